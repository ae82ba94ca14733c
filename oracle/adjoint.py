"""Gradients of L = 1/2 ||u(T) - u_target||^2 through the fine integration (oracle).

TEST INFRASTRUCTURE ONLY -- see the package docstring.

The converged Parareal result is the serial fine solution (Section 3.1,
interface conditions; Section 3.2, finite termination), so the gradient of the
loss through the solver is the gradient through M = N*m explicit-Euler steps
  u_{n+1} = A u_n,   A = I + nu*dt*L_h,
with dt fixed by the slicing (independent of nu).  With g = u_M - u_target and
the adjoint states mu_M = g, mu_n = A^T mu_{n+1}:
  dL/du0 = mu_0 = (A^T)^M g
  dL/dnu = sum_{n=0}^{M-1} mu_{n+1}^T (dt * L_h u_n).
A is symmetric and commutes with L_h, so these also have the closed forms
  dL/du0 = A^M g            (a serial fine run started from g)
  dL/dnu = M * dt * g^T L_h u_{M-1}.
"""
from __future__ import annotations

import numpy as np

from . import heat


def loss(uT: np.ndarray, target: np.ndarray) -> float:
    d = uT - target
    return 0.5 * float(np.vdot(d, d))


def forward_uT(u0: np.ndarray, r: float, M: int) -> np.ndarray:
    return heat.fine(u0, r, M)


def grad_closed_form(u0: np.ndarray, target: np.ndarray, r: float, M: int,
                     dt: float, h: float):
    """(dL/du0, dL/dnu) from the closed forms above."""
    u_prev = heat.fine(u0, r, M - 1)          # u_{M-1}
    uT = heat.fine_step(u_prev, r)            # u_M
    g = uT - target
    dldu0 = heat.fine(g, r, M)
    lap = heat.laplacian_h2(u_prev) / (h * h)
    dldnu = M * dt * float(np.vdot(g, lap))
    return dldu0, dldnu


def grad_reverse(u0: np.ndarray, target: np.ndarray, r: float, M: int,
                 dt: float, h: float):
    """Plain reverse sweep that stores every forward state (small sizes only)."""
    states = [u0]
    for _ in range(M):
        states.append(heat.fine_step(states[-1], r))
    mu = states[-1] - target
    dldnu = 0.0
    for n in range(M - 1, -1, -1):
        lap = heat.laplacian_h2(states[n]) / (h * h)
        dldnu += float(np.vdot(mu, dt * lap))       # mu_{n+1}^T dA/dnu u_n
        mu = heat.fine_step(mu, r)                  # A^T mu (A symmetric)
    return mu, dldnu

