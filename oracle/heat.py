"""Discretised heat problem, fine propagator F and coarse propagator G (oracle).

TEST INFRASTRUCTURE ONLY -- see the package docstring.

The paper leaves F and G abstract (Section 3.1: F is an accurate solve of one
slice's subproblem, G a cheap approximate one) and in its experiment uses
implicit time integrators on a finite-element mesh (Section 5.1).  Here, as the
workloads prescribe, F is m explicit-Euler steps of the standard
(2d+1)-point finite-difference Laplacian and G is one backward-Euler step of
the same Laplacian, both with zero Dirichlet ghost values.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass(frozen=True)
class Discretisation:
    dim: int
    n: int
    h: float
    nslices: int
    dT: float      # slice length T/N
    m: int         # fine steps per slice
    dt: float      # fine step dT/m
    r: float       # nu*dt/h^2  (explicit Euler mesh ratio)
    s: float       # nu*dT/h^2  (backward Euler mesh ratio)


def discretise(dim: int, n: int, nu: float, T: float, nslices: int,
               dt_nominal: float) -> Discretisation:
    """Time decomposition [T_{i-1}, T_i] of equal length (Section 3.1) and the
    fine step count: the smallest m with dT/m <= dt_nominal (up to 1e-9 slack
    for ratios that are integers in exact arithmetic)."""
    h = 1.0 / (n + 1)
    dT = T / nslices
    m = max(1, math.ceil(dT / dt_nominal - 1e-9))
    dt = dT / m
    return Discretisation(dim, n, h, nslices, dT, m, dt, nu * dt / (h * h),
                          nu * dT / (h * h))


def laplacian_h2(u: np.ndarray) -> np.ndarray:
    """h^2 * L_h u: sum over axes of u(x-e) + u(x+e) - 2u(x), zero outside."""
    out = -2.0 * u.ndim * u
    for ax in range(u.ndim):
        lo = [slice(None)] * u.ndim
        hi = [slice(None)] * u.ndim
        lo[ax] = slice(0, -1)
        hi[ax] = slice(1, None)
        out[tuple(hi)] += u[tuple(lo)]     # left neighbour
        out[tuple(lo)] += u[tuple(hi)]     # right neighbour
    return out


def fine_step(u: np.ndarray, r: float) -> np.ndarray:
    """One explicit-Euler step u + dt*nu*L_h u = u + r * h^2 L_h u."""
    return u + r * laplacian_h2(u)


def fine(u: np.ndarray, r: float, m: int) -> np.ndarray:
    """F: m explicit-Euler steps over one slice (the accurate propagator)."""
    for _ in range(m):
        u = fine_step(u, r)
    return u


def serial_fine(u0: np.ndarray, r: float, m: int, nslices: int) -> np.ndarray:
    """lambda*_0 = u0, lambda*_i = F(lambda*_{i-1}): the sequential composition
    of F over all slices that Parareal must reproduce (Section 3.1, and the
    interface conditions (itf_cond)).  Returns shape (N+1,) + u0.shape."""
    out = np.empty((nslices + 1,) + u0.shape)
    out[0] = u0
    for i in range(1, nslices + 1):
        out[i] = fine(out[i - 1], r, m)
    return out


def be_apply(y: np.ndarray, s: float) -> np.ndarray:
    """(I - nu*dT*L_h) y = y - s * h^2 L_h y, the backward-Euler matrix."""
    return y - s * laplacian_h2(y)


def coarse_thomas(x: np.ndarray, s: float) -> np.ndarray:
    """G in 1D: solve tridiag(-s, 1+2s, -s) w = x by the Thomas algorithm
    (Gaussian elimination without pivoting; the matrix is strictly diagonally
    dominant)."""
    n = x.shape[0]
    a = -s
    b = 1.0 + 2.0 * s
    c = -s
    cp = np.empty(n)
    dp = np.empty(n)
    cp[0] = c / b
    dp[0] = x[0] / b
    for i in range(1, n):
        den = b - a * cp[i - 1]
        cp[i] = c / den
        dp[i] = (x[i] - a * dp[i - 1]) / den
    w = np.empty(n)
    w[n - 1] = dp[n - 1]
    for i in range(n - 2, -1, -1):
        w[i] = dp[i] - cp[i] * w[i + 1]
    return w


def coarse_cg(x: np.ndarray, s: float, tol: float = 1e-12, maxit: int = 0):
    """G in 2D/3D: textbook (Hestenes-Stiefel) conjugate gradients on the
    symmetric positive definite backward-Euler system, started from x0 = b,
    stopped when ||r||_2 <= tol * ||b||_2.  Returns (w, iterations)."""
    b = x
    if maxit <= 0:
        maxit = 10 * b.shape[0] + 10
    w = b.copy()
    res = b - be_apply(w, s)
    p = res.copy()
    rr = float(np.vdot(res, res))
    bnorm = math.sqrt(float(np.vdot(b, b)))
    it = 0
    while it < maxit and math.sqrt(rr) > tol * bnorm:
        q = be_apply(p, s)
        alpha = rr / float(np.vdot(p, q))
        w = w + alpha * p
        res = res - alpha * q
        rr_new = float(np.vdot(res, res))
        p = res + (rr_new / rr) * p
        rr = rr_new
        it += 1
    return w, it


def fine_theta(u: np.ndarray, r: float, m: int, theta: float, tol: float = 1e-12) -> np.ndarray:
    """Implicit F: m steps of the theta-method for u_t = nu L_h u (the paper's
    experiments use implicit fine integrators, Section 5.1: theta = 1/2 is the
    trapezoidal rule, theta = 1 backward Euler).  Each step solves
        (I - theta r h^2 L_h) u' = (I + (1 - theta) r h^2 L_h) u,
    the left-hand matrix being the backward-Euler matrix with s = theta r, by
    Thomas in 1D and by the textbook CG of coarse_cg otherwise (x0 = the
    right-hand side, ||res||_2 <= tol ||rhs||_2)."""
    for _ in range(m):
        b = u + ((1.0 - theta) * r) * laplacian_h2(u) if theta != 1.0 else u
        if u.ndim == 1:
            u = coarse_thomas(b, theta * r)
        else:
            u = coarse_cg(b, theta * r, tol)[0]
    return u


def serial_fine_theta(u0: np.ndarray, r: float, m: int, nslices: int, theta: float,
                      tol: float = 1e-12) -> np.ndarray:
    """serial_fine with the implicit F of fine_theta."""
    out = np.empty((nslices + 1,) + u0.shape)
    out[0] = u0
    for i in range(1, nslices + 1):
        out[i] = fine_theta(out[i - 1], r, m, theta, tol)
    return out


def be_matrix(dim: int, n: int, s: float) -> np.ndarray:
    """Dense backward-Euler matrix (tiny n only), for brute-force pins."""
    N = n ** dim
    M = np.empty((N, N))
    e = np.zeros((n,) * dim)
    for j in range(N):
        e.flat[:] = 0.0
        e.flat[j] = 1.0
        M[:, j] = be_apply(e, s).ravel()
    return M


def fine_matrix_step(dim: int, n: int, r: float) -> np.ndarray:
    """Dense one-step explicit-Euler matrix I + r h^2 L_h (tiny n only)."""
    N = n ** dim
    M = np.empty((N, N))
    e = np.zeros((n,) * dim)
    for j in range(N):
        e.flat[:] = 0.0
        e.flat[j] = 1.0
        M[:, j] = fine_step(e, r).ravel()
    return M


class Propagators:
    """F and G bound to one discretisation (G: Thomas in 1D, CG otherwise)."""

    def __init__(self, disc: Discretisation, cg_tol: float = 1e-12,
                 coarse: str = "auto", theta: float = 0.0):
        self.disc = disc
        self.cg_tol = cg_tol
        self.theta = theta      # 0: explicit Euler F; 1/2, 1: implicit F (fine_theta)
        if coarse == "auto":
            coarse = "thomas" if disc.dim == 1 else "cg"
        self.coarse = coarse
        self.cg_iters = []

    def F(self, u: np.ndarray) -> np.ndarray:
        if self.theta:
            return fine_theta(u, self.disc.r, self.disc.m, self.theta, self.cg_tol)
        return fine(u, self.disc.r, self.disc.m)

    def G(self, u: np.ndarray) -> np.ndarray:
        if self.coarse == "thomas":
            return coarse_thomas(u, self.disc.s)
        if self.coarse == "dense":
            M = be_matrix(self.disc.dim, self.disc.n, self.disc.s)
            return np.linalg.solve(M, u.ravel()).reshape(u.shape)
        w, it = coarse_cg(u, self.disc.s, self.cg_tol)
        self.cg_iters.append(it)
        return w
