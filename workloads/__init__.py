"""Seeded synthetic inputs for the heat-equation Parareal workloads.

This module only describes problems and draws their initial data.  It holds
none of the method's arithmetic (no time stepping, no solves, no step-count
derivation): both the CPU oracle and the HIP library receive what it produces
and derive everything else on their own.

Problem statement (paper, Section 3.1, equation (pde) and the time
decomposition that follows it): heat equation u_t = nu * Laplace(u) on the unit
interval / square / cube, zero Dirichlet boundary, interior grid points
x_j = j*h, h = 1/(n+1), j = 1..n, stored C-order with x fastest.

Draw order per workload (NumPy PCG64, ``default_rng(seed)``):
  heat1d   seed 0: z = standard_normal(8); u0 = sum_k (z_k/k) sin(k pi x)
  heat2d   seed 1: centres uniform(0.1, 0.9, (16, 2)), widths uniform(0.02, 0.1, 16)
  heat3d   seed 2: centres uniform(0.1, 0.9, (32, 3)), widths uniform(0.02, 0.1, 32),
                   noise normal(0, 0.01, n^3)  (0.01 is the standard deviation)
  batched  seed 3: per problem, in order: side, log10 nu, slice count, the 256
                   sine-mode amplitudes (k_x, k_y <= 16, a = z / sqrt(kx^2+ky^2))
  adjoint  seed 4: u0 centres/widths (16 bumps), then target centres/widths
                   (8 bumps, amplitude 0.5)
  heat3d_long seed 5: as heat3d (32 bumps + noise) on 128^3, 64 slices of 100
                   fine steps each: the paper's regime of a slice 100 fine
                   steps long (Section 5.1), which the 256^3 workload, with
                   less than one step per slice, does not reach
A Gaussian bump is exp(-|x - c|^2 / (2 sigma^2)) with amplitude 1; bumps near a
wall are simply cut by the zero boundary.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Tuple

import numpy as np

__all__ = [
    "Problem", "grid", "bumps", "sine_modes_1d", "sine_modes_2d",
    "heat1d", "heat2d", "heat3d", "heat3d_long", "adjoint2d", "batched", "by_name",
]


@dataclasses.dataclass
class Problem:
    """One heat problem: geometry, physics, slicing, solver knobs and u0."""
    name: str
    dim: int
    n: int                 # interior points per dimension
    nu: float              # diffusivity
    T: float               # end time
    nslices: int           # number of time slices N (the paper's p)
    dt_nominal: float      # requested fine step; the solver rounds it down so
                           # that an integer number of steps fills a slice
    eps: float = 1e-10     # Parareal stopping threshold on ||lambda^k - lambda^{k-1}||_inf
    cg_tol: float = 1e-12  # relative residual for the backward-Euler solve (dim >= 2)
    u0: Optional[np.ndarray] = None          # shape (n,)*dim, float64
    target: Optional[np.ndarray] = None      # adjoint workloads only

    @property
    def npts(self) -> int:
        return self.n ** self.dim

    @property
    def h(self) -> float:
        return 1.0 / (self.n + 1)


def grid(n: int) -> np.ndarray:
    """Interior coordinates j*h, j = 1..n, h = 1/(n+1)."""
    return np.arange(1, n + 1, dtype=np.float64) / (n + 1)


def bumps(n: int, dim: int, centres: np.ndarray, widths: np.ndarray,
          amplitude: float = 1.0) -> np.ndarray:
    """Sum of Gaussian bumps on the interior grid, built from separable factors."""
    x = grid(n)
    out = np.zeros((n,) * dim, dtype=np.float64)
    for c, s in zip(centres, widths):
        f = [np.exp(-(x - c[d]) ** 2 / (2.0 * s * s)) for d in range(dim)]
        if dim == 1:
            out += f[0]
        elif dim == 2:
            out += np.outer(f[1], f[0])            # index [y, x]
        else:
            out += f[2][:, None, None] * f[1][None, :, None] * f[0][None, None, :]
    return amplitude * out


def sine_modes_1d(n: int, amps: np.ndarray) -> np.ndarray:
    x = grid(n)
    k = np.arange(1, len(amps) + 1)
    return (amps[:, None] * np.sin(np.pi * k[:, None] * x[None, :])).sum(axis=0)


def sine_modes_2d(n: int, amps: np.ndarray) -> np.ndarray:
    """amps[ky-1, kx-1] * sin(kx pi x) sin(ky pi y), array index [y, x]."""
    x = grid(n)
    kk = np.arange(1, amps.shape[0] + 1)
    sx = np.sin(np.pi * kk[:, None] * x[None, :])        # [k, x]
    return np.einsum("ab,ay,bx->yx", amps, sx, sx)


def heat1d(n: int = 127) -> Problem:
    rng = np.random.default_rng(0)
    z = rng.standard_normal(8)
    amps = z / np.arange(1, 9)
    h = 1.0 / (n + 1)
    p = Problem("heat1d", 1, n, 1.0, 0.1, 16, 0.4 * h * h)
    p.u0 = sine_modes_1d(n, amps)
    p.amps = amps  # type: ignore[attr-defined]
    return p


def heat2d(n: int = 1024, nslices: int = 64, T: float = 1e-3) -> Problem:
    rng = np.random.default_rng(1)
    centres = rng.uniform(0.1, 0.9, (16, 2))
    widths = rng.uniform(0.02, 0.1, 16)
    h = 1.0 / (n + 1)
    p = Problem("heat2d", 2, n, 1.0, T, nslices, 0.2 * h * h)
    p.u0 = bumps(n, 2, centres, widths)
    return p


def heat3d(n: int = 256, nslices: int = 128, T: float = 2e-4) -> Problem:
    rng = np.random.default_rng(2)
    centres = rng.uniform(0.1, 0.9, (32, 3))
    widths = rng.uniform(0.02, 0.1, 32)
    noise = rng.normal(0.0, 0.01, n ** 3)
    h = 1.0 / (n + 1)
    p = Problem("heat3d", 3, n, 0.5, T, nslices, 0.15 * h * h)
    p.u0 = bumps(n, 3, centres, widths) + noise.reshape(n, n, n)
    return p


HEAT3D_LONG_STEPS = 100   # fine steps per slice, dt = 0.15 h^2


def heat3d_long(n: int = 128, nslices: int = 64, steps: int = HEAT3D_LONG_STEPS) -> Problem:
    rng = np.random.default_rng(5)
    centres = rng.uniform(0.1, 0.9, (32, 3))
    widths = rng.uniform(0.02, 0.1, 32)
    noise = rng.normal(0.0, 0.01, n ** 3)
    h = 1.0 / (n + 1)
    dt = 0.15 * h * h
    p = Problem("heat3d_long", 3, n, 0.5, nslices * steps * dt, nslices, dt)
    p.u0 = bumps(n, 3, centres, widths) + noise.reshape(n, n, n)
    return p


def adjoint2d(n: int = 512, nslices: int = 32, T: float = 5e-3) -> Problem:
    rng = np.random.default_rng(4)
    c0 = rng.uniform(0.1, 0.9, (16, 2))
    s0 = rng.uniform(0.02, 0.1, 16)
    c1 = rng.uniform(0.1, 0.9, (8, 2))
    s1 = rng.uniform(0.02, 0.1, 8)
    h = 1.0 / (n + 1)
    p = Problem("adjoint2d", 2, n, 1.0, T, nslices, 0.2 * h * h)
    p.u0 = bumps(n, 2, c0, s0)
    p.target = bumps(n, 2, c1, s1, amplitude=0.5)
    return p


BATCH_SIDES = (64, 128, 256, 512)
BATCH_STEPS_PER_SLICE = 64   # fine steps per slice, dt = 0.2 h^2 / nu


def batched(count: int = 512, sides: Tuple[int, ...] = BATCH_SIDES,
            max_slices: int = 64, modes: int = 16) -> List[Problem]:
    """Independent 2D problems of uneven side, diffusivity and slice count.

    Each problem has dt = 0.2 h^2/nu and T = N * 64 * dt, so every slice holds
    exactly 64 fine steps.  ``sides``/``max_slices`` may be shrunk for tests;
    the draws are made in the same order either way.
    """
    rng = np.random.default_rng(3)
    out = []
    kk = np.arange(1, modes + 1)
    norm = np.sqrt(kk[:, None] ** 2 + kk[None, :] ** 2)
    for b in range(count):
        side = int(sides[rng.integers(0, len(sides))])
        nu = float(10.0 ** rng.uniform(-1.0, 1.0))
        ns = int(rng.integers(8, max_slices + 1))
        amps = rng.standard_normal((modes, modes)) / norm
        h = 1.0 / (side + 1)
        dt = 0.2 * h * h / nu
        p = Problem(f"batched[{b}]", 2, side, nu, ns * BATCH_STEPS_PER_SLICE * dt, ns, dt)
        p.u0 = sine_modes_2d(side, amps)
        out.append(p)
    return out


def by_name(name: str) -> Problem:
    return {"heat1d": heat1d, "heat2d": heat2d, "heat3d": heat3d, "heat3d_long": heat3d_long,
            "adjoint2d": adjoint2d}[name]()
