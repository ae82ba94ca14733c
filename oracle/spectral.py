"""Exact sine-mode closed forms of F, G and Parareal (oracle).

TEST INFRASTRUCTURE ONLY -- see the package docstring.

With zero Dirichlet values the grid functions sin(k pi x_j), k = 1..n, are the
eigenvectors of the finite-difference Laplacian, with eigenvalue
-mu_k/h^2, mu_k = 4 sin^2(k pi h / 2) per dimension (tensor products and sums in
2D/3D).  Both propagators are diagonal in that basis:
  F (m explicit-Euler steps):  f_k = (1 - r mu_k)^m
  G (one backward-Euler step): g_k = 1 / (1 + s mu_k)
so every quantity the method computes has a per-mode scalar form.  Section 3.1
writes the linear case as G(l) = cal_G l + delta and F(l) = cal_F l + zeta; for
the heat problem delta = zeta = 0, and equation (pr) per mode is the scalar
recurrence l_n^{k+1} = g l_{n-1}^{k+1} + (f - g) l_{n-1}^k, l_n^0 = g^n l_0,
whose solution is
  l_n^k = l_0 * sum_{j=0}^{min(k,n)} C(n, j) (f - g)^j g^(n-j)
(check: k = 0 gives g^n; Pascal's rule C(n-1,j) + C(n-1,j-1) = C(n,j) gives the
recurrence; k >= n gives (g + f - g)^n = f^n, the serial fine value, which is
the finite termination of Section 3.2).  The discrete sine transform (DST-I,
orthonormal) is a library routine that moves between grid and mode values.
"""
from __future__ import annotations

import math
import os

import numpy as np
import scipy.fft


_WORKERS = max(1, min(16, os.cpu_count() or 1))


def dst(u: np.ndarray) -> np.ndarray:
    """Orthonormal DST-I over every axis (its own inverse); the library
    routine's own threads share the 1D transforms of large grids."""
    return scipy.fft.dstn(u, type=1, norm="ortho", workers=_WORKERS)


idst = dst


def mode_mu(dim: int, n: int) -> np.ndarray:
    """mu(k) = sum_d 4 sin^2(k_d pi h / 2), array shaped like a grid function."""
    h = 1.0 / (n + 1)
    k = np.arange(1, n + 1)
    m1 = 4.0 * np.sin(k * np.pi * h / 2.0) ** 2
    mu = np.zeros((n,) * dim)
    for d in range(dim):
        shape = [1] * dim
        shape[d] = n
        mu = mu + m1.reshape(shape)
    return mu


def symbols(dim: int, n: int, r: float, m: int, s: float):
    """Per-mode amplification of F and G."""
    mu = mode_mu(dim, n)
    return (1.0 - r * mu) ** m, 1.0 / (1.0 + s * mu)


def fine(u: np.ndarray, r: float, m: int) -> np.ndarray:
    f, _ = symbols(u.ndim, u.shape[0], r, m, 0.0)
    return idst(f * dst(u))


def coarse(u: np.ndarray, s: float) -> np.ndarray:
    _, g = symbols(u.ndim, u.shape[0], 0.0, 1, s)
    return idst(g * dst(u))


def serial_fine(u0: np.ndarray, r: float, m: int, nslices: int, slices=None) -> np.ndarray:
    """lambda*_i = F^i u0 for the requested slices (default: all 0..N)."""
    if slices is None:
        slices = range(nslices + 1)
    f, _ = symbols(u0.ndim, u0.shape[0], r, m, 0.0)
    u0h = dst(u0)
    return np.stack([idst(f ** i * u0h) for i in slices])


def parareal_coefficients(f: np.ndarray, g: np.ndarray, slice_index: int, k: int) -> np.ndarray:
    """sum_{j=0}^{min(k,n)} C(n, j) (f-g)^j g^(n-j), elementwise over modes."""
    n = slice_index
    out = np.zeros_like(f)
    d = f - g
    for j in range(0, min(k, n) + 1):
        out += float(math.comb(n, j)) * d ** j * g ** (n - j)
    return out


def parareal_sync(u0: np.ndarray, r: float, m: int, s: float, k: int,
                  slices) -> np.ndarray:
    """Synchronous Parareal iterate lambda_i^k (exact G, exact arithmetic up to
    rounding) for the requested slice indices."""
    f, g = symbols(u0.ndim, u0.shape[0], r, m, s)
    u0h = dst(u0)
    return np.stack([idst(parareal_coefficients(f, g, i, k) * u0h) for i in slices])


def parareal_sync_change(u0: np.ndarray, r: float, m: int, s: float, k: int,
                         slices) -> np.ndarray:
    """lambda_i^k - lambda_i^{k-1} of synchronous Parareal with exact G for the
    requested slices: by the closed form above only the j = k term changes,
    C(i, k) (f - g)^k g^(i-k) per mode (zero for slices i < k, which are
    already exact).  Its max norm over all slices is the change of the
    stopping test, eq. (thresh)."""
    f, g = symbols(u0.ndim, u0.shape[0], r, m, s)
    u0h = dst(u0)
    d = f - g
    out = []
    for i in slices:
        if i < k or k < 1:
            out.append(np.zeros_like(u0))
        else:
            out.append(idst(float(math.comb(i, k)) * d ** k * g ** (i - k) * u0h))
    return np.stack(out)
