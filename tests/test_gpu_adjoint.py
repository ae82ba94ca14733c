"""Adjoint gradient (dL/du0, dL/dnu) on the GPU vs the oracle and central FD.

Bar: <= 1e-6 relative against the CPU reference gradient (the closed forms of
the oracle; the spectral closed form at full size), and central differences
within the noise bound 1e-6 |g| + 10 eps_mach |L| / eps_fd.
"""
import math

import numpy as np
import pytest

import workloads
from oracle import adjoint, heat, spectral

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2110_10762_amd as pr  # noqa: E402

DEV = "cuda:0"


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def disc_of(p):
    return heat.discretise(p.dim, p.n, p.nu, p.T, p.nslices, p.dt_nominal)


def gpu_grad(p, driver="fine"):
    prob = pr.Problem(pr.config_of(p))
    lam = torch.empty((p.nslices + 1,) + p.u0.shape, dtype=torch.float64, device=DEV)
    if driver == "fine":
        prob.solve_fine(dev(p.u0), lam)
    else:
        prob.solve_sync(dev(p.u0), lam)
    gT = lam[-1] - dev(p.target)
    d0 = torch.empty_like(gT)
    dnu = prob.grad(lam, gT.contiguous(), d0)
    return d0.cpu().numpy(), dnu, lam


@pytest.mark.parametrize("n,N,T", [(63, 4, 1e-2), (40, 6, 2e-2)])
def test_grad_vs_oracle_closed_form(n, N, T):
    p = workloads.adjoint2d(n=n, nslices=N, T=T)
    d = disc_of(p)
    M = d.m * d.nslices
    g0, gnu = adjoint.grad_closed_form(p.u0, p.target, d.r, M, d.dt, d.h)
    d0, dnu, _ = gpu_grad(p)
    assert np.max(np.abs(d0 - g0)) <= 1e-10 * np.max(np.abs(g0))
    assert abs(dnu - gnu) <= 1e-9 * abs(gnu)
    g1, gnu1 = adjoint.grad_reverse(p.u0, p.target, d.r, M, d.dt, d.h)
    assert abs(dnu - gnu1) <= 1e-9 * abs(gnu1)


def test_grad_1d_and_3d_vs_oracle():
    p = workloads.heat1d()
    p.target = 0.3 * np.sin(2 * np.pi * workloads.grid(p.n))
    d = disc_of(p)
    M = d.m * d.nslices
    g0, gnu = adjoint.grad_closed_form(p.u0, p.target, d.r, M, d.dt, d.h)
    d0, dnu, _ = gpu_grad(p)
    assert np.max(np.abs(d0 - g0)) <= 1e-10 * np.max(np.abs(g0))
    assert abs(dnu - gnu) <= 1e-9 * abs(gnu)
    p = workloads.heat3d(n=16, nslices=3, T=3e-3)
    p.target = 0.5 * p.u0[::-1].copy()
    d = disc_of(p)
    M = d.m * d.nslices
    g0, gnu = adjoint.grad_closed_form(p.u0, p.target, d.r, M, d.dt, d.h)
    d0, dnu, _ = gpu_grad(p)
    assert np.max(np.abs(d0 - g0)) <= 1e-10 * np.max(np.abs(g0))
    assert abs(dnu - gnu) <= 1e-9 * abs(gnu)


def test_grad_full_size_vs_spectral_closed_form():
    # the adjoint workload at full size: 512^2, 32 slices, 206 steps per slice
    p = workloads.adjoint2d()
    d = disc_of(p)
    M = d.m * d.nslices
    f, _ = spectral.symbols(2, p.n, d.r, 1, 0.0)        # one-step amplification
    u0h = spectral.dst(p.u0)
    uT = spectral.idst(f ** M * u0h)
    g = uT - p.target
    want0 = spectral.idst(f ** M * spectral.dst(g))
    u_prev = spectral.idst(f ** (M - 1) * u0h)
    want_nu = M * d.dt * float(np.vdot(g, heat.laplacian_h2(u_prev))) / d.h ** 2
    d0, dnu, lam = gpu_grad(p, driver="sync")        # checkpoints from Parareal to 1e-10
    assert np.max(np.abs(d0 - want0)) <= 1e-6 * np.max(np.abs(want0))
    assert abs(dnu - want_nu) <= 1e-6 * abs(want_nu)


def test_grad_vs_central_fd_on_gpu():
    p = workloads.adjoint2d(n=95, nslices=4, T=4e-3)
    d = disc_of(p)
    d0, dnu, _ = gpu_grad(p)

    def L(nu, u0):
        prob = pr.Problem(pr.config_of(p, nu=nu))
        lam = torch.empty((p.nslices + 1,) + p.u0.shape, dtype=torch.float64, device=DEV)
        prob.solve_fine(dev(u0), lam)
        r = lam[-1] - dev(p.target)
        return 0.5 * float((r * r).sum())

    e = 1e-6
    L0 = L(p.nu, p.u0)
    fd = (L(p.nu + e, p.u0) - L(p.nu - e, p.u0)) / (2 * e)
    assert abs(fd - dnu) <= 1e-6 * abs(dnu) + 10 * 2.2e-16 * abs(L0) / e
    rng = np.random.default_rng(4)
    for _ in range(4):
        v = rng.standard_normal(p.u0.shape)
        v /= np.linalg.norm(v)
        fdu = (L(p.nu, p.u0 + e * v) - L(p.nu, p.u0 - e * v)) / (2 * e)
        assert abs(fdu - float(np.vdot(d0, v))) <= 1e-6 * np.linalg.norm(d0) + 10 * 2.2e-16 * abs(L0) / e


def test_autograd_function():
    p = workloads.adjoint2d(n=48, nslices=4, T=1e-2)
    d = disc_of(p)
    M = d.m * d.nslices
    u0 = dev(p.u0).requires_grad_(True)
    nu = torch.tensor(p.nu, dtype=torch.float64, device=DEV, requires_grad=True)
    uT = pr.heat_parareal(u0, nu, 2, p.n, p.T, p.nslices, p.dt_nominal, eps=1e-12, driver="sync")
    loss = 0.5 * ((uT - dev(p.target)) ** 2).sum()
    loss.backward()
    g0, gnu = adjoint.grad_closed_form(p.u0, p.target, d.r, M, d.dt, d.h)
    assert np.max(np.abs(u0.grad.cpu().numpy() - g0)) <= 1e-6 * np.max(np.abs(g0))
    assert abs(nu.grad.item() - gnu) <= 1e-6 * abs(gnu)
