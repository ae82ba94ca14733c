"""Pins of the CPU oracle against facts fixed by the paper and the mathematics.

Each test checks the oracle against something other than itself: closed forms
written out here, dense brute force, library solvers, the paper's stated
invariants (finite termination, fixed-point equivalence, synchronous as a
special case of asynchronous, stale input gives F, kappa >= k).
"""
import math

import numpy as np
import pytest

import workloads
from oracle import adjoint, heat, parareal, spectral


def _disc(p):
    return heat.discretise(p.dim, p.n, p.nu, p.T, p.nslices, p.dt_nominal)


# ---------------------------------------------------------------- P1: fine propagator

@pytest.mark.parametrize("k", [1, 3, 17, 64, 127])
def test_fine_sine_mode_amplification_1d(k):
    # explicit Euler on sin(k pi x_j): factor 1 - 4 r sin^2(k pi h/2) per step
    n, r, m = 127, 0.4, 256
    h = 1.0 / (n + 1)
    x = np.arange(1, n + 1) * h
    u0 = np.sin(k * np.pi * x)
    amp = (1.0 - 4.0 * r * math.sin(k * math.pi * h / 2) ** 2) ** m
    got = heat.fine(u0, r, m)
    assert np.max(np.abs(got - amp * u0)) <= 1e-13 * max(1.0, abs(amp)) + 1e-15


@pytest.mark.parametrize("dim,n,kvec", [(2, 31, (2, 5)), (2, 31, (31, 1)), (3, 15, (1, 4, 9))])
def test_fine_tensor_mode_amplification(dim, n, kvec):
    r, m = 0.9 / (2 * dim), 40
    h = 1.0 / (n + 1)
    x = np.arange(1, n + 1) * h
    u0 = np.ones((n,) * dim)
    mu = 0.0
    for d, kd in enumerate(kvec):              # array axis 0 is the slowest coordinate
        shape = [1] * dim
        shape[dim - 1 - d] = n
        u0 = u0 * np.sin(kd * np.pi * x).reshape(shape)
        mu += 4.0 * math.sin(kd * math.pi * h / 2) ** 2
    amp = (1.0 - r * mu) ** m
    got = heat.fine(u0, r, m)
    assert np.max(np.abs(got - amp * u0)) <= 1e-13


def test_fine_heat1d_closed_form():
    # the 1D workload's u0 is a sum of 8 discrete eigenmodes: u(T) has a closed form
    p = workloads.heat1d()
    d = _disc(p)
    assert (d.m, d.dt, d.r) == (256, 2.44140625e-05, 0.4)
    x = workloads.grid(p.n)
    M = d.m * d.nslices
    exact = np.zeros(p.n)
    for k, a in enumerate(p.amps, start=1):
        exact += a * (1 - 4 * d.r * math.sin(k * math.pi * d.h / 2) ** 2) ** M * np.sin(k * np.pi * x)
    got = heat.serial_fine(p.u0, d.r, d.m, d.nslices)[-1]
    assert np.max(np.abs(got - exact)) <= 1e-13 * np.max(np.abs(exact))


@pytest.mark.parametrize("dim,n", [(1, 9), (2, 5), (3, 3)])
def test_fine_dense_brute_force(dim, n):
    rng = np.random.default_rng(11)
    u0 = rng.standard_normal((n,) * dim)
    r, m = 0.15, 23
    A = np.eye(n ** dim)
    h2 = (n + 1) ** 2
    # build I + r*h^2*L_h by hand from the stencil definition
    idx = np.arange(n ** dim).reshape((n,) * dim)
    for p in range(n ** dim):
        c = np.unravel_index(p, (n,) * dim)
        A[p, p] -= 2 * dim * r
        for ax in range(dim):
            for sgn in (-1, 1):
                q = list(c)
                q[ax] += sgn
                if 0 <= q[ax] < n:
                    A[p, idx[tuple(q)]] += r
    want = np.linalg.matrix_power(A, m) @ u0.ravel()
    assert np.allclose(heat.fine(u0, r, m).ravel(), want, rtol=0, atol=1e-13)
    assert h2 > 0


# ---- implicit fine propagators (theta-method: trapezoidal 1/2, backward Euler 1)

def _stencil_matrix(dim, n):
    """h^2 L_h as a dense matrix, built point by point from the stencil."""
    N = n ** dim
    A = np.zeros((N, N))
    idx = np.arange(N).reshape((n,) * dim)
    for p in range(N):
        c = np.unravel_index(p, (n,) * dim)
        A[p, p] = -2.0 * dim
        for ax in range(dim):
            for sgn in (-1, 1):
                q = list(c)
                q[ax] += sgn
                if 0 <= q[ax] < n:
                    A[p, idx[tuple(q)]] = 1.0
    return A


@pytest.mark.parametrize("theta", [0.5, 1.0])
@pytest.mark.parametrize("dim,n,kvec,r", [(1, 127, (5,), 3.0), (2, 31, (2, 7), 0.8), (3, 11, (1, 3, 9), 2.5)])
def test_fine_theta_mode_amplification(theta, dim, n, kvec, r):
    # on a discrete eigenmode with h^2 L_h eigenvalue -mu, one theta-step
    # multiplies by (1 - (1 - theta) r mu) / (1 + theta r mu); unconditionally
    # stable, so r may exceed the explicit limit 1/(2d)
    m = 7
    h = 1.0 / (n + 1)
    x = np.arange(1, n + 1) * h
    u0 = np.ones((n,) * dim)
    mu = 0.0
    for d, kd in enumerate(kvec):
        shape = [1] * dim
        shape[dim - 1 - d] = n
        u0 = u0 * np.sin(kd * np.pi * x).reshape(shape)
        mu += 4.0 * math.sin(kd * math.pi * h / 2) ** 2
    amp = ((1.0 - (1.0 - theta) * r * mu) / (1.0 + theta * r * mu)) ** m
    got = heat.fine_theta(u0, r, m, theta)
    assert np.max(np.abs(got - amp * u0)) <= 1e-11


@pytest.mark.parametrize("theta", [0.5, 1.0])
@pytest.mark.parametrize("dim,n", [(1, 9), (2, 5), (3, 3)])
def test_fine_theta_dense_brute_force(theta, dim, n):
    rng = np.random.default_rng(12)
    u0 = rng.standard_normal((n,) * dim)
    r, m = 1.7, 9
    A = _stencil_matrix(dim, n)
    I = np.eye(n ** dim)
    step = np.linalg.solve(I - theta * r * A, I + (1.0 - theta) * r * A)
    want = np.linalg.matrix_power(step, m) @ u0.ravel()
    assert np.allclose(heat.fine_theta(u0, r, m, theta).ravel(), want, rtol=0, atol=1e-11)


@pytest.mark.parametrize("theta", [0.5, 1.0])
def test_sync_finite_termination_implicit_fine_bitwise(theta):
    # finite termination holds for any F (Section 3.2): with the implicit F,
    # k = N reproduces the serial implicit integration bit for bit
    p = workloads.heat2d(n=15, nslices=5, T=2e-2)
    d = heat.discretise(p.dim, p.n, p.nu, p.T, p.nslices, 4 * p.dt_nominal)
    props = heat.Propagators(d, cg_tol=1e-12, theta=theta)
    res = parareal.parareal_sync(p.u0, props.F, props.G, d.nslices, eps=0.0)
    ser = heat.serial_fine_theta(p.u0, d.r, d.m, d.nslices, theta)
    assert res.iters == d.nslices
    assert np.array_equal(res.lam, ser)


def test_discretise_rounding_rule():
    # slice length divided into the fewest steps not above the requested one
    d = heat.discretise(2, 1024, 1.0, 1e-3, 64, 0.2 / 1025 ** 2)
    assert d.m == 83 and d.dt <= 0.2 / 1025 ** 2
    d = heat.discretise(3, 256, 0.5, 2e-4, 128, 0.15 / 257 ** 2)
    assert d.m == 1 and abs(d.r - 0.05160078125) < 1e-15
    d = heat.discretise(2, 512, 1.0, 5e-3, 32, 0.2 / 513 ** 2)
    assert d.m == 206


# ---------------------------------------------------------------- P2: coarse propagator

@pytest.mark.parametrize("n,s", [(31, 0.3), (127, 102.4), (64, 1e-3)])
def test_thomas_vs_dense_solve(n, s):
    rng = np.random.default_rng(n)
    x = rng.standard_normal(n)
    T = np.diag(np.full(n, 1 + 2 * s)) + np.diag(np.full(n - 1, -s), 1) + np.diag(np.full(n - 1, -s), -1)
    want = np.linalg.solve(T, x)
    got = heat.coarse_thomas(x, s)
    assert np.max(np.abs(got - want)) <= 1e-13 * np.max(np.abs(want))


@pytest.mark.parametrize("dim,n,s", [(2, 15, 16.42), (2, 9, 0.05), (3, 7, 0.0516), (3, 5, 40.0)])
def test_cg_vs_dense_solve(dim, n, s):
    rng = np.random.default_rng(dim * 100 + n)
    x = rng.standard_normal((n,) * dim)
    M = heat.be_matrix(dim, n, s)
    want = np.linalg.solve(M, x.ravel()).reshape(x.shape)
    got, it = heat.coarse_cg(x, s, 1e-12)
    assert it > 0
    assert np.max(np.abs(got - want)) <= 1e-10 * np.max(np.abs(want))
    # residual criterion actually met
    res = x - heat.be_apply(got, s)
    assert np.linalg.norm(res) <= 1e-12 * np.linalg.norm(x) * 1.0001


def test_be_matrix_is_the_stencil():
    # (I - s h^2 L_h): diagonal 1 + 2 d s, off-diagonals -s at grid neighbours
    M = heat.be_matrix(2, 4, 0.7)
    assert np.allclose(np.diag(M), 1 + 4 * 0.7)
    assert np.allclose(M, M.T)
    assert M[0, 1] == -0.7 and M[0, 4] == -0.7 and M[0, 5] == 0.0 and M[3, 4] == 0.0


def test_coarse_on_sine_mode():
    n, s, k = 63, 16.42, 7
    h = 1.0 / (n + 1)
    x = np.arange(1, n + 1) * h
    u = np.outer(np.sin(k * np.pi * x), np.sin(2 * np.pi * x))
    mu = 4 * math.sin(k * math.pi * h / 2) ** 2 + 4 * math.sin(2 * math.pi * h / 2) ** 2
    got, _ = heat.coarse_cg(u, s, 1e-13)
    assert np.max(np.abs(got - u / (1 + s * mu))) <= 1e-11


@pytest.mark.parametrize("dim,n,N", [(1, 31, 6), (2, 15, 5), (3, 7, 4)])
def test_spectral_serial_fine_vs_stencil_all_slices(dim, n, N):
    # the modal serial fine run against the stencil one (itself pinned to the
    # sine-mode amplification and to dense matrix powers), every slice
    rng = np.random.default_rng(40 + dim)
    u0 = rng.standard_normal((n,) * dim)
    r, m = 0.8 / (2 * dim), 11
    want = heat.serial_fine(u0, r, m, N)
    got = spectral.serial_fine(u0, r, m, N)
    assert got.shape == want.shape
    for i in range(N + 1):
        assert np.max(np.abs(got[i] - want[i])) <= 1e-13 * max(1.0, np.max(np.abs(want[i]))), i
    sub = spectral.serial_fine(u0, r, m, N, slices=[N, 0, 2])
    assert np.max(np.abs(sub - want[[N, 0, 2]])) <= 1e-13 * np.max(np.abs(want))


def test_spectral_serial_fine_heat1d_closed_form_every_slice():
    # lambda*_i of the 1D workload written out mode by mode:
    # sum_k a_k (1 - 4 r sin^2(k pi h / 2))^(i m) sin(k pi x)
    p = workloads.heat1d()
    d = _disc(p)
    x = workloads.grid(p.n)
    got = spectral.serial_fine(p.u0, d.r, d.m, d.nslices)
    for i in range(d.nslices + 1):
        want = np.zeros(p.n)
        for k, a in enumerate(p.amps, start=1):
            want += a * (1 - 4 * d.r * math.sin(k * math.pi * d.h / 2) ** 2) ** (i * d.m) * np.sin(k * np.pi * x)
        assert np.max(np.abs(got[i] - want)) <= 1e-13 * np.max(np.abs(want)), i


def test_spectral_serial_fine_anisotropic_mode():
    # a 2D mode with different wave numbers along the two axes: each slice
    # multiplies it by (1 - r (mu_kx + mu_ky))^m
    n, r, m, N = 40, 0.2, 13, 7
    h = 1.0 / (n + 1)
    x = np.arange(1, n + 1) * h
    u0 = np.outer(np.sin(3 * np.pi * x), np.sin(11 * np.pi * x))
    mu = 4 * math.sin(3 * math.pi * h / 2) ** 2 + 4 * math.sin(11 * math.pi * h / 2) ** 2
    got = spectral.serial_fine(u0, r, m, N)
    for i in range(N + 1):
        assert np.max(np.abs(got[i] - (1 - r * mu) ** (i * m) * u0)) <= 1e-13, i


def test_spectral_parareal_sync_endpoints():
    # k = 0 is the coarse sweep g^i u0 (dense solves); k >= i is the serial
    # fine value (finite termination)
    rng = np.random.default_rng(12)
    n, r, m, s, N = 6, 0.2, 9, 1.7, 5
    u0 = rng.standard_normal((n, n))
    Mg = heat.be_matrix(2, n, s)
    lam = u0.ravel()
    k0 = spectral.parareal_sync(u0, r, m, s, 0, range(N + 1))
    for i in range(N + 1):
        assert np.max(np.abs(k0[i].ravel() - lam)) <= 1e-12 * np.max(np.abs(lam)), i
        lam = np.linalg.solve(Mg, lam)
    ser = heat.serial_fine(u0, r, m, N)
    for i in range(N + 1):
        got = spectral.parareal_sync(u0, r, m, s, i, [i])[0]
        assert np.max(np.abs(got - ser[i])) <= 1e-12 * np.max(np.abs(ser[i])), i


def test_spectral_sync_change_vs_iterates_and_deltas():
    # the closed-form change of one iteration against the difference of two
    # closed-form iterates, and its max norm against the stencil/Thomas
    # oracle's recorded changes on the 1D workload
    p = workloads.heat1d()
    d = _disc(p)
    N = d.nslices
    props = heat.Propagators(d)
    res = parareal.parareal_sync(p.u0, props.F, props.G, N, eps=0.0)
    for k in (1, 2, 5, 9, 14):
        ch = spectral.parareal_sync_change(p.u0, d.r, d.m, d.s, k, range(N + 1))
        diff = (spectral.parareal_sync(p.u0, d.r, d.m, d.s, k, range(N + 1))
                - spectral.parareal_sync(p.u0, d.r, d.m, d.s, k - 1, range(N + 1)))
        assert np.max(np.abs(ch - diff)) <= 1e-14 + 1e-12 * np.max(np.abs(ch)), k
        assert not np.any(ch[:k])
        got = float(np.max(np.abs(ch)))
        assert abs(got - res.deltas[k - 1]) <= 1e-9 * res.deltas[k - 1] + 1e-15, k


def test_spectral_propagators_vs_dense():
    rng = np.random.default_rng(5)
    u = rng.standard_normal((7, 7))
    s, r, m = 3.3, 0.2, 9
    Mg = heat.be_matrix(2, 7, s)
    assert np.allclose(spectral.coarse(u, s).ravel(), np.linalg.solve(Mg, u.ravel()), atol=1e-13)
    assert np.allclose(spectral.fine(u, r, m), heat.fine(u, r, m), atol=1e-13)


# ---------------------------------------------------------------- P3/P4: synchronous Parareal

def _sync_1d(keep=True):
    p = workloads.heat1d()
    d = _disc(p)
    pr = heat.Propagators(d)
    return p, d, parareal.parareal_sync(p.u0, pr.F, pr.G, d.nslices, eps=0.0, keep_history=keep)


def test_sync_iterates_vs_binomial_closed_form():
    # every (k, slice) iterate of the 1D workload, per-mode closed form
    p, d, res = _sync_1d()
    x = workloads.grid(p.n)
    for k in range(0, d.nslices + 1):
        lam = res.history[k]
        for i in range(d.nslices + 1):
            want = np.zeros(p.n)
            for kk, a in enumerate(p.amps, start=1):
                mu = 4 * math.sin(kk * math.pi * d.h / 2) ** 2
                f = (1 - d.r * mu) ** d.m
                g = 1 / (1 + d.s * mu)
                c = sum(math.comb(i, j) * (f - g) ** j * g ** (i - j) for j in range(min(k, i) + 1))
                want += a * c * np.sin(kk * np.pi * x)
            assert np.max(np.abs(lam[i] - want)) <= 1e-12 * max(1.0, np.max(np.abs(want))), (k, i)


def test_sync_finite_termination_bitwise():
    p, d, res = _sync_1d(keep=False)
    ser = heat.serial_fine(p.u0, d.r, d.m, d.nslices)
    assert res.iters == d.nslices
    assert np.array_equal(res.lam, ser)


def test_sync_exact_slices_freeze_bitwise():
    # after iteration k, slices 0..k equal the serial fine values exactly
    p, d, res = _sync_1d()
    ser = heat.serial_fine(p.u0, d.r, d.m, d.nslices)
    for k in range(d.nslices + 1):
        assert np.array_equal(res.history[k][: k + 1], ser[: k + 1])


def test_sync_heat1d_stopping():
    p = workloads.heat1d()
    d = _disc(p)
    pr = heat.Propagators(d)
    res = parareal.parareal_sync(p.u0, pr.F, pr.G, d.nslices, eps=p.eps)
    assert res.iters == 15 and res.deltas[-1] < 1e-10 <= res.deltas[-2]
    ser = heat.serial_fine(p.u0, d.r, d.m, d.nslices)
    assert np.max(np.abs(res.lam - ser)) < 1e-11


def test_sync_2d_small_vs_spectral_and_dense_all_at_once():
    # 2D, CG coarse solve, every iterate vs the closed form with exact G
    p = workloads.heat2d(n=15, nslices=6, T=2e-2)
    d = _disc(p)
    pr = heat.Propagators(d, cg_tol=1e-13)
    res = parareal.parareal_sync(p.u0, pr.F, pr.G, d.nslices, eps=0.0, keep_history=True)
    for k in (0, 1, 2, 4, 6):
        want = spectral.parareal_sync(p.u0, d.r, d.m, d.s, k, range(d.nslices + 1))
        scale = np.max(np.abs(want))
        assert np.max(np.abs(res.history[k] - want)) <= 1e-11 * scale, k


def test_all_at_once_fixed_point():
    # Section 3.1: lambda* solves the block lower-bidiagonal system A lambda = b,
    # and Parareal is the preconditioned Richardson iteration with M
    n, dim, N, r, m, s = 5, 2, 4, 0.2, 6, 1.2
    rng = np.random.default_rng(9)
    u0 = rng.standard_normal((n,) * dim)
    Fm = np.linalg.matrix_power(heat.fine_matrix_step(dim, n, r), m)
    Gm = np.linalg.inv(heat.be_matrix(dim, n, s))
    P = n ** dim
    A = np.eye((N + 1) * P)
    Mb = np.eye((N + 1) * P)
    for i in range(1, N + 1):
        A[i * P:(i + 1) * P, (i - 1) * P:i * P] = -Fm
        Mb[i * P:(i + 1) * P, (i - 1) * P:i * P] = -Gm
    b = np.zeros((N + 1) * P)
    b[:P] = u0.ravel()
    lam_star = np.linalg.solve(A, b).reshape((N + 1,) + u0.shape)
    assert np.allclose(lam_star, heat.serial_fine(u0, r, m, N), atol=1e-12)
    # Richardson iteration lambda <- (I - M^-1 A) lambda + M^-1 b from the coarse guess
    Fp = lambda x: heat.fine(x, r, m)
    Gp = lambda x: np.linalg.solve(heat.be_matrix(dim, n, s), x.ravel()).reshape(x.shape)
    res = parareal.parareal_sync(u0, Fp, Gp, N, eps=0.0, keep_history=True)
    lam = np.linalg.solve(Mb, b)
    assert np.allclose(lam, res.history[0].ravel(), atol=1e-12)
    for k in range(1, N + 1):
        lam = lam - np.linalg.solve(Mb, A @ lam - b)
        assert np.allclose(lam, res.history[k].ravel(), atol=1e-11), k


# ---------------------------------------------------------------- P6/P7: asynchronous Parareal

def _tiny():
    # a case where alpha~ = ||G|| + ||F - G|| < 1 (infinity norm), dense G
    dim, n, r, m = 2, 5, 0.25, 32
    s = r * m
    Fm = np.linalg.matrix_power(heat.fine_matrix_step(dim, n, r), m)
    Gm = np.linalg.inv(heat.be_matrix(dim, n, s))
    Fp = lambda x: heat.fine(x, r, m)
    Gp = lambda x: np.linalg.solve(heat.be_matrix(dim, n, s), x.ravel()).reshape(x.shape)
    rng = np.random.default_rng(21)
    u0 = rng.standard_normal((n,) * dim)
    return u0, Fp, Gp, Fm, Gm, r, m


def test_async_sync_schedule_equals_sync_bitwise():
    p = workloads.heat1d()
    d = _disc(p)
    pr = heat.Propagators(d)
    sync = parareal.parareal_sync(p.u0, pr.F, pr.G, d.nslices, eps=0.0, kmax=7, keep_history=True)
    st = parareal.replay(p.u0, pr.F, pr.G, d.nslices, parareal.sync_schedule(d.nslices, 7))
    for i in range(d.nslices + 1):
        for k in range(8):
            assert np.array_equal(st.versions[i][k if i > 0 else 0], sync.history[k][i])


def test_async_stale_input_gives_fine_exactly():
    p = workloads.heat1d()
    d = _disc(p)
    pr = heat.Propagators(d)
    st = parareal.AsyncReplay(p.u0, pr.F, pr.G, d.nslices)
    st.step(3, 0)            # slice 3 reads the predecessor it already used
    assert np.array_equal(st.versions[3][-1], pr.F(st.versions[2][0]))
    st.step(2, 0)
    st.step(3, 1)            # fresh input: a genuine correction
    assert not np.array_equal(st.versions[3][-1], pr.F(st.versions[2][0]))
    st.step(3, 1)            # stale again: exactly F of that input
    assert np.array_equal(st.versions[3][-1], pr.F(st.versions[2][1]))


def test_async_per_update_error_bound():
    # proof of the asynchronous error theorem: each update obeys
    # ||l_i - l*_i|| <= ||G|| ||x_new - l*|| + ||F - G|| ||x_old - l*||
    u0, Fp, Gp, Fm, Gm, r, m = _tiny()
    N = 6
    star = heat.serial_fine(u0, r, m, N)
    nG = np.abs(Gm).sum(1).max()
    nFG = np.abs(Fm - Gm).sum(1).max()
    rng = np.random.default_rng(3)
    st = parareal.AsyncReplay(u0, Fp, Gp, N)
    for _ in range(60):
        i = int(rng.integers(1, N + 1))
        hi = st.newest(i - 1)
        j = int(rng.integers(st.f_ver[i], hi + 1))
        xo = st.versions[i - 1][st.f_ver[i]]
        xn = st.versions[i - 1][j]
        st.step(i, j)
        err = np.abs(st.versions[i][-1] - star[i]).max()
        bound = nG * np.abs(xn - star[i - 1]).max() + nFG * np.abs(xo - star[i - 1]).max()
        assert err <= bound * (1 + 1e-12) + 1e-14


@pytest.mark.parametrize("seed,delay", [(0, 0), (1, 2), (2, 5)])
def test_async_random_schedules_converge_and_terminate(seed, delay):
    p = workloads.heat1d()
    d = _disc(p)
    pr = heat.Propagators(d)
    star = heat.serial_fine(p.u0, d.r, d.m, d.nslices)
    st = parareal.run_random(p.u0, pr.F, pr.G, d.nslices, seed=seed, max_delay=delay, exact=True)
    assert st.converged_exact()
    assert np.array_equal(st.current(), star)         # finite termination, bit for bit
    sync = parareal.parareal_sync(p.u0, pr.F, pr.G, d.nslices, eps=p.eps)
    assert st.kappa >= sync.iters                     # kappa(k~) >= k (Section 4.2)
    st2 = parareal.run_random(p.u0, pr.F, pr.G, d.nslices, seed=seed, max_delay=delay, eps=p.eps)
    assert st2.converged_tol(p.eps)
    assert np.max(np.abs(st2.current() - star)) < 1e-10 * np.max(np.abs(star))


def _stale_tail_state(K):
    # 1D workload after K synchronous sweeps; slice N then re-reads the
    # predecessor version it already used until its own change is 0 (stale
    # input gives F exactly), and slices 1..N-1 make two more sweeps reading
    # their newest predecessor while slice N does not update
    p = workloads.heat1d()
    d = _disc(p)
    pr = heat.Propagators(d)
    N = d.nslices
    st = parareal.replay(p.u0, pr.F, pr.G, N, parareal.sync_schedule(N, K))
    st.step(N, st.f_ver[N])
    st.step(N, st.f_ver[N])
    for _ in range(2):
        for i in range(1, N):
            st.step(i, st.newest(i - 1))
    return st, N


def test_async_tolerance_stop_rejects_a_stale_predecessor():
    # every slice's last change is below eps, but the predecessor slice N last
    # read has moved by more than eps since: the tolerance stop must refuse
    st, N = _stale_tail_state(8)
    last = max(st.delta[1:])
    actual = float(np.max(np.abs(st.versions[N - 1][-1] - st.versions[N - 1][st.g_ver[N]])))
    eps = 2.5e-7
    assert st.delta[N] == 0.0 and last < eps <= actual
    assert min(st.k[1:]) > 0
    assert not st.converged_tol(eps)
    # the same state passes once eps exceeds the recorded drift of every input
    assert st.staleness(N) < 1e-6 and st.converged_tol(1e-6)


def test_async_tolerance_stop_accepts_small_drift_only():
    st, N = _stale_tail_state(10)
    assert max(st.delta[1:]) < 1e-8
    drift = st.staleness(N)
    assert 3e-8 < drift < 1e-7
    assert st.converged_tol(1e-7)
    assert not st.converged_tol(3e-8)      # all changes < 3e-8, drift is not
    # a slice that never updated blocks the stop whatever its recorded change
    fresh = parareal.AsyncReplay(np.ones(3), lambda x: x, lambda x: x, 2)
    fresh.step(1, 0)
    assert fresh.delta[2] == np.inf and not fresh.converged_tol(1.0)


@pytest.mark.parametrize("seed", [5, 6])
def test_async_drift_bounds_the_true_staleness(seed):
    # the recorded changes bound, by the triangle inequality, how far the
    # newest predecessor is from the one a slice last read
    p = workloads.heat2d(n=9, nslices=5, T=2e-2)
    d = _disc(p)
    pr = heat.Propagators(d, cg_tol=1e-13)
    rng = np.random.default_rng(seed)
    st = parareal.AsyncReplay(p.u0, pr.F, pr.G, d.nslices)
    for _ in range(80):
        i = int(rng.integers(1, d.nslices + 1))
        hi = st.newest(i - 1)
        st.step(i, int(rng.integers(max(st.f_ver[i], hi - 3), hi + 1)))
        for s in range(2, d.nslices + 1):
            if st.g_ver[s] < 0:
                continue
            true = float(np.max(np.abs(st.versions[s - 1][-1] - st.versions[s - 1][st.g_ver[s]])))
            assert true <= st.staleness(s) * (1 + 1e-12) + 1e-300


@pytest.mark.parametrize("seed", [0, 3])
def test_async_resets_still_reach_the_fixed_point(seed):
    # slices that lose their state mid-run (start again from the initial
    # guess) perturb the iteration once; the fair, bounded-delay schedule still
    # reaches the serial fine solution bit for bit (finite termination), and
    # the tolerance stop still lands within the bar
    p = workloads.heat1d()
    d = _disc(p)
    pr = heat.Propagators(d)
    star = heat.serial_fine(p.u0, d.r, d.m, d.nslices)
    resets = {3: 4, 7: 9, 12: 15, 16: 2}
    st = parareal.run_random(p.u0, pr.F, pr.G, d.nslices, seed=seed, max_delay=2, exact=True, resets=resets)
    assert st.converged_exact()
    assert np.array_equal(st.current(), star)
    st2 = parareal.run_random(p.u0, pr.F, pr.G, d.nslices, seed=seed, max_delay=2, eps=p.eps, resets=resets)
    assert st2.converged_tol(p.eps)
    assert np.max(np.abs(st2.current() - star)) < 1e-10 * np.max(np.abs(star))


def test_async_reset_restarts_from_the_initial_guess():
    # after a reset the next update is exactly the first update of Algorithm 2
    # with the newest predecessor as coarse input: F(lambda_{i-1}^0) +
    # G(x_new) - lambda_i^0
    p = workloads.heat1d()
    d = _disc(p)
    pr = heat.Propagators(d)
    st = parareal.replay(p.u0, pr.F, pr.G, d.nslices, parareal.sync_schedule(d.nslices, 5))
    st.reset(4)
    assert st.final_from[4] == -1 and st.final_from[9] == -1 and st.final_from[3] >= 0
    j = st.newest(3)
    st.step(4, j)
    want = pr.F(st.versions[3][0]) + (pr.G(st.versions[3][j]) - st.versions[4][0])
    assert np.array_equal(st.versions[4][-1], want)


def test_async_contraction_when_alpha_below_one():
    u0, Fp, Gp, Fm, Gm, r, m = _tiny()
    N = 8
    at = np.abs(Gm).sum(1).max() + np.abs(Fm - Gm).sum(1).max()
    assert at < 1
    star = heat.serial_fine(u0, r, m, N)
    st = parareal.run_random(u0, Fp, Gp, N, seed=4, max_delay=2, max_rounds=3)
    e3 = np.abs(st.current() - star).max()
    e0 = np.abs(parareal.coarse_sweep(u0, Gp, N) - star).max()
    assert e3 < e0


def test_sync_error_theorem_bound():
    # Theorem on synchronous error: ||l^k - l*|| <= alpha^k ||l^0 - l*||
    u0, Fp, Gp, Fm, Gm, r, m = _tiny()
    N = 8
    th = np.abs(Gm).sum(1).max()
    alpha = (1 - th ** N) / (1 - th) * np.abs(Fm - Gm).sum(1).max()
    star = heat.serial_fine(u0, r, m, N)
    res = parareal.parareal_sync(u0, Fp, Gp, N, eps=0.0, keep_history=True)
    e0 = np.abs(res.history[0] - star).max()
    for k in range(1, N + 1):
        assert np.abs(res.history[k] - star).max() <= alpha ** k * e0 * (1 + 1e-9) + 1e-15


# ---------------------------------------------------------------- P8: gradients

def test_gradient_closed_form_vs_reverse_and_fd():
    p = workloads.adjoint2d(n=15, nslices=4, T=2e-2)
    d = _disc(p)
    M = d.m * d.nslices
    g0, gnu = adjoint.grad_closed_form(p.u0, p.target, d.r, M, d.dt, d.h)
    g1, gnu1 = adjoint.grad_reverse(p.u0, p.target, d.r, M, d.dt, d.h)
    assert np.max(np.abs(g0 - g1)) <= 1e-12 * np.max(np.abs(g0))
    assert abs(gnu - gnu1) <= 1e-10 * abs(gnu)

    def L_of(u0, nu):
        r = nu * d.dt / d.h ** 2
        return adjoint.loss(heat.fine(u0, r, M), p.target)

    e = 1e-6
    fd_nu = (L_of(p.u0, p.nu + e) - L_of(p.u0, p.nu - e)) / (2 * e)
    L0 = L_of(p.u0, p.nu)
    assert abs(fd_nu - gnu) <= 1e-6 * abs(gnu) + 10 * 2.2e-16 * abs(L0) / e
    rng = np.random.default_rng(4)
    for _ in range(4):
        dirn = rng.standard_normal(p.u0.shape)
        dirn /= np.linalg.norm(dirn)
        fd = (L_of(p.u0 + e * dirn, p.nu) - L_of(p.u0 - e * dirn, p.nu)) / (2 * e)
        assert abs(fd - float(np.vdot(g0, dirn))) <= 1e-6 * np.linalg.norm(g0) + 10 * 2.2e-16 * abs(L0) / e


def test_gradient_vs_dense_transpose():
    n, dim, r, M = 4, 2, 0.2, 13
    rng = np.random.default_rng(8)
    u0 = rng.standard_normal((n, n))
    tgt = rng.standard_normal((n, n))
    A = heat.fine_matrix_step(dim, n, r)
    AM = np.linalg.matrix_power(A, M)
    g = AM @ u0.ravel() - tgt.ravel()
    want = AM.T @ g
    got, _ = adjoint.grad_reverse(u0, tgt, r, M, 1e-3, 1 / (n + 1))
    assert np.allclose(got.ravel(), want, atol=1e-13)


def test_golden_heat1d_regression():
    # stored by tests/golden/make_golden.py from this oracle; guards later edits
    import json, os
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "heat1d_sync.json")))
    p = workloads.heat1d()
    d = _disc(p)
    pr = heat.Propagators(d)
    res = parareal.parareal_sync(p.u0, pr.F, pr.G, d.nslices, eps=p.eps)
    assert res.iters == g["sync_iters"] == 15
    assert np.array_equal(res.lam[-1], np.array(g["sync_lambda_N"]))
    assert np.array_equal(heat.serial_fine(p.u0, d.r, d.m, d.nslices)[-1], np.array(g["serial_fine_uT"]))
