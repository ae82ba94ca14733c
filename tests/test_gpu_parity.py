"""GPU-vs-oracle parity of the HIP library, called through the C ABI.

Tolerance: the FP64 results must match the oracle within 1e-10 relative in
the max norm (the workloads' stated bar); the fine propagator alone matches
to ~1e-13 and is checked tighter.
"""
import math

import numpy as np
import pytest

import workloads
from oracle import heat, parareal, spectral

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2110_10762_amd as pr  # noqa: E402

DEV = "cuda:0"
TOL = 1e-10


def rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def disc_of(p):
    return heat.discretise(p.dim, p.n, p.nu, p.T, p.nslices, p.dt_nominal)


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def states(rng, count, shape):
    return rng.standard_normal((count,) + shape)


# ------------------------------------------------------------------ fine propagator

@pytest.mark.parametrize("n,steps", [(127, 256), (5, 3), (64, 100), (1000, 40)])
def test_fine_1d(n, steps):
    rng = np.random.default_rng(n)
    x = states(rng, 3, (n,))
    prob = pr.Problem(pr.make_config(1, n, 1.0, 1.0, 2, 0.4 / (n + 1) ** 2))
    r = prob.info().r
    y = torch.empty_like(dev(x))
    prob.apply_fine(dev(x), y, 3, steps)
    got = y.cpu().numpy()
    for c in range(3):
        assert rel(got[c], heat.fine(x[c], r, steps)) <= 1e-12


# n >= 64 XP: strips flush with both boundaries (one strip at n = 128 for
# XP = 2, two up to 240, then interior strips); smaller n: odd extension
@pytest.mark.parametrize("n", [63, 100, 1, 128, 129, 240, 241, 300])
def test_fine_2d_all_shapes_bitwise_and_vs_oracle(n):
    rng = np.random.default_rng(7 + n)
    cnt = 3
    x = states(rng, cnt, (n, n))
    prob = pr.Problem(pr.make_config(2, n, 1.0, 1.0, cnt, 0.2 / (n + 1) ** 2))
    r = prob.info().r
    steps = 19
    want = [heat.fine(x[c], r, steps) for c in range(cnt)]
    ref_bits = None
    for (d, rows, xp, sw) in pr.fine_shapes(2):
        prob.set_fine_shape(d, rows, xp)
        y = torch.empty_like(dev(x))
        prob.apply_fine(dev(x), y, cnt, steps)
        got = y.cpu().numpy()
        for c in range(cnt):
            assert rel(got[c], want[c]) <= 1e-12, (d, rows, xp)
        if ref_bits is None:
            ref_bits = got
        else:   # every kernel shape evaluates the same per-point formula
            assert np.array_equal(got, ref_bits), (d, rows, xp)


def test_fine_3d_depth_shapes_wide():
    # the z-marching kernels of depth 2-4 at a size of several x strips (n =
    # 130 > 64 - 2D), y strips and z segments, with a step count no depth
    # divides: against the oracle and bit for bit against one step per pass
    n, steps = 130, 9
    rng = np.random.default_rng(17)
    x = states(rng, 2, (n, n, n))
    prob = pr.Problem(pr.make_config(3, n, 0.5, 1.0, 2, 0.15 / (n + 1) ** 2))
    r = prob.info().r
    want = [heat.fine(x[c], r, steps) for c in range(2)]
    outs = {}
    for (d, rows, xp, sw) in pr.fine_shapes(3):
        prob.set_fine_shape(d, rows, xp)
        y = torch.empty_like(dev(x))
        prob.apply_fine(dev(x), y, 2, steps)
        outs[(d, rows, xp)] = y.cpu().numpy()
    depths = sorted({k[0] for k in outs})
    assert depths[0] == 1 and depths[-1] >= 4
    ref = outs[[k for k in outs if k[0] == 1][0]]
    for k, got in outs.items():
        for c in range(2):
            assert rel(got[c], want[c]) <= 1e-12, k
        assert np.array_equal(got, ref), k


@pytest.mark.parametrize("n", [31, 40, 2])
def test_fine_3d_all_shapes(n):
    rng = np.random.default_rng(3 + n)
    x = states(rng, 2, (n, n, n))
    prob = pr.Problem(pr.make_config(3, n, 0.5, 1.0, 2, 0.15 / (n + 1) ** 2))
    r = prob.info().r
    steps = 5
    want = [heat.fine(x[c], r, steps) for c in range(2)]
    ref_bits = None
    for (d, rows, xp, sw) in pr.fine_shapes(3):
        prob.set_fine_shape(d, rows, xp)
        y = torch.empty_like(dev(x))
        prob.apply_fine(dev(x), y, 2, steps)
        got = y.cpu().numpy()
        for c in range(2):
            assert rel(got[c], want[c]) <= 1e-12, (rows, xp)
        if ref_bits is None:
            ref_bits = got
        else:
            assert np.array_equal(got, ref_bits)


def test_fine_2d_full_size_sampled():
    # full 2D workload size, one slice, vs the exact modal form
    p = workloads.heat2d()
    d = disc_of(p)
    prob = pr.Problem(pr.config_of(p))
    x = dev(p.u0)
    y = torch.empty_like(x)
    prob.apply_fine(x, y, 1, d.m)
    want = spectral.fine(p.u0, d.r, d.m)
    assert rel(y.cpu().numpy(), want) <= 1e-12


# ------------------------------------------------------------------ coarse propagator

@pytest.mark.parametrize("n,s_scale", [(127, 1.0), (31, 1.0), (2000, 1.0), (1, 1.0)])
def test_coarse_thomas(n, s_scale):
    rng = np.random.default_rng(n)
    x = states(rng, 4, (n,))
    prob = pr.Problem(pr.make_config(1, n, 1.0, 0.1, 16, 0.4 / (n + 1) ** 2))
    s = prob.info().s
    y = torch.empty_like(dev(x))
    prob.apply_coarse(dev(x), y, 4)
    got = y.cpu().numpy()
    for c in range(4):
        # scan order differs from sequential elimination; cond ~ 4s here
        assert rel(got[c], heat.coarse_thomas(x[c], s)) <= 1e-11


@pytest.mark.parametrize("dim,n", [(2, 63), (2, 130), (3, 24), (3, 1)])
def test_coarse_cg(dim, n):
    rng = np.random.default_rng(dim * 1000 + n)
    x = states(rng, 2, (n,) * dim)
    T = 1e-3 if dim == 2 else 2e-4
    prob = pr.Problem(pr.make_config(dim, n, 1.0, T, 4, 0.2 / (n + 1) ** 2 / dim))
    s = prob.info().s
    y = torch.empty_like(dev(x))
    its = prob.apply_coarse(dev(x), y, 2)
    got = y.cpu().numpy()
    for c in range(2):
        want, it = heat.coarse_cg(x[c], s, 1e-12)
        assert rel(got[c], want) <= TOL
        exact = spectral.coarse(x[c], s)
        assert rel(got[c], exact) <= 1e-10
    assert its > 0


@pytest.mark.parametrize("n", [1, 2, 3, 10, 53, 54, 55, 64, 65, 108, 109, 130])
def test_coarse_pcg_vs_plain_and_oracle(n):
    # the preconditioned CG (default in 2D) on ragged grids: strip borders at
    # multiples of 54 columns, segments of 16 rows, a grid smaller than the
    # halo (n <= 5); against the oracle's textbook CG, the exact G and the
    # unpreconditioned GPU solver
    rng = np.random.default_rng(4000 + n)
    x = states(rng, 2, (n, n))
    cfg = dict(dim=2, n=n, nu=1.0, T=1e-3, nslices=4, dt_nominal=0.1 / (n + 1) ** 2)
    pcg = pr.Problem(pr.make_config(**cfg))
    plain = pr.Problem(pr.make_config(**cfg, cg_precond=-1))
    s = pcg.info().s
    y = torch.empty_like(dev(x))
    y0 = torch.empty_like(dev(x))
    its = pcg.apply_coarse(dev(x), y, 2)
    its0 = plain.apply_coarse(dev(x), y0, 2)
    got, got0 = y.cpu().numpy(), y0.cpu().numpy()
    for c in range(2):
        want, _ = heat.coarse_cg(x[c], s, 1e-12)
        assert rel(got[c], want) <= TOL, c
        assert rel(got[c], spectral.coarse(x[c], s)) <= TOL, c
        assert rel(got[c], got0[c]) <= TOL, c
    assert its <= its0


def test_coarse_pcg_iterations_full_size():
    # 1024^2, s = 16.4: the polynomial preconditioner cuts the CG iterations
    # by more than 3x (condition number ~132 -> ~6)
    p = workloads.heat2d()
    d = disc_of(p)
    x = dev(p.u0)
    y = torch.empty_like(x)
    y0 = torch.empty_like(x)
    its = pr.Problem(pr.config_of(p)).apply_coarse(x, y, 1)
    its0 = pr.Problem(pr.config_of(p, cg_precond=-1)).apply_coarse(x, y0, 1)
    print(f"1024^2 coarse solve: {its} preconditioned vs {its0} plain CG iterations", flush=True)
    assert 3 * its < its0
    exact = spectral.coarse(p.u0, d.s)
    assert rel(y.cpu().numpy(), exact) <= TOL
    assert rel(y0.cpu().numpy(), exact) <= TOL


def test_pcg_rejects_unsupported_degree():
    with pytest.raises(pr.PRError) as e:
        pr.Problem(pr.make_config(2, 16, 1.0, 1e-3, 4, 1e-5, cg_precond=3))
    assert e.value.code == pr.PR_EINVAL


# ------------------------------------------------------------------ synchronous Parareal

def run_sync(p, eps=None, kmax=0, **over):
    prob = pr.Problem(pr.config_of(p, eps=p.eps if eps is None else eps, kmax=kmax, **over))
    lam = torch.empty((p.nslices + 1,) + p.u0.shape, dtype=torch.float64, device=DEV)
    st = pr.Stats(p.nslices, p.nslices + 1)
    prob.solve_sync(dev(p.u0), lam, st, allow_notconv=True)
    return prob, lam.cpu().numpy(), st


def test_sync_heat1d_vs_oracle_and_golden():
    import json, os
    p = workloads.heat1d()
    _, lam, st = run_sync(p)
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "heat1d_sync.json")))
    assert st.iters == g["sync_iters"] == 15
    assert st.converged == 1
    assert rel(lam[-1], np.array(g["sync_lambda_N"])) <= TOL
    for k, (a, b) in enumerate(zip(st.deltas, g["sync_deltas"])):
        assert abs(a - b) <= 1e-10 * max(abs(b), 1e-3) + 1e-14, k


@pytest.mark.parametrize("k", [1, 2, 3, 7])
def test_sync_fixed_iterations_1d(k):
    p = workloads.heat1d()
    d = disc_of(p)
    _, lam, st = run_sync(p, eps=0.0, kmax=k)
    props = heat.Propagators(d)
    ref = parareal.parareal_sync(p.u0, props.F, props.G, d.nslices, eps=0.0, kmax=k)
    assert st.iters == k
    assert rel(lam, ref.lam) <= TOL
    for a, b in zip(st.deltas, ref.deltas):
        assert abs(a - b) <= 1e-10 * b + 1e-15


def test_sync_finite_termination_bitwise_gpu():
    # lambda^N == the GPU serial fine solution, bit for bit (1D and 2D)
    for p in (workloads.heat1d(), workloads.heat2d(n=40, nslices=5, T=2e-2)):
        prob, lam, st = run_sync(p, eps=0.0)
        assert st.iters == p.nslices
        ser = torch.empty((p.nslices + 1,) + p.u0.shape, dtype=torch.float64, device=DEV)
        prob.solve_fine(dev(p.u0), ser)
        assert np.array_equal(lam, ser.cpu().numpy())
        d = disc_of(p)
        assert rel(lam, heat.serial_fine(p.u0, d.r, d.m, d.nslices)) <= 1e-12


# n = 70 and 130: two and three column strips of the coarse solver, the last
# one ragged
@pytest.mark.parametrize("precond", [0, -1])
@pytest.mark.parametrize("n,N,T", [(31, 8, 2e-2), (70, 6, 5e-3), (130, 5, 5e-3)])
def test_sync_2d_vs_oracle(n, N, T, precond):
    p = workloads.heat2d(n=n, nslices=N, T=T)
    d = disc_of(p)
    _, lam, st = run_sync(p, cg_precond=precond)
    props = heat.Propagators(d, cg_tol=p.cg_tol)
    ref = parareal.parareal_sync(p.u0, props.F, props.G, d.nslices, eps=p.eps)
    assert st.iters == ref.iters
    assert rel(lam, ref.lam) <= TOL
    assert rel(lam[-1], ref.lam[-1]) <= TOL


def test_sync_3d_small_vs_oracle():
    p = workloads.heat3d(n=20, nslices=6, T=4e-3)
    d = disc_of(p)
    _, lam, st = run_sync(p, eps=0.0, kmax=3)
    props = heat.Propagators(d, cg_tol=p.cg_tol)
    ref = parareal.parareal_sync(p.u0, props.F, props.G, d.nslices, eps=0.0, kmax=3)
    assert rel(lam, ref.lam) <= TOL


def test_sync_3d_ragged_vs_oracle():
    # n = 70: two x-strips per row (the marching CG phases cross a strip
    # border), the second one ragged
    p = workloads.heat3d(n=70, nslices=3, T=2e-3)
    d = disc_of(p)
    _, lam, st = run_sync(p, eps=0.0, kmax=2)
    props = heat.Propagators(d, cg_tol=p.cg_tol)
    ref = parareal.parareal_sync(p.u0, props.F, props.G, d.nslices, eps=0.0, kmax=2)
    assert rel(lam, ref.lam) <= TOL


def test_serial_fine_2d_vs_spectral():
    p = workloads.heat2d(n=255, nslices=4, T=2e-4)
    d = disc_of(p)
    prob = pr.Problem(pr.config_of(p))
    lam = torch.empty((p.nslices + 1,) + p.u0.shape, dtype=torch.float64, device=DEV)
    prob.solve_fine(dev(p.u0), lam)
    want = spectral.serial_fine(p.u0, d.r, d.m, d.nslices)
    assert rel(lam.cpu().numpy(), want) <= 1e-12


# ------------------------------------------------------------------ errors through the ABI

def test_abi_errors():
    with pytest.raises(pr.PRError) as e:
        pr.Problem(pr.make_config(4, 10, 1.0, 1.0, 2, 1e-3))
    assert e.value.code == pr.PR_EINVAL
    with pytest.raises(pr.PRError) as e:
        pr.Problem(pr.make_config(2, 10, 1.0, 1.0, 2, 1.0))     # r >> 1/4
    assert e.value.code == pr.PR_EUNSTABLE
    with pytest.raises(pr.PRError) as e:
        pr.Problem(pr.make_config(2, 10, -1.0, 1.0, 2, 1e-4))
    assert e.value.code == pr.PR_EINVAL
    prob = pr.Problem(pr.make_config(1, 10, 1.0, 1.0, 2, 1e-3))
    with pytest.raises(pr.PRError):
        prob.solve_sync(0, 0)
    # buffers of the wrong size never reach a kernel
    u0 = torch.zeros(10, dtype=torch.float64, device=DEV)
    lam = torch.zeros(3 * 10, dtype=torch.float64, device=DEV)
    with pytest.raises(ValueError):
        prob.solve_sync(u0[:9], lam)
    with pytest.raises(ValueError):
        prob.solve_sync(u0, lam[:29])
    with pytest.raises(ValueError):
        prob.apply_fine(u0, lam, 2)
    prob.solve_sync(u0, lam)
    prob.apply_fine(lam, lam.clone(), 3)
    prob.close()
    prob.close()
