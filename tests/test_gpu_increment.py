"""Coarse solves on the change of their input (G is linear, Section 3.1):
same fixed point, same finite termination, iterates within the CG tolerance
of the literal G(new) - G(old) form the oracle computes."""
import numpy as np
import pytest

import workloads
from oracle import heat, parareal

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2110_10762_amd as pr  # noqa: E402

DEV = "cuda:0"


def rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def disc_of(p):
    return heat.discretise(p.dim, p.n, p.nu, p.T, p.nslices, p.dt_nominal)


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def sync(p, incr, eps=None, kmax=0):
    prob = pr.Problem(pr.config_of(p, eps=p.eps if eps is None else eps, kmax=kmax, coarse_increment=incr))
    lam = torch.empty((p.nslices + 1,) + p.u0.shape, dtype=torch.float64, device=DEV)
    st = pr.Stats(p.nslices, p.nslices + 1)
    prob.solve_sync(dev(p.u0), lam, st, allow_notconv=True)
    return prob, lam.cpu().numpy(), st


@pytest.mark.parametrize("which", ["1d", "2d", "3d"])
def test_sync_increment_vs_oracle(which):
    if which == "1d":
        p = workloads.heat1d()
    elif which == "2d":
        p = workloads.heat2d(n=70, nslices=8, T=1e-2)
    else:
        p = workloads.heat3d(n=20, nslices=6, T=4e-3)
    d = disc_of(p)
    props = heat.Propagators(d, cg_tol=p.cg_tol)
    ref = parareal.parareal_sync(p.u0, props.F, props.G, d.nslices, eps=p.eps)
    _, lam, st = sync(p, 1)
    assert st.iters == ref.iters
    assert rel(lam, ref.lam) <= 1e-10
    for k in (1, 3):
        refk = parareal.parareal_sync(p.u0, props.F, props.G, d.nslices, eps=0.0, kmax=k)
        _, lamk, _ = sync(p, 1, eps=0.0, kmax=k)
        assert rel(lamk, refk.lam) <= 1e-10


def test_sync_increment_finite_termination_bitwise():
    for p in (workloads.heat1d(), workloads.heat2d(n=40, nslices=5, T=2e-2)):
        prob, lam, st = sync(p, 1, eps=0.0)
        ser = torch.empty_like(dev(lam))
        prob.solve_fine(dev(p.u0), ser)
        assert np.array_equal(lam, ser.cpu().numpy())


def test_async_increment_modes():
    p = workloads.heat2d(n=64, nslices=8, T=1e-2)
    d = disc_of(p)
    star = heat.serial_fine(p.u0, d.r, d.m, d.nslices)
    for mode in (pr.PR_ASYNC_FREE, pr.PR_ASYNC_EXACT):
        prob = pr.Problem(pr.config_of(p, coarse_increment=1))
        prob.set_async_options(mode=mode, time_limit_s=30.0)
        lam = torch.empty((p.nslices + 1,) + p.u0.shape, dtype=torch.float64, device=DEV)
        st = pr.Stats(p.nslices)
        prob.solve_async(dev(p.u0), lam, st)
        assert st.converged == 1
        if mode == pr.PR_ASYNC_EXACT:
            ser = torch.empty_like(lam)
            prob.solve_fine(dev(p.u0), ser)
            assert torch.equal(lam, ser)
        else:
            assert rel(lam.cpu().numpy(), star) <= 1e-10


def test_async_replay_of_sync_schedule_equals_sync_increment_1d():
    p = workloads.heat1d()
    N, K = p.nslices, 5
    rows = [[] for _ in range(N + 1)]
    for i, j in parareal.sync_schedule(N, K):
        rows[i].append(j)
    sched = []
    for i in range(1, N + 1):
        sched += rows[i] + [-1] * (K - len(rows[i]))
    prob = pr.Problem(pr.config_of(p, coarse_increment=1))
    prob.set_async_options(mode=pr.PR_ASYNC_REPLAY, max_local_iters=K, schedule=sched, time_limit_s=30.0)
    lam = torch.empty((N + 1, p.n), dtype=torch.float64, device=DEV)
    prob.solve_async(dev(p.u0), lam)
    _, ls, _ = sync(p, 1, eps=0.0, kmax=K)
    assert np.array_equal(lam.cpu().numpy(), ls)


def test_batched_increment_matches_literal():
    probs = workloads.batched(count=10, sides=(32, 64), max_slices=9)
    outs = []
    for incr in (0, 1):
        h = pr.Problem([pr.config_of(q, coarse_increment=incr) for q in probs])
        u0 = dev(np.concatenate([q.u0.ravel() for q in probs]))
        lam = torch.empty(sum((q.nslices + 1) * q.n * q.n for q in probs), dtype=torch.float64, device=DEV)
        _, st = h.solve_batch(u0, lam)
        outs.append((lam.cpu().numpy(), [s.iters for s in st]))
    assert outs[0][1] == outs[1][1]
    assert rel(outs[1][0], outs[0][0]) <= 1e-10
