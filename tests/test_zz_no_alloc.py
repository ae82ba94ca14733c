"""The allocation-free coarse propagator, called through the C ABI, against
the handle-based pr_apply_coarse (same solver, same launch: same bits) and
the oracle's textbook CG; two calls in a row, the second on a smaller input,
so the second must not depend on what the first left in the shared array."""
import ctypes

import numpy as np
import pytest

from oracle import heat

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2110_10762_amd as pr  # noqa: E402

DEV = "cuda:0"


def rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def static_apply(cfg, x, y, count):
    lib = pr.load_library()
    its = ctypes.c_longlong()
    stream = torch.cuda.current_stream().cuda_stream
    rc = lib.pr_apply_coarse_static(ctypes.byref(cfg), 0, ctypes.c_void_p(stream),
                                    ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                                    count, ctypes.byref(its))
    return rc, its.value


def handle_apply(cfg, x, count):
    prob = pr.Problem(cfg)
    y = torch.empty_like(x)
    its = prob.apply_coarse(x, y, count)
    prob.close()
    return y, its


@pytest.mark.parametrize("dim,sizes", [(2, [(1024, 3), (130, 2)]), (3, [(101, 2), (40, 1)])])
def test_static_coarse_matches_handle_and_oracle(dim, sizes):
    rng = np.random.default_rng(500 + dim)
    for n, count in sizes:      # the second call is smaller than the first
        print(f"static coarse apply: dim={dim} n={n} count={count}", flush=True)
        T = 1e-3 if dim == 2 else 2e-4
        cfg = pr.make_config(dim, n, 1.0, T, 4, 0.2 / (n + 1) ** 2 / dim)
        xs = rng.standard_normal((count,) + (n,) * dim)
        x = torch.from_numpy(xs).to(DEV)
        y = torch.full_like(x, np.nan)
        rc, its = static_apply(cfg, x, y, count)
        assert rc == pr.PR_OK, pr.load_library().pr_last_error().decode()
        want, its_h = handle_apply(cfg, x, count)
        assert its == its_h
        assert torch.equal(y, want)
        got = y.cpu().numpy()
        s = pr.Problem(cfg).info().s
        for c in range(min(count, 1 if n > 200 else count)):
            ref, _ = heat.coarse_cg(xs[c], s, 1e-12)
            assert rel(got[c], ref) <= 1e-10


def test_static_coarse_rejects_what_it_cannot_hold():
    lib = pr.load_library()
    x = torch.zeros(8, dtype=torch.float64, device=DEV)
    y = torch.zeros(8, dtype=torch.float64, device=DEV)
    its = ctypes.c_longlong()
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    big = pr.make_config(2, 1025, 1.0, 1e-3, 4, 0.2 / 1026 ** 2)      # 1025^2 > 2^20 points
    rc = lib.pr_apply_coarse_static(ctypes.byref(big), 0, stream, ctypes.c_void_p(x.data_ptr()),
                                    ctypes.c_void_p(y.data_ptr()), 1, ctypes.byref(its))
    assert rc == pr.PR_EINVAL and b"exceeds" in lib.pr_last_error()
    one_d = pr.make_config(1, 8, 1.0, 0.1, 4, 0.4 / 81)
    rc = lib.pr_apply_coarse_static(ctypes.byref(one_d), 0, stream, ctypes.c_void_p(x.data_ptr()),
                                    ctypes.c_void_p(y.data_ptr()), 1, ctypes.byref(its))
    assert rc == pr.PR_EINVAL
    ok = pr.make_config(2, 2, 1.0, 1e-3, 4, 0.2 / 9)
    rc = lib.pr_apply_coarse_static(ctypes.byref(ok), 0, stream, ctypes.c_void_p(x.data_ptr()),
                                    ctypes.c_void_p(x.data_ptr()), 1, ctypes.byref(its))
    assert rc == pr.PR_EINVAL     # aliasing
