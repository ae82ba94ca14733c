"""Benchmark: fine-stencil GLUPS + % HBM roofline; async vs sync Parareal
time to 1e-10, on the 2D heat workload (1024^2 interior points, 64 slices,
nu = 1, T = 1e-3, fine dt = 0.2 h^2 -> 83 explicit-Euler steps per slice,
backward-Euler coarse step solved by CG to 1e-12).

One step = one synchronous and one asynchronous Parareal solve of that
workload to ||lambda^k - lambda^{k-1}||_inf < 1e-10, both starting from u0
already resident in HBM (the whole hot path: coarse sweep, fine propagation
of every slice, coarse solves, fused correction + change norm, and the two
drivers).  `value` = fine-stencil GLUPS: the lattice-site updates of the
fine-propagator launches inside the timed synchronous solves over those
launches' own duration (device events around each launch); the whole step's
rate (all fine updates of both solves over the wall time of the timed steps)
is reported beside it.

Untimed extras (outside the timed region, skipped with --no-extras): the 2D
fine sweep at every sliding-window depth D, the 3D workload (256^3, 128
slices), a supplementary 3D case with slices of 100 fine steps (128^3, 64
slices), the 512-problem batch (hipGraph, autotuned fine kernel) and the
adjoint gradient (512^2, 32 slices), each compared at sampled outputs with the
library's own serial fine integration (their agreement with the oracle is
checked by the GPU tests).

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-extras]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, published
ASYNC_DEPTH = 12        # fine steps per pass inside the persistent asynchronous kernel (2D)

# Bytes per launch moved between L2 and the memory fabric, from two rocprofv3
# --pmc runs (FETCH_SIZE scaled by 1.994, WRITE_SIZE by 1.000: the factors a
# plain copy of known size gives), kept in profiles/.  They describe the
# kernel sources whose code (comments aside) has this digest and are reported
# as null once that code changes.
PROFILED_SOURCES = "2a4660fdd90cacf5"
PROFILED_TRAFFIC = {"async": 390.40 + 258.26,      # GB, one launch
                    "fine": 0.4954 + 0.4745,       # GB, mean over the sync solve's passes
                    "sweep": 17.191 + 11.129}      # GB, mean over the sync solve's sweeps


def sources_digest():
    """Digest of the kernel sources' code (comments and blank space dropped)."""
    import glob
    import hashlib
    import re
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_2110_10762_amd", "csrc", "*"))):
        with open(f) as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()[:16]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-slices", type=int, default=96)
    ap.add_argument("--only", choices=["both", "sync", "async"], default="both",
                    help="restrict the step to one driver (profiling runs)")
    ap.add_argument("--no-pipelined", action="store_true",
                    help="skip the untimed pipelined synchronous solve (Algorithm 1)")
    ap.add_argument("--no-increment", action="store_true",
                    help="skip the untimed runs with coarse solves on input changes")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the untimed 3D, batched and adjoint runs")
    ap.add_argument("--extras-only", action="store_true",
                    help="run only the untimed 3D, batched and adjoint runs and print them "
                         "(profiling of those kernels); no benchmark line")
    return ap.parse_args()


def cpu_info():
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    return model, os.cpu_count() or 1, avail


def _fine_worker(args):
    """One process of the multi-core oracle leg: the oracle's F on one slice."""
    import numpy as np
    from oracle import heat
    u, r, m = args
    t = time.perf_counter()
    heat.fine(np.asarray(u), r, m)
    return time.perf_counter() - t


def cpu_baseline(p, nslices_sample):
    """The oracle on the host cores, on bounded samples of the workloads:
    (1) its fine propagator F, single core, over `nslices_sample` slices of
    83 explicit-Euler steps on the 1024^2 grid; (2) the same F on independent
    slice states spread over the host cores (one process per slice, as the F
    sweep of synchronous Parareal is spread); (3) its synchronous Parareal
    solve of the 1D workload (n = 127, 16 slices) to 1e-10, single core."""
    import multiprocessing as mp
    import numpy as np
    import workloads
    from oracle import heat, parareal
    model, ncpu, avail = cpu_info()
    d = heat.discretise(p.dim, p.n, p.nu, p.T, p.nslices, p.dt_nominal)
    u = p.u0.copy()
    t = time.perf_counter()
    for _ in range(nslices_sample):
        u = heat.fine(u, d.r, d.m)
    dt = time.perf_counter() - t
    lups = nslices_sample * d.m * p.n * p.n
    out = {"value": lups / dt / 1e9, "unit": "GLUPS", "cores": 1, "kind": "oracle",
           "sample": f"oracle fine propagator F over {nslices_sample} slices of the workload "
                     f"({nslices_sample}x{d.m} explicit-Euler steps on the 1024^2 grid), "
                     f"{dt:.1f} s, single-threaded NumPy",
           "cpu_model": model, "nproc": ncpu, "cores_available": avail}
    # (2) multi-core: one process per slice state, all cores busy
    procs = max(1, min(avail, 16))
    states = 8 * procs
    env_keep = {k: os.environ.get(k) for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")}
    for k in env_keep:
        os.environ[k] = "1"
    try:
        ctx = mp.get_context("spawn")
        with ctx.Pool(procs) as pool:
            pool.map(_fine_worker, [(p.u0, d.r, 1)] * procs)       # start-up outside the timing
            t = time.perf_counter()
            pool.map(_fine_worker, [(p.u0, d.r, d.m)] * states)
            dtm = time.perf_counter() - t
    finally:
        for k, v in env_keep.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    out["multicore"] = {"value": states * d.m * p.n * p.n / dtm / 1e9, "unit": "GLUPS", "cores": procs,
                        "kind": "oracle",
                        "sample": f"oracle F on {states} independent slice states of the 1024^2 workload "
                                  f"({d.m} steps each) in {procs} processes, {dtm:.1f} s"}
    # (3) the oracle's synchronous Parareal time to 1e-10 on the 1D workload
    p1 = workloads.heat1d()
    d1 = heat.discretise(p1.dim, p1.n, p1.nu, p1.T, p1.nslices, p1.dt_nominal)
    props = heat.Propagators(d1)
    t = time.perf_counter()
    res = parareal.parareal_sync(p1.u0, props.F, props.G, d1.nslices, eps=1e-10)
    t1 = time.perf_counter() - t
    t = time.perf_counter()
    heat.serial_fine(p1.u0, d1.r, d1.m, d1.nslices)
    t2 = time.perf_counter() - t
    out["heat1d_time_to_tol"] = {"sync_s": t1, "k": res.iters, "serial_fine_s": t2, "cores": 1,
                                 "kind": "oracle", "sample": "the whole 1D workload (n = 127, N = 16)"}
    return out


def run_extras(dev):
    """Untimed runs: the 2D fine sweep at every sliding-window depth, and the
    other workloads (3D, batched, adjoint).  The workloads'
    agreement with the oracle at these sizes is checked by the GPU tests
    (test_gpu_fullsize, test_gpu_batched, test_gpu_adjoint); here each result
    is compared with the library's own serial fine integration."""
    import numpy as np
    import torch

    import paper_2110_10762_amd as pr
    import workloads

    out = {}
    # ---- fine sweep of the 2D workload (64 states x 83 steps) by every
    # sliding-window depth D: bytes per lattice update fall as 16/D while the
    # arithmetic per pass grows with D
    p = workloads.heat2d()
    N = p.nslices
    prob = pr.Problem(pr.config_of(p))
    info = prob.info()
    xs = torch.rand((N, p.n, p.n), dtype=torch.float64, device=dev)
    ys = torch.empty_like(xs)
    npts = N * p.n * p.n
    table = []
    for d, rows, xp, sw in pr.fine_shapes(2):
        if not sw or xp != 2:
            continue
        prob.set_fine_shape(d, rows, xp)
        prob.apply_fine(xs, ys, N, info.m)
        torch.cuda.synchronize()
        reps = 5
        t = time.perf_counter()
        for _ in range(reps):
            prob.apply_fine(xs, ys, N, info.m)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t) / reps * 1e3
        passes = -(-info.m // d)
        gbs = passes * 16.0 * npts / (ms * 1e-3) / 1e9
        table.append({"kernel": f"k_fine2d_sw<{xp},{d}>", "D": d, "rows": "auto" if rows >= 1000 else rows,
                      "passes": passes, "sweep_ms": ms, "glups": npts * info.m / (ms * 1e-3) / 1e9,
                      "alg_bytes_per_lup": passes * 16.0 / info.m, "alg_GBps": gbs, "hbm_frac": gbs / HBM_PEAK_GBS})
    out["fine_depth"] = {"workload": "heat2d n=1024^2, 64 states x 83 explicit steps", "shapes": table}
    prob.close()
    del xs, ys
    torch.cuda.empty_cache()

    # ---- 3D: 256^3, 128 slices (m = 1 explicit step per slice)
    p = workloads.heat3d()
    N = p.nslices
    prob = pr.Problem(pr.config_of(p, eps=1e-10))
    prob.set_async_options(mode=pr.PR_ASYNC_FREE, time_limit_s=200.0)
    info = prob.info()
    u0 = torch.from_numpy(p.u0).to(dev)
    lam = torch.empty((N + 1,) + p.u0.shape, dtype=torch.float64, device=dev)
    sample = [1, N // 2, N]
    st = pr.Stats()
    prob.solve_fine(u0, lam, st)
    ser_ms = st.wall_ms
    ser = torch.stack([lam[i].clone() for i in sample])
    sref = ser.abs().max().item()
    npts = p.n ** 3
    xs = lam[:N]
    ys = torch.empty_like(xs[:N])
    prob.apply_fine(xs, ys, N, info.m)
    torch.cuda.synchronize()
    t = time.perf_counter()
    prob.apply_fine(xs, ys, N, info.m)
    sweep_ms = (time.perf_counter() - t) * 1e3
    del ys
    res = {"workload": "heat3d n=256^3 N=128 nu=0.5 T=2e-4 dt=0.15h^2 (m=1), CG 1e-12",
           "serial_fine_ms": ser_ms,
           "fine_sweep": {"ms": sweep_ms, "glups": N * info.m * npts / (sweep_ms * 1e-3) / 1e9,
                          "hbm_frac": N * info.m * 16.0 * npts / (sweep_ms * 1e-3) / 1e9 / HBM_PEAK_GBS}}
    for drv in ("sync", "async"):
        st = pr.Stats(N, N + 1) if drv == "sync" else pr.Stats(N)
        (prob.solve_sync if drv == "sync" else prob.solve_async)(u0, lam, st)
        got = torch.stack([lam[i] for i in sample])
        r = {"ms": st.wall_ms, "iters": st.iters, "cg_iters": st.cg_iters,
             "rel_err_vs_gpu_serial_fine": (got - ser).abs().max().item() / sref}
        if drv == "sync":
            r["fine_ms"], r["coarse_ms"] = st.fine_ms, st.coarse_ms
            # set-up 24 B from x0 = b (initial sweep, then 24 to store lambda^0
            # and w^0); afterwards each set-up carries the previous slice's
            # correction: 64 (read x0, v, w_new, w_old, lambda_old; write x, r,
            # lambda), and the last slice of an iteration corrects in a pass of
            # 40 (the same reads, write lambda)
            c_bytes = (st.cg_iters * 64.0 + N * (24.0 + 24.0) + (st.g_solves - N) * 64.0
                       + st.g_skipped * 40.0) * npts
            r["roofline_sweep"] = {"kernel": "k_sweep_cg<3>", "bound": "hbm",
                                   "achieved": c_bytes / (st.coarse_ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS,
                                   "unit": "GB/s", "frac": c_bytes / (st.coarse_ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
        else:
            r["kappa"], r["teams"], r["kernel_ms"] = st.kappa, st.teams, st.kernel_ms
            r["updates"] = st.kernel_updates
            # mean per team of the time its leader spent per phase
            r["team_ms"] = {"fine": st.team_fine_ms, "copy": st.team_copy_ms, "coarse": st.team_coarse_ms,
                            "correction": st.team_corr_ms, "total": st.team_total_ms}
        res[drv] = r
    out["heat3d"] = res
    prob.close()
    del lam, xs, ser, u0
    torch.cuda.empty_cache()

    # ---- 3D with long slices: 128^3, 64 slices of 100 fine steps (the paper's
    # ratio of slice length to fine step), labelled apart from the 256^3 workload
    p = workloads.heat3d_long()
    N = p.nslices
    prob = pr.Problem(pr.config_of(p, eps=1e-10))
    prob.set_async_options(mode=pr.PR_ASYNC_FREE, time_limit_s=200.0)
    info = prob.info()
    u0 = torch.from_numpy(p.u0).to(dev)
    lam = torch.empty((N + 1,) + p.u0.shape, dtype=torch.float64, device=dev)
    sample = [1, N // 2, N]
    st = pr.Stats()
    prob.solve_fine(u0, lam, st)
    ser_ms = st.wall_ms
    ser = torch.stack([lam[i].clone() for i in sample])
    sref = ser.abs().max().item()
    npts = p.n ** 3
    xs = lam[:N].clone()
    ys = torch.empty_like(xs)
    prob.apply_fine(xs, ys, N, info.m)
    torch.cuda.synchronize()
    t = time.perf_counter()
    prob.apply_fine(xs, ys, N, info.m)
    torch.cuda.synchronize()
    sweep_ms = (time.perf_counter() - t) * 1e3
    del xs, ys
    res = {"workload": "heat3d_long n=128^3 N=64 nu=0.5 dt=0.15h^2, 100 fine steps per slice (s = 7.5), CG 1e-12",
           "label": "supplementary: the paper's slice of 100 fine steps; not one of the benchmark's configurations",
           "serial_fine_ms": ser_ms,
           "fine_sweep": {"kernel": f"k_fine3d_tb (depth {info.tb_depth}, rows {info.tile_rows})", "ms": sweep_ms,
                          "glups": N * info.m * npts / (sweep_ms * 1e-3) / 1e9,
                          "hbm_frac": N * -(-info.m // info.tb_depth) * 16.0 * npts / (sweep_ms * 1e-3) / 1e9
                          / HBM_PEAK_GBS}}
    for drv in ("sync", "async"):
        st = pr.Stats(N, N + 1) if drv == "sync" else pr.Stats(N)
        (prob.solve_sync if drv == "sync" else prob.solve_async)(u0, lam, st)
        got = torch.stack([lam[i] for i in sample])
        r = {"ms": st.wall_ms, "iters": st.iters, "cg_iters": st.cg_iters,
             "rel_err_vs_gpu_serial_fine": (got - ser).abs().max().item() / sref}
        if drv == "sync":
            r["fine_ms"], r["coarse_ms"] = st.fine_ms, st.coarse_ms
            r["C_F_ms"] = sweep_ms / N
            r["C_G_ms"] = st.coarse_ms / max(1, st.g_solves)
        else:
            r["kappa"], r["teams"] = st.kappa, st.teams
        res[drv] = r
    out["heat3d_long"] = res
    prob.close()
    del lam, ser, u0
    torch.cuda.empty_cache()

    # ---- batched: 512 independent 2D problems, hipGraph, autotuned fine kernel
    probs = workloads.batched()
    h = pr.Problem([pr.config_of(q) for q in probs])
    t = time.perf_counter()
    h.autotune(-1, reps=1)
    tune_s = time.perf_counter() - t
    h.set_graph(True)
    u0 = torch.from_numpy(np.concatenate([q.u0.ravel() for q in probs])).to(dev)
    total = sum((q.nslices + 1) * q.n * q.n for q in probs)
    lam = torch.empty(total, dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    t = time.perf_counter()
    _, stb = h.solve_batch(u0, lam)
    torch.cuda.synchronize()
    wall_b = time.perf_counter() - t
    lups = sum(x.fine_lups for x in stb)
    work = [q.nslices * q.n * q.n for q in probs]
    pick = sorted({int(np.argmin(work)), int(np.argmax(work)), 0, len(probs) // 2})
    errs = []
    off = [0]
    for q in probs:
        off.append(off[-1] + (q.nslices + 1) * q.n * q.n)
    for b in pick:
        q = probs[b]
        one = pr.Problem(pr.config_of(q))
        ref = torch.empty((q.nslices + 1, q.n, q.n), dtype=torch.float64, device=dev)
        one.solve_fine(torch.from_numpy(q.u0).to(dev), ref)
        got = lam[off[b]: off[b + 1]].reshape(ref.shape)
        errs.append((got - ref).abs().max().item() / ref.abs().max().item())
        one.close()
    out["batched"] = {"workload": "512 2D problems, side in {64,128,256,512}, nu log-uniform [0.1,10], "
                                  "N in 8..64, 64 fine steps per slice, CG 1e-12, sync to 1e-10",
                      "wall_ms": wall_b * 1e3, "glups": lups / wall_b / 1e9, "graph": True,
                      "autotune_s": tune_s, "max_k": max(x.iters for x in stb),
                      "all_converged": all(x.converged == 1 for x in stb),
                      "sampled_problems": pick,
                      "max_rel_err_vs_gpu_serial_fine": max(errs)}
    h.close()
    del lam, u0
    torch.cuda.empty_cache()

    # ---- adjoint: dL/du0 and dL/dnu at 512^2, 32 slices
    p = workloads.adjoint2d()
    prob = pr.Problem(pr.config_of(p))
    info = prob.info()
    lam = torch.empty((p.nslices + 1,) + p.u0.shape, dtype=torch.float64, device=dev)
    prob.solve_fine(torch.from_numpy(p.u0).to(dev), lam)
    gT = (lam[-1] - torch.from_numpy(p.target).to(dev)).contiguous()
    d0 = torch.empty_like(gT)
    prob.grad(lam, gT, d0)
    torch.cuda.synchronize()
    t = time.perf_counter()
    dnu = prob.grad(lam, gT, d0)
    torch.cuda.synchronize()
    g_ms = (time.perf_counter() - t) * 1e3
    # central difference of L in nu through the library's serial fine runs
    eps = 1e-6

    def loss(nu):
        q = pr.Problem(pr.config_of(p, nu=nu))
        lq = torch.empty_like(lam)
        q.solve_fine(torch.from_numpy(p.u0).to(dev), lq)
        q.close()
        return 0.5 * ((lq[-1] - torch.from_numpy(p.target).to(dev)) ** 2).sum().item()

    fd = (loss(p.nu + eps) - loss(p.nu - eps)) / (2 * eps)
    out["adjoint"] = {"workload": "adjoint2d n=512^2 N=32 T=5e-3 dt=0.2h^2 (m=%d)" % info.m,
                      "grad_ms": g_ms, "dL_dnu": dnu, "dL_dnu_central_fd": fd,
                      "rel_diff_fd": abs(fd - dnu) / abs(dnu)}
    prob.close()
    return out


def fine_kernel_name(info):
    if info.sliding:
        return f"k_fine2d_sw<{info.xpts},{info.tb_depth}> (rows {info.tile_rows})"
    return f"k_fine2d<{info.xpts},{info.tile_rows},{info.tb_depth}>"


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: the library runs on one GPU; the method's slices would shard "
              "over GPUs by contiguous blocks, but no multi-GPU path is built or timed",
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_2110_10762_amd as pr
    import workloads

    pr.load_library()          # fails loudly if the HIP library is missing
    dev = torch.device("cuda:0")
    if args.extras_only:
        print(json.dumps(run_extras(dev)), flush=True)
        torch.cuda.synchronize()
        return
    p = workloads.heat2d()
    prob = pr.Problem(pr.config_of(p, eps=1e-10))
    info = prob.info()
    N, npts, m = p.nslices, p.n * p.n, info.m
    u0 = torch.from_numpy(p.u0).to(dev)
    lam_s = torch.empty((N + 1, p.n, p.n), dtype=torch.float64, device=dev)
    lam_a = torch.empty_like(lam_s)
    ser = torch.empty_like(lam_s)
    prob.set_async_options(mode=pr.PR_ASYNC_FREE, time_limit_s=200.0)

    # serial fine reference (outside the timed region): accuracy and baseline time
    stf = pr.Stats()
    prob.solve_fine(u0, ser, stf)
    prob.solve_fine(u0, ser, stf)
    serial_ms = stf.wall_ms

    def step(rec):
        if args.only in ("both", "sync"):
            st = pr.Stats(N, N + 1)
            prob.solve_sync(u0, lam_s, st)
            rec["sync"].append(st.as_dict())
        if args.only in ("both", "async"):
            st = pr.Stats(N)
            prob.solve_async(u0, lam_a, st)
            rec["async"].append(st.as_dict())

    warm = {"sync": [], "async": []}
    for _ in range(args.warmup):
        step(warm)
    rec = {"sync": [], "async": []}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(rec)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    # ---- outside the timed region: the fine sweep alone (every slice, m steps)
    #      and both drivers with coarse solves on input changes (linear G)
    xs = lam_s[:N].clone()
    ys = torch.empty_like(xs)
    prob.apply_fine(xs, ys, N, m)
    t1 = time.perf_counter()
    for _ in range(5):
        prob.apply_fine(xs, ys, N, m)
    sweep_ms = (time.perf_counter() - t1) / 5 * 1e3
    fine_sweep = {"kernel": fine_kernel_name(info), "ms": sweep_ms,
                  "glups": N * m * npts / (sweep_ms * 1e-3) / 1e9,
                  "hbm_frac": N * -(-m // info.tb_depth) * 16.0 * npts / (sweep_ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
    incr = {}
    if not args.no_increment:
        pi = pr.Problem(pr.config_of(p, eps=1e-10, coarse_increment=1))
        pi.set_async_options(mode=pr.PR_ASYNC_FREE, time_limit_s=200.0)
        lam_i = torch.empty_like(lam_s)
        for drv in (("sync", "async") if args.only == "both" else (args.only,)):
            st = pr.Stats(N, N + 1) if drv == "sync" else pr.Stats(N)
            (pi.solve_sync if drv == "sync" else pi.solve_async)(u0, lam_i, st)
            incr[drv] = {"ms": st.wall_ms, "iters": st.iters, "cg_iters": st.cg_iters,
                         "rel_err_vs_serial_fine": (lam_i - ser).abs().max().item() / ser.abs().max().item()}
        pi.close()
        del lam_i

    # the pipelined synchronous driver (Algorithm 1, per-slice waits, the
    # default async teams), also outside the timed region
    pipe = None
    if not args.no_pipelined and args.only == "both":
        prob.set_async_options(mode=pr.PR_ASYNC_PIPELINED, time_limit_s=200.0)
        lam_p = torch.empty_like(lam_s)
        st = pr.Stats(N)
        prob.solve_async(u0, lam_p, st)
        pipe = {"ms": st.wall_ms, "iters": st.iters,
                "rel_err_vs_serial_fine": (lam_p - ser).abs().max().item() / ser.abs().max().item()}
        prob.set_async_options(mode=pr.PR_ASYNC_FREE, time_limit_s=200.0)
        del lam_p

    sref = ser.abs().max().item()
    err_s = (lam_s - ser).abs().max().item() / sref if rec["sync"] else None
    err_a = (lam_a - ser).abs().max().item() / sref if rec["async"] else None

    lups = sum(s["fine_lups"] for s in rec["sync"]) + sum(s["fine_lups"] for s in rec["async"])
    whole_job = lups / wall / 1e9

    # ---- roofline objects (algorithmic bytes per launch / live event durations)
    # Algorithmic bytes per point: F pass 16 (read + write the state).  2D
    # preconditioned CG (sync sweep and async teams): iteration 64 (reads r,
    # u, p, x; writes the same four), set-up (one march) 32 from x0 = b (read
    # b, write x, r0, u0) in the initial sweep, 40 from the last coarse value
    # (read x0 and b, write x, r0, u0) afterwards.
    # Unpreconditioned 2D CG (cg_precond = -1; products recomputed from r and
    # p): iteration 48 (reads r, p_old, x; writes p, x, r'), set-up 24.
    # Correction 48 (read v, w_new, w_old, lambda_old, write lambda, w); in
    # the initial sweep 24 (read w_new, write lambda, w).  The synchronous
    # sweep with the preconditioned CG carries each slice's correction in the
    # set-up march of the next slice's solve: that set-up moves 72 (read x0, v,
    # w_new, w_old, lambda_old; write x, r0, u0, lambda) and the last slice's
    # correction of an iteration is a pass of 40 (the same reads, write
    # lambda).
    D = info.tb_depth
    passes = -(-m // D)
    cg_it_b, cg_set_b, cg_warm_b = (64.0, 32.0, 40.0) if info.cg_precond else (48.0, 24.0, 24.0)
    fine_kernel = fine_kernel_name(info)
    rl = {}
    if rec["sync"]:
        s = rec["sync"]
        f_ms = sum(x["fine_ms"] for x in s)
        f_bytes = sum(x["fine_lups"] for x in s) / m * passes * 16.0
        f_launches = sum(x["iters"] for x in s) * passes
        rl["fine"] = {"kernel": fine_kernel, "bound": "hbm",
                      "achieved": f_bytes / (f_ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                      "launches": f_launches, "avg_launch_ms": f_ms / f_launches,
                      "glups": sum(x["fine_lups"] for x in s) / (f_ms * 1e-3) / 1e9}
        c_ms = sum(x["coarse_ms"] for x in s)
        if info.cg_precond:   # corrections carried by the set-ups
            c_bytes = sum((x["cg_iters"] * cg_it_b + N * (cg_set_b + 24.0) + (x["g_solves"] - N) * 72.0
                           + x["g_skipped"] * 40.0) * npts for x in s)
        else:
            c_bytes = sum((x["cg_iters"] * cg_it_b + N * (cg_set_b + 24.0) + (x["g_solves"] - N) * (cg_warm_b + 48.0)
                           + x["g_skipped"] * 48.0) * npts for x in s)
        c_launches = sum(x["iters"] + 1 for x in s)
        rl["sweep"] = {"kernel": "k_sweep_cg<2,true>" if info.cg_precond else "k_sweep_cg<2,false>", "bound": "hbm", "achieved": c_bytes / (c_ms * 1e-3) / 1e9,
                       "peak": HBM_PEAK_GBS, "unit": "GB/s", "launches": c_launches,
                       "avg_launch_ms": c_ms / c_launches}
    if rec["async"]:
        a = rec["async"]
        k_ms = sum(x["kernel_ms"] for x in a)
        a_passes = -(-m // ASYNC_DEPTH)
        a_bytes = 0.0
        for x in a:
            upd = x["kernel_updates"]
            solves = x["g_solves"] - N          # minus the initial coarse sweep
            # per update: F passes, predecessor copy 16, correction + next slot
            # 40 (read v, w_new, w_old and the current slot; write the next)
            a_bytes += (upd * (a_passes * 16.0 + 16.0 + 40.0) + x["kernel_cg_iters"] * cg_it_b
                        + solves * cg_warm_b) * npts
        rl["async"] = {"kernel": f"k_async<2,2,0,{ASYNC_DEPTH},false,{'true' if info.cg_precond else 'false'}>",
                       "bound": "hbm",
                       "achieved": a_bytes / (k_ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "launches": len(a), "avg_launch_ms": k_ms / len(a)}
    same_sources = sources_digest() == PROFILED_SOURCES
    for key, r in rl.items():
        r["frac"] = r["achieved"] / r["peak"]
        r["traffic"] = PROFILED_TRAFFIC.get(key) if same_sources else None
        r["traffic_unit"] = "GB per launch"
        r["algorithmic_GB_per_launch"] = r["achieved"] * r["avg_launch_ms"] * 1e-3
    dom = max(rl, key=lambda k: rl[k]["avg_launch_ms"] * rl[k]["launches"])
    roofline = dict(rl[dom])

    # the headline: fine-stencil GLUPS of the F launches of the timed sync solves
    if rec["sync"]:
        value = sum(x["fine_lups"] for x in rec["sync"]) / (sum(x["fine_ms"] for x in rec["sync"]) * 1e-3) / 1e9
    else:
        value = whole_job
    extras = {}
    if not args.no_extras:
        extras = run_extras(dev)
    out = {
        "metric": "fine-stencil GLUPS + % HBM roofline; async vs sync Parareal time-to-1e-10",
        "value": value,
        "value_is": "fine-stencil GLUPS of the fine-propagator launches in the timed synchronous solves",
        "whole_job_glups": whole_job,
        "unit": "GLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "heat2d n=1024^2 N=64 nu=1 T=1e-3 dt=0.2h^2 (m=83), CG 1e-12; "
                               "one sync + one async Parareal solve to 1e-10 per step",
                   "parallelism": "time slices on one GPU (persistent teams for async)"},
        "roofline": roofline,
        "roofline_fine": rl.get("fine"),
        "fine_sweep": fine_sweep,
        "time_to_tol_ms_increment": incr,
        "time_to_tol_ms_pipelined_sync": pipe,
        "roofline_kernels": rl,
        "time_to_tol_ms": {
            "sync": float(np.median([x["wall_ms"] for x in rec["sync"]])) if rec["sync"] else None,
            "async": float(np.median([x["wall_ms"] for x in rec["async"]])) if rec["async"] else None,
            "serial_fine": serial_ms},
        "k_sync": rec["sync"][-1]["iters"] if rec["sync"] else None,
        "kappa_async": rec["async"][-1]["kappa"] if rec["async"] else None,
        "rel_err_vs_serial_fine": {"sync": err_s, "async": err_a},
        "cg_iters": {"sync": rec["sync"][-1]["cg_iters"] if rec["sync"] else None,
                     "async": rec["async"][-1]["cg_iters"] if rec["async"] else None},
    }
    out.update(extras)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(p, args.cpu_sample_slices)
    prob.close()
    torch.cuda.synchronize()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
