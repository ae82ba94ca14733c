"""Delay study: pipelined synchronous Parareal (Algorithm 1, per-slice waits)
against asynchronous Parareal (Algorithm 2) under emulated message latency,
on the 2D heat workload (1024^2 interior points, 64 slices, nu = 1, T = 1e-3,
fine dt = 0.2 h^2, backward-Euler coarse step by CG to 1e-12, stop at 1e-10).

Three team layouts: one team per slice (the paper's p = N processors), one
team per XCD, and the library's default of four teams of two XCDs, each of
the last two holding a contiguous block of slices.  A published slice value
becomes readable by the successor only `latency` after its publication, the
emulated transfer of Section 4.1.  For every latency both drivers run to the
tolerance; the lines report wall time, k, kappa, the per-team costs C_F and
C_G measured inside the launch, and, for one team per slice, the times the
cost models of Section 4.1 predict from them:
    pipelined, Proposition (latency on every message):
        init + p C_G + k (C_F + C_G + (p - 1 - (k+1)/2) L)
    pipelined, the paper's remark that with regular delays only the first
    wave pays:  init + p C_G + k (C_F + C_G) + (p - 2) L
    async, Proposition:  init + p C_G + kappa (C_F + C_G)
where init is the initial coarse sweep (done by the whole GPU here) and p C_G
the first wave of coarse solves down the pipeline.

    python bench_delays.py [--latency-ms 0,10,30,100] [--teams N]
"""
import argparse
import json
import os
import sys

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--latency-ms", default="0,3,10,30,100")
    ap.add_argument("--teams", default="64,8,4", help="team counts (64: one per slice)")
    ap.add_argument("--gpus", type=int, default=1)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench_delays.py: one GPU only", file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_2110_10762_amd as pr
    import workloads

    pr.load_library()
    p = workloads.heat2d()
    N = p.nslices
    prob = pr.Problem(pr.config_of(p, eps=1e-10))
    u0 = torch.from_numpy(p.u0).to("cuda:0")
    lam = torch.empty((N + 1, p.n, p.n), dtype=torch.float64, device="cuda:0")
    ser = torch.empty_like(lam)
    prob.solve_fine(u0, ser)
    sref = ser.abs().max().item()

    st = pr.Stats(N, N + 1)
    prob.solve_sync(u0, lam, st)
    print(json.dumps({"driver": "bulk_sync", "wall_ms": st.wall_ms, "k": st.iters,
                      "rel_err": (lam - ser).abs().max().item() / sref}), flush=True)

    for teams in [min(int(x), N) for x in args.teams.split(",")]:
      for lat_ms in [float(x) for x in args.latency_ms.split(",")]:
        for mode, name in ((pr.PR_ASYNC_PIPELINED, "pipelined_sync"), (pr.PR_ASYNC_FREE, "async")):
            prob.set_async_options(mode=mode, teams=teams, latency_us=lat_ms * 1e3, time_limit_s=300.0)
            st = pr.Stats(N)
            prob.solve_async(u0, lam, st)
            upd = max(st.kernel_updates, 1)
            solves = max(st.g_solves - N, 1)
            # per-team costs measured in the launch: one fine propagation, one coarse solve
            c_f = st.team_fine_ms * st.teams / upd
            c_g = st.team_coarse_ms * st.teams / solves
            c_init = st.coarse_ms          # the initial coarse sweep (whole GPU here)
            models = {}
            if teams == N:
                if mode == pr.PR_ASYNC_PIPELINED:
                    k = st.iters
                    models["every_message"] = c_init + N * c_g + k * (c_f + c_g + (N - 1 - (k + 1) / 2) * lat_ms)
                    models["first_wave"] = c_init + N * c_g + k * (c_f + c_g) + (N - 2) * lat_ms
                else:
                    models["proposition"] = c_init + N * c_g + st.kappa * (c_f + c_g)
            print(json.dumps({"driver": name, "teams": st.teams, "latency_ms": lat_ms, "wall_ms": st.wall_ms,
                              "k": st.iters, "kappa": st.kappa, "g_solves": st.g_solves,
                              "C_F_ms": c_f, "C_G_ms": c_g, "init_ms": c_init,
                              "model_ms": models, "converged": st.converged,
                              "rel_err": (lam - ser).abs().max().item() / sref}), flush=True)


if __name__ == "__main__":
    main()
