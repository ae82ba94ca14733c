"""Writes the stored expected values under tests/golden/ from the CPU oracle only.

The paper prints no worked numerical example, so every stored value here comes
from the oracle (pinned by tests/test_oracle_pins.py) on the seeded workloads.
Run:  python tests/golden/make_golden.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads  # noqa: E402
from oracle import heat, parareal  # noqa: E402


def main():
    p = workloads.heat1d()
    d = heat.discretise(p.dim, p.n, p.nu, p.T, p.nslices, p.dt_nominal)
    pr = heat.Propagators(d)
    res = parareal.parareal_sync(p.u0, pr.F, pr.G, d.nslices, eps=p.eps)
    ser = heat.serial_fine(p.u0, d.r, d.m, d.nslices)
    out = {
        "workload": "heat1d n=127 N=16 nu=1 T=0.1 dt=0.4h^2 (seed 0)",
        "m": d.m, "dt": d.dt, "r": d.r, "s": d.s,
        "sync_iters": res.iters,
        "sync_deltas": res.deltas,
        "sync_lambda_N": res.lam[-1].tolist(),
        "serial_fine_uT": ser[-1].tolist(),
    }
    with open(os.path.join(HERE, "heat1d_sync.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
