"""Write the autotune database of the fused step kernel for a set of grids.

    python -m paper_1301_5058_amd.tune_db OUT.jsonl [--effort 1] [--only 2048/fp32/rk2+noise]

For every (grid, precision) below, a solver is created on the workload's
fields and kc_autotune times the candidate configurations; the winners are
appended to OUT.jsonl (the format read through KC_AUTOTUNE_CACHE).  The
shipped paper_1301_5058_amd/tuning/gfx950.jsonl was written this way on an
MI355X.
"""
import argparse
import os
import sys

import numpy as np
import torch

from . import workload
from .solver import Solver

GRIDS = [  # (nx, n0, a, chi, precision, integrator)
    (128, 0.8, 0.5, 0.5, "fp32", "euler"), (128, 0.8, 0.5, 0.5, "fp64", "euler"),
    (512, 0.35, 0.5, 2.0, "fp32", "euler"),
    (4096, 0.5, 0.5, 1.0, "fp32", "euler"), (4096, 0.5, 0.5, 1.0, "fp64", "euler"),
    (16384, 0.35, 0.5, 2.0, "fp32", "euler"),
    (4096, 0.5, 0.5, 1.0, "fp32", "rk2"), (4096, 0.5, 0.5, 1.0, "fp64", "rk2"),
    (4096, 0.5, 0.5, 1.0, "fp32", "euler+noise"),
    (2048, 0.71, 0.5, 5.0, "fp32", "rk2+noise"),  # the paper's own runs
]
NOISE = {"sigma0": 1.0, "amp": 0.5, "seed": 2013}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("out")
    ap.add_argument("--effort", type=int, default=1)
    ap.add_argument("--only", default=None,
                    help="comma-separated NX/PRECISION/INTEGRATOR entries, e.g. 2048/fp32/rk2+noise")
    a = ap.parse_args()
    only = None if a.only is None else set(a.only.split(","))
    os.environ["KC_AUTOTUNE_CACHE"] = os.path.abspath(a.out)
    for nx, n0, amp, chi, prec, integ in GRIDS:
        if only is not None and "%d/%s/%s" % (nx, prec, integ) not in only:
            continue
        b, n, s = workload.fields(nx, nx, n0, amp, 0)
        dt = workload.config_dt(b, n, s)
        if prec == "fp64":
            b, n, s = (x.astype(np.float64) for x in (b, n, s))
        noise = NOISE if integ.endswith("+noise") else None
        S = Solver(nx, nx, dt=dt, chi=chi, precision=prec, integrator=integ.split("+")[0],
                   noise=noise)
        S.set_fields(*(torch.from_numpy(x).cuda() for x in ((b, n) if noise else (b, n, s))))
        g = S.autotune(effort=a.effort, use_cache=True)
        print("%5d^2 %s %s: tsteps=%d rows=%d prefetch=%d waves/strip=%d  %.1f GCell/s"
              % ((nx, prec, integ) + S.tuning() + (S.strip_waves(), g)), flush=True)
        S.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
