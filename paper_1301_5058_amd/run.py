"""Run one single-instance configuration of the solver and print its rate.

    python -m paper_1301_5058_amd.run [--nx 4096] [--ny NX] [--precision fp32|fp64]
        [--integrator euler|rk2] [--noise] [--chi 1.0] [--n0 0.5] [--amp 0.5]
        [--steps 400] [--warmup 100] [--tuning T,ROWS,PF[,WAVES]] [--paper-set NAME]
        [--copy-ref-mib M]

The workload is the seeded synthetic one of the library's benchmarks (uniform
nutrient n0, the Gaussian inoculum at the centre, sigma = 1 + amp U[-1, 1] per
cell, dt = 0.2 h^2 / max(D_n, max sigma n b)); with --noise the agar field is
redrawn at every cell and step (sigma0 = 1, amplitude amp); with --paper-set the
grid, cell width, inoculum, noise and step of one of the paper's figure sets
(Sec. 3) are used instead, at the larger sensitivity of the set.  Fields stay
on the device; the timed region is `steps` steps (HIP events on the solver's
stream).  The tuning comes from the shipped autotune table unless --tuning
fixes it.  Prints one JSON line.  Used to drive profilers over one kernel
configuration at a time; --copy-ref-mib first makes a plain device copy of M
MiB, against which byte counters are calibrated.
"""
import argparse
import json
import os
import sys


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--nx", type=int, default=4096)
    ap.add_argument("--ny", type=int, default=0)
    ap.add_argument("--precision", choices=("fp32", "fp64"), default="fp32")
    ap.add_argument("--integrator", choices=("euler", "rk2"), default="euler")
    ap.add_argument("--noise", action="store_true")
    ap.add_argument("--chi", type=float, default=1.0)
    ap.add_argument("--n0", type=float, default=0.5)
    ap.add_argument("--amp", type=float, default=0.5)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--tuning", default="")
    ap.add_argument("--paper-set", default="")
    ap.add_argument("--copy-ref-mib", type=int, default=0)
    a = ap.parse_args(argv)

    import numpy as np
    import torch

    from . import workload
    from .solver import Solver

    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    os.environ.setdefault("KC_AUTOTUNE_CACHE",
                          os.path.join(root, "paper_1301_5058_amd", "tuning", "gfx950.jsonl"))
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    if a.copy_ref_mib:
        # a plain device copy of known size, against which profiler byte
        # counters are calibrated
        x = torch.ones(a.copy_ref_mib * 262144, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        y.copy_(x)
        torch.cuda.synchronize()
        del x, y
    if a.paper_set:
        ps = workload.PAPER_SETS[a.paper_set]
        geo = workload.PAPER_2D
        nx = ny = a.nx if a.nx != 4096 else geo["cells"]
        h = geo["length"] / nx
        b, n = workload.paper_fields(nx, geo["length"], ps["n0"])
        dt = workload.paper_dt(nx, geo["length"], ps["sigma0"], ps["n0"], ps["dt"])
        noise = dict(sigma0=ps["sigma0"], amp=geo["amp"], seed=1)
        S = Solver(nx, ny, h=h, dt=dt, chi=ps["chi"][-1], precision=a.precision,
                   b_thr=0.5 * ps["n0"], stream=stream, integrator="rk2", noise=noise)
        fields = (b, n)
        integrator = "rk2"
    else:
        nx, ny = a.nx, a.ny or a.nx
        b, n, s = workload.fields(nx, ny, a.n0, a.amp, 0)
        dt = workload.config_dt(b, n, s)
        noise = dict(sigma0=1.0, amp=a.amp, seed=2013) if a.noise else None
        if a.precision == "fp64":
            b, n, s = (x.astype(np.float64) for x in (b, n, s))
        S = Solver(nx, ny, dt=dt, chi=a.chi, precision=a.precision, b_thr=0.5 * a.n0,
                   stream=stream, integrator=a.integrator, noise=noise)
        fields = (b, n) if noise else (b, n, s)
        integrator = a.integrator
    S.set_fields(*(torch.from_numpy(x).cuda() for x in fields))
    if a.tuning:
        vals = [int(v) for v in a.tuning.split(",")]
        S.set_tuning(*vals)
    else:
        S.autotune(effort=0, use_cache=True)
    T, rows, pf = S.tuning()
    waves = S.strip_waves()
    S.step(a.warmup)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    S.step(a.steps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    m, nu, r = S.diagnostics()
    S.close()
    out = {"nx": nx, "ny": ny, "precision": a.precision, "integrator": integrator,
           "noise": noise is not None, "steps": a.steps, "tsteps": T, "rows": rows, "prefetch": pf,
           "waves_per_strip": waves,
           "ms": round(ms, 4), "gcell_steps_s": round(nx * ny * a.steps / (ms * 1e-3) / 1e9, 2),
           "mass": m, "nutrient": nu, "envelope_radius": r}
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
