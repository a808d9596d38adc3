"""Benchmark: explicit chemotaxis step on a 4096 x 4096 FP32 grid, one MI355X.

    python bench.py [--gpus 1] [--steps 50000] [--warmup 1000] [--no-cpu-baseline]

Workload (seeded, synthetic; the paper's set-up of Sec. 3): uniform nutrient
n0 = 0.5, Gaussian inoculum b_max = 0.7 / radius 6 cells at the centre, agar
field sigma = 1 + 0.5 U[-1, 1] per cell (seed 0), chi = 1 (receptor law),
theta = kappa = D_n = 1, h = 1, dt = 0.2 h^2 / max(D_n, max sigma n b).
A step is one time step of the whole grid; every 100 steps the diagnostics
(mass, nutrient, envelope radius) are sampled into a device series, as a run
that tracks the colony envelope does.  Inputs are resident in HBM before the
timed region.  Prints one JSON line.
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, 8 TB/s
BYTES_PER_CELL_LAUNCH = {"fp32": 20, "fp64": 40}  # read b, n, sigma; write b', n'
SAMPLE_EVERY = 100
METRIC = "GCell-updates/s & % HBM peak (4096^2 FP32); velocity-map pts/s at <=2% err"
STEP_SOURCES = ("paper_1301_5058_amd/csrc/kc_step.hip", "paper_1301_5058_amd/csrc/kc_stream.h",
                "paper_1301_5058_amd/csrc/kc_device.h")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "step_stream_4096_fp32_traffic.txt")


def kernel_hash():
    h = hashlib.sha256()
    for rel in STEP_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(tsteps):
    """HBM bytes per step-kernel launch from the committed PMC summary, or None
    when the summary is missing, for another fused depth, or for older kernel
    sources."""
    try:
        txt = open(TRAFFIC_FILE).read()
    except OSError:
        return None
    kv = dict(re.findall(r"^(\w+)\s*=\s*(\S+)", txt, flags=re.M))
    if kv.get("kernel_sources_sha256_16") != kernel_hash() or int(kv.get("tsteps", -1)) != tsteps:
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_baseline(b, n, s, dt, chi, budget_s=15.0):
    """The FP64 oracle on the host cores, on a bounded number of steps of the
    same 4096^2 fields (calibrated to ~budget_s of CPU time)."""
    import numpy as np
    import oracle
    b64, n64, s64 = (a.astype(np.float64) for a in (b, n, s))
    t0 = time.perf_counter()
    oracle.run(b64, n64, s64, 1.0, dt, 2, chi=chi)
    per = (time.perf_counter() - t0) / 2
    steps = int(max(4, min(20000, budget_s / max(per, 1e-9))))
    t0 = time.perf_counter()
    oracle.run(b64, n64, s64, 1.0, dt, steps, chi=chi)
    el = time.perf_counter() - t0
    cells = b.size
    return {"value": round(cells * steps / el / 1e9, 5), "unit": "GCell-updates/s",
            "cores": oracle.threads(), "kind": "oracle",
            "sample": "FP64 C oracle, %d steps of the same %dx%d fields (%.1f s)"
                      % (steps, b.shape[1], b.shape[0], el)}


def run(args):
    import numpy as np
    import torch
    from paper_1301_5058_amd import workload
    from paper_1301_5058_amd.solver import Solver

    cfg = workload.SINGLE_4096
    nx, ny, chi = cfg["nx"], cfg["ny"], cfg["chi"]
    b, n, s = workload.fields(nx, ny, cfg["n0"], cfg["a"], cfg["seed"])
    dt = workload.config_dt(b, n, s)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    tb, tn, ts = (torch.from_numpy(a).to(dev) for a in (b, n, s))
    stream = torch.cuda.current_stream()
    S = Solver(nx, ny, dt=dt, chi=chi, precision="fp32", b_thr=0.5 * cfg["n0"], stream=stream)
    S.set_fields(tb, tn, ts)
    tsteps, rows, pf = S.tuning()

    nsamp = args.steps // SAMPLE_EVERY + 2
    series = torch.zeros((nsamp, 5), dtype=torch.float64, device=dev)

    # warmup (same code path)
    left = args.warmup
    while left > 0:
        k = min(SAMPLE_EVERY, left)
        S.step(k)
        left -= k
    torch.cuda.synchronize()

    # timed region: HIP events on the solver's stream around every chunk
    nchunks = (args.steps + SAMPLE_EVERY - 1) // SAMPLE_EVERY
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2 * nchunks + 1)]
    torch.cuda.synchronize()
    t_wall = time.perf_counter()
    ev[0].record(stream)
    left, i = args.steps, 0
    launches = 0
    while left > 0:
        k = min(SAMPLE_EVERY, left)
        S.step(k)
        launches += (k // tsteps) + (1 if k % tsteps else 0)
        ev[2 * i + 1].record(stream)
        S.diagnostics_device(series[i])
        ev[2 * i + 2].record(stream)
        left -= k
        i += 1
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_wall
    total_ms = ev[0].elapsed_time(ev[2 * nchunks])
    step_ms = sum(ev[2 * j].elapsed_time(ev[2 * j + 1]) for j in range(nchunks))

    cells = nx * ny
    value = cells * args.steps / (total_ms / 1e3) / 1e9
    launch_ms = step_ms / launches
    alg_bytes = BYTES_PER_CELL_LAUNCH["fp32"] * cells
    achieved = alg_bytes / (launch_ms / 1e3) / 1e9
    traffic = measured_traffic(tsteps)
    last = series[nchunks - 1].cpu().numpy()
    out = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "GCell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(total_ms / args.steps, 6),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "single instance 4096x4096 FP32, n0=0.5, sigma amplitude 0.5, "
                               "chi=1 receptor law, forward Euler, diagnostics every 100 steps",
                   "nx": nx, "ny": ny, "dt": dt, "chi": chi, "tsteps": tsteps, "rows": rows,
                   "prefetch": pf},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic,
                     "kernel": "step_stream<float,T=%d>" % tsteps,
                     "launch_us": round(launch_ms * 1e3, 3),
                     "alg_bytes_per_launch": alg_bytes},
        "effective_hbm_frac": round(value * 1e9 * 20 / (HBM_PEAK_GBS * 1e9), 4),
        "wall_s": round(wall, 3),
        "final_diag": {"t": float(last[0]), "mass": float(last[1]), "nutrient": float(last[2]),
                       "envelope_radius": float(last[3]), "area_radius": float(last[4])},
    }
    S.close()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(b, n, s, dt, chi)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50000)
    ap.add_argument("--warmup", type=int, default=1000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only; --gpus %d is not supported "
              "(the multi-GPU domain decomposition is a design, not code)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)
    if args.steps < 1 or args.warmup < 0:
        print("bench.py: --steps must be >= 1 and --warmup >= 0", file=sys.stderr)
        sys.exit(2)
    out = run(args)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
