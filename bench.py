"""Benchmark: explicit chemotaxis step on a 4096 x 4096 FP32 grid, one MI355X.

    python bench.py [--gpus 1] [--steps 500] [--warmup 10] [--no-cpu-baseline]
                    [--no-extras] [--copy-ref-mib M]

Workload (seeded, synthetic; the paper's set-up of Sec. 3): uniform nutrient
n0 = 0.5, Gaussian inoculum b_max = 0.7 / radius 6 cells at the centre, agar
field sigma = 1 + 0.5 U[-1, 1] per cell (seed 0), chi = 1 (receptor law),
theta = kappa = D_n = 1, h = 1, dt = 0.2 h^2 / max(D_n, max sigma n b).
One benchmark step is one pass of the whole hot path: 100 time steps of the
grid followed by the diagnostics (mass, nutrient, envelope and area radius,
folded into the last step launch) sampled into a device series, as a run that
tracks the colony envelope does; the defaults time 500 such steps (50,000 time
steps) after 10 (1,000 time steps) of warm-up.  The value is cell-updates
(cells x time steps) per second.  Inputs are resident in HBM before the timed
region.  Prints one JSON line.

The line also carries, under "extras", the other workloads of the solver:
the FP64 variant, chi = 0, the two-stage Runge-Kutta integrator (FP32 and
FP64) and the per-step agar noise at 4096^2, the 16384^2 grid (20,000 steps), the 256-instance batched
sweep (30,000 steps), the velocity map (surrogate with solver fallback) and
the 1-D front-speed experiment of Sec. 4.2.  --no-extras skips them.
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
# VALU issue rate: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz (one lane-op per lane per clock)
VALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12
# algorithmic VALU lane-operations per cell-update of an interior cell (receptor
# law): coefficients 8 (sigma n b: 2 mul; chi-weighted b^2 term: 2 mul; (1+n)^2: add,
# mul; reciprocal; product), two faces 2 x 7 (two differences, compare, select,
# diffusivity sum, product, fused multiply-add), two net fluxes 2 x 3, update 5
OPS_PER_CELL_UPDATE = 33
# a two-stage Runge-Kutta step: two Euler stages and the average (add, multiply)
# of b and n
OPS_PER_RK2_UPDATE = 2 * OPS_PER_CELL_UPDATE + 4
BYTES_PER_CELL_LAUNCH = {"fp32": 20, "fp64": 40}  # read b, n, sigma; write b', n'
# per-step agar noise: sigma is drawn in the kernel, not read (read b, n; write b', n'),
# and each cell-update draws it: Philox4x32-10 is 10 rounds of two 32 x 32 -> 64
# multiplies and two three-way XORs per call of four cells (10 per cell), then the
# sum of the word's halves, its conversion and one FMA
BYTES_PER_CELL_LAUNCH_NOISE = {"fp32": 16, "fp64": 32}
OPS_PER_NOISE_DRAW = 13
# per-step agar noise of the 4096^2 workload: sigma = 1 + 0.5 Delta, redrawn every step
NOISE_4096 = {"sigma0": 1.0, "amp": 0.5, "seed": 2013}
SAMPLE_EVERY = 100  # time steps per benchmark step (one diagnostics sample each)
T_START = time.perf_counter()
# published MI355X FP32 vector peak (packed FMA) and the non-packed half of it
FP32_PEAK_TFLOPS = 157.3
FP32_NONPACKED_TFLOPS = 78.6
# floating-point operations per cell-update (FMA = 2) of the textbook per-cell
# form, which evaluates each of a cell's four face fluxes itself: coefficients 8,
# four faces 4 x 8, two net fluxes 6, update 9 = 55.  This implementation shares
# each face between its two cells and needs 33 VALU operations (39 flops).
FLOPS_PER_CELL_UPDATE = 55
METRIC = "GCell-updates/s & % HBM peak (4096^2 FP32); velocity-map pts/s at <=2% err"
STEP_SOURCES = ("paper_1301_5058_amd/csrc/kc_step.hip", "paper_1301_5058_amd/csrc/kc_step_kernels.h",
                "paper_1301_5058_amd/csrc/kc_stream_f32_euler.hip",
                "paper_1301_5058_amd/csrc/kc_stream_f32_euler4.hip",
                "paper_1301_5058_amd/csrc/kc_stream.h", "paper_1301_5058_amd/csrc/kc_device.h",
                "paper_1301_5058_amd/build.py")
# PMC summaries of the bench kernel, one pair per profiled configuration
TRAFFIC_FILES = [os.path.join(ROOT, "profiles", f) for f in
                 ("step_stream_4096_fp32_traffic.txt", "step_split_4096_fp32_traffic.txt")]
COUNTERS_FILES = [os.path.join(ROOT, "profiles", f) for f in
                  ("step_stream_4096_fp32_counters.txt", "step_split_4096_fp32_counters.txt")]
# The two 4096^2 FP32 configurations (tsteps, rows, prefetch, wavefronts per
# strip) that the autotuner ranks within a few per cent of each other, in an
# order that changes from one MI355X to another: the shipped database's pick
# (one wavefront per strip) and the split kernel's.  bench.py times both on
# the GPU it runs on and keeps the faster; both are profiled under profiles/.
CANDIDATES_4096 = [(4, 35, 4, 1), (4, 46, 4, 2)]
# shipped autotune database (written by paper_1301_5058_amd/tune_db.py on an MI355X);
# grids without an entry are timed on the spot
os.environ.setdefault("KC_AUTOTUNE_CACHE",
                      os.path.join(ROOT, "paper_1301_5058_amd", "tuning", "gfx950.jsonl"))


def _code_only(text, python=False):
    """Source text without comments and blank lines (C/C++ `//` and `/* */`
    comments outside string literals, or Python `#` comments), so that editing
    a comment leaves the hash of the kernel sources unchanged."""
    out, i, n = [], 0, len(text)
    while i < n:
        c = text[i]
        if c == '"' or c == "'":  # a literal, copied as it stands
            j = i + 1
            while j < n and text[j] != c and text[j] != "\n":
                j += 2 if text[j] == "\\" else 1
            out.append(text[i:j + 1])
            i = j + 1
        elif python and c == "#":
            while i < n and text[i] != "\n":
                i += 1
        elif not python and text.startswith("//", i):
            while i < n and text[i] != "\n":
                i += 1
        elif not python and text.startswith("/*", i):
            j = text.find("*/", i + 2)
            i = n if j < 0 else j + 2
        else:
            out.append(c)
            i += 1
    lines = [ln.rstrip() for ln in "".join(out).splitlines()]
    return "\n".join(ln for ln in lines if ln.strip())


def kernel_hash():
    """Hash of the step kernel's sources (code only) and build flags; the PMC
    summaries under profiles/ record the hash of the sources they measured."""
    h = hashlib.sha256()
    for rel in STEP_SOURCES:
        with open(os.path.join(ROOT, rel), encoding="utf-8") as f:
            h.update(_code_only(f.read(), python=rel.endswith(".py")).encode())
    return h.hexdigest()[:16]


def _tuning_matches(kv, tsteps, rows, prefetch, waves):
    return (int(kv.get("tsteps", -1)), int(kv.get("rows", -1)), int(kv.get("prefetch", -1)),
            int(kv.get("waves", 1))) == (tsteps, rows, prefetch, waves)


def _summary(paths, tsteps, rows, prefetch, waves):
    """(path, key-value pairs) of the PMC summary among `paths` that was taken
    for this configuration and the current kernel sources, or None."""
    for path in paths:
        try:
            txt = open(path).read()
        except OSError:
            continue
        kv = dict(re.findall(r"^(\w+)\s*=\s*(\S+)", txt, flags=re.M))
        if kv.get("kernel_sources_sha256_16") == kernel_hash() and \
                _tuning_matches(kv, tsteps, rows, prefetch, waves):
            return path, kv
    return None


def measured_traffic(tsteps, rows, prefetch, waves=1):
    """HBM bytes per step-kernel launch from the committed PMC summary, or None
    when no summary was taken for this configuration and these kernel sources."""
    found = _summary(TRAFFIC_FILES, tsteps, rows, prefetch, waves)
    try:
        return float(found[1]["hbm_bytes_per_launch"]) if found else None
    except (KeyError, ValueError):
        return None


def measured_counters(tsteps, rows, prefetch, waves=1):
    """VALU counters of the step kernel from the committed PMC summary (issued
    VALU instructions per useful cell-update, VALU busy fraction), or None when
    no summary was taken for this configuration and these kernel sources."""
    found = _summary(COUNTERS_FILES, tsteps, rows, prefetch, waves)
    if not found:
        return None
    try:
        return {"valu_issued_per_update": float(found[1]["valu_issued_per_update"]),
                "valu_busy": float(found[1]["valu_busy"]),
                "source": os.path.relpath(found[0], ROOT)}
    except (KeyError, ValueError):
        return None


def cpu_baseline(b, n, s, dt, chi, budget_s=15.0):
    """The FP64 oracle on the host cores, on a bounded number of steps of the
    same 4096^2 fields (calibrated to ~budget_s of CPU time)."""
    import numpy as np
    import oracle
    build = oracle.use_native()  # the same arithmetic, built for this host's CPU
    b64, n64, s64 = (a.astype(np.float64) for a in (b, n, s))
    t0 = time.perf_counter()
    oracle.run(b64, n64, s64, 1.0, dt, 2, chi=chi)
    per = (time.perf_counter() - t0) / 2
    steps = int(max(4, min(20000, budget_s / max(per, 1e-9))))
    t0 = time.perf_counter()
    oracle.run(b64, n64, s64, 1.0, dt, steps, chi=chi)
    el = time.perf_counter() - t0
    cells = b.size
    cores = oracle.threads()
    # the same oracle on one thread, a few steps (about a third of the budget)
    oracle.set_threads(1)
    try:
        t0 = time.perf_counter()
        oracle.run(b64, n64, s64, 1.0, dt, 1, chi=chi)
        per1 = time.perf_counter() - t0
        steps1 = int(max(1, min(200, budget_s / 3 / max(per1, 1e-9))))
        t0 = time.perf_counter()
        oracle.run(b64, n64, s64, 1.0, dt, steps1, chi=chi)
        el1 = time.perf_counter() - t0
    finally:
        oracle.set_threads(cores)
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), "")
    except OSError:
        pass
    return {"value": round(cells * steps / el / 1e9, 5), "unit": "GCell-updates/s",
            "cores": cores, "kind": "oracle",
            "sample": "FP64 C oracle, %d steps of the same %dx%d fields (%.1f s)"
                      % (steps, b.shape[1], b.shape[0], el),
            "build": build,
            "single_thread": {"value": round(cells * steps1 / el1 / 1e9, 5), "steps": steps1,
                              "seconds": round(el1, 2)},
            "host": {"cpu_model": model, "nproc": os.cpu_count()}}


def progress(msg):
    """Progress line on stderr (stdout carries only the JSON result)."""
    print("[bench %.0fs] %s" % (time.perf_counter() - T_START, msg), file=sys.stderr, flush=True)


def launch_probe(S, stream, launches=60):
    """Average duration (ms) of one fused launch of the current depth, from
    HIP events on the solver's stream around `launches` back-to-back launches."""
    import torch
    T = S.tuning()[0]
    S.step(T * 4)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    S.step(T * launches)
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / launches


def copy_bandwidth(mib=1024, reps=5):
    """GB/s (bytes read + written) of a plain device-to-device copy of `mib`
    MiB, best of `reps`, timed with HIP events: what HBM delivers to a
    streaming kernel on this GPU."""
    import torch
    x = torch.ones(mib * 262144, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    y.copy_(x)
    best = 1e30
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        y.copy_(x)
        e1.record()
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1))
    del x, y
    return 2 * mib * 1048576 / (best * 1e-3) / 1e9


def roofline(precision, cells, tsteps, launch_ms, ops_per_update=OPS_PER_CELL_UPDATE,
             bytes_per_cell=None):
    """Roofline of the fused step kernel: the bound (HBM or VALU) with the
    larger fraction of its peak is reported as the kernel's bound."""
    if bytes_per_cell is None:
        bytes_per_cell = BYTES_PER_CELL_LAUNCH[precision]
    bytes_per = bytes_per_cell * cells
    gbs = bytes_per / (launch_ms / 1e3) / 1e9
    tops = ops_per_update * cells * tsteps / (launch_ms / 1e3) / 1e12
    hbm = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(gbs / HBM_PEAK_GBS, 4), "alg_bytes_per_launch": bytes_per}
    alu = {"bound": "alu", "achieved": round(tops, 3), "peak": round(VALU_PEAK_TOPS, 2),
           "unit": "Tops/s", "frac": round(tops / VALU_PEAK_TOPS, 4),
           "alg_ops_per_launch": ops_per_update * cells * tsteps}
    return (alu, hbm) if alu["frac"] > hbm["frac"] else (hbm, alu)


def timed_run(S, stream, steps, series=None):
    """`steps` time steps with diagnostics every SAMPLE_EVERY steps; returns
    elapsed ms."""
    import torch
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    left, i = steps, 0
    while left > 0:
        k = min(SAMPLE_EVERY, left)
        if series is not None:
            S.step_sample(k, series[i])  # diagnostics fused into the last launch
        else:
            S.step(k)
        left -= k
        i += 1
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1)


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
    if args.copy_ref_mib:
        # a plain device copy of known size, so that profiler byte counters can
        # be calibrated against it (used by the PMC runs that write profiles/)
        x = torch.ones(args.copy_ref_mib * 262144, dtype=torch.float32, device=dev)
        y = torch.empty_like(x)
        y.copy_(x)
        torch.cuda.synchronize()
        del x, y
    tb, tn, ts = (torch.from_numpy(a).to(dev) for a in (b, n, s))
    stream = torch.cuda.current_stream()
    S = Solver(nx, ny, dt=dt, chi=chi, precision="fp32", b_thr=0.5 * cfg["n0"], stream=stream)
    S.set_fields(tb, tn, ts)
    tuned = S.autotune(effort=0 if args.quick_tune else 1, use_cache=True)
    choice = None
    if args.tuning:
        S.set_tuning(*(int(v) for v in args.tuning.split(",")))
    elif not args.quick_tune:
        # the faster of the two profiled configurations on this GPU (best of
        # two probes of 40 launches each), then the fields again from the start
        us = [1e30] * len(CANDIDATES_4096)
        for _ in range(2):
            for k, cand in enumerate(CANDIDATES_4096):
                S.set_tuning(*cand)
                us[k] = min(us[k], launch_probe(S, stream, 40) * 1e3)
        best = CANDIDATES_4096[us.index(min(us))]
        S.set_tuning(*best)
        S.set_fields(tb, tn, ts)
        choice = {"candidates": [list(c) for c in CANDIDATES_4096],
                  "launch_us": [round(u, 2) for u in us]}
    tsteps, rows, pf = S.tuning()
    waves = S.strip_waves()
    progress("autotuned 4096^2 fp32: T=%d rows=%d prefetch=%d waves/strip=%d (%.1f GCell/s)"
             % (tsteps, rows, pf, waves, tuned))

    time_steps = args.steps * SAMPLE_EVERY
    series = torch.zeros((args.steps + 1, 5), dtype=torch.float64, device=dev)
    if args.warmup:  # the same code path
        timed_run(S, stream, args.warmup * SAMPLE_EVERY, series)
    torch.cuda.synchronize()

    t_wall = time.perf_counter()
    total_ms = timed_run(S, stream, time_steps, series)
    wall = time.perf_counter() - t_wall
    cells = nx * ny
    value = cells * time_steps / (total_ms / 1e3) / 1e9
    last = series[args.steps - 1].cpu().numpy()

    progress("timed %d steps (%d time steps): %.1f GCell/s" % (args.steps, time_steps, value))
    launch_ms = launch_probe(S, stream)
    main_rl, other_rl = roofline("fp32", cells, tsteps, launch_ms)
    main_rl["traffic"] = measured_traffic(tsteps, rows, pf, waves)
    main_rl["kernel"] = "%s<float,T=%d,PF=%d>" % ("step_split" if waves == 2 else "step_stream",
                                                 tsteps, pf)
    main_rl["launch_us"] = round(launch_ms * 1e3, 3)
    main_rl["other_bound"] = other_rl
    # context for the HBM figures: a plain 1 GiB device-to-device copy
    other_rl["copy_gbs"] = round(copy_bandwidth(), 1)
    # the same launch priced in flops: 55 per update against the published
    # FP32 peak (which counts packed FMAs, not used here) and its non-packed half
    tflops = FLOPS_PER_CELL_UPDATE * cells * tsteps / (launch_ms / 1e3) / 1e12
    main_rl["flop_view"] = {"flops_per_update": FLOPS_PER_CELL_UPDATE,
                            "achieved_tflops": round(tflops, 2),
                            "frac_of_157_3": round(tflops / FP32_PEAK_TFLOPS, 4),
                            "frac_of_nonpacked_78_6": round(tflops / FP32_NONPACKED_TFLOPS, 4)}
    main_rl["counters"] = measured_counters(tsteps, rows, pf, waves)
    # the same lane-operation rate against twice the issue rate: FP32 VALU
    # instructions with at most two VGPR sources issue at up to that rate from
    # enough wavefronts per SIMD on gfx950 (three-source FMAs do not)
    main_rl["frac_of_2x_issue_rate"] = round(main_rl["achieved"] / (2 * VALU_PEAK_TOPS), 4) \
        if main_rl["bound"] == "alu" else None
    S.close()

    out = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "GCell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(total_ms / args.steps, 6),
        "time_steps_per_step": SAMPLE_EVERY,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "single instance 4096x4096 FP32, n0=0.5, sigma amplitude 0.5, "
                               "chi=1 receptor law, forward Euler; one step = 100 time steps "
                               "+ fused diagnostics",
                   "nx": nx, "ny": ny, "dt": dt, "chi": chi, "tsteps": tsteps, "rows": rows,
                   "prefetch": pf, "waves_per_strip": waves, "autotune_gcell_s": round(tuned, 1),
                   "configuration_choice": choice},
        "roofline": main_rl,
        # 20 B per cell-update against 8 TB/s: above 1 because a launch reads
        # and writes each cell once for 4 time steps (temporal blocking)
        "effective_hbm_frac": round(value * 1e9 * 20 / (HBM_PEAK_GBS * 1e9), 4),
        "wall_s": round(wall, 3),
        "final_diag": {"t": float(last[0]), "mass": float(last[1]), "nutrient": float(last[2]),
                       "envelope_radius": float(last[3]), "area_radius": float(last[4])},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(b, n, s, dt, chi)
        progress("cpu baseline: %.3f GCell/s on %d threads"
                 % (out["cpu_baseline"]["value"], out["cpu_baseline"]["cores"]))
    if not args.no_extras:
        out["extras"] = extras(args)
    return out


def single_variant(nx, n0, a, chi, precision, steps, tune_effort=0, integrator="euler",
                   noise=None):
    """GCell-updates/s of one single-instance configuration (autotuned); with
    integrator="rk2" an update is one two-stage Runge-Kutta step, with noise
    (dict sigma0, amp, seed) the agar field is redrawn at every step."""
    import numpy as np
    import torch
    from paper_1301_5058_amd import workload
    from paper_1301_5058_amd.solver import Solver
    b, n, s = workload.fields(nx, nx, n0, a, 0)
    dt = workload.config_dt(b, n, s)
    if precision == "fp64":
        b, n, s = (x.astype(np.float64) for x in (b, n, s))
    stream = torch.cuda.current_stream()
    S = Solver(nx, nx, dt=dt, chi=chi, precision=precision, b_thr=0.5 * n0, stream=stream,
               integrator=integrator, noise=noise)
    if noise is None:
        S.set_fields(*(torch.from_numpy(x).cuda() for x in (b, n, s)))
    else:
        S.set_fields(*(torch.from_numpy(x).cuda() for x in (b, n)))
    S.autotune(effort=tune_effort, use_cache=True)
    T, rows, pf = S.tuning()
    waves = S.strip_waves()
    S.step(100)
    ms = timed_run(S, stream, steps)
    lm = launch_probe(S, stream, 20)
    ops = OPS_PER_RK2_UPDATE if integrator == "rk2" else OPS_PER_CELL_UPDATE
    nbytes = None
    if noise is not None:
        ops += OPS_PER_NOISE_DRAW
        nbytes = BYTES_PER_CELL_LAUNCH_NOISE[precision]
    rl, other = roofline(precision, nx * nx, T, lm, ops, nbytes)
    S.close()
    return {"gcell_s": round(nx * nx * steps / (ms / 1e3) / 1e9, 2), "steps": steps,
            "integrator": integrator, "noise": noise is not None, "tsteps": T, "rows": rows,
            "prefetch": pf, "waves_per_strip": waves,
            "launch_us": round(lm * 1e3, 2), "roofline_bound": rl["bound"],
            "roofline_frac": rl["frac"], "other_bound": other["bound"],
            "other_frac": other["frac"]}


def hires(steps):
    """The 16384^2 grid (n0 = 0.35, chi = 2, a = 0.5).  Its 512^2 companion run
    in the same kernel configuration is checked against the oracle by the GPU
    tests (tests/test_parity_gpu.py), not here."""
    import torch
    from paper_1301_5058_amd import workload
    from paper_1301_5058_amd.solver import Solver
    c = workload.HIRES_16384
    b, n, s = workload.fields(c["nx"], c["ny"], c["n0"], c["a"], c["seed"])
    dt = workload.config_dt(b, n, s)
    stream = torch.cuda.current_stream()
    S = Solver(c["nx"], c["ny"], dt=dt, chi=c["chi"], b_thr=0.5 * c["n0"], stream=stream)
    S.set_fields(*(torch.from_numpy(x).cuda() for x in (b, n, s)))
    del b, n, s
    S.autotune(effort=0, use_cache=True)
    T, rows, pf = S.tuning()
    waves = S.strip_waves()
    series = torch.zeros((steps // SAMPLE_EVERY + 2, 5), dtype=torch.float64, device="cuda")
    ms = timed_run(S, stream, steps, series)
    d = series[steps // SAMPLE_EVERY - 1].cpu().numpy()
    S.close()
    res = {"nx": c["nx"], "steps": steps, "gcell_s": round(c["nx"] * c["ny"] * steps / (ms / 1e3) / 1e9, 2),
           "tsteps": T, "rows": rows, "prefetch": pf, "waves_per_strip": waves,
           "seconds": round(ms / 1e3, 3),
           "final_envelope_radius": float(d[3]), "final_area_radius": float(d[4])}
    return res


def sweep(steps=30000, every=100):
    """The 256-instance parameter sweep, in the batch's tuned launch mode."""
    import numpy as np
    import torch
    from paper_1301_5058_amd import workload
    from paper_1301_5058_amd.batch import Batch
    from paper_1301_5058_amd.surrogate import Surrogate
    insts = workload.sweep()
    descs, cells = [], 0
    t0 = time.perf_counter()
    B = None
    fields = []
    for d in insts:
        b, n, s = workload.fields(d["nx"], d["ny"], d["n0"], d["a"], d["seed"])
        dt = workload.config_dt(b, n, s)
        descs.append(dict(nx=d["nx"], ny=d["ny"], dt=dt, chi=d["chi"], b_thr=0.5 * d["n0"]))
        fields.append((b, n, s))
        cells += d["nx"] * d["ny"]
    B = Batch(descs, max_samples=steps // every + 1)
    for k, (b, n, s) in enumerate(fields):
        B.set_fields(k, b, n, s)
    del fields
    setup = time.perf_counter() - t0
    B.autotune(every, effort=0)
    T, rows, pf, _ = B.tuning()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    B.run(steps, every)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    lo = np.full(len(insts), 24.0)
    hi = np.array([0.8 * d["nx"] / 2 for d in insts])
    v, npts = B.fit_velocity(lo, hi, radius="area")
    ve, _ = B.fit_velocity(lo, hi, radius="envelope")
    B.close()
    S = Surrogate(len(insts))  # only for the library's closed-form speed bound (ks_cbar)
    cb = S.cbar(np.array([[d["n0"], d["chi"], d["a"]] for d in insts])).astype(np.float64)
    S.close()
    ok = np.isfinite(v)
    return {"instances": len(insts), "cells": cells, "steps": steps, "tsteps": T,
            "prefetch": pf, "seconds": round(ms / 1e3, 3),
            "gcell_s": round(cells * steps / (ms / 1e3) / 1e9, 2),
            "instances_per_s": round(len(insts) / (ms / 1e3), 2),
            "setup_s": round(setup, 2), "velocities_fitted": int(ok.sum()),
            "v_over_cbar_median": float(np.median(v[ok] / cb[ok])),
            "v_envelope_over_area_median": float(np.nanmedian(ve / v))}


def extras(args):
    from paper_1301_5058_amd import velocity_map
    ex = {}
    ex["fp64_4096"] = single_variant(4096, 0.5, 0.5, 1.0, "fp64", 5000)
    progress("fp64 4096^2: %s" % ex["fp64_4096"])
    ex["chi0_4096_fp32"] = single_variant(4096, 0.5, 0.5, 0.0, "fp32", 20000)
    progress("chi=0 4096^2: %s" % ex["chi0_4096_fp32"])
    ex["rk2_4096_fp32"] = single_variant(4096, 0.5, 0.5, 1.0, "fp32", 20000, integrator="rk2")
    progress("rk2 4096^2: %s" % ex["rk2_4096_fp32"])
    ex["rk2_4096_fp64"] = single_variant(4096, 0.5, 0.5, 1.0, "fp64", 4000, integrator="rk2")
    progress("rk2 fp64 4096^2: %s" % ex["rk2_4096_fp64"])
    # the paper's agar noise: sigma redrawn at every cell and step (Philox4x32-10)
    ex["noise_4096_fp32"] = single_variant(4096, 0.5, 0.5, 1.0, "fp32", 20000,
                                           noise=NOISE_4096)
    progress("noise 4096^2: %s" % ex["noise_4096_fp32"])
    ex["hires_16384"] = hires(20000)
    progress("16384^2: %s" % ex["hires_16384"])
    ex["sweep_256"] = sweep()
    progress("sweep: %s" % ex["sweep_256"])
    ex["velocity_map"] = velocity_map.run_velocity_map()
    progress("velocity map: %s" % ex["velocity_map"])
    ex["front1d"] = front1d_speeds()
    progress("1-D fronts: %s" % ex["front1d"])
    ex["paper_sets_2048"] = paper_sets()
    progress("paper sets: %s" % ex["paper_sets_2048"])
    return ex


def paper_sets():
    """The paper's 2-D figure sets (Sec. 3) at 2048^2 on L = 680: RK2 with sigma
    redrawn at every cell and step, each column to its captions' last time;
    envelope radii, the high/low sensitivity ratio and the shape at that time."""
    from paper_1301_5058_amd import colony, workload
    out, cells_steps, gpu_s = {}, 0.0, 0.0
    for name in workload.PAPER_SETS:
        res, _ = colony.run_set(name)
        cols = []
        for c in res["columns"]:
            i, r = c["info"], c["snapshots"][-1]
            cells_steps += i["cells"] ** 2 * i["steps"]
            gpu_s += i["gpu_s"]
            cols.append({"chi0": i["chi"], "dt": i["dt"], "steps": i["steps"], "t": round(r["t"], 2),
                         "envelope_speed": None if i["speed"] is None else round(i["speed"], 5),
                         "r_env": round(r["r_env"], 2), "compactness": round(r["compactness"], 3),
                         "axis_diag": round(r["axis_diag"], 3),
                         "arcs_half_r_env": r["rings"][0]["arcs"],
                         "b_centre_over_peak": round(r["b_centre"] / r["b_peak"], 3),
                         "tuning": i["tuning"]})
        out[name] = {"sigma0": res["sigma0"], "n0": res["n0"], "columns": cols,
                     "r_env_ratio": [round(v, 3) for v in res["r_env_ratio"]]}
    return {"cells": workload.PAPER_2D["cells"], "length": workload.PAPER_2D["length"],
            "gpu_s": round(gpu_s, 2), "gcell_steps_s": round(cells_steps / gpu_s * 1e-9, 1),
            "sets": out}


def front1d_speeds():
    """The 1-D front experiment of Sec. 4.2: 30 (n0, chi0) grids in one batch,
    front speeds against the closed-form bound c-bar and the threshold speed
    c* of the scalar front equation."""
    from paper_1301_5058_amd import front1d
    r = front1d.run_front1d()
    v1, v2 = r["velocity_halves"]
    spread = resolution_spread(r["cells"])
    # "steady": the speeds over the two halves of the window agree within 10 %
    # (a travelling front); otherwise the window speed is the mean of a
    # transient (strong chemotaxis bursts ahead and decelerates, poor nutrient
    # stalls).  "resolution_spread": how far the FP64 oracle's speed on this
    # grid lies from its speed on the finest grid of its resolution study
    # (tests/golden/front1d_resolution.txt; null where the study has no row);
    # "resolved": that spread is below 2 %.  "above_cbar": faster than c-bar
    # by more than that spread plus the 1 % FP32 / FP64 bar.
    rows = []
    for p, v, st, a, b, cb, cs, te in zip(r["points"], r["velocity"], r["steady"], v1, v2,
                                          r["cbar"], r["cstar"], r["t_end"]):
        sp = spread.get((round(p[0], 2), round(p[1], 1)))
        rows.append({"n0": p[0], "chi0": p[1], "v": round(float(v), 5), "steady": bool(st),
                     "v_halves": [round(float(a), 5), round(float(b), 5)],
                     "t_end": round(float(te), 5),
                     "resolution_spread": None if sp is None else round(sp, 5),
                     "resolved": None if sp is None else bool(sp <= 0.02),
                     "above_cbar": bool(v > cb * (1.0 + 0.01 + (sp or 0.0))),
                     "cbar": round(float(cb), 5), "cstar": round(float(cs), 5),
                     "v_over_cbar": round(float(v / cb), 4),
                     "v_over_cstar": round(float(v / cs), 4)})
    return {"cells": r["cells"], "steps": r["steps"], "window": list(r["window"]),
            "gpu_s": round(r["gpu_s"], 3), "wall_s": round(r["wall_s"], 3), "fronts": rows}


def resolution_spread(cells):
    """{(n0, chi0): |v(cells) - v(finest)| / v(finest)} from the oracle's
    resolution study of the 1-D experiment (a text table in tests/golden)."""
    path = os.path.join(ROOT, "tests", "golden", "front1d_resolution.txt")
    tab = {}
    try:
        for line in open(path):
            if line.startswith("#") or not line.strip():
                continue
            f = line.split()
            tab.setdefault((round(float(f[0]), 2), round(float(f[1]), 1)), {})[int(f[2])] = \
                float(f[7])
    except OSError:
        return {}
    out = {}
    for key, by_cells in tab.items():
        finest = max(by_cells)
        if cells in by_cells and finest > cells and by_cells[finest] > 0:
            out[key] = abs(by_cells[cells] - by_cells[finest]) / by_cells[finest]
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500,
                    help="benchmark steps of %d time steps + diagnostics each" % SAMPLE_EVERY)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--quick-tune", action="store_true")
    ap.add_argument("--copy-ref-mib", type=int, default=0)
    ap.add_argument("--tuning", default="",
                    help="T,ROWS,PF,WAVES: run this configuration (profiling runs)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: the solver runs on one GPU; --gpus %d is not supported "
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
