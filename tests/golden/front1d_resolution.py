"""Grid-resolution study of the one-dimensional front experiment (Sec. 4.2,
system velo-system-1d) with the FP64 oracle only.

    python tests/golden/front1d_resolution.py [--jobs 5] [--cells 400,800,1600,3200] [--points hard|all]

For each (n0, chi0) below (`hard`: the six points whose fronts are fastest,
burst or stall; `all`: the experiment's 30) and each grid of `cells` cells on
[0, 20] the oracle
runs the experiment's set-up (constant sensitivity, sigma = 1, the cut
inoculum 0.71 exp(-x^2 / 6.25), forward Euler at the experiment's time step
0.2 h^2 / max(D_n, sigma0 n0 (n0 + b_M)(1 + chi0 n0)), which scales with h^2)
and samples the front position -- the largest x of a cell with
b >= min(0.5, n0 / 2) --
at the same physical times on every grid (every 100 steps of the 400-cell
grid).  A run stops once the front has passed x = 17.5 or at the time a front
moving at a quarter of the bound c-bar of Sec. 4.1 needs to cross [7.5, 17].
Written out per run: the time step, the final time, the final front position,
the least-squares speed over the window x in [9, 17] and over its two halves
(NaN when fewer than three samples fall in it), and the speed over the last
quarter of the run.  Rows are merged into front1d_resolution.txt beside this
script (a new row replaces the one with the same n0, chi0 and cells); the GPU
tests compare the library's 400-cell runs with the rows of the hard points,
and the benchmark flags a front as resolved when its 400-cell speed is within
1 % of the speed on the finest grid of the table.
"""
import argparse
import math
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

POINTS = [(4.0, 10.0), (4.0, 5.0), (3.0, 10.0), (2.0, 2.5), (0.71, 0.0), (0.35, 0.0)]
ALL_POINTS = [(n0, chi) for n0 in (0.35, 0.71, 1.07, 2.0, 3.0, 4.0)
              for chi in (0.0, 1.0, 2.5, 5.0, 10.0)]
CELLS = (400, 800, 1600, 3200)
LENGTH, B_MAX, R0, CUT, SIGMA0 = 20.0, 0.71, 2.5, 3.0, 1.0
WINDOW = (9.0, 17.0)
BASE_CELLS, BASE_EVERY = 400, 100


def fields(cells, n0):
    h = LENGTH / cells
    x = (np.arange(cells, dtype=np.float64) + 0.5) * h
    b = B_MAX * np.exp(-x * x / (R0 * R0))
    b[x > CUT * R0] = 0.0
    b = b.astype(np.float32).astype(np.float64)[None, :]
    n = np.full((1, cells), float(np.float32(n0)))
    s = np.full((1, cells), float(np.float32(SIGMA0)))
    return b, n, s


def time_step(cells, n0, chi):
    h = LENGTH / cells
    m = max(1.0, SIGMA0 * n0 * (n0 + B_MAX) * (1.0 + chi * n0))
    return float(np.float32(0.2 * h * h / m))


def slope(t, r, lo, hi):
    import oracle
    sel = (r >= lo) & (r <= hi)
    if sel.sum() < 3:
        return math.nan
    return float(oracle.fit_velocity(t[sel], r[sel], lo, hi)[0])


def run_one(args):
    n0, chi, cells = args
    import oracle
    oracle.set_threads(1)
    h = LENGTH / cells
    dt = time_step(cells, n0, chi)
    every = BASE_EVERY * (cells // BASE_CELLS) ** 2
    t_end = 4.0 * (WINDOW[1] - CUT * R0) / oracle.cbar(n0, chi)
    b, n, s = fields(cells, n0)
    ts, rs = [], []
    k = 0
    t0 = time.perf_counter()
    while True:
        b, n = oracle.run(b, n, s, h, dt, every, chi=chi, chi_law=1)
        k += every
        t = k * dt
        r = oracle.diag(b, n, h, min(0.5, 0.5 * n0), cx=-0.5, cy=0.0)[2]
        ts.append(t)
        rs.append(r)
        if r >= WINDOW[1] + 0.5 or t >= t_end:
            break
    ts, rs = np.array(ts), np.array(rs)
    mid = 0.5 * (WINDOW[0] + WINDOW[1])
    q = ts >= 0.75 * ts[-1]
    v_last = float(np.polyfit(ts[q], rs[q], 1)[0]) if q.sum() >= 3 else math.nan
    return dict(n0=n0, chi=chi, cells=cells, dt=dt, steps=k, t_end=float(ts[-1]),
                r_end=float(rs[-1]), v=slope(ts, rs, *WINDOW), v1=slope(ts, rs, WINDOW[0], mid),
                v2=slope(ts, rs, mid, WINDOW[1]), v_last=v_last, cbar=float(oracle.cbar(n0, chi)),
                seconds=time.perf_counter() - t0)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=5)
    ap.add_argument("--cells", default=",".join(str(c) for c in CELLS))
    ap.add_argument("--points", choices=("hard", "all"), default="hard")
    a = ap.parse_args()
    cells = [int(c) for c in a.cells.split(",")]
    points = POINTS if a.points == "hard" else ALL_POINTS
    jobs = [(n0, chi, c) for c in cells for (n0, chi) in points]
    # longest runs first
    jobs.sort(key=lambda j: -j[2])
    rows = []
    with ProcessPoolExecutor(a.jobs) as ex:
        for r in ex.map(run_one, jobs):
            print("n0 %.2f chi0 %4.1f cells %4d: v %.5g (halves %.5g %.5g), v/cbar %.4f, "
                  "r_end %.3f at t %.4g, %.0f s" % (r["n0"], r["chi"], r["cells"], r["v"], r["v1"],
                                                     r["v2"], r["v"] / r["cbar"], r["r_end"],
                                                     r["t_end"], r["seconds"]), flush=True)
            rows.append(r)
    out = os.path.join(HERE, "front1d_resolution.txt")
    cols = ("n0", "chi", "cells", "dt", "steps", "t_end", "r_end", "v", "v1", "v2", "v_last", "cbar")
    new = {(round(r["n0"], 2), round(r["chi"], 1), r["cells"]) for r in rows}
    if os.path.exists(out):
        for line in open(out):
            if line.startswith("#") or not line.strip():
                continue
            f = line.split()
            old = dict(zip(cols, [float(x) for x in f]))
            old["cells"], old["steps"] = int(f[2]), int(f[4])
            if (round(old["n0"], 2), round(old["chi"], 1), old["cells"]) not in new:
                rows.append(old)
    rows.sort(key=lambda r: (-r["n0"], -r["chi"], r["cells"]))
    with open(out, "w") as f:
        f.write("# Resolution study of the 1-D front experiment of Sec. 4.2 (system velo-system-1d),\n"
                "# FP64 oracle only; written by tests/golden/front1d_resolution.py.\n"
                "# Columns: n0 chi0 cells dt steps t_end r_end v v_first_half v_second_half "
                "v_last_quarter cbar\n"
                "# v: least-squares front speed over x in [9, 17]; halves [9, 13], [13, 17];\n"
                "# cbar: the bound of Sec. 4.1 (eqs. c-bar-chi0, c-bar-0) at sigma0 = 1.\n")
        for r in rows:
            f.write("%.2f %.1f %d %.9g %d %.9g %.9g %.9g %.9g %.9g %.9g %.9g\n"
                    % (r["n0"], r["chi"], r["cells"], r["dt"], r["steps"], r["t_end"], r["r_end"],
                       r["v"], r["v1"], r["v2"], r["v_last"], r["cbar"]))
    print("wrote", out)


if __name__ == "__main__":
    main()
