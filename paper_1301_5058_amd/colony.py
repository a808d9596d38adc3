"""The paper's two-dimensional colony runs (Sec. 3, Figs. set1 - set4) at full
scale, and a description of each snapshot's shape.

    python -m paper_1301_5058_amd.colony [--sets set1,set3b] [--cells 2048]
                                         [--json OUT.json] [--png DIR]

Every run is one Solver on the paper's set-up (the recipe is in workload.py:
N = 2048, L = 680, inoculum b_M exp(-(x^2+y^2)/6.25), uniform n0, sigma =
sigma0 (1 + Delta) redrawn per cell and step, two-stage Runge-Kutta); all
time stepping happens in libkc.so.  At each caption time the bacterial field
is copied to the host and described by `morphology`:

  r_env        envelope radius: largest distance from the centre of a cell
               with b >= b_thr (b_thr = n0 / 2)
  r_area       radius of the disk with the colony's area (cells with b >= b_thr)
  compactness  (r_area / r_env)^2: 1 for a disk, small for a branched colony
  rings        for rings of radius f r_env (f = 0.5, 0.75, 0.9): the fraction
               of the ring inside the colony ("cover") and the number of
               separate arcs it crosses ("arcs"; a closed ring is 1 arc, cover 1)
  axis_diag    the colony's reach along the grid axes over its reach along the
               diagonals (largest distance of a colony cell within pi/16 of
               the direction): 1 for a round envelope, sqrt 2 for a rhomboid
               with its corners on the axes (the grid artefact of the paper's
               coarsest mesh, Sec. 3.2)
  b_centre     b at the centre, b_peak its maximum (a depression at the centre
               shows as b_centre < b_peak)

and each run by its envelope speed: the least-squares slope of r_env(t) over
the caption times at which the envelope has not reached the wall.

The paper prints pictures, not numbers; what it states (faster envelopes with
chi0, branches merging into a disk at sigma0 = 4, n0 = 0.71, chi0 = 7.5, disks
at n0 = 1.07, sigma0 = 4) is read off these quantities.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

from . import workload

RING_FRACTIONS = (0.5, 0.75, 0.9)


def _ring(mask, cx, cy, rho):
    """(cover, arcs) of the circle of radius rho cells about (cx, cy), sampled at
    about four points per cell of arc length and read at the nearest cell."""
    ny, nx = mask.shape
    k = max(64, int(math.ceil(8.0 * math.pi * rho)))
    th = 2.0 * math.pi * (np.arange(k) + 0.5) / k
    x = np.clip(np.rint(cx + rho * np.cos(th)).astype(np.int64), 0, nx - 1)
    y = np.clip(np.rint(cy + rho * np.sin(th)).astype(np.int64), 0, ny - 1)
    on = mask[y, x]
    if on.all():
        return 1.0, 1
    # arcs = runs of consecutive samples inside, counted around the circle
    starts = on & ~np.roll(on, 1)
    return float(on.mean()), int(starts.sum())


def morphology(b, h, b_thr, cx=None, cy=None, rings=RING_FRACTIONS):
    """Shape of the colony {b >= b_thr} of one bacterial field [ny, nx] (cell
    width h; centre (cx, cy) in cell indices, default the grid's centre)."""
    b = np.asarray(b)
    ny, nx = b.shape
    cx = (nx - 1) / 2.0 if cx is None else float(cx)
    cy = (ny - 1) / 2.0 if cy is None else float(cy)
    mask = b.astype(np.float64) >= b_thr
    cells = int(mask.sum())
    jc, ic = int(round(cy)), int(round(cx))
    out = dict(cells=cells, b_peak=float(b.max()), b_centre=float(b[jc, ic]))
    if cells == 0:
        out.update(r_env=0.0, r_area=0.0, compactness=0.0, axis_diag=float("nan"),
                   rings=[dict(f=f, cover=0.0, arcs=0) for f in rings])
        return out
    jj, ii = np.nonzero(mask)
    dx, dy = ii - cx, jj - cy
    dist = np.hypot(dx, dy)
    d = dist.max()
    r_env = h * float(d)
    # angle from the nearest axis, in [0, pi/4]
    ax = np.arctan2(np.minimum(np.abs(dx), np.abs(dy)), np.maximum(np.abs(dx), np.abs(dy)))
    near_axis, near_diag = ax <= math.pi / 16, ax >= math.pi / 4 - math.pi / 16
    r_axis = float(dist[near_axis].max()) if near_axis.any() else 0.0
    r_diag = float(dist[near_diag].max()) if near_diag.any() else 0.0
    r_area = h * math.sqrt(cells / math.pi)
    out.update(r_env=r_env, r_area=r_area, compactness=(r_area / r_env) ** 2 if r_env > 0 else 1.0,
               axis_diag=r_axis / r_diag if r_diag > 0 else float("inf"))
    rr = []
    for f in rings:
        cover, arcs = _ring(mask, cx, cy, f * d)
        rr.append(dict(f=f, cover=cover, arcs=arcs))
    out["rings"] = rr
    return out


def envelope_speed(snapshots, half_side, wall=0.95):
    """Least-squares slope of r_env against t over the snapshots whose envelope
    has not reached `wall` of the half side (None with fewer than two)."""
    pts = [(r["t"], r["r_env"]) for r in snapshots if r["r_env"] < wall * half_side]
    if len(pts) < 2:
        return None
    t = np.array([p[0] for p in pts])
    r = np.array([p[1] for p in pts])
    tc = t - t.mean()
    return float(np.dot(tc, r - r.mean()) / np.dot(tc, tc))


def run_case(sigma0, n0, chi, times, dt_paper, cells=2048, length=680.0, seed=1,
             precision="fp32", keep_fields=False, log=None, chunk_cell_steps=5e12):
    """One run of the paper's set-up; returns (records, fields) with one record
    per caption time (fields: the FP32 bacterial field at each time, or [])."""
    import torch

    from .solver import Solver

    c = workload.PAPER_2D
    h = length / cells
    dt = workload.paper_dt(cells, length, sigma0, n0, dt_paper, amp=c["amp"], b_max=c["b_max"])
    b, n = workload.paper_fields(cells, length, n0, b_max=c["b_max"], r0=c["r0"], cut=c["cut"])
    if precision == "fp64":
        b, n = b.astype(np.float64), n.astype(np.float64)
    noise = dict(sigma0=sigma0, amp=c["amp"], seed=seed)
    b_thr = 0.5 * n0
    S = Solver(cells, cells, h=h, dt=dt, chi=chi, precision=precision, integrator="rk2",
               noise=noise, b_thr=b_thr)
    try:
        S.set_fields(torch.from_numpy(b).cuda(), torch.from_numpy(n).cuda())
        S.autotune(effort=0, use_cache=True)
        tuning = S.tuning() + (S.strip_waves(),)
        chunk = max(1, int(chunk_cell_steps / (cells * cells)))
        recs, keep = [], []
        done, gpu_ms = 0, 0.0
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        for t in times:
            k = int(round(t / dt))
            while done < k:
                # chunks of about half a minute of GPU time on the largest meshes
                m = min(k - done, chunk)
                e0.record(S.stream)
                S.step(m)
                e1.record(S.stream)
                e1.synchronize()
                gpu_ms += e0.elapsed_time(e1)
                done += m
                if log and done < k:
                    log("    ... step %d of %d" % (done, k))
            gb, gn = S.get_fields()
            tt, mass, nut, renv_dev, rarea_dev = S.diagnostics_all()
            r = morphology(gb, h, b_thr)
            bb, nn = gb.astype(np.float64), gn.astype(np.float64)
            snb = sigma0 * (1.0 + c["amp"]) * float(np.max(nn * bb))
            r.update(t_caption=t, t=tt, steps=k, mass=mass, nutrient=nut,
                     r_env_device=renv_dev, r_area_device=rarea_dev,
                     min_b=float(bb.min()), min_n=float(nn.min()), max_n=float(nn.max()),
                     # dt over the explicit bound with the largest sigma n b seen
                     dt_over_bound=dt * 4.0 * max(1.0, snb) / (h * h))
            recs.append(r)
            if keep_fields:
                keep.append(np.asarray(gb, dtype=np.float32))
            if log:
                log("  chi0=%-4g t=%7.1f steps=%7d r_env=%7.2f r_area=%7.2f compact=%.3f "
                    "axis/diag=%.3f arcs=%s cover=%s b_c/b_pk=%.3f/%.3f"
                    % (chi, tt, k, r["r_env"], r["r_area"], r["compactness"], r["axis_diag"],
                       "/".join("%d" % g["arcs"] for g in r["rings"]),
                       "/".join("%.2f" % g["cover"] for g in r["rings"]),
                       r["b_centre"], r["b_peak"]))
        info = dict(sigma0=sigma0, n0=n0, chi=chi, dt=dt, dt_paper=dt_paper, h=h, cells=cells,
                    seed=seed, precision=precision, tuning=list(tuning), steps=done,
                    gpu_s=gpu_ms * 1e-3,
                    gcell_s=cells * cells * done / (gpu_ms * 1e-3) * 1e-9 if gpu_ms > 0 else 0.0)
        for r in recs:
            r.update(chi=chi)
        info["speed"] = envelope_speed(recs, 0.5 * length)
        return dict(info=info, snapshots=recs), keep
    finally:
        S.close()


def run_set(name, cells=2048, length=680.0, seed=1, precision="fp32", keep_fields=False, log=None):
    """Both columns of one figure set (same noise seed for both sensitivities)."""
    s = workload.PAPER_SETS[name]
    cols, fields = [], []
    for chi in s["chi"]:
        if log:
            log("%s: sigma0=%g n0=%g chi0=%g" % (name, s["sigma0"], s["n0"], chi))
        res, f = run_case(s["sigma0"], s["n0"], chi, s["times"], s["dt"], cells=cells,
                          length=length, seed=seed, precision=precision,
                          keep_fields=keep_fields, log=log)
        cols.append(res)
        fields.append(f)
    lo, hi = cols[0]["snapshots"], cols[1]["snapshots"]
    ratio = [b["r_env"] / a["r_env"] if a["r_env"] > 0 else float("inf") for a, b in zip(lo, hi)]
    return dict(set=name, sigma0=s["sigma0"], n0=s["n0"], chi=list(s["chi"]), columns=cols,
                r_env_ratio=ratio), fields


def grid_study(name, chi, cells_list, length=680.0, seed=1, precision="fp32", keep_fields=False,
               log=None):
    """One column of a figure set on several meshes of the same square (the
    paper's grid-size check, Sec. 3.2: N = 1024 ... 8192 at sigma0 = 1,
    n0 = 0.71, chi0 = 5).  The step follows each mesh's explicit bound."""
    s = workload.PAPER_SETS[name]
    cols, fields = [], []
    for cells in cells_list:
        if log:
            log("%s chi0=%g on %d^2 cells (h = %.4f)" % (name, chi, cells, length / cells))
        res, f = run_case(s["sigma0"], s["n0"], chi, s["times"], s["dt"], cells=cells,
                          length=length, seed=seed, precision=precision,
                          keep_fields=keep_fields, log=log)
        cols.append(res)
        fields.append(f)
    return dict(set=name, sigma0=s["sigma0"], n0=s["n0"], chi=chi, cells=list(cells_list),
                columns=cols), fields


def save_png(path, columns, vmax=None, side=512):
    """Montage of a figure set: one column per sensitivity, one row per time,
    each field block-averaged to side x side and shown in grey (black = 0)."""
    from PIL import Image

    rows = len(columns[0])
    tiles = []
    for col in columns:
        out = []
        for f in col:
            k = max(1, f.shape[0] // side)
            g = f[: f.shape[0] // k * k, : f.shape[1] // k * k]
            g = g.reshape(g.shape[0] // k, k, g.shape[1] // k, k).mean(axis=(1, 3))
            out.append(g)
        tiles.append(out)
    top = vmax if vmax is not None else max(float(t.max()) for c in tiles for t in c) or 1.0
    th, tw = tiles[0][0].shape
    pad = 4
    img = np.full((rows * (th + pad) - pad, len(tiles) * (tw + pad) - pad), 255, np.uint8)
    for ci, c in enumerate(tiles):
        for ri, t in enumerate(c):
            v = np.clip(t / top, 0.0, 1.0)
            img[ri * (th + pad): ri * (th + pad) + th, ci * (tw + pad): ci * (tw + pad) + tw] = \
                (255.0 * v).astype(np.uint8)
    Image.fromarray(img).save(path)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--sets", default=",".join(workload.PAPER_SETS))
    ap.add_argument("--cells", type=int, default=workload.PAPER_2D["cells"])
    ap.add_argument("--length", type=float, default=workload.PAPER_2D["length"])
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--precision", default="fp32", choices=("fp32", "fp64"))
    ap.add_argument("--json", default=None, help="write the records here")
    ap.add_argument("--png", default=None, help="write one montage per set into this folder")
    ap.add_argument("--grid", default=None,
                    help="comma-separated mesh sizes: run the grid-size study instead of the sets")
    ap.add_argument("--grid-set", default="set1")
    ap.add_argument("--grid-chi", type=float, default=5.0)
    a = ap.parse_args(argv)
    here = os.path.dirname(os.path.abspath(__file__))
    os.environ.setdefault("KC_AUTOTUNE_CACHE", os.path.join(here, "tuning", "gfx950.jsonl"))

    def log(msg):
        print(msg, flush=True)

    t0 = time.time()
    out = []
    if a.grid:
        meshes = [int(v) for v in a.grid.split(",")]
        res, fields = grid_study(a.grid_set, a.grid_chi, meshes, length=a.length, seed=a.seed,
                                 precision=a.precision, keep_fields=a.png is not None, log=log)
        for c in res["columns"]:
            i = c["info"]
            log("  %d^2: dt=%.6g, %d steps in %.2f s of GPU time, %.1f GCell/s, tuning %s"
                % (i["cells"], i["dt"], i["steps"], i["gpu_s"], i["gcell_s"], tuple(i["tuning"])))
        if a.png:
            os.makedirs(a.png, exist_ok=True)
            save_png(os.path.join(a.png, "grid_%s.png" % a.grid_set), fields)
        out.append(res)
    for name in ([] if a.grid else a.sets.split(",")):
        res, fields = run_set(name, cells=a.cells, length=a.length, seed=a.seed,
                              precision=a.precision, keep_fields=a.png is not None, log=log)
        log("%s: r_env(chi0=%g) / r_env(chi0=%g) = %s" % (
            name, res["chi"][1], res["chi"][0], " ".join("%.2f" % r for r in res["r_env_ratio"])))
        for c in res["columns"]:
            i = c["info"]
            log("  chi0=%g: envelope speed %s, dt=%.6g (paper %.6g), %d steps in %.2f s of GPU "
                "time, %.1f GCell/s, tuning %s"
                % (i["chi"], "-" if i["speed"] is None else "%.4f" % i["speed"], i["dt"],
                   i["dt_paper"], i["steps"], i["gpu_s"], i["gcell_s"], tuple(i["tuning"])))
        if a.png:
            os.makedirs(a.png, exist_ok=True)
            save_png(os.path.join(a.png, "%s.png" % name), fields)
        out.append(res)
    if a.json:
        with open(a.json, "w") as f:
            json.dump(out, f, indent=1)
    log("all sets: %.1f s wall" % (time.time() - t0))
    return 0


if __name__ == "__main__":
    sys.exit(main())
