"""Envelope-velocity maps: batched solver sweeps, the learned surrogate, and
the routing between them.

A point is (n0, chi, a): initial nutrient, chemotactic strength (receptor law)
and agar-noise amplitude.  Its velocity is measured by running the solver on
a side x side grid (512^2 by default) from the seeded inoculum and fitting
the slope of the radius over the fixed window [4 r0, 102.4] cells
(kb_fit_velocity).  The grid is twice the window's reach so that its walls
do not change the speed: over this window a 512^2 grid agrees with a 2048^2
one within the seed-to-seed spread, while a 256^2 grid, whose walls the
window nearly touches, is up to a fifth slower for slow colonies.  The
surrogate answers points inside the convex hull of its training inputs; the
others go to the batched solver.  This module only chooses instances and
moves arrays; the solver, the fit, the network and the hull test run in
libkc.so.
"""
import math
import time

import numpy as np
import torch

from . import workload
from .batch import Batch
from .surrogate import Surrogate, he_uniform, hull_facets

R0 = 6.0
SAMPLE_EVERY = 100


WINDOW = (4.0 * R0, 0.8 * 256 / 2.0)  # radii fitted, in cells


def window(h=1.0):
    return WINDOW[0] * h, WINDOW[1] * h


def solver_velocities(points, side, steps, seeds=(0,), tune=True, max_batch=1024,
                      radius="area"):
    """Velocity of every (point, seed) pair: returns (v [m, len(seeds)], npts, gpu_seconds).

    gpu_seconds is the device time of the runs and fits (events on the batch
    stream), not the host-side generation of the initial fields.  The radius
    window is WINDOW on every grid."""
    points = np.asarray(points, dtype=np.float64)
    m = len(points)
    pairs = [(i, s) for i in range(m) for s in seeds]
    v = np.full((m, len(seeds)), np.nan)
    npts = np.zeros((m, len(seeds)), dtype=np.int32)
    lo, hi = window()
    gpu_s = 0.0
    for c0 in range(0, len(pairs), max_batch):
        chunk = pairs[c0:c0 + max_batch]
        descs, fields = [], []
        for (i, s) in chunk:
            n0, chi, a = points[i]
            b, n, sg = workload.fields(side, side, n0, a, int(s), r0=R0)
            dt = workload.config_dt(b, n, sg)
            descs.append(dict(nx=side, ny=side, dt=dt, chi=chi, b_thr=0.5 * n0))
            fields.append((b, n, sg))
        B = Batch(descs, max_samples=steps // SAMPLE_EVERY + 1)
        for k, (b, n, sg) in enumerate(fields):
            B.set_fields(k, b, n, sg)
        if tune:
            B.autotune(SAMPLE_EVERY, effort=0)
        st = torch.cuda.current_stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(st)
        B.run(steps, SAMPLE_EVERY)
        vv, nn = B.fit_velocity(lo, hi, radius=radius)
        e1.record(st)
        torch.cuda.synchronize()
        gpu_s += e0.elapsed_time(e1) / 1e3
        for k, (i, s) in enumerate(chunk):
            v[i, seeds.index(s)] = vv[k]
            npts[i, seeds.index(s)] = nn[k]
        B.close()
    return v, npts, gpu_s


class VelocityMap:
    """Surrogate trained on solver velocities, with solver fallback outside its hull."""

    IN_SHIFT = (0.75, 1.0, 0.3)
    IN_SCALE = (0.45, 1.0, 0.2)

    def __init__(self, max_points=1 << 19, seed=0):
        self.S = Surrogate(max_points)
        self.S.set_params(he_uniform(seed))
        self.trained = False

    # full-batch Adam, stepped learning rate (iterations, rate)
    SCHEDULE = ((6000, 3e-3), (6000, 1e-3), (6000, 3e-4), (4000, 1e-4))

    def fit(self, X, v, schedule=SCHEDULE):
        """Train on velocities v > 0 at points X in log-target mode (the loss
        weighs relative errors; velocities span more than a decade)."""
        X = np.asarray(X, dtype=np.float32)
        v = np.asarray(v, dtype=np.float32)
        ok = np.isfinite(v) & (v > 0)
        X, v = X[ok], v[ok]
        lv = np.log(v.astype(np.float64))
        self.S.set_normalization(self.IN_SHIFT, self.IN_SCALE, float(np.mean(lv)),
                                 float(np.std(lv) + 1e-12), log_target=True)
        loss = None
        for iters, lr in schedule:
            loss = self.S.train(X, v, iters=iters, batch=len(X), lr=lr)
        self.S.set_hull(hull_facets(X.astype(np.float64)), tol=1e-6)
        self.trained = True
        return loss

    def query(self, X, side, steps, seeds=(0,)):
        """Velocities of X: surrogate inside the hull, solver outside.

        Returns (v, inside mask, timing dict)."""
        X = np.asarray(X, dtype=np.float32)
        st = torch.cuda.current_stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e0.record(st)
        inside = self.S.inside(X)
        v = self.S.predict(X)
        e1.record(st)
        torch.cuda.synchronize()
        sur_s = e0.elapsed_time(e1) / 1e3
        host_s = time.perf_counter() - t0
        out = v.astype(np.float64)
        fb = np.nonzero(~inside)[0]
        solver_s = 0.0
        if len(fb):
            vs, _, solver_s = solver_velocities(X[fb].astype(np.float64), side, steps, seeds)
            out[fb] = np.nanmean(vs, axis=1)
        return out, inside, dict(surrogate_gpu_s=sur_s, surrogate_wall_s=host_s,
                                 fallback_points=int(len(fb)), fallback_gpu_s=solver_s)


# ---------------------------------------------------------------------------
# The velocity-map workload: (n0, chi, a) in [0.3, 1.2] x [0, 2] x [0.1, 0.5]
# ---------------------------------------------------------------------------
BOX_LO = np.array([0.3, 0.0, 0.1])
BOX_HI = np.array([1.2, 2.0, 0.5])


def design_grid(per_axis=16):
    """Full-factorial training design (per_axis^3 points, faces included, so the
    hull of the design is the whole box)."""
    ax = [np.linspace(BOX_LO[i], BOX_HI[i], per_axis) for i in range(3)]
    g = np.stack(np.meshgrid(*ax, indexing="ij"), -1).reshape(-1, 3)
    return g


def run_velocity_map(side=512, steps=8000, per_axis=16, held_out=64, ref_seeds=(101, 102, 103, 104),
                     query=512, band=256, seed=7, ref_side_large=2048, train_seeds=(0, 1),
                     log=None):
    """Train the surrogate on solver velocities, compare it on held-out points
    with the seed-averaged solver (the reference velocities), and time a query
    map with fallback.  With ref_side_large the held-out references are also
    taken on that larger grid over the same radius window (no wall within
    reach), which shows what the training grid's walls do to the velocities.

    Returns a dict of the measurements (all velocities by the area radius)."""
    rng = np.random.default_rng(seed)
    out = dict(protocol=dict(side=side, steps=steps, sample_every=SAMPLE_EVERY, radius="area",
                             window=list(window()), box_lo=BOX_LO.tolist(),
                             box_hi=BOX_HI.tolist()))
    # 1. training velocities from the batched solver (mean over train_seeds per point)
    X = design_grid(per_axis)
    t0 = time.perf_counter()
    # the mean over train_seeds agar fields: the per-seed spread (about 1 %) is
    # noise the network would otherwise fit
    v, npts, gpu_train = solver_velocities(X, side, steps, seeds=tuple(train_seeds))
    v = np.nanmean(v, axis=1)
    if log:
        log("training velocities: %d points" % len(X))
    host_train = time.perf_counter() - t0
    ok = np.isfinite(v)
    out["train"] = dict(points=int(len(X)), seeds=len(train_seeds), finite=int(ok.sum()),
                        solver_gpu_s=round(gpu_train, 3), wall_s=round(host_train, 2),
                        solver_pts_per_s=round(len(X) * len(train_seeds) / gpu_train, 2))
    # 2. surrogate training on the GPU
    vm = VelocityMap()
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    loss = vm.fit(X[ok], v[ok])
    e1.record(st)
    torch.cuda.synchronize()
    out["fit"] = dict(iters=sum(i for i, _ in vm.SCHEDULE), batch="full", target="log v",
                      final_loss=loss, gpu_s=round(e0.elapsed_time(e1) / 1e3, 3))
    # 3. held-out reference: random interior points, solver averaged over seeds
    H = BOX_LO + (BOX_HI - BOX_LO) * rng.uniform(0.02, 0.98, (held_out, 3))
    vr, _, gpu_ref = solver_velocities(H, side, steps, seeds=tuple(ref_seeds))
    if log:
        log("held-out references on %d^2" % side)
    vref = np.nanmean(vr, axis=1)
    spread = np.nanstd(vr, axis=1) / vref
    pred = vm.S.predict(H.astype(np.float32)).astype(np.float64)
    rel = np.abs(pred - vref) / vref
    # the closed-form bound with one fitted scale (what the method gives without the network)
    cb_tr = vm.S.cbar(X[ok].astype(np.float32)).astype(np.float64)
    scale = float(np.sum(cb_tr * v[ok]) / np.sum(cb_tr * cb_tr))
    cb_h = vm.S.cbar(H.astype(np.float32)).astype(np.float64)
    rel_cb = np.abs(scale * cb_h - vref) / vref
    out["held_out"] = dict(points=int(held_out), seeds=len(ref_seeds),
                           ref_seed_spread_median=float(np.median(spread)),
                           surrogate_rel_err_median=float(np.median(rel)),
                           surrogate_rel_err_p95=float(np.quantile(rel, 0.95)),
                           surrogate_rel_err_max=float(np.max(rel)),
                           surrogate_within_2pct=float(np.mean(rel <= 0.02)),
                           scaled_cbar_rel_err_median=float(np.median(rel_cb)),
                           scaled_cbar_rel_err_p95=float(np.quantile(rel_cb, 0.95)),
                           cbar_scale=scale, ref_gpu_s=round(gpu_ref, 3))
    if ref_side_large:
        vl, _, gpu_l = solver_velocities(H, ref_side_large, steps, seeds=tuple(ref_seeds),
                                         max_batch=64)
        vlarge = np.nanmean(vl, axis=1)
        if log:
            log("held-out references on %d^2" % ref_side_large)
        rel_l = np.abs(pred - vlarge) / vlarge
        wall = (vref - vlarge) / vlarge
        out["held_out_large"] = dict(side=int(ref_side_large), points=int(held_out),
                                     seeds=len(ref_seeds),
                                     ref_seed_spread_median=float(np.median(
                                         np.nanstd(vl, axis=1) / vlarge)),
                                     training_grid_vs_large_median=float(np.median(wall)),
                                     training_grid_vs_large_max_abs=float(np.max(np.abs(wall))),
                                     surrogate_rel_err_median=float(np.median(rel_l)),
                                     surrogate_rel_err_p95=float(np.quantile(rel_l, 0.95)),
                                     surrogate_rel_err_max=float(np.max(rel_l)),
                                     surrogate_within_2pct=float(np.mean(rel_l <= 0.02)),
                                     ref_gpu_s=round(gpu_l, 3))
    # 4. query map: query x query (n0, chi) at a = 0.3 inside the box, plus a band outside
    n0q, chq = np.meshgrid(np.linspace(BOX_LO[0], BOX_HI[0], query),
                           np.linspace(BOX_LO[1], BOX_HI[1], query), indexing="ij")
    Q = np.stack([n0q.ravel(), chq.ravel(), np.full(query * query, 0.3)], 1)
    nb = int(round(np.sqrt(band)))
    bn, bc = np.meshgrid(np.linspace(1.21, 1.4, nb), np.linspace(2.01, 2.5, nb), indexing="ij")
    Bq = np.stack([bn.ravel(), bc.ravel(), np.full(nb * nb, 0.3)], 1)
    allq = np.concatenate([Q, Bq], 0)
    vals, inside, tm = vm.query(allq, side, steps)
    total_s = tm["surrogate_gpu_s"] + tm["fallback_gpu_s"]
    out["query"] = dict(points=int(len(allq)), inside=int(inside.sum()),
                        fallback=tm["fallback_points"], surrogate_gpu_s=round(tm["surrogate_gpu_s"], 5),
                        fallback_gpu_s=round(tm["fallback_gpu_s"], 3),
                        pts_per_s_with_fallback=round(len(allq) / total_s, 1),
                        pts_per_s_plain_solver=out["train"]["solver_pts_per_s"],
                        speedup=round((len(allq) / total_s) / out["train"]["solver_pts_per_s"], 1))
    vm.S.close()
    return out


def main(argv=None):
    import argparse
    import json
    import os
    import sys
    ap = argparse.ArgumentParser(description="velocity surrogate: training, held-out check, query map")
    ap.add_argument("--ref-side-large", type=int, default=2048,
                    help="also take the held-out references on this larger grid (0: no)")
    ap.add_argument("--json", default=None)
    a = ap.parse_args(argv)
    here = os.path.dirname(os.path.abspath(__file__))
    os.environ.setdefault("KC_AUTOTUNE_CACHE", os.path.join(here, "tuning", "gfx950.jsonl"))
    def log(msg):
        print("[velocity map] " + msg, file=sys.stderr, flush=True)

    out = run_velocity_map(ref_side_large=a.ref_side_large, log=log)
    txt = json.dumps(out, indent=1)
    print(txt, flush=True)
    if a.json:
        with open(a.json, "w") as f:
            f.write(txt)
    return 0


if __name__ == "__main__":
    import sys
    sys.exit(main())
