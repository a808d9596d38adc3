"""The one-dimensional front-speed experiment of Sec. 4.2 on the batched solver.

For every (n0, chi0) of the experiment one 1 x cells grid on [0, length] runs
the system velo-system-1d (constant sensitivity, sigma = sigma0): all
instances in one batch (kb_* calls), the front position sampled on the device
as the envelope radius about x = 0 (centre at cell index -1/2, threshold
b_thr = min(0.5, n0 / 2): Sec. 4.2 follows the point where b is about one
half, and n0 / 2 where the plateau n0 stays below that), and its velocity fitted on the device over the window of
front positions up to the front's own end time (its first sample past the
window, or the time a quarter-c-bar front needs to cross it).  The velocities
are compared with the
closed-form bound c-bar(n0, chi0) of Sec. 4.1 (ks_cbar) and with the threshold
speed c* of the scalar front equation (ks_cstar); the speeds over the
two halves of the window tell a steady front from one that still changes
speed (slow fronts that deplete the nutrient ahead of them decelerate).  This
module only
chooses instances and moves arrays; every computation runs in libkc.so.
"""
import math
import time

import numpy as np
import torch

from . import workload
from .batch import Batch
from .surrogate import Surrogate

SAMPLE_EVERY = 100


def instances(cells=None, n0s=None, chis=None):
    """(descriptors, fields) of the experiment's grid of (n0, chi0)."""
    c = workload.FRONT1D
    cells = int(cells or c["cells"])
    n0s = c["n0"] if n0s is None else n0s
    chis = c["chi"] if chis is None else chis
    h = c["length"] / cells
    descs, fields = [], []
    for n0 in n0s:
        for chi in chis:
            b, n, s = workload.front1d_fields(cells, c["length"], n0, c["b_max"], c["r0"], c["cut"],
                                              c["sigma0"])
            dt = workload.front1d_dt(cells, c["length"], n0, chi, c["b_max"], c["sigma0"])
            descs.append(dict(nx=cells, ny=1, h=h, dt=dt, chi=float(chi),
                              b_thr=workload.front1d_threshold(n0, c["threshold"]),
                              cx=-0.5, cy=0.0, n0=float(n0)))
            fields.append((b, n, s))
    return descs, fields


def speed_bounds(points, sigma0=1.0, threshold=False):
    """c-bar(n0, chi0) sqrt(sigma0) for rows (n0, chi0) from the library
    (ks_cbar); with threshold=True also the threshold speeds c* (ks_cstar)."""
    X = np.zeros((len(points), 3), dtype=np.float32)
    X[:, :2] = np.asarray(points, dtype=np.float32)
    S = Surrogate(max(1, len(points)))
    try:
        cb = S.cbar(X, sigma0).astype(np.float64)
        if threshold:
            return cb, S.cstar(X, sigma0).astype(np.float64)
        return cb
    finally:
        S.close()


def steps_needed(descs, cbar, reach, min_speed_frac=0.5):
    """Steps after which every front has passed `reach`, if it moves at least
    min_speed_frac of its bound (a multiple of SAMPLE_EVERY)."""
    t = max(reach / (min_speed_frac * cb) / d["dt"] for d, cb in zip(descs, cbar))
    return int(math.ceil(t / SAMPLE_EVERY)) * SAMPLE_EVERY


def run_front1d(cells=None, n0s=None, chis=None, steps=None):
    """Run the experiment; returns a dict with the velocities, the bounds and
    the device time."""
    c = workload.FRONT1D
    descs, fields = instances(cells, n0s, chis)
    pts = [(d["n0"], d["chi"]) for d in descs]
    cbar, cstar = speed_bounds(pts, c["sigma0"], threshold=True)
    lo, hi = c["window"]
    # A front's run ends at its first sample past hi + 1/2, or at the time a
    # front moving at a quarter of c-bar needs to cross from the inoculum's
    # edge to hi (a slow front that stalls ends there); its speed is fitted
    # over the samples up to that end.
    t_cap = 4.0 * (hi - c["cut"] * c["r0"]) / np.asarray(cbar, dtype=np.float64)
    if steps is None:
        steps = steps_needed(descs, cbar, hi)
        longest = max(tc / d["dt"] for tc, d in zip(t_cap, descs))
        steps = max(steps, int(math.ceil(longest / SAMPLE_EVERY)) * SAMPLE_EVERY)
    B = Batch(descs, chi_law="constant", max_samples=steps // SAMPLE_EVERY + 1)
    try:
        for k, (b, n, s) in enumerate(fields):
            B.set_fields(k, b, n, s)
        st = torch.cuda.current_stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e0.record(st)
        B.run(steps, SAMPLE_EVERY)
        series = B.series()
        t_end = np.empty(len(descs))
        for k in range(len(descs)):
            ts, rs = series[k, :, 0], series[k, :, 3]
            stop = np.nonzero((rs >= hi + 0.5) | (ts >= t_cap[k]))[0]
            t_end[k] = ts[stop[0]] if len(stop) else ts[-1]
        v, npts = B.fit_velocity(lo, hi, radius="envelope", t_max=t_end)
        mid = 0.5 * (lo + hi)
        v1, _ = B.fit_velocity(lo, mid, radius="envelope", t_max=t_end)
        v2, _ = B.fit_velocity(mid, hi, radius="envelope", t_max=t_end)
        e1.record(st)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
    finally:
        B.close()
    # a front is steady when its speeds over the two halves of the window agree
    steady = np.isfinite(v1) & np.isfinite(v2) & (np.abs(v1 - v2) <= 0.1 * np.abs(v))
    return dict(points=pts, velocity=v, samples=npts, cbar=cbar, cstar=cstar, steps=steps,
                velocity_halves=(v1, v2), steady=steady, t_end=t_end,
                dt=[d["dt"] for d in descs], cells=descs[0]["nx"], window=(lo, hi),
                gpu_s=e0.elapsed_time(e1) / 1e3, wall_s=wall, series=series)
