"""Envelope-velocity maps: batched solver sweeps, the learned surrogate, and
the routing between them.

A point is (n0, chi, a): initial nutrient, chemotactic strength (receptor law)
and agar-noise amplitude.  Its velocity is measured by running the solver on
a side x side grid from the seeded inoculum and fitting the slope of the
envelope radius over the window [4 r0, 0.8 side/2] (kb_fit_velocity).  The
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


def window(side, h=1.0):
    return 4.0 * R0 * h, 0.8 * side * h / 2.0


def solver_velocities(points, side, steps, seeds=(0,), tune=True, max_batch=1024,
                      radius="area"):
    """Velocity of every (point, seed) pair: returns (v [m, len(seeds)], npts, gpu_seconds).

    gpu_seconds is the device time of the runs and fits (events on the batch
    stream), not the host-side generation of the initial fields."""
    points = np.asarray(points, dtype=np.float64)
    m = len(points)
    pairs = [(i, s) for i in range(m) for s in seeds]
    v = np.full((m, len(seeds)), np.nan)
    npts = np.zeros((m, len(seeds)), dtype=np.int32)
    lo, hi = window(side)
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

    def fit(self, X, v, iters=4000, batch=512, lr=2e-3):
        X = np.asarray(X, dtype=np.float32)
        v = np.asarray(v, dtype=np.float32)
        ok = np.isfinite(v)
        X, v = X[ok], v[ok]
        self.S.set_normalization(self.IN_SHIFT, self.IN_SCALE, float(np.mean(v)),
                                 float(np.std(v) + 1e-12))
        loss = self.S.train(X, v, iters=iters, batch=min(batch, len(X)), lr=lr)
        self.S.set_hull(hull_facets(X.astype(np.float64)), tol=1e-9)
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
