"""Python face of the batched sweep (kb_* calls of include/kb.h).

Batch wraps one kb_batch: many FP32 instances of the solver with their own
grid, time step, rates and agar field, advanced together by one launch per
time block; the envelope radius R(t), mass and nutrient of every
instance are sampled on the device, and fit_velocity() returns dR/dt per
instance.  Every computation happens in libkc.so.
"""
import ctypes
import math

import numpy as np
import torch

from . import native as N


class Batch:
    def __init__(self, instances, chi_law="receptor", max_samples=1024, stream=None):
        self.count = len(instances)
        arr = (N.KbInstance * self.count)()
        self.shapes = []
        for k, d in enumerate(instances):
            I = arr[k]
            I.nx, I.ny = int(d["nx"]), int(d["ny"])
            I.h, I.dt = float(d.get("h", 1.0)), float(d["dt"])
            I.D_n, I.theta = float(d.get("D_n", 1.0)), float(d.get("theta", 1.0))
            I.kappa, I.chi = float(d.get("kappa", 1.0)), float(d.get("chi", 0.0))
            I.b_thr = float(d.get("b_thr", 0.5))
            I.cx = math.nan if d.get("cx") is None else float(d["cx"])
            I.cy = math.nan if d.get("cy") is None else float(d["cy"])
            self.shapes.append((I.ny, I.nx))
        self.max_samples = int(max_samples)
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        h = ctypes.c_void_p()
        law = N.KC_CHI_RECEPTOR if chi_law == "receptor" else N.KC_CHI_CONSTANT
        N.check(N.lib().kb_create(self.count, arr, law, self.max_samples,
                                  ctypes.c_void_p(stream.cuda_stream), ctypes.byref(h)))
        self.h = h

    def _chk(self, code):
        return N.check(code, self.h, kind="kb")

    def set_fields(self, k, b, n, sigma):
        shape = self.shapes[k]
        keep = []
        ptrs = []
        mem = None
        for a in (b, n, sigma):
            if isinstance(a, torch.Tensor) and a.is_cuda:
                if a.dtype != torch.float32 or tuple(a.shape) != shape:
                    raise ValueError("instance %d fields must be float32 %s" % (k, shape))
                a = a.contiguous()
                m = N.KC_MEM_DEVICE
                ptrs.append(ctypes.c_void_p(a.data_ptr()))
            else:
                a = np.ascontiguousarray(a, dtype=np.float32)
                if a.shape != shape:
                    raise ValueError("instance %d fields must have shape %s" % (k, shape))
                m = N.KC_MEM_HOST
                ptrs.append(ctypes.c_void_p(a.ctypes.data))
            if mem is not None and m != mem:
                raise ValueError("fields must all be host arrays or all device tensors")
            mem = m
            keep.append(a)
        self._chk(N.lib().kb_set_fields(self.h, int(k), ptrs[0], ptrs[1], ptrs[2], mem))

    def run(self, nsteps, sample_every):
        self._chk(N.lib().kb_run(self.h, int(nsteps), int(sample_every)))

    def nsamples(self):
        ns = ctypes.c_int32()
        self._chk(N.lib().kb_series(self.h, None, ctypes.byref(ns), N.KC_MEM_HOST))
        return ns.value

    def series(self):
        """[count, nsamples, 5] array of (t, mass, nutrient, envelope radius, area radius)."""
        out = np.zeros((self.count, self.max_samples, 5), dtype=np.float64)
        ns = ctypes.c_int32()
        self._chk(N.lib().kb_series(self.h, ctypes.c_void_p(out.ctypes.data), ctypes.byref(ns),
                                    N.KC_MEM_HOST))
        return out[:, :ns.value, :]

    def get_fields(self, k):
        b = np.empty(self.shapes[k], dtype=np.float32)
        n = np.empty_like(b)
        self._chk(N.lib().kb_get_fields(self.h, int(k), ctypes.c_void_p(b.ctypes.data),
                                        ctypes.c_void_p(n.ctypes.data), N.KC_MEM_HOST))
        return b, n

    def fit_velocity(self, r_lo, r_hi, radius="envelope", t_max=None):
        """Device least-squares dR/dt over the samples with r_lo <= R <= r_hi
        (and t <= t_max when given: kb_fit_velocity_until)."""
        lo = np.ascontiguousarray(np.broadcast_to(np.asarray(r_lo, np.float64), (self.count,)))
        hi = np.ascontiguousarray(np.broadcast_to(np.asarray(r_hi, np.float64), (self.count,)))
        v = np.empty(self.count, dtype=np.float64)
        npts = np.empty(self.count, dtype=np.int32)
        sel = 0 if radius == "envelope" else 1
        if t_max is None:
            self._chk(N.lib().kb_fit_velocity(self.h, sel, ctypes.c_void_p(lo.ctypes.data),
                                              ctypes.c_void_p(hi.ctypes.data),
                                              ctypes.c_void_p(v.ctypes.data),
                                              ctypes.c_void_p(npts.ctypes.data)))
        else:
            tm = np.ascontiguousarray(np.broadcast_to(np.asarray(t_max, np.float64), (self.count,)))
            self._chk(N.lib().kb_fit_velocity_until(self.h, sel, ctypes.c_void_p(lo.ctypes.data),
                                                    ctypes.c_void_p(hi.ctypes.data),
                                                    ctypes.c_void_p(tm.ctypes.data),
                                                    ctypes.c_void_p(v.ctypes.data),
                                                    ctypes.c_void_p(npts.ctypes.data)))
        return v, npts

    def set_tuning(self, tsteps=0, rows=None, prefetch=0, persistent=-1):
        rp = None
        if rows is not None:
            r = np.ascontiguousarray(np.broadcast_to(np.asarray(rows, np.int32), (self.count,)))
            rp = ctypes.c_void_p(r.ctypes.data)
        self._chk(N.lib().kb_set_tuning(self.h, int(tsteps), rp, int(prefetch), int(persistent)))

    def tuning(self):
        t, p, q = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        rows = np.empty(self.count, dtype=np.int32)
        self._chk(N.lib().kb_get_tuning(self.h, ctypes.byref(t), ctypes.c_void_p(rows.ctypes.data),
                                        ctypes.byref(p), ctypes.byref(q)))
        return t.value, rows, p.value, q.value

    def autotune(self, sample_every, effort=0):
        self._chk(N.lib().kb_autotune(self.h, int(effort), int(sample_every)))

    def set_spin_limit(self, polls):
        self._chk(N.lib().kb_set_spin_limit(self.h, int(polls)))

    def steps(self):
        s = ctypes.c_int64()
        self._chk(N.lib().kb_steps(self.h, ctypes.byref(s)))
        return s.value

    def close(self):
        if getattr(self, "h", None):
            N.lib().kb_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
