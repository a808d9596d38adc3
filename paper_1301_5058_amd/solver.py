"""Python face of the single-instance solver (kc_* calls of include/kc.h).

Solver wraps one kc_ctx.  Fields go in and out as numpy arrays (host memory)
or torch tensors on the GPU (device memory); the context's stream is torch's
current stream unless one is given.  Every computation happens in libkc.so.
"""
import ctypes
import math

import numpy as np
import torch

from . import native as N


def _np_dtype(precision):
    return np.float32 if precision == N.KC_FP32 else np.float64


def _torch_dtype(precision):
    return torch.float32 if precision == N.KC_FP32 else torch.float64


class Solver:
    def __init__(self, nx, ny, h=1.0, dt=0.2, chi=0.0, chi_law="receptor", precision="fp32",
                 D_n=1.0, theta=1.0, kappa=1.0, b_thr=0.5, cx=None, cy=None, step0=0,
                 stream=None, integrator="euler", noise=None):
        self.nx, self.ny, self.h, self.dt = int(nx), int(ny), float(h), float(dt)
        p = N.default_params()
        p.D_n, p.theta, p.kappa, p.chi = float(D_n), float(theta), float(kappa), float(chi)
        p.chi_law = N.KC_CHI_RECEPTOR if chi_law == "receptor" else N.KC_CHI_CONSTANT
        p.precision = N.KC_FP32 if precision == "fp32" else N.KC_FP64
        p.b_thr = float(b_thr)
        p.cx = math.nan if cx is None else float(cx)
        p.cy = math.nan if cy is None else float(cy)
        p.step0 = int(step0)
        if integrator not in ("euler", "rk2"):
            raise ValueError("integrator must be 'euler' or 'rk2'")
        p.integrator = N.KC_EULER if integrator == "euler" else N.KC_RK2
        if noise is not None:
            # per-step agar noise: dict(sigma0=..., amp=..., seed=...)
            p.noise = N.KC_NOISE_PER_STEP
            p.sigma0 = float(noise.get("sigma0", 1.0))
            p.noise_amp = float(noise["amp"])
            p.noise_seed = int(noise.get("seed", 0))
        self.noise = noise
        self.precision = p.precision
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        g = N.KcGrid(self.nx, self.ny)
        ctx = ctypes.c_void_p()
        N.check(N.lib().kc_create(ctypes.byref(g), self.h, self.dt, ctypes.byref(p),
                                  ctypes.c_void_p(stream.cuda_stream), ctypes.byref(ctx)))
        self.ctx = ctx

    # -- fields ---------------------------------------------------------------
    def _arg(self, a):
        """(pointer, mem kind, keep-alive) for a numpy array or torch tensor."""
        if isinstance(a, torch.Tensor):
            if a.dtype != _torch_dtype(self.precision) or tuple(a.shape) != (self.ny, self.nx):
                raise ValueError("field must be %s of shape (%d, %d)"
                                 % (_torch_dtype(self.precision), self.ny, self.nx))
            a = a.contiguous()
            if a.is_cuda:
                return ctypes.c_void_p(a.data_ptr()), N.KC_MEM_DEVICE, a
            a = a.numpy()
        a = np.ascontiguousarray(a, dtype=_np_dtype(self.precision))
        if a.shape != (self.ny, self.nx):
            raise ValueError("field must have shape (%d, %d)" % (self.ny, self.nx))
        return ctypes.c_void_p(a.ctypes.data), N.KC_MEM_HOST, a

    def set_fields(self, b, n, sigma=None):
        """sigma may be None with per-step noise (the library draws it)."""
        (pb, mb, kb), (pn, mn, kn) = self._arg(b), self._arg(n)
        if sigma is None:
            ps, ms = ctypes.c_void_p(None), mb
        else:
            ps, ms, ks = self._arg(sigma)
        if not (mb == mn == ms):
            raise ValueError("b, n and sigma must all be host arrays or all device tensors")
        N.check(N.lib().kc_set_fields(self.ctx, pb, pn, ps, mb), self.ctx)

    def get_fields(self, device=False):
        if device:
            b = torch.empty((self.ny, self.nx), dtype=_torch_dtype(self.precision), device="cuda")
            n = torch.empty_like(b)
            N.check(N.lib().kc_get_fields(self.ctx, ctypes.c_void_p(b.data_ptr()),
                                          ctypes.c_void_p(n.data_ptr()), N.KC_MEM_DEVICE), self.ctx)
            return b, n
        b = np.empty((self.ny, self.nx), dtype=_np_dtype(self.precision))
        n = np.empty_like(b)
        N.check(N.lib().kc_get_fields(self.ctx, ctypes.c_void_p(b.ctypes.data),
                                      ctypes.c_void_p(n.ctypes.data), N.KC_MEM_HOST), self.ctx)
        return b, n

    # -- time stepping ----------------------------------------------------------
    def step(self, nsteps):
        N.check(N.lib().kc_step(self.ctx, int(nsteps)), self.ctx)

    def step_sample(self, nsteps, out5):
        """nsteps steps, then {t, mass, nutrient, envelope radius, area radius}
        of the new level into out5 (a contiguous float64 CUDA tensor of >= 5
        elements), fused into the last step launch; enqueued."""
        if out5.dtype != torch.float64 or not out5.is_cuda or out5.numel() < 5 or \
                not out5.is_contiguous():
            raise ValueError("out5 must be a contiguous float64 CUDA tensor with >= 5 elements")
        N.check(N.lib().kc_step_sample(self.ctx, int(nsteps), ctypes.c_void_p(out5.data_ptr())),
                self.ctx)

    def step_sample_noalloc(self, nsteps, out5):
        """step_sample through kc_step_sample_noalloc: the same results, with
        the diagnostics partials in the library's fixed device scratch (no
        device allocation in the call)."""
        if out5.dtype != torch.float64 or not out5.is_cuda or out5.numel() < 5 or \
                not out5.is_contiguous():
            raise ValueError("out5 must be a contiguous float64 CUDA tensor with >= 5 elements")
        N.check(N.lib().kc_step_sample_noalloc(self.ctx, int(nsteps),
                                               ctypes.c_void_p(out5.data_ptr())), self.ctx)

    def diagnostics(self):
        m, nu, r = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        N.check(N.lib().kc_diagnostics(self.ctx, ctypes.byref(m), ctypes.byref(nu),
                                       ctypes.byref(r)), self.ctx)
        return m.value, nu.value, r.value

    def diagnostics_device(self, out5):
        """Enqueue {t, mass, nutrient, envelope radius, area radius} into a
        contiguous float64 CUDA tensor of >= 5 elements."""
        if out5.dtype != torch.float64 or not out5.is_cuda or out5.numel() < 5 or \
                not out5.is_contiguous():
            raise ValueError("out5 must be a contiguous float64 CUDA tensor with >= 5 elements")
        N.check(N.lib().kc_diagnostics_device(self.ctx, ctypes.c_void_p(out5.data_ptr())), self.ctx)

    def diagnostics_all(self):
        """(t, mass, nutrient, envelope radius, area radius), synchronous."""
        out = torch.zeros(5, dtype=torch.float64, device="cuda")
        self.diagnostics_device(out)
        self.stream.synchronize()
        return tuple(float(v) for v in out.cpu().numpy())

    def time(self):
        t, s = ctypes.c_double(), ctypes.c_int64()
        N.check(N.lib().kc_time(self.ctx, ctypes.byref(t), ctypes.byref(s)))
        return t.value, s.value

    # -- kernel configuration ---------------------------------------------------
    def set_tuning(self, tsteps=0, rows=0, prefetch=0, waves=0):
        """waves: wavefronts per strip (1 or 2; 0 keeps the current value)."""
        N.check(N.lib().kc_set_tuning(self.ctx, int(tsteps), int(rows), int(prefetch)), self.ctx)
        if waves:
            N.check(N.lib().kc_set_strip_waves(self.ctx, int(waves)), self.ctx)

    def strip_waves(self):
        w = ctypes.c_int32()
        N.check(N.lib().kc_get_strip_waves(self.ctx, ctypes.byref(w)))
        return w.value

    def tuning(self):
        t, r, p = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        N.check(N.lib().kc_get_tuning(self.ctx, ctypes.byref(t), ctypes.byref(r), ctypes.byref(p)))
        return t.value, r.value, p.value

    def autotune(self, effort=0, use_cache=True):
        """Time candidate kernel configurations on this solver's fields and keep
        the fastest; returns its rate in 1e9 cell-updates/s (0 if cached)."""
        g = ctypes.c_double()
        N.check(N.lib().kc_autotune(self.ctx, int(effort), 1 if use_cache else 0, ctypes.byref(g)),
                self.ctx)
        return g.value

    def use_reference_kernel(self, on=True):
        N.check(N.lib().kc_set_reference_kernel(self.ctx, 1 if on else 0), self.ctx)

    def close(self):
        if getattr(self, "ctx", None):
            N.lib().kc_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
