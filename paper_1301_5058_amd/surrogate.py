"""Python face of the velocity surrogate (ks_* calls of include/ks.h).

Surrogate wraps one ks_model: a 3 -> 64 -> 64 -> 64 -> 1 BF16 MLP trained and
evaluated by the library's MFMA kernels.  Its training hull (the convex hull
of the training inputs) is handed to the library as facet planes; points
outside it are the ones a caller sends to the batched solver instead.
"""
import ctypes

import numpy as np
import torch

from . import native as N

NPARAM = 8641


def he_uniform(seed):
    """Initial parameters: He-uniform weights, zero biases (seeded, host side)."""
    rng = np.random.default_rng(seed)
    p = np.zeros(NPARAM, dtype=np.float32)

    def fill(off, fan_out, fan_in):
        lim = np.sqrt(6.0 / fan_in)
        p[off:off + fan_out * fan_in] = rng.uniform(-lim, lim, fan_out * fan_in)

    fill(0, 64, 3)
    fill(256, 64, 64)
    fill(4416, 64, 64)
    fill(8576, 1, 64)
    return p


def hull_facets(points):
    """Facet planes {a, b} (a.x + b <= 0 inside) of the convex hull of points [n, 3]."""
    from scipy.spatial import ConvexHull
    h = ConvexHull(np.asarray(points, dtype=np.float64))
    return np.ascontiguousarray(h.equations, dtype=np.float64)


class Surrogate:
    def __init__(self, max_points, stream=None):
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        self.max_points = int(max_points)
        h = ctypes.c_void_p()
        N.check(N.lib().ks_create(self.max_points, ctypes.c_void_p(stream.cuda_stream),
                                  ctypes.byref(h)))
        self.h = h

    def _chk(self, code):
        if code != N.KC_OK:
            raise N.KcError(code, N.lib().ks_last_error(self.h).decode() or
                            N.lib().kc_strerror(code).decode())

    @staticmethod
    def _x(X):
        X = np.ascontiguousarray(X, dtype=np.float32)
        if X.ndim != 2 or X.shape[1] != 3:
            raise ValueError("X must be [n, 3]")
        return X

    def set_params(self, p):
        p = np.ascontiguousarray(p, dtype=np.float32)
        assert p.shape == (NPARAM,)
        self._chk(N.lib().ks_set_params(self.h, p.ctypes.data_as(ctypes.c_void_p)))

    def get_params(self):
        p = np.empty(NPARAM, dtype=np.float32)
        self._chk(N.lib().ks_get_params(self.h, p.ctypes.data_as(ctypes.c_void_p)))
        return p

    def set_normalization(self, in_shift, in_scale, out_shift, out_scale, log_target=False):
        a = np.ascontiguousarray(in_shift, dtype=np.float64)
        b = np.ascontiguousarray(in_scale, dtype=np.float64)
        self.norm = (a.copy(), b.copy(), float(out_shift), float(out_scale), bool(log_target))
        self._chk(N.lib().ks_set_normalization(self.h, a.ctypes.data_as(ctypes.c_void_p),
                                               b.ctypes.data_as(ctypes.c_void_p),
                                               float(out_shift), float(out_scale),
                                               1 if log_target else 0))

    def train(self, X, v, iters, batch, lr):
        X = self._x(X)
        v = np.ascontiguousarray(v, dtype=np.float32)
        loss = ctypes.c_double()
        self._chk(N.lib().ks_train(self.h, X.ctypes.data_as(ctypes.c_void_p),
                                   v.ctypes.data_as(ctypes.c_void_p), len(X), int(iters),
                                   int(batch), float(lr), N.KC_MEM_HOST, ctypes.byref(loss)))
        return loss.value

    def grad(self, X, v):
        X = self._x(X)
        v = np.ascontiguousarray(v, dtype=np.float32)
        g = np.empty(NPARAM, dtype=np.float32)
        loss = ctypes.c_double()
        self._chk(N.lib().ks_grad(self.h, X.ctypes.data_as(ctypes.c_void_p),
                                  v.ctypes.data_as(ctypes.c_void_p), len(X),
                                  g.ctypes.data_as(ctypes.c_void_p), ctypes.byref(loss),
                                  N.KC_MEM_HOST))
        return g, loss.value

    def predict(self, X):
        X = self._x(X)
        v = np.empty(len(X), dtype=np.float32)
        self._chk(N.lib().ks_predict(self.h, X.ctypes.data_as(ctypes.c_void_p), len(X),
                                     v.ctypes.data_as(ctypes.c_void_p), N.KC_MEM_HOST))
        return v

    def predict_device(self, X, out):
        """X: float32 CUDA tensor [n, 3]; out: float32 CUDA tensor [n] (enqueued)."""
        self._chk(N.lib().ks_predict(self.h, ctypes.c_void_p(X.data_ptr()), X.shape[0],
                                     ctypes.c_void_p(out.data_ptr()), N.KC_MEM_DEVICE))

    def set_hull(self, facets, tol=1e-9):
        f = np.ascontiguousarray(facets, dtype=np.float64)
        self._chk(N.lib().ks_hull_set(self.h, f.ctypes.data_as(ctypes.c_void_p), len(f),
                                      float(tol)))

    def inside(self, X):
        X = self._x(X)
        o = np.empty(len(X), dtype=np.uint8)
        self._chk(N.lib().ks_hull_test(self.h, X.ctypes.data_as(ctypes.c_void_p), len(X),
                                       o.ctypes.data_as(ctypes.c_void_p), N.KC_MEM_HOST))
        return o.astype(bool)

    def cbar(self, X, sigma0=1.0):
        X = self._x(X)
        o = np.empty(len(X), dtype=np.float32)
        self._chk(N.lib().ks_cbar(self.h, X.ctypes.data_as(ctypes.c_void_p), len(X),
                                  float(sigma0), o.ctypes.data_as(ctypes.c_void_p),
                                  N.KC_MEM_HOST))
        return o

    def cstar(self, X, sigma0=1.0):
        """Threshold speed c*(n0, chi0) of the scalar front equation (ks_cstar)."""
        X = self._x(X)
        o = np.empty(len(X), dtype=np.float32)
        self._chk(N.lib().ks_cstar(self.h, X.ctypes.data_as(ctypes.c_void_p), len(X),
                                   float(sigma0), o.ctypes.data_as(ctypes.c_void_p),
                                   N.KC_MEM_HOST))
        return o

    def close(self):
        if getattr(self, "h", None):
            N.lib().ks_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
