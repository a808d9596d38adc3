"""ctypes binding of libkc.so (C ABI in include/kc.h): argument marshalling only.

torch is imported first so that libkc.so binds to the HIP runtime torch has
already loaded (one runtime per process).  There is no CPU fallback: when the
library is missing, every entry point raises.
"""
import ctypes
import os

import torch  # noqa: F401  (loads the process's HIP runtime before libkc.so)

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libkc.so")

KC_OK, KC_EINVAL, KC_ENONFINITE, KC_EUNSTABLE, KC_ESTATE, KC_ENOMEM, KC_EHIP = 0, -1, -2, -3, -4, -5, -6
KC_FP32, KC_FP64 = 0, 1
KC_CHI_RECEPTOR, KC_CHI_CONSTANT = 0, 1
KC_MEM_HOST, KC_MEM_DEVICE = 0, 1
KC_EULER, KC_RK2 = 0, 1
KC_NOISE_STATIC, KC_NOISE_PER_STEP = 0, 1

c_int32, c_int64, c_double, c_void_p = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p
P_double = ctypes.POINTER(c_double)


class KcGrid(ctypes.Structure):
    _fields_ = [("nx", c_int32), ("ny", c_int32)]


class KcParams(ctypes.Structure):
    _fields_ = [("D_n", c_double), ("theta", c_double), ("kappa", c_double), ("chi", c_double),
                ("chi_law", c_int32), ("precision", c_int32), ("b_thr", c_double),
                ("cx", c_double), ("cy", c_double), ("step0", c_int64), ("integrator", c_int32),
                ("noise", c_int32), ("sigma0", c_double), ("noise_amp", c_double),
                ("noise_seed", ctypes.c_uint64)]


class KbInstance(ctypes.Structure):
    _fields_ = [("nx", c_int32), ("ny", c_int32), ("h", c_double), ("dt", c_double),
                ("D_n", c_double), ("theta", c_double), ("kappa", c_double), ("chi", c_double),
                ("b_thr", c_double), ("cx", c_double), ("cy", c_double)]


class KcError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (status %d)" % (msg, code))
        self.code = code


_SIGS = {
    # name: (restype, argtypes)
    "kc_default_params": (None, [ctypes.POINTER(KcParams)]),
    "kc_create": (c_int32, [ctypes.POINTER(KcGrid), c_double, c_double, ctypes.POINTER(KcParams),
                            c_void_p, ctypes.POINTER(c_void_p)]),
    "kc_set_fields": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_int32]),
    "kc_step": (c_int32, [c_void_p, c_int64]),
    "kc_diagnostics": (c_int32, [c_void_p, P_double, P_double, P_double]),
    "kc_diagnostics_device": (c_int32, [c_void_p, c_void_p]),
    "kc_step_sample": (c_int32, [c_void_p, c_int64, c_void_p]),
    "kc_step_sample_noalloc": (c_int32, [c_void_p, c_int64, c_void_p]),
    "kc_get_fields": (c_int32, [c_void_p, c_void_p, c_void_p, c_int32]),
    "kc_time": (c_int32, [c_void_p, P_double, ctypes.POINTER(c_int64)]),
    "kc_suggest_dt": (c_double, [c_double, c_double, c_double]),
    "kc_check_fields": (c_int32, [c_int32, c_int32, c_int32, c_void_p, c_void_p, c_void_p,
                                  P_double]),
    "kc_check_step": (c_int32, [c_int32, c_int32, c_int32, c_void_p, c_void_p, c_void_p, c_double,
                                c_double, ctypes.POINTER(KcParams), P_double]),
    "kc_set_tuning": (c_int32, [c_void_p, c_int32, c_int32, c_int32]),
    "kc_set_strip_waves": (c_int32, [c_void_p, c_int32]),
    "kc_get_strip_waves": (c_int32, [c_void_p, ctypes.POINTER(c_int32)]),
    "kc_get_tuning": (c_int32, [c_void_p, ctypes.POINTER(c_int32), ctypes.POINTER(c_int32),
                                ctypes.POINTER(c_int32)]),
    "kc_set_reference_kernel": (c_int32, [c_void_p, c_int32]),
    "kc_autotune": (c_int32, [c_void_p, c_int32, c_int32, P_double]),
    "kc_destroy": (None, [c_void_p]),
    "kc_strerror": (ctypes.c_char_p, [c_int32]),
    "kc_last_error": (ctypes.c_char_p, [c_void_p]),
    # batch (kb.h)
    "kb_create": (c_int32, [c_int32, ctypes.POINTER(KbInstance), c_int32, c_int32, c_void_p,
                            ctypes.POINTER(c_void_p)]),
    "kb_set_fields": (c_int32, [c_void_p, c_int32, c_void_p, c_void_p, c_void_p, c_int32]),
    "kb_run": (c_int32, [c_void_p, c_int64, c_int32]),
    "kb_series": (c_int32, [c_void_p, c_void_p, ctypes.POINTER(c_int32), c_int32]),
    "kb_get_fields": (c_int32, [c_void_p, c_int32, c_void_p, c_void_p, c_int32]),
    "kb_fit_velocity": (c_int32, [c_void_p, c_int32, c_void_p, c_void_p, c_void_p, c_void_p]),
    "kb_fit_velocity_until": (c_int32, [c_void_p, c_int32, c_void_p, c_void_p, c_void_p, c_void_p,
                                        c_void_p]),
    "kb_set_tuning": (c_int32, [c_void_p, c_int32, c_void_p, c_int32, c_int32]),
    "kb_get_tuning": (c_int32, [c_void_p, ctypes.POINTER(c_int32), c_void_p,
                                ctypes.POINTER(c_int32), ctypes.POINTER(c_int32)]),
    "kb_set_spin_limit": (c_int32, [c_void_p, c_int64]),
    "kb_autotune": (c_int32, [c_void_p, c_int32, c_int32]),
    "kb_steps": (c_int32, [c_void_p, ctypes.POINTER(c_int64)]),
    "kb_destroy": (None, [c_void_p]),
    "kb_last_error": (ctypes.c_char_p, [c_void_p]),
    # surrogate (ks.h)
    "ks_create": (c_int32, [c_int32, c_void_p, ctypes.POINTER(c_void_p)]),
    "ks_set_params": (c_int32, [c_void_p, c_void_p]),
    "ks_get_params": (c_int32, [c_void_p, c_void_p]),
    "ks_set_normalization": (c_int32, [c_void_p, c_void_p, c_void_p, c_double, c_double,
                                       c_int32]),
    "ks_train": (c_int32, [c_void_p, c_void_p, c_void_p, c_int32, c_int32, c_int32, c_double,
                           c_int32, P_double]),
    "ks_grad": (c_int32, [c_void_p, c_void_p, c_void_p, c_int32, c_void_p, P_double, c_int32]),
    "ks_predict": (c_int32, [c_void_p, c_void_p, c_int32, c_void_p, c_int32]),
    "ks_hull_set": (c_int32, [c_void_p, c_void_p, c_int32, c_double]),
    "ks_hull_test": (c_int32, [c_void_p, c_void_p, c_int32, c_void_p, c_int32]),
    "ks_cbar": (c_int32, [c_void_p, c_void_p, c_int32, c_double, c_void_p, c_int32]),
    "ks_cstar": (c_int32, [c_void_p, c_void_p, c_int32, c_double, c_void_p, c_int32]),
    "ks_destroy": (None, [c_void_p]),
    "ks_last_error": (ctypes.c_char_p, [c_void_p]),
}

_lib = None


def lib():
    """The loaded library (raises when libkc.so has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libkc.so is not built (%s); run `python -m paper_1301_5058_amd.build`"
                               % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def check(code, ctx=None, kind="kc"):
    """Raise KcError for a negative status (message from the kc or kb handle)."""
    if code != KC_OK:
        L = lib()
        msg = ""
        if ctx:
            msg = (L.kc_last_error(ctx) if kind == "kc" else L.kb_last_error(ctx)).decode()
        raise KcError(code, msg or L.kc_strerror(code).decode())
    return code


def default_params():
    p = KcParams()
    lib().kc_default_params(ctypes.byref(p))
    return p
