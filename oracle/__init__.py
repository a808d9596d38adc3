"""FP64 CPU oracle for the explicit step of the normalised chemotaxis system.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark are its only users.  The product library never imports,
links or calls anything here, and nothing here imports the product package.

Contents
  step / run / diag   plain C loops (kc_oracle.c), driven through ctypes;
                      eqs. eqnadim / eqbadim of Sec. 2.4 with no-flux
                      boundaries (eq. bconds), forward Euler or the
                      two-stage Runge-Kutta method (Sec. 3) built from it.
  run_noise           the same steps with the agar field redrawn at every
                      step from a counter-based generator (Philox4x32-10).
  cbar, bstar         closed-form speed bound of Sec. 4.1 (eqs. c-bar-chi0,
                      c-bar-0) -- see cbar.py.
  fit_velocity        least-squares slope of an envelope-radius series.
  cstar               threshold speed of travelling fronts of the scalar
                      equation of Sec. 4.1 by shooting (the appendix) -- see
                      fronts.py.
  mlp_ref             FP64 forward / backward of the velocity surrogate MLP.
"""
import ctypes
import hashlib
import os
import subprocess
import tempfile

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "kc_oracle.c")
_LIB_PATH = os.path.join(_HERE, "libkc_oracle.so")
_lib = None

CHI_RECEPTOR = 0
CHI_CONSTANT = 1


FLAGS = ["-O3", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared", "-std=c99"]


def _native_path():
    """Per-host path of the -march=native build (never shipped with the tree:
    another machine's CPU may lack the instructions)."""
    h = hashlib.sha256()
    with open(_SRC, "rb") as f:
        h.update(f.read())
    try:
        with open("/proc/cpuinfo") as f:
            h.update("".join(ln for ln in f if ln.startswith(("model name", "flags"))).encode())
    except OSError:
        pass
    return os.path.join(tempfile.gettempdir(), "kc_oracle_native_%s.so" % h.hexdigest()[:16])


def build(force=False, native=False):
    """Compile kc_oracle.c with gcc (-O3, OpenMP, no FMA contraction); with
    native=True also -march=native, into a per-host file.  The flags leave the
    arithmetic unchanged: no contraction, and no reassociation of sums (no
    -ffast-math), so both builds give the same bits."""
    path = _native_path() if native else _LIB_PATH
    if not force and os.path.exists(path) and os.path.getmtime(path) >= os.path.getmtime(_SRC):
        return path
    tmp = path + ".tmp%d" % os.getpid()
    cmd = ["gcc"] + FLAGS + (["-march=native"] if native else []) + ["-o", tmp, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, path)
    return path


def use_native():
    """Switch this process to the -march=native build (the CPU-baseline timing
    leg); returns its gcc flags."""
    global _lib
    _lib = _bind(ctypes.CDLL(build(native=True)))
    return " ".join(["gcc"] + FLAGS + ["-march=native"])


def _load():
    global _lib
    if _lib is None:
        _lib = _bind(ctypes.CDLL(build()))
    return _lib


def _bind(lib):
    dp = ctypes.POINTER(ctypes.c_double)
    lib.oracle_step.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                ctypes.c_double, ctypes.c_int, dp, dp, dp, dp, dp]
    lib.oracle_step.restype = None
    lib.oracle_run.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                               ctypes.c_double, ctypes.c_double, ctypes.c_double,
                               ctypes.c_double, ctypes.c_int, dp, dp, dp, ctypes.c_long]
    lib.oracle_run.restype = ctypes.c_int
    lib.oracle_run_rk2.argtypes = lib.oracle_run.argtypes
    lib.oracle_run_rk2.restype = ctypes.c_int
    u32p = ctypes.POINTER(ctypes.c_uint32)
    lib.oracle_philox4x32_10.argtypes = [u32p, u32p, u32p]
    lib.oracle_philox4x32_10.restype = None
    lib.oracle_noise_delta.argtypes = [ctypes.c_uint64, ctypes.c_int64, ctypes.c_int,
                                       ctypes.c_int]
    lib.oracle_noise_delta.restype = ctypes.c_double
    lib.oracle_run_noise.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                     ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                     ctypes.c_double, ctypes.c_double, ctypes.c_int, dp, dp,
                                     ctypes.c_double, ctypes.c_double, ctypes.c_uint64,
                                     ctypes.c_int64, ctypes.c_long, ctypes.c_int]
    lib.oracle_run_noise.restype = ctypes.c_int
    lib.oracle_diag.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, dp, dp,
                                ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                dp, dp, dp, dp]
    lib.oracle_diag.restype = None
    lib.oracle_threads.argtypes = []
    lib.oracle_threads.restype = ctypes.c_int
    lib.oracle_set_threads.argtypes = [ctypes.c_int]
    lib.oracle_set_threads.restype = None
    return lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _params(p):
    return (float(p.get("D_n", 1.0)), float(p.get("theta", 1.0)), float(p.get("kappa", 1.0)),
            float(p.get("chi", 0.0)), int(p.get("chi_law", CHI_RECEPTOR)))


def step(b, n, sigma, h, dt, **p):
    """One forward-Euler step; returns new (b, n) as float64 arrays [ny, nx]."""
    lib = _load()
    b, n, sigma = _f64(b), _f64(n), _f64(sigma)
    ny, nx = b.shape
    bo, no = np.empty_like(b), np.empty_like(n)
    lib.oracle_step(nx, ny, float(h), float(dt), *_params(p),
                    _ptr(b), _ptr(n), _ptr(sigma), _ptr(bo), _ptr(no))
    return bo, no


def run(b, n, sigma, h, dt, nsteps, integrator="euler", **p):
    """nsteps steps of forward Euler (integrator="euler") or of the two-stage
    Runge-Kutta method of kc_oracle.c (integrator="rk2"); returns (b, n) as
    new float64 arrays."""
    lib = _load()
    b, n, sigma = _f64(b).copy(), _f64(n).copy(), _f64(sigma)
    ny, nx = b.shape
    if integrator not in ("euler", "rk2"):
        raise ValueError("integrator must be 'euler' or 'rk2'")
    fn = lib.oracle_run if integrator == "euler" else lib.oracle_run_rk2
    rc = fn(nx, ny, float(h), float(dt), *_params(p),
            _ptr(b), _ptr(n), _ptr(sigma), int(nsteps))
    if rc != 0:
        raise MemoryError("oracle_run: out of memory")
    return b, n


def philox4x32_10(counter, key):
    """The raw Philox4x32-10 generator (4 words out of 4 counter and 2 key words)."""
    lib = _load()
    c = (ctypes.c_uint32 * 4)(*[int(v) & 0xffffffff for v in counter])
    k = (ctypes.c_uint32 * 2)(*[int(v) & 0xffffffff for v in key])
    o = (ctypes.c_uint32 * 4)()
    lib.oracle_philox4x32_10(c, k, o)
    return [int(v) for v in o]


def noise_delta(seed, step, i, j):
    """The triangular agar perturbation Delta of cell (i, j) at time step `step`."""
    return float(_load().oracle_noise_delta(int(seed), int(step), int(i), int(j)))


def run_noise(b, n, h, dt, nsteps, sigma0, amp, seed, step0=0, integrator="euler", **p):
    """nsteps steps with the agar field sigma0 (1 + amp Delta) redrawn at every
    step (steps step0, step0 + 1, ...); returns (b, n) as new float64 arrays."""
    lib = _load()
    b, n = _f64(b).copy(), _f64(n).copy()
    ny, nx = b.shape
    integ = {"euler": 0, "rk2": 1}[integrator]
    rc = lib.oracle_run_noise(nx, ny, float(h), float(dt), *_params(p), _ptr(b), _ptr(n),
                              float(sigma0), float(amp), int(seed), int(step0), int(nsteps), integ)
    if rc != 0:
        raise MemoryError("oracle_run_noise: out of memory")
    return b, n


def diag(b, n, h, b_thr, cx=None, cy=None, area=False):
    """(mass, nutrient, envelope radius) of one level -- plus the area radius
    when area=True; the centre defaults to the grid centre."""
    lib = _load()
    b, n = _f64(b), _f64(n)
    ny, nx = b.shape
    cx = (nx - 1) / 2.0 if cx is None else float(cx)
    cy = (ny - 1) / 2.0 if cy is None else float(cy)
    m, nu, r, ra = ctypes.c_double(), ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    lib.oracle_diag(nx, ny, float(h), _ptr(b), _ptr(n), float(b_thr), cx, cy,
                    ctypes.byref(m), ctypes.byref(nu), ctypes.byref(r), ctypes.byref(ra))
    if area:
        return m.value, nu.value, r.value, ra.value
    return m.value, nu.value, r.value


def threads():
    """OpenMP threads the oracle step uses."""
    return int(_load().oracle_threads())


def set_threads(n):
    """Run the following oracle calls on n OpenMP threads (timing only)."""
    _load().oracle_set_threads(int(n))


from .cbar import bstar, cbar, psi  # noqa: E402,F401
from .velocity import fit_velocity  # noqa: E402,F401
from .fronts import cstar, threshold_speed  # noqa: E402,F401
