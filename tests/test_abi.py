"""C ABI checks that need no GPU: the library loads, exports every symbol its
headers declare, and rejects bad arguments before any device work."""
import ctypes
import glob
import math
import os
import re

import numpy as np
import pytest

from paper_1301_5058_amd import native as N

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        src = open(h).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        for m in re.finditer(r"^[A-Za-z_][\w \*]*?\b(k[a-z]_\w+)\s*\(", src, flags=re.M):
            names.add(m.group(1))
    return sorted(names)


def test_headers_declare_the_entry_points():
    names = _declared()
    for must in ("kc_create", "kc_set_fields", "kc_step", "kc_diagnostics", "kc_destroy"):
        assert must in names


def test_library_exports_every_declared_symbol():
    L = N.lib()
    missing = [n for n in _declared() if not hasattr(L, n)]
    assert not missing, missing


def test_strerror_and_null_context():
    L = N.lib()
    for code in (0, -1, -2, -3, -4, -5, -6):
        assert L.kc_strerror(code)
    assert L.kc_strerror(-99) == b"unknown status"
    L.kc_destroy(None)
    assert L.kc_step(None, 1) == N.KC_EINVAL
    assert L.kc_step_sample(None, 1, None) == N.KC_EINVAL
    assert L.kc_step_sample_noalloc(None, 1, None) == N.KC_EINVAL
    assert L.kc_set_fields(None, None, None, None, 0) == N.KC_EINVAL
    assert L.kc_diagnostics(None, None, None, None) == N.KC_EINVAL
    assert L.kc_get_fields(None, None, None, 0) == N.KC_EINVAL
    assert L.kc_set_tuning(None, 1, 1, 2) == N.KC_EINVAL
    assert L.kc_set_strip_waves(None, 1) == N.KC_EINVAL
    w = ctypes.c_int32()
    assert L.kc_get_strip_waves(None, ctypes.byref(w)) == N.KC_EINVAL
    assert L.kc_time(None, None, None) == N.KC_EINVAL
    assert L.kc_last_error(None) == b"null context"


def _create(nx=16, ny=16, h=1.0, dt=0.1, **kw):
    L = N.lib()
    p = N.default_params()
    for k, v in kw.items():
        setattr(p, k, v)
    g = N.KcGrid(nx, ny)
    ctx = ctypes.c_void_p()
    rc = L.kc_create(ctypes.byref(g), h, dt, ctypes.byref(p), None, ctypes.byref(ctx))
    if rc == N.KC_OK:
        L.kc_destroy(ctx)
    return rc, ctx


@pytest.mark.parametrize("kw", [dict(nx=0), dict(ny=-3), dict(h=0.0), dict(h=math.nan),
                                dict(dt=0.0), dict(dt=-1.0), dict(dt=math.inf),
                                dict(D_n=-1.0), dict(theta=-0.1), dict(kappa=math.nan),
                                dict(chi=-2.0), dict(chi_law=7), dict(precision=3),
                                dict(nx=1 << 21), dict(step0=-1), dict(b_thr=math.nan),
                                dict(integrator=2), dict(noise=2),
                                dict(noise=1, noise_amp=1.0 + 1e-12), dict(noise=1, noise_amp=-0.1),
                                dict(noise=1, noise_amp=math.nan), dict(noise=1, sigma0=0.0),
                                dict(noise=1, sigma0=math.inf)])
def test_create_rejects_bad_arguments(kw):
    rc, ctx = _create(**kw)
    assert rc == N.KC_EINVAL
    assert not ctx.value


def test_create_accepts_the_papers_full_noise_amplitude():
    # sigma = sigma0 (1 + Delta) (Sec. 3): amplitude 1 passes the argument checks
    # (without a GPU the call then fails with KC_EHIP, with one it succeeds)
    rc, _ = _create(noise=1, noise_amp=1.0, sigma0=4.0, integrator=1)
    assert rc != N.KC_EINVAL


def test_create_rejects_null_outputs():
    L = N.lib()
    p = N.default_params()
    g = N.KcGrid(8, 8)
    assert L.kc_create(ctypes.byref(g), 1.0, 0.1, ctypes.byref(p), None, None) == N.KC_EINVAL
    ctx = ctypes.c_void_p()
    assert L.kc_create(None, 1.0, 0.1, ctypes.byref(p), None, ctypes.byref(ctx)) == N.KC_EINVAL
    assert L.kc_create(ctypes.byref(g), 1.0, 0.1, None, None, ctypes.byref(ctx)) == N.KC_EINVAL


def test_create_without_device_reports_hip_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    rc, ctx = _create()
    assert rc == N.KC_EHIP and not ctx.value


def _check(b, n, s, precision=N.KC_FP32, nx=None, ny=None):
    L = N.lib()
    dt = np.float32 if precision == N.KC_FP32 else np.float64
    b, n, s = (np.ascontiguousarray(a, dtype=dt) for a in (b, n, s))
    ny_, nx_ = b.shape
    mx = ctypes.c_double(-1)
    rc = L.kc_check_fields(nx_ if nx is None else nx, ny_ if ny is None else ny, precision,
                           b.ctypes.data, n.ctypes.data, s.ctypes.data, ctypes.byref(mx))
    return rc, mx.value


@pytest.mark.parametrize("precision", [N.KC_FP32, N.KC_FP64])
def test_check_fields(precision):
    rng = np.random.default_rng(0)
    b = rng.uniform(0, 0.7, (5, 6))
    n = rng.uniform(0, 1, (5, 6))
    s = rng.uniform(0.5, 1.5, (5, 6))
    rc, mx = _check(b, n, s, precision)
    assert rc == N.KC_OK
    dt = np.float32 if precision == N.KC_FP32 else np.float64
    ref = np.max(b.astype(dt).astype(np.float64) * n.astype(dt) * s.astype(dt))
    assert mx == pytest.approx(ref, rel=1e-15)
    for bad in (math.nan, math.inf, -1e-30):
        for which in range(3):
            arrs = [b.copy(), n.copy(), s.copy()]
            arrs[which][2, 3] = bad
            assert _check(*arrs, precision)[0] == N.KC_ENONFINITE
    assert _check(b, n, s, precision, nx=0)[0] == N.KC_EINVAL
    assert _check(b, n, s, 9)[0] == N.KC_EINVAL
    L = N.lib()
    assert L.kc_check_fields(6, 5, precision, None, None, None, None) == N.KC_EINVAL


def test_suggest_dt():
    L = N.lib()
    assert L.kc_suggest_dt(1.0, 1.0, 0.3) == pytest.approx(0.2)
    assert L.kc_suggest_dt(0.5, 1.0, 2.0) == pytest.approx(0.2 * 0.25 / 2.0)
    assert L.kc_suggest_dt(0.0, 1.0, 1.0) == 0.0


def _kb_create(count=2, law=0, cap=10, **kw):
    L = N.lib()
    arr = (N.KbInstance * max(count, 1))()
    for k in range(max(count, 1)):
        I = arr[k]
        I.nx, I.ny, I.h, I.dt = 32, 32, 1.0, 0.1
        I.D_n = I.theta = I.kappa = 1.0
        I.chi, I.b_thr, I.cx, I.cy = 0.5, 0.4, math.nan, math.nan
        for key, v in kw.items():
            setattr(I, key, v)
    h = ctypes.c_void_p()
    rc = L.kb_create(count, arr, law, cap, None, ctypes.byref(h))
    if rc == N.KC_OK:
        L.kb_destroy(h)
    return rc, h


@pytest.mark.parametrize("args", [dict(count=0), dict(law=5), dict(cap=0), dict(nx=0),
                                  dict(dt=-1.0), dict(h=math.inf), dict(chi=-1.0),
                                  dict(kappa=math.nan), dict(ny=1 << 17), dict(b_thr=math.nan)])
def test_batch_create_rejects_bad_arguments(args):
    rc, h = _kb_create(**args)
    assert rc == N.KC_EINVAL and not h.value


def test_batch_null_handles():
    L = N.lib()
    L.kb_destroy(None)
    assert L.kb_run(None, 10, 10) == N.KC_EINVAL
    assert L.kb_set_fields(None, 0, None, None, None, 0) == N.KC_EINVAL
    assert L.kb_series(None, None, None, 0) == N.KC_EINVAL
    assert L.kb_set_spin_limit(None, 5) == N.KC_EINVAL
    assert L.kb_last_error(None) == b"null batch"


def _check_step(b, n, s, h, dt, **kw):
    L = N.lib()
    p = N.default_params()
    for k, v in kw.items():
        setattr(p, k, v)
    b, n = np.ascontiguousarray(b, np.float32), np.ascontiguousarray(n, np.float32)
    sp = None if s is None else np.ascontiguousarray(s, np.float32)
    dmax = ctypes.c_double()
    rc = L.kc_check_step(b.shape[1], b.shape[0], N.KC_FP32, b.ctypes.data, n.ctypes.data,
                         None if sp is None else sp.ctypes.data, h, dt, ctypes.byref(p),
                         ctypes.byref(dmax))
    return rc, dmax.value


def _outflow_bound(b, n, s, chi, receptor, D_n=1.0):
    """The largest dt of the two documented bounds, by a direct numpy loop."""
    ny, nx = b.shape
    D = s * n * b
    rate = 0.0
    for y in range(ny):
        for x in range(nx):
            dsum = up = 0.0
            for xq, yq in ((x + 1, y), (x - 1, y), (x, y + 1), (x, y - 1)):
                if 0 <= xq < nx and 0 <= yq < ny:
                    dsum += 0.5 * (D[y, x] + D[yq, xq])
                    up += max(n[yq, xq] - n[y, x], 0.0)
            ch = 1.0 / (1.0 + n[y, x]) ** 2 if receptor else 1.0
            rate = max(rate, dsum + chi * D[y, x] * ch * up)
    return 1.0 / max(4.0 * max(D_n, D.max()), rate)


def _chemotactic_front(nx=16, ny=12):
    # b = 0.5 everywhere, nutrient 0.1 on the left half and 1.0 on the right:
    # the cells left of the jump send their bacteria up the nutrient step
    b = np.full((ny, nx), 0.5)
    n = np.full((ny, nx), 0.1)
    n[:, nx // 2:] = 1.0
    s = np.ones((ny, nx))
    return b, n, s


def test_stability_check_counts_the_chemotactic_outflow():
    import oracle
    b, n, s = _chemotactic_front()
    chi, dt = 200.0, 0.2
    # the diffusive bound alone accepts dt = 0.2: max sigma n b = 0.5 <= D_n = 1
    mx = ctypes.c_double()
    L = N.lib()
    bf, nf, sf = (np.ascontiguousarray(a, np.float32) for a in (b, n, s))
    assert L.kc_check_fields(16, 12, N.KC_FP32, bf.ctypes.data, nf.ctypes.data, sf.ctypes.data,
                             ctypes.byref(mx)) == N.KC_OK
    assert dt <= 1.0 / (4.0 * max(1.0, mx.value))
    # ... but one step of that size drives b negative next to the jump (oracle)
    ob, _ = oracle.step(bf, nf, sf, 1.0, dt, chi=chi, chi_law=N.KC_CHI_CONSTANT)
    assert ob.min() < 0
    rc, dmax = _check_step(b, n, s, 1.0, dt, chi=chi, chi_law=N.KC_CHI_CONSTANT)
    assert rc == N.KC_EUNSTABLE
    # the bound it reports: left of the jump, the face diffusivities
    # 3 x 0.05 + (0.05 + 0.5) / 2 plus chi sigma n b (1.0 - 0.1) up the jump
    assert dmax == pytest.approx(1.0 / (0.425 + chi * 0.05 * 0.9), rel=1e-6)
    assert dmax == pytest.approx(_outflow_bound(b, n, s, chi, False), rel=1e-6)
    # a step of that size keeps b >= 0 on these fields (the bound is for the
    # fields it is given: the pile-up it causes at the jump needs a smaller
    # step afterwards), and the check accepts it
    rc2, _ = _check_step(b, n, s, 1.0, dmax, chi=chi, chi_law=N.KC_CHI_CONSTANT)
    assert rc2 == N.KC_OK
    ob, _ = oracle.step(bf, nf, sf, 1.0, dmax, chi=chi, chi_law=N.KC_CHI_CONSTANT)
    assert ob.min() >= 0
    # the receptor law divides the chemotactic coefficient by (1 + n)^2
    _, dmax_r = _check_step(b, n, s, 1.0, dt, chi=chi, chi_law=N.KC_CHI_RECEPTOR)
    assert dmax_r == pytest.approx(_outflow_bound(b, n, s, chi, True), rel=1e-6)
    assert dmax_r > dmax
    # no chemotaxis: only the diffusive bound, 1 / (4 max(D_n, sigma n b))
    rc0, dmax0 = _check_step(b, n, s, 1.0, dt, chi=0.0)
    assert rc0 == N.KC_OK and dmax0 == pytest.approx(0.25, rel=1e-12)


def test_stability_check_with_per_step_noise_takes_the_largest_sigma():
    b, n, s = _chemotactic_front()
    # sigma0 (1 + a) = 3 scales every diffusivity and the chemotactic coefficient
    rc, dmax = _check_step(b, n, None, 1.0, 0.05, chi=20.0, chi_law=N.KC_CHI_CONSTANT,
                           noise=N.KC_NOISE_PER_STEP, sigma0=2.0, noise_amp=0.5)
    want = _outflow_bound(b, n, 3.0 * s, 20.0, False)
    assert dmax == pytest.approx(want, rel=1e-6)
    assert rc == N.KC_OK and 0.05 <= want
    assert _check_step(b, n, None, 1.0, 1.01 * want, chi=20.0, chi_law=N.KC_CHI_CONSTANT,
                       noise=N.KC_NOISE_PER_STEP, sigma0=2.0, noise_amp=0.5)[0] == N.KC_EUNSTABLE
    assert _check_step(b, n, None, 1.0, 0.05, chi=20.0)[0] == N.KC_EINVAL  # static sigma needed
    bad = b.copy()
    bad[3, 4] = np.nan
    assert _check_step(bad, n, s, 1.0, 0.05)[0] == N.KC_ENONFINITE
    assert _check_step(b, n, s, 1.0, -1.0)[0] == N.KC_EINVAL
