"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Tolerances
  FP32 fields vs the FP64 oracle, normwise max|x - x_ref| / max|x_ref| per
  field: <= 1e-4 after 2000 steps; mass and envelope radius within 0.5 %.
  FP64 fields vs the oracle: <= 1e-10 normwise (the two differ only in the
  order of rounding: explicit FMAs and face-wise sums).
  Any fused launch shape vs the one-step reference kernel: bitwise equal.
"""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_1301_5058_amd import workload

pytestmark = pytest.mark.gpu


def _solver(nx, ny, dt, **kw):
    from paper_1301_5058_amd.solver import Solver
    return Solver(nx, ny, dt=dt, **kw)


def run_gpu(b, n, s, steps, dt, precision="fp32", tuning=None, ref=False, **kw):
    ny, nx = b.shape
    S = _solver(nx, ny, dt, precision=precision, **kw)
    if tuning:
        S.set_tuning(*tuning)
    if ref:
        S.use_reference_kernel()
    if precision == "fp64":
        b, n, s = (np.asarray(a, np.float64) for a in (b, n, s))
    S.set_fields(b, n, s)
    S.step(steps)
    bo, no = S.get_fields()
    d = S.diagnostics()
    S.close()
    return bo, no, d


def normwise(x, ref):
    return float(np.max(np.abs(np.asarray(x, np.float64) - ref)) / np.max(np.abs(ref)))


# ----------------------------------------------------------------------------
# The small workload (128^2, 2000 steps) against the oracle
# ----------------------------------------------------------------------------
@pytest.fixture(scope="module")
def small_oracle():
    c = workload.SMALL_128
    b, n, s = workload.fields(c["nx"], c["ny"], c["n0"], c["a"], c["seed"])
    dt = workload.config_dt(b, n, s)
    ob, on = oracle.run(b, n, s, 1.0, dt, c["steps"], chi=c["chi"])
    od = oracle.diag(ob, on, 1.0, 0.5 * c["n0"])
    return (b, n, s, dt), (ob, on, od)


def test_small_workload_fp32_matches_oracle(small_oracle):
    (b, n, s, dt), (ob, on, od) = small_oracle
    c = workload.SMALL_128
    gb, gn, gd = run_gpu(b, n, s, c["steps"], dt, chi=c["chi"], b_thr=0.5 * c["n0"])
    eb, en = normwise(gb, ob), normwise(gn, on)
    print("fp32 128^2 x 2000: normwise b %.3e n %.3e" % (eb, en))
    assert eb <= 1e-4 and en <= 1e-4
    assert abs(gd[0] - od[0]) / od[0] <= 5e-3
    assert abs(gd[1] - od[1]) / od[1] <= 5e-3
    assert od[2] > 10.0 and abs(gd[2] - od[2]) / od[2] <= 5e-3


def test_small_workload_fp64_matches_oracle(small_oracle):
    (b, n, s, dt), (ob, on, od) = small_oracle
    c = workload.SMALL_128
    gb, gn, gd = run_gpu(b, n, s, c["steps"], dt, precision="fp64", chi=c["chi"],
                         b_thr=0.5 * c["n0"])
    eb, en = normwise(gb, ob), normwise(gn, on)
    print("fp64 128^2 x 2000: normwise b %.3e n %.3e" % (eb, en))
    assert eb <= 1e-10 and en <= 1e-10
    assert gd[0] == pytest.approx(od[0], rel=1e-12)
    assert gd[1] == pytest.approx(od[1], rel=1e-12)
    assert gd[2] == od[2]


# ----------------------------------------------------------------------------
# One step, element by element, on random data (several tiles + ragged tails)
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("nx,ny", [(700, 150), (257, 31), (1, 40), (40, 1), (1, 1), (2, 3)])
@pytest.mark.parametrize("law", ["receptor", "constant"])
def test_one_step_elementwise(nx, ny, law):
    rng = np.random.default_rng(nx * 1000 + ny)
    b = rng.uniform(0.0, 0.8, (ny, nx)).astype(np.float32)
    b[rng.uniform(size=(ny, nx)) < 0.2] = 0.0  # degenerate cells
    n = rng.uniform(0.0, 1.2, (ny, nx)).astype(np.float32)
    s = rng.uniform(0.2, 1.8, (ny, nx)).astype(np.float32)
    dt = 0.05
    kw = dict(chi=1.3, chi_law=law, D_n=1.1, theta=0.9, kappa=1.2)
    ob, on = oracle.step(b, n, s, 1.0, dt, D_n=1.1, theta=0.9, kappa=1.2, chi=1.3,
                         chi_law=0 if law == "receptor" else 1)
    for prec, tol in (("fp64", 4e-16), ("fp32", 1e-6)):
        gb, gn, _ = run_gpu(b, n, s, 1, dt, precision=prec, **kw)
        scale = max(np.max(np.abs(ob)), np.max(np.abs(on)))
        assert np.max(np.abs(gb - ob)) <= tol * 8 * scale, prec
        assert np.max(np.abs(gn - on)) <= tol * 8 * scale, prec


# ----------------------------------------------------------------------------
# Fused launches reproduce the reference kernel bit for bit
# ----------------------------------------------------------------------------
# (560, 203): a last strip column of 64-80 output columns and a short last strip row
SHAPES = [(128, 128), (700, 150), (257, 31), (1, 64), (64, 1), (5, 3), (300, 97), (560, 203)]
# (steps per launch, rows per strip, prefetch[, wavefronts per strip])
TUNINGS = [(1, 1, 2), (2, 7, 4), (3, 32, 2), (4, 5, 4), (6, 16, 4), (8, 3, 2), (2, 1000, 2),
           (2, 7, 4, 2), (4, 5, 2, 2), (4, 35, 4, 2), (6, 16, 2, 2), (8, 3, 4, 2), (2, 1000, 2, 2),
           (3, 9, 2, 2)]


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("nx,ny", SHAPES)
def test_fused_launches_bitwise_equal_to_reference(precision, nx, ny):
    b, n, s = workload.fields(nx, ny, 0.8, 0.5, 7, r0=max(1.0, min(nx, ny) / 8.0))
    rng = np.random.default_rng(nx + 7 * ny)
    b = np.maximum(b, rng.uniform(0, 0.3, b.shape).astype(np.float32) *
                   (rng.uniform(size=b.shape) < 0.3))
    dt = 0.1
    steps = 13
    for law in ("receptor", "constant"):
        rb, rn, rd = run_gpu(b, n, s, steps, dt, precision=precision, ref=True, chi=1.7,
                             chi_law=law)
        for tune in TUNINGS:
            gb, gn, gd = run_gpu(b, n, s, steps, dt, precision=precision, tuning=tune, chi=1.7,
                                 chi_law=law)
            assert np.array_equal(gb, rb) and np.array_equal(gn, rn), (law, tune)
            assert gd == rd


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_every_launch_shape_bitwise_equal_to_reference(precision):
    # the whole product of the compiled kernels (Euler 1-8 steps and Runge-Kutta
    # 1-3 steps per launch, both sensitivity laws, both prefetch depths, one or
    # two wavefronts per strip) at short, medium and whole-grid strip heights, on
    # grids of odd and even width and with short last strip rows
    import itertools
    bad = []
    for nx, ny in ((257, 31), (560, 203), (129, 300)):
        b, n, s = workload.fields(nx, ny, 0.8, 0.5, 3, r0=max(1.0, min(nx, ny) / 8.0))
        rng = np.random.default_rng(5 * nx + ny)
        b = np.maximum(b, rng.uniform(0, 0.3, b.shape).astype(np.float32) *
                       (rng.uniform(size=b.shape) < 0.3))
        for law, (integ, depths) in itertools.product(
                ("receptor", "constant"), (("euler", (1, 2, 3, 4, 6, 8)), ("rk2", (1, 2, 3)))):
            rb, rn, _ = run_gpu(b, n, s, 13, 0.1, precision=precision, ref=True, chi=1.7,
                                chi_law=law, integrator=integ)
            for d, rows, pf, w in itertools.product(depths, (3, 16, 1000), (2, 4), (1, 2)):
                gb, gn, _ = run_gpu(b, n, s, 13, 0.1, precision=precision,
                                    tuning=(d, rows, pf, w), chi=1.7, chi_law=law,
                                    integrator=integ)
                if not (np.array_equal(gb, rb) and np.array_equal(gn, rn)):
                    bad.append((nx, ny, law, integ, d, rows, pf, w))
    assert not bad, bad


# Grids whose last strip column holds few output columns: FP32 launches of up to
# four levels fold its strips into bands of one wavefront (8 to 16 bands here).
FOLD_SHAPES = [(1000, 77), (520, 130), (760, 45), (1016, 33)]


def test_folded_last_column_bitwise_equal_to_reference():
    import itertools
    bad = []
    for nx, ny in FOLD_SHAPES:
        b, n, s = workload.fields(nx, ny, 0.8, 0.5, 11, r0=max(1.0, min(nx, ny) / 8.0))
        rng = np.random.default_rng(nx + ny)
        b = np.maximum(b, rng.uniform(0, 0.3, b.shape).astype(np.float32) *
                       (rng.uniform(size=b.shape) < 0.3))
        for law, (integ, depths) in itertools.product(
                ("receptor", "constant"), (("euler", (1, 2, 3, 4)), ("rk2", (1, 2)))):
            rb, rn, rd = run_gpu(b, n, s, 9, 0.1, ref=True, chi=1.7, chi_law=law,
                                 integrator=integ)
            for d, rows, pf, w in itertools.product(depths, (3, 5, 12, 40), (2, 4), (1, 2)):
                gb, gn, gd = run_gpu(b, n, s, 9, 0.1, tuning=(d, rows, pf, w), chi=1.7,
                                     chi_law=law, integrator=integ)
                if not (np.array_equal(gb, rb) and np.array_equal(gn, rn) and gd == rd):
                    bad.append((nx, ny, law, integ, d, rows, pf, w))
    assert not bad, bad


# ----------------------------------------------------------------------------
# Resume, determinism, diagnostics
# ----------------------------------------------------------------------------
def test_resume_is_bitwise():
    b, n, s = workload.fields(200, 160, 0.8, 0.5, 1)
    dt = workload.config_dt(b, n, s)
    full_b, full_n, full_d = run_gpu(b, n, s, 600, dt, chi=0.5)
    hb, hn, _ = run_gpu(b, n, s, 300, dt, chi=0.5)
    S = _solver(200, 160, dt, chi=0.5, step0=300)
    S.set_fields(hb, hn, s)
    assert S.time() == (pytest.approx(300 * dt), 300)
    S.step(300)
    rb, rn = S.get_fields()
    rd = S.diagnostics()
    t, k = S.time()
    S.close()
    assert k == 600 and t == 600 * dt
    assert np.array_equal(rb, full_b) and np.array_equal(rn, full_n) and rd == full_d


def test_runs_are_deterministic_and_diagnostics_match_oracle_on_same_fields():
    b, n, s = workload.fields(333, 211, 0.7, 0.4, 2)
    dt = workload.config_dt(b, n, s)
    r1 = run_gpu(b, n, s, 500, dt, chi=1.0, b_thr=0.35)
    r2 = run_gpu(b, n, s, 500, dt, chi=1.0, b_thr=0.35)
    assert np.array_equal(r1[0], r2[0]) and r1[2] == r2[2]
    m, nu, rad = oracle.diag(r1[0], r1[1], 1.0, 0.35)
    assert r1[2][0] == pytest.approx(m, rel=1e-13)
    assert r1[2][1] == pytest.approx(nu, rel=1e-13)
    assert r1[2][2] == rad


def test_diagnostics_device_and_time():
    b, n, s = workload.fields(64, 48, 0.8, 0.5, 0)
    S = _solver(64, 48, 0.04, chi=0.5, h=0.5, b_thr=0.4, cx=10.0, cy=7.5)
    S.set_fields(b, n, s)
    S.step(37)
    out = torch.zeros(10, dtype=torch.float64, device="cuda")
    S.diagnostics_device(out[5:])
    torch.cuda.synchronize()
    gb, gn = S.get_fields()
    m, nu, r, ra = oracle.diag(gb, gn, 0.5, 0.4, cx=10.0, cy=7.5, area=True)
    o = out.cpu().numpy()
    assert np.all(o[:5] == 0.0)
    assert o[5] == 37 * 0.04
    assert o[6] == pytest.approx(m, rel=1e-13) and o[7] == pytest.approx(nu, rel=1e-13)
    assert o[8] == r and o[9] == ra and ra > 0
    S.close()


# ----------------------------------------------------------------------------
# Error paths through the ABI
# ----------------------------------------------------------------------------
def test_error_paths():
    from paper_1301_5058_amd import native as N
    b, n, s = workload.fields(32, 32, 0.8, 0.5, 0)
    S = _solver(32, 32, 0.2)
    with pytest.raises(N.KcError) as e:
        S.step(1)
    assert e.value.code == N.KC_ESTATE
    with pytest.raises(N.KcError) as e:
        S.diagnostics()
    assert e.value.code == N.KC_ESTATE
    bad = torch.tensor(b, device="cuda")
    bad[3, 4] = float("nan")
    with pytest.raises(N.KcError) as e:
        S.set_fields(bad, torch.tensor(n, device="cuda"), torch.tensor(s, device="cuda"))
    assert e.value.code == N.KC_ENONFINITE
    neg = torch.tensor(s, device="cuda")
    neg[0, 0] = -1.0
    with pytest.raises(N.KcError) as e:
        S.set_fields(torch.tensor(b, device="cuda"), torch.tensor(n, device="cuda"), neg)
    assert e.value.code == N.KC_ENONFINITE
    S.set_fields(torch.tensor(b, device="cuda"), torch.tensor(n, device="cuda"),
                 torch.tensor(s, device="cuda"))
    S.step(3)
    # wavefronts per strip: 1 or 2 only; a depth that does not split in halves
    # of whole steps runs one wavefront per strip with the same bits
    for w in (0, 3, -1):
        assert N.lib().kc_set_strip_waves(S.ctx, w) == N.KC_EINVAL
    S.set_tuning(3, 8, 2, 2)
    assert S.strip_waves() == 2
    S.step(3)
    S.close()
    T = _solver(32, 32, 0.3)  # 0.3 > 1/(4 * 1) : unstable for D_n = 1
    with pytest.raises(N.KcError) as e:
        T.set_fields(b, n, s)
    assert e.value.code == N.KC_EUNSTABLE
    T.close()


# ----------------------------------------------------------------------------
# Full-size workloads in the benchmark's launch configuration: sampled cells
# ----------------------------------------------------------------------------
def _oracle_cell(b, n, s, dt, steps, j, i, reach=1, **kw):
    """Oracle value of cell (j, i) after `steps` steps, from the window of
    cells within `reach * steps + 1` of it (cells farther away cannot reach
    it; reach = Euler stages per step)."""
    ny, nx = b.shape
    w = reach * steps + 1
    j0, j1, i0, i1 = max(0, j - w), min(ny, j + w + 1), max(0, i - w), min(nx, i + w + 1)
    # a window edge inside the domain acts as a wall; it is more than
    # `reach * steps` cells away from (j, i), so the value at (j, i) is exact.
    wb, wn = oracle.run(b[j0:j1, i0:i1], n[j0:j1, i0:i1], s[j0:j1, i0:i1], 1.0, dt, steps, **kw)
    return wb[j - j0, i - i0], wn[j - j0, i - i0]


def _sample_points(nx, ny, rng, k=120):
    cx, cy = (nx - 1) // 2, (ny - 1) // 2
    pts = [(0, 0), (0, nx - 1), (ny - 1, 0), (ny - 1, nx - 1), (cy, cx), (0, cx), (cy, 0),
           (ny - 1, cx), (cy, nx - 1)]
    pts += [(cy + int(dy), cx + int(dx)) for dy, dx in rng.integers(-20, 21, (k // 2, 2))]
    pts += [tuple(p) for p in np.stack([rng.integers(0, ny, k // 2), rng.integers(0, nx, k // 2)], 1)]
    return pts


@pytest.mark.parametrize("cfg,launches", [(workload.SINGLE_4096, 3), (workload.HIRES_16384, 1)])
def test_full_size_sampled_cells_match_oracle(cfg, launches):
    from paper_1301_5058_amd.solver import Solver
    nx, ny = cfg["nx"], cfg["ny"]
    b, n, s = workload.fields(nx, ny, cfg["n0"], cfg["a"], cfg["seed"])
    dt = workload.config_dt(b, n, s)
    S = Solver(nx, ny, dt=dt, chi=cfg["chi"], b_thr=0.5 * cfg["n0"])
    S.set_fields(torch.from_numpy(b).cuda(), torch.from_numpy(n).cuda(), torch.from_numpy(s).cuda())
    # the launch configuration the benchmark times (shipped tuning database)
    tuning = _shipped_tuning("|%dx%d|fp32|receptor" % (nx, ny), exact=True)
    assert tuning is not None
    S.set_tuning(*tuning)
    T = S.tuning()[0]
    steps = T * launches
    # make the colony non-trivial first, in the same configuration
    S.step(steps)
    gb, gn = S.get_fields()
    S.close()
    rng = np.random.default_rng(11)
    worst = 0.0
    for (j, i) in _sample_points(nx, ny, rng):
        eb, en = _oracle_cell(b, n, s, dt, steps, j, i, chi=cfg["chi"])
        worst = max(worst, abs(gb[j, i] - eb), abs(gn[j, i] - en))
    print("%dx%d, %d steps (T=%d): worst sampled abs error %.3e" % (nx, ny, steps, T, worst))
    assert worst <= 2e-6


# ----------------------------------------------------------------------------
# Long horizon: the 512^2 crop of the 16384^2 workload (n0 = 0.35, chi = 2),
# 20000 steps, in the kernel configuration the shipped tuning database gives
# the 16384^2 grid.  The FP32 error of the 128^2 workload after 2000 steps
# (2.5e-5) grown linearly to 20000 steps is 2.5e-4 (measured here: 1.5e-4 for
# b, 4e-5 for n); the bar is twice that, 5e-4.
# ----------------------------------------------------------------------------
def _shipped_tuning(key_part, exact=False):
    import json
    import os
    path = os.path.join(os.path.dirname(__file__), "..", "paper_1301_5058_amd", "tuning",
                        "gfx950.jsonl")
    for line in open(path):
        e = json.loads(line)
        if (e["key"].endswith(key_part) if exact else key_part in e["key"]):
            return e["tsteps"], e["rows"], e["prefetch"], e.get("waves", 1)
    return None


def test_crop_512_long_run_matches_oracle():
    k = workload.CROP_512
    b, n, s = workload.fields(k["nx"], k["ny"], k["n0"], k["a"], k["seed"])
    dt = workload.config_dt(b, n, s)
    tuning = _shipped_tuning("|16384x16384|fp32|receptor")
    assert tuning is not None
    S = _solver(k["nx"], k["ny"], dt, chi=k["chi"], b_thr=0.5 * k["n0"])
    S.set_tuning(*tuning)
    S.set_fields(b, n, s)
    S.step(k["steps"])
    gb, gn = S.get_fields()
    _, mass_g, _, _, area_g = S.diagnostics_all()
    S.close()
    ob, on = oracle.run(b, n, s, 1.0, dt, k["steps"], chi=k["chi"])
    od = oracle.diag(ob, on, 1.0, 0.5 * k["n0"], area=True)
    eb, en = normwise(gb, ob), normwise(gn, on)
    mass = abs(mass_g - od[0]) / od[0]
    print("512^2 x %d steps, tuning %s: normwise b %.3e n %.3e, mass %.3e, area radius %.6f vs %.6f"
          % (k["steps"], tuning, eb, en, mass, area_g, od[3]))
    assert eb <= 5e-4 and en <= 5e-4
    assert mass <= 5e-4
    assert abs(area_g - od[3]) <= 0.005 * od[3]


def test_bench_configuration_whole_field_matches_oracle():
    # the benchmark's own path: the 4096^2 FP32 workload (chi = 1) in the shipped
    # tuning and in the other configuration bench.py may pick on a given GPU (4
    # steps per launch, 46-row strips, prefetch 4, two wavefronts per strip),
    # kc_step_sample every 100 steps, 2000 steps; every cell of both fields
    # against the FP64 oracle, and the last sample's mass and radii
    from paper_1301_5058_amd.solver import Solver
    cfg = workload.SINGLE_4096
    nx, ny = cfg["nx"], cfg["ny"]
    b, n, s = workload.fields(nx, ny, cfg["n0"], cfg["a"], cfg["seed"])
    dt = workload.config_dt(b, n, s)
    shipped = _shipped_tuning("|4096x4096|fp32|receptor", exact=True)
    assert shipped is not None
    steps, every = 2000, 100
    ob, on = oracle.run(b, n, s, 1.0, dt, steps, chi=cfg["chi"])
    m, nu, r, ra = oracle.diag(ob, on, 1.0, 0.5 * cfg["n0"], area=True)
    runs = []
    for tuning in sorted({tuple(shipped), (4, 46, 4, 2)}):
        S = Solver(nx, ny, dt=dt, chi=cfg["chi"], b_thr=0.5 * cfg["n0"])
        S.set_fields(torch.from_numpy(b).cuda(), torch.from_numpy(n).cuda(),
                     torch.from_numpy(s).cuda())
        S.set_tuning(*tuning)
        series = torch.zeros((steps // every, 5), dtype=torch.float64, device="cuda")
        for i in range(steps // every):
            S.step_sample(every, series[i])
        gb, gn = S.get_fields()
        last = series[-1].cpu().numpy()
        S.close()
        eb, en = normwise(gb, ob), normwise(gn, on)
        print("4096^2 x %d steps, tuning %s: normwise b %.3e n %.3e; mass %.9g (oracle %.9g), "
              "envelope radius %.6f (%.6f), area radius %.6f (%.6f)"
              % (steps, tuning, eb, en, last[1], m, last[3], r, last[4], ra))
        assert last[0] == pytest.approx(steps * dt, rel=1e-15)
        assert eb <= 1e-4 and en <= 1e-4
        assert abs(last[1] - m) <= 5e-3 * m and abs(last[2] - nu) <= 5e-3 * nu
        assert abs(last[3] - r) <= 5e-3 * r and abs(last[4] - ra) <= 5e-3 * ra
        runs.append((gb, gn))
    # every launch shape gives the same bits
    assert all(np.array_equal(g[0], runs[0][0]) and np.array_equal(g[1], runs[0][1]) for g in runs)


# ----------------------------------------------------------------------------
# Autotuner: picks a valid configuration, leaves the state alone, uses its cache
# ----------------------------------------------------------------------------
def test_autotune_keeps_state_and_caches(tmp_path, monkeypatch):
    cache = tmp_path / "tune.jsonl"
    monkeypatch.setenv("KC_AUTOTUNE_CACHE", str(cache))
    b, n, s = workload.fields(520, 300, 0.8, 0.5, 3)
    dt = workload.config_dt(b, n, s)
    ref_b, ref_n, ref_d = run_gpu(b, n, s, 40, dt, chi=0.7)
    S = _solver(520, 300, dt, chi=0.7)
    S.set_fields(b, n, s)
    S.step(1)
    before = S.get_fields()
    g = S.autotune(effort=0, use_cache=True)
    assert g > 0
    after = S.get_fields()
    assert np.array_equal(before[0], after[0]) and np.array_equal(before[1], after[1])
    t1 = S.tuning()
    assert t1[0] in (1, 2, 3, 4) and t1[1] >= 1 and t1[2] in (2, 4)
    S.step(39)
    gb, gn = S.get_fields()
    assert np.array_equal(gb, ref_b) and np.array_equal(gn, ref_n)
    assert cache.read_text().count('"key"') == 1
    S.set_tuning(1, 8, 2)
    # answered by the cache: the tuning and the rate stored with it
    assert S.autotune(effort=0, use_cache=True) == round(g, 3)
    assert S.tuning() == t1
    S.close()
