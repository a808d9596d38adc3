"""The two-stage Runge-Kutta integrator (Sec. 3) on the GPU, through the C ABI.

u' = (u + E(E(u))) / 2 with E one forward-Euler step.  Tolerances as for
forward Euler (tests/test_parity_gpu.py): FP32 fields within 1e-4 normwise of
the FP64 oracle after 2000 steps, FP64 within 1e-10; every fused launch shape
bitwise equal to the reference path (two global-memory Euler launches, the
second averaging with the step's input).
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1301_5058_amd import workload
from test_parity_gpu import _oracle_cell, _sample_points, normwise, run_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def small_rk2_oracle():
    c = workload.SMALL_128
    b, n, s = workload.fields(c["nx"], c["ny"], c["n0"], c["a"], c["seed"])
    dt = workload.config_dt(b, n, s)
    ob, on = oracle.run(b, n, s, 1.0, dt, c["steps"], integrator="rk2", chi=c["chi"])
    od = oracle.diag(ob, on, 1.0, 0.5 * c["n0"])
    return (b, n, s, dt), (ob, on, od)


@pytest.mark.parametrize("precision,tol", [("fp32", 1e-4), ("fp64", 1e-10)])
def test_rk2_small_workload_matches_oracle(small_rk2_oracle, precision, tol):
    (b, n, s, dt), (ob, on, od) = small_rk2_oracle
    c = workload.SMALL_128
    gb, gn, gd = run_gpu(b, n, s, c["steps"], dt, precision=precision, integrator="rk2",
                         chi=c["chi"], b_thr=0.5 * c["n0"])
    eb, en = normwise(gb, ob), normwise(gn, on)
    print("rk2 %s 128^2 x 2000: normwise b %.3e n %.3e" % (precision, eb, en))
    assert eb <= tol and en <= tol
    assert abs(gd[0] - od[0]) / od[0] <= (5e-3 if precision == "fp32" else 1e-12)
    assert od[2] > 10.0 and abs(gd[2] - od[2]) / od[2] <= 5e-3


def test_rk2_differs_from_euler():
    # the integrator flag reaches the kernels: one step of each differs
    b, n, s = workload.fields(96, 80, 0.8, 0.5, 2)
    dt = workload.config_dt(b, n, s)
    e = run_gpu(b, n, s, 1, dt, chi=0.5)
    r = run_gpu(b, n, s, 1, dt, chi=0.5, integrator="rk2")
    ob, on = oracle.run(b, n, s, 1.0, dt, 1, integrator="rk2", chi=0.5)
    assert not np.array_equal(e[0], r[0])
    assert normwise(r[0], ob) <= 1e-6 and normwise(r[1], on) <= 1e-6


SHAPES = [(128, 128), (700, 150), (257, 31), (1, 64), (64, 1), (5, 3), (300, 97), (560, 203)]
TUNINGS = [(1, 1, 2), (1, 9, 4), (2, 7, 4), (2, 35, 2), (3, 16, 4), (3, 3, 2), (4, 1000, 4),
           (2, 7, 2, 2), (2, 19, 4, 2), (2, 1000, 2, 2), (1, 5, 2, 2)]


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("nx,ny", SHAPES)
def test_rk2_fused_launches_bitwise_equal_to_reference(precision, nx, ny):
    b, n, s = workload.fields(nx, ny, 0.8, 0.5, 7, r0=max(1.0, min(nx, ny) / 8.0))
    rng = np.random.default_rng(nx + 7 * ny)
    b = np.maximum(b, rng.uniform(0, 0.3, b.shape).astype(np.float32) *
                   (rng.uniform(size=b.shape) < 0.3))
    dt = 0.1
    steps = 11
    for law in ("receptor", "constant"):
        rb, rn, rd = run_gpu(b, n, s, steps, dt, precision=precision, ref=True, chi=1.7,
                             chi_law=law, integrator="rk2")
        for tune in TUNINGS:
            gb, gn, gd = run_gpu(b, n, s, steps, dt, precision=precision, tuning=tune, chi=1.7,
                                 chi_law=law, integrator="rk2")
            assert np.array_equal(gb, rb) and np.array_equal(gn, rn), (law, tune)
            assert gd == rd


def test_rk2_full_size_sampled_cells_match_oracle():
    from paper_1301_5058_amd.solver import Solver
    cfg = workload.SINGLE_4096
    nx, ny = cfg["nx"], cfg["ny"]
    b, n, s = workload.fields(nx, ny, cfg["n0"], cfg["a"], cfg["seed"])
    dt = workload.config_dt(b, n, s)
    S = Solver(nx, ny, dt=dt, chi=cfg["chi"], b_thr=0.5 * cfg["n0"], integrator="rk2")
    S.set_fields(torch.from_numpy(b).cuda(), torch.from_numpy(n).cuda(), torch.from_numpy(s).cuda())
    T = S.tuning()[0]
    steps = 2 * T
    S.step(steps)
    gb, gn = S.get_fields()
    S.close()
    rng = np.random.default_rng(12)
    worst = 0.0
    for (j, i) in _sample_points(nx, ny, rng, k=60):
        eb, en = _oracle_cell(b, n, s, dt, steps, j, i, reach=2, chi=cfg["chi"], integrator="rk2")
        worst = max(worst, abs(gb[j, i] - eb), abs(gn[j, i] - en))
    print("rk2 %dx%d, %d steps (T=%d): worst sampled abs error %.3e" % (nx, ny, steps, T, worst))
    assert worst <= 2e-6


def test_rk2_autotune_and_cache_key(tmp_path, monkeypatch):
    cache = tmp_path / "tune.jsonl"
    monkeypatch.setenv("KC_AUTOTUNE_CACHE", str(cache))
    from paper_1301_5058_amd.solver import Solver
    b, n, s = workload.fields(520, 300, 0.8, 0.5, 3)
    dt = workload.config_dt(b, n, s)
    ref = run_gpu(b, n, s, 9, dt, chi=0.7, integrator="rk2")
    S = Solver(520, 300, dt=dt, chi=0.7, integrator="rk2")
    S.set_fields(b, n, s)
    assert S.autotune(effort=0, use_cache=True) > 0
    t = S.tuning()
    assert 1 <= t[0] <= 3
    S.step(9)
    gb, gn = S.get_fields()
    assert np.array_equal(gb, ref[0]) and np.array_equal(gn, ref[1])
    S.close()
    text = cache.read_text()
    assert text.count('"key"') == 1 and "|rk2" in text
