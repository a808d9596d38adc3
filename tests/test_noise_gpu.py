"""Per-step agar noise (Sec. 3) on the GPU, through the C ABI.

sigma = sigma0 (1 + a Delta), Delta triangular, redrawn at every cell and
time step from Philox4x32-10 (kc.h).  The FP64 kernels draw exactly the
oracle's sigma and match it to 1e-10 normwise; FP32 within 1e-4 after 2000
steps as for the static field; every fused launch shape bitwise equals the
reference kernel; runs split into pieces equal one run.
"""
import numpy as np
import pytest

import oracle
from paper_1301_5058_amd import workload
from test_parity_gpu import normwise

pytestmark = pytest.mark.gpu

NOISE = dict(sigma0=1.0, amp=0.5, seed=(3 << 32) | 77)


def _run(b, n, steps, dt, precision="fp32", tuning=None, ref=False, noise=NOISE, pieces=(),
         **kw):
    from paper_1301_5058_amd.solver import Solver
    ny, nx = b.shape
    S = Solver(nx, ny, dt=dt, precision=precision, noise=noise, **kw)
    if tuning:
        S.set_tuning(*tuning)
    if ref:
        S.use_reference_kernel()
    dtp = np.float32 if precision == "fp32" else np.float64
    S.set_fields(b.astype(dtp), n.astype(dtp))
    done = 0
    for p in pieces:
        S.step(p)
        done += p
    S.step(steps - done)
    out = S.get_fields()
    S.close()
    return out


def _fields(nx, ny, seed=0):
    b, n, _ = workload.fields(nx, ny, 0.8, 0.0, seed)
    return b, n


@pytest.mark.parametrize("integrator", ["euler", "rk2"])
def test_noise_fp64_matches_oracle(integrator):
    b, n = _fields(96, 80)
    dt = 0.2 / max(1.0, 0.8 * 0.7 * 1.5)  # the usual 0.2 h^2 / max(D_n, max sigma n b)
    steps = 300
    gb, gn = _run(b, n, steps, dt, precision="fp64", integrator=integrator, chi=0.5)
    ob, on = oracle.run_noise(b, n, 1.0, dt, steps, NOISE["sigma0"], NOISE["amp"], NOISE["seed"],
                              integrator=integrator, chi=0.5)
    print("noise fp64 %s: normwise b %.2e n %.2e" % (integrator, normwise(gb, ob), normwise(gn, on)))
    assert normwise(gb, ob) <= 1e-10 and normwise(gn, on) <= 1e-10


def test_noise_small_workload_fp32_matches_oracle():
    c = workload.SMALL_128
    b, n = _fields(c["nx"], c["ny"])
    dt = 0.2 / max(1.0, 0.8 * 0.7 * 1.5)
    gb, gn = _run(b, n, c["steps"], dt, chi=c["chi"])
    ob, on = oracle.run_noise(b, n, 1.0, dt, c["steps"], NOISE["sigma0"], NOISE["amp"],
                              NOISE["seed"], chi=c["chi"])
    print("noise fp32 128^2 x 2000: normwise b %.2e n %.2e" % (normwise(gb, ob), normwise(gn, on)))
    assert normwise(gb, ob) <= 1e-4 and normwise(gn, on) <= 1e-4
    # the agar noise changes the run
    sb, _, _ = workload.fields(c["nx"], c["ny"], 0.8, 0.0, 0)
    ones = np.ones_like(b)
    qb, _ = oracle.run(b, n, ones, 1.0, dt, c["steps"], chi=c["chi"])
    assert normwise(gb, qb) > 1e-3


SHAPES = [(128, 128), (257, 31), (64, 1), (1, 40), (300, 97), (560, 203)]
TUNINGS = [(1, 1, 2), (2, 7, 4), (3, 16, 2), (4, 35, 4), (8, 3, 4), (6, 1000, 2),
           (2, 7, 4, 2), (4, 35, 2, 2), (8, 3, 2, 2)]


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("nx,ny", SHAPES)
def test_noise_fused_launches_bitwise_equal_to_reference(precision, nx, ny):
    b, n = _fields(nx, ny, 5)
    rng = np.random.default_rng(nx * 3 + ny)
    b = np.maximum(b, rng.uniform(0, 0.3, b.shape).astype(np.float32) *
                   (rng.uniform(size=b.shape) < 0.3))
    dt = 0.08
    for integ, tunes in (("euler", TUNINGS),
                         ("rk2", [(1, 5, 2), (2, 9, 4), (3, 100, 4), (2, 19, 2, 2), (2, 4, 4, 2)])):
        rb, rn = _run(b, n, 11, dt, precision=precision, ref=True, integrator=integ, chi=1.3)
        for t in tunes:
            gb, gn = _run(b, n, 11, dt, precision=precision, tuning=t, integrator=integ, chi=1.3)
            assert np.array_equal(gb, rb) and np.array_equal(gn, rn), (integ, t)


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_noise_every_launch_shape_bitwise_equal_to_reference(precision):
    # every compiled depth (Euler 1-8 steps, Runge-Kutta 1-3), short / medium /
    # single-row-of-strips heights, both prefetch depths, one or two wavefronts
    # per strip, on grids of odd and even width and with short last strip rows
    import itertools
    bad = []
    for nx, ny in ((257, 31), (560, 203), (129, 300)):
        b, n = _fields(nx, ny, 5)
        rng = np.random.default_rng(nx * 3 + ny)
        b = np.maximum(b, rng.uniform(0, 0.3, b.shape).astype(np.float32) *
                       (rng.uniform(size=b.shape) < 0.3))
        for integ, depths in (("euler", (1, 2, 3, 4, 6, 8)), ("rk2", (1, 2, 3))):
            rb, rn = _run(b, n, 13, 0.08, precision=precision, ref=True, integrator=integ,
                          chi=1.3)
            for d, rows, pf, w in itertools.product(depths, (3, 16, 1000), (2, 4), (1, 2)):
                gb, gn = _run(b, n, 13, 0.08, precision=precision, tuning=(d, rows, pf, w),
                              integrator=integ, chi=1.3)
                if not (np.array_equal(gb, rb) and np.array_equal(gn, rn)):
                    bad.append((nx, ny, integ, d, rows, pf, w))
    assert not bad, bad


def test_noise_folded_last_column_bitwise_equal_to_reference():
    # grids whose last strip column folds (FP32 launches of up to four levels)
    import itertools
    from test_parity_gpu import FOLD_SHAPES
    bad = []
    for nx, ny in FOLD_SHAPES:
        b, n = _fields(nx, ny, 7)
        rng = np.random.default_rng(nx + ny)
        b = np.maximum(b, rng.uniform(0, 0.3, b.shape).astype(np.float32) *
                       (rng.uniform(size=b.shape) < 0.3))
        for integ, depths in (("euler", (1, 2, 3, 4)), ("rk2", (1, 2))):
            rb, rn = _run(b, n, 9, 0.08, ref=True, integrator=integ, chi=1.3)
            for d, rows, pf, w in itertools.product(depths, (3, 5, 12, 40), (2, 4), (1, 2)):
                gb, gn = _run(b, n, 9, 0.08, tuning=(d, rows, pf, w), integrator=integ, chi=1.3)
                if not (np.array_equal(gb, rb) and np.array_equal(gn, rn)):
                    bad.append((nx, ny, integ, d, rows, pf, w))
    assert not bad, bad


def test_noise_runs_split_seeded_and_resumed():
    b, n = _fields(300, 200, 2)
    dt = 0.2 / max(1.0, 0.8 * 0.7 * 1.5)  # the usual 0.2 h^2 / max(D_n, max sigma n b)
    one = _run(b, n, 40, dt, chi=0.5)
    split = _run(b, n, 40, dt, chi=0.5, pieces=(3, 13, 7))
    assert np.array_equal(one[0], split[0]) and np.array_equal(one[1], split[1])
    other = _run(b, n, 40, dt, chi=0.5, noise=dict(NOISE, seed=NOISE["seed"] + 1))
    assert not np.array_equal(one[0], other[0])
    # resuming at step0 = 15 from the state after 15 steps continues the same draws
    from paper_1301_5058_amd.solver import Solver
    S = Solver(300, 200, dt=dt, chi=0.5, noise=NOISE)
    S.set_fields(b, n)
    S.step(15)
    mb, mn = S.get_fields()
    S.close()
    S = Solver(300, 200, dt=dt, chi=0.5, noise=NOISE, step0=15)
    S.set_fields(mb, mn)
    S.step(25)
    rb, rn = S.get_fields()
    S.close()
    assert np.array_equal(rb, one[0]) and np.array_equal(rn, one[1])


def test_noise_stability_bound_uses_the_largest_drawn_sigma():
    from paper_1301_5058_amd.native import KcError
    from paper_1301_5058_amd.solver import Solver
    b, n, _ = workload.fields(64, 64, 2.0, 0.0, 0)
    # max n b = 2 * 0.7 = 1.4 > D_n: with sigma up to 1.5 the bound is
    # 1 / (4 * 2.1) = 0.119 (with sigma = 1 it would be 0.179)
    S = Solver(64, 64, dt=0.15, chi=0.5, noise=NOISE)
    with pytest.raises(KcError):
        S.set_fields(b, n)
    S.close()
    S = Solver(64, 64, dt=0.11, chi=0.5, noise=NOISE)
    S.set_fields(b, n)
    S.close()
