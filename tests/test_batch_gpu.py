"""Batched sweep (kb_*) on the GPU: every instance of a batch must reproduce
the single-instance solver bit for bit, the device-side samples must equal
the single-instance diagnostics, the persistent launch must equal one launch
per time block, and the velocity fit must equal the oracle's fit of the same
series."""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_1301_5058_amd import workload

pytestmark = pytest.mark.gpu

INSTANCES = [
    dict(nx=64, ny=64, n0=0.8, a=0.5, chi=0.5, seed=1),
    dict(nx=100, ny=77, n0=1.1, a=0.2, chi=1.7, seed=2),
    dict(nx=300, ny=130, n0=0.4, a=0.4, chi=0.0, seed=3),
    dict(nx=1, ny=50, n0=0.9, a=0.3, chi=1.0, seed=4),
    dict(nx=257, ny=256, n0=0.6, a=0.1, chi=2.0, seed=5),
    dict(nx=33, ny=3, n0=0.7, a=0.5, chi=0.3, seed=6),
]


def _setup(insts, law="receptor", **kw):
    from paper_1301_5058_amd.batch import Batch
    fields, descs = [], []
    for d in insts:
        b, n, s = workload.fields(d["nx"], d["ny"], d["n0"], d["a"], d["seed"],
                                  r0=max(1.0, min(6.0, min(d["nx"], d["ny"]) / 6.0)))
        dt = workload.config_dt(b, n, s)
        fields.append((b, n, s))
        descs.append(dict(nx=d["nx"], ny=d["ny"], dt=dt, chi=d["chi"], b_thr=0.5 * d["n0"]))
    B = Batch(descs, chi_law=law, **kw)
    for k, (b, n, s) in enumerate(fields):
        B.set_fields(k, b, n, s)
    return B, fields, descs


def _single(b, n, s, desc, steps, every, law="receptor"):
    from paper_1301_5058_amd.solver import Solver
    S = Solver(desc["nx"], desc["ny"], dt=desc["dt"], chi=desc["chi"], chi_law=law,
               b_thr=desc["b_thr"])
    S.set_fields(b, n, s)
    diags = []
    for _ in range(steps // every):
        S.step(every)
        diags.append(S.diagnostics_all())
    fb, fn = S.get_fields()
    S.close()
    return fb, fn, np.array(diags)


@pytest.mark.parametrize("law", ["receptor", "constant"])
def test_batch_matches_single_instance_bitwise(law):
    steps, every = 120, 20
    B, fields, descs = _setup(INSTANCES, law=law, max_samples=64)
    B.run(steps, every)
    ser = B.series()
    assert ser.shape == (len(INSTANCES), steps // every, 5)
    for k, ((b, n, s), d) in enumerate(zip(fields, descs)):
        fb, fn, diags = _single(b, n, s, d, steps, every, law)
        gb, gn = B.get_fields(k)
        assert np.array_equal(gb, fb) and np.array_equal(gn, fn), k
        assert np.array_equal(ser[k][:, [0, 3, 4]], diags[:, [0, 3, 4]])
        np.testing.assert_allclose(ser[k, :, 1:3], diags[:, 1:3], rtol=1e-13, atol=0)
    B.close()


def test_persistent_equals_per_block_launches_and_any_tuning():
    steps, every = 96, 24
    ref = None
    for tune in [dict(persistent=0, tsteps=1), dict(persistent=1, tsteps=2),
                 dict(persistent=1, tsteps=4, rows=5, prefetch=2),
                 dict(persistent=1, tsteps=8, rows=64), dict(persistent=0, tsteps=3, rows=7)]:
        B, _, _ = _setup(INSTANCES, max_samples=16)
        B.set_tuning(**tune)
        B.run(steps // 2, every)
        B.run(steps // 2, every)
        got = (B.series(), [B.get_fields(k) for k in range(len(INSTANCES))])
        assert B.steps() == steps
        B.close()
        if ref is None:
            ref = got
            continue
        # fields, times and radii are exact; the double sums are folded per strip,
        # so another strip partition changes their rounding only
        assert np.array_equal(got[0][..., [0, 3, 4]], ref[0][..., [0, 3, 4]]), tune
        np.testing.assert_allclose(got[0][..., 1:3], ref[0][..., 1:3], rtol=1e-13, atol=0)
        for (a, b_), (c, d) in zip(got[1], ref[1]):
            assert np.array_equal(a, c) and np.array_equal(b_, d), tune


def test_instance_matches_oracle():
    d = INSTANCES[1]
    B, fields, descs = _setup([d], max_samples=8)
    B.run(400, 100)
    gb, gn = B.get_fields(0)
    b, n, s = fields[0]
    ob, on = oracle.run(b, n, s, 1.0, descs[0]["dt"], 400, chi=d["chi"])
    assert np.max(np.abs(gb - ob)) / np.max(ob) <= 1e-4
    assert np.max(np.abs(gn - on)) / np.max(on) <= 1e-4
    m, nu, r, ra = oracle.diag(ob, on, 1.0, descs[0]["b_thr"], area=True)
    ser = B.series()
    assert abs(ser[0, -1, 1] - m) / m <= 5e-3 and abs(ser[0, -1, 3] - r) <= max(1.0, 5e-3 * r)
    assert abs(ser[0, -1, 4] - ra) <= 5e-3 * ra
    B.close()


def test_velocity_fit_equals_oracle_fit_of_same_series():
    insts = [dict(nx=160, ny=160, n0=0.9, a=0.3, chi=c, seed=k) for k, c in enumerate((0.0, 2.0))]
    B, _, _ = _setup(insts, max_samples=64)
    B.run(3000, 100)
    ser = B.series()
    lo, hi = np.array([8.0, 8.0]), np.array([60.0, 60.0])
    for col, radius in ((3, "envelope"), (4, "area")):
        v, npts = B.fit_velocity(lo, hi, radius=radius)
        for k in range(2):
            vo, ko = oracle.fit_velocity(ser[k, :, 0], ser[k, :, col], lo[k], hi[k])
            assert npts[k] == ko and ko >= 3
            assert v[k] == pytest.approx(vo, rel=1e-12)
        # chemotaxis speeds the envelope up (abstract; Sec. 3.1; Sec. 4.1 eq. speedinq)
        assert v[1] > v[0] > 0
    v2, n2 = B.fit_velocity(1e6, 2e6)
    assert np.all(np.isnan(v2)) and np.all(n2 == 0)
    # kb_fit_velocity_until: only the samples up to each instance's t_max
    t_max = np.array([ser[0, 17, 0], ser[1, 24, 0]])
    v3, n3 = B.fit_velocity(lo, hi, t_max=t_max)
    for k in range(2):
        sel = ser[k, :, 0] <= t_max[k]
        vo, ko = oracle.fit_velocity(ser[k, sel, 0], ser[k, sel, 3], lo[k], hi[k])
        assert n3[k] == ko and v3[k] == pytest.approx(vo, rel=1e-12)
    v4, _ = B.fit_velocity(lo, hi, t_max=np.inf)
    assert np.array_equal(v4, B.fit_velocity(lo, hi)[0])
    from paper_1301_5058_amd import native as N
    with pytest.raises(N.KcError) as e:
        B.fit_velocity(lo, hi, t_max=np.nan)
    assert e.value.code == N.KC_EINVAL
    B.close()


def test_error_paths_and_bounded_wait():
    from paper_1301_5058_amd import native as N
    from paper_1301_5058_amd.batch import Batch
    B = Batch([dict(nx=512, ny=512, dt=0.2, chi=0.5, b_thr=0.4)], max_samples=4)
    with pytest.raises(N.KcError) as e:
        B.run(10, 10)
    assert e.value.code == N.KC_ESTATE
    b, n, s = workload.fields(512, 512, 0.8, 0.5, 0)
    B.set_fields(0, b, n, s)
    with pytest.raises(N.KcError) as e:
        B.run(15, 10)
    assert e.value.code == N.KC_EINVAL
    with pytest.raises(N.KcError) as e:
        B.run(50, 10)  # 5 samples > capacity 4
    assert e.value.code == N.KC_EINVAL
    # a one-poll bound on the persistent kernel's waits: items of the second
    # time block are handed out while the first block is still running, so a
    # wait cannot be satisfied at its first poll and the launch stops cleanly
    B.set_tuning(tsteps=1, rows=8, persistent=1)
    B.set_spin_limit(1)
    with pytest.raises(N.KcError) as e:
        B.run(40, 10)
    assert e.value.code == N.KC_EHIP
    # the stopped launch may have overwritten part of a level: the fields must be
    # set again before the batch runs or returns them
    B.set_spin_limit(1 << 23)
    with pytest.raises(N.KcError) as e:
        B.run(40, 10)
    assert e.value.code == N.KC_ESTATE
    with pytest.raises(N.KcError) as e:
        B.get_fields(0)
    assert e.value.code == N.KC_ESTATE
    B.set_fields(0, b, n, s)
    B.run(40, 10)
    assert B.nsamples() == 4
    B.close()


def test_batch_autotune_keeps_results():
    steps, every = 60, 20
    B0, _, _ = _setup(INSTANCES, max_samples=8)
    B0.run(steps, every)
    ref = (B0.series(), [B0.get_fields(k) for k in range(len(INSTANCES))])
    B0.close()
    B, _, _ = _setup(INSTANCES, max_samples=8)
    B.autotune(every, effort=0)
    T, rows, pf, _p = B.tuning()
    assert every % T == 0 and np.all(rows >= 1) and pf in (2, 4) and _p == 0
    B.run(steps, every)
    ser = B.series()
    assert np.array_equal(ser[..., [0, 3, 4]], ref[0][..., [0, 3, 4]])
    np.testing.assert_allclose(ser[..., 1:3], ref[0][..., 1:3], rtol=1e-13, atol=0)
    for k in range(len(INSTANCES)):
        gb, gn = B.get_fields(k)
        assert np.array_equal(gb, ref[1][k][0]) and np.array_equal(gn, ref[1][k][1])
    B.close()


ROWS = [(400, 0.71, 5.0), (64, 1.07, 2.5), (333, 2.0, 0.0), (512, 0.35, 10.0), (5, 1.0, 1.0),
        (257, 3.0, 1.0)]


@pytest.mark.parametrize("law", ["constant", "receptor"])
def test_single_row_batch_matches_the_single_instance_solver(law):
    """A batch of single rows (ny = 1, at most 512 cells: the 1-D front
    experiment's shape) runs in one launch per kb_run; every instance equals
    the single-instance solver on the same nx x 1 grid: fields bit for bit,
    time and radii exactly, mass and nutrient to 1e-13."""
    from paper_1301_5058_amd.batch import Batch
    from paper_1301_5058_amd.solver import Solver
    c = workload.FRONT1D
    descs, fields = [], []
    for nx, n0, chi in ROWS:
        h = c["length"] / 400
        b, n, s = workload.front1d_fields(nx, nx * h, n0)
        s = (s * np.linspace(0.7, 1.3, nx, dtype=np.float32)[None, :]).astype(np.float32)
        dt = workload.front1d_dt(nx, nx * h, n0, chi)
        descs.append(dict(nx=nx, ny=1, h=h, dt=dt, chi=chi, b_thr=0.5 * n0, cx=-0.5, cy=0.0))
        fields.append((b, n, s))
    every, blocks = 70, 9  # 70 steps between samples: not a multiple of any launch depth
    B = Batch(descs, chi_law=law, max_samples=2 * blocks)
    for k, (b, n, s) in enumerate(fields):
        B.set_fields(k, b, n, s)
    B.run(every * 5, every)
    B.run(every * (blocks - 5), every)  # a second run continues the series
    series = B.series()
    out = [B.get_fields(k) for k in range(len(descs))]
    B.close()
    for k, d in enumerate(descs):
        b, n, s = fields[k]
        S = Solver(d["nx"], 1, h=d["h"], dt=d["dt"], chi=d["chi"], chi_law=law,
                   b_thr=d["b_thr"], cx=-0.5, cy=0.0)
        S.set_fields(b, n, s)
        for i in range(blocks):
            S.step(every)
            t, mass, nut, re, ra = S.diagnostics_all()
            row = series[k, i]
            assert row[0] == t and row[3] == re and row[4] == ra, (k, i, row, (t, re, ra))
            np.testing.assert_allclose(row[1:3], [mass, nut], rtol=1e-13, atol=0)
        gb, gn = S.get_fields()
        S.close()
        assert np.array_equal(out[k][0], gb) and np.array_equal(out[k][1], gn), k
