"""Host side of the paper-scale colony runs: the paper's set-up (Sec. 3) and the
shape measures of a snapshot, checked on shapes whose answers are known by
construction (a disk, a star of k arms, an annulus, an empty field)."""
import math

import numpy as np
import pytest

from paper_1301_5058_amd import workload
from paper_1301_5058_amd.colony import envelope_speed, morphology


def _grid(side):
    c = (side - 1) / 2.0
    j, i = np.meshgrid(np.arange(side, dtype=np.float64), np.arange(side, dtype=np.float64),
                       indexing="ij")
    return i - c, j - c


def test_disk_is_compact_and_closed():
    x, y = _grid(401)
    R, h = 150.0, 0.5
    b = (np.hypot(x, y) <= R).astype(np.float32)
    m = morphology(b, h, 0.5)
    # the farthest lattice point inside the disk lies within one cell of R
    assert h * (R - 1) <= m["r_env"] <= h * R
    assert m["r_area"] == pytest.approx(h * R, rel=0.01)
    assert m["compactness"] == pytest.approx(1.0, abs=0.02)
    for r in m["rings"]:
        assert r["cover"] == 1.0 and r["arcs"] == 1
    assert m["b_centre"] == m["b_peak"] == 1.0
    assert m["cells"] == int(b.sum())
    assert m["axis_diag"] == pytest.approx(1.0, abs=0.01)


@pytest.mark.parametrize("shape,ratio", [("diamond", math.sqrt(2)), ("square", 1 / math.sqrt(2))])
def test_axis_diagonal_reach(shape, ratio):
    x, y = _grid(401)
    R = 180.0
    inside = (np.abs(x) + np.abs(y) <= R) if shape == "diamond" else \
        (np.maximum(np.abs(x), np.abs(y)) <= R / math.sqrt(2))
    m = morphology(inside.astype(np.float32), 1.0, 0.5)
    assert m["axis_diag"] == pytest.approx(ratio, rel=0.02)
    # a diamond's corners lie on the axes: its envelope radius is R
    if shape == "diamond":
        assert m["r_env"] == pytest.approx(R, abs=1.0)


@pytest.mark.parametrize("k", [3, 7, 12])
def test_star_arms_are_counted_as_arcs(k):
    x, y = _grid(501)
    R, w = 240.0, 6.0
    d = np.hypot(x, y)
    mask = np.zeros(x.shape, dtype=bool)
    for a in range(k):
        # arm a along angle 2 pi a / k; arm 0 lies on the +x axis, where the
        # ring's samples wrap around from the last to the first
        th = 2.0 * math.pi * a / k
        along = x * math.cos(th) + y * math.sin(th)
        perp = -x * math.sin(th) + y * math.cos(th)
        mask |= (along >= 0) & (np.abs(perp) <= w / 2) & (d <= R)
    b = np.where(mask, 0.8, 0.0).astype(np.float32)
    m = morphology(b, 1.0, 0.4)
    assert m["r_env"] == pytest.approx(R, abs=1.0)
    for r in m["rings"]:
        assert r["arcs"] == k
        rho = r["f"] * m["r_env"]
        assert r["cover"] == pytest.approx(k * (w + 1) / (2 * math.pi * rho), rel=0.25)
    # area of k arms of width ~w and length R against the disk of radius R
    assert m["compactness"] == pytest.approx(k * (w + 1) * R / (math.pi * R * R), rel=0.25)
    assert m["compactness"] < 0.2


def test_annulus_shows_a_central_depression():
    x, y = _grid(201)
    d = np.hypot(x, y)
    b = (0.9 * np.exp(-((d - 40.0) / 15.0) ** 2)).astype(np.float32)
    m = morphology(b, 1.0, 0.3)
    assert m["b_centre"] < 0.2 * m["b_peak"]
    # the inner hole is not part of the colony: the ring at half the envelope
    # radius lies in the band and is closed
    assert m["rings"][0]["arcs"] == 1 and m["rings"][0]["cover"] == 1.0
    assert m["compactness"] < 0.9


def test_empty_field():
    m = morphology(np.zeros((32, 40), np.float32), 1.0, 0.1)
    assert m["cells"] == 0 and m["r_env"] == 0.0 and m["r_area"] == 0.0
    assert all(r["arcs"] == 0 for r in m["rings"])


def test_off_centre_colony_uses_the_given_centre():
    x, y = _grid(101)
    b = (np.hypot(x - 20, y + 10) <= 8).astype(np.float32)
    m = morphology(b, 1.0, 0.5, cx=50 + 20, cy=50 - 10)
    assert m["r_env"] == pytest.approx(8.0, abs=1.0)
    assert m["compactness"] == pytest.approx(1.0, abs=0.1)


def test_paper_inoculum():
    """b_M exp(-(x^2+y^2)/6.25) in physical coordinates about the centre of the
    square (eq. inibacexp), cut beyond three radii; uniform nutrient."""
    c = workload.PAPER_2D
    cells, L = 256, 680.0 * 256 / 2048  # the paper's h on a smaller square
    h = L / cells
    b, n = workload.paper_fields(cells, L, 0.71)
    assert n.dtype == np.float32 and np.all(n == np.float32(0.71))
    X = (np.arange(cells) + 0.5) * h - L / 2
    xx, yy = np.meshgrid(X, X)
    r2 = xx ** 2 + yy ** 2
    want = c["b_max"] * np.exp(-r2 / 6.25)
    inside = r2 <= (c["cut"] * c["r0"]) ** 2 * (1 - 1e-12)
    np.testing.assert_allclose(b[inside], want[inside].astype(np.float32), rtol=2e-7)
    assert np.all(b[r2 > (c["cut"] * c["r0"]) ** 2 * (1 + 1e-12)] == 0)
    assert b.max() == np.float32(c["b_max"] * math.exp(-h * h / 12.5))


def test_paper_time_steps():
    """The paper's step where it keeps the explicit bound, else 0.95 of it."""
    h = 680.0 / 2048
    s1 = workload.PAPER_SETS["set1"]
    dt1 = workload.paper_dt(2048, 680.0, s1["sigma0"], s1["n0"], s1["dt"])
    assert dt1 == float(np.float32(0.02315))
    # Set 1's captions: 30000, 60000 and 90000 steps
    assert [round(t / dt1) for t in s1["times"][:3]] == [30000, 60000, 90000]
    for name in ("set2", "set3a", "set3b", "set4"):
        s = workload.PAPER_SETS[name]
        dt = workload.paper_dt(2048, 680.0, s["sigma0"], s["n0"], s["dt"])
        B = 0.5 * (s["n0"] + 0.71)
        bound = h * h / (4 * max(1.0, 2 * s["sigma0"] * B * B))
        assert dt < s["dt"] and dt == pytest.approx(0.95 * bound, rel=1e-6)
        # the library's own check on the initial fields: sigma0 (1 + a) max(n b)
        assert dt <= h * h / (4 * max(1.0, 2 * s["sigma0"] * s["n0"] * 0.71))


def test_envelope_speed_is_the_least_squares_slope_before_the_wall():
    snaps = [dict(t=t, r_env=5.0 + 0.25 * t + e) for t, e in ((10, 0.1), (20, -0.1), (30, 0.0))]
    # slope 0.25 plus that of the offsets: (-10 * 0.1 + 10 * 0.0) / 200 = -0.005
    assert envelope_speed(snaps, 100.0) == pytest.approx(0.245, abs=1e-12)
    # a snapshot at the wall is left out; with one left there is no slope
    snaps.append(dict(t=400.0, r_env=99.0))
    assert envelope_speed(snaps, 100.0) == pytest.approx(0.245, abs=1e-12)
    assert envelope_speed(snaps[:1] + snaps[3:], 100.0) is None
