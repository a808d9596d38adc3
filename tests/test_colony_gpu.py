"""The paper's two-dimensional set-up (Sec. 3) on the GPU, through the C ABI:
cell width 680 / 2048, noise amplitude 1 (sigma = sigma0 (1 + Delta), so sigma
reaches 0 and 2 sigma0), the two-stage Runge-Kutta method, sensitivities up to
chi0 = 7.5, against the oracle; and the colony runner's records against the
library's own diagnostics."""
import numpy as np
import pytest
import torch

import oracle
from paper_1301_5058_amd import colony, workload
from test_parity_gpu import normwise

pytestmark = pytest.mark.gpu

H = 680.0 / 2048


def _solver(cells, s, chi, precision, seed=1, step0=0):
    from paper_1301_5058_amd.solver import Solver
    dt = workload.paper_dt(2048, 680.0, s["sigma0"], s["n0"], s["dt"])
    noise = dict(sigma0=s["sigma0"], amp=1.0, seed=seed)
    S = Solver(cells, cells, h=H, dt=dt, chi=chi, precision=precision, integrator="rk2",
               noise=noise, b_thr=0.5 * s["n0"], step0=step0)
    return S, dt, noise


@pytest.mark.parametrize("name,chi,steps", [("set1", 5.0, 1500), ("set3b", 7.5, 2500),
                                            ("set4", 7.5, 2500)])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_paper_setup_small_square_matches_oracle(name, chi, steps, precision):
    """A 160^2 square at the paper's cell width from the paper's inoculum."""
    s = workload.PAPER_SETS[name]
    cells = 160
    b, n = workload.paper_fields(cells, cells * H, s["n0"])
    S, dt, noise = _solver(cells, s, chi, precision)
    dtp = np.float32 if precision == "fp32" else np.float64
    S.set_fields(b.astype(dtp), n.astype(dtp))
    S.step(steps)
    gb, gn = S.get_fields()
    S.close()
    ob, on = oracle.run_noise(b, n, H, dt, steps, noise["sigma0"], 1.0, noise["seed"],
                              integrator="rk2", chi=chi)
    eb, en = normwise(gb, ob), normwise(gn, on)
    print("%s chi0=%g %s, %d steps: normwise b %.2e n %.2e" % (name, chi, precision, steps, eb, en))
    tol = 1e-10 if precision == "fp64" else 1e-4
    assert eb <= tol and en <= tol
    # the colony has spread beyond the inoculum's support (radius 7.5)
    assert colony.morphology(ob, H, 0.5 * s["n0"])["r_env"] > 8.0


def test_paper_scale_grid_matches_oracle_in_the_runner_configuration(monkeypatch):
    """2048^2 with the kernel configuration the colony runner picks (the
    shipped tuning table), two launches from a state that has bacteria in every
    strip, against the oracle over the whole grid."""
    import os
    monkeypatch.setenv("KC_AUTOTUNE_CACHE", os.path.join(
        os.path.dirname(colony.__file__), "tuning", "gfx950.jsonl"))
    s = workload.PAPER_SETS["set3b"]
    cells, chi = 2048, 7.5
    b, n = workload.paper_fields(cells, 680.0, s["n0"])
    rng = np.random.default_rng(5)
    b = np.maximum(b, (rng.uniform(0, 0.4, b.shape) * (rng.uniform(size=b.shape) < 0.3))
                   .astype(np.float32))
    n = (n * rng.uniform(0.85, 1.0, n.shape)).astype(np.float32)
    S, dt, noise = _solver(cells, s, chi, "fp32", seed=9, step0=123456)
    S.set_fields(torch.from_numpy(b).cuda(), torch.from_numpy(n).cuda())
    S.autotune(effort=0, use_cache=True)
    tuning = S.tuning()
    steps = 2 * tuning[0]
    S.step(steps)
    gb, gn = S.get_fields()
    S.close()
    ob, on = oracle.run_noise(b, n, H, dt, steps, noise["sigma0"], 1.0, noise["seed"],
                              step0=123456, integrator="rk2", chi=chi)
    eb, en = normwise(gb, ob), normwise(gn, on)
    print("2048^2 rk2 noise, tuning %s, %d steps: normwise b %.2e n %.2e"
          % (tuning, steps, eb, en))
    assert eb <= 1e-5 and en <= 1e-5


def test_colony_runner_records():
    """run_case on a 512^2 square at the paper's cell width: host measures agree
    with the device diagnostics, the step keeps the explicit bound, b stays
    >= 0, and chemotaxis moves the envelope faster (Sec. 3)."""
    s = workload.PAPER_SETS["set3b"]
    times = (10.0, 20.0)
    out = {}
    for chi in (0.0, 7.5):
        res, fields = colony.run_case(s["sigma0"], s["n0"], chi, times, s["dt"], cells=512,
                                      length=512 * H, keep_fields=True)
        info, snaps = res["info"], res["snapshots"]
        assert info["dt"] == workload.paper_dt(2048, 680.0, s["sigma0"], s["n0"], s["dt"])
        assert [r["steps"] for r in snaps] == [round(t / info["dt"]) for t in times]
        assert len(fields) == 2 and fields[0].shape == (512, 512)
        prev = 0.0
        for r in snaps:
            assert r["t"] == pytest.approx(r["steps"] * info["dt"], rel=1e-12)
            assert r["r_env"] == pytest.approx(r["r_env_device"], rel=1e-12)
            assert r["r_area"] == pytest.approx(r["r_area_device"], rel=1e-12)
            assert r["min_b"] >= 0.0 and r["max_n"] <= s["n0"] * (1 + 1e-6)
            assert r["dt_over_bound"] <= 1.0
            assert r["r_env"] > prev
            prev = r["r_env"]
        out[chi] = snaps[-1]["r_env"]
    print("r_env at t=20: chi0=0 %.2f, chi0=7.5 %.2f" % (out[0.0], out[7.5]))
    assert out[7.5] > out[0.0]


def test_grid_study_runs_each_mesh_at_its_own_bound():
    """The grid-size study (Sec. 3.2) on two meshes of one square: each mesh
    takes the step of its own explicit bound, reaches the same caption times,
    and the colony's physical size agrees between the meshes."""
    L = 512 * H
    res, fields = colony.grid_study("set4", 0.0, [256, 512], length=L, keep_fields=True)
    assert res["cells"] == [256, 512] and len(fields) == 2
    a, b = (c["info"] for c in res["columns"])
    assert a["h"] == pytest.approx(2 * b["h"]) and a["dt"] > b["dt"]
    s = workload.PAPER_SETS["set4"]
    for c in res["columns"]:
        i = c["info"]
        assert i["dt"] == workload.paper_dt(i["cells"], L, s["sigma0"], s["n0"], s["dt"])
        assert [r["t_caption"] for r in c["snapshots"]] == list(s["times"])
        for r in c["snapshots"]:
            assert abs(r["t"] - r["t_caption"]) <= i["dt"]
    # first caption time, before either colony reaches the wall: radii within 25 %
    ra, rb = (c["snapshots"][0]["r_env"] for c in res["columns"])
    print("set4 chi0=0 r_env at t=33: 256^2 %.2f, 512^2 %.2f" % (ra, rb))
    assert 0 < ra < 0.95 * L / 2 and 0 < rb < 0.95 * L / 2
    assert abs(ra - rb) <= 0.25 * rb
