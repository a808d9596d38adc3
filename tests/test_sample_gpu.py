"""kc_step_sample: steps with the diagnostics fused into the last launch.

Against kc_step followed by kc_diagnostics_device on the same state: the
fields are the same bits, time and both radii the same numbers (a maximum and
a count), mass and nutrient the same sums in another order.  Every integrator,
noise mode and precision; launch depths that do not divide the step count (the
last launch is then a shallower kernel); ragged grids; a second call whose
strip count outgrows the partials buffer.
"""
import numpy as np
import pytest
import torch

from paper_1301_5058_amd import workload

pytestmark = pytest.mark.gpu

NOISE = dict(sigma0=1.0, amp=0.5, seed=5)


def _state(nx, ny):
    b, n, s = workload.fields(nx, ny, 0.8, 0.5, 3)
    rng = np.random.default_rng(nx + 7 * ny)
    b = np.maximum(b, (rng.uniform(0, 0.6, b.shape) * (rng.uniform(size=b.shape) < 0.2))
                   .astype(np.float32))
    return b, n, s


def _solver(nx, ny, precision, integrator, noise, tuning):
    from paper_1301_5058_amd.solver import Solver
    S = Solver(nx, ny, dt=0.05, chi=1.1, precision=precision, integrator=integrator,
               noise=NOISE if noise else None, b_thr=0.3)
    b, n, s = _state(nx, ny)
    if precision == "fp64":
        b, n, s = (x.astype(np.float64) for x in (b, n, s))
    S.set_fields(b, n, None if noise else s)
    S.set_tuning(*tuning)
    return S


CASES = [("euler", (4, 35, 4)), ("euler", (3, 7, 2)), ("euler", (8, 16, 4)), ("euler", (1, 1, 4)),
         ("rk2", (2, 9, 4)), ("rk2", (3, 100, 2)), ("euler", (4, 35, 2, 2)), ("rk2", (2, 9, 4, 2))]


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("noise", [False, True])
@pytest.mark.parametrize("integrator,tuning", CASES)
@pytest.mark.parametrize("nx,ny", [(300, 97), (128, 128), (64, 1), (560, 203)])
def test_step_sample_equals_step_then_diagnostics(precision, noise, integrator, tuning, nx, ny):
    steps = 11
    A = _solver(nx, ny, precision, integrator, noise, tuning)
    oa = torch.zeros(5, dtype=torch.float64, device="cuda")
    A.step(steps)
    A.diagnostics_device(oa)
    fa = A.get_fields()
    A.close()
    B = _solver(nx, ny, precision, integrator, noise, tuning)
    ob = torch.zeros(5, dtype=torch.float64, device="cuda")
    B.step_sample(steps, ob)
    fb = B.get_fields()
    B.close()
    torch.cuda.synchronize()
    a, b = oa.cpu().numpy(), ob.cpu().numpy()
    assert np.array_equal(fa[0], fb[0]) and np.array_equal(fa[1], fb[1])
    assert a[0] == b[0] and a[3] == b[3] and a[4] == b[4]
    assert a[1] > 0 and a[3] > 0
    np.testing.assert_allclose(b[1:3], a[1:3], rtol=1e-13, atol=0)


def test_step_sample_series_and_buffer_growth():
    """A series sampled with kc_step_sample equals one sampled with
    kc_diagnostics_device, through a tuning change that multiplies the strip
    count (the partials buffer grows between calls)."""
    nx, ny = 512, 384
    series = []
    for fused in (False, True):
        S = _solver(nx, ny, "fp32", "euler", False, (4, 120, 4))
        out = torch.zeros((6, 5), dtype=torch.float64, device="cuda")
        for i in range(6):
            if i == 3:
                S.set_tuning(2, 3, 2)  # ~40x the strips
            if fused:
                S.step_sample(7, out[i])
            else:
                S.step(7)
                S.diagnostics_device(out[i])
        torch.cuda.synchronize()
        series.append((out.cpu().numpy(), S.get_fields()))
        S.close()
    (sa, fa), (sb, fb) = series
    assert np.array_equal(fa[0], fb[0]) and np.array_equal(fa[1], fb[1])
    assert np.array_equal(sa[:, [0, 3, 4]], sb[:, [0, 3, 4]])
    np.testing.assert_allclose(sb[:, 1:3], sa[:, 1:3], rtol=1e-13, atol=0)


def test_step_sample_rejects_bad_arguments():
    from paper_1301_5058_amd.native import KcError
    S = _solver(64, 64, "fp32", "euler", False, (4, 16, 4))
    out = torch.zeros(5, dtype=torch.float64, device="cuda")
    with pytest.raises(KcError):
        S.step_sample(0, out)
    with pytest.raises(ValueError):
        S.step_sample(1, torch.zeros(5, dtype=torch.float32, device="cuda"))
    S.close()


def test_step_sample_with_the_reference_kernel():
    """With the reference kernel selected kc_step_sample is kc_step then
    kc_diagnostics_device: the same numbers exactly."""
    outs = []
    for fused in (False, True):
        S = _solver(100, 60, "fp32", "rk2", True, (2, 9, 4))
        S.use_reference_kernel()
        o = torch.zeros(5, dtype=torch.float64, device="cuda")
        if fused:
            S.step_sample(5, o)
        else:
            S.step(5)
            S.diagnostics_device(o)
        torch.cuda.synchronize()
        outs.append((o.cpu().numpy(), S.get_fields()))
        S.close()
    (a, fa), (b, fb) = outs
    assert np.array_equal(a, b)
    assert np.array_equal(fa[0], fb[0]) and np.array_equal(fa[1], fb[1])
