"""kc_step_sample_noalloc (the entry point for callers that cannot allocate)
against kc_step_sample: same fields and diagnostics, on two calls in a row
with the second on a smaller grid, and the strip limit of its scratch."""
import numpy as np
import pytest
import torch

from paper_1301_5058_amd import native as N
from paper_1301_5058_amd import workload

pytestmark = pytest.mark.gpu


def _pair(nx, ny, steps, tuning=None, **kw):
    from paper_1301_5058_amd.solver import Solver
    b, n, s = workload.fields(nx, ny, 0.6, 0.5, 7)
    dt = workload.config_dt(b, n, s)
    if kw.get("precision") == "fp64":
        b, n, s = (x.astype(np.float64) for x in (b, n, s))
    out = []
    for noalloc in (False, True):
        S = Solver(nx, ny, dt=dt, chi=1.0, b_thr=0.3, **kw)
        S.set_fields(*(torch.from_numpy(x).cuda() for x in ((b, n) if "noise" in kw else (b, n, s))))
        if tuning:
            S.set_tuning(*tuning)
        o5 = torch.zeros(5, dtype=torch.float64, device="cuda")
        series = []
        for k in steps:
            (S.step_sample_noalloc if noalloc else S.step_sample)(k, o5)
            torch.cuda.synchronize()
            series.append(o5.cpu().numpy().copy())
        out.append((np.array(series), S.get_fields()))
        S.close()
    return out


@pytest.mark.parametrize("kw", [dict(), dict(integrator="rk2"), dict(precision="fp64"),
                                dict(noise=dict(sigma0=1.0, amp=0.5, seed=9))])
def test_noalloc_equals_step_sample_on_two_grids(kw):
    # first call: a 1000 x 700 grid; second: a smaller 300 x 200 grid in a new
    # context (fewer strips, so the scratch keeps stale partials of the first
    # call beyond what the second writes)
    for nx, ny, steps in ((1000, 700, (37, 100, 5)), (300, 200, (13, 40))):
        (sa, fa), (sb, fb) = _pair(nx, ny, steps, **kw)
        print(nx, ny, kw, sa[-1], sb[-1])
        assert np.array_equal(sa, sb)
        assert np.array_equal(fa[0], fb[0]) and np.array_equal(fa[1], fb[1])


def test_noalloc_rejects_more_strips_than_its_scratch_and_the_reference_kernel():
    from paper_1301_5058_amd.solver import Solver
    nx, ny = 4096, 8192  # 17 strips across; one-row strips give 139264 > 131072
    S = Solver(nx, ny, dt=0.2, chi=0.5, b_thr=0.3)
    b = torch.zeros((ny, nx), dtype=torch.float32, device="cuda")
    n = torch.full((ny, nx), 0.5, dtype=torch.float32, device="cuda")
    s = torch.ones((ny, nx), dtype=torch.float32, device="cuda")
    S.set_fields(b, n, s)
    S.set_tuning(4, 1, 4)
    o5 = torch.zeros(5, dtype=torch.float64, device="cuda")
    with pytest.raises(N.KcError) as e:
        S.step_sample_noalloc(4, o5)
    assert e.value.code == N.KC_EINVAL and "strips" in str(e.value)
    assert S.time()[1] == 0  # nothing was enqueued
    S.set_tuning(4, 2, 4)  # 69632 strips: fits
    S.step_sample_noalloc(4, o5)
    torch.cuda.synchronize()
    assert o5[0].item() == pytest.approx(0.8) and o5[2].item() == pytest.approx(0.5 * nx * ny)
    S.use_reference_kernel(True)
    with pytest.raises(N.KcError) as e:
        S.step_sample_noalloc(4, o5)
    assert e.value.code == N.KC_EINVAL
    S.close()
