"""Surrogate MLP kernels (ks_*) against the FP64 reference network."""
import numpy as np
import pytest

import oracle
from oracle import mlp_ref

pytestmark = pytest.mark.gpu

MAPS = dict(in_shift=(0.75, 1.0, 0.3), in_scale=(0.45, 1.0, 0.2), out_shift=0.3, out_scale=0.2)


def _model(maxp=70000, seed=0, log_target=False):
    from paper_1301_5058_amd.surrogate import Surrogate, he_uniform
    S = Surrogate(maxp)
    S.set_normalization(MAPS["in_shift"], MAPS["in_scale"], MAPS["out_shift"], MAPS["out_scale"],
                        log_target=log_target)
    p = he_uniform(seed)
    rng = np.random.default_rng(seed + 100)
    p[192:256] = rng.uniform(-0.2, 0.2, 64)     # non-zero biases exercise every term
    p[4352:4416] = rng.uniform(-0.2, 0.2, 64)
    p[8512:8576] = rng.uniform(-0.2, 0.2, 64)
    p[8640] = 0.1
    S.set_params(p)
    return S, p


def _data(n, seed=1):
    rng = np.random.default_rng(seed)
    X = np.stack([rng.uniform(0.3, 1.2, n), rng.uniform(0, 2, n), rng.uniform(0.1, 0.5, n)],
                 1).astype(np.float32)
    y = (np.array([oracle.cbar(a, b) for a, b in X[:, :2].astype(np.float64)]) *
         (1.0 + 0.1 * X[:, 2])).astype(np.float32)
    return X, y


@pytest.mark.parametrize("n", [1, 37, 1000, 4096])
def test_gradient_matches_reference(n):
    S, p = _model()
    X, y = _data(n)
    g, loss = S.grad(X, y)
    lr, gr = mlp_ref.loss_and_grad(p.astype(np.float64), X.astype(np.float64), y, **MAPS)
    assert loss == pytest.approx(lr, rel=2e-3)
    for name, off, shape in mlp_ref.LAYOUT:
        size = int(np.prod(shape)) if shape else 1
        a, b = g[off:off + size].astype(np.float64), gr[off:off + size]
        err = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)
        print("%s rel err %.2e" % (name, err))
        assert err <= 2e-2, name
    S.close()


def test_log_target_mode_matches_reference():
    S, p = _model(log_target=True)
    X, y = _data(777, 6)
    g, loss = S.grad(X, y)
    lr, gr = mlp_ref.loss_and_grad(p.astype(np.float64), X.astype(np.float64), y, log_target=True,
                                   **MAPS)
    assert loss == pytest.approx(lr, rel=2e-3)
    assert np.linalg.norm(g - gr) <= 2e-2 * np.linalg.norm(gr)
    v = S.predict(X)
    vr, _ = mlp_ref.forward(p.astype(np.float64), X.astype(np.float64), log_target=True, **MAPS)
    assert np.max(np.abs(v - vr) / vr) <= 1e-2 * MAPS["out_scale"] * 5
    S.close()


def test_predict_matches_reference():
    S, p = _model()
    X, _ = _data(5003, 2)
    v = S.predict(X)
    vr, _ = mlp_ref.forward(p.astype(np.float64), X.astype(np.float64), **MAPS)
    assert np.max(np.abs(v - vr)) <= 1e-2 * MAPS["out_scale"]
    S.close()


def test_training_fits_a_smooth_velocity_law():
    S, _ = _model()
    X, y = _data(4096, 3)
    Xt, yt = _data(512, 4)
    l0 = S.grad(X, y)[1]
    loss = S.train(X, y, iters=3000, batch=1024, lr=2e-3)
    assert loss < 0.02 * l0
    rel = np.abs(S.predict(Xt) - yt) / yt
    print("held-out median rel err %.4f, p95 %.4f" % (np.median(rel), np.quantile(rel, 0.95)))
    assert np.median(rel) < 0.02
    S.close()


def test_hull_and_speed_bound_kernels():
    from paper_1301_5058_amd.surrogate import hull_facets
    S, _ = _model()
    rng = np.random.default_rng(5)
    pts = np.stack([rng.uniform(0.3, 1.2, 400), rng.uniform(0, 2, 400), rng.uniform(0.1, 0.5, 400)], 1)
    F = hull_facets(pts)
    S.set_hull(F, tol=1e-9)
    Q = np.stack([rng.uniform(0.1, 1.5, 3000), rng.uniform(-0.5, 2.5, 3000),
                  rng.uniform(0.0, 0.6, 3000)], 1).astype(np.float32)
    d = Q.astype(np.float64) @ F[:, :3].T + F[:, 3]
    want = np.all(d <= 1e-9, axis=1)
    got = S.inside(Q)
    clear = np.min(np.abs(d), axis=1) > 1e-6  # away from the facets
    assert np.array_equal(got[clear], want[clear]) and want.any() and (~want).any()
    cb = S.cbar(Q[:, :], sigma0=1.0)
    ref = np.array([oracle.cbar(float(a), float(max(b, 0.0))) for a, b in Q[:, :2]])
    ok = Q[:, 1] >= 0
    np.testing.assert_allclose(cb[ok], ref[ok], rtol=2e-6)
    S.close()


def test_threshold_speed_kernel_matches_oracle():
    pts = [(0.35, 0.0), (0.71, 10.0), (1.07, 5.0), (2.0, 0.0), (2.0, 2.5), (3.0, 1.0),
           (4.0, 10.0), (0.5, 0.3)]
    X = np.array([[n0, chi, 0.3] for n0, chi in pts], dtype=np.float32)
    from paper_1301_5058_amd.surrogate import Surrogate
    S = Surrogate(16)
    got = S.cstar(X).astype(np.float64)
    got2 = S.cstar(X[:3], sigma0=2.0).astype(np.float64)
    bad = S.cstar(np.array([[0.0, 1.0, 0.3], [1.0, -1.0, 0.3]], dtype=np.float32))
    S.close()
    for k, (n0, chi) in enumerate(pts):
        ref = oracle.cstar(float(np.float32(n0)), float(np.float32(chi)))
        print("c*(%.2f, %.1f) = %.6f (oracle %.6f)" % (n0, chi, got[k], ref))
        assert abs(got[k] - ref) <= 1e-5 * ref
    for k in range(3):
        n0, chi = pts[k]
        assert abs(got2[k] - oracle.cstar(n0, chi, 2.0)) <= 1e-5 * got2[k]
    assert np.all(np.isnan(bad))


def test_gradient_elementwise_against_reference():
    # every entry of every tensor against the FP64 network with the same
    # bfloat16 rounding points; the differences left are float32 accumulation
    # and bfloat16 roundings that fall on the other side of a tie
    S, p = _model()
    X, y = _data(1000, 9)
    g, _ = S.grad(X, y)
    _, gr = mlp_ref.loss_and_grad(p.astype(np.float64), X.astype(np.float64), y, **MAPS)
    for name, off, shape in mlp_ref.LAYOUT:
        size = int(np.prod(shape)) if shape else 1
        a, b = g[off:off + size].astype(np.float64), gr[off:off + size]
        err = np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-30)
        print("%s max elementwise err / max|g| %.2e" % (name, err))
        assert err <= 2e-2, name
    S.close()


def test_adam_steps_match_reference_adam():
    # ks_train with one full-batch iteration applies Adam to the gradient that
    # ks_grad returns at the same parameters (same kernel, same partials, same
    # summation order).  The FP64 Adam of the oracle fed those gradients must
    # reproduce the parameters after every step, element by element, to the
    # float32 rounding of the parameters and the moments.
    S, p = _model()
    X, y = _data(300, 8)
    lr = 1e-3
    theta = p.astype(np.float64)
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    k = 6
    for t in range(1, k + 1):
        g, _ = S.grad(X, y)
        S.train(X, y, iters=1, batch=len(X), lr=lr)
        theta, m, v = mlp_ref.adam_step(theta, g.astype(np.float64), m, v, t, lr)
        got = S.get_params().astype(np.float64)
        err = np.abs(got - theta)
        tol = t * (1.2e-7 * np.abs(theta) + 4e-6 * lr) + 1e-30
        print("step %d: max |p - p_ref| %.3e, max err / tol %.3f, max |step| %.3e"
              % (t, err.max(), np.max(err / tol), np.max(np.abs(got - p))))
        assert np.all(err <= tol), t
    # the same steps again with the oracle's own gradients: the trajectories
    # differ only where a gradient entry is near zero and its float32 value
    # has a different sign or size (Adam normalises every entry to about lr)
    theta = p.astype(np.float64)
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    S.set_params(p)
    S.train(X, y, iters=3, batch=len(X), lr=lr)
    for t in range(1, 4):
        _, gr = mlp_ref.loss_and_grad(theta, X.astype(np.float64), y, **MAPS)
        theta, m, v = mlp_ref.adam_step(theta, gr, m, v, t, lr)
    d = np.abs(S.get_params().astype(np.float64) - theta)
    print("3 steps, oracle gradients: median |dp| %.2e, p99 %.2e, max %.2e (lr %.0e)"
          % (np.median(d), np.quantile(d, 0.99), d.max(), lr))
    assert np.quantile(d, 0.99) <= 0.1 * 3 * lr and d.max() <= 2 * 3 * lr
    S.close()
