"""Pins of the FP64 reference network (the surrogate's gradient oracle)."""
import numpy as np
import pytest

from oracle import mlp_ref


def _setup(seed=0, n=37):
    rng = np.random.default_rng(seed)
    p = np.zeros(mlp_ref.NPARAM)
    p[0:192] = rng.uniform(-1, 1, 192)
    p[192:256] = rng.uniform(-0.1, 0.1, 64)
    p[256:4352] = rng.uniform(-0.3, 0.3, 4096)
    p[4352:4416] = rng.uniform(-0.1, 0.1, 64)
    p[4416:8512] = rng.uniform(-0.3, 0.3, 4096)
    p[8512:8576] = rng.uniform(-0.1, 0.1, 64)
    p[8576:8640] = rng.uniform(-0.3, 0.3, 64)
    p[8640] = 0.05
    X = np.stack([rng.uniform(0.3, 1.2, n), rng.uniform(0, 2, n), rng.uniform(0.1, 0.5, n)], 1)
    y = rng.uniform(0.1, 0.6, n)
    maps = dict(in_shift=(0.75, 1.0, 0.3), in_scale=(0.45, 1.0, 0.2), out_shift=0.3,
                out_scale=0.2)
    return p, X, y, maps


def test_bf16_rounding_is_round_to_nearest_even():
    # 1 + 2^-8 is a tie between 1 and 1 + 2^-7: even mantissa wins (1.0)
    assert mlp_ref.bf16(1.0 + 2 ** -8) == 1.0
    assert mlp_ref.bf16(1.0 + 3 * 2 ** -8) == 1.0 + 2 ** -6
    assert mlp_ref.bf16(1.0 + 2 ** -8 + 2 ** -20) == 1.0 + 2 ** -7
    assert mlp_ref.bf16(-3.0) == -3.0
    x = np.linspace(-5, 5, 1001)
    assert np.max(np.abs(mlp_ref.bf16(x) - x) / np.maximum(np.abs(x), 1e-30)) <= 2 ** -8 + 1e-12


def test_gelu_derivative_matches_finite_difference():
    z = np.linspace(-6, 6, 241)
    h = 1e-6
    fd = (mlp_ref.gelu(z + h) - mlp_ref.gelu(z - h)) / (2 * h)
    assert np.max(np.abs(fd - mlp_ref.gelu_grad(z))) <= 1e-8
    # g(z) = z Phi(z): g(0) = 0, g(z) -> z for large z, -> 0 for very negative z
    assert mlp_ref.gelu(np.array([0.0]))[0] == 0.0
    assert abs(mlp_ref.gelu(np.array([8.0]))[0] - 8.0) < 1e-12


def test_plain_gradient_matches_central_differences():
    p, X, y, maps = _setup()
    loss, g = mlp_ref.loss_and_grad(p, X, y, emulate_bf16=False, **maps)
    rng = np.random.default_rng(3)
    idx = np.concatenate([rng.choice(np.arange(0, 192), 6), rng.choice(np.arange(192, 8641), 30),
                          [8640, 8575, 4351, 255]])
    h = 1e-6
    for i in idx:
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        lp = mlp_ref.loss_and_grad(pp, X, y, emulate_bf16=False, **maps)[0]
        lm = mlp_ref.loss_and_grad(pm, X, y, emulate_bf16=False, **maps)[0]
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])), i


def test_bf16_emulation_stays_close_to_the_plain_network():
    p, X, y, maps = _setup(1, 200)
    _, g0 = mlp_ref.loss_and_grad(p, X, y, emulate_bf16=False, **maps)
    _, g1 = mlp_ref.loss_and_grad(p, X, y, emulate_bf16=True, **maps)
    for name, off, shape in mlp_ref.LAYOUT:
        size = int(np.prod(shape)) if shape else 1
        a, b = g0[off:off + size], g1[off:off + size]
        assert np.linalg.norm(a - b) <= 5e-2 * np.linalg.norm(a) + 1e-12, name


def test_pack_unpack_roundtrip():
    p, *_ = _setup()
    assert np.array_equal(mlp_ref.pack(mlp_ref.unpack(p)), p)


def test_adam_constant_gradient_moves_lr_per_step():
    # With a constant gradient g the bias-corrected moments are exactly g and
    # g^2 at every step, so each step moves lr g / (|g| + eps): after k steps
    # the closed form p0 - k lr g / (|g| + eps).
    rng = np.random.default_rng(4)
    p0 = rng.uniform(-1, 1, 50)
    g = rng.uniform(-2, 2, 50) * 10.0 ** rng.integers(-6, 2, 50)
    p, m, v = p0.copy(), np.zeros(50), np.zeros(50)
    lr = 3e-3
    for t in range(1, 26):
        p, m, v = mlp_ref.adam_step(p, g, m, v, t, lr)
        want = p0 - t * lr * g / (np.abs(g) + 1e-8)
        np.testing.assert_allclose(p, want, rtol=0, atol=1e-13 * t)


def test_adam_matches_torch_adam_on_a_gradient_sequence():
    # the library routine torch.optim.Adam (float64, CPU) on the same gradients
    import torch
    rng = np.random.default_rng(5)
    p0 = rng.uniform(-1, 1, 200)
    grads = [rng.normal(0, 1, 200) * 10.0 ** rng.integers(-9, 1, 200) for _ in range(40)]
    w = torch.tensor(p0.copy(), dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([w], lr=2e-3, betas=(0.9, 0.999), eps=1e-8, foreach=False)
    p, m, v = p0.copy(), np.zeros(200), np.zeros(200)
    for t, g in enumerate(grads, start=1):
        opt.zero_grad()
        w.grad = torch.tensor(g, dtype=torch.float64)
        opt.step()
        p, m, v = mlp_ref.adam_step(p, g, m, v, t, 2e-3)
        np.testing.assert_allclose(p, w.detach().numpy(), rtol=0, atol=1e-14)


def test_adam_first_step_is_lr_times_the_gradient_sign():
    # first step from zero moments: mhat = g, vhat = g^2
    g = np.array([3.0, -1e-3, 0.0, 2e-12])
    p, m, v = mlp_ref.adam_step(np.zeros(4), g, np.zeros(4), np.zeros(4), 1, 0.5)
    np.testing.assert_allclose(p, -0.5 * g / (np.abs(g) + 1e-8), rtol=1e-15, atol=0)
    np.testing.assert_allclose(m, 0.1 * g, rtol=1e-14)
    np.testing.assert_allclose(v, 0.001 * g * g, rtol=1e-13)
