"""Pins of the learned-closure oracle: gradients against central differences,
closed-form properties of the stress model, Adam's first step, BF16 rounding."""
import numpy as np
import pytest

from oracle import mlp


def test_parameter_count():
    assert mlp.N_PARAMS == 5254
    p = mlp.init_params(0)
    assert np.allclose(mlp.unflatten(mlp.flatten(p))["W2"], p["W2"])


def test_gradients_match_central_differences():
    rng = np.random.default_rng(1)
    p = mlp.init_params(2)
    for k in p:  # nonzero biases so every parameter is exercised
        p[k] = p[k] + 0.05 * rng.standard_normal(p[k].shape)
    x = rng.standard_normal((40, mlp.N_IN))
    t = rng.standard_normal((40, mlp.N_OUT))
    t[:, :3] -= t[:, :3].mean(axis=1, keepdims=True)
    L, g = mlp.loss_and_grad(p, x, t)
    h = 1e-5  # central differences: truncation ~h^2, rounding ~1e-16 L / h
    worst = 0.0
    for k in mlp.ORDER:
        flat = p[k].ravel()
        for idx in rng.choice(flat.size, size=min(12, flat.size), replace=False):
            old = flat[idx]
            flat[idx] = old + h
            Lp, _ = mlp.loss_and_grad(p, x, t)
            flat[idx] = old - h
            Lm, _ = mlp.loss_and_grad(p, x, t)
            flat[idx] = old
            fd = (Lp - Lm) / (2 * h)
            an = g[k].ravel()[idx]
            worst = max(worst, abs(fd - an) / max(abs(fd), abs(an), 1e-2))
    assert worst < 1e-7, worst


def test_stress_is_symmetric_deviatoric_and_scales_with_gradient_squared():
    rng = np.random.default_rng(3)
    p = mlp.init_params(4)
    G = rng.standard_normal((30, 3, 3))
    d = rng.uniform(0.05, 0.2, 30)
    t1 = mlp.tau(p, G, d, 0.1)
    assert np.abs(t1[:, :3].sum(axis=1)).max() < 1e-14 * np.abs(t1).max()
    # features depend on G / |G| only, the prefactor on |G|^2
    t3 = mlp.tau(p, 3.0 * G, d, 0.1)
    assert np.abs(t3 - 9.0 * t1).max() < 1e-12 * np.abs(t3).max()
    assert np.abs(mlp.tau(p, np.zeros((2, 3, 3)), [0.1, 0.1], 0.1)).max() == 0.0


def test_adam_first_step_is_signed_learning_rate():
    """At step 1 the bias-corrected moments are g and g^2, so the update is
    -lr g / (|g| + eps)."""
    rng = np.random.default_rng(5)
    p = mlp.init_params(6)
    g = {k: rng.standard_normal(v.shape) for k, v in p.items()}
    p0 = {k: v.copy() for k, v in p.items()}
    mlp.adam_step(p, g, {}, lr=1e-3, step=1)
    for k in p:
        assert np.allclose(p[k], p0[k] - 1e-3 * g[k] / (np.abs(g[k]) + 1e-8), rtol=0, atol=1e-15)


def test_bf16_rounding():
    one = 1.0
    assert mlp.bf16_round(one)[()] == 1.0
    assert mlp.bf16_round(1 + 2.0 ** -8)[()] == 1.0               # tie -> even
    assert mlp.bf16_round(1 + 3 * 2.0 ** -9)[()] == 1 + 2.0 ** -7  # above the tie -> up
    assert mlp.bf16_round(1 + 3 * 2.0 ** -8)[()] == 1 + 2.0 ** -6  # tie -> even (up)
    x = np.random.default_rng(7).standard_normal(1000)
    r = mlp.bf16_round(x)
    assert np.abs(r - x).max() <= np.abs(x).max() * 2.0 ** -8


def test_training_reduces_loss():
    rng = np.random.default_rng(8)
    p = mlp.init_params(9)
    x = rng.standard_normal((256, mlp.N_IN))
    t = np.tanh(x[:, :6])
    t[:, :3] -= t[:, :3].mean(axis=1, keepdims=True)
    st = {}
    L0, _ = mlp.loss_and_grad(p, x, t)
    for s in range(1, 201):
        _, g = mlp.loss_and_grad(p, x, t)
        mlp.adam_step(p, g, st, 3e-3, s)
    L1, _ = mlp.loss_and_grad(p, x, t)
    assert L1 < 0.2 * L0
