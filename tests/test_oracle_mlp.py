"""Pins of the oracle's radiance-cache network (an addition of this project,
not in the paper) against finite differences and closed forms (no GPU)."""
import math

import numpy as np
import pytest

import oracle

NP = oracle.N_PARAMS


def rand_params(seed, scale=0.3):
    rng = np.random.default_rng(seed)
    return rng.normal(0, scale, NP) * np.sqrt(2.0 / 64)


def test_param_count():
    """76 -> 64 x 4 -> 3 with biases: 76*64+64 + 3*(64*64+64) + 64*3+3."""
    assert NP == 76 * 64 + 64 + 3 * (64 * 64 + 64) + 64 * 3 + 3 == 17603


def test_encoding_closed_form():
    rng = np.random.default_rng(0)
    p = rng.random((5, 3)).astype(np.float32)
    d = rng.normal(size=(5, 3)).astype(np.float32)
    s = rng.random(5).astype(np.float32)
    f = oracle.nrc_encode(p, d, s)
    for a in range(3):
        for k in range(12):
            arg = (2.0 ** k) * math.pi * p[:, a].astype(np.float64)
            assert np.allclose(f[:, 24 * a + 2 * k], np.sin(arg), atol=1e-6)
            assert np.allclose(f[:, 24 * a + 2 * k + 1], np.cos(arg), atol=1e-6)
    assert np.array_equal(f[:, 72:75], d) and np.array_equal(f[:, 75], s)


def test_backward_matches_finite_differences():
    P = rand_params(1, scale=1.0)
    rng = np.random.default_rng(2)
    x = rng.normal(size=(7, 76))
    dy = rng.normal(size=(7, 3))
    y, g = oracle.mlp_backward(P, x, dy)
    assert np.allclose(y, oracle.mlp_forward(P, x))
    f = lambda q: float((oracle.mlp_forward(q, x) * dy).sum())
    idx = rng.choice(NP, 300, replace=False)
    idx = np.concatenate([idx, [0, 4863, 4864 + 63, NP - 1, NP - 4]])  # first/last weights and biases
    h = 1e-6
    for i in idx:
        e = np.zeros(NP)
        e[i] = h
        fd = (f(P + e) - f(P - e)) / (2 * h)
        assert g[i] == pytest.approx(fd, rel=1e-5, abs=1e-7)


def test_loss_gradient_matches_finite_differences():
    rng = np.random.default_rng(3)
    y = rng.normal(size=(6, 3))
    t = rng.random((6, 3))
    loss, dy = oracle.nrc_loss_grad(y, t)
    # relative L2 with the denominator held constant (stop-gradient)
    den = y ** 2 + 0.01
    assert loss == pytest.approx(((y - t) ** 2 / den).mean())
    assert np.allclose(dy, 2 * (y - t) / den / y.size)


def test_adam_closed_forms():
    """First Adam step with bias correction moves every parameter by
    lr * g / (|g| + eps); zero gradients leave parameters unchanged."""
    rng = np.random.default_rng(4)
    p = rng.normal(size=100)
    g = rng.normal(size=100)
    g[:5] = 0
    m = np.zeros(100)
    v = np.zeros(100)
    p0 = p.copy()
    oracle.adam_step(p, g, m, v, 1, lr=1e-3)
    assert np.allclose(p, p0 - 1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-9, atol=1e-15)
    assert np.array_equal(p[:5], p0[:5])


def test_training_reduces_loss():
    """Property: Adam on the relative-L2 loss fits a smooth target."""
    rng = np.random.default_rng(5)
    P = rand_params(6)
    pos = rng.random((256, 3)).astype(np.float32)
    x = oracle.nrc_encode(pos, np.tile([0, 0, 1], (256, 1)), np.zeros(256)).astype(np.float64)
    tgt = np.stack([pos[:, 0], pos[:, 1] ** 2, 0.5 + 0 * pos[:, 2]], 1).astype(np.float64)
    m = np.zeros(NP)
    v = np.zeros(NP)
    first = None
    for step in range(1, 201):
        y = oracle.mlp_forward(P, x)
        loss, dy = oracle.nrc_loss_grad(y, tgt)
        first = loss if first is None else first
        _, g = oracle.mlp_backward(P, x, dy)
        oracle.adam_step(P, g, m, v, step, lr=3e-3)
    assert loss < 0.2 * first
