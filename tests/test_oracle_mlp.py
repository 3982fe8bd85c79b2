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
    s = (rng.random(5) * 20).astype(np.float32)
    s[0], s[1] = 0.0, 20.0
    f = oracle.nrc_encode(p, d, s, 20.0)
    for a in range(3):
        for k in range(12):
            arg = (2.0 ** k) * math.pi * p[:, a].astype(np.float64)
            assert np.allclose(f[:, 24 * a + 2 * k], np.sin(arg), atol=1e-6)
            assert np.allclose(f[:, 24 * a + 2 * k + 1], np.cos(arg), atol=1e-6)
    assert np.array_equal(f[:, 72:75], d)
    assert f[0, 75] == 0.0 and f[1, 75] == 1.0
    assert np.allclose(f[:, 75], np.log1p(s.astype(np.float64)) / math.log1p(20.0), rtol=1e-7)


def test_bf16_rounding_matches_torch():
    """The oracle's bfloat16 rounding against torch's CPU conversion (an
    independent implementation of round-to-nearest-even)."""
    import torch
    rng = np.random.default_rng(11)
    x = np.concatenate([rng.normal(size=4000).astype(np.float32),
                        (rng.normal(size=1000) * 1e-38).astype(np.float32),  # subnormals
                        (rng.normal(size=1000) * 1e30).astype(np.float32)])
    # exact ties (lower 16 bits 0x8000) with even and odd upper halves, and
    # values one unit either side of a tie
    u = rng.integers(0x3F000000, 0x47000000, 2000, dtype=np.uint32) & np.uint32(0xFFFF0000)
    ties = np.concatenate([u | 0x8000, u | 0x7FFF, u | 0x8001, (u | 0x10000) | 0x8000]).view(np.float32)
    x = np.concatenate([x, ties, np.float32([0.0, -0.0, 1.0, 3.3895314e38])])
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    assert np.array_equal(oracle.bf16_round(x).view(np.uint32), ref.view(np.uint32))


def sparse_int_params(seed):
    """Weights in {-1, 0, 1} with few nonzeros per row and integer biases,
    so every activation, error and product of the BF16-operand mode is a
    small integer (exact in bfloat16)."""
    rng = np.random.default_rng(seed)
    P = np.zeros(NP)
    dims = [76, 64, 64, 64, 64, 3]
    o = 0
    for l in range(5):
        fi, fo = dims[l], dims[l + 1]
        W = np.zeros((fo, fi))
        nnz = 8 if l == 0 else 2
        for r in range(fo):
            cols = rng.choice(fi, nnz, replace=False)
            W[r, cols] = rng.choice([-1.0, 1.0], nnz)
        P[o:o + fo * fi] = W.ravel()
        P[o + fo * fi:o + fo * fi + fo] = rng.integers(-2, 3, fo)
        o += fo * fi + fo
    assert o == NP
    return P


def test_bf16_mode_is_exact_on_representable_networks():
    """When every operand is exactly representable in bfloat16 the
    BF16-operand mode must equal the FP64 network bit for bit."""
    P = sparse_int_params(7)
    rng = np.random.default_rng(8)
    x = rng.integers(0, 2, (9, 76)).astype(np.float64)
    dy = rng.integers(-1, 2, (9, 3)).astype(np.float64)
    y64, g64 = oracle.mlp_backward(P, x, dy, bf16=False)
    y16, g16 = oracle.mlp_backward(P, x, dy, bf16=True)
    assert np.abs(y64).max() > 4 and np.abs(g64).max() > 4  # not a trivial network
    assert np.array_equal(y64, y16) and np.array_equal(g64, g16)
    assert np.array_equal(oracle.mlp_forward(P, x, bf16=True), y64)


def test_bf16_mode_rounds_layer_inputs():
    """A chain passing feature 0 through unit 0 of every layer: the input
    1 + 2^-8 is a tie and rounds to 1 (even), 1 + 3 * 2^-9 rounds up to
    1 + 2^-7; the FP64 network keeps both exactly."""
    P = np.zeros(NP)
    dims = [76, 64, 64, 64, 64, 3]
    o = 0
    for l in range(5):
        fi, fo = dims[l], dims[l + 1]
        P[o] = 1.0  # W_l[0][0]
        o += fo * fi + fo
    x = np.zeros((2, 76))
    x[0, 0] = 1 + 2 ** -8
    x[1, 0] = 1 + 3 * 2 ** -9
    assert np.array_equal(oracle.mlp_forward(P, x)[:, 0], x[:, 0])
    assert np.array_equal(oracle.mlp_forward(P, x, bf16=True)[:, 0], [1.0, 1 + 2 ** -7])


def test_bf16_mode_close_to_fp64():
    """Property: on a random network the BF16-operand results stay close
    to the exact network: each rounded operand carries a relative error of
    at most 2^-9, outputs pass 5 roundings of layer inputs, and gradients
    about twice as many, with cancellation in the batch sums on top (a few
    percent)."""
    P = rand_params(12, scale=1.0)
    rng = np.random.default_rng(13)
    x = oracle.nrc_encode(rng.random((64, 3)), rng.normal(size=(64, 3)), rng.random(64), 1.0).astype(np.float64)
    dy = rng.normal(size=(64, 3))
    y64, g64 = oracle.mlp_backward(P, x, dy)
    y16, g16 = oracle.mlp_backward(P, x, dy, bf16=True)
    assert np.linalg.norm(y16 - y64) <= 0.03 * np.linalg.norm(y64)
    assert np.linalg.norm(g16 - g64) <= 0.1 * np.linalg.norm(g64)
    assert not np.array_equal(y16, y64)


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
    x = oracle.nrc_encode(pos, np.tile([0, 0, 1], (256, 1)), np.zeros(256), 1.0).astype(np.float64)
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


def test_weight_average_closed_forms():
    """Bias-corrected exponential average: constant weights give themselves;
    two steps give (b w1 + w2) / (1 + b)."""
    rng = np.random.default_rng(14)
    c = rng.normal(size=50)
    ema = np.zeros(50)
    for t in range(1, 6):
        out = oracle.ema_step(ema, c, 0.9, t)
        assert np.allclose(out, c, rtol=1e-14, atol=0)
    w1, w2 = rng.normal(size=50), rng.normal(size=50)
    ema = np.zeros(50)
    oracle.ema_step(ema, w1, 0.95, 1)
    out = oracle.ema_step(ema, w2, 0.95, 2)
    assert np.allclose(out, (0.95 * w1 + w2) / 1.95, rtol=1e-14, atol=1e-16)
