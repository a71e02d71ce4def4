"""Pins of the FP64 reference of the warm-start network (CPU).

The network is not in the paper, so nothing the paper prints pins it; its
pins are the definition of a derivative (central differences), a network
whose output is known in closed form, Adam's first step, the BF16 rounding
rule on chosen values, and the input encoding on hand-worked indices.
"""
import numpy as np
import pytest

from oracle import mlp


def _rand_params(rng, scale=0.2):
    return rng.normal(0.0, scale, mlp.NPARAMS)


def test_layout_size():
    assert mlp.NPARAMS == 32 * 256 + 256 + 2 * (256 * 256 + 256) + 256 + 1 == 140289


def test_encoding_l16_is_the_index_bits_in_order():
    rng = np.random.default_rng(0)
    idx = rng.integers(0, 2**32, 50, dtype=np.uint64)
    X = mlp.encode(idx, 16)
    for r, i in enumerate(idx):
        bits = [(int(i) >> (31 - s)) & 1 for s in range(32)]
        assert X[r].tolist() == [2.0 * b - 1 for b in bits]


def test_encoding_short_window_by_hand():
    """l = 12: positions 1..8 then 5..12.  a = 1 followed by zeros, b = all
    zeros except its last symbol: a_1 is the top bit (2*11+1 = 23), b_12 is
    bit 0."""
    idx = (1 << 23) | 1
    x = mlp.encode([idx], 12)[0]
    assert x[0] == 1.0 and x[1] == -1.0                # (a_1, b_1)
    assert all(v == -1.0 for v in x[2:30])
    assert x[30] == -1.0 and x[31] == 1.0              # (a_12, b_12)
    assert mlp.positions(12) == [1, 2, 3, 4, 5, 6, 7, 8, 5, 6, 7, 8, 9, 10, 11, 12]


def test_bf16_rounding_rule():
    vals = np.array([1.0, 1 + 2**-8, 1 + 3 * 2**-8, 1 + 2**-7 + 2**-8, -2.5, 1 + 2**-9, 3.0e38])
    out = mlp.bf16(vals)
    # 1 + 2^-8 is a tie between 1 and 1 + 2^-7: even mantissa (1) wins;
    # 1 + 3*2^-8 is a tie between 1 + 2^-7 and 1 + 2^-6: even (1 + 2^-6) wins
    assert out.tolist()[:6] == [1.0, 1.0, 1 + 2**-6, 1 + 2**-6, -2.5, 1.0]
    assert np.isfinite(out[6])


def test_closed_form_network():
    """Only input 0 reaches the output: y = 0.5 * 3 * 2 * relu(x_0 + 0.5) + 0.25."""
    p = np.zeros(mlp.NPARAMS)
    P = mlp.unpack(p)
    P["W1"][0, 0] = 1.0
    P["b1"][0] = 0.5
    P["W2"][0, 0] = 2.0
    P["W3"][0, 0] = 3.0
    P["w4"][0] = 0.5
    P["b4"][0] = 0.25
    X = np.zeros((3, 32))
    X[:, 0] = [1.0, -1.0, 0.0]
    for b in (False, True):
        y, _ = mlp.forward(p, X, bf16_ops=b)
        assert y.tolist() == [4.75, 0.25, 1.75]


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(1)
    p = _rand_params(rng)
    X = mlp.encode(rng.integers(0, 2**32, 16, dtype=np.uint64), 16)
    t = rng.normal(0, 1, 16)

    def loss(q):
        y, _ = mlp.forward(q, X, bf16_ops=False)
        return mlp.mse(y, t)[0]

    y, cache = mlp.forward(p, X, bf16_ops=False)
    _, dy = mlp.mse(y, t)
    g = mlp.backward(cache, dy)
    picks = np.concatenate([rng.choice(mlp.NPARAMS, 60, replace=False),
                            [o for o, _ in mlp.OFFSETS.values()]])
    eps = 1e-6
    for k in picks:
        e = np.zeros_like(p)
        e[k] = eps
        fd = (loss(p + e) - loss(p - e)) / (2 * eps)
        assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(fd)), (k, fd, g[k])


def test_adam_first_step_closed_form():
    """From m = v = 0 the bias-corrected moments are g and g^2, so the first
    step moves every parameter by -lr g / (|g| + eps)."""
    rng = np.random.default_rng(2)
    p = rng.normal(size=100)
    g = rng.normal(size=100)
    q, m, v = mlp.adam(p, g, np.zeros(100), np.zeros(100), 1, 1e-3)
    np.testing.assert_allclose(q, p - 1e-3 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    np.testing.assert_allclose(m, 0.1 * g)
    np.testing.assert_allclose(v, 0.001 * g * g)
