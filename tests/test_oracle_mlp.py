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


def _r(x):
    """BF16 rounding written from its definition: nearest value with 8
    significant bits, ties to the even one (exact rational arithmetic)."""
    from fractions import Fraction
    x = Fraction(x)
    if x == 0:
        return 0.0
    s = -1 if x < 0 else 1
    x = abs(x)
    e = 0
    while x >= 2:
        x /= 2
        e += 1
    while x < 1:
        x *= 2
        e -= 1
    q = x * 128  # in [128, 256)
    f = int(q)
    rem = q - f
    if rem > Fraction(1, 2) or (rem == Fraction(1, 2) and f % 2 == 1):
        f += 1
    return float(s * Fraction(f, 128) * Fraction(2) ** e)


def test_adam_later_steps_closed_form():
    """Kingma and Ba's bias correction at t = 2, 3: with a constant gradient
    every step moves by -lr g / (|g| + eps) (the corrected moments are g and
    g^2); with g, -g, g the corrected first moment is -(1-b1) g / (1+b1) at
    t = 2 and (1-b1)(1 - b1 (1-b1)) g / (1-b1^3) at t = 3."""
    b1, b2, lr, eps = 0.9, 0.999, 1e-3, 1e-8
    rng = np.random.default_rng(4)
    p0 = rng.normal(size=50)
    g = rng.normal(size=50)
    p, m, v = p0, np.zeros(50), np.zeros(50)
    for t in (1, 2, 3):
        q, m, v = mlp.adam(p, g, m, v, t, lr)
        np.testing.assert_allclose(q - p, -lr * g / (np.abs(g) + eps), rtol=1e-12, atol=1e-18)
        p = q
    p, m, v = p0, np.zeros(50), np.zeros(50)
    p1, m, v = mlp.adam(p, g, m, v, 1, lr)
    p2, m, v = mlp.adam(p1, -g, m, v, 2, lr)
    mhat2 = -(1 - b1) * g / (1 + b1)
    np.testing.assert_allclose(p2 - p1, -lr * mhat2 / (np.abs(g) + eps), rtol=1e-10, atol=1e-18)
    p3, m, v = mlp.adam(p2, g, m, v, 3, lr)
    mhat3 = (1 - b1) * (1 - b1 * (1 - b1)) * g / (1 - b1 ** 3)
    np.testing.assert_allclose(p3 - p2, -lr * mhat3 / (np.abs(g) + eps), rtol=1e-10, atol=1e-18)


def _one_path(vals):
    """A network with one live path: input 0 (and 1) -> unit 0 -> unit 0 ->
    unit 0 -> output, with the given weights and biases."""
    p = np.zeros(mlp.NPARAMS)
    P = mlp.unpack(p)
    P["W1"][0, 0], P["W1"][0, 1], P["b1"][0] = vals["w1a"], vals["w1b"], vals["b1"]
    P["W2"][0, 0], P["b2"][0] = vals["w2"], vals["b2"]
    P["W3"][0, 0], P["b3"][0] = vals["w3"], vals["b3"]
    P["w4"][0], P["b4"][0] = vals["w4"], vals["b4"]
    return p


def test_bf16_forward_rounds_weights_and_activations_not_biases():
    """Values none of which is a BF16 number: the weights and each layer's
    activation are rounded, the biases are not; computed here from the BF16
    definition (an independent rounding routine) by hand, one path."""
    v = {"w1a": 0.3, "w1b": 0.17, "b1": 0.1, "w2": 0.7, "b2": 0.05, "w3": 1.3, "b3": -0.02,
         "w4": 0.9, "b4": 0.01}
    p = _one_path(v)
    X = np.zeros((1, 32))
    X[0, 0], X[0, 1] = 1.0, -1.0
    a1 = _r(max(_r(0.3) - _r(0.17) + 0.1, 0.0))
    a2 = _r(max(_r(0.7) * a1 + 0.05, 0.0))
    a3 = _r(max(_r(1.3) * a2 - 0.02, 0.0))
    y_ref = _r(0.9) * a3 + 0.01
    y, cache = mlp.forward(p, X, bf16_ops=True)
    assert abs(y[0] - y_ref) <= 1e-15
    assert (cache["a1"][0, 0], cache["a2"][0, 0], cache["a3"][0, 0]) == (a1, a2, a3)
    # the plain network differs by far more than that
    assert abs(mlp.forward(p, X, bf16_ops=False)[0][0] - y_ref) > 1e-4


def test_bf16_gradients_round_at_the_kernel_points():
    """One live path, one sample, dy = 0.3: dZ3 = bf16(fp32(dy) fp32(w4)),
    dZ2 = bf16(dZ3 w3), dZ1 = bf16(dZ2 w2), each weight's gradient dZ times
    the layer input; checked through the bias gradients (b_k's gradient is
    dZ_k) and the weight gradients, against the BF16 definition by hand."""
    v = {"w1a": 0.5, "w1b": 0.25, "b1": 0.5, "w2": 0.7, "b2": 0.0, "w3": 1.3, "b3": 0.0,
         "w4": 0.9, "b4": 0.0}
    p = _one_path(v)
    X = np.zeros((1, 32))
    X[0, 0], X[0, 1] = 1.0, -1.0
    y, cache = mlp.forward(p, X, bf16_ops=True)
    dy = np.array([0.3])
    g = mlp.unpack(mlp.backward(cache, dy, bf16_grads=True))
    dz3 = _r(float(np.float32(0.3) * np.float32(_r(0.9))))
    dz2 = _r(dz3 * _r(1.3))
    dz1 = _r(dz2 * _r(0.7))
    assert (g["b3"][0], g["b2"][0], g["b1"][0]) == (dz3, dz2, dz1)
    assert g["W3"][0, 0] == dz3 * cache["a2"][0, 0] and g["W1"][0, 1] == -dz1
    assert g["w4"][0] == 0.3 * cache["a3"][0, 0] and g["b4"][0] == 0.3
    # the exact gradient keeps the unrounded products
    ge = mlp.unpack(mlp.backward(cache, dy, bf16_grads=False))
    assert ge["b2"][0] == 0.3 * _r(0.9) * _r(1.3) and ge["b2"][0] != dz2


def test_bf16_gradients_equal_the_exact_ones_on_a_bf16_exact_network():
    """The closed-form network with targets that make dy = +-1/4: every
    back-propagated value is a BF16 number, so both gradient forms agree bit
    for bit."""
    p = np.zeros(mlp.NPARAMS)
    P = mlp.unpack(p)
    P["W1"][0, 0], P["b1"][0], P["W2"][0, 0], P["W3"][0, 0], P["w4"][0], P["b4"][0] = \
        1.0, 0.5, 2.0, 3.0, 0.5, 0.25
    X = np.zeros((4, 32))
    X[:, 0] = [1.0, -1.0, 0.0, 1.0]
    y, cache = mlp.forward(p, X, bf16_ops=True)
    t = y - np.array([0.5, -0.5, 0.5, -0.5])
    _, dy = mlp.mse(y, t)
    assert np.all(np.abs(dy) == 0.25)
    assert np.array_equal(mlp.backward(cache, dy, bf16_grads=True),
                          mlp.backward(cache, dy, bf16_grads=False))
