"""FP64 reference of the warm-start network (test infrastructure).

The network is not part of the paper: it is a learned initial table for the
iteration of Algorithm 2, whose limit does not depend on the starting table
(F is monotone and translation invariant, hence non-expansive).  It maps a
tuple of two binary head strings to a guess of the normalised converged table
value v[A] - v[0]:

    x (32 inputs) -> relu(W1 x + b1) -> relu(W2 . + b2) -> relu(W3 . + b3) -> w4 . + b4

Inputs: the symbols at the window positions P(l) = (1..8, l-7..l) of string
a and string b, slot 2j = a_{P_j}, slot 2j+1 = b_{P_j}, symbol s -> 2s - 1.
For l = 16 this is the 32 index bits in order; for shorter windows the last
eight positions keep their distance from the end of the window.

The GPU computes every matrix product with BF16 operands and FP32
accumulation: weight matrices are the BF16 rounding (to nearest, ties to
even) of FP32 master weights, and the activations fed to the next layer are
rounded to BF16 after the ReLU.  forward() models exactly those roundings
(bf16=True) in FP64 arithmetic otherwise; with bf16=False it is the plain
FP64 network used for gradient checks.  Gradients are taken with respect to
the weights as used (the BF16 rounding passes gradients unchanged).
"""
from __future__ import annotations

import numpy as np

IN = 32
WIDTH = 256
LAYOUT = [("W1", (WIDTH, IN)), ("b1", (WIDTH,)), ("W2", (WIDTH, WIDTH)), ("b2", (WIDTH,)),
          ("W3", (WIDTH, WIDTH)), ("b3", (WIDTH,)), ("w4", (WIDTH,)), ("b4", (1,))]


def _offsets():
    out, o = {}, 0
    for name, shape in LAYOUT:
        n = int(np.prod(shape))
        out[name] = (o, shape)
        o += n
    return out, o


OFFSETS, NPARAMS = _offsets()


def unpack(flat):
    flat = np.asarray(flat)
    return {k: flat[o:o + int(np.prod(s))].reshape(s) for k, (o, s) in OFFSETS.items()}


def positions(h):
    """1-based window positions feeding the 16 input pairs."""
    if h < 8:
        raise ValueError("the encoding needs l >= 8")
    return list(range(1, 9)) + list(range(h - 7, h + 1))


def encode(idx, h):
    """(B, 32) float64 inputs for sigma = d = 2 indices at window length h.
    Bit layout of an index: position p of string a at bit 2(h-p)+1, of b at
    bit 2(h-p) (interleaved pair, Sec. 3.2)."""
    idx = np.asarray(idx, dtype=np.uint64)
    X = np.empty((idx.size, IN), dtype=np.float64)
    for j, p in enumerate(positions(h)):
        a = (idx >> np.uint64(2 * (h - p) + 1)) & np.uint64(1)
        b = (idx >> np.uint64(2 * (h - p))) & np.uint64(1)
        X[:, 2 * j] = 2.0 * a.astype(np.float64) - 1.0
        X[:, 2 * j + 1] = 2.0 * b.astype(np.float64) - 1.0
    return X


def bf16(x):
    """Round to BF16 (via FP32, each step to nearest, ties to even); return FP64."""
    f = np.asarray(x, dtype=np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + np.uint64(0x7FFF) + ((u >> np.uint64(16)) & np.uint64(1))) >> np.uint64(16)
    return (u.astype(np.uint32) << np.uint32(16)).view(np.float32).astype(np.float64)


def forward(flat, X, bf16_ops=True):
    p = unpack(np.asarray(flat, dtype=np.float64))
    q = (lambda a: bf16(a)) if bf16_ops else (lambda a: a)
    W1, W2, W3, w4 = q(p["W1"]), q(p["W2"]), q(p["W3"]), q(p["w4"])
    z1 = X @ W1.T + p["b1"]
    h1 = np.maximum(z1, 0.0)
    a1 = q(h1)
    z2 = a1 @ W2.T + p["b2"]
    h2 = np.maximum(z2, 0.0)
    a2 = q(h2)
    z3 = a2 @ W3.T + p["b3"]
    h3 = np.maximum(z3, 0.0)
    a3 = q(h3)
    y = a3 @ w4 + p["b4"][0]
    cache = {"X": X, "a1": a1, "a2": a2, "a3": a3, "W1": W1, "W2": W2, "W3": W3, "w4": w4,
             "z1": z1, "z2": z2, "z3": z3, "m1": z1 > 0, "m2": z2 > 0, "m3": z3 > 0}
    return y, cache


def mse(y, t):
    """Mean squared error and its gradient with respect to y."""
    r = np.asarray(y, np.float64) - np.asarray(t, np.float64)
    return float(np.mean(r * r)), 2.0 * r / r.size


def backward(cache, dy, bf16_grads=False):
    """Gradient of the loss with respect to every parameter (flat FP64 vector).

    bf16_grads=False: the exact gradient of forward() (ReLU' from the sign of
    the pre-activation).  bf16_grads=True: the rounding the GPU applies to the
    back-propagated signal, in FP64 otherwise: ReLU' is read off the stored
    BF16 activation (a > 0), the output layer's dZ3 = dy * w4 is formed in
    FP32 and rounded to BF16, and each dZ that meets a weight matrix on its
    way down (dZ2 = dZ3 W3, dZ1 = dZ2 W2) is rounded to BF16 after its
    product; weight and bias gradients are exact sums of those."""
    g = {}
    dy = np.asarray(dy, np.float64)
    g["w4"] = cache["a3"].T @ dy
    g["b4"] = np.array([dy.sum()])
    if bf16_grads:
        m3, m2, m1 = cache["a3"] > 0, cache["a2"] > 0, cache["a1"] > 0
        prod = np.outer(dy.astype(np.float32), cache["w4"].astype(np.float32))  # FP32 products
        dz3 = bf16(prod.astype(np.float64)) * m3
        g["W3"] = dz3.T @ cache["a2"]
        g["b3"] = dz3.sum(0)
        dz2 = bf16(dz3 @ cache["W3"]) * m2
        g["W2"] = dz2.T @ cache["a1"]
        g["b2"] = dz2.sum(0)
        dz1 = bf16(dz2 @ cache["W2"]) * m1
    else:
        dz3 = np.outer(dy, cache["w4"]) * cache["m3"]
        g["W3"] = dz3.T @ cache["a2"]
        g["b3"] = dz3.sum(0)
        dz2 = (dz3 @ cache["W3"]) * cache["m2"]
        g["W2"] = dz2.T @ cache["a1"]
        g["b2"] = dz2.sum(0)
        dz1 = (dz2 @ cache["W2"]) * cache["m1"]
    g["W1"] = dz1.T @ cache["X"]
    g["b1"] = dz1.sum(0)
    cache["dz3"], cache["dz2"], cache["dz1"] = dz3, dz2, dz1
    out = np.empty(NPARAMS)
    for k, (o, s) in OFFSETS.items():
        out[o:o + int(np.prod(s))] = g[k].reshape(-1)
    return out


def adam(p, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (Kingma and Ba, ICLR 2015, Algorithm 1); returns new (p, m, v)."""
    m = beta1 * m + (1 - beta1) * g
    v = beta2 * v + (1 - beta2) * g * g
    mhat = m / (1 - beta1 ** t)
    vhat = v / (1 - beta2 ** t)
    return p - lr * mhat / (np.sqrt(vhat) + eps), m, v
