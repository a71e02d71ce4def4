"""Pins of the oracle's general F and of its certificate's rounding.

The binary case of Sec. 2.1.1 writes F for sigma = d = 2 as a four-row case
table per head pair (eqs. (7)-(9)), an independent formulation of the general
Algorithm 1.  It is evaluated here in exact rational arithmetic on strings:

* on dyadic tables it must equal the oracle's general F bit for bit;
* on arbitrary double tables it gives the exact W = u + 2R - F(u + R, u) of
  Algorithm 2, and the oracle's directed rounding must bound it: every W
  rounded up, hence E up and the bound d (R - E) down, within a few ulps.

For non-negative tables the literal 0 of the head-pair row "both heads equal
z" is never the maximum, so the case table agrees with skipping that branch.
"""
from fractions import Fraction
from itertools import product

import numpy as np
import pytest


def _strings(h):
    return ["".join(p) for p in product("01", repeat=h)]


def _index(a, b):
    """Interleave a and b, a first (Sec. 3.2)."""
    return int("".join(x + y for x, y in zip(a, b)), 2)


def _F_binary(v1, v2, h):
    """eqs. (7)-(9) on exact values; v1, v2 map (a, b) -> Fraction."""
    T = lambda s: s[1:]
    out = {}
    for a in _strings(h):
        for b in _strings(h):
            def Fz(z):
                o = "1" if z == "0" else "0"
                ha, hb = a[0], b[0]
                if ha == z and hb == z:
                    return Fraction(0)
                if ha == z and hb == o:
                    return (v1[(a, T(b) + "0")] + v1[(a, T(b) + "1")]) / 2
                if ha == o and hb == z:
                    return (v1[(T(a) + "0", b)] + v1[(T(a) + "1", b)]) / 2
                return sum(v2[(T(a) + c1, T(b) + c2)] for c1 in "01" for c2 in "01") / 4
            s = 1 if a[0] == b[0] else 0
            out[(a, b)] = s + max(Fz("0"), Fz("1"))
    return out


def _as_map(arr, h):
    return {(a, b): Fraction(float(arr[_index(a, b)])) for a in _strings(h) for b in _strings(h)}


@pytest.mark.parametrize("h", [1, 2, 3, 4])
def test_general_F_equals_binary_case_table(orc, h):
    rng = np.random.default_rng(100 + h)
    N = 4 ** h
    lag1 = rng.integers(0, 1 << 10, N) / 64.0
    lag2 = rng.integers(0, 1 << 10, N) / 64.0
    F = orc.sweep(2, 2, h, [lag1, lag2])
    Fb = _F_binary(_as_map(lag1, h), _as_map(lag2, h), h)
    for a in _strings(h):
        for b in _strings(h):
            assert Fraction(float(F[_index(a, b)])) == Fb[(a, b)]


@pytest.mark.parametrize("h,seed", [(1, 0), (1, 1), (2, 2), (2, 3), (3, 4)])
def test_certificate_rounding_bounds_exact_value(orc, h, seed):
    rng = np.random.default_rng(seed)
    N = 4 ** h
    prev = rng.random(N) * 7.0
    u = prev + rng.random(N) * 0.5 + 0.25
    c = orc.certify(2, 2, h, u, prev)
    assert c["R"] == np.max(u - prev)
    R = Fraction(c["R"])
    um = _as_map(u, h)
    shifted = {k: v + R for k, v in um.items()}
    Fex = _F_binary(shifted, um, h)           # F(v_d + R, v_d)
    Wex = {k: um[k] + 2 * R - Fex[k] for k in um}
    idx = np.arange(N, dtype=np.uint64)
    Wor = orc.certify_W_at(2, 2, h, u, c["R"], idx)
    for a in _strings(h):
        for b in _strings(h):
            w_or = Fraction(float(Wor[_index(a, b)]))
            w_ex = Wex[(a, b)]
            assert w_or >= w_ex
            assert w_or - w_ex <= Fraction(2.0 ** -44)
    maxW_ex = max(Wex.values())
    E_ex = max(Fraction(0), maxW_ex)
    bound_ex = 2 * (R - E_ex)
    assert Fraction(c["maxW"]) >= maxW_ex
    assert Fraction(c["bound"]) <= bound_ex
    assert bound_ex - Fraction(c["bound"]) <= Fraction(2.0 ** -43)
    assert c["argmax_W"] == int(np.argmax(Wor))


def test_certificate_nonfinite_is_counted(orc):
    N = 16
    u = np.ones(N)
    prev = np.zeros(N)
    u[5] = np.nan
    c = orc.certify(2, 2, 2, u, prev)
    assert c["nonfinite"] >= 1


def test_summation_tree_convention(orc):
    """Reading of an unstated detail: the sigma^k appended tuples (c_1..c_k)
    are summed by a balanced binary tree, left half first; for sigma = 2 the
    leaves are the tuples with c_1 = 0 in lexicographic order, each followed
    by its complement, so a lag-2 group (c_1 c_2 = 00, 01, 10, 11) is summed
    as (00 + 11) + (01 + 10).  Entries around 2^53, where the rounding of a
    sum depends on the association, tell that order from the lexicographic
    one and from the transposed one: for the 0/0 pair x = 0 of l = 1 the
    group is lag-2 entries 0..3."""
    big = 2.0 ** 53
    a, b, c, d = big, 1.0, 0.5, -big          # members 00, 01, 10, 11
    lag2 = np.array([a, b, c, d])
    lag1 = np.zeros(4)
    F = orc.sweep(2, 2, 1, [lag1, lag2])
    paired = ((a + d) + (b + c)) / 4       # 3/8
    lexicographic = ((a + b) + (c + d)) / 4  # 0
    transposed = ((a + c) + (b + d)) / 4   # 1/4
    assert len({paired, lexicographic, transposed}) == 3
    assert F[0] == 1.0 + paired


def test_sigma4_summation_order(orc):
    """Reading for sigma = 4: the sixteen all-advance tuples of a 0/0 pair
    are summed in the order 01 10 23 32 | 02 20 13 31 | 03 30 12 21 |
    00 33 11 22 (pairs {ab, ba} grouped by a xor b, then {aa, ~a~a}), a
    balanced tree over that list.  Values around 2^53 tell it from the
    lexicographic order: at l = 1 the group of the 0/0 pair is lag-2
    entries 0..15 (index 4 c_1 + c_2)."""
    big = 2.0 ** 53
    lag2 = np.zeros(16)
    lag2[1], lag2[4] = big, 1.0        # a pair of the new order: big + 1 rounds to big
    lag2[2], lag2[3] = -big, 1.0       # siblings in lexicographic order instead
    lag1 = np.zeros(16)
    F = orc.sweep(4, 2, 1, [lag1, lag2])
    order = [1, 4, 11, 14, 2, 8, 7, 13, 3, 12, 6, 9, 0, 15, 5, 10]

    def tree(v):
        v = list(v)
        while len(v) > 1:
            v = [v[i] + v[i + 1] for i in range(0, len(v), 2)]
        return v[0]
    new = tree(lag2[order]) / 16
    lexicographic = tree(lag2) / 16
    assert new != lexicographic
    assert F[0] == 1.0 + new


@pytest.mark.parametrize("sigma,d,h", [(2, 2, 2), (2, 2, 3), (2, 3, 2), (4, 2, 2)])
def test_tree_keeps_string_exchange_bit_for_bit(orc, sigma, d, h):
    """With the summation orders of the readings (complement-paired for
    sigma = 2, pairs {ab, ba} grouped by a xor b for sigma = 4), a sweep of
    tables symmetric under exchanging strings 1 and 2 returns a table with
    the same symmetry bit for bit: the all-advance leaves map to sibling
    leaves or sibling groups, a branch moving strings 1 and 2 keeps its
    pairs, and (d = 3) a branch moving one of them and string 3 becomes the
    branch moving the other, with its leaves in the same order.  Random
    values over sixty binades make any other association of the all-advance
    group round differently somewhere."""
    n = sigma ** (d * h)
    rng = np.random.default_rng(7 + d * 10 + h + sigma)
    swap = np.empty(n, dtype=np.int64)
    for i in range(n):
        s = orc.decode(sigma, d, h, i).copy()
        s[[0, 1]] = s[[1, 0]]
        swap[i] = orc.encode(sigma, d, h, s)
    lags = []
    for _ in range(d):
        v = rng.standard_normal(n) * np.exp2(rng.integers(-30, 30, n).astype(np.float64))
        lags.append(np.maximum(v, v[swap]))
    out = orc.sweep(sigma, d, h, lags)
    assert np.array_equal(out, out[swap])


@pytest.mark.parametrize("sigma,d,h,n", [(3, 2, 1, 80), (2, 2, 1, 60), (2, 2, 2, 120)])
def test_keep_best_prefers_the_later_iterate_on_ties(orc, sigma, d, h, n):
    """Algorithm 2 replaces the triplet when R - E >= r - eps, so among equal
    certificates the last one is kept."""
    best, hist, _ = orc.feasible_triplet(sigma, d, h, n, 1)
    rho = hist[:, 3] / d
    top = np.max(rho)
    last = int(hist[np.nonzero(rho == top)[0][-1], 0])
    assert best["sweep"] == last
    if sigma == 3:
        assert np.count_nonzero(rho == top) > 1
