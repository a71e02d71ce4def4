"""Pins of the oracle's index layout and of the symmetries F must have.

CPU only.  Values are dyadic rationals with few bits wherever an identity is
checked exactly, so FP64 sums are exact and the summation order is immaterial.
"""
import numpy as np
import pytest


def _zero_start(orc, sigma, d, h, sweeps):
    N = sigma ** (d * h)
    ring = [np.zeros(N) for _ in range(d)]
    hist = []
    for _ in range(sweeps):
        new = orc.sweep(sigma, d, h, ring)
        ring = [new] + ring[:-1]
        hist.append(new)
    return hist


def _dyadic(rng, n, bits=6, scale=8):
    return rng.integers(0, scale << bits, size=n).astype(np.float64) / (1 << bits)


# ------------------------------------------------------------ layout (Sec. 3.2)
def test_interleaved_pair_example(orc):
    """Sec. 3.2: a = 1011 and b = 0010 interleave (a first) to 10001110."""
    assert orc.encode(2, 2, 4, [[1, 0, 1, 1], [0, 0, 1, 0]]) == 0b10001110
    assert orc.decode(2, 2, 4, 0b10001110).tolist() == [[1, 0, 1, 1], [0, 0, 1, 0]]


@pytest.mark.parametrize("h", [1, 2, 3, 4])
def test_head_quarters(orc, h):
    """Sec. 3.2: pairs below 2^(2l-2) start 0/0, pairs from 2^(2l-1)+2^(2l-2)
    on start 1/1, and the ones between start differently."""
    N = 4 ** h
    for i in range(N):
        a0, b0 = orc.decode(2, 2, h, i)[:, 0]
        if i < N // 4:
            assert (a0, b0) == (0, 0)
        elif i < N // 2 + N // 4:
            assert a0 != b0
        else:
            assert (a0, b0) == (1, 1)


@pytest.mark.parametrize("h", [1, 2, 3])
def test_complement_index(orc, h):
    """eq. (10): index 2^(2l) - 1 - i holds the complemented pair of index i."""
    N = 4 ** h
    for i in range(N):
        assert (orc.decode(2, 2, h, N - 1 - i) == 1 - orc.decode(2, 2, h, i)).all()


@pytest.mark.parametrize("h", [2, 3, 4])
def test_match_and_advance_b_successor_indices(orc, h):
    """Algorithms 4 and 5 give the successor indices in the interleaved layout:
    a 0/0 pair x reads lag-2 entries 4x .. 4x+3; a 0/1 pair x (advance b)
    reads lag-1 entries i, i+1 with i = (a bits of x) | ((b bits of x, head
    bit cleared) << 2).  With random dyadic lags the oracle's F must equal
    1 + their mean at 0/0 pairs and be at least their mean at 0/1 pairs."""
    rng = np.random.default_rng(7)
    N = 4 ** h
    lag1, lag2 = _dyadic(rng, N), _dyadic(rng, N)
    F = orc.sweep(2, 2, h, [lag1, lag2])
    a_bits = int("10" * h, 2)
    b_bits = int("01" * h, 2)
    for x in range(N // 4):
        assert F[x] == 1 + (lag2[4 * x] + lag2[4 * x + 1] + lag2[4 * x + 2] + lag2[4 * x + 3]) / 4
    for x in range(N // 4, N // 2):
        bx = x & b_bits & ~(1 << (2 * h - 2))
        i = (x & a_bits) | ((bx << 2) & (N - 1))
        assert F[x] >= (lag1[i] + lag1[i + 1]) / 2


# ------------------------------------------------------------ symmetries of F
@pytest.mark.parametrize("sigma,d,h", [(2, 2, 3), (2, 2, 4), (2, 3, 2), (4, 2, 2)])
def test_symbol_xor_symmetry_of_iterates(orc, sigma, d, h):
    """Relabelling every symbol by c -> c xor m (complement for sigma = 2,
    Sec. 3.3) leaves LCS lengths unchanged, so the iterates are invariant.
    With the pairwise tree over lexicographically ordered appended tuples this
    holds bit for bit, also after many sweeps with rounding."""
    N = sigma ** (d * h)
    hist = _zero_start(orc, sigma, d, h, 40)
    for m in range(1, sigma):
        perm = np.array([orc.encode(sigma, d, h, orc.decode(sigma, d, h, i) ^ m) for i in range(N)])
        for v in hist:
            assert np.array_equal(v[perm], v)


@pytest.mark.parametrize("sigma,d,h", [(2, 2, 3), (3, 2, 2), (2, 3, 2)])
def test_string_and_alphabet_permutations_dyadic(orc, sigma, d, h):
    """Permuting the d strings, or the alphabet, permutes the coordinates of
    F.  Checked exactly on dyadic lags (exact sums)."""
    rng = np.random.default_rng(11)
    N = sigma ** (d * h)
    lags = [_dyadic(rng, N) for _ in range(d)]
    F = orc.sweep(sigma, d, h, lags)
    syms = [orc.decode(sigma, d, h, i) for i in range(N)]
    # string permutation: reverse the order of the strings
    perm = np.array([orc.encode(sigma, d, h, s[::-1]) for s in syms])
    Fp = orc.sweep(sigma, d, h, [lg[np.argsort(perm)] for lg in lags])
    # lag'[perm[i]] = lag[i]  =>  F'[perm[i]] = F[i]
    assert np.array_equal(Fp[perm], F)
    # alphabet permutation: a cyclic shift of the symbols
    perm2 = np.array([orc.encode(sigma, d, h, (s + 1) % sigma) for s in syms])
    Fq = orc.sweep(sigma, d, h, [lg[np.argsort(perm2)] for lg in lags])
    assert np.array_equal(Fq[perm2], F)


def test_match_head_invariance(orc):
    """A tuple whose strings share a head z reads only the appended tails (eq.
    (2)), so v[z a', z b'] does not depend on z."""
    h = 3
    hist = _zero_start(orc, 2, 2, h, 30)
    N = 4 ** h
    for v in hist:
        assert np.array_equal(v[: N // 4], v[3 * N // 4:])


@pytest.mark.parametrize("sigma,d,h", [(2, 2, 3), (2, 3, 2), (4, 2, 1)])
def test_iterates_nondecreasing_from_zero(orc, sigma, d, h):
    """F is monotone (feasible-triplet lemma, property 1) and v_d >= 0 = v_{d-1},
    so the zero-start iterates never decrease; round-to-nearest preserves it."""
    hist = _zero_start(orc, sigma, d, h, 60)
    for a, b in zip(hist, hist[1:]):
        assert np.all(b >= a)


@pytest.mark.parametrize("sigma,d,h", [(2, 2, 3), (2, 3, 2), (4, 2, 2), (3, 2, 2)])
def test_translation_invariance_and_monotonicity(orc, sigma, d, h):
    """Property 2 of the feasible-triplet lemma, F(v + c 1) = F(v) + c 1, and
    property 1, v <= w => F(v) <= F(w).  Exact on dyadic data for sigma in
    {2, 4}; for sigma = 3 the division by 3 rounds, so a few ulps are allowed."""
    rng = np.random.default_rng(3)
    N = sigma ** (d * h)
    lags = [_dyadic(rng, N) for _ in range(d)]
    F = orc.sweep(sigma, d, h, lags)
    for c in (0.5, 3.25, -2.0):
        Fc = orc.sweep(sigma, d, h, [lg + c for lg in lags])
        if sigma in (2, 4):
            assert np.array_equal(Fc, F + c)
        else:
            np.testing.assert_allclose(Fc, F + c, rtol=0, atol=8 * np.spacing(np.max(np.abs(F)) + 4))
    bumped = [lg + _dyadic(rng, N, scale=1) for lg in lags]
    assert np.all(orc.sweep(sigma, d, h, bumped) >= F)
