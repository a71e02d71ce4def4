"""Pins of the oracle's F against the definition of W_n (Sec. 2.1).

W_n(a_1..a_d) is evaluated exactly by enumerating every random tail and
running the textbook LCS recurrence (no part of the iteration is used).  Two
facts must then hold:

* eq. (4) is an inequality about W itself: W_n >= F(W_{n-1}, ..., W_{n-d})
  coordinate-wise.  A wrong lag, branch or mean in F breaks it.
* From the zero start (a lower bound for W_0 .. W_{d-1}), monotonicity of F
  gives v_n <= W_n for every n.

For sigma in {2, 4} every W value is a dyadic rational with a small
denominator, so the FP64 evaluation of F on it is exact and the comparisons
are exact.  For sigma = 3 W is rounded to FP64 first and a 1e-12 slack is
allowed.
"""
import itertools
from fractions import Fraction

import numpy as np
import pytest

CASES = [  # sigma, d, h, n_max
    (2, 2, 1, 8),
    (2, 2, 2, 7),
    (2, 2, 3, 5),
    (4, 2, 1, 4),
    (3, 2, 1, 5),
    (2, 3, 1, 5),
    (2, 3, 2, 4),
]


def _W_table(orc, sigma, d, h, n):
    N = sigma ** (d * h)
    den = sigma ** (d * n)
    out = []
    for idx in range(N):
        sym = orc.decode(sigma, d, h, idx)
        out.append(Fraction(orc.brute_W_sum(sigma, d, h, n, sym), den))
    return out


@pytest.mark.parametrize("sigma,d,h,n_max", CASES, ids=lambda v: str(v))
def test_F_is_a_lower_bound_on_W_and_iterates_stay_below_W(orc, sigma, d, h, n_max):
    exact = sigma in (2, 4)
    tol = 0.0 if exact else 1e-12
    W = {n: _W_table(orc, sigma, d, h, n) for n in range(0, n_max + 1)}
    Wf = {n: np.array([float(x) for x in W[n]]) for n in W}
    if exact:
        for n in W:
            assert all(Fraction(float(x)) == x for x in W[n])
    # W_0 is the LCS of the heads themselves: zero start is below it
    assert all(x >= 0 for x in W[0])
    # eq. (4) on the exact W
    for n in range(d, n_max + 1):
        lags = [Wf[n - k] for k in range(1, d + 1)]
        F = orc.sweep(sigma, d, h, lags)
        assert np.all(Wf[n] >= F - tol), (n, np.max(F - Wf[n]))
    # zero-start iterates v_n <= W_n
    N = sigma ** (d * h)
    ring = [np.zeros(N) for _ in range(d)]  # ring[k-1] = lag k
    for n in range(d, n_max + 1):
        new = orc.sweep(sigma, d, h, ring)
        assert np.all(new <= Wf[n] + tol), (n, np.max(new - Wf[n]))
        ring = [new] + ring[:-1]


def test_W_small_values_by_hand(orc):
    """Three values enumerated by hand for sigma = d = 2, l = 1.

    W_0(0, 0) = L(0, 0) = 1.
    W_1(0, 1): tails (x, y) in {0,1}^2 and splits (i_1, i_2) in {(1,0), (0,1)}
    give max(L(0x, 1), L(0, 1y)) = 1, 0, 1, 1 for (x, y) = 00, 01, 10, 11,
    so W_1(0, 1) = 3/4.
    W_1(0, 0): L(0x, 0) = L(0, 0y) = 1 for every tail, so W_1(0, 0) = 1."""
    assert orc.brute_W_sum(2, 2, 1, 0, [0, 0]) == 1
    assert orc.brute_W_sum(2, 2, 1, 1, [0, 1]) == 3
    assert orc.brute_W_sum(2, 2, 1, 1, [0, 0]) == 4
