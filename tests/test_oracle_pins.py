"""Pins of the CPU oracle to values the paper prints and to closed forms.

Everything here runs on the CPU (no GPU marker).
"""
import math
import os
from fractions import Fraction

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rows(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return [line.split() for line in f if line.strip() and not line.startswith("#")]


def floor6(x):
    return math.floor(x * 1e6 + 1e-9) / 1e6


def _converged_bound(orc, sigma, d, h):
    N = sigma ** (d * h)
    n, cad = (600, 1) if N < 5000 else (250, 5)
    best, _, _ = orc.feasible_triplet(sigma, d, h, n, cad)
    return best["bound"]


# ---------------------------------------------------------------- Table 2
@pytest.mark.parametrize("row", [r for r in _rows("table2_binary_bounds.txt") if int(r[0]) <= 7],
                         ids=lambda r: f"l{r[0]}")
def test_table2_binary_bounds(orc, row):
    """Table 2 (Sec. 4): gamma_{2,2} bound at l, floored at the 6th decimal."""
    h, printed = int(row[0]), float(row[1])
    n, cad = (200, 1) if h <= 6 else (200, 4)
    best, _, _ = orc.feasible_triplet(2, 2, h, n, cad)
    assert floor6(best["bound"]) == pytest.approx(printed, abs=1e-12)


@pytest.mark.slow
def test_table2_l8(orc):
    best, _, _ = orc.feasible_triplet(2, 2, 8, 200, 4)
    assert floor6(best["bound"]) == pytest.approx(0.776860, abs=1e-12)


# ---------------------------------------------------------------- Appendix C
_APPC = _rows("appendixC_bounds.txt")


@pytest.mark.parametrize("row", [r for r in _APPC if r[4] == "ok"],
                         ids=lambda r: f"l{r[0]}-s{r[1]}-d{r[2]}")
def test_appendix_c_bounds(orc, row):
    """Appendix C cells: printed value is floor6 or nearest-6 of the bound."""
    h, sigma, d, printed = int(row[0]), int(row[1]), int(row[2]), float(row[3])
    b = _converged_bound(orc, sigma, d, h)
    candidates = {round(floor6(b), 6), round(b, 6)}
    assert any(abs(c - printed) < 1e-12 for c in candidates), (b, printed)


@pytest.mark.parametrize("row", [r for r in _APPC if r[4] == "typo"],
                         ids=lambda r: f"l{r[0]}-s{r[1]}-d{r[2]}")
def test_appendix_c_flagged_cells_contradict_table3(orc, row):
    """The two flagged cells exceed Table 3's best bound for the same (sigma, d),
    which a run at l = 1 cannot do (bounds grow with l); the iteration gives 8/13."""
    h, sigma, d, printed = int(row[0]), int(row[1]), int(row[2]), float(row[3])
    best3 = {(int(r[0]), int(r[1])): float(r[3]) for r in _rows("table3_general_bounds.txt")}
    assert printed > best3[(sigma, d)]
    b = _converged_bound(orc, sigma, d, h)
    assert abs(b - 8 / 13) < 1e-6
    assert b < best3[(sigma, d)]


# ---------------------------------------------------------------- closed forms, l = 1
@pytest.mark.parametrize("sigma", [2, 3, 4, 5, 6])
def test_l1_d2_closed_form(orc, sigma):
    """l = 1, d = 2.  With M the value of a match pair and X of a mismatch pair,
    eq. (2) gives M_n = 1 + S_{n-2} and every branch of eq. (3) gives
    X_n = S_{n-1}, where S = (M + (sigma-1) X) / sigma (each branch averages a
    full row, column or table), so sigma S_n = 1 + S_{n-2} + (sigma-1) S_{n-1}.
    Putting S_n = r n + c gives 0 = 1 - 2r - (sigma-1) r, so r = 1/(sigma+1)
    and the bound d r = 2/(sigma+1).
    The certified bound approaches it from below and never exceeds it."""
    best, hist, _ = orc.feasible_triplet(sigma, 2, 1, 400, 1)
    limit = 2.0 / (sigma + 1)
    assert best["bound"] <= limit + 1e-15
    assert limit - best["bound"] < 1e-9
    assert np.all(hist[:, 3] <= limit + 1e-15)


def test_l1_worked_trajectory(orc):
    """sigma = d = 2, l = 1, zero start, in exact arithmetic.

    By the complement symmetry two values exist: M (pairs 00, 11) and X (01,
    10).  Eq. (2): M_n = 1 + (M_{n-2} + X_{n-2})/2.  Eq. (3): both branches of
    a mismatch pair average one match and one mismatch entry of lag 1, so
    X_n = (M_{n-1} + X_{n-1})/2.  All values are dyadic, so FP64 is exact and
    the oracle must reproduce them bit for bit.  The certificate of
    Algorithm 2 on these values: R = max(dM, dX), W_match = M + 2R - (1 + S),
    W_mis = X + 2R - (S + R) with S the mean of u; bound = 2 (R - max(0, W))."""
    M = {0: Fraction(0), 1: Fraction(0)}
    X = {0: Fraction(0), 1: Fraction(0)}
    for n in range(2, 12):
        M[n] = 1 + (M[n - 2] + X[n - 2]) / 2
        X[n] = (M[n - 1] + X[n - 1]) / 2
    assert [M[n] for n in range(2, 7)] == [1, 1, Fraction(3, 2), Fraction(7, 4), Fraction(17, 8)]
    assert [X[n] for n in range(2, 7)] == [0, Fraction(1, 2), Fraction(3, 4), Fraction(9, 8),
                                          Fraction(23, 16)]
    sweeps = 10
    best, hist, ring = orc.feasible_triplet(2, 2, 1, sweeps, 1, want_ring=True)
    n_last = 1 + sweeps
    # index layout: 0 = (0,0), 1 = (0,1), 2 = (1,0), 3 = (1,1)
    assert ring[0].tolist() == [float(M[n_last]), float(X[n_last]), float(X[n_last]), float(M[n_last])]
    assert ring[1].tolist() == [float(M[n_last - 1]), float(X[n_last - 1]), float(X[n_last - 1]),
                                float(M[n_last - 1])]
    exp_bounds = []
    best_rho, best_bound = Fraction(0), Fraction(0)
    for n in range(2, n_last + 1):
        S = (M[n] + X[n]) / 2
        R = max(M[n] - M[n - 1], X[n] - X[n - 1])
        W = max(M[n] + 2 * R - (1 + S), X[n] + 2 * R - (S + R))
        E = max(Fraction(0), W)
        exp_bounds.append(2 * (R - E))
        if R - E >= best_rho:
            best_rho, best_bound = R - E, 2 * (R - E)
    assert hist[:, 3].tolist() == [float(b) for b in exp_bounds]
    # the first iterates: n = 2..6 give -1, 1/2, 1/4, 5/8, 9/16 (keep-best keeps 5/8 at n = 6)
    assert exp_bounds[:5] == [-1, Fraction(1, 2), Fraction(1, 4), Fraction(5, 8), Fraction(9, 16)]
    assert best["bound"] == float(best_bound)


# ---------------------------------------------------------------- monotone in l, below Lueker
def test_bounds_increase_with_l_and_stay_below_upper_bound(orc):
    """Table 2 grows with l; every bound stays below the upper bound 0.826280
    quoted in the abstract."""
    prev = 0.0
    for h in range(1, 7):
        best, _, _ = orc.feasible_triplet(2, 2, h, 200, 1)
        assert best["bound"] > prev
        assert best["bound"] < 0.826280
        prev = best["bound"]
