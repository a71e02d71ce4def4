"""Pins of the oracle's largest-r certificate (lemma of Sec. 2.1 with eps = 0).

For a table u the lemma accepts (u, r, 0) when F(u + (d-1) r, .., u) >= u + d r
holds at every coordinate; the oracle computes the largest such r as
min_A max_z c_z(A) / k_z with every step rounded down.  It is pinned here to
things other than that formula:

* the hand-derived worked example at l = 1 (tests/golden);
* the lemma's inequality itself, evaluated in exact rational arithmetic with
  the binary case table of eqs. (7)-(9): it must hold at the computed r and
  fail a hair above it (so r is rigorous and within that hair of optimal);
* Algorithm 2's own W (a different formula in the oracle) at R = r: its max
  must be zero up to rounding, and positive just above r;
* the limits at l = 1 (2/(sigma+1) for d = 2, 2/3 for sigma = 2, d = 3), Table 2
  at convergence, and the dominance over Algorithm 2's certificate of the
  same table, which only chooses another r.
"""
import math
import os
from fractions import Fraction

import numpy as np
import pytest

from test_oracle_certificate import _F_binary, _as_map, _index, _strings

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden_rows(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return [line.split() for line in f if line.strip() and not line.startswith("#")]


def _trajectory(orc, sigma, d, h, sweeps):
    """Zero-start ring after each sweep: list of (u, prev)."""
    N = sigma ** (d * h)
    ring = [np.zeros(N) for _ in range(d)]
    out = []
    for _ in range(sweeps):
        ring = [orc.sweep(sigma, d, h, ring)] + ring[:-1]
        out.append((ring[0], ring[1]))
    return out


def test_worked_example_l1(orc):
    (sweeps, r_star, bound_star, argmin, alg2) = _golden_rows("optimal_certificate_l1.txt")[0]
    u, prev = _trajectory(orc, 2, 2, 1, int(sweeps))[-1]
    assert u[0] == 17 / 8 and u[1] == 23 / 16 and prev[0] == 7 / 4 and prev[1] == 9 / 8
    c = orc.certify_optimal(2, 2, 1, u)
    assert (c["r"], c["bound"], c["argmin"], c["nonfinite"]) == \
        (float(r_star), float(bound_star), int(argmin), 0)
    assert orc.certify(2, 2, 1, u, prev)["bound"] == float(alg2)


def _lemma_holds(u_map, r, h):
    """F(u + r, u) >= u + 2 r at every coordinate, exactly (sigma = d = 2)."""
    shifted = {k: v + r for k, v in u_map.items()}
    F = _F_binary(shifted, u_map, h)
    return all(F[k] >= u_map[k] + 2 * r for k in u_map)


@pytest.mark.parametrize("h,seed", [(1, 0), (1, 1), (2, 2), (2, 3), (3, 4), (3, 5)])
def test_computed_r_is_feasible_and_tight_in_exact_arithmetic(orc, h, seed):
    """Non-dyadic tables, so every rounding of the oracle matters: the computed
    r satisfies the lemma's inequality with eps = 0 exactly, and r + 2^-40
    violates it somewhere."""
    rng = np.random.default_rng(200 + seed)
    N = 4 ** h
    u = rng.random(N) * 7.0 + rng.integers(0, 3, N)
    c = orc.certify_optimal(2, 2, h, u)
    r = Fraction(c["r"])
    um = _as_map(u, h)
    assert _lemma_holds(um, r, h)
    assert not _lemma_holds(um, r + Fraction(2) ** -40, h)
    assert Fraction(c["bound"]) <= 2 * r
    assert 2 * r - Fraction(c["bound"]) <= Fraction(2) ** -50


SHAPES = [(2, 2, 1), (2, 2, 2), (2, 2, 3), (2, 2, 4), (3, 2, 1), (3, 2, 2), (4, 2, 1), (4, 2, 2),
          (2, 3, 1), (2, 3, 2), (2, 3, 3)]


@pytest.mark.parametrize("sigma,d,h", SHAPES, ids=lambda v: str(v))
def test_agrees_with_algorithm2_W(orc, sigma, d, h):
    """Algorithm 2's W = u + dR - F(u + (d-1)R, .., u), evaluated by the
    oracle's own W function (rounded up), is <= 0 up to rounding at R = r
    (so E = 0 there) and positive at every coordinate attaining r once R is
    2^-30 above it."""
    rng = np.random.default_rng(300 + 17 * sigma + 5 * d + h)
    N = sigma ** (d * h)
    u = rng.random(N) * 5.0
    c = orc.certify_optimal(sigma, d, h, u)
    idx = np.arange(N, dtype=np.uint64)
    W = orc.certify_W_at(sigma, d, h, u, c["r"], idx)
    assert np.max(W) <= 2.0 ** -44
    W_above = orc.certify_W_at(sigma, d, h, u, c["r"] + 2.0 ** -30, idx)
    assert W_above[c["argmin"]] > 0.0
    ratios = orc.optimal_ratio_at(sigma, d, h, u, idx)
    assert np.min(ratios) == c["r"] and int(np.argmin(ratios)) == c["argmin"]


@pytest.mark.parametrize("sigma,d,h,sweeps", [(2, 2, 1, 40), (2, 2, 3, 60), (4, 2, 1, 40),
                                              (4, 2, 2, 40), (2, 3, 2, 60), (3, 2, 2, 40)])
def test_dominates_algorithm2_on_the_same_table(orc, sigma, d, h, sweeps):
    """Algorithm 2 certifies the same table with one particular r (the last
    step R), so the largest feasible r gives a bound at least as large, up to
    the rounding of the two computations."""
    for t, (u, prev) in enumerate(_trajectory(orc, sigma, d, h, sweeps), 1):
        a2 = orc.certify(sigma, d, h, u, prev)["bound"]
        opt = orc.certify_optimal(sigma, d, h, u)["bound"]
        assert opt >= a2 - 4 * math.ulp(max(abs(a2), 1.0)), (t, opt, a2)


@pytest.mark.parametrize("sigma,d,limit", [(2, 2, Fraction(2, 3)), (3, 2, Fraction(1, 2)),
                                           (4, 2, Fraction(2, 5)), (2, 3, Fraction(2, 3))])
def test_l1_limit(orc, sigma, d, limit):
    """At l = 1 the iteration's growth is the closed form 2/(sigma+1) for
    d = 2 (and 2/3 for sigma = 2, d = 3); the certificate of a converged table
    reaches it from below."""
    u, _ = _trajectory(orc, sigma, d, 1, 300)[-1]
    b = Fraction(orc.certify_optimal(sigma, d, 1, u)["bound"])
    assert b <= limit
    assert limit - b < Fraction(1, 10 ** 12)


@pytest.mark.parametrize("h,printed", [(2, 0.727272), (3, 0.747922), (4, 0.758576),
                                       (5, 0.765446), (6, 0.770273)])
def test_table2_at_convergence(orc, h, printed):
    """Table 2 (Sec. 4, floored at the 6th decimal) from the converged table."""
    u, _ = _trajectory(orc, 2, 2, h, 200)[-1]
    b = orc.certify_optimal(2, 2, h, u)["bound"]
    assert math.floor(b * 1e6 + 1e-9) / 1e6 == pytest.approx(printed, abs=1e-12)


def test_division_by_three_is_rounded_down(orc):
    """sigma = 2, d = 3, l = 1: the all-match tuple 000 has one branch moving
    all three strings, so its ratio is c / 3 with c = 1 + mean(u) - u[0].
    The computed ratio never exceeds c / 3, for either sign of c, and is within
    two ulps of it."""
    for u0, rest in [(0.0, 0.0), (0.1, 0.7), (5.0, 0.3), (3.0, 1.0), (1e-300, 0.0)]:
        u = np.full(8, rest)
        u[0] = u0
        q = orc.optimal_ratio_at(2, 3, 1, u, np.array([0], np.uint64))[0]
        s = sum(Fraction(float(v)) for v in u)
        c = 1 + s / 8 - Fraction(u0)
        exact = c / 3
        assert Fraction(q) <= exact
        assert exact - Fraction(q) <= 2 * Fraction(math.ulp(float(exact)))


def test_nonfinite_table(orc):
    u = np.linspace(0.0, 3.0, 16)
    u[6] = np.nan
    c = orc.certify_optimal(2, 2, 2, u)
    assert c["nonfinite"] >= 1 and c["r"] == -math.inf


def test_string_and_index_examples_agree():
    """The helpers borrowed from the case-table tests index as Sec. 3.2 does."""
    assert _index("1011", "0010") == int("10001110", 2)
    assert len(_strings(3)) == 8


def test_zero_ratio_is_positive_zero(orc):
    """A constant table: every mismatch tuple has c = 0 exactly (a zero that
    round-down subtraction makes -0); the reported r is +0."""
    u = np.full(16, 2.5)
    c = orc.certify_optimal(2, 2, 2, u)
    assert c["r"] == 0.0 and math.copysign(1.0, c["r"]) == 1.0
    assert math.copysign(1.0, c["bound"]) == 1.0
