"""Pins of the oracle's two-array iteration (a reading of the remark of
Sec. 3.3 that the recurrence can run on two arrays).

One step is u_new = F(u, u - R, .., u - (d-1) R), the shift added to each
branch mean; R is the mean growth of the previous step over a fixed sample of
4096 coordinates.  Pinned here against things other than that code:

* on dyadic tables (every operation exact) one step equals the plain sweep of
  the ring whose lag k is u - (k-1) R, bit for bit;
* on non-dyadic tables, the binary case table (eqs. (7)-(9)) in exact
  rational arithmetic on the maps (u, u - R), within a few ulps;
* the rate: an exact constant growth gives that constant; the sample lies in
  the stored half of the index range and is spread over it;
* the limits: 2/(sigma+1) at l = 1 for d = 2 and 2/3 for sigma = 2, d = 3,
  Table 2 for l <= 7, Appendix C cells, and the ring's own converged bound at
  l = 8 (the two iterations share their fixed points);
* the string-exchange and relabelling symmetries survive a step bit for bit
  (the shifts are uniform), as the folded GPU kernels need.
"""
import math
import os
from fractions import Fraction

import numpy as np
import pytest

from test_oracle_certificate import _F_binary, _as_map, _index, _strings

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rows(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return [l.split() for l in f if l.strip() and not l.startswith("#")]


@pytest.mark.parametrize("sigma,d,h", [(2, 2, 3), (2, 2, 4), (4, 2, 2), (2, 3, 3), (3, 2, 2)])
def test_step_is_the_ring_sweep_of_the_extrapolated_ring(orc, sigma, d, h):
    """Dyadic table and rate: every sum, mean and shift is exact, so the step
    equals the sweep of the ring [u, u - R, .., u - (d-1) R] exactly."""
    rng = np.random.default_rng(7 + h)
    N = sigma ** (d * h)
    u = rng.integers(0, 512, N) / 64.0
    R = 0.375
    ring = [u - k * R for k in range(d)]
    if sigma == 3:  # thirds are not exact: only the structure is compared
        assert np.allclose(orc.two_array_step(sigma, d, h, u, R), orc.sweep(sigma, d, h, ring),
                           rtol=0, atol=1e-12)
    else:
        assert np.array_equal(orc.two_array_step(sigma, d, h, u, R), orc.sweep(sigma, d, h, ring))


@pytest.mark.parametrize("h", [1, 2, 3])
def test_step_against_the_binary_case_table_in_exact_arithmetic(orc, h):
    rng = np.random.default_rng(40 + h)
    N = 4 ** h
    u = rng.random(N) * 7.0
    R = 0.3817
    got = orc.two_array_step(2, 2, h, u, R)
    um = _as_map(u, h)
    shifted = {k: v - Fraction(R) for k, v in um.items()}
    exact = _F_binary(um, shifted, h)
    for (a, b), v in exact.items():
        g = Fraction(float(got[_index(a, b)]))
        assert abs(g - v) <= 4 * Fraction(2) ** -52 * max(1, abs(v)), (a, b)


def test_constant_growth_gives_its_rate(orc):
    rng = np.random.default_rng(3)
    for sigma, d, h in [(2, 2, 7), (4, 2, 3), (2, 3, 4), (2, 2, 2)]:
        N = sigma ** (d * h)
        u = rng.integers(0, 1 << 20, N) / 1024.0
        for c in (0.0, 0.5, -3.25, 2.0 ** -20):
            assert orc.sample_growth(sigma, d, h, u + c, u) == c


def test_rate_is_the_sample_mean(orc):
    sigma, d, h = 2, 2, 8
    N = 4 ** h
    rng = np.random.default_rng(5)
    u, v = rng.random(N), rng.random(N) + 0.4
    c = orc.sample_coordinates(sigma, d, h).astype(np.int64)
    exact = sum(Fraction(float(v[i] - u[i])) for i in c) / len(c)
    got = Fraction(orc.sample_growth(sigma, d, h, v, u))
    assert abs(got - exact) <= 4096 * Fraction(2) ** -53


@pytest.mark.parametrize("sigma,d,h", [(2, 2, 8), (4, 2, 4), (2, 3, 6), (2, 2, 3)])
def test_sample_coordinates(orc, sigma, d, h):
    """In the stored half (string-1 head 0), distinct when that half holds at
    least 4096 coordinates, and spread: every top bit pattern below the head
    occurs when the half is large."""
    c = orc.sample_coordinates(sigma, d, h)
    N = sigma ** (d * h)
    ns = N // sigma
    assert c.size == orc.SAMPLE and np.all(c < ns)
    for i in (0, 1, 4095):
        assert c[i] == (i * 0x9E3779B97F4A7C15) % (1 << 64) % ns
    if ns >= 4096:
        assert np.unique(c).size == 4096
        top = (c >> np.uint64(int(math.log2(ns)) - 4)) & np.uint64(15)
        assert np.unique(top).size == 16
    else:
        assert np.unique(c).size == ns


@pytest.mark.parametrize("sigma,d,limit", [(2, 2, Fraction(2, 3)), (3, 2, Fraction(1, 2)),
                                           (4, 2, Fraction(2, 5)), (2, 3, Fraction(2, 3))])
def test_l1_limit(orc, sigma, d, limit):
    """At l = 1 the bound tends to 2/(sigma+1) for d = 2 and 2/3 for sigma = 2,
    d = 3 (Appendix C, l = 1)."""
    for cert in ("feasible", "optimal"):
        best, _, _ = orc.two_array_run(sigma, d, 1, 150, 1, cert)
        assert best["bound"] <= float(limit) + 1e-15
        assert abs(best["bound"] - float(limit)) <= 1e-9, (cert, best)


@pytest.mark.parametrize("h", [2, 3, 4, 5, 6, 7])
def test_table2(orc, h):
    printed = {int(r[0]): float(r[1]) for r in _rows("table2_binary_bounds.txt")}[h]
    best, _, _ = orc.two_array_run(2, 2, h, 60 + 20 * h, 1, "optimal")
    assert math.floor(best["bound"] * 1e6) / 1e6 == printed


@pytest.mark.parametrize("sigma,d,h", [(4, 2, 2), (4, 2, 3), (2, 3, 2), (2, 3, 3)])
def test_appendix_c(orc, sigma, d, h):
    cell = [float(r[3]) for r in _rows("appendixC_bounds.txt")
            if (int(r[0]), int(r[1]), int(r[2])) == (h, sigma, d) and r[4] == "ok"]
    assert cell
    best, _, _ = orc.two_array_run(sigma, d, h, 150, 1, "optimal")
    assert abs(best["bound"] - cell[0]) <= 1e-6 or math.floor(best["bound"] * 1e6) / 1e6 == cell[0]


@pytest.mark.slow
def test_same_limit_as_the_ring_at_l8(orc):
    """Both iterations converge to the same certified bound (their fixed
    points agree); the two-array one is certified here with both kinds."""
    ring_best, _, _ = orc.feasible_triplet(2, 2, 8, 200, 1)
    ring_opt = max(orc.certify_optimal(2, 2, 8, u)["bound"]
                   for u in [orc.feasible_triplet(2, 2, 8, 200, 200, want_ring=True)[2][0]])
    for cert in ("feasible", "optimal"):
        best, _, (u, up, R) = orc.two_array_run(2, 2, 8, 160, 4, cert)
        assert abs(best["bound"] - ring_best["bound"]) <= 1e-9, cert
        assert abs(best["bound"] - ring_opt) <= 1e-9
        assert abs(2 * R - ring_best["bound"]) <= 1e-8  # the rate is the limit's r


@pytest.mark.parametrize("sigma,d,h", [(2, 2, 4), (4, 2, 3), (2, 3, 4)])
def test_step_keeps_the_symmetries(orc, sigma, d, h):
    """A table invariant under c -> c xor m and under exchanging strings 1 and
    2 stays so after a step, bit for bit (the folded kernels rely on it)."""
    import torch
    import seeded_inputs as si
    u = si.table(sigma, d, h, seed=77, exchange=True).numpy()
    new = orc.two_array_step(sigma, d, h, u, 0.41)
    idx = torch.arange(sigma ** (d * h))
    assert np.array_equal(new, new[si.representative(idx, sigma, d, h).numpy()])
    assert np.array_equal(new, new[si.exchanged(idx, sigma, d, h).numpy()])


def test_rate_converges_to_r_and_growth_is_uniform(orc):
    """Near the limit every coordinate grows by the same r = bound / d."""
    best, _, (u, up, R) = orc.two_array_run(2, 2, 6, 150, 1, "optimal")
    g = u - up
    assert g.max() - g.min() <= 1e-10
    assert abs(R - best["bound"] / 2) <= 1e-10


def test_sampled_step_is_the_whole_step_there(orc):
    rng = np.random.default_rng(9)
    for sigma, d, h in [(2, 2, 5), (4, 2, 2), (2, 3, 3)]:
        N = sigma ** (d * h)
        u = rng.random(N) * 5
        idx = np.unique(rng.integers(0, N, 200)).astype(np.uint64)
        whole = orc.two_array_step(sigma, d, h, u, 0.37)
        assert np.array_equal(orc.two_array_step_at(sigma, d, h, u, 0.37, idx), whole[idx.astype(np.int64)])
