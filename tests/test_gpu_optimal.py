"""GPU parity of the largest-r certificate (lcsb_certify_optimal) against the
CPU oracle, and full-size checks of both certificates on the exchange-folded
kernels the benchmarks run.

The largest-r certificate of a table u is r = min_A max_z c_z(A) / k_z (lemma
of Sec. 2.1 with eps = 0), every step rounded toward -inf; the GPU must give
the oracle's r, bound, lowest minimising index and non-finite count bit for
bit on the same seeded inputs.  Full-size tables are too large for the
oracle's whole-table pass, so there a known extreme is planted: raising u (and
prev, so R stays) on one symmetry orbit by far more than the table's spread
makes that orbit's lowest index the argmax of W and the argmin of the ratio,
wherever it lies in the index range; the certificate must find exactly that
index, with the oracle's value there, and every sampled coordinate must be on
the right side of it.
"""
import math
import sys

import numpy as np
import pytest
import torch

import oracle
import seeded_inputs as si

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def pk():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    import paper_2407_10925_amd as pk
    return pk


def _host(t):
    return t.detach().cpu().numpy()


def _full(L, got):
    idx = torch.arange(L.n, dtype=torch.int64)
    return _host(got)[si.representative(idx, L.sigma, L.d, L.h).numpy()]


def _same_opt(gpu, ref, sigma=None):
    """The GPU's largest-r certificate against the oracle's: r, bound, the
    lowest minimising index and the non-finite count (GPU counts stored
    coordinates; times sigma gives the oracle's count over all indices)."""
    assert gpu["kind"] == 1
    assert gpu["R"] == ref["r"] and gpu["rho"] == ref["r"], (gpu["R"], ref["r"])
    assert math.copysign(1.0, gpu["R"]) == math.copysign(1.0, ref["r"])
    assert gpu["bound"] == ref["bound"], (gpu["bound"], ref["bound"])
    assert gpu["E"] == 0.0 and gpu["maxW"] == 0.0
    assert gpu["argmax_W"] == ref["argmin"], (gpu["argmax_W"], ref["argmin"])
    nf = gpu["nonfinite"] * (sigma or 1)
    assert nf == ref["nonfinite"], (nf, ref["nonfinite"])


# ------------------------------------------------------------------ zero-start trajectories
@pytest.mark.parametrize("sigma,d,h,sweeps", [(2, 2, 6, 100), (2, 2, 1, 40), (2, 2, 2, 60),
                                              (4, 2, 1, 40), (4, 2, 2, 60), (2, 3, 1, 40),
                                              (2, 3, 3, 80)], ids=lambda v: str(v))
def test_optimal_certificate_on_the_zero_start_trajectory(pk, sigma, d, h, sweeps):
    """Every sweep of the plain FP64 iteration from zero: the largest-r
    certificate of the newest table equals the oracle's bit for bit, the best
    one follows Algorithm 2's keep rule on rho = r, and it is never below
    Algorithm 2's certificate of the same table by more than rounding."""
    say(f"largest-r certificate, zero start sigma={sigma} d={d} h={h} sweeps={sweeps}")
    L = pk.Lcsb(sigma, d, h, "f64")
    L.init_zero()
    N = sigma ** (d * h)
    ring = [np.zeros(N) for _ in range(d)]
    best_rho, best_sweep = 0.0, 0
    for t in range(1, sweeps + 1):
        L.iterate(1)
        ring = [oracle.sweep(sigma, d, h, ring)] + ring[:-1]
        cur, best = L.certify_optimal()
        ref = oracle.certify_optimal(sigma, d, h, ring[0])
        _same_opt(cur, ref)
        assert cur["sweep"] == t
        if ref["r"] >= best_rho:
            best_rho, best_sweep = ref["r"], t
        assert (best["rho"], best["sweep"]) == (best_rho, best_sweep)
        alg2 = oracle.certify(sigma, d, h, ring[0], ring[1])
        assert cur["bound"] >= alg2["bound"] - 1e-12


# ------------------------------------------------------------------ seeded tables
CASES = [(2, 2, h) for h in (1, 2, 3, 5, 8, 10)] + [(4, 2, h) for h in (1, 2, 3, 4)] + \
        [(2, 3, h) for h in (1, 2, 3, 5, 6)]


@pytest.mark.parametrize("sigma,d,h", CASES, ids=lambda v: str(v))
@pytest.mark.parametrize("exchange", [False, True], ids=["plain", "exchange"])
def test_optimal_certificate_of_seeded_tables(pk, sigma, d, h, exchange):
    """Seeded FP64 tables, symmetric in the two strings or not (the folded and
    the unfolded kernels), before and after one sweep."""
    say(f"largest-r certificate, seeded sigma={sigma} d={d} h={h} exchange={exchange}")
    lags = [si.table(sigma, d, h, seed=210 + k, exchange=exchange) for k in range(d)]
    L = pk.Lcsb(sigma, d, h, "f64")
    L.load_ring([x.cuda() for x in lags])
    assert L.swap_symmetric() == (exchange and h >= 2)
    cur, _ = L.certify_optimal()
    _same_opt(cur, oracle.certify_optimal(sigma, d, h, lags[0].numpy()))
    L.iterate(1)
    new = oracle.sweep(sigma, d, h, [x.numpy() for x in lags])
    cur, _ = L.certify_optimal()
    _same_opt(cur, oracle.certify_optimal(sigma, d, h, new))


@pytest.mark.parametrize("sigma,d,h", [(2, 2, 3), (2, 2, 6), (4, 2, 2), (4, 2, 3), (2, 3, 3),
                                       (2, 3, 5)], ids=lambda v: str(v))
def test_optimal_certificate_reads_only_lower_entries(pk, sigma, d, h):
    """On an exchange-symmetric ring the folded pass reads one entry of each
    exchanged pair: with every upper entry set to NaN its certificate is
    unchanged."""
    say(f"largest-r certificate, poisoned upper entries sigma={sigma} d={d} h={h}")
    u = si.table(sigma, d, h, seed=230, exchange=True)
    L = pk.Lcsb(sigma, d, h, "f64")
    L.load_ring([u.cuda()] * d)
    assert L.swap_symmetric()
    idx = torch.arange(L.stored)
    twin = si.representative(si.exchanged(idx, sigma, d, h), sigma, d, h)
    upper = (twin < idx).cuda()
    assert bool(upper.any())
    buf, _ = L.lag(1)
    buf[upper] = float("nan")
    cur, _ = L.certify_optimal()
    _same_opt(cur, oracle.certify_optimal(sigma, d, h, u.numpy()))


@pytest.mark.parametrize("sigma,d,h,exchange", [(2, 2, 5, False), (2, 2, 5, True), (4, 2, 2, False),
                                                (4, 2, 2, True), (2, 3, 3, False), (2, 3, 3, True),
                                                (2, 3, 1, False)], ids=lambda v: str(v))
@pytest.mark.parametrize("scale", [1e-300, 2.0 ** -1021], ids=["tiny", "subnormal"])
def test_optimal_certificate_of_tiny_and_subnormal_tables(pk, sigma, d, h, exchange, scale):
    """Values near and below the smallest normal double: the halving of the
    k = 2 ratio, the 1/3 of d = 3 and every round-down step round here."""
    say(f"largest-r certificate, tiny sigma={sigma} d={d} h={h} exchange={exchange}")
    u = si.table(sigma, d, h, seed=240, scale=scale, exchange=exchange)
    L = pk.Lcsb(sigma, d, h, "f64")
    L.load_ring([u.cuda()] * d)
    cur, _ = L.certify_optimal()
    _same_opt(cur, oracle.certify_optimal(sigma, d, h, u.numpy()))


@pytest.mark.parametrize("sigma,d,h,exchange", [(2, 2, 4, False), (2, 2, 4, True), (2, 2, 1, False),
                                                (4, 2, 2, False), (4, 2, 2, True), (2, 3, 3, False),
                                                (2, 3, 3, True)], ids=lambda v: str(v))
def test_optimal_certificate_of_nonfinite_tables(pk, sigma, d, h, exchange):
    """NaN, +inf and -inf entries: a NaN branch never wins the max over
    branches, so such coordinates get -inf (or +inf) ratios; the certificate
    reports them and is never kept."""
    say(f"largest-r certificate, non-finite sigma={sigma} d={d} h={h} exchange={exchange}")
    n = sigma ** (d * h)
    u = si.table(sigma, d, h, seed=250, exchange=exchange)
    for j, bad in ((3, float("nan")), (11, float("inf")), (7, -float("inf"))):
        if exchange and h >= 2:
            u[si.orbit(j % n, sigma, d, h)] = bad
        else:
            rep = si.representative(torch.arange(n), sigma, d, h)
            u[rep == rep[j % n]] = bad
    L = pk.Lcsb(sigma, d, h, "f64")
    L.load_ring([u.cuda()] * d)
    cur, best = L.certify_optimal(allow_nonfinite=True)
    ref = oracle.certify_optimal(sigma, d, h, u.numpy())
    assert ref["nonfinite"] > 0
    _same_opt(cur, ref, sigma)
    assert best["bound"] == 0.0 and best["sweep"] == 0


@pytest.mark.parametrize("sigma,d,h,exchange", [(2, 2, 4, False), (2, 2, 9, True), (4, 2, 3, True),
                                                (2, 3, 5, True), (2, 3, 4, False)],
                         ids=lambda v: str(v))
def test_optimal_certificate_of_fp32_tables(pk, sigma, d, h, exchange):
    """FP32 tables are certified as their exact FP64 values; the offset they
    are stored relative to cancels in c = b + mean - u."""
    say(f"largest-r certificate, FP32 sigma={sigma} d={d} h={h} exchange={exchange}")
    u = si.table(sigma, d, h, seed=260, dtype=torch.float32, exchange=exchange)
    L = pk.Lcsb(sigma, d, h, "f32")
    L.load_ring([u.cuda()] * d, offsets=[3.25] * d)
    cur, _ = L.certify_optimal()
    _same_opt(cur, oracle.certify_optimal(sigma, d, h, u.numpy()))


def test_run_driver_with_the_optimal_certificate(pk, tmp_path):
    """lcsb_run with certificate = optimal takes the largest-r certificate at
    its cadence: the same best as the host loop, and an earlier stop than
    Algorithm 2's certificate for the same target.  Its log holds one JSON
    line per certificate."""
    import json
    sigma, d, h = 2, 2, 6
    say("lcsb_run with the largest-r certificate")
    target = 0.7702
    L = pk.Lcsb(sigma, d, h, "f64")
    L.init_zero()
    log = tmp_path / "certs.jsonl"
    cur, best, certs, why = L.run(cadence=4, max_sweeps=400, target=target, certificate="optimal",
                                  log=log)
    assert why == "target" and best["kind"] == 1 and best["bound"] >= target
    rows = [json.loads(x) for x in log.read_text().splitlines()]
    assert len(rows) == certs and [r["sweep"] for r in rows] == [4 * (k + 1) for k in range(certs)]
    assert all(r["kind"] == "optimal" and r["E"] == 0.0 for r in rows)
    assert rows[-1]["best_bound"] == best["bound"] and rows[-1]["bound"] == cur["bound"]
    assert all(b["seconds"] >= a["seconds"] for a, b in zip(rows, rows[1:]))
    N = 4 ** h
    ring = [np.zeros(N), np.zeros(N)]
    t, best_ref = 0, None
    while True:
        for _ in range(4):
            ring = [oracle.sweep(sigma, d, h, ring), ring[0]]
        t += 4
        ref = oracle.certify_optimal(sigma, d, h, ring[0])
        if best_ref is None or ref["r"] >= best_ref["r"]:
            best_ref = dict(ref, sweep=t)
        if best_ref["bound"] >= target:
            break
    assert (best["bound"], best["sweep"], certs) == (best_ref["bound"], best_ref["sweep"], t // 4)
    M = pk.Lcsb(sigma, d, h, "f64")
    M.init_zero()
    _, best2, _, why2 = M.run(cadence=4, max_sweeps=400, target=target)
    assert why2 == "target" and best2["sweep"] >= best["sweep"]


# ------------------------------------------------------------------ full size, planted extremes
def _host_full(stored_dev, sigma, d, h, chunk=1 << 26):
    """All n values of a seeded input table (given as its stored entries on the
    device), gathered through the representative index, on the host."""
    n = sigma ** (d * h)
    out = np.empty(n, dtype=_host(stored_dev[:1]).dtype)
    for lo in range(0, n, chunk):
        idx = torch.arange(lo, min(n, lo + chunk), dtype=torch.int64, device=stored_dev.device)
        out[lo:lo + idx.numel()] = _host(stored_dev[si.representative(idx, sigma, d, h)])
    return out


FULL = [(2, 2, 14, "f64"), (2, 2, 16, "f32"), (2, 2, 16, "f64"), (4, 2, 8, "f32"),
        (2, 3, 10, "f32"), (2, 2, 17, "f32")]


@pytest.mark.timeout(900)
@pytest.mark.parametrize("sigma,d,h,dt", FULL, ids=lambda v: str(v))
def test_full_size_exchange_folded_sweep_and_certificates(pk, sigma, d, h, dt):
    """The exchange-folded kernels at the sizes the benchmarks use (l = 17:
    2^34 indices, stored entries above 2^32).  A seeded exchange-symmetric ring
    takes the folded path; one sweep is checked at sampled coordinates (FP64
    bit for bit, FP32 within its bound), R against the oracle over the whole
    table (l <= 16), and for planted orbits spread over the index range both
    certificates find the planted index with the oracle's value there."""
    n = sigma ** (d * h)
    ns = n // sigma
    es = 8 if dt == "f64" else 4
    tdt = torch.float64 if dt == "f64" else torch.float32
    need = (2 * d + 1) * ns * es + 8 * 2**30
    torch.cuda.empty_cache()  # what earlier tests left in the allocator's cache
    free, _ = torch.cuda.mem_get_info()
    if free < need:
        pytest.skip(f"needs {need / 2**30:.0f} GiB of free device memory")
    tag = f"sigma={sigma} d={d} l={h} {dt} exchange-symmetric"
    say(f"{tag}: generating the seeded ring on the device")
    src = [si.stored_table(sigma, d, h, seed=300 + k, dtype=tdt, device="cuda") for k in range(d)]
    L = pk.Lcsb(sigma, d, h, dt)
    L.load_ring(src)
    assert L.swap_symmetric(), "the seeded ring must take the exchange-folded kernels"
    small = h <= 16
    say(f"{tag}: copying u{' and prev' if small else ''} to the host")
    u = _host_full(src[0], sigma, d, h)
    prev = _host_full(src[1], sigma, d, h) if small else None
    idx_t = si.sample_indices(n, 20000, seed=11)
    idx = idx_t.numpy().astype(np.uint64)

    # planted orbits: the lowest index of each lies at the start, in the middle,
    # at the top of the stored range and (l = 17) above 2^32
    where = [5, ns // 2 + 12345, ns - 3]
    if n > 2**33:
        where += [2**32 + 77, 2**33 - 1000]
    bufs = [L.lag(k)[0] for k in (1, 2)]
    for j in where:
        orb = si.orbit(j, sigma, d, h)
        low = orb[0]
        stored = sorted({o for o in orb if o < ns})
        say(f"{tag}: planted orbit at {low} (stored members {stored})")
        keep = [b[stored].clone() for b in bufs]
        bump = 1000.0
        for b in bufs:  # u and prev raised alike: R is unchanged, W and the ratio move
            b[stored] += bump
        u_keep = u[orb].copy()
        u[orb] += u.dtype.type(bump)  # the same addition, in the same precision, on the host
        cur, _ = L.certify()
        assert cur["argmax_W"] == low, (cur["argmax_W"], low)
        w = oracle.certify_W_at_table(sigma, d, h, u, cur["R"], np.array([low], np.uint64))
        assert w[0] == cur["maxW"]
        opt, _ = L.certify_optimal()
        assert opt["argmax_W"] == low, (opt["argmax_W"], low)
        q = oracle.optimal_ratio_at(sigma, d, h, u, np.array([low], np.uint64))
        assert q[0] == opt["R"]
        qs = oracle.optimal_ratio_at(sigma, d, h, u, idx)
        assert np.all(qs >= opt["R"]) and np.all(qs[idx < low] > opt["R"])
        u[orb] = u_keep
        for b, kp in zip(bufs, keep):
            b[stored] = kp
    say(f"{tag}: certificates of the unplanted ring")
    cur, _ = L.certify()
    opt, _ = L.certify_optimal()
    if small:
        R, _ = oracle.max_diff(u, prev)
        assert cur["R"] == R
    w_arg = oracle.certify_W_at_table(sigma, d, h, u, cur["R"], np.array([cur["argmax_W"]], np.uint64))
    assert w_arg[0] == cur["maxW"]
    w_s = oracle.certify_W_at_table(sigma, d, h, u, cur["R"], idx)
    assert np.all(w_s <= cur["maxW"]) and np.all(w_s[idx < cur["argmax_W"]] < cur["maxW"])
    q_arg = oracle.optimal_ratio_at(sigma, d, h, u, np.array([opt["argmax_W"]], np.uint64))
    assert q_arg[0] == opt["R"]
    q_s = oracle.optimal_ratio_at(sigma, d, h, u, idx)
    assert np.all(q_s >= opt["R"]) and np.all(q_s[idx < opt["argmax_W"]] > opt["R"])
    if not small:
        del L, src, bufs
        torch.cuda.empty_cache()
        return
    say(f"{tag}: one sweep, sampled")
    L.iterate(1)
    assert L.swap_symmetric()
    got, o_new = L.lag(1)
    got_s = got[si.representative(idx_t.cuda(), sigma, d, h)].double().cpu().numpy() + o_new
    lags = [u, prev] + ([_host_full(src[2], sigma, d, h)] if d == 3 else [])
    ref = oracle.sweep_at_tables(sigma, d, h, lags, idx)
    if dt == "f64":
        assert np.array_equal(got_s, ref)
    else:
        assert np.max(np.abs(got_s - ref)) <= 8 * 2.0 ** -24 * (16 * 8.0 + 2)
    del L, src, bufs, got
    torch.cuda.empty_cache()
