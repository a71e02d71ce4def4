"""Branch-mean sweeps (lcsb_bind_means; the sigma = d = 2 ring and two-array
pair) against the entry-reading sweep and the oracle.  A ring with mean buffers bound reads one
mean per branch (Ma, Mab) instead of the entries, writes the entries only on
the last d sweeps of each lcsb_iterate call, and re-derives the means after
anything else writes the tables.  Every table a caller sees, the offsets and
every certificate field are the same, bit for bit, as without the means:
along zero-start trajectories in chunks of 1 .. 64 sweeps, after writes
through lcsb_lag, across lcsb_run, lcsb_upcast, checkpoints and unbinding,
and at the benchmark's full size (l = 16 FP32, l = 14 FP64)."""
import math
import sys

import numpy as np
import pytest
import torch

import oracle
import seeded_inputs as si

pytestmark = pytest.mark.gpu

CERT_FIELDS = ("R", "E", "maxW", "rho", "bound", "argmax_W", "nonfinite", "kind", "sweep")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def pk():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    import paper_2407_10925_amd as pk
    return pk


def _pair(pk, h, dtype, iteration="ring", d=2, sigma=2):
    T = pk.Lcsb(sigma, d, h, dtype, iteration=iteration)
    M = pk.Lcsb(sigma, d, h, dtype, iteration=iteration, means=True)
    T.init_zero()
    M.init_zero()
    assert T.swap_symmetric() and M.swap_symmetric()
    return T, M


def _same_certs(T, M, tag=""):
    for kind in ("feasible", "optimal"):
        if kind == "feasible":
            (ct, bt), (cm, bm) = T.certify(), M.certify()
        else:
            (ct, bt), (cm, bm) = T.certify_optimal(), M.certify_optimal()
        for f in CERT_FIELDS:
            for x, y in ((ct, cm), (bt, bm)):
                same = x[f] == y[f] or (isinstance(x[f], float) and math.isnan(x[f])
                                        and math.isnan(y[f]))
                assert same, (tag, kind, f, x[f], y[f])


def _same_tables_host(T, M, tag=""):
    """Every lag as stored and as FP64 true values (read_table leaves the
    means of the mean context in use)."""
    for k in range(1, T.lags + 1):
        for as_f64 in (False, True):
            a, b = T.read_table(k, as_f64), M.read_table(k, as_f64)
            if not np.array_equal(a, b):
                bad = int(np.nonzero(a != b)[0][0])
                raise AssertionError(f"{tag} lag {k} as_f64={as_f64}: entry {bad} "
                                     f"{a[bad]!r} vs {b[bad]!r}")


@pytest.mark.parametrize("h", [3, 6])
def test_means_trajectory_matches_the_oracle(pk, h):
    """FP64 zero start, in chunks that cross lcsb_iterate calls (1, 1, 2, 3, 5,
    8, 13, 27 sweeps): lags 1 and 2 equal the oracle's ring, entry for entry."""
    say(f"means vs oracle: h={h}")
    M = pk.Lcsb(2, 2, h, "f64", means=True)
    M.init_zero()
    N = 4 ** h
    ring = [np.zeros(N), np.zeros(N)]
    done = 0
    for chunk in (1, 1, 2, 3, 5, 8, 13, 27):
        for _ in range(chunk):
            ring = [oracle.sweep(2, 2, h, ring), ring[0]]
        M.iterate(chunk)
        done += chunk
        for k in (1, 2):
            got = M.read_table(k)
            assert np.array_equal(got, ring[k - 1][: N // 2]), (done, k)


@pytest.mark.parametrize("h", [3, 4, 5, 8, 10])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_means_ring_matches_the_entry_ring(pk, h, dtype):
    say(f"means vs entries: h={h} {dtype}")
    T, M = _pair(pk, h, dtype)
    done = 0
    for chunk in (1, 2, 7, 40, 64, 0, 1):
        T.iterate(chunk)
        M.iterate(chunk)
        done += chunk
        _same_tables_host(T, M, f"after {done}")
        _same_certs(T, M, f"after {done}")


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_writes_through_lag_are_seen_by_the_next_sweep(pk, dtype):
    """Values planted through lcsb_lag (both members of an exchanged pair, so
    the ring stays symmetric) in lag 1 and in lag 2: the mean context derives
    its means again and follows the entry context."""
    h = 7
    say(f"means after writes through lcsb_lag: {dtype}")
    T, M = _pair(pk, h, dtype)
    T.iterate(9)
    M.iterate(9)
    n = 4 ** h
    am = int("10" * h, 2)
    for k, i in ((1, 0x1357), (2, 0x0ace)):  # stored indices (below n/2 = 8192)
        e = ((i & am) >> 1) | ((i & (am >> 1)) << 1)
        if e >= n // 2:
            e ^= n - 1
        for L in (T, M):
            t, _ = L.lag(k)
            t[i] = t[i] + 0.375
            if e != i:
                t[e] = t[e] + 0.375
        torch.cuda.synchronize()
    assert T.swap_symmetric() and M.swap_symmetric()
    for chunk in (1, 4):
        T.iterate(chunk)
        M.iterate(chunk)
        _same_tables_host(T, M, f"planted, +{chunk}")
        _same_certs(T, M, f"planted, +{chunk}")


def test_run_upcast_checkpoint_and_unbind(pk, tmp_path):
    """lcsb_run (largest-r certificate every 8 sweeps) stops at the same sweep
    with the same bound; the FP32 ring upcast to an FP64 ring (buffers of its
    own) polishes the same; a checkpoint of the mean context resumes into a
    fresh mean context; unbinding the means leaves the entry sweep in charge."""
    h = 10
    say("means: run, upcast, checkpoint, unbind")
    res = []
    for means in (False, True):
        L = pk.Lcsb(2, 2, h, "f32", means=means)
        L.init_zero()
        cur, best, certs, why = L.run(8, max_sweeps=160, stop_delta=1e-9, certificate="optimal")
        P = pk.Lcsb(2, 2, h, "f64", means=means)
        P.upcast(L)
        P.iterate(24)
        res.append((cur["sweep"], best["bound"], best["argmax_W"], certs, why,
                    P.read_table(1).tobytes(), P.read_table(2).tobytes()))
        del L, P
    assert res[0] == res[1]

    T, M = _pair(pk, h, "f64")
    T.iterate(11)
    M.iterate(11)
    path = str(tmp_path / "means.ckpt")
    M.save(path)
    R = pk.Lcsb(2, 2, h, "f64", means=True)
    R.load(path)
    for L in (T, R):
        L.iterate(13)
    _same_tables_host(T, R, "resumed")
    _same_certs(T, R, "resumed")
    M._lib.lcsb_bind_means(M._ctx, None, 0)
    M.iterate(13)
    _same_tables_host(T, M, "unbound")


@pytest.mark.parametrize("h,dtype,first,rest", [(16, "f32", 3, 17), (14, "f64", 3, 29)])
def test_means_full_size_matches_the_entry_ring(pk, h, dtype, first, rest):
    """The benchmark's sizes: whole lags compared on the device after sweeps
    that cross an lcsb_iterate call, and both certificates."""
    say(f"means full size: h={h} {dtype} {first}+{rest} sweeps")
    torch.cuda.empty_cache()
    T, M = _pair(pk, h, dtype)
    for chunk in (first, rest):
        T.iterate(chunk)
        M.iterate(chunk)
    _same_certs(T, M, "full size")
    for k in (1, 2):
        a, ao = T.lag(k)
        b, bo = M.lag(k)
        assert ao == bo
        assert torch.equal(a, b), k
    del T, M
    torch.cuda.empty_cache()


def test_means_l17_fp32_matches_the_entry_ring_sampled(pk):
    """l = 17 FP32 (2^34 indices, stored entries and mean indices past 2^32):
    the mean ring and the entry ring, run one after the other (both do not fit
    together), agree on 2^20 sampled entries of lags 1 and 2, their offsets and
    both certificates after 6 sweeps (3 + 3, crossing an lcsb_iterate call)."""
    h = 17
    say("means vs entries at l=17 FP32, sampled")
    torch.cuda.empty_cache()
    got = []
    for means in (True, False):
        L = pk.Lcsb(2, 2, h, "f32", means=means)
        L.init_zero()
        L.iterate(3)
        L.iterate(3)
        cf, _ = L.certify()
        co, _ = L.certify_optimal()
        idx = si.sample_indices(L.stored, 1 << 20, seed=17).to(L.device)
        lags = []
        for k in (1, 2):
            t, off = L.lag(k)
            lags.append((t[idx].cpu().numpy(), off))
        got.append((lags, cf, co))
        del L, t
        torch.cuda.empty_cache()
    (lm, cfm, com), (le, cfe, coe) = got
    for (a, ao), (b, bo) in zip(lm, le):
        assert ao == bo
        assert np.array_equal(a, b)
    for x, y in ((cfm, cfe), (com, coe)):
        for f in CERT_FIELDS:
            assert x[f] == y[f], (f, x[f], y[f])


# ------------------------------------------------------------------ two arrays
# The two-array rate samples 4096 entries of the new table after every sweep;
# with means bound those values are recomputed from the same means
# (launch_means_samples) and the rate read from them.

@pytest.mark.parametrize("h", [3, 6])
def test_two_array_means_matches_the_oracle(pk, h):
    say(f"two-array means vs oracle: h={h}")
    _, hist, (u, u_prev, R) = oracle.two_array_run(2, 2, h, 30, cadence=30, certificate="optimal")
    M = pk.Lcsb(2, 2, h, "f64", iteration="two_array", means=True)
    M.init_zero()
    for chunk in (1, 4, 25):
        M.iterate(chunk)
    N = 4 ** h
    assert np.array_equal(M.read_table(1), u[: N // 2])
    assert np.array_equal(M.read_table(2), u_prev[: N // 2])
    assert M.rate() == R
    cp, _ = M.certify_optimal()
    c = hist[-1]["cert"]
    assert (cp["R"], cp["bound"], cp["argmax_W"], cp["nonfinite"]) == \
        (c["r"], c["bound"], c["argmin"], c["nonfinite"])


@pytest.mark.parametrize("h", [3, 5, 8, 10])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_two_array_means_matches_the_entry_pair(pk, h, dtype):
    say(f"two-array means vs entries: h={h} {dtype}")
    T, M = _pair(pk, h, dtype, "two_array")
    done = 0
    for chunk in (1, 2, 7, 40, 64, 0, 1):
        T.iterate(chunk)
        M.iterate(chunk)
        done += chunk
        assert T.rate() == M.rate(), done
        _same_tables_host(T, M, f"after {done}")
        _same_certs(T, M, f"after {done}")


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_two_array_means_run_and_writes_through_lag(pk, dtype):
    """lcsb_run (largest-r certificate every 8 sweeps) stops alike; a write
    through lcsb_lag (both members of an exchanged pair) re-derives the means
    and makes the next rate read the old table's entries again."""
    h = 9
    say(f"two-array means: run, writes through lcsb_lag: {dtype}")
    res = []
    for means in (False, True):
        L = pk.Lcsb(2, 2, h, dtype, iteration="two_array", means=means)
        L.init_zero()
        cur, best, certs, why = L.run(8, max_sweeps=200, stop_delta=1e-9, certificate="optimal")
        res.append((cur["sweep"], best["bound"], best["argmax_W"], certs, why, L.rate()))
        del L
    assert res[0] == res[1]
    T, M = _pair(pk, h, dtype, "two_array")
    T.iterate(5)
    M.iterate(5)
    n = 4 ** h
    am = int("10" * h, 2)
    i = 0x1b3c1  # a stored index (below n/2 = 131072)
    e = ((i & am) >> 1) | ((i & (am >> 1)) << 1)
    if e >= n // 2:
        e ^= n - 1
    for L in (T, M):
        t, _ = L.lag(1)
        t[i] = t[i] + 0.625
        if e != i:
            t[e] = t[e] + 0.625
    torch.cuda.synchronize()
    for chunk in (1, 6):
        T.iterate(chunk)
        M.iterate(chunk)
        assert T.rate() == M.rate()
        _same_tables_host(T, M, f"planted, +{chunk}")
        _same_certs(T, M, f"planted, +{chunk}")


def test_two_array_means_full_size(pk):
    """l = 16 FP32: whole tables on the device, the rate and both
    certificates after sweeps that cross an lcsb_iterate call."""
    say("two-array means full size: h=16 f32 3+13 sweeps")
    torch.cuda.empty_cache()
    T, M = _pair(pk, 16, "f32", "two_array")
    for chunk in (3, 13):
        T.iterate(chunk)
        M.iterate(chunk)
        assert T.rate() == M.rate()
    _same_certs(T, M, "full size")
    for k in (1, 2):
        a, ao = T.lag(k)
        b, bo = M.lag(k)
        assert ao == bo
        assert torch.equal(a, b), k
    del T, M
    torch.cuda.empty_cache()


# ------------------------------------------------------------------ sigma = 2, d = 3
# M1, M3 of lag 1, M12, M23 of lag 2 and M123 of lag 3 (m1_index .. m123_index).

@pytest.mark.parametrize("h", [3, 4])
def test_d3_means_trajectory_matches_the_oracle(pk, h):
    say(f"d=3 means vs oracle: h={h}")
    M = pk.Lcsb(2, 3, h, "f64", means=True)
    M.init_zero()
    N = 8 ** h
    ring = [np.zeros(N)] * 3
    done = 0
    for chunk in (1, 1, 2, 3, 5, 8, 20):
        for _ in range(chunk):
            ring = [oracle.sweep(2, 3, h, ring), ring[0], ring[1]]
        M.iterate(chunk)
        done += chunk
        for k in (1, 2, 3):
            assert np.array_equal(M.read_table(k), ring[k - 1][: N // 2]), (done, k)


@pytest.mark.parametrize("h", [3, 4, 6, 8])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_d3_means_ring_matches_the_entry_ring(pk, h, dtype):
    say(f"d=3 means vs entries: h={h} {dtype}")
    T, M = _pair(pk, h, dtype, d=3)
    done = 0
    for chunk in (1, 2, 7, 40, 0, 1):
        T.iterate(chunk)
        M.iterate(chunk)
        done += chunk
        _same_tables_host(T, M, f"after {done}")
        _same_certs(T, M, f"after {done}")


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_d3_means_writes_through_lag(pk, dtype):
    h = 5
    say(f"d=3 means after writes through lcsb_lag: {dtype}")
    T, M = _pair(pk, h, dtype, d=3)
    T.iterate(7)
    M.iterate(7)
    n = 8 ** h
    for k, i in ((1, 0x2a5b), (3, 0x1c3d)):  # stored indices (below n/2 = 16384)
        # the exchanged twin: strings 1 and 2 swapped in every slot, complemented
        # when that puts a 1 at string 1's head
        r3 = (n - 1) // 7
        e = (i & r3) | ((i & (r3 << 2)) >> 1) | ((i & (r3 << 1)) << 1)
        if e >= n // 2:
            e ^= n - 1
        for L in (T, M):
            t, _ = L.lag(k)
            t[i] = t[i] + 0.375
            if e != i:
                t[e] = t[e] + 0.375
        torch.cuda.synchronize()
    assert T.swap_symmetric() and M.swap_symmetric()
    for chunk in (1, 5):
        T.iterate(chunk)
        M.iterate(chunk)
        _same_tables_host(T, M, f"planted, +{chunk}")
        _same_certs(T, M, f"planted, +{chunk}")


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_d3_means_full_size(pk, dtype):
    """The benchmark's (2, 3, 10): whole lags on the device and both
    certificates after sweeps that cross an lcsb_iterate call."""
    say(f"d=3 means full size: h=10 {dtype}")
    torch.cuda.empty_cache()
    T, M = _pair(pk, 10, dtype, d=3)
    for chunk in (4, 20):
        T.iterate(chunk)
        M.iterate(chunk)
    _same_certs(T, M, "full size")
    for k in (1, 2, 3):
        a, ao = T.lag(k)
        b, bo = M.lag(k)
        assert ao == bo
        assert torch.equal(a, b), k
    del T, M
    torch.cuda.empty_cache()


# ------------------------------------------------------------------ sigma = 4, d = 2
# M4a of lag 1 and M4ab of lag 2 (m4a_index, m4ab_index); sixteen lanes of a
# hexadecet exchange values by shuffles.

def _twin4(i, h):
    """The exchanged tuple of stored index i: the two strings' symbols swapped
    in every 4-bit slot, relabelled so that string 1's head is 0."""
    n = 16 ** h
    a = 0xCCCCCCCCCCCCCCCC & (n - 1)
    b = 0x3333333333333333 & (n - 1)
    x = ((i & a) >> 2) | ((i & b) << 2)
    m = (x >> (4 * h - 2)) & 3
    return x ^ (m * ((n - 1) // 3))


@pytest.mark.parametrize("h", [3])
def test_s4_means_trajectory_matches_the_oracle(pk, h):
    say(f"sigma=4 means vs oracle: h={h}")
    M = pk.Lcsb(4, 2, h, "f64", means=True)
    M.init_zero()
    N = 16 ** h
    ring = [np.zeros(N)] * 2
    done = 0
    for chunk in (1, 1, 2, 3, 5, 8, 20):
        for _ in range(chunk):
            ring = [oracle.sweep(4, 2, h, ring), ring[0]]
        M.iterate(chunk)
        done += chunk
        for k in (1, 2):
            assert np.array_equal(M.read_table(k), ring[k - 1][: N // 4]), (done, k)


@pytest.mark.parametrize("h", [3, 4, 5, 7])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_s4_means_ring_matches_the_entry_ring(pk, h, dtype):
    say(f"sigma=4 means vs entries: h={h} {dtype}")
    T, M = _pair(pk, h, dtype, sigma=4)
    done = 0
    for chunk in (1, 2, 7, 40, 0, 1):
        T.iterate(chunk)
        M.iterate(chunk)
        done += chunk
        _same_tables_host(T, M, f"after {done}")
        _same_certs(T, M, f"after {done}")


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_s4_means_writes_through_lag(pk, dtype):
    h = 4
    say(f"sigma=4 means after writes through lcsb_lag: {dtype}")
    T, M = _pair(pk, h, dtype, sigma=4)
    T.iterate(7)
    M.iterate(7)
    for k, i in ((1, 0x2a5b), (2, 0x1c3d)):  # stored indices (below n/4 = 16384)
        e = _twin4(i, h)
        assert e < 16 ** h // 4
        for L in (T, M):
            t, _ = L.lag(k)
            t[i] = t[i] + 0.375
            if e != i:
                t[e] = t[e] + 0.375
        torch.cuda.synchronize()
    assert T.swap_symmetric() and M.swap_symmetric()
    for chunk in (1, 5):
        T.iterate(chunk)
        M.iterate(chunk)
        _same_tables_host(T, M, f"planted, +{chunk}")
        _same_certs(T, M, f"planted, +{chunk}")


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_s4_means_full_size(pk, dtype):
    """The benchmark's (4, 2, 8), 2^30 stored entries (32-bit indices at the
    2^32 limit): whole lags on the device and both certificates after sweeps
    that cross an lcsb_iterate call."""
    say(f"sigma=4 means full size: h=8 {dtype}")
    torch.cuda.empty_cache()
    T, M = _pair(pk, 8, dtype, sigma=4)
    for chunk in (4, 20):
        T.iterate(chunk)
        M.iterate(chunk)
    _same_certs(T, M, "full size")
    for k in (1, 2):
        a, ao = T.lag(k)
        b, bo = M.lag(k)
        assert ao == bo
        assert torch.equal(a, b), k
    del T, M
    torch.cuda.empty_cache()


def test_s4_means_l9_fp32_matches_the_entry_ring_sampled(pk):
    """sigma = 4, l = 9 FP32 (2^36 indices, 2^34 stored: the kernel's 64-bit
    index arithmetic): the mean ring and the entry ring, run one after the
    other (both do not fit together), agree on 2^20 sampled entries of lags 1
    and 2, their offsets and both certificates after 6 sweeps (3 + 3, crossing
    an lcsb_iterate call)."""
    h = 9
    need = 3 * 4 * (16 ** h // 4) + 3 * 4 * (16 ** h // 16 + 16 ** h // 64) + 4 * 2**30
    torch.cuda.empty_cache()
    free, _ = torch.cuda.mem_get_info()
    if free < need:
        pytest.skip(f"needs {need / 2**30:.0f} GiB of free device memory")
    say("sigma=4 means vs entries at l=9 FP32, sampled")
    got = []
    for means in (True, False):
        L = pk.Lcsb(4, 2, h, "f32", means=means)
        L.init_zero()
        L.iterate(3)
        L.iterate(3)
        cf, _ = L.certify()
        co, _ = L.certify_optimal()
        idx = si.sample_indices(L.stored, 1 << 20, seed=19).to(L.device)
        lags = []
        for k in (1, 2):
            t, off = L.lag(k)
            lags.append((t[idx].cpu().numpy(), off))
        got.append((lags, cf, co))
        del L, t
        torch.cuda.empty_cache()
    (lm, cfm, com), (le, cfe, coe) = got
    for (a, ao), (b, bo) in zip(lm, le):
        assert ao == bo
        assert np.array_equal(a, b)
    for x, y in ((cfm, cfe), (com, coe)):
        for f in CERT_FIELDS:
            assert x[f] == y[f], (f, x[f], y[f])


def test_d3_means_l11_fp32_matches_the_entry_ring_sampled(pk):
    """sigma = 2, d = 3, l = 11 FP32 (2^33 indices, 2^32 stored: the kernel's
    64-bit index arithmetic): the mean ring and the entry ring, one after the
    other, agree on 2^20 sampled entries of lags 1 to 3, their offsets and
    both certificates after 7 sweeps (3 + 4, crossing an lcsb_iterate call)."""
    h = 11
    n = 8 ** h
    need = 4 * 4 * (n // 2) + 4 * 4 * (n // 4 + n // 4 + n // 8 + n // 8 + n // 16) + 4 * 2**30
    torch.cuda.empty_cache()
    free, _ = torch.cuda.mem_get_info()
    if free < need:
        pytest.skip(f"needs {need / 2**30:.0f} GiB of free device memory")
    say("d=3 means vs entries at l=11 FP32, sampled")
    got = []
    for means in (True, False):
        L = pk.Lcsb(2, 3, h, "f32", means=means)
        L.init_zero()
        L.iterate(3)
        L.iterate(4)
        cf, _ = L.certify()
        co, _ = L.certify_optimal()
        idx = si.sample_indices(L.stored, 1 << 20, seed=23).to(L.device)
        lags = []
        for k in (1, 2, 3):
            t, off = L.lag(k)
            lags.append((t[idx].cpu().numpy(), off))
        got.append((lags, cf, co))
        del L, t
        torch.cuda.empty_cache()
    (lm, cfm, com), (le, cfe, coe) = got
    for (a, ao), (b, bo) in zip(lm, le):
        assert ao == bo
        assert np.array_equal(a, b)
    for x, y in ((cfm, cfe), (com, coe)):
        for f in CERT_FIELDS:
            assert x[f] == y[f], (f, x[f], y[f])


# ------------------------------------------------------------------ sigma = 4, two arrays
# The rate's sample values recomputed from M4a and M4ab (means_samples4).

@pytest.mark.parametrize("h", [3])
def test_s4_two_array_means_matches_the_oracle(pk, h):
    say(f"sigma=4 two-array means vs oracle: h={h}")
    _, hist, (u, u_prev, R) = oracle.two_array_run(4, 2, h, 30, cadence=30, certificate="optimal")
    M = pk.Lcsb(4, 2, h, "f64", iteration="two_array", means=True)
    M.init_zero()
    for chunk in (1, 4, 25):
        M.iterate(chunk)
    N = 16 ** h
    assert np.array_equal(M.read_table(1), u[: N // 4])
    assert np.array_equal(M.read_table(2), u_prev[: N // 4])
    assert M.rate() == R
    cp, _ = M.certify_optimal()
    c = hist[-1]["cert"]
    assert (cp["R"], cp["bound"], cp["argmax_W"], cp["nonfinite"]) == \
        (c["r"], c["bound"], c["argmin"], c["nonfinite"])


@pytest.mark.parametrize("h", [3, 4, 6])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_s4_two_array_means_matches_the_entry_pair(pk, h, dtype):
    say(f"sigma=4 two-array means vs entries: h={h} {dtype}")
    T, M = _pair(pk, h, dtype, "two_array", sigma=4)
    done = 0
    for chunk in (1, 2, 7, 40, 0, 1):
        T.iterate(chunk)
        M.iterate(chunk)
        done += chunk
        assert T.rate() == M.rate(), done
        _same_tables_host(T, M, f"after {done}")
        _same_certs(T, M, f"after {done}")


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_s4_two_array_means_run_and_writes_through_lag(pk, dtype):
    """lcsb_run stops alike with and without means; a write through lcsb_lag
    (both members of an exchanged pair) re-derives the means."""
    h = 4
    say(f"sigma=4 two-array means: run, writes through lcsb_lag: {dtype}")
    res = []
    for means in (False, True):
        L = pk.Lcsb(4, 2, h, dtype, iteration="two_array", means=means)
        L.init_zero()
        cur, best, certs, why = L.run(8, max_sweeps=200, stop_delta=1e-9, certificate="optimal")
        res.append((cur["sweep"], best["bound"], best["argmax_W"], certs, why, L.rate()))
        del L
    assert res[0] == res[1]
    T, M = _pair(pk, h, dtype, "two_array", sigma=4)
    T.iterate(5)
    M.iterate(5)
    i = 0x2a5b
    e = _twin4(i, h)
    for L in (T, M):
        t, _ = L.lag(1)
        t[i] = t[i] + 0.625
        if e != i:
            t[e] = t[e] + 0.625
    torch.cuda.synchronize()
    for chunk in (1, 6):
        T.iterate(chunk)
        M.iterate(chunk)
        assert T.rate() == M.rate()
        _same_tables_host(T, M, f"planted, +{chunk}")
        _same_certs(T, M, f"planted, +{chunk}")


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_s4_two_array_means_full_size(pk, dtype):
    """(4, 2, 8): whole tables on the device, the rate and both certificates
    after sweeps that cross an lcsb_iterate call."""
    say(f"sigma=4 two-array means full size: h=8 {dtype}")
    torch.cuda.empty_cache()
    T, M = _pair(pk, 8, dtype, "two_array", sigma=4)
    for chunk in (3, 13):
        T.iterate(chunk)
        M.iterate(chunk)
        assert T.rate() == M.rate()
    _same_certs(T, M, "full size")
    for k in (1, 2):
        a, ao = T.lag(k)
        b, bo = M.lag(k)
        assert ao == bo
        assert torch.equal(a, b), k
    del T, M
    torch.cuda.empty_cache()


# ------------------------------------------------------------------ d = 3, two arrays
# The rate's sample values recomputed from the five means (means_samples3).

@pytest.mark.parametrize("h", [3, 4])
def test_d3_two_array_means_matches_the_oracle(pk, h):
    say(f"d=3 two-array means vs oracle: h={h}")
    _, hist, (u, u_prev, R) = oracle.two_array_run(2, 3, h, 30, cadence=30, certificate="optimal")
    M = pk.Lcsb(2, 3, h, "f64", iteration="two_array", means=True)
    M.init_zero()
    for chunk in (1, 4, 25):
        M.iterate(chunk)
    N = 8 ** h
    assert np.array_equal(M.read_table(1), u[: N // 2])
    assert np.array_equal(M.read_table(2), u_prev[: N // 2])
    assert M.rate() == R
    cp, _ = M.certify_optimal()
    c = hist[-1]["cert"]
    assert (cp["R"], cp["bound"], cp["argmax_W"], cp["nonfinite"]) == \
        (c["r"], c["bound"], c["argmin"], c["nonfinite"])


@pytest.mark.parametrize("h", [3, 4, 6, 8])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_d3_two_array_means_matches_the_entry_pair(pk, h, dtype):
    say(f"d=3 two-array means vs entries: h={h} {dtype}")
    T, M = _pair(pk, h, dtype, "two_array", d=3)
    done = 0
    for chunk in (1, 2, 7, 40, 0, 1):
        T.iterate(chunk)
        M.iterate(chunk)
        done += chunk
        assert T.rate() == M.rate(), done
        _same_tables_host(T, M, f"after {done}")
        _same_certs(T, M, f"after {done}")


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_d3_two_array_means_run_and_writes_through_lag(pk, dtype):
    """lcsb_run stops alike with and without means; a write through lcsb_lag
    (both members of an exchanged pair) re-derives the means."""
    h = 5
    say(f"d=3 two-array means: run, writes through lcsb_lag: {dtype}")
    res = []
    for means in (False, True):
        L = pk.Lcsb(2, 3, h, dtype, iteration="two_array", means=means)
        L.init_zero()
        cur, best, certs, why = L.run(8, max_sweeps=200, stop_delta=1e-9, certificate="optimal")
        res.append((cur["sweep"], best["bound"], best["argmax_W"], certs, why, L.rate()))
        del L
    assert res[0] == res[1]
    T, M = _pair(pk, h, dtype, "two_array", d=3)
    T.iterate(5)
    M.iterate(5)
    n = 8 ** h
    i = 0x2a5b
    r3 = (n - 1) // 7
    e = (i & r3) | ((i & (r3 << 2)) >> 1) | ((i & (r3 << 1)) << 1)
    if e >= n // 2:
        e ^= n - 1
    for L in (T, M):
        t, _ = L.lag(1)
        t[i] = t[i] + 0.625
        if e != i:
            t[e] = t[e] + 0.625
    torch.cuda.synchronize()
    for chunk in (1, 6):
        T.iterate(chunk)
        M.iterate(chunk)
        assert T.rate() == M.rate()
        _same_tables_host(T, M, f"planted, +{chunk}")
        _same_certs(T, M, f"planted, +{chunk}")


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_d3_two_array_means_full_size(pk, dtype):
    """(2, 3, 10): whole tables on the device, the rate and both certificates
    after sweeps that cross an lcsb_iterate call."""
    say(f"d=3 two-array means full size: h=10 {dtype}")
    torch.cuda.empty_cache()
    T, M = _pair(pk, 10, dtype, "two_array", d=3)
    for chunk in (3, 13):
        T.iterate(chunk)
        M.iterate(chunk)
        assert T.rate() == M.rate()
    _same_certs(T, M, "full size")
    for k in (1, 2):
        a, ao = T.lag(k)
        b, bo = M.lag(k)
        assert ao == bo
        assert torch.equal(a, b), k
    del T, M
    torch.cuda.empty_cache()
