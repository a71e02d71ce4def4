"""GPU parity of the two-array iteration (lcsb_create_iter with
LCSB_ITER_TWO_ARRAY) against the CPU oracle's two-array policy.

FP64: every table, every rate and every certificate bit for bit with
oracle.two_array_step / sample_growth / certify / certify_optimal on the same
inputs; FP32: one step within the FP32 bound of the FP64 oracle step on the
same exact values, and the FP32 run polished in FP64 reaches the ring's
converged bound.  Inputs come from tests/seeded_inputs.py.
"""
import math
import sys

import numpy as np
import pytest
import torch

import oracle
import seeded_inputs as si

pytestmark = pytest.mark.gpu

CERT_KEYS = ("R", "maxW", "E", "rho", "bound", "argmax_W", "nonfinite")


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


def _same_cert(gpu, ref):
    for k in CERT_KEYS:
        assert gpu[k] == ref[k], (k, gpu[k], ref[k])


def _same_opt(gpu, ref):
    assert (gpu["R"], gpu["bound"], gpu["argmax_W"], gpu["nonfinite"]) == \
        (ref["r"], ref["bound"], ref["argmin"], ref["nonfinite"])


def _fp32_bound(v_max, delta_max):
    """FP32 error of one sweep on exact float inputs, as derived for the
    ring's FP32 sweep (tests/test_gpu_sweep.py): u (8 V + 5 D + 3), u = 2^-24,
    |stored value| <= V, |delta_k| <= D (here the shifts -(k-1) R), plus 1%."""
    return 1.01 * 2.0 ** -24 * (8 * v_max + 5 * delta_max + 3)


@pytest.mark.parametrize("sigma,d,h,sweeps", [(2, 2, 6, 120), (2, 2, 1, 40), (2, 2, 2, 60),
                                              (4, 2, 1, 40), (4, 2, 2, 60), (2, 3, 1, 40),
                                              (2, 3, 3, 80)], ids=lambda v: str(v))
def test_fp64_zero_start_two_array_trajectory_is_bit_exact(pk, sigma, d, h, sweeps):
    """Every sweep from zero: the table, the rate of the next sweep, Algorithm
    2's certificate (u against the table before it) and the largest-r one."""
    say(f"two-array FP64 zero start sigma={sigma} d={d} h={h} sweeps={sweeps}")
    L = pk.Lcsb(sigma, d, h, "f64", iteration="two_array")
    assert L.nbuf == 2
    L.init_zero()
    assert L.swap_symmetric() == (h >= 2)
    N = sigma ** (d * h)
    u, up = np.zeros(N), np.zeros(N)
    R = oracle.sample_growth(sigma, d, h, u, up)
    assert L.rate() == R == 0.0
    for t in range(1, sweeps + 1):
        new = oracle.two_array_step(sigma, d, h, u, R)
        R = oracle.sample_growth(sigma, d, h, new, u)
        up, u = u, new
        L.iterate(1)
        assert L.rate() == R, f"rate after sweep {t}"
        got, off = L.lag(1)
        assert off == 0.0
        assert np.array_equal(_full(L, got), u), f"sweep {t}"
        cur, _ = L.certify()
        _same_cert(cur, oracle.certify(sigma, d, h, u, up))
        opt, _ = L.certify_optimal()
        _same_opt(opt, oracle.certify_optimal(sigma, d, h, u))
    assert L.swap_symmetric() == (h >= 2)


CASES = [(2, 2, h) for h in (1, 2, 3, 5, 8)] + [(4, 2, h) for h in (1, 2, 3)] + \
        [(2, 3, h) for h in (1, 2, 3, 5)]


@pytest.mark.parametrize("sigma,d,h", CASES, ids=lambda v: str(v))
@pytest.mark.parametrize("exchange", [False, True], ids=["plain", "exchange"])
def test_fp64_seeded_two_array_steps(pk, sigma, d, h, exchange):
    """Seeded tables (folded and unfolded kernels, every shift delta_k in
    play): the rate taken from the loaded pair, then three steps."""
    say(f"two-array FP64 seeded sigma={sigma} d={d} h={h} exchange={exchange}")
    u = si.table(sigma, d, h, seed=400, exchange=exchange).numpy()
    up = si.table(sigma, d, h, seed=401, exchange=exchange).numpy() - 0.3
    L = pk.Lcsb(sigma, d, h, "f64", iteration="two_array")
    L.load_ring([torch.from_numpy(u).cuda(), torch.from_numpy(up).cuda()])
    assert L.swap_symmetric() == (exchange and h >= 2)
    R = oracle.sample_growth(sigma, d, h, u, up)
    assert L.rate() == R
    for t in range(3):
        new = oracle.two_array_step(sigma, d, h, u, R)
        R = oracle.sample_growth(sigma, d, h, new, u)
        u = new
        L.iterate(1)
        assert np.array_equal(_full(L, L.lag(1)[0]), u), f"step {t}"
        assert L.rate() == R


@pytest.mark.parametrize("sigma,d,h,exchange", [(2, 2, 4, False), (2, 2, 9, True), (4, 2, 3, True),
                                                (4, 2, 2, False), (2, 3, 5, True), (2, 3, 1, False),
                                                (2, 2, 1, False)], ids=lambda v: str(v))
def test_fp32_two_array_step(pk, sigma, d, h, exchange):
    """FP32 tables with offsets: the rate (offset difference plus the sample
    mean of the stored values) and one step against the FP64 oracle on the
    same exact values, within the FP32 bounds."""
    say(f"two-array FP32 sigma={sigma} d={d} h={h} exchange={exchange}")
    u = si.table(sigma, d, h, seed=410, dtype=torch.float32, exchange=exchange)
    up = si.table(sigma, d, h, seed=411, dtype=torch.float32, exchange=exchange)
    offs = [2.5, 1.75]
    L = pk.Lcsb(sigma, d, h, "f32", iteration="two_array")
    L.load_ring([u.cuda(), up.cuda()], offsets=offs)
    u64 = u.numpy().astype(np.float64) + offs[0]
    up64 = up.numpy().astype(np.float64) + offs[1]
    R = L.rate()
    R_ref = oracle.sample_growth(sigma, d, h, u64, up64)
    assert abs(R - R_ref) <= 1e-12
    L.iterate(1)
    got, o_new = L.lag(1)
    val = o_new + _full(L, got).astype(np.float64)
    ref = oracle.two_array_step(sigma, d, h, u64, R)
    assert np.max(np.abs(val - ref)) <= _fp32_bound(8.0, (d - 1) * abs(R))
    assert _host(got)[0] == 0.0  # entry 0 is the reference entry


def test_fp32_two_array_polished_in_fp64_reaches_the_ring_bound(pk):
    """sigma = d = 2, l = 8: FP32 two-array sweeps from zero, then the ring
    converted to FP64 (in place, inside the FP64 buffers) and polished: the
    best largest-r certificate comes within 1e-9 of the ring's converged
    bound (the oracle's Algorithm 2 run)."""
    sigma, d, h = 2, 2, 8
    say("two-array FP32 + FP64 polish, l = 8")
    ring_best, _, _ = oracle.feasible_triplet(sigma, d, h, 200, 4)
    P = pk.Lcsb(sigma, d, h, "f64", iteration="two_array")
    S = pk.Lcsb(sigma, d, h, "f32", iteration="two_array",
                bufs=[b.view(torch.float32) for b in P.bufs])
    S.init_zero()
    S.run(cadence=8, max_sweeps=400, min_gain=2e-5, certificate="optimal")
    P.upcast(S)
    assert abs(P.rate() - S.rate()) <= 1e-6
    _, best, _, why = P.run(cadence=4, max_sweeps=400, target=ring_best["bound"] - 1e-9,
                            certificate="optimal")
    say(f"polished {best['bound']:.12f} ring {ring_best['bound']:.12f} ({why})")
    assert why == "target" and abs(best["bound"] - ring_best["bound"]) <= 1e-9


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_two_array_checkpoint_resume_is_bit_identical(pk, tmp_path, dt):
    sigma, d, h = 2, 3, 4
    say(f"two-array checkpoint {dt}")
    A = pk.Lcsb(sigma, d, h, dt, iteration="two_array")
    A.init_zero()
    A.iterate(13)
    A.certify_optimal()
    path = str(tmp_path / "two.ckpt")
    A.save(path)
    B = pk.Lcsb(sigma, d, h, dt, iteration="two_array")
    B.load(path)
    assert B.rate() == A.rate() and B.status() == A.status()
    A.iterate(9)
    B.iterate(9)
    assert torch.equal(A.lag(1)[0], B.lag(1)[0]) and A.lag(1)[1] == B.lag(1)[1]
    assert A.certify_optimal()[0] == B.certify_optimal()[0]
    R = pk.Lcsb(sigma, d, h, dt)  # a ring context refuses a two-array checkpoint
    with pytest.raises(pk.LcsbError):
        R.load(path)


def test_two_array_needs_fewer_sweeps_than_the_ring(pk):
    """sigma = d = 2, l = 10, FP64 from zero, certified every 2 sweeps with
    the largest-r certificate: sweeps to the ring's converged bound - 1e-9,
    two-array against ring (both bit-exact iterations; the count is what the
    two-array form buys)."""
    sigma, d, h = 2, 2, 10
    R = pk.Lcsb(sigma, d, h, "f64")
    R.init_zero()
    _, bestB, _, _ = R.run(cadence=2, max_sweeps=600, certificate="optimal")
    assert bestB["bound"] > 0.78
    target = bestB["bound"] - 1e-9
    counts = {}
    for it in ("ring", "two_array"):
        L = pk.Lcsb(sigma, d, h, "f64", iteration=it)
        L.init_zero()
        _, best, _, why = L.run(cadence=2, max_sweeps=2000, target=target, certificate="optimal")
        assert why == "target"
        counts[it] = best["sweep"]
    say(f"sweeps to B - 1e-9 at l = 10: {counts}")
    assert counts["two_array"] < counts["ring"]


@pytest.mark.timeout(600)
def test_fp64_two_array_h14_sampled_and_converged_bound(pk):
    """sigma = d = 2, l = 14 (2^28 indices, two FP64 tables of 1 GiB): one step
    from a seeded exchange-symmetric pair bit-exact at sampled coordinates,
    its rate bit-exact, then the iteration from zero to convergence reaches
    Table 2's 0.787017."""
    sigma, d, h = 2, 2, 14
    say("two-array l = 14: seeded step")
    u_dev = si.stored_table(sigma, d, h, seed=420, device="cuda")
    up_dev = si.stored_table(sigma, d, h, seed=421, device="cuda")
    L = pk.Lcsb(sigma, d, h, "f64", iteration="two_array")
    L.load_ring([u_dev, up_dev])
    assert L.swap_symmetric()
    n = L.n
    idx_all = torch.arange(n, dtype=torch.int64, device="cuda")
    u = _host(u_dev[si.representative(idx_all, sigma, d, h)])
    up = _host(up_dev[si.representative(idx_all, sigma, d, h)])
    del idx_all
    R = oracle.sample_growth(sigma, d, h, u, up)
    assert L.rate() == R
    L.iterate(1)
    idx = si.sample_indices(n, 20000, seed=13)
    got = L.lag(1)[0][si.representative(idx.cuda(), sigma, d, h)].cpu().numpy()
    ref = oracle.two_array_step_at(sigma, d, h, u, R, idx.numpy().astype(np.uint64))
    assert np.array_equal(got, ref)
    del L, u_dev, up_dev
    torch.cuda.empty_cache()
    say("two-array l = 14: from zero to convergence")
    L = pk.Lcsb(sigma, d, h, "f64", iteration="two_array")
    L.init_zero()
    cur, best, certs, why = L.run(cadence=8, max_sweeps=1600, stop_delta=1e-10,
                                  certificate="optimal")
    say(f"two-array l = 14: {best['bound']:.12f} after {cur['sweep']} sweeps ({why})")
    assert why == "converged"
    assert math.floor(best["bound"] * 1e6) / 1e6 == 0.787017


@pytest.mark.timeout(900)
@pytest.mark.parametrize("sigma,d,h", [(4, 2, 8), (2, 3, 10), (2, 2, 16)], ids=lambda v: str(v))
def test_fp64_two_array_full_size_seeded_step_sampled(pk, sigma, d, h):
    """The generality shapes and l = 16 at their full sizes (2^32, 2^30 and
    2^32 tuples), in the library's own launch shapes: one two-array step from
    a seeded exchange-symmetric pair, bit-exact with the oracle at 20000
    sampled coordinates (plus the head-class boundaries), and the rate that
    step used bit-exact."""
    n = sigma ** (d * h)
    torch.cuda.empty_cache()
    free, _ = torch.cuda.mem_get_info()
    need = 4 * 8 * n // sigma + 8 * 2**30  # the seeded pair and the context's two tables
    if free < need:
        pytest.skip(f"needs {need / 2**30:.0f} GiB of free device memory")
    tag = f"({sigma},{d},{h}) FP64 two-array"
    say(f"{tag}: seeded pair")
    u_dev = si.stored_table(sigma, d, h, seed=430, device="cuda")
    up_dev = si.stored_table(sigma, d, h, seed=431, device="cuda")
    L = pk.Lcsb(sigma, d, h, "f64", iteration="two_array")
    L.load_ring([u_dev, up_dev])
    assert L.swap_symmetric()
    rate = L.rate()
    L.iterate(1)
    idx = si.sample_indices(n, 20000, seed=17)
    got = L.lag(1)[0][si.representative(idx.cuda(), sigma, d, h)].cpu().numpy()
    del L
    torch.cuda.empty_cache()
    say(f"{tag}: full tables to the host")
    full = []
    for t in (u_dev, up_dev):
        out = np.empty(n, dtype=np.float64)
        for lo in range(0, n, 1 << 28):
            ii = torch.arange(lo, min(n, lo + (1 << 28)), dtype=torch.int64, device="cuda")
            out[lo:lo + ii.numel()] = t[si.representative(ii, sigma, d, h)].cpu().numpy()
            del ii
        full.append(out)
    del u_dev, up_dev
    torch.cuda.empty_cache()
    R = oracle.sample_growth(sigma, d, h, full[0], full[1])
    assert rate == R
    ref = oracle.two_array_step_at(sigma, d, h, full[0], R, idx.numpy().astype(np.uint64))
    assert np.array_equal(got, ref)


def _table3(sigma, d):
    import pathlib
    for line in (pathlib.Path(__file__).parent / "golden" / "table3_general_bounds.txt").read_text().splitlines():
        f = line.split()
        if f and not f[0].startswith("#") and (int(f[0]), int(f[1])) == (sigma, d):
            return int(f[2]), float(f[3])
    raise KeyError((sigma, d))


def _converge(pk, sigma, d, h, iteration):
    L = pk.Lcsb(sigma, d, h, "f64", iteration=iteration)
    L.init_zero()
    cur, best, _, why = L.run(16, max_sweeps=800, stop_delta=1e-10, certificate="optimal")
    assert why == "converged"
    del L
    torch.cuda.empty_cache()
    return best["bound"], cur["sweep"]


@pytest.mark.timeout(600)
@pytest.mark.parametrize("sigma,d,h", [(2, 3, 11), (4, 2, 9)], ids=lambda v: str(v))
def test_fp64_two_array_one_string_length_past_table3(pk, sigma, d, h):
    """One l past the l of Table 3's bound for (sigma, d) = (2, 3) and (4, 2),
    in FP64 on one GPU (two folded tables of 2^32 and 2^34 entries: 64 and
    256 GiB): the two-array iteration from zero, certified with the largest-r
    certificate every 16 sweeps to convergence, certifies a bound above
    Table 3's (0.711548 at l = 10 and 0.614333 at l = 8).  At (2, 3, 11) the
    ring of four tables (128 GiB) converges to the same bound within 1e-9."""
    l_paper, paper = _table3(sigma, d)
    assert h == l_paper + 1
    torch.cuda.empty_cache()
    free, _ = torch.cuda.mem_get_info()
    need = 2 * 8 * sigma ** (d * h) // sigma + 4 * 2**30
    if free < need:
        pytest.skip(f"needs {need / 2**30:.0f} GiB of free device memory")
    say(f"({sigma},{d},{h}) FP64 two-array to convergence")
    B, sweeps = _converge(pk, sigma, d, h, "two_array")
    say(f"({sigma},{d},{h}): {B:.12f} after {sweeps} sweeps (Table 3 at l = {l_paper}: {paper})")
    assert B > paper + 1e-3
    if (sigma, d) == (2, 3):
        Bring, _ = _converge(pk, sigma, d, h, "ring")
        assert abs(Bring - B) <= 1e-9


@pytest.mark.parametrize("dtype,iteration", [("f64", "ring"), ("f32", "ring"), ("f32", "two_array"),
                                             ("f64", "two_array_packed")], ids=lambda v: str(v))
def test_read_table_copies_the_lag_to_the_host(pk, dtype, iteration):
    """lcsb_read_table: the stored entries as stored, and as FP64 true values
    (an FP32 table widened and its offset added), equal to the device table."""
    L = pk.Lcsb(2, 2, 7, dtype, iteration=iteration)
    L.init_zero()
    L.iterate(9)
    for k in (1, 2):
        dev, off = L.lag(k)
        ref = dev.cpu().numpy()
        raw = L.read_table(k, as_f64=False)
        assert raw.dtype == ref.dtype and np.array_equal(raw, ref)
        true = L.read_table(k, as_f64=True)
        assert true.dtype == np.float64
        assert np.array_equal(true, off + ref.astype(np.float64))
