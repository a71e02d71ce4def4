"""The allocation-free certificate (lcsb_certify_optimal_noalloc, called
through the C ABI) against the context-based lcsb_certify_optimal on the same
tables: r, bound, lowest minimising index and non-finite count bit for bit.
Two calls in a row, the second on a smaller table, share the static scratch;
each must match."""
import ctypes as C
import sys

import numpy as np
import pytest
import torch

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


def _noalloc(pk, sigma, d, h, dt, table, exchange):
    from paper_2407_10925_amd import _capi
    lib = _capi.load()
    out = torch.full((4,), float("nan"), dtype=torch.float64, device="cuda")
    code = _capi.LCSB_F64 if dt == "f64" else _capi.LCSB_F32
    stream = torch.cuda.current_stream().cuda_stream
    _capi.check(lib.lcsb_certify_optimal_noalloc(sigma, d, h, code, C.c_void_p(table.data_ptr()),
                                                  int(exchange), C.c_void_p(out.data_ptr()),
                                                  C.c_void_p(stream)))
    torch.cuda.synchronize()
    o = out.cpu()
    ints = o.view(torch.int64)
    return {"r": o[0].item(), "bound": o[1].item(), "arg": int(ints[2]), "nonfinite": int(ints[3])}


def _context(pk, sigma, d, h, dt, table):
    L = pk.Lcsb(sigma, d, h, dt)
    L.load_ring([table] * d)
    cur, _ = L.certify_optimal(allow_nonfinite=True)
    return {"r": cur["R"], "bound": cur["bound"], "arg": cur["argmax_W"],
            "nonfinite": cur["nonfinite"]}, L.swap_symmetric()


def _table(sigma, d, h, dt, seed, exchange):
    tdt = torch.float64 if dt == "f64" else torch.float32
    return si.table(sigma, d, h, seed=seed, dtype=tdt, exchange=exchange)[: sigma ** (d * h) // sigma].cuda()


@pytest.mark.parametrize("sigma,d,dt,exchange", [(2, 2, "f64", True), (2, 2, "f32", False),
                                                 (4, 2, "f32", True), (2, 3, "f64", True),
                                                 (2, 3, "f32", False)], ids=lambda v: str(v))
def test_noalloc_matches_the_context_certificate_twice(pk, sigma, d, dt, exchange):
    big, small = {(2, 2): (9, 4), (4, 2): (4, 2), (2, 3): (6, 3)}[(sigma, d)]
    for h in (big, small):  # the second call is on a smaller table, in the same scratch
        say(f"noalloc certificate sigma={sigma} d={d} l={h} {dt} exchange={exchange}")
        t = _table(sigma, d, h, dt, seed=500 + h, exchange=exchange)
        ref, sym = _context(pk, sigma, d, h, dt, t)
        assert sym == exchange
        got = _noalloc(pk, sigma, d, h, dt, t, exchange)
        assert got == ref, (got, ref)
        if exchange:  # reading every entry gives the same bits
            assert _noalloc(pk, sigma, d, h, dt, t, False) == ref


def test_noalloc_rejects_bad_arguments(pk):
    from paper_2407_10925_amd import _capi
    lib = _capi.load()
    out = torch.zeros(4, dtype=torch.float64, device="cuda")
    t = torch.zeros(4 ** 4, dtype=torch.float64, device="cuda")
    o, tp = C.c_void_p(out.data_ptr()), C.c_void_p(t.data_ptr())
    assert lib.lcsb_certify_optimal_noalloc(2, 2, 19, 0, tp, 0, o, None) == _capi.LCSB_EINVAL
    assert lib.lcsb_certify_optimal_noalloc(3, 2, 4, 0, tp, 0, o, None) == _capi.LCSB_EUNSUPPORTED
    assert lib.lcsb_certify_optimal_noalloc(2, 2, 4, 0, None, 0, o, None) == _capi.LCSB_EINVAL
    assert lib.lcsb_certify_optimal_noalloc(2, 2, 4, 0, C.c_void_p(t.data_ptr() + 8), 0, o,
                                            None) == _capi.LCSB_EINVAL
    assert b"aligned" in lib.lcsb_last_error()
