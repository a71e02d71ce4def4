"""The C-ABI library loads and exports what include/lcsb.h declares; host-only
argument checks.  No call here touches a GPU."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lcsb.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lcsb_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_2407_10925_amd import _capi
    if not os.path.exists(_capi.LIB_PATH):
        pytest.fail("liblcsb.so is not built (run python -m paper_2407_10925_amd.build)")
    return _capi.load()


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert len(names) >= 12
    for n in names:
        assert hasattr(lib, n), n


def test_create_validates_arguments(lib):
    from paper_2407_10925_amd import _capi
    ctx = C.c_void_p()
    assert lib.lcsb_create(3, 2, 2, 0, C.byref(ctx)) == _capi.LCSB_EUNSUPPORTED
    assert lib.lcsb_create(2, 4, 2, 0, C.byref(ctx)) == _capi.LCSB_EUNSUPPORTED
    assert lib.lcsb_create(2, 2, 0, 0, C.byref(ctx)) == _capi.LCSB_EINVAL
    assert lib.lcsb_create(2, 2, 19, 0, C.byref(ctx)) == _capi.LCSB_EINVAL  # 2^38 > 2^36
    assert lib.lcsb_create(2, 2, 6, 7, C.byref(ctx)) == _capi.LCSB_EINVAL
    assert b"dtype" in lib.lcsb_last_error()
    assert lib.lcsb_create(2, 2, 6, 0, None) == _capi.LCSB_EINVAL
    assert lib.lcsb_create_iter(2, 2, 6, 0, 3, C.byref(ctx)) == _capi.LCSB_EINVAL
    assert b"iteration" in lib.lcsb_last_error()
    for d, iteration, nbuf in ((2, 0, 3), (3, 0, 4), (2, 1, 2), (3, 1, 2)):
        assert lib.lcsb_create_iter(2, d, 3, 0, iteration, C.byref(ctx)) == 0
        nb = C.c_int()
        assert lib.lcsb_query(ctx, C.byref(nb), None, None, None) == 0
        assert nb.value == nbuf
        rate = C.c_double()
        assert lib.lcsb_rate(ctx, C.byref(rate)) == _capi.LCSB_ESTATE  # not initialised
        assert lib.lcsb_destroy(ctx) == 0
    # packed tables: sigma = d = 2, l >= 2 only; one entry per exchange orbit
    for sigma, d, h in ((4, 2, 3), (2, 3, 3), (2, 2, 1)):
        assert lib.lcsb_create_iter(sigma, d, h, 0, 2, C.byref(ctx)) == _capi.LCSB_EUNSUPPORTED
    for h, dtype in ((2, 0), (3, 1), (18, 0)):
        assert lib.lcsb_create_iter(2, 2, h, dtype, 2, C.byref(ctx)) == 0
        nb, ent, bpb = C.c_int(), C.c_uint64(), C.c_uint64()
        assert lib.lcsb_query(ctx, C.byref(nb), C.byref(ent), C.byref(bpb), None) == 0
        assert (nb.value, ent.value) == (2, 4 ** (h - 1) + 2 ** h)
        assert bpb.value == ent.value * (8 if dtype == 0 else 4)
        assert lib.lcsb_destroy(ctx) == 0


@pytest.mark.parametrize("sigma,d,h,dtype,n,elem", [(2, 2, 6, 0, 4096, 8), (2, 2, 16, 1, 2**32, 4),
                                                    (4, 2, 8, 1, 2**32, 4), (2, 3, 10, 1, 2**30, 4),
                                                    (2, 2, 17, 1, 2**34, 4)])
def test_query_sizes(lib, sigma, d, h, dtype, n, elem):
    ctx = C.c_void_p()
    assert lib.lcsb_create(sigma, d, h, dtype, C.byref(ctx)) == 0
    nbuf, ent, bpb, ws = C.c_int(), C.c_uint64(), C.c_uint64(), C.c_uint64()
    assert lib.lcsb_query(ctx, C.byref(nbuf), C.byref(ent), C.byref(bpb), C.byref(ws)) == 0
    # tables are folded: the n / sigma indices whose string-1 head is 0
    assert (nbuf.value, ent.value, bpb.value) == (d + 1, n // sigma, n // sigma * elem)
    assert ws.value > 0 and ws.value % 256 == 0
    assert lib.lcsb_destroy(ctx) == 0


def test_call_order_is_enforced_without_a_gpu(lib):
    from paper_2407_10925_amd import _capi
    ctx = C.c_void_p()
    assert lib.lcsb_create(2, 2, 4, 0, C.byref(ctx)) == 0
    assert lib.lcsb_iterate(ctx, 1) == _capi.LCSB_ESTATE
    assert lib.lcsb_certify(ctx, None, None) == _capi.LCSB_ESTATE
    assert lib.lcsb_certify_optimal(ctx, None, None) == _capi.LCSB_ESTATE
    assert lib.lcsb_read_table(ctx, 1, None, 1) == _capi.LCSB_ESTATE
    assert lib.lcsb_init_zero(ctx) == _capi.LCSB_ESTATE
    # bind checks pointers before storing anything
    assert lib.lcsb_bind(ctx, None, 3, None, None) == _capi.LCSB_EINVAL
    bufs = (C.c_void_p * 3)(256, 512, 256)  # aliasing, never dereferenced
    assert lib.lcsb_bind(ctx, bufs, 3, C.c_void_p(1024), None) == _capi.LCSB_EINVAL
    bufs = (C.c_void_p * 3)(256, 512, 768)
    assert lib.lcsb_bind(ctx, bufs, 3, C.c_void_p(1000), None) == _capi.LCSB_EINVAL  # misaligned ws
    assert lib.lcsb_bind(ctx, bufs, 2, C.c_void_p(1024), None) == _capi.LCSB_EINVAL
    assert lib.lcsb_destroy(ctx) == 0
    assert lib.lcsb_destroy(None) == 0


def test_branch_mean_buffers_are_checked_without_a_gpu(lib):
    """lcsb_query_means / lcsb_bind_means: sizes for sigma = d = 2 folded
    tables (Ma, n/4 entries, then Mab, n/8, then the 4096 sample values of the
    two-array rate, each at a 256-byte boundary) and for the sigma = 2, d = 3
    and sigma = 4, d = 2 rings, the two-array pairs of every such shape,
    refusals for packed tables, l < 3 and other shapes,
    and pointer checks before anything is stored (no buffer is dereferenced)."""
    from paper_2407_10925_amd import _capi
    mb = C.c_uint64()
    for (sigma, d, h, it) in ((2, 3, 2, 1), (4, 2, 2, 1), (4, 2, 2, 0), (2, 2, 2, 0), (2, 3, 2, 0), (2, 2, 5, 2)):
        ctx = C.c_void_p()
        assert lib.lcsb_create_iter(sigma, d, h, 0, it, C.byref(ctx)) == 0
        assert lib.lcsb_query_means(ctx, C.byref(mb)) == _capi.LCSB_EUNSUPPORTED, (sigma, d, h, it)
        assert lib.lcsb_destroy(ctx) == 0
    for dtype, elem in ((0, 8), (1, 4)):
        ctx = C.c_void_p()
        assert lib.lcsb_create(2, 2, 5, dtype, C.byref(ctx)) == 0
        n = 4 ** 5
        assert lib.lcsb_query_means(ctx, C.byref(mb)) == 0

        def up(b):
            return (b + 255) // 256 * 256
        assert mb.value == up(up((n // 4) * elem) + (n // 8) * elem) + 4096 * elem
        means = (C.c_void_p * 3)(4096, 8192, 12288)
        assert lib.lcsb_bind_means(ctx, means, 3) == _capi.LCSB_ESTATE  # before lcsb_bind
        bufs = (C.c_void_p * 3)(256, 512, 768)
        assert lib.lcsb_bind(ctx, bufs, 3, C.c_void_p(1024), None) == 0
        assert lib.lcsb_bind_means(ctx, means, 2) == _capi.LCSB_EINVAL
        assert lib.lcsb_bind_means(ctx, (C.c_void_p * 3)(4096, 8200, 12288), 3) == _capi.LCSB_EINVAL
        assert lib.lcsb_bind_means(ctx, (C.c_void_p * 3)(4096, 512, 12288), 3) == _capi.LCSB_EINVAL
        assert lib.lcsb_bind_means(ctx, (C.c_void_p * 3)(4096, 4096, 12288), 3) == _capi.LCSB_EINVAL
        assert lib.lcsb_bind_means(ctx, (C.c_void_p * 3)(4096, 1024, 12288), 3) == _capi.LCSB_EINVAL
        assert lib.lcsb_bind_means(ctx, means, 3) == 0
        assert lib.lcsb_bind_means(ctx, None, 0) == 0  # unbind
        assert lib.lcsb_destroy(ctx) == 0
    for sigma, d, h in ((2, 2, 5), (4, 2, 3), (2, 3, 4)):  # the two-array pairs take them too
        ctx = C.c_void_p()
        assert lib.lcsb_create_iter(sigma, d, h, 0, 1, C.byref(ctx)) == 0
        assert lib.lcsb_query_means(ctx, C.byref(mb)) == 0
        assert lib.lcsb_destroy(ctx) == 0
    # sigma = 2, d = 3 ring: M1, M3 (n/4 each), M12, M23 (n/8), M123 (n/16), the sample
    for dtype, elem in ((0, 8), (1, 4)):
        ctx = C.c_void_p()
        assert lib.lcsb_create(2, 3, 4, dtype, C.byref(ctx)) == 0
        assert lib.lcsb_query_means(ctx, C.byref(mb)) == 0
        n, at = 8 ** 4, 0
        for part in (n // 4, n // 4, n // 8, n // 8, n // 16):
            at = (at + part * elem + 255) // 256 * 256
        assert mb.value == at + 4096 * elem
        assert lib.lcsb_destroy(ctx) == 0
    # sigma = 4, d = 2 ring: M4a (n/16 entries), M4ab (n/64), the sample
    for dtype, elem in ((0, 8), (1, 4)):
        ctx = C.c_void_p()
        assert lib.lcsb_create(4, 2, 3, dtype, C.byref(ctx)) == 0
        assert lib.lcsb_query_means(ctx, C.byref(mb)) == 0
        n, at = 16 ** 3, 0
        for part in (n // 16, n // 64):
            at = (at + part * elem + 255) // 256 * 256
        assert mb.value == at + 4096 * elem
        assert lib.lcsb_destroy(ctx) == 0


def test_python_binding_refuses_without_gpu():
    import torch
    import paper_2407_10925_amd as pk
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(RuntimeError):
        pk.Lcsb(2, 2, 4)


def test_build_rejects_kernels_that_spill():
    """The build parses hipcc's resource-usage remarks and names every kernel
    with scratch memory (the forward kernel's weight ring counts its own
    outstanding loads and would miscount compiler-issued spill traffic)."""
    from paper_2407_10925_amd import build as B
    remarks = "\n".join([
        "x.hip:1:1: remark: Function Name: _Z4goodv [-Rpass-analysis=kernel-resource-usage]",
        "x.hip:1:1: remark:     VGPRs: 12 [-Rpass-analysis=kernel-resource-usage]",
        "x.hip:1:1: remark:     ScratchSize [bytes/lane]: 0 [-Rpass-analysis=kernel-resource-usage]",
        "x.hip:9:1: remark: Function Name: _Z5spillv [-Rpass-analysis=kernel-resource-usage]",
        "x.hip:9:1: remark:     ScratchSize [bytes/lane]: 28 [-Rpass-analysis=kernel-resource-usage]",
    ])
    assert B.scratch_users(remarks) == [("_Z5spillv", 28)]
    assert B.scratch_users("") == []


# ------------------------------------------------------------------ checkpoint files
_HDR = "<8sIiiiiiQqdddddqQQq3d3QQ"  # the checkpoint header of include/lcsb.h's lcsb_save


def _hash64(data: bytes) -> int:
    """The header/table hash: 8-byte little-endian words, zero-padded tail."""
    h, m = 0x243F6A8885A308D3, (1 << 64) - 1
    for i in range(0, len(data), 8):
        w = int.from_bytes(data[i:i + 8].ljust(8, b"\0"), "little")
        h = ((h ^ w) * 0x9E3779B97F4A7C15) & m
        h ^= h >> 29
    return h


def _header(sigma, d, h, dtype, stored, iteration=0, version=2):
    import struct
    body = struct.pack(_HDR[:-1], b"LCSBRING", version, sigma, d, h, dtype, iteration, stored, 5,
                       0.5, 0.25, 0.0, -1.0, 0.25, 4, 0, 0, 0, 0.0, 0.0, 0.0, 1, 2, 3)
    return body + struct.pack("<Q", _hash64(body))


def test_checkpoint_header_is_checked_before_the_ring_is_touched(lib, tmp_path):
    """Every refusal here happens before any device access (the ring pointers
    are not device memory: this runs without a GPU)."""
    import struct
    from paper_2407_10925_amd import _capi
    assert struct.calcsize(_HDR) == 176
    ctx = C.c_void_p()
    assert lib.lcsb_create(2, 2, 4, 0, C.byref(ctx)) == 0
    assert lib.lcsb_load(ctx, str(tmp_path / "x").encode()) == _capi.LCSB_ESTATE  # not bound
    bufs = (C.c_void_p * 3)(256, 512, 768)
    assert lib.lcsb_bind(ctx, bufs, 3, C.c_void_p(1024), None) == 0
    assert lib.lcsb_save(ctx, str(tmp_path / "x").encode()) == _capi.LCSB_ESTATE  # no ring yet
    assert lib.lcsb_load(ctx, None) == _capi.LCSB_EINVAL
    assert lib.lcsb_load(ctx, str(tmp_path / "missing").encode()) == _capi.LCSB_ECKPT
    stored, tbytes = 4 ** 4 // 2, 8 * 4 ** 4 // 2
    good = _header(2, 2, 4, 0, stored)
    cases = {
        "short": good[:100],
        "magic": b"LCSBRINX" + good[8:],
        "hash": good[:40] + b"\x07" + good[41:],
        "shape": _header(2, 2, 5, 0, 4 ** 5 // 2) + bytes(2 * 8 * 4 ** 5 // 2),
        "dtype": _header(2, 2, 4, 1, stored) + bytes(2 * 4 * stored),
        "iteration": _header(2, 2, 4, 0, stored, iteration=1) + bytes(2 * tbytes),
        "version": _header(2, 2, 4, 0, stored, version=1) + bytes(2 * tbytes),
        "truncated": good + bytes(2 * tbytes - 8),
        "too long": good + bytes(2 * tbytes + 8),
    }
    for name, blob in cases.items():
        p = tmp_path / name
        p.write_bytes(blob)
        assert lib.lcsb_load(ctx, str(p).encode()) == _capi.LCSB_ECKPT, name
        assert b"checkpoint" in lib.lcsb_last_error() or str(p).encode() in lib.lcsb_last_error()
    assert lib.lcsb_iterate(ctx, 1) == _capi.LCSB_ESTATE  # still not initialised
    assert lib.lcsb_destroy(ctx) == 0
