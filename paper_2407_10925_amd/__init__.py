"""gfx950 implementation of the lower-bound iteration of arXiv 2407.10925.

The computation lives in ``liblcsb.so`` (HIP kernels behind the C ABI of
``include/lcsb.h``).  This module only allocates the ring and workspace as
PyTorch device tensors, passes their addresses and the current HIP stream,
and converts results; it computes nothing itself.  Importing it does not
need a GPU; constructing :class:`Lcsb` does, and raises if the library has
not been built.
"""
from __future__ import annotations

import ctypes as C

from . import _capi
from ._capi import (LCSB_F32, LCSB_F64, Cert, LcsbError, check)

__all__ = ["Lcsb", "LcsbError", "LCSB_F32", "LCSB_F64", "create"]

_DTYPES = {"f64": LCSB_F64, "f32": LCSB_F32}


class Lcsb:
    """One ring of d+1 tables for (sigma, d, h) on one GPU.

    Methods mirror the C entry points: init_zero, load_ring, iterate,
    certify, lag, status, upcast, destroy.
    """

    def __init__(self, sigma: int, d: int, h: int, dtype: str = "f64", device=None):
        import torch

        if dtype not in _DTYPES:
            raise ValueError(f"dtype must be one of {list(_DTYPES)}")
        if not torch.cuda.is_available():
            raise RuntimeError("Lcsb needs a HIP device (torch.cuda.is_available() is False)")
        lib = _capi.load()
        self.sigma, self.d, self.h, self.dtype = sigma, d, h, dtype
        self.device = torch.device(device if device is not None else "cuda")
        if self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        self._lib = lib
        ctx = C.c_void_p()
        check(lib.lcsb_create(sigma, d, h, _DTYPES[dtype], C.byref(ctx)))
        self._ctx = ctx
        nbuf, n, bpb, wsb = C.c_int(), C.c_uint64(), C.c_uint64(), C.c_uint64()
        check(lib.lcsb_query(ctx, C.byref(nbuf), C.byref(n), C.byref(bpb), C.byref(wsb)))
        self.nbuf, self.n = nbuf.value, n.value
        tdt = torch.float64 if dtype == "f64" else torch.float32
        self.torch_dtype = tdt
        self.bufs = [torch.empty(self.n, dtype=tdt, device=self.device) for _ in range(self.nbuf)]
        self.ws = torch.empty(wsb.value, dtype=torch.uint8, device=self.device)
        self.stream = torch.cuda.current_stream(self.device)
        ptrs = (C.c_void_p * self.nbuf)(*[b.data_ptr() for b in self.bufs])
        check(lib.lcsb_bind(ctx, ptrs, self.nbuf, C.c_void_p(self.ws.data_ptr()),
                            C.c_void_p(self.stream.cuda_stream)))

    # ------------------------------------------------------------------ C calls
    def init_zero(self):
        check(self._lib.lcsb_init_zero(self._ctx))

    def load_ring(self, tables, offsets=None):
        """tables[k-1] = lag k, device tensors of the ring's dtype and size."""
        if len(tables) != self.d:
            raise ValueError(f"need {self.d} tables")
        for t in tables:
            if t.dtype != self.torch_dtype or t.numel() != self.n or not t.is_contiguous() \
                    or t.device != self.device:
                raise ValueError("table dtype, size, layout or device does not match the ring")
        self._keep = list(tables)
        ptrs = (C.c_void_p * self.d)(*[t.data_ptr() for t in tables])
        offs = None
        if offsets is not None:
            offs = (C.c_double * self.d)(*[float(o) for o in offsets])
        check(self._lib.lcsb_load_ring(self._ctx, ptrs, self.d, offs))

    def iterate(self, k: int = 1):
        check(self._lib.lcsb_iterate(self._ctx, int(k)))

    def certify(self, allow_nonfinite: bool = False):
        """Returns (current, best) certificates as dicts (synchronises)."""
        cur, best = Cert(), Cert()
        rc = self._lib.lcsb_certify(self._ctx, C.byref(cur), C.byref(best))
        if rc != 0 and not (allow_nonfinite and rc == _capi.LCSB_ENONFINITE):
            check(rc)
        return cur.as_dict(), best.as_dict()

    def lag(self, k: int = 1):
        """(tensor aliasing lag k, its FP64 offset).  Valid until the next sweep."""
        p, off = C.c_void_p(), C.c_double()
        check(self._lib.lcsb_lag(self._ctx, k, C.byref(p), C.byref(off)))
        for b in self.bufs:
            if b.data_ptr() == p.value:
                return b, off.value
        raise RuntimeError("lag pointer does not match a ring buffer")

    def status(self):
        s, best = C.c_int64(), Cert()
        check(self._lib.lcsb_status(self._ctx, C.byref(s), C.byref(best)))
        return s.value, best.as_dict()

    def upcast(self, src: "Lcsb"):
        """Fill this FP64 ring from the FP32 ring ``src`` (FP64 polish)."""
        check(self._lib.lcsb_upcast(src._ctx, self._ctx))

    def destroy(self):
        if getattr(self, "_ctx", None) is not None and self._ctx.value:
            self._lib.lcsb_destroy(self._ctx)
            self._ctx = C.c_void_p()

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def create(sigma: int, d: int, h: int, dtype: str = "f64", device=None) -> Lcsb:
    return Lcsb(sigma, d, h, dtype, device)
