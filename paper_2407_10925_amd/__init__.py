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

__all__ = ["Lcsb", "Mlp", "LcsbError", "LCSB_F32", "LCSB_F64", "create"]

_DTYPES = {"f64": LCSB_F64, "f32": LCSB_F32}


class Lcsb:
    """One ring of d+1 tables for (sigma, d, h) on one GPU.

    ``n`` = sigma^(d h) is the number of table indices; every table stores the
    ``stored`` = n / sigma lowest ones (string-1 head 0), the others being
    equal to their image under the symbol relabelling.  Methods mirror the C
    entry points: init_zero, load_ring, iterate, certify, run, lag, status,
    upcast, save, load, swap_symmetric, destroy.
    """

    def __init__(self, sigma: int, d: int, h: int, dtype: str = "f64", device=None,
                 bufs=None, iteration: str = "ring", means: bool = False):
        """``bufs``: optional ring buffers to bind instead of allocating, d + 1
        (2 for the two-array iteration) contiguous device tensors of at least
        the ring's bytes each (for an FP32 ring inside an FP64 ring's memory,
        ``[b.view(torch.float32) for b in P.bufs]``; see :meth:`upcast`).
        ``iteration``: "ring" (Algorithm 2), "two_array" or "two_array_packed"
        (lcsb_create_iter; packed tables hold ``stored`` = packed_entries
        entries, one per exchange orbit).  ``means``: allocate and bind the
        branch-mean buffers (lcsb_bind_means; folded tables of h >= 3, rings and
        two-array pairs: sigma = 2 with d = 2 or 3, sigma = 4 with d = 2)."""
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
        self.iteration = iteration
        check(lib.lcsb_create_iter(sigma, d, h, _DTYPES[dtype], _capi.ITERATIONS[iteration],
                                   C.byref(ctx)))
        self.lags = d if iteration == "ring" else 2
        self._ctx = ctx
        nbuf, n, bpb, wsb = C.c_int(), C.c_uint64(), C.c_uint64(), C.c_uint64()
        check(lib.lcsb_query(ctx, C.byref(nbuf), C.byref(n), C.byref(bpb), C.byref(wsb)))
        self.nbuf, self.stored = nbuf.value, n.value
        self.n = sigma ** (d * h)
        tdt = torch.float64 if dtype == "f64" else torch.float32
        self.torch_dtype = tdt
        if bufs is None:
            self.bufs = [torch.empty(self.stored, dtype=tdt, device=self.device)
                         for _ in range(self.nbuf)]
        else:
            if len(bufs) != self.nbuf or any(
                    b.dtype != tdt or b.numel() < self.stored or not b.is_contiguous()
                    or b.device != self.device for b in bufs):
                raise ValueError(f"need {self.nbuf} contiguous {tdt} device buffers of at least "
                                 f"{self.stored} elements")
            self.bufs = [b[:self.stored] for b in bufs]
        self.ws = torch.empty(wsb.value, dtype=torch.uint8, device=self.device)
        self.stream = torch.cuda.current_stream(self.device)
        ptrs = (C.c_void_p * self.nbuf)(*[b.data_ptr() for b in self.bufs])
        check(lib.lcsb_bind(ctx, ptrs, self.nbuf, C.c_void_p(self.ws.data_ptr()),
                            C.c_void_p(self.stream.cuda_stream)))
        self.means = []
        if means:
            mb = C.c_uint64()
            check(lib.lcsb_query_means(ctx, C.byref(mb)))
            self.means = [torch.empty(mb.value, dtype=torch.uint8, device=self.device)
                          for _ in range(self.nbuf)]
            mptrs = (C.c_void_p * self.nbuf)(*[b.data_ptr() for b in self.means])
            check(lib.lcsb_bind_means(ctx, mptrs, self.nbuf))

    # ------------------------------------------------------------------ C calls
    def init_zero(self):
        check(self._lib.lcsb_init_zero(self._ctx))

    def load_ring(self, tables, offsets=None):
        """tables[k-1] = lag k: device tensors of the ring's dtype holding all n
        indices or only the stored ones (the first ``stored`` values are used)."""
        if len(tables) != self.lags:
            raise ValueError(f"need {self.lags} tables")
        for t in tables:
            if t.dtype != self.torch_dtype or t.numel() not in (self.n, self.stored) \
                    or not t.is_contiguous() or t.device != self.device:
                raise ValueError("table dtype, size, layout or device does not match the ring")
        self._keep = list(tables)
        ptrs = (C.c_void_p * self.lags)(*[t.data_ptr() for t in tables])
        offs = None
        if offsets is not None:
            offs = (C.c_double * self.lags)(*[float(o) for o in offsets])
        check(self._lib.lcsb_load_ring(self._ctx, ptrs, self.lags, offs))

    def iterate(self, k: int = 1):
        check(self._lib.lcsb_iterate(self._ctx, int(k)))

    def certify(self, allow_nonfinite: bool = False):
        """Returns (current, best) certificates as dicts (synchronises)."""
        cur, best = Cert(), Cert()
        rc = self._lib.lcsb_certify(self._ctx, C.byref(cur), C.byref(best))
        if rc != 0 and not (allow_nonfinite and rc == _capi.LCSB_ENONFINITE):
            check(rc)
        return cur.as_dict(), best.as_dict()

    def certify_optimal(self, allow_nonfinite: bool = False):
        """lcsb_certify_optimal: the largest r with (u, r, 0) a feasible
        triplet for the newest table u.  Returns (current, best) as dicts
        (synchronises)."""
        cur, best = Cert(), Cert()
        rc = self._lib.lcsb_certify_optimal(self._ctx, C.byref(cur), C.byref(best))
        if rc != 0 and not (allow_nonfinite and rc == _capi.LCSB_ENONFINITE):
            check(rc)
        return cur.as_dict(), best.as_dict()

    def run(self, cadence: int, first: int = 0, max_sweeps: int = 1 << 40,
            target: float = float("nan"), stop_delta: float = 0.0, min_gain: float = 0.0,
            certificate: str = "feasible", log: str = None):
        """lcsb_run: sweep and certify every `cadence` sweeps (the first
        certificate after `first`) until the best bound reaches `target`,
        consecutive certificates move by less than `stop_delta`, a positive
        best bound gains less than `min_gain` in a period, or `max_sweeps`.
        `certificate`: "feasible" (Algorithm 2, lcsb_certify) or "optimal"
        (lcsb_certify_optimal).  `log`: a file that gets one JSON line per
        certificate.  Returns (current, best, certificates, reason)."""
        pol = _capi.RunPolicy(int(cadence), int(first), int(max_sweeps), float(target),
                              float(stop_delta), float(min_gain),
                              _capi.CERT_KINDS[certificate],
                              None if log is None else str(log).encode())
        cur, best, certs, why = Cert(), Cert(), C.c_int64(), C.c_int()
        check(self._lib.lcsb_run(self._ctx, C.byref(pol), C.byref(cur), C.byref(best),
                                 C.byref(certs), C.byref(why)))
        return cur.as_dict(), best.as_dict(), certs.value, _capi.LCSB_STOP_NAMES[why.value]

    def lag(self, k: int = 1):
        """(tensor aliasing the stored entries of lag k, its FP64 offset).
        Valid until the next sweep."""
        p, off = C.c_void_p(), C.c_double()
        check(self._lib.lcsb_lag(self._ctx, k, C.byref(p), C.byref(off)))
        for b in self.bufs:
            if b.data_ptr() == p.value:
                return b, off.value
        raise RuntimeError("lag pointer does not match a ring buffer")

    def read_table(self, k: int = 1, as_f64: bool = True):
        """lcsb_read_table: lag k's stored entries copied to a host numpy array,
        as FP64 true values (FP32 tables widened, offset added) or as stored."""
        import numpy as np
        dt = np.float64 if (as_f64 or self.dtype == "f64") else np.float32
        out = np.empty(self.stored, dtype=dt)
        check(self._lib.lcsb_read_table(self._ctx, int(k), C.c_void_p(out.ctypes.data),
                                        1 if as_f64 else 0))
        return out

    def rate(self) -> float:
        """The rate R the next two-array sweep uses (synchronises)."""
        r = C.c_double()
        check(self._lib.lcsb_rate(self._ctx, C.byref(r)))
        return r.value

    def status(self):
        s, best = C.c_int64(), Cert()
        check(self._lib.lcsb_status(self._ctx, C.byref(s), C.byref(best)))
        return s.value, best.as_dict()

    def swap_symmetric(self) -> bool:
        """Whether the ring is known to be symmetric in strings 1 and 2
        (sigma = 2, d = 2 or 3): sweeps and certificates then move half the
        bytes."""
        v = C.c_int()
        check(self._lib.lcsb_swap_symmetric(self._ctx, C.byref(v)))
        return bool(v.value)

    def init_seed_mlp(self, mlp: "Mlp", rate: float):
        """Fill the ring from the warm-start network: lag 2 = u, lag 1 = u + rate."""
        check(self._lib.lcsb_init_seed_mlp(self._ctx, C.c_void_p(mlp.params.data_ptr()),
                                           C.c_void_p(mlp.wbf16.data_ptr()), float(rate)))

    def save(self, path: str):
        """Checkpoint the ring, its offsets, sweep count and best certificate."""
        check(self._lib.lcsb_save(self._ctx, str(path).encode()))

    def load(self, path: str):
        """Restore a checkpoint written by :meth:`save` for the same shape."""
        check(self._lib.lcsb_load(self._ctx, str(path).encode()))

    def upcast(self, src: "Lcsb"):
        """Fill this FP64 ring from the FP32 ring ``src`` (FP64 polish); in place
        when ``src`` was bound to this ring's buffers."""
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


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


class Mlp:
    """Warm-start network state on one device: FP32 master parameters, their
    BF16 copy, Adam moments and a training workspace for one batch size.
    Methods mirror the lcsb_mlp_* entry points."""

    def __init__(self, device=None, seed: int = 2407, batch: int = 8192):
        import torch
        self._lib = _capi.load()
        self.device = torch.device(device if device is not None else "cuda")
        n = _capi.LCSB_MLP_NPARAMS
        self.params = torch.empty(n, dtype=torch.float32, device=self.device)
        self.wbf16 = torch.empty(n, dtype=torch.int16, device=self.device)
        self.m = torch.zeros(n, dtype=torch.float32, device=self.device)
        self.v = torch.zeros(n, dtype=torch.float32, device=self.device)
        self.grad = torch.zeros(n, dtype=torch.float32, device=self.device)
        self.t = 0
        self.stream = torch.cuda.current_stream(self.device)
        check(self._lib.lcsb_mlp_init(_ptr(self.params), seed, self._s()))
        self.to_bf16()
        self.set_batch(batch)

    def _s(self):
        return C.c_void_p(self.stream.cuda_stream)

    def set_batch(self, batch: int):
        import torch
        b = C.c_uint64()
        check(self._lib.lcsb_mlp_workspace(batch, C.byref(b)))
        self.batch = batch
        self.ws = torch.empty(b.value, dtype=torch.uint8, device=self.device)
        self.idx = torch.empty(batch, dtype=torch.int64, device=self.device)
        self.target = torch.empty(batch, dtype=torch.float32, device=self.device)
        self.y = torch.empty(batch, dtype=torch.float32, device=self.device)
        self.dy = torch.empty(batch, dtype=torch.float32, device=self.device)
        self.loss_dev = torch.zeros(1, dtype=torch.float64, device=self.device)

    def load(self, params):
        """Copy FP32 parameters in (device tensor) and refresh the BF16 copy."""
        self.params.copy_(params)
        self.to_bf16()

    def to_bf16(self):
        check(self._lib.lcsb_mlp_to_bf16(_ptr(self.params), _ptr(self.wbf16), self._s()))

    def sample(self, table, h: int, seed: int):
        dt = LCSB_F32 if table.dtype == _torch_f32() else LCSB_F64
        check(self._lib.lcsb_mlp_sample(_ptr(table), dt, h, seed, self.batch, _ptr(self.idx),
                                        _ptr(self.target), self._s()))

    def forward(self, idx, h: int, y, keep: bool = False):
        check(self._lib.lcsb_mlp_forward(_ptr(self.params), _ptr(self.wbf16), _ptr(idx), h,
                                         idx.numel(), _ptr(self.ws) if keep else None, _ptr(y),
                                         self._s()))

    def loss(self, y, target, dy):
        check(self._lib.lcsb_mlp_loss(_ptr(y), _ptr(target), y.numel(), _ptr(dy),
                                      _ptr(self.loss_dev), self._s()))

    def backward(self, idx, h: int, dy):
        check(self._lib.lcsb_mlp_backward(_ptr(self.wbf16), _ptr(idx), h, _ptr(dy), idx.numel(),
                                          _ptr(self.ws), _ptr(self.grad), self._s()))

    def adam(self, lr: float, beta1=0.9, beta2=0.999, eps=1e-8):
        self.t += 1
        check(self._lib.lcsb_mlp_adam(_ptr(self.params), _ptr(self.wbf16), _ptr(self.grad),
                                      _ptr(self.m), _ptr(self.v), lr, beta1, beta2, eps, self.t,
                                      self._s()))

    def train_step(self, table, h: int, seed: int, lr: float):
        """Sample a batch from `table`, one forward/backward/Adam step; the
        batch loss stays on the device (self.loss_dev)."""
        self.sample(table, h, seed)
        self.forward(self.idx, h, self.y, keep=True)
        self.loss(self.y, self.target, self.dy)
        self.backward(self.idx, h, self.dy)
        self.adam(lr)


def _torch_f32():
    import torch
    return torch.float32


def create(sigma: int, d: int, h: int, dtype: str = "f64", device=None) -> Lcsb:
    return Lcsb(sigma, d, h, dtype, device)
