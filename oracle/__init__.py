"""CPU oracle for the lower-bound iteration of arXiv 2407.10925.

TEST INFRASTRUCTURE.  Only the tests, the package smoke check and the
benchmark's CPU-baseline leg import this package; the GPU library never does,
and the two share no code.

``oracle.c`` holds the iteration, the certificate and the brute-force W_n
(all FP64, single-threaded); this module only builds it with gcc and marshals
numpy arrays through ctypes.  ``mlp.py`` holds the FP64 reference of the
warm-start network.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

GCC_FLAGS = ["-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
             "-frounding-math", "-fno-fast-math"]


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so next to it (gcc, no GPU)."""
    global _lib
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", *GCC_FLAGS, _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
        _lib = None
    return _LIB


class Cert(C.Structure):
    _fields_ = [("R", C.c_double), ("maxW", C.c_double), ("E", C.c_double),
                ("bound", C.c_double), ("rho", C.c_double),
                ("argmax_W", C.c_uint64), ("nonfinite", C.c_uint64)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class CertOpt(C.Structure):
    _fields_ = [("r", C.c_double), ("bound", C.c_double), ("argmin", C.c_uint64),
                ("nonfinite", C.c_uint64)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = C.CDLL(_LIB)
        P = C.POINTER
        L.or_num_entries.restype = C.c_uint64
        L.or_num_entries.argtypes = [C.c_int, C.c_int, C.c_int]
        L.or_decode.argtypes = [C.c_int, C.c_int, C.c_int, C.c_uint64, P(C.c_int)]
        L.or_encode.restype = C.c_uint64
        L.or_encode.argtypes = [C.c_int, C.c_int, C.c_int, P(C.c_int)]
        L.or_sweep.argtypes = [C.c_int, C.c_int, C.c_int, P(P(C.c_double)), P(C.c_double)]
        L.or_sweep_at.argtypes = [C.c_int, C.c_int, C.c_int, P(P(C.c_double)),
                                  P(C.c_uint64), C.c_uint64, P(C.c_double)]
        L.or_sweep_at_f32.argtypes = [C.c_int, C.c_int, C.c_int, P(P(C.c_float)),
                                      P(C.c_uint64), C.c_uint64, P(C.c_double)]
        L.or_certify_W_at_f32.argtypes = [C.c_int, C.c_int, C.c_int, P(C.c_float), C.c_double,
                                          P(C.c_uint64), C.c_uint64, P(C.c_double)]
        L.or_max_diff.argtypes = [P(C.c_double), P(C.c_double), C.c_uint64, P(C.c_double),
                                  P(C.c_uint64)]
        L.or_max_diff_f32.argtypes = [P(C.c_float), P(C.c_float), C.c_uint64, P(C.c_double),
                                      P(C.c_uint64)]
        L.or_certify.argtypes = [C.c_int, C.c_int, C.c_int, P(C.c_double), P(C.c_double), P(Cert)]
        L.or_certify_W_at.argtypes = [C.c_int, C.c_int, C.c_int, P(C.c_double), C.c_double,
                                      P(C.c_uint64), C.c_uint64, P(C.c_double)]
        L.or_feasible_triplet.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int64, C.c_int64,
                                          P(C.c_double), P(C.c_double), P(C.c_double)]
        L.or_certify_optimal.argtypes = [C.c_int, C.c_int, C.c_int, P(C.c_double), P(CertOpt)]
        L.or_certify_optimal_f32.argtypes = [C.c_int, C.c_int, C.c_int, P(C.c_float), P(CertOpt)]
        L.or_optimal_ratio_at.argtypes = [C.c_int, C.c_int, C.c_int, P(C.c_double), P(C.c_uint64),
                                          C.c_uint64, P(C.c_double)]
        L.or_optimal_ratio_at_f32.argtypes = [C.c_int, C.c_int, C.c_int, P(C.c_float),
                                              P(C.c_uint64), C.c_uint64, P(C.c_double)]
        L.or_brute_W.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, P(C.c_int), P(C.c_uint64)]
        L.or_two_array_step.argtypes = [C.c_int, C.c_int, C.c_int, P(C.c_double), C.c_double,
                                        P(C.c_double)]
        L.or_two_array_step_at.argtypes = [C.c_int, C.c_int, C.c_int, P(C.c_double), C.c_double,
                                           P(C.c_uint64), C.c_uint64, P(C.c_double)]
        L.or_sample_growth.argtypes = [C.c_int, C.c_int, C.c_int, P(C.c_double), P(C.c_double),
                                       P(C.c_double)]
        L.or_sample_coordinates.argtypes = [C.c_int, C.c_int, C.c_int, P(C.c_uint64)]
        _lib = L
    return _lib


def _dptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a


def _check(rc, what):
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed with code {rc}")


def num_entries(sigma, d, h):
    return int(lib().or_num_entries(sigma, d, h))


def decode(sigma, d, h, idx):
    """Symbols of the tuple at ``idx`` as a (d, h) int array (column 0 = heads)."""
    out = np.zeros(d * h, dtype=np.int32)
    _check(lib().or_decode(sigma, d, h, idx, out.ctypes.data_as(C.POINTER(C.c_int))), "decode")
    return out.reshape(d, h)


def encode(sigma, d, h, sym):
    s = np.ascontiguousarray(np.asarray(sym, dtype=np.int32).reshape(-1))
    return int(lib().or_encode(sigma, d, h, s.ctypes.data_as(C.POINTER(C.c_int))))


def _lag_array(lags):
    arrs = [_f64(x) for x in lags]
    ptrs = (C.POINTER(C.c_double) * len(arrs))(*[_dptr(a) for a in arrs])
    return arrs, ptrs


def sweep(sigma, d, h, lags):
    """F(lag_1, ..., lag_d) over every coordinate; lags[k-1] is lag k."""
    assert len(lags) == d
    arrs, ptrs = _lag_array(lags)
    out = np.empty(num_entries(sigma, d, h), dtype=np.float64)
    _check(lib().or_sweep(sigma, d, h, ptrs, _dptr(out)), "sweep")
    return out


def sweep_at(sigma, d, h, lags, idx):
    assert len(lags) == d
    arrs, ptrs = _lag_array(lags)
    idx = np.ascontiguousarray(idx, dtype=np.uint64)
    out = np.empty(idx.size, dtype=np.float64)
    _check(lib().or_sweep_at(sigma, d, h, ptrs, idx.ctypes.data_as(C.POINTER(C.c_uint64)),
                             idx.size, _dptr(out)), "sweep_at")
    return out


def _is_f32(a):
    return isinstance(a, np.ndarray) and a.dtype == np.float32


def _fptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_float))


def sweep_at_tables(sigma, d, h, lags, idx):
    """sweep_at for float64 or float32 tables (float32 read as exact doubles)."""
    if all(_is_f32(x) for x in lags):
        arrs = [np.ascontiguousarray(x) for x in lags]
        ptrs = (C.POINTER(C.c_float) * len(arrs))(*[_fptr(a) for a in arrs])
        idx = np.ascontiguousarray(idx, dtype=np.uint64)
        out = np.empty(idx.size, dtype=np.float64)
        _check(lib().or_sweep_at_f32(sigma, d, h, ptrs, idx.ctypes.data_as(C.POINTER(C.c_uint64)),
                                     idx.size, _dptr(out)), "sweep_at_f32")
        return out
    return sweep_at(sigma, d, h, lags, idx)


def certify_W_at_table(sigma, d, h, u, R, idx):
    if _is_f32(u):
        u = np.ascontiguousarray(u)
        idx = np.ascontiguousarray(idx, dtype=np.uint64)
        out = np.empty(idx.size, dtype=np.float64)
        _check(lib().or_certify_W_at_f32(sigma, d, h, _fptr(u), float(R),
                                         idx.ctypes.data_as(C.POINTER(C.c_uint64)), idx.size,
                                         _dptr(out)), "certify_W_at_f32")
        return out
    return certify_W_at(sigma, d, h, u, R, idx)


def max_diff(u, prev):
    """R of Algorithm 2 alone: (max_j (u - prev)[j], lowest arg)."""
    R, arg = C.c_double(), C.c_uint64()
    if _is_f32(u) and _is_f32(prev):
        u, prev = np.ascontiguousarray(u), np.ascontiguousarray(prev)
        _check(lib().or_max_diff_f32(_fptr(u), _fptr(prev), u.size, C.byref(R), C.byref(arg)),
               "max_diff_f32")
    else:
        u, prev = _f64(u), _f64(prev)
        _check(lib().or_max_diff(_dptr(u), _dptr(prev), u.size, C.byref(R), C.byref(arg)),
               "max_diff")
    return R.value, int(arg.value)


def certify(sigma, d, h, u, prev):
    """Certificate of the newest vector u (prev = the vector before it)."""
    u = _f64(u)
    prev = _f64(prev)
    c = Cert()
    _check(lib().or_certify(sigma, d, h, _dptr(u), _dptr(prev), C.byref(c)), "certify")
    return c.as_dict()


def certify_W_at(sigma, d, h, u, R, idx):
    u = _f64(u)
    idx = np.ascontiguousarray(idx, dtype=np.uint64)
    out = np.empty(idx.size, dtype=np.float64)
    _check(lib().or_certify_W_at(sigma, d, h, _dptr(u), float(R),
                                 idx.ctypes.data_as(C.POINTER(C.c_uint64)), idx.size,
                                 _dptr(out)), "certify_W_at")
    return out


def certify_optimal(sigma, d, h, u):
    """Largest r with (u, r, 0) a feasible triplet: dict(r, bound, argmin,
    nonfinite), r = min_A max_z c_z(A) / k_z rounded down, bound = d r.
    float32 tables are read as exact doubles."""
    c = CertOpt()
    if _is_f32(u):
        u = np.ascontiguousarray(u)
        _check(lib().or_certify_optimal_f32(sigma, d, h, _fptr(u), C.byref(c)), "certify_optimal")
    else:
        u = _f64(u)
        _check(lib().or_certify_optimal(sigma, d, h, _dptr(u), C.byref(c)), "certify_optimal")
    return c.as_dict()


def optimal_ratio_at(sigma, d, h, u, idx):
    """max_z c_z(A) / k_z (rounded down) at the coordinates idx."""
    idx = np.ascontiguousarray(idx, dtype=np.uint64)
    out = np.empty(idx.size, dtype=np.float64)
    ip = idx.ctypes.data_as(C.POINTER(C.c_uint64))
    if _is_f32(u):
        u = np.ascontiguousarray(u)
        _check(lib().or_optimal_ratio_at_f32(sigma, d, h, _fptr(u), ip, idx.size, _dptr(out)),
               "optimal_ratio_at")
    else:
        u = _f64(u)
        _check(lib().or_optimal_ratio_at(sigma, d, h, _dptr(u), ip, idx.size, _dptr(out)),
               "optimal_ratio_at")
    return out


def feasible_triplet(sigma, d, h, n_sweeps, cadence=1, want_ring=False):
    """Algorithm 2 from the zero ring.  Returns (best, history, ring).

    best = dict(sweep, r, eps, bound); history = (k, 4) array of
    (sweep, R, E, bound) per certified sweep; ring = (d, N) lag 1..d or None.
    """
    nh = n_sweeps // cadence
    hist = np.zeros(max(nh, 1) * 4, dtype=np.float64)
    best = np.zeros(4, dtype=np.float64)
    N = num_entries(sigma, d, h)
    ring = np.zeros(d * N, dtype=np.float64) if want_ring else None
    _check(lib().or_feasible_triplet(sigma, d, h, n_sweeps, cadence, _dptr(hist), _dptr(best),
                                     _dptr(ring) if want_ring else None), "feasible_triplet")
    return ({"sweep": int(best[0]), "r": best[1], "eps": best[2], "bound": best[3]},
            hist[: nh * 4].reshape(nh, 4),
            ring.reshape(d, N) if want_ring else None)


SAMPLE = 4096  # coordinates of the two-array iteration's rate sample


def two_array_step(sigma, d, h, u, R):
    """u_new = F(u, u - R, .., u - (d-1) R), the shift added to each branch
    mean (a reading of the two-array remark of Sec. 3.3)."""
    u = _f64(u)
    out = np.empty(u.size, dtype=np.float64)
    _check(lib().or_two_array_step(sigma, d, h, _dptr(u), float(R), _dptr(out)), "two_array_step")
    return out


def two_array_step_at(sigma, d, h, u, R, idx):
    """two_array_step at the coordinates idx only."""
    u = _f64(u)
    idx = np.ascontiguousarray(idx, dtype=np.uint64)
    out = np.empty(idx.size, dtype=np.float64)
    _check(lib().or_two_array_step_at(sigma, d, h, _dptr(u), float(R),
                                      idx.ctypes.data_as(C.POINTER(C.c_uint64)), idx.size,
                                      _dptr(out)), "two_array_step_at")
    return out


def sample_growth(sigma, d, h, u_new, u):
    """The rate of the next two-array step: mean of u_new - u over the sample."""
    u_new, u = _f64(u_new), _f64(u)
    R = C.c_double()
    _check(lib().or_sample_growth(sigma, d, h, _dptr(u_new), _dptr(u), C.byref(R)),
           "sample_growth")
    return R.value


def sample_coordinates(sigma, d, h):
    out = np.empty(SAMPLE, dtype=np.uint64)
    _check(lib().or_sample_coordinates(sigma, d, h, out.ctypes.data_as(C.POINTER(C.c_uint64))),
           "sample_coordinates")
    return out


def two_array_run(sigma, d, h, n_sweeps, cadence=1, certificate="feasible", u0=None, u1=None):
    """The two-array iteration from u1 (newest) and u0 (the table before it;
    both zero by default), certified every `cadence` steps with Algorithm 2's
    certificate (u and the table before it) or the largest-r one.  Returns
    (best, history, (u, u_prev, R)); best and each history entry are dicts
    with keys sweep, rho, bound (history entries also hold the certificate)."""
    N = num_entries(sigma, d, h)
    u_prev = np.zeros(N) if u0 is None else _f64(u0).copy()
    u = np.zeros(N) if u1 is None else _f64(u1).copy()
    R = sample_growth(sigma, d, h, u, u_prev)
    best = {"sweep": 0, "rho": 0.0, "bound": 0.0}
    hist = []
    for t in range(1, n_sweeps + 1):
        new = two_array_step(sigma, d, h, u, R)
        R = sample_growth(sigma, d, h, new, u)
        u_prev, u = u, new
        if t % cadence:
            continue
        if certificate == "optimal":
            c = certify_optimal(sigma, d, h, u)
            rho, ok = c["r"], c["nonfinite"] == 0
        else:
            c = certify(sigma, d, h, u, u_prev)
            rho, ok = c["rho"], c["nonfinite"] == 0
        hist.append({"sweep": t, "rho": rho, "bound": c["bound"], "cert": c, "R_next": R})
        if ok and rho >= best["rho"]:  # Algorithm 2's keep rule
            best = {"sweep": t, "rho": rho, "bound": c["bound"]}
    return best, hist, (u, u_prev, R)


def brute_W_sum(sigma, d, h, n, heads):
    """Integer sum over all sigma^(d n) tails; W_n = sum / sigma^(d n)."""
    a = np.ascontiguousarray(np.asarray(heads, dtype=np.int32).reshape(-1))
    assert a.size == d * h
    s = C.c_uint64(0)
    _check(lib().or_brute_W(sigma, d, h, n, a.ctypes.data_as(C.POINTER(C.c_int)), C.byref(s)),
           "brute_W")
    return int(s.value)
