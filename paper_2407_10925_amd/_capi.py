"""ctypes declarations of the C ABI in include/lcsb.h (argument marshalling only)."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblcsb.so")

LCSB_OK = 0
LCSB_EINVAL = -1
LCSB_ENOMEM = -2
LCSB_EHIP = -3
LCSB_ESTATE = -4
LCSB_EUNSUPPORTED = -5
LCSB_ENONFINITE = -6
LCSB_ECKPT = -7
LCSB_F64 = 0
LCSB_F32 = 1
LCSB_MLP_NPARAMS = 140289

_NAMES = {0: "LCSB_OK", -1: "LCSB_EINVAL", -2: "LCSB_ENOMEM", -3: "LCSB_EHIP",
          -4: "LCSB_ESTATE", -5: "LCSB_EUNSUPPORTED", -6: "LCSB_ENONFINITE",
          -7: "LCSB_ECKPT"}


class LcsbError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__(f"{_NAMES.get(code, code)}: {message}")
        self.code = code


LCSB_STOP_NAMES = {0: "max_sweeps", 1: "target", 2: "converged", 3: "floor"}
LCSB_ITER_RING = 0
LCSB_ITER_TWO_ARRAY = 1
LCSB_ITER_TWO_ARRAY_PACKED = 2
ITERATIONS = {"ring": LCSB_ITER_RING, "two_array": LCSB_ITER_TWO_ARRAY,
              "two_array_packed": LCSB_ITER_TWO_ARRAY_PACKED}
LCSB_CERT_FEASIBLE = 0
LCSB_CERT_OPTIMAL = 1
CERT_KINDS = {"feasible": LCSB_CERT_FEASIBLE, "optimal": LCSB_CERT_OPTIMAL}


class RunPolicy(C.Structure):
    _fields_ = [("cadence", C.c_int64), ("first", C.c_int64), ("max_sweeps", C.c_int64),
                ("target", C.c_double), ("stop_delta", C.c_double), ("min_gain", C.c_double),
                ("certificate", C.c_int64), ("log_path", C.c_char_p)]


class Cert(C.Structure):
    _fields_ = [("bound", C.c_double), ("R", C.c_double), ("E", C.c_double),
                ("maxW", C.c_double), ("rho", C.c_double), ("sweep", C.c_int64),
                ("argmax_W", C.c_uint64), ("nonfinite", C.c_uint64), ("kind", C.c_int64)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


_lib = None
P = C.c_void_p


def load():
    """Load the in-tree liblcsb.so; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is missing: build it first (python -m paper_2407_10925_amd.build)")
    L = C.CDLL(LIB_PATH)
    L.lcsb_last_error.restype = C.c_char_p
    L.lcsb_last_error.argtypes = []
    L.lcsb_create.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, C.POINTER(P)]
    L.lcsb_create_iter.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.POINTER(P)]
    L.lcsb_rate.argtypes = [P, C.POINTER(C.c_double)]
    L.lcsb_query.argtypes = [P, C.POINTER(C.c_int), C.POINTER(C.c_uint64), C.POINTER(C.c_uint64),
                             C.POINTER(C.c_uint64)]
    L.lcsb_bind.argtypes = [P, C.POINTER(P), C.c_int, P, P]
    L.lcsb_query_means.argtypes = [P, C.POINTER(C.c_uint64)]
    L.lcsb_bind_means.argtypes = [P, C.POINTER(P), C.c_int]
    L.lcsb_init_zero.argtypes = [P]
    L.lcsb_load_ring.argtypes = [P, C.POINTER(P), C.c_int, C.POINTER(C.c_double)]
    L.lcsb_iterate.argtypes = [P, C.c_int64]
    L.lcsb_certify.argtypes = [P, C.POINTER(Cert), C.POINTER(Cert)]
    L.lcsb_certify_optimal.argtypes = [P, C.POINTER(Cert), C.POINTER(Cert)]
    L.lcsb_certify_optimal_noalloc.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, P, C.c_int, P,
                                               P]
    L.lcsb_lag.argtypes = [P, C.c_int, C.POINTER(P), C.POINTER(C.c_double)]
    L.lcsb_read_table.argtypes = [P, C.c_int, P, C.c_int]
    L.lcsb_status.argtypes = [P, C.POINTER(C.c_int64), C.POINTER(Cert)]
    L.lcsb_swap_symmetric.argtypes = [P, C.POINTER(C.c_int)]
    L.lcsb_upcast.argtypes = [P, P]
    L.lcsb_run.argtypes = [P, C.POINTER(RunPolicy), C.POINTER(Cert), C.POINTER(Cert),
                           C.POINTER(C.c_int64), C.POINTER(C.c_int)]
    L.lcsb_save.argtypes = [P, C.c_char_p]
    L.lcsb_load.argtypes = [P, C.c_char_p]
    L.lcsb_destroy.argtypes = [P]
    L.lcsb_mlp_workspace.argtypes = [C.c_int64, C.POINTER(C.c_uint64)]
    L.lcsb_mlp_init.argtypes = [P, C.c_uint64, P]
    L.lcsb_mlp_to_bf16.argtypes = [P, P, P]
    L.lcsb_mlp_sample.argtypes = [P, C.c_int, C.c_int, C.c_uint64, C.c_int64, P, P, P]
    L.lcsb_mlp_forward.argtypes = [P, P, P, C.c_int, C.c_int64, P, P, P]
    L.lcsb_mlp_loss.argtypes = [P, P, C.c_int64, P, P, P]
    L.lcsb_mlp_backward.argtypes = [P, P, C.c_int, P, C.c_int64, P, P, P]
    L.lcsb_mlp_adam.argtypes = [P, P, P, P, P, C.c_float, C.c_float, C.c_float, C.c_float,
                                C.c_int64, P]
    L.lcsb_init_seed_mlp.argtypes = [P, P, P, C.c_double]
    for name in ("lcsb_create", "lcsb_create_iter", "lcsb_rate", "lcsb_query", "lcsb_bind", "lcsb_init_zero", "lcsb_load_ring",
                 "lcsb_iterate", "lcsb_certify", "lcsb_certify_optimal",
                 "lcsb_certify_optimal_noalloc", "lcsb_lag", "lcsb_read_table", "lcsb_status", "lcsb_swap_symmetric",
                 "lcsb_upcast",
                 "lcsb_run", "lcsb_save", "lcsb_load", "lcsb_destroy", "lcsb_mlp_workspace", "lcsb_mlp_init", "lcsb_mlp_to_bf16",
                 "lcsb_mlp_sample", "lcsb_mlp_forward", "lcsb_mlp_loss", "lcsb_mlp_backward",
                 "lcsb_mlp_adam", "lcsb_init_seed_mlp"):
        getattr(L, name).restype = C.c_int
    _lib = L
    return L


def check(rc: int) -> int:
    if rc != LCSB_OK:
        raise LcsbError(rc, load().lcsb_last_error().decode(errors="replace"))
    return rc
