"""ctypes view of libtssvd.so (the C ABI declared in include/tssvd.h).

Only argument marshalling lives here.  Loading fails loudly when the library has not
been built: there is no fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtssvd.so")

TSSVD_N_MAX = 100
TSSVD_TSQR_N_MAX = 128
TSSVD_NOALLOC_SCRATCH_BYTES = 64 << 20

OK, E_INVALID_ARG, E_WORKSPACE, E_HIP, E_UNSUPPORTED = 0, 1, 2, 3, 4
F64, F32 = 0, 1
PREC_FP64, PREC_MIXED = 0, 1
ORTHO_AUTO, ORTHO_ONCE, ORTHO_TWICE = 0, 1, 2
NUM_NONFINITE, NUM_NO_CONVERGENCE = 1, 2
FLAG_F32_MFMA_FINAL = 1
FLAG_NO_A_COPY = 2
FLAG_GRAM = 4
FLAG_LU = 8
FLAG_MIX = 16

# every exported symbol declared in include/tssvd.h
EXPORTS = (
    "tssvd_default_opts", "tssvd_status_string", "tssvd_version",
    "tsqr_workspace_bytes", "tsqr",
    "tssvd_workspace_bytes", "tssvd", "tssvd_noalloc",
    "lowrank_svd_workspace_bytes", "lowrank_svd",
    "lowrank_svd_backward_workspace_bytes", "lowrank_svd_backward",
    "tssvd_profile_enable", "tssvd_profile_read",
)

PROF_AX, PROF_ATQ, PROF_LEAF_FACTOR, PROF_LEAF_APPLY = 0, 1, 2, 3
PROF_AX_BF16, PROF_ATQ_BF16, PROF_AX_FINAL, PROF_ATQ_FINAL = 4, 5, 6, 7
PROF_AX_BF16C, PROF_ATQ_BF16C = 8, 9
PROF_NAMES = {0: "gemm_ax_f64", 1: "gemm_atq_f64", 2: "tsqr_leaf_factor", 3: "tsqr_leaf_apply",
              4: "ax_bf16", 5: "atq_bf16", 6: "ax_final", 7: "atq_final", 8: "ax_bf16c",
              9: "atq_bf16c"}


class Opts(C.Structure):
    _fields_ = [("prec", C.c_int32), ("ortho", C.c_int32), ("working_precision", C.c_double),
                ("reorth_tol", C.c_double), ("max_jacobi_sweeps", C.c_int32),
                ("flags", C.c_int32), ("seed", C.c_uint64)]


class Info(C.Structure):
    _fields_ = [("numstat", C.c_int32), ("rank", C.c_int32), ("sweeps", C.c_int32),
                ("reorth", C.c_int32), ("ortho", C.c_double)]


_lib = None

P, I64, I32, SZ = C.c_void_p, C.c_int64, C.c_int32, C.c_size_t


def _declare(lib):
    lib.tssvd_default_opts.argtypes = [C.POINTER(Opts)]
    lib.tssvd_default_opts.restype = None
    lib.tssvd_status_string.argtypes = [C.c_int]
    lib.tssvd_status_string.restype = C.c_char_p
    lib.tssvd_version.argtypes = []
    lib.tssvd_version.restype = C.c_int
    lib.tsqr_workspace_bytes.argtypes = [I64, I64, I32, C.POINTER(SZ)]
    lib.tsqr.argtypes = [P, I32, I64, I64, I64, P, I64, P, I64, P, SZ, P]
    lib.tssvd_workspace_bytes.argtypes = [I64, I64, I32, C.POINTER(Opts), C.POINTER(SZ)]
    lib.tssvd.argtypes = [P, I32, I64, I64, I64, P, I64, P, P, I64, P, P, SZ, C.POINTER(Opts), P]
    lib.tssvd_noalloc.argtypes = [P, I32, I64, I64, I64, P, I64, P, P, I64, P, C.POINTER(Opts), P]
    lib.lowrank_svd_workspace_bytes.argtypes = [I64, I64, I64, I64, I64, I32, C.POINTER(Opts),
                                                C.POINTER(SZ)]
    lib.lowrank_svd.argtypes = [P, I32, I64, I64, I64, I64, I64, I64, P, P, I64, P, P, I64, P,
                                P, SZ, C.POINTER(Opts), P]
    lib.lowrank_svd_backward_workspace_bytes.argtypes = [I64, I64, I64, I64, I64, I32,
                                                         C.POINTER(Opts), C.POINTER(SZ)]
    lib.lowrank_svd_backward.argtypes = [P, I32, I64, I64, I64, I64, I64, I64, P, P, I64, P, P,
                                         I64, P, P, P, P, I64, P, P, SZ, C.POINTER(Opts), P]
    lib.tssvd_profile_enable.argtypes = [C.c_int]
    lib.tssvd_profile_enable.restype = C.c_int
    lib.tssvd_profile_read.argtypes = [C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_int64)]
    lib.tssvd_profile_read.restype = C.c_int
    for name in ("tsqr_workspace_bytes", "tsqr", "tssvd_workspace_bytes", "tssvd", "tssvd_noalloc",
                 "lowrank_svd_workspace_bytes", "lowrank_svd",
                 "lowrank_svd_backward_workspace_bytes", "lowrank_svd_backward"):
        getattr(lib, name).restype = C.c_int


def lib():
    """The loaded library (raises if it was never built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with `python -m paper_1612_08709_amd.build` "
                "(there is no CPU fallback)")
        handle = C.CDLL(LIB_PATH)
        _declare(handle)
        _lib = handle
    return _lib


def status_string(st: int) -> str:
    return lib().tssvd_status_string(st).decode()


def check(st: int, what: str):
    if st == OK:
        return
    msg = f"{what}: {status_string(st)} (status {st})"
    if st in (E_INVALID_ARG, E_WORKSPACE, E_UNSUPPORTED):
        raise ValueError(msg)
    raise RuntimeError(msg)


def profile_enable(on: bool):
    lib().tssvd_profile_enable(1 if on else 0)


def profile_read(kind: int):
    """(total_ms, launches) recorded for one kernel kind since profile_enable(True)."""
    ms, cnt = C.c_double(), C.c_int64()
    check(lib().tssvd_profile_read(kind, C.byref(ms), C.byref(cnt)), "tssvd_profile_read")
    return ms.value, cnt.value


def default_opts() -> Opts:
    o = Opts()
    lib().tssvd_default_opts(C.byref(o))
    return o
