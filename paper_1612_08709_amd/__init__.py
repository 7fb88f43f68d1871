"""MI355X (gfx950) tall-skinny and randomized low-rank SVD.

Python entry points with the names of the C ABI in ``include/tssvd.h``.  They only
marshal arguments: torch allocates device memory (outputs and the workspace) and
supplies the current HIP stream; every arithmetic step runs in libtssvd's kernels.

    Q, R          = tsqr(A)                      # Algorithm 1 step 2 (TSQR)
    U, S, V, info = tssvd(A, ...)                # Algorithms 1-2
    U, S, V, info = lowrank_svd(A, k, l, q, ...) # Algorithm 7
    gA            = lowrank_svd_backward(...)    # VJP of lowrank_svd (Omega fixed)
    LowRankSVD.apply(A, Omega, k, l, q)          # torch.autograd.Function wrapper
"""
from __future__ import annotations

import ctypes as C

import torch

from . import _native as N
from ._native import (F32, F64, ORTHO_AUTO, ORTHO_ONCE, ORTHO_TWICE, PREC_FP64,  # noqa: F401
                      PREC_MIXED, TSSVD_N_MAX, TSSVD_TSQR_N_MAX, FLAG_F32_MFMA_FINAL,
                      FLAG_NO_A_COPY, FLAG_GRAM, FLAG_LU, FLAG_MIX)

__all__ = ["tsqr", "tssvd", "tssvd_noalloc", "lowrank_svd", "lowrank_svd_backward", "LowRankSVD", "make_opts",
           "PREC_FP64", "PREC_MIXED", "ORTHO_AUTO", "ORTHO_ONCE", "ORTHO_TWICE",
           "FLAG_F32_MFMA_FINAL", "FLAG_NO_A_COPY", "FLAG_GRAM",
           "FLAG_LU", "FLAG_MIX"]


def _dtype_code(t: torch.Tensor) -> int:
    if t.dtype == torch.float64:
        return F64
    if t.dtype == torch.float32:
        return F32
    raise ValueError(f"A must be float64 or float32, got {t.dtype}")


def _check_matrix(A: torch.Tensor, name="A"):
    if not A.is_cuda:
        raise ValueError(f"{name} must be a device (HIP) tensor")
    if A.dim() != 2 or A.stride(1) != 1 or A.stride(0) < A.shape[1]:
        raise ValueError(f"{name} must be a 2-D row-major tensor with unit column stride")


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else C.c_void_p(0)


def _stream(device) -> C.c_void_p:
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _check_omega(Omega, n: int, l: int, device):
    """The sketch is read as a contiguous n x l float64 device array (or is None)."""
    if Omega is None:
        return
    if Omega.dtype != torch.float64 or tuple(Omega.shape) != (n, l) or \
            not Omega.is_contiguous() or Omega.device != torch.device(device):
        raise ValueError("Omega must be a contiguous float64 n x l tensor on A's device")


def _check_cotangent(t, shape, name, device):
    """A cotangent, when given, must have the shape of the output it belongs to."""
    if t is None:
        return None
    if tuple(t.shape) != tuple(shape) or t.device != torch.device(device):
        raise ValueError(f"{name} must have shape {tuple(shape)} and live on A's device")
    return t.to(torch.float64).contiguous()


def _workspace(nbytes: int, device) -> torch.Tensor:
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


def make_opts(prec=PREC_FP64, ortho=ORTHO_AUTO, working_precision=0.0, reorth_tol=1e-13,
              max_jacobi_sweeps=30, seed=None, flags=0) -> N.Opts:
    o = N.default_opts()
    o.flags = int(flags)
    o.prec, o.ortho = int(prec), int(ortho)
    o.working_precision = float(working_precision)
    o.reorth_tol = float(reorth_tol)
    o.max_jacobi_sweeps = int(max_jacobi_sweeps)
    if seed is not None:
        o.seed = int(seed) & ((1 << 64) - 1)
    return o


class _InfoBuf:
    """Device-side tssvd_info record, read back after a synchronization."""

    def __init__(self, device):
        self.t = torch.zeros(C.sizeof(N.Info), dtype=torch.uint8, device=device)

    @property
    def ptr(self):
        return C.c_void_p(self.t.data_ptr())

    def read(self) -> dict:
        raw = bytes(self.t.cpu().numpy().tobytes())
        info = N.Info.from_buffer_copy(raw)
        return dict(numstat=info.numstat, rank=info.rank, sweeps=info.sweeps,
                    reorth=info.reorth, ortho=info.ortho)


def tsqr(A: torch.Tensor, want_q: bool = True):
    """A = Q R by TSQR.  Returns (Q or None, R), float64."""
    _check_matrix(A)
    m, n = A.shape
    lib = N.lib()
    nb = C.c_size_t()
    N.check(lib.tsqr_workspace_bytes(m, n, _dtype_code(A), C.byref(nb)), "tsqr_workspace_bytes")
    work = _workspace(nb.value, A.device)
    Q = torch.empty(m, n, dtype=torch.float64, device=A.device) if want_q else None
    R = torch.empty(n, n, dtype=torch.float64, device=A.device)
    st = lib.tsqr(_ptr(A), _dtype_code(A), m, n, A.stride(0), _ptr(Q), n, _ptr(R), n,
                  _ptr(work), nb.value, _stream(A.device))
    N.check(st, "tsqr")
    return Q, R


def tssvd(A: torch.Tensor, opts: N.Opts | None = None, **kw):
    """Thin SVD of a tall-skinny A.  Returns (U, S, V, info) with info a dict (synchronizes)."""
    _check_matrix(A)
    m, n = A.shape
    o = opts if opts is not None else make_opts(**kw)
    lib = N.lib()
    nb = C.c_size_t()
    N.check(lib.tssvd_workspace_bytes(m, n, _dtype_code(A), C.byref(o), C.byref(nb)),
            "tssvd_workspace_bytes")
    work = _workspace(nb.value, A.device)
    U = torch.empty(m, n, dtype=torch.float64, device=A.device)
    S = torch.empty(n, dtype=torch.float64, device=A.device)
    V = torch.empty(n, n, dtype=torch.float64, device=A.device)
    info = _InfoBuf(A.device)
    st = lib.tssvd(_ptr(A), _dtype_code(A), m, n, A.stride(0), _ptr(U), n, _ptr(S), _ptr(V), n,
                   info.ptr, _ptr(work), nb.value, C.byref(o), _stream(A.device))
    N.check(st, "tssvd")
    return U, S, V, info.read()


def tssvd_noalloc(A: torch.Tensor, opts: N.Opts | None = None, **kw):
    """tssvd through the entry point that takes no workspace (the library's fixed per-GPU
    scratch array).  Returns (U, S, V, info) like tssvd."""
    _check_matrix(A)
    m, n = A.shape
    o = opts if opts is not None else make_opts(**kw)
    U = torch.empty(m, n, dtype=torch.float64, device=A.device)
    S = torch.empty(n, dtype=torch.float64, device=A.device)
    V = torch.empty(n, n, dtype=torch.float64, device=A.device)
    info = _InfoBuf(A.device)
    with torch.cuda.device(A.device):
        st = N.lib().tssvd_noalloc(_ptr(A), _dtype_code(A), m, n, A.stride(0), _ptr(U), n,
                                   _ptr(S), _ptr(V), n, info.ptr, C.byref(o),
                                   _stream(A.device))
    N.check(st, "tssvd_noalloc")
    return U, S, V, info.read()


class LowrankCall:
    """A reusable, pre-planned lowrank_svd call (workspace and outputs allocated once)."""

    def __init__(self, A: torch.Tensor, k: int, l: int, q: int, opts: N.Opts | None = None,
                 **kw):
        _check_matrix(A)
        self.A, self.k, self.l, self.q = A, int(k), int(l), int(q)
        self.m, self.n = A.shape
        self.o = opts if opts is not None else make_opts(**kw)
        lib = N.lib()
        nb = C.c_size_t()
        N.check(lib.lowrank_svd_workspace_bytes(self.m, self.n, self.k, self.l, self.q,
                                                _dtype_code(A), C.byref(self.o), C.byref(nb)),
                "lowrank_svd_workspace_bytes")
        self.nbytes = nb.value
        dev = A.device
        self.work = _workspace(nb.value, dev)
        self.U = torch.empty(self.m, self.k, dtype=torch.float64, device=dev)
        self.S = torch.empty(self.k, dtype=torch.float64, device=dev)
        self.V = torch.empty(self.n, self.k, dtype=torch.float64, device=dev)
        self.info = _InfoBuf(dev)

    def run(self, Omega: torch.Tensor | None = None):
        _check_omega(Omega, self.n, self.l, self.A.device)
        st = N.lib().lowrank_svd(_ptr(self.A), _dtype_code(self.A), self.m, self.n,
                                 self.A.stride(0), self.k, self.l, self.q, _ptr(Omega),
                                 _ptr(self.U), self.k, _ptr(self.S), _ptr(self.V), self.k,
                                 self.info.ptr, _ptr(self.work), self.nbytes, C.byref(self.o),
                                 _stream(self.A.device))
        N.check(st, "lowrank_svd")
        return self.U, self.S, self.V


def lowrank_svd(A: torch.Tensor, k: int, l: int, q: int, Omega: torch.Tensor | None = None,
                opts: N.Opts | None = None, **kw):
    """Rank-k SVD by Algorithm 7.  Returns (U, S, V, info)."""
    call = LowrankCall(A, k, l, q, opts, **kw)
    U, S, V = call.run(Omega)
    return U, S, V, call.info.read()


def lowrank_svd_backward(A, k, l, q, Omega, U, S, V, gU=None, gS=None, gV=None,
                         opts: N.Opts | None = None, **kw):
    """dL/dA for cotangents (gU, gS, gV) of lowrank_svd's outputs; returns gA (A's dtype)."""
    _check_matrix(A)
    m, n = A.shape
    k, l, q = int(k), int(l), int(q)
    _check_omega(Omega, n, l, A.device)
    # the cotangents are passed as contiguous float64 arrays, so their row strides are k;
    # the library reads gU and gV with the ldu / ldv strides (U and V themselves are not read)
    gU = _check_cotangent(gU, (m, k), "gU", A.device)
    gS = _check_cotangent(gS, (k,), "gS", A.device)
    gV = _check_cotangent(gV, (n, k), "gV", A.device)
    o = opts if opts is not None else make_opts(**kw)
    lib = N.lib()
    nb = C.c_size_t()
    N.check(lib.lowrank_svd_backward_workspace_bytes(m, n, k, l, q, _dtype_code(A), C.byref(o),
                                                     C.byref(nb)),
            "lowrank_svd_backward_workspace_bytes")
    work = _workspace(nb.value, A.device)
    gA = torch.empty_like(A)
    info = _InfoBuf(A.device)
    st = lib.lowrank_svd_backward(_ptr(A), _dtype_code(A), m, n, A.stride(0), k, l, q,
                                  _ptr(Omega), _ptr(U), k, _ptr(S), _ptr(V), k,
                                  _ptr(gU), _ptr(gS), _ptr(gV), _ptr(gA),
                                  gA.stride(0), info.ptr, _ptr(work), nb.value, C.byref(o),
                                  _stream(A.device))
    N.check(st, "lowrank_svd_backward")
    return gA


class LowRankSVD(torch.autograd.Function):
    """(U, S, V) = lowrank_svd(A) with a hand-written backward; Omega is held fixed."""

    @staticmethod
    def forward(ctx, A, Omega, k, l, q, opts=None):
        U, S, V, _ = lowrank_svd(A, k, l, q, Omega, opts)
        ctx.save_for_backward(A, Omega, U, S, V)
        ctx.cfg = (k, l, q, opts)
        return U, S, V

    @staticmethod
    def backward(ctx, gU, gS, gV):
        A, Omega, U, S, V = ctx.saved_tensors
        k, l, q, opts = ctx.cfg
        gA = lowrank_svd_backward(A, k, l, q, Omega, U, S, V, gU, gS, gV, opts)
        return gA, None, None, None, None, None
