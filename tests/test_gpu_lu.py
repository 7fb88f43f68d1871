"""GPU parity of LU-based subspace tracking (TSSVD_FLAG_LU): lowrank_svd with the
intermediate bases of Algorithm 5 from a tournament-pivoted LU, through the C ABI, vs the
CPU oracle's Algorithm 7 with partial-pivoting LU tracking (``lowrank_ref(...,
tracking="lu")``) on the same inputs.

The two sides pivot differently (a tournament over row groups on the GPU, one column-wide
search in the oracle), so their L factors differ; both span the same columns, so the
outputs agree to rounding amplified by the conditioning of the tracked bases.  Inputs
plant a decaying spectrum with a gap after k, where that amplification is small.
"""
import numpy as np
import pytest
import torch

from oracle import checks
from oracle.lowrank_ref import lowrank_ref
from synth import matrices as sm

from gpu_util import col_sin, dev, flush_print, host, sigma_rel

pytestmark = pytest.mark.gpu

T = pytest.importorskip("paper_1612_08709_amd")


def _planted(m, n, workload, decay=8.0, r=None):
    sigma = np.exp(-np.arange((r or min(m, n))) / decay)
    return sm.planted(m, n, sigma, workload=workload), sigma


def _lowrank(A, Om, k, q, dtype=torch.float64, flags=T.FLAG_LU, **kw):
    U, S, V, info = T.lowrank_svd(dev(A, dtype), k, Om.shape[1], q, dev(Om), flags=flags, **kw)
    torch.cuda.synchronize()
    return host(U), host(S), host(V), info


# (m, n, k, l, q): l = 8 .. 60 covers the three register widths (16, 32, 64 columns);
# m and n from below one 256-row group to several tree levels, with ragged last groups
@pytest.mark.parametrize("m,n,k,l,q", [(1000, 37, 5, 8, 1), (3000, 400, 20, 30, 2),
                                       (5000, 300, 10, 16, 3), (2049, 257, 12, 24, 2),
                                       (20000, 700, 50, 60, 2), (70001, 1200, 20, 33, 1),
                                       (4000, 500, 10, 20, 0)])
def test_lu_lowrank_vs_oracle(m, n, k, l, q):
    flush_print("case lu lowrank", m, n, k, l, q)
    A, sigma = _planted(m, n, 500 + l, r=min(m, n, 400))
    Om = sm.sketch(n, l, 500 + l)
    U, S, V, info = _lowrank(A, Om, k, q)
    Ur, Sr, Vr = lowrank_ref(A, Om, k, q, tracking="lu")
    flush_print(f"  sigma rel {sigma_rel(S, Sr):.2e} U sin {np.max(col_sin(U, Ur)):.2e} "
                f"V sin {np.max(col_sin(V, Vr)):.2e}")
    assert sigma_rel(S, Sr) < 1e-11
    assert np.max(col_sin(U, Ur)) < 1e-8 and np.max(col_sin(V, Vr)) < 1e-8
    assert checks.ortho_spec(U) < 1e-13 and checks.ortho_spec(V) < 1e-13
    assert np.all(np.diff(S) <= 0)


@pytest.mark.parametrize("m,n,k,l,q", [(5000, 400, 64, 64, 1), (1000, 50, 1, 1, 2)])
def test_lu_width_limits(m, n, k, l, q):
    """l = 64 (the widest register row, k = l) and l = 1 (one pivot per group).  With k = l
    the trailing triplets sit at the edge of the sketch: rounding in the tracked subspaces
    moves every sigma_j by O(eps sigma_1), so all are bounded absolutely (1e-13 sigma_1) and
    the leading half relatively."""
    flush_print("case lu limits", m, n, k, l, q)
    A, _ = _planted(m, n, 540 + l, r=min(m, n, 300))
    Om = sm.sketch(n, l, 540 + l)
    U, S, V, _ = _lowrank(A, Om, k, q)
    Ur, Sr, Vr = lowrank_ref(A, Om, k, q, tracking="lu")
    h = k // 2 + 1
    assert np.max(np.abs(S - Sr)) <= 1e-13 * Sr[0] and sigma_rel(S[:h], Sr[:h]) < 1e-11
    assert np.max(col_sin(U[:, :h], Ur[:, :h])) < 1e-8
    assert checks.ortho_spec(U) < 1e-13 and checks.ortho_spec(V) < 1e-13


def test_lu_tracking_matches_qr_tracking_on_gpu():
    """Same column spaces: the LU route and the default route agree to rounding."""
    A, _ = _planted(30000, 1000, 531, r=400)
    Om = sm.sketch(1000, 40, 531)
    Ul, Sl, Vl, _ = _lowrank(A, Om, 30, 3)
    Uq, Sq, Vq, _ = _lowrank(A, Om, 30, 3, flags=0)
    assert sigma_rel(Sl, Sq) < 1e-11
    assert np.max(col_sin(Ul, Uq)) < 1e-8 and np.max(col_sin(Vl, Vq)) < 1e-8


def test_lu_float32_storage_and_mixed_precision():
    """float32 A: the FP64 path matches the oracle on the upcast matrix; the mixed path
    (bfloat16 power steps on the LU bases) keeps the residual of the FP64 path."""
    A, _ = _planted(20000, 1500, 532, decay=15.0, r=300)
    A32 = A.astype(np.float32)
    A64 = A32.astype(np.float64)
    Om = sm.sketch(1500, 60, 532)
    U, S, V, _ = _lowrank(A32, Om, 50, 3, dtype=torch.float32)
    Ur, Sr, Vr = lowrank_ref(A64, Om, 50, 3, tracking="lu")
    assert sigma_rel(S, Sr) < 1e-11
    assert np.max(col_sin(U[:, :40], Ur[:, :40])) < 1e-8
    Um, Sm, Vm, _ = _lowrank(A32, Om, 50, 3, dtype=torch.float32, prec=T.PREC_MIXED)
    assert checks.ortho_spec(Um) <= 1e-12 and checks.ortho_spec(Vm) <= 1e-12
    e = checks.spectral_residual(A64, Um, Sm, Vm, tol=1e-9)
    er = checks.spectral_residual(A64, Ur, Sr, Vr, tol=1e-9)
    flush_print(f"  residual mixed {e:.6e} oracle {er:.6e}")
    assert abs(e - er) <= 1e-6 * Sr[0]


def test_lu_singular_pivot_block_falls_back_to_householder_q():
    """A with 5 nonzero rows: every sketch Y has 5 nonzero rows, the sixth pivot is zero, so
    the first basis falls back to the TSQR's Q; the exact SVD of the rank-5 A comes back."""
    m, n, k, l = 3000, 400, 5, 10
    A = np.zeros((m, n))
    A[:5] = sm.gaussian((5, n), workload=533, stream="A")
    Om = sm.sketch(n, l, 533)
    U, S, V, _ = _lowrank(A, Om, k, 2)
    Ue, Se, Vhe = np.linalg.svd(A, full_matrices=False)
    np.testing.assert_allclose(S, Se[:k], rtol=1e-12)
    assert np.max(col_sin(U, Ue[:, :k])) < 1e-10 and np.max(col_sin(V, Vhe[:k].T)) < 1e-10


def test_lu_flag_argument_errors():
    A = dev(np.ones((300, 80)))
    Om = dev(sm.sketch(80, 10, 534))
    with pytest.raises(ValueError):                       # LU and Gram routes together
        T.lowrank_svd(A, 5, 10, 1, Om, flags=T.FLAG_LU | T.FLAG_GRAM)
    with pytest.raises(ValueError):                       # with the paper's discard rule
        T.lowrank_svd(A, 5, 10, 1, Om, flags=T.FLAG_LU, working_precision=1e-11)
    A2 = dev(np.ones((300, 200)))
    with pytest.raises(ValueError):                       # l above 64
        T.lowrank_svd(A2, 5, 65, 1, dev(sm.sketch(200, 65, 534)), flags=T.FLAG_LU)
    U, S, V, _ = T.lowrank_svd(A, 5, 10, 1, Om)
    with pytest.raises(ValueError):                       # no derivative through LU bases
        T.lowrank_svd_backward(A, 5, 10, 1, Om, U, S, V, gS=torch.ones_like(S), flags=T.FLAG_LU)
