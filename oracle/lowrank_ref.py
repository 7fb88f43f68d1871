"""Randomized low-rank SVD, oracle side: Algorithm 7 = Algorithm 5 feeding Algorithm 6.

Algorithm 5 (randomized subspace iteration, Halko-Martinsson-Tropp 4.4):
    Q~_0 = Omega (n x l, supplied by the caller — the random draw is an input)
    for j = 1..q:  Y_j = A Q~_{j-1};  Y_j = Q_j R_j;  Y~_j = A^* Q_j;  Y~_j = Q~_j R~_j
    Y = A Q~_q;  Y = Q R using double orthonormalization (Algorithm 2 form)
Algorithm 6 (direct SVD, HMT 5.1):
    B = Q^* A;  B = U~ Sigma V^*;  U = Q U~
Truncation to the leading k <= l triplets and the sign convention of
``oracle.signs`` are applied at the end.

Reading (Section 3): the factorizations inside Algorithm 5 only track a
subspace, and the paper notes that the trailing SVD steps of Algorithm 1 are
superfluous there; any orthonormal basis of the same column space leaves the
final U, Sigma, V unchanged.  The oracle therefore takes Q from a Householder
QR directly.  With wp > 0 (the paper's discard rule) the basis may lose
columns.  No random mixing is applied before these factorizations: the printed
Algorithm 7 errors are identical across independent runs, which a random
mixing at a rank threshold would not give.

For single-precision inputs every product is formed in double precision from
the stored values (exact upcast), in row blocks to bound host memory.
"""
from __future__ import annotations

import numpy as np

from .lu_ref import lu_basis
from .signs import apply_sign_rule
from .tssvd_ref import tsqr_ref

_BLOCK = 1 << 16


def _a_times(A: np.ndarray, X: np.ndarray) -> np.ndarray:
    """A @ X in float64 (A may be float32), row-blocked."""
    m = A.shape[0]
    out = np.empty((m, X.shape[1]))
    for r0 in range(0, m, _BLOCK):
        out[r0:r0 + _BLOCK] = np.asarray(A[r0:r0 + _BLOCK], dtype=np.float64) @ X
    return out


def _at_times(A: np.ndarray, Q: np.ndarray) -> np.ndarray:
    """A^T @ Q in float64, summing row blocks in order."""
    out = np.zeros((A.shape[1], Q.shape[1]))
    for r0 in range(0, A.shape[0], _BLOCK):
        out += np.asarray(A[r0:r0 + _BLOCK], dtype=np.float64).T @ Q[r0:r0 + _BLOCK]
    return out


def lowrank_ref(A: np.ndarray, Omega: np.ndarray, k: int, q: int, wp: float = 0.0,
                return_basis: bool = False, tracking: str = "qr"):
    """Rank-k approximation U diag(sigma) V^T of A via Algorithm 7.

    tracking="lu" takes the intermediate bases of Algorithm 5 from an LU factorization
    with partial pivoting (``oracle.lu_ref``) instead of QR; the last step is unchanged.
    Returns (U m x k, sigma k, V n x k[, Q]).  Columns past the numerical rank
    are zero with sigma = 0.
    """
    m, n = A.shape
    Omega = np.asarray(Omega, dtype=np.float64)
    l = Omega.shape[1]
    if not (0 < k <= l < min(m, n)):
        raise ValueError("need 0 < k <= l < min(m, n)")
    if tracking not in ("qr", "lu") or (tracking == "lu" and wp > 0.0):
        raise ValueError("tracking is 'qr', or 'lu' without the discard rule")

    def orth(Y):
        return tsqr_ref(Y, wp)[0]

    track = orth if tracking == "qr" else lu_basis
    Qt = Omega                                          # step 1
    for _ in range(q):                                  # steps 2-7
        Qj = track(_a_times(A, Qt))                     # Y_j = A Q~_{j-1};  Y_j = Q_j R_j
        Qt = track(_at_times(A, Qj))                    # Y~_j = A^* Q_j;  Y~_j = Q~_j R~_j
    Q = tsqr_ref(orth(_a_times(A, Qt)), wp)[0]          # last step, orthonormalized twice (Alg. 2)
    B = _at_times(A, Q).T                               # Alg. 6: B = Q^* A  (r x n)
    Ub, s, Vh = np.linalg.svd(B, full_matrices=False)   # B = U~ Sigma V^*
    r = min(k, s.size)
    U = np.zeros((m, k))
    V = np.zeros((n, k))
    so = np.zeros(k)
    U[:, :r] = Q @ Ub[:, :r]                            # U = Q U~
    V[:, :r] = Vh[:r].T
    so[:r] = s[:r]
    U, V = apply_sign_rule(U, V)
    if return_basis:
        return U, so, V, Q
    return U, so, V
