"""Gram-based SVD, oracle side: Algorithms 3 and 4 of the paper (Section 2) and
Algorithm 8 (Section 3), in plain float64.  Test infrastructure only.

Algorithm 3 (tall-skinny SVD from the Gram matrix):
    (1) B = A^* A,  (2) eigendecomposition B = V D V^*,  (3) U~ = A V,
    (4) Sigma = Euclidean norms of the columns of U~ (explicit normalization, the
        paper's remark on normalizing),
    (5) discard entries of Sigma below max(Sigma) * sqrt(wp), with their columns
        of U~ and V,
    (6) U = U~ Sigma^{-1}.
Algorithm 4 (the same with double orthonormalization):
    steps (1)-(6) give Y = U~ Sigma~^{-1}, Sigma~, V~; then
    Z = Y^* Y = W D W^*,  Q~ = Y W,  T = column norms of Q~ (discard below
    max(T) sqrt(wp)),  Q = Q~ T^{-1},  R = T W^* Sigma~ V~^*,
    R = P Sigma V^* (SVD),  U = Q P.
Algorithm 8: Algorithm 5 (randomized subspace iteration) taking its
intermediate orthonormal factors from Algorithm 3 and its last one from
Algorithm 4, then Algorithm 6 (B = Q^* A, B = U~ Sigma V^*, U = Q U~).

numpy's symmetric eigensolver and SVD serve as the eigendecomposition and SVD
steps; nothing else is reordered or fused.  Outputs are thin and zero-padded
past the kept rank like ``oracle.tssvd_ref``; column signs follow
``oracle.signs``.
"""
from __future__ import annotations

import numpy as np

from .lowrank_ref import _a_times, _at_times
from .signs import apply_sign_rule


def _eig_desc(B: np.ndarray):
    """Eigendecomposition of a symmetric matrix, eigenvalues in descending order."""
    d, V = np.linalg.eigh(B)
    order = np.argsort(-d, kind="stable")
    return d[order], V[:, order]


def _normalize(Yt: np.ndarray, wp: float):
    """Column norms of Yt, the discard at sqrt(wp), and the normalized kept columns.

    Returns (Y, norms, keep): Y = Yt[:, keep] / norms[keep].
    """
    # pairwise summation over each (contiguous) column: error ~ log2(m) eps even when the
    # squares are all equal, where a running sum would drift by up to m eps
    cols = np.ascontiguousarray(Yt.T)
    norms = np.sqrt(np.add.reduce(cols * cols, axis=1))
    if norms.size == 0:
        return Yt, norms, np.arange(0)
    thr = norms.max() * np.sqrt(wp) if wp > 0.0 else 0.0
    keep = np.nonzero((norms > 0.0) & ~(norms < thr))[0]
    return Yt[:, keep] / norms[keep], norms, keep


def alg3(A: np.ndarray, wp: float = 0.0):
    """Algorithm 3: returns (U m x r, sigma r, V n x r), columns in the eigenvalue order."""
    A = np.asarray(A, dtype=np.float64)
    B = A.T @ A                                           # (1) Gram matrix
    _, V = _eig_desc(B)                                   # (2) B = V D V^*
    Ut = A @ V                                            # (3) U~ = A V
    U, norms, keep = _normalize(Ut, wp)                   # (4)-(6)
    return U, norms[keep], V[:, keep]


def alg4(A: np.ndarray, wp: float = 0.0):
    """Algorithm 4: returns (U m x r, sigma r, V n x r), sigma descending."""
    Y, s1, V1 = alg3(A, wp)                               # Alg. 3 steps, Y = U~ Sigma~^{-1}
    Z = Y.T @ Y                                           # Z = Y^* Y
    _, W = _eig_desc(Z)                                   # Z = W D W^*
    Qt = Y @ W                                            # Q~ = Y W
    Q, t, keep = _normalize(Qt, wp)                       # T, discard, Q = Q~ T^{-1}
    R = (t[keep][:, None] * W[:, keep].T) @ (s1[:, None] * V1.T)   # R = T W^* Sigma~ V~^*
    P, s, Vh = np.linalg.svd(R, full_matrices=False)      # R = P Sigma V^*
    return Q @ P, s, Vh.T                                 # U = Q P


def gram_svd_ref(A: np.ndarray, wp: float = 0.0, double: bool = True, sign_rule: bool = True):
    """Thin SVD of a tall-skinny A by Algorithm 4 (double=True) or Algorithm 3.

    Returns (U m x n, sigma n, V n x n, rank), sigma descending and zero past the rank.
    """
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    if m < n:
        raise ValueError("tall-skinny SVD needs m >= n")
    U, s, V = alg4(A, wp) if double else alg3(A, wp)
    if not double:  # Alg. 3 orders by eigenvalue; report by singular value
        order = np.argsort(-s, kind="stable")
        U, s, V = U[:, order], s[order], V[:, order]
    r = s.size
    Uo, Vo, so = np.zeros((m, n)), np.zeros((n, n)), np.zeros(n)
    Uo[:, :r], Vo[:, :r], so[:r] = U, V, s
    if sign_rule:
        Uo, Vo = apply_sign_rule(Uo, Vo)
    return Uo, so, Vo, r


def lowrank_gram_ref(A: np.ndarray, Omega: np.ndarray, k: int, q: int, wp: float = 0.0):
    """Rank-k approximation U diag(sigma) V^T of A via Algorithm 8.

    Returns (U m x k, sigma k, V n x k); columns past the kept rank are zero.
    """
    m, n = A.shape
    Omega = np.asarray(Omega, dtype=np.float64)
    l = Omega.shape[1]
    if not (0 < k <= l < min(m, n)):
        raise ValueError("need 0 < k <= l < min(m, n)")
    Qt = Omega                                            # Alg. 5 step 1
    for _ in range(q):
        Qj = alg3(_a_times(A, Qt), wp)[0]                 # Y_j = A Q~_{j-1}; Q_j by Alg. 3
        Qt = alg3(_at_times(A, Qj), wp)[0]                # Y~_j = A^* Q_j; Q~_j by Alg. 3
    Q = alg4(_a_times(A, Qt), wp)[0]                      # last step by Alg. 4
    B = _at_times(A, Q).T                                 # Alg. 6: B = Q^* A
    Ub, s, Vh = np.linalg.svd(B, full_matrices=False)
    r = min(k, s.size)
    U, V, so = np.zeros((m, k)), np.zeros((n, k)), np.zeros(k)
    U[:, :r] = Q @ Ub[:, :r]
    V[:, :r] = Vh[:r].T
    so[:r] = s[:r]
    U, V = apply_sign_rule(U, V)
    return U, so, V
