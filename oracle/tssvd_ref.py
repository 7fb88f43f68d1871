"""Tall-skinny SVD, oracle side: Algorithms 1 and 2 of the paper (Section 2).

The result the method reaches is the thin SVD of A (unique up to the sign of
each singular pair when the singular values are distinct).  The steps below
are taken in the paper's order:

  Alg. 1  (1) optional random orthogonal mixing B* = A Omega^*,
          (2) QR factorization B* = Q R (LAPACK Householder QR stands in for TSQR:
              both compute the same Householder factorization up to rounding),
          (3) discard rows of R whose |diagonal| < wp * |R_11| (and columns of Q),
          (4) SVD R = U~ Sigma V~^*,  (5) U = Q U~,  (6) V = Omega^* V~.
  Alg. 2  same, but (4') a second QR of Q~ = Q R, discard again, T = R R~,
          SVD of T, U = Q U~.

Outputs are "thin": U is m x n, V is n x n, sigma has n entries; singular
triplets beyond the numerical rank (after the discard rule) are zero columns
with sigma = 0.  Column signs follow ``oracle.signs``.
"""
from __future__ import annotations

import numpy as np

from .philox import philox_normal
from .signs import apply_sign_rule


def discard_rule(R: np.ndarray, wp: float) -> np.ndarray:
    """Indices of rows of R to keep under the working-precision rule of Algorithms 1-2.

    A diagonal entry counts as numerically zero when it is less (in absolute
    value) than the first diagonal entry times the working precision.  wp <= 0
    keeps every row.
    """
    d = np.abs(np.diag(R))
    if wp <= 0.0 or d.size == 0:
        return np.arange(R.shape[0])
    return np.nonzero(~(d < wp * d[0]))[0]


def haar_mix(n: int, seed: int) -> np.ndarray:
    """The n x n random orthogonal mixing Omega of Algorithm 1 step (1) (Remark on randomness):
    Omega = Q diag(sign(diag R)) for the QR factorization G = Q R of an n x n matrix G of
    Philox4x32-10 standard normals keyed by ``seed`` (``oracle.philox`` layout), which is
    Haar-distributed.  The paper's own D F S D~ F S~ is a fast stand-in for such a matrix;
    only its orthogonality and randomness enter the method.
    """
    G = philox_normal(n, n, seed)
    Q, R = np.linalg.qr(G)
    return Q * np.sign(np.diag(R))


def tsqr_ref(Y: np.ndarray, wp: float = 0.0, mix: np.ndarray | None = None):
    """One QR factorization Y Omega^* = Q R with the discard rule applied.

    Returns (Q, R) with Q: m x r orthonormal columns, R: r x l.
    ``mix`` is the optional orthogonal mixing matrix Omega (l x l).
    """
    Y = np.asarray(Y, dtype=np.float64)
    B = Y @ mix.T if mix is not None else Y
    Q, R = np.linalg.qr(B, mode="reduced")
    keep = discard_rule(R, wp)
    return Q[:, keep], R[keep, :]


def tssvd_ref(A: np.ndarray, wp: float = 0.0, double: bool = True,
              mix: np.ndarray | None = None, sign_rule: bool = True):
    """Thin SVD of a tall-skinny A by Algorithm 2 (double=True) or Algorithm 1.

    Returns (U, sigma, V, rank).
    """
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    if m < n:
        raise ValueError("tall-skinny SVD needs m >= n")
    Qt, Rt = tsqr_ref(A, wp, mix)                       # steps 1-3
    if double:
        Q, R = tsqr_ref(Qt, wp)                         # Alg. 2 steps 4-5
        T = R @ Rt                                      # Alg. 2 step 6
    else:
        Q, T = Qt, Rt
    Ut, s, Vh = np.linalg.svd(T, full_matrices=False)   # SVD of the small factor
    U = Q @ Ut                                          # U = Q U~
    V = Vh.T
    if mix is not None:
        V = mix.T @ V                                   # V = Omega^{-1} V~
    r = s.size
    Uo = np.zeros((m, n))
    Vo = np.zeros((n, n))
    so = np.zeros(n)
    Uo[:, :r], Vo[:, :r], so[:r] = U, V, s
    if sign_rule:
        Uo, Vo = apply_sign_rule(Uo, Vo)
    return Uo, so, Vo, r
