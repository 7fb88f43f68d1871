"""LU-based subspace tracking, oracle side — test infrastructure only.

Section 3 (the discussion of the power iterations): the intermediate factorizations of
Algorithm 5 only carry a column space forward, so the orthonormal factor Q may be replaced
by the lower triangular/trapezoidal factor L of an LU factorization.  With partial
pivoting, P Y = L U, and the rows of L put back in Y's order form P^T L = Y U^{-1}, which
spans the columns of Y whenever U is nonsingular.

``lu_basis`` writes Gaussian elimination with partial pivoting out step by step (the
largest |entry| of the remaining column is the pivot, the lowest row index among equal
ones).  The last step of Algorithm 5 keeps the double orthonormalization of Algorithm 2;
``oracle.lowrank_ref(..., tracking="lu")`` runs the whole of Algorithm 7 that way.
"""
from __future__ import annotations

import numpy as np


def lu_factor_gepp(Y: np.ndarray):
    """Gaussian elimination with partial pivoting of a tall Y (m x l, m >= l).

    Returns (rows, L, U): rows[i] is the row of Y eliminated at step i (its first l entries
    are the pivot order), L (m x l) unit lower trapezoidal in that row order, U (l x l)
    upper triangular, with Y[rows] = L @ U.  A column with no nonzero entry left gets a
    zero pivot and no elimination.
    """
    W = np.array(Y, dtype=np.float64, copy=True)
    m, l = W.shape
    if m < l:
        raise ValueError("LU basis needs m >= l")
    rows = np.arange(m)
    for j in range(l):
        p = j + int(np.argmax(np.abs(W[j:, j])))        # first index of the largest |entry|
        if p != j:
            W[[j, p]] = W[[p, j]]
            rows[[j, p]] = rows[[p, j]]
        piv = W[j, j]
        if piv != 0.0:
            W[j + 1:, j] /= piv                           # multipliers: column j of L
            W[j + 1:, j + 1:] -= np.outer(W[j + 1:, j], W[j, j + 1:])
    L = np.tril(W, -1)
    L[np.arange(l), np.arange(l)] = 1.0
    U = np.triu(W[:l])
    return rows, L, U


def lu_basis(Y: np.ndarray) -> np.ndarray:
    """The tracking basis P^T L (= Y U^{-1}), rows in Y's order."""
    rows, L, _ = lu_factor_gepp(Y)
    B = np.empty_like(L)
    B[rows] = L
    return B
