"""Accuracy metrics of the paper's tables (Table "heads"), oracle side.

* ``maxentry_ortho(U)``  = MaxEntry(|U^* U - I|), the paper's orthonormality metric.
* ``ortho_spec(U)``      = ||U^* U - I||_2 (spectral norm; bounds MaxEntry from above).
* ``spectral_residual``  = ||A - U Sigma V^*||_2 estimated by the power method, as
  the paper does with 20 iterations (Section 2); optionally run to convergence.

U^* U is accumulated in double precision over row blocks that are then summed
pairwise (a binary tree), so the rounding error grows like log(m) rather than
m; a plain running sum over millions of rows would already err at 1e-14.
"""
from __future__ import annotations

import numpy as np

_BLOCK = 4096


def gram_pairwise(U: np.ndarray) -> np.ndarray:
    """U^T U in float64 with pairwise summation of row-block Gram matrices."""
    m = U.shape[0]
    parts = [np.asarray(U[r0:r0 + _BLOCK], dtype=np.float64).T @ np.asarray(U[r0:r0 + _BLOCK], dtype=np.float64)
             for r0 in range(0, m, _BLOCK)]
    if not parts:
        return np.zeros((U.shape[1], U.shape[1]))
    while len(parts) > 1:
        nxt = [parts[i] + parts[i + 1] for i in range(0, len(parts) - 1, 2)]
        if len(parts) % 2:
            nxt.append(parts[-1])
        parts = nxt
    return parts[0]


def _gram_minus_identity(U: np.ndarray, cols: int | None = None) -> np.ndarray:
    G = gram_pairwise(U)
    c = G.shape[0] if cols is None else cols
    return G[:c, :c] - np.eye(c)


def maxentry_ortho(U: np.ndarray, cols: int | None = None) -> float:
    """MaxEntry(|U^* U - I|) over the first ``cols`` columns (all by default)."""
    return float(np.max(np.abs(_gram_minus_identity(U, cols)))) if U.shape[1] else 0.0


def ortho_spec(U: np.ndarray, cols: int | None = None) -> float:
    """||U^* U - I||_2 over the first ``cols`` columns (all by default)."""
    return float(np.linalg.norm(_gram_minus_identity(U, cols), 2)) if U.shape[1] else 0.0


def spectral_residual(A: np.ndarray, U: np.ndarray, s: np.ndarray, V: np.ndarray,
                      iters: int = 20, seed: int = 12345, tol: float | None = None,
                      max_iters: int = 200) -> float:
    """Power-method estimate of ||A - U diag(s) V^T||_2.

    E x is applied implicitly as A x - U (s * (V^T x)).  With ``tol`` set the
    iteration continues past ``iters`` until the estimate changes by less than
    ``tol`` relatively (at most ``max_iters``).
    """
    rng = np.random.default_rng(seed)
    n = A.shape[1]
    x = rng.standard_normal(n)
    x /= np.linalg.norm(x)
    blk = 1 << 16

    def e_mul(x):
        y = np.empty(A.shape[0])
        for r0 in range(0, A.shape[0], blk):
            y[r0:r0 + blk] = np.asarray(A[r0:r0 + blk], dtype=np.float64) @ x
        return y - U @ (s * (V.T @ x))

    def et_mul(y):
        z = np.zeros(n)
        for r0 in range(0, A.shape[0], blk):
            z += np.asarray(A[r0:r0 + blk], dtype=np.float64).T @ y[r0:r0 + blk]
        return z - V @ (s * (U.T @ y))

    est = 0.0
    it = 0
    while True:
        y = e_mul(x)
        new = float(np.linalg.norm(y))
        z = et_mul(y)
        nz = float(np.linalg.norm(z))
        it += 1
        done = it >= iters and (tol is None or abs(new - est) <= tol * max(new, 1e-300) or it >= max_iters)
        est = new
        if done or nz == 0.0:
            return est
        x = z / nz
