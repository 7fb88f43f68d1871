"""Vector-Jacobian product of the randomized low-rank SVD, oracle side.

The gradient asked for is that of the implemented forward map
A -> (U, Sigma, V) of Algorithm 7 with the sketch Omega held fixed.  The
oracle obtains it by reverse-mode differentiation (torch, CPU, float64)
through the very steps of ``lowrank_ref``: products with A, Householder QR
(``torch.linalg.qr``), the SVD of B = Q^* A and the truncation to k.  The
sign convention is applied with signs treated as constants (they are locally
constant wherever w^T v_j != 0).

The scalar loss is  L = sum_j w_j sigma_j + <G_U, U> + <G_V, V>.
"""
from __future__ import annotations

import math

import numpy as np
import torch

_G = (math.sqrt(5.0) - 1.0) / 2.0


def _sign_ref(n: int) -> torch.Tensor:
    t = torch.arange(1, n + 1, dtype=torch.float64) * _G
    return t - torch.floor(t) - 0.5


def lowrank_torch(A: torch.Tensor, Omega: torch.Tensor, k: int, q: int):
    """Algorithm 7 in torch float64 (differentiable in A)."""
    Qt = Omega
    for _ in range(q):
        Q, _r = torch.linalg.qr(A @ Qt)
        Qt, _r = torch.linalg.qr(A.T @ Q)
    Q, _r = torch.linalg.qr(A @ Qt)
    Q, _r = torch.linalg.qr(Q)                          # second orthonormalization
    B = Q.T @ A
    Ub, s, Vh = torch.linalg.svd(B, full_matrices=False)
    U = Q @ Ub[:, :k]
    V = Vh[:k].T
    sgn = torch.where(_sign_ref(V.shape[0]) @ V.detach() < 0, -1.0, 1.0).to(torch.float64)
    return U * sgn, s[:k], V * sgn


def loss_value(U, s, V, w, GU, GV):
    return (w * s).sum() + (GU * U).sum() + (GV * V).sum()


def grad_ref(A: np.ndarray, Omega: np.ndarray, k: int, q: int, w: np.ndarray,
             GU: np.ndarray, GV: np.ndarray):
    """Return (dL/dA, L) for the loss above, float64 numpy."""
    At = torch.tensor(np.asarray(A, dtype=np.float64), requires_grad=True)
    Om = torch.tensor(np.asarray(Omega, dtype=np.float64))
    U, s, V = lowrank_torch(At, Om, k, q)
    L = loss_value(U, s, V, torch.tensor(w), torch.tensor(GU), torch.tensor(GV))
    L.backward()
    return At.grad.numpy().copy(), float(L.detach())


def loss_ref(A: np.ndarray, Omega: np.ndarray, k: int, q: int, w, GU, GV) -> float:
    with torch.no_grad():
        U, s, V = lowrank_torch(torch.tensor(np.asarray(A, dtype=np.float64)),
                                torch.tensor(np.asarray(Omega, dtype=np.float64)), k, q)
        return float(loss_value(U, s, V, torch.tensor(w), torch.tensor(GU), torch.tensor(GV)))
