"""Sign convention for singular vectors (oracle side).

A singular triplet (u_j, sigma_j, v_j) is defined only up to a common sign.
The paper leaves the choice open.  Convention used throughout: flip (u_j, v_j)
so that w^T v_j >= 0 for the fixed reference vector

    w_i = frac((i + 1) * g) - 1/2,   g = (sqrt(5) - 1) / 2,   i = 0 .. n-1,

evaluated in IEEE double precision.  w has no symmetry, so w^T v_j vanishes
only on a measure-zero set; tests also check the margin |w^T v_j|.
"""
from __future__ import annotations

import math

import numpy as np

_G = (math.sqrt(5.0) - 1.0) / 2.0


def sign_reference(n: int) -> np.ndarray:
    t = np.arange(1, n + 1, dtype=np.float64) * _G
    return t - np.floor(t) - 0.5


def apply_sign_rule(U: np.ndarray, V: np.ndarray):
    """Return copies of U, V with column signs fixed by the convention above."""
    w = sign_reference(V.shape[0])
    s = w @ V
    flip = np.where(s < 0.0, -1.0, 1.0)
    return U * flip, V * flip
