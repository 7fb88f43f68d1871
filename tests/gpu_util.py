"""Helpers for the GPU parity tests (comparison of the HIP path with the CPU oracle)."""
import numpy as np
import torch

DEV = "cuda:0"


def dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to(DEV)


def host(t):
    return t.detach().cpu().numpy()


def sigma_rel(s, ref):
    ref = np.asarray(ref)
    nz = ref > 0
    return float(np.max(np.abs(s[nz] - ref[nz]) / ref[nz])) if nz.any() else 0.0


def col_sin(U, Ur):
    """Per-column sin of the angle between U[:, j] and Ur[:, j] (sign-free).

    Computed from the chord d = |u - sign(u.v) v| of the normalized columns,
    sin = d sqrt(1 - d^2/4), which keeps full precision for tiny angles.
    Zero columns on both sides count as equal.
    """
    nu = np.linalg.norm(U, axis=0)
    nr = np.linalg.norm(Ur, axis=0)
    u = U / np.where(nu > 0, nu, 1.0)
    v = Ur / np.where(nr > 0, nr, 1.0)
    sg = np.where(np.sum(u * v, axis=0) < 0, -1.0, 1.0)
    d = np.linalg.norm(u - sg * v, axis=0)
    return d * np.sqrt(np.maximum(0.0, 1.0 - d * d / 4.0))


def flush_print(*a):
    print(*a, flush=True)
