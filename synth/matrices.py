"""Seeded synthetic matrices (NumPy, host).

Every generator is a pure function of its arguments and a seed.  Seeds are
derived from ``SeedSequence([ROOT_SEED, workload, stream])`` so that each
workload and each random object (left factor, right factor, noise, sketch,
cotangents, finite-difference directions) has its own independent stream.

Matrix families:

* ``planted``: A = U0 diag(sigma) V0^T (+ noise), U0/V0 Haar-distributed
  (QR of a Gaussian matrix, columns multiplied by the signs of diag(R)).
* ``dct_planted``: the paper's test matrices, A = U Sigma V^* with U and V the
  orthonormal DCT-II bases (Section 2, equations for the test matrix and its
  spectrum; Section 3 restricts the spectrum to the first l values).
* ``paper_spectrum``: sigma_j = exp((j-1)/(count-1) * ln 1e-20).
* ``staircase``: the Devil's-staircase spectrum of Appendix B.
"""
from __future__ import annotations

import math

import numpy as np

ROOT_SEED = 161208709

STREAM = {"U0": 0, "V0": 1, "noise": 2, "omega": 3, "w": 4, "GU": 5, "GV": 6,
          "fd": 7, "A": 8, "mix": 9, "power": 10}


def rng_for(workload: int, stream: str | int, sub: int = 0) -> np.random.Generator:
    s = STREAM[stream] if isinstance(stream, str) else int(stream)
    return np.random.default_rng(np.random.SeedSequence([ROOT_SEED, int(workload), s, int(sub)]))


def seed64(workload: int, stream: str | int, sub: int = 0) -> int:
    """A 63-bit integer seed for generators that take a plain integer (torch)."""
    s = STREAM[stream] if isinstance(stream, str) else int(stream)
    st = np.random.SeedSequence([ROOT_SEED, int(workload), s, int(sub)]).generate_state(2, np.uint32)
    return int((int(st[0]) << 31) ^ int(st[1])) & ((1 << 63) - 1)


def round_to_bf16(x: np.ndarray) -> np.ndarray:
    """Round to the nearest bfloat16-representable value (ties to even), returned as float64."""
    f = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def haar(rng: np.random.Generator, m: int, n: int) -> np.ndarray:
    """m x n matrix with orthonormal columns, Haar-distributed (sign-corrected QR of a Gaussian)."""
    g = rng.standard_normal((m, n))
    q, r = np.linalg.qr(g)
    d = np.sign(np.diag(r))
    d[d == 0] = 1.0
    return q * d


def planted(m: int, n: int, sigma, workload: int, noise: float = 0.0, rank: int | None = None,
            sub: int = 0) -> np.ndarray:
    """A = U0 diag(sigma) V0^T + noise * N(0,1), float64, row-major."""
    sigma = np.asarray(sigma, dtype=np.float64)
    r = len(sigma) if rank is None else rank
    sigma = sigma[:r]
    u0 = haar(rng_for(workload, "U0", sub), m, r)
    v0 = haar(rng_for(workload, "V0", sub), n, r)
    a = (u0 * sigma) @ v0.T
    if noise:
        a += noise * rng_for(workload, "noise", sub).standard_normal((m, n))
    return np.ascontiguousarray(a)


def planted_factors(m: int, n: int, sigma, workload: int, sub: int = 0):
    """Return (U0, sigma, V0) used by ``planted`` without noise."""
    sigma = np.asarray(sigma, dtype=np.float64)
    r = len(sigma)
    return (haar(rng_for(workload, "U0", sub), m, r), sigma,
            haar(rng_for(workload, "V0", sub), n, r))


def sketch(n: int, l: int, workload: int, sub: int = 0) -> np.ndarray:
    """Gaussian n x l sketch whose entries are exactly representable in bfloat16."""
    return round_to_bf16(rng_for(workload, "omega", sub).standard_normal((n, l)))


def gaussian(shape, workload: int, stream: str, sub: int = 0) -> np.ndarray:
    return rng_for(workload, stream, sub).standard_normal(shape)


def dct_basis(m: int, cols: int) -> np.ndarray:
    """First ``cols`` orthonormal DCT-II basis vectors of length m, as columns."""
    i = np.arange(m, dtype=np.float64)[:, None]
    k = np.arange(cols, dtype=np.float64)[None, :]
    c = np.cos(np.pi * (2.0 * i + 1.0) * k / (2.0 * m))
    scale = np.full(cols, math.sqrt(2.0 / m))
    scale[0] = math.sqrt(1.0 / m)
    return c * scale


def paper_spectrum(count: int, total: int | None = None) -> np.ndarray:
    """sigma_j = exp((j-1)/(total-1) * ln(1e-20)), j = 1..count (total defaults to count)."""
    total = count if total is None else total
    j = np.arange(1, count + 1, dtype=np.float64)
    return np.exp((j - 1.0) / (total - 1.0) * math.log(1e-20))


def dct_planted(m: int, n: int, sigma) -> np.ndarray:
    """A = U Sigma V^T with U, V orthonormal DCT-II bases and diag(Sigma) = sigma (zero beyond)."""
    sigma = np.asarray(sigma, dtype=np.float64)
    r = len(sigma)
    return np.ascontiguousarray((dct_basis(m, r) * sigma) @ dct_basis(n, r).T)


def staircase(k: int) -> np.ndarray:
    """Devil's-staircase singular values (Appendix B), descending.

    For j = 0..k-1 take round(j * 8^6 / k) (single precision, half rounded up),
    write it in octal, map every nonzero octal digit to binary 1, read the
    result in binary, and rescale by 1 / (2^6 (1 - 2^-6)) so values lie in [0, 1].
    """
    out = np.empty(k, dtype=np.float64)
    scale = np.float32(8.0 ** 6)
    for j in range(k):
        x = (np.float32(j) * scale) / np.float32(k)
        r = int(math.floor(float(x) + 0.5))
        digits = "".join("0" if ch == "0" else "1" for ch in format(r, "o"))
        out[j] = int(digits, 2) / 2.0 ** 6 / (1.0 - 2.0 ** -6)
    return np.sort(out)[::-1].copy()


# --------------------------------------------------------------------------------------------
# Workloads.  Sizes follow the tall-skinny and randomized low-rank experiments (Sections 2 and 3).
# --------------------------------------------------------------------------------------------

def workload_spec(w: int) -> dict:
    if w == 1:
        return dict(kind="tssvd", m=10_000, n=20, dtype="f64",
                    sigma=10.0 ** (-(np.arange(1, 21) - 1) / 4.0))
    if w == 2:
        return dict(kind="lowrank", m=200_000, n=2_000, dtype="f64", noise=1e-8,
                    sigma=1.0 / np.arange(1, 2001), k=20, l=30, q=2)
    if w == 3:
        return dict(kind="tssvd", m=4_000_000, n=100, dtype="f32",
                    sigma=np.logspace(0.0, -6.0, 100))
    if w == 4:
        return dict(kind="lowrank", m=500_000, n=8_000, dtype="f32", noise=1e-5, rank=600,
                    sigma=np.exp(-np.arange(1, 601) / 15.0), k=50, l=60, q=3)
    if w == 5:
        return dict(kind="grad", m=100_000, n=1_000, dtype="f32",
                    sigma=1.0 / np.arange(1, 1001), k=16, l=24, q=2)
    raise ValueError(f"unknown workload {w}")
