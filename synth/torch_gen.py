"""Seeded synthetic matrices generated with torch, on any device.

Used where the host generator would be too slow (millions of rows).  The
recipe is the same as ``synth.matrices.planted``: Haar factors from the
sign-corrected QR of a Gaussian matrix, a planted spectrum, optional Gaussian
noise, then a round-to-nearest cast to the storage dtype.  The random streams
differ from NumPy's, so a test must hand the very same bytes to both sides.
Like the rest of ``synth`` this holds no step of the SVD method.
"""
from __future__ import annotations

import numpy as np
import torch

from .matrices import seed64


def _gen(device, workload: int, stream: str, sub: int = 0) -> torch.Generator:
    g = torch.Generator(device=device)
    g.manual_seed(seed64(workload, stream, sub))
    return g


def haar(m: int, n: int, workload: int, stream: str, device, sub: int = 0) -> torch.Tensor:
    g = torch.randn(m, n, generator=_gen(device, workload, stream, sub), device=device,
                    dtype=torch.float64)
    q, r = torch.linalg.qr(g)
    d = torch.sign(torch.diagonal(r))
    d[d == 0] = 1.0
    return q * d


def planted(m: int, n: int, sigma, workload: int, device, noise: float = 0.0,
            dtype=torch.float64, rank: int | None = None, sub: int = 0,
            chunk_rows: int = 65536) -> torch.Tensor:
    """A = U0 diag(sigma) V0^T + noise * N(0,1), built in row chunks and cast to ``dtype``."""
    sigma = np.asarray(sigma, dtype=np.float64)
    r = len(sigma) if rank is None else int(rank)
    s = torch.tensor(sigma[:r], dtype=torch.float64, device=device)
    u0 = haar(m, r, workload, "U0", device, sub)
    v0 = haar(n, r, workload, "V0", device, sub)
    w = (v0 * s).T.contiguous()  # r x n
    a = torch.empty(m, n, dtype=dtype, device=device)
    gn = _gen(device, workload, "noise", sub) if noise else None
    for r0 in range(0, m, chunk_rows):
        r1 = min(m, r0 + chunk_rows)
        blk = u0[r0:r1] @ w
        if noise:
            blk += noise * torch.randn(r1 - r0, n, generator=gn, device=device, dtype=torch.float64)
        a[r0:r1] = blk.to(dtype)
    del u0, v0, w
    return a


def gaussian(shape, workload: int, stream: str, device, sub: int = 0,
             dtype=torch.float64) -> torch.Tensor:
    return torch.randn(*shape, generator=_gen(device, workload, stream, sub), device=device,
                       dtype=torch.float64).to(dtype)


def sketch(n: int, l: int, workload: int, device, sub: int = 0) -> torch.Tensor:
    """Gaussian n x l sketch, entries exactly representable in bfloat16, held as float64."""
    g = gaussian((n, l), workload, "omega", device, sub)
    return g.to(torch.float32).to(torch.bfloat16).to(torch.float64)
