"""Philox4x32-10 and Box-Muller normals, oracle side.

Philox4x32 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as
1, 2, 3", SC'11): a 128-bit counter (c0, c1, c2, c3) and a 64-bit key
(k0, k1).  One round multiplies c0 and c2 by the constants M0 = 0xD2511F53
and M1 = 0xCD9E8D57 into 64-bit products (hi, lo) and outputs
(hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0); the key is advanced by the Weyl
increments (0x9E3779B9, 0xBB67AE85) before every round after the first.
Ten rounds.

Sketch layout (the library's convention when no sketch is passed in): the
n x l sketch is filled in row-major order, four entries per counter value
t = 0, 1, ...: counter (t mod 2^32, t div 2^32, 0, 0), key (seed mod 2^32,
seed div 2^32).  Each output word x maps to u = (x + 1/2) 2^-32 in (0, 1),
and the pairs (u0, u1), (u2, u3) give two normals each by Box-Muller:
sqrt(-2 ln u_a) * (cos 2 pi u_b, sin 2 pi u_b).
"""
from __future__ import annotations

import numpy as np

M0, M1 = 0xD2511F53, 0xCD9E8D57
W0, W1 = 0x9E3779B9, 0xBB67AE85
MASK = 0xFFFFFFFF


def philox4x32_10(ctr, key):
    """Vectorized Philox4x32-10. ctr: (..., 4) uint64 holding 32-bit words; key: (2,) ints."""
    c = [np.asarray(ctr[..., i], dtype=np.uint64) for i in range(4)]
    k0 = np.uint64(key[0] & MASK)
    k1 = np.uint64(key[1] & MASK)
    m0, m1 = np.uint64(M0), np.uint64(M1)
    mask = np.uint64(MASK)
    for r in range(10):
        if r:
            k0 = np.uint64((int(k0) + W0) & MASK)
            k1 = np.uint64((int(k1) + W1) & MASK)
        p0 = m0 * c[0]
        p1 = m1 * c[2]
        hi0, lo0 = p0 >> np.uint64(32), p0 & mask
        hi1, lo1 = p1 >> np.uint64(32), p1 & mask
        c = [(hi1 ^ c[1] ^ k0) & mask, lo1, (hi0 ^ c[3] ^ k1) & mask, lo0]
    return np.stack(c, axis=-1)


def philox_normal(n: int, l: int, seed: int) -> np.ndarray:
    """n x l float64 standard normals laid out as described in the module docstring."""
    total = n * l
    nt = (total + 3) // 4
    t = np.arange(nt, dtype=np.uint64)
    ctr = np.zeros((nt, 4), dtype=np.uint64)
    ctr[:, 0] = t & np.uint64(MASK)
    ctr[:, 1] = t >> np.uint64(32)
    key = (int(seed) & MASK, (int(seed) >> 32) & MASK)
    x = philox4x32_10(ctr, key).astype(np.float64)
    u = (x + 0.5) * 2.0 ** -32
    r0 = np.sqrt(-2.0 * np.log(u[:, 0]))
    r1 = np.sqrt(-2.0 * np.log(u[:, 2]))
    z = np.stack([r0 * np.cos(2.0 * np.pi * u[:, 1]), r0 * np.sin(2.0 * np.pi * u[:, 1]),
                  r1 * np.cos(2.0 * np.pi * u[:, 3]), r1 * np.sin(2.0 * np.pi * u[:, 3])], axis=1)
    return z.reshape(-1)[:total].reshape(n, l)
