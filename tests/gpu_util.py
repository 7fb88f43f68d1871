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


def gram_pairwise_gpu(U, block=4096, group=256):
    """U^T U in float64 on the device: Gram matrices of 4096-row blocks, added pairwise (a
    binary tree), so the rounding error grows like log(m) rather than m.  This is the
    summation order of the oracle's checker; a single long GEMM over millions of rows
    already errs at ~1e-14."""
    m, n = U.shape
    parts = []
    for g0 in range(0, m, block * group):
        rows = min(m - g0, block * group)
        nb = (rows + block - 1) // block
        Ub = torch.zeros(nb * block, n, dtype=torch.float64, device=U.device)
        Ub[:rows] = U[g0:g0 + rows]
        Ub = Ub.view(nb, block, n)
        parts.append(torch.bmm(Ub.transpose(1, 2).contiguous(), Ub))
    G = torch.cat(parts) if parts else torch.zeros(1, n, n, dtype=torch.float64,
                                                   device=U.device)
    while G.shape[0] > 1:
        if G.shape[0] % 2:
            G = torch.cat([G, torch.zeros_like(G[:1])])
        G = G[0::2] + G[1::2]
    return G[0]


def ortho_gpu(U):
    """||U^T U - I||_2 in float64, the Gram summed pairwise on the device."""
    G = gram_pairwise_gpu(U)
    G -= torch.eye(G.shape[0], dtype=G.dtype, device=G.device)
    return float(np.linalg.norm(G.cpu().numpy(), 2))


def residual_gpu(A, U, S, V, tol=1e-10, max_iters=400, seed=12345, chunk=50_000):
    """Power-method estimate of ||A - U diag(S) V^T||_2 for a large device matrix A.

    Same iteration as the oracle's checker (E x applied implicitly as A x - U (S (V^T x)),
    continued until the estimate changes by less than ``tol`` relatively), with the
    products A x and A^T y done in float64 on the device over row chunks of A.
    """
    g = torch.Generator(device="cpu").manual_seed(seed)
    n = A.shape[1]
    x = torch.randn(n, generator=g, dtype=torch.float64).to(A.device)
    x /= torch.linalg.norm(x)

    def a_mul(x):
        return torch.cat([A[r0:r0 + chunk].double() @ x for r0 in range(0, A.shape[0], chunk)])

    def at_mul(y):
        z = torch.zeros(n, dtype=torch.float64, device=A.device)
        for r0 in range(0, A.shape[0], chunk):
            z += A[r0:r0 + chunk].double().T @ y[r0:r0 + chunk]
        return z

    est = 0.0
    for it in range(max_iters):
        y = a_mul(x) - U @ (S * (V.T @ x))
        z = at_mul(y) - V @ (S * (U.T @ y))
        new = float(torch.sqrt(torch.linalg.norm(z)))
        x = z / torch.linalg.norm(z)
        if it > 0 and abs(new - est) <= tol * new:
            return new
        est = new
    return est
