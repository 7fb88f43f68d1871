"""GPU parity of lowrank_svd_backward (vector-Jacobian product, sketch held fixed).

References: the oracle's torch-float64 autograd through the same algorithm (G1), central
finite differences of the GPU forward itself, and, for an exactly rank-l matrix, the
gradient of the exact truncated SVD (closed-form thin-SVD derivative on LAPACK factors).
"""
import numpy as np
import pytest
import torch

from oracle import grad_ref
from synth import matrices as sm

from gpu_util import dev, flush_print, host

pytestmark = pytest.mark.gpu

T = pytest.importorskip("paper_1612_08709_amd")


def _instance(m, n, k, l, q, workload, exact_rank=False, dtype=np.float64):
    sigma = 1.0 / np.arange(1, min(m, n) + 1)
    if exact_rank:
        sigma = sigma[:l]
    A = sm.planted(m, n, sigma, workload=workload).astype(dtype)
    Om = sm.sketch(n, l, workload)
    w = sm.gaussian(k, workload, "w")
    GU = sm.gaussian((m, k), workload, "GU")
    GV = sm.gaussian((n, k), workload, "GV")
    return A, Om, w, GU, GV


def _gpu_grad(A, Om, k, l, q, w, GU, GV, dtype=torch.float64, use_gu=True, use_gv=True):
    Ad, Omd = dev(A, dtype), dev(Om)
    U, S, V, _ = T.lowrank_svd(Ad, k, l, q, Omd)
    gA = T.lowrank_svd_backward(Ad, k, l, q, Omd, U, S, V,
                                dev(GU) if use_gu else None, dev(w),
                                dev(GV) if use_gv else None)
    torch.cuda.synchronize()
    return host(gA).astype(np.float64)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("m,n,k,l,q", [(300, 80, 5, 8, 1), (1000, 200, 10, 16, 2),
                                       (2000, 50, 16, 24, 2), (777, 333, 7, 7, 0),
                                       (4099, 517, 20, 30, 3)])
def test_backward_vs_oracle_autograd(m, n, k, l, q):
    flush_print("case backward", m, n, k, l, q)
    A, Om, w, GU, GV = _instance(m, n, k, l, q, 80 + l)
    g = _gpu_grad(A, Om, k, l, q, w, GU, GV)
    gr, _ = grad_ref.grad_ref(A, Om, k, q, w, GU, GV)
    r = _rel(g, gr)
    flush_print(f"  rel diff vs torch autograd {r:.2e}")
    assert r <= 1e-9


def test_backward_partial_cotangents():
    A, Om, w, GU, GV = _instance(1500, 120, 6, 12, 2, 90)
    g = _gpu_grad(A, Om, 6, 12, 2, w, GU, GV, use_gu=False, use_gv=False)
    gr, _ = grad_ref.grad_ref(A, Om, 6, 2, w, 0 * GU, 0 * GV)
    assert _rel(g, gr) <= 1e-9
    g2 = _gpu_grad(A, Om, 6, 12, 2, w, GU, GV, use_gv=False)
    gr2, _ = grad_ref.grad_ref(A, Om, 6, 2, w, GU, 0 * GV)
    assert _rel(g2, gr2) <= 1e-9


def test_backward_vs_central_differences_of_gpu_forward():
    """FD instance of the differentiation workload: 2,000 x 50, sigma_j = 1/j, k=16, l=24, q=2;
    32 seeded unit directions, each with the best of three step sizes."""
    m, n, k, l, q = 2000, 50, 16, 24, 2
    A, Om, w, GU, GV = _instance(m, n, k, l, q, 5)
    g = _gpu_grad(A, Om, k, l, q, w, GU, GV)
    Omd = dev(Om)

    def loss(Ah):
        U, S, V, _ = T.lowrank_svd(dev(Ah), k, l, q, Omd)
        torch.cuda.synchronize()
        return float(np.sum(w * host(S)) + np.sum(GU * host(U)) + np.sum(GV * host(V)))

    rng = sm.rng_for(5, "fd")
    worst = 0.0
    for _ in range(32):
        E = rng.standard_normal(A.shape)
        E /= np.linalg.norm(E)
        exact = float(np.sum(g * E))
        best = min(abs((loss(A + h * E) - loss(A - h * E)) / (2 * h) - exact)
                   for h in (1e-3, 1e-4, 1e-5))
        worst = max(worst, best / max(1.0, abs(exact)))
    flush_print(f"  worst FD relative error {worst:.2e}")
    assert worst <= 1e-6


def _exact_truncated_svd_grad(A, k, w, GU, GV):
    """dL/dA of L = sum w_j s_j + <GU, U_k> + <GV, V_k> for the exact top-k SVD of A.

    Thin-SVD derivative (Townsend, "Differentiating the singular value decomposition"),
    Abar = U[(F o (U^T Ubar - Ubar^T U)) S + diag(Sbar) + S (F o (V^T Vbar - Vbar^T V))]V^T
           + (I - U U^T) Ubar S^-1 V^T,  F_ij = 1/(s_j^2 - s_i^2),
    with the cotangents zero past column k.  Entries of F between two indices >= k multiply
    zero cotangents and are set to 0 (they are 1/0 for the repeated zero singular values).
    """
    m, n = A.shape
    U, s, Vh = np.linalg.svd(A, full_matrices=False)
    V = Vh.T
    Ub = np.zeros((m, n)); Ub[:, :k] = GU
    Vb = np.zeros((n, n)); Vb[:, :k] = GV
    Sb = np.zeros(n); Sb[:k] = w
    # sign convention of the outputs (same as the library and the oracle)
    from oracle import sign_reference
    sg = np.where(sign_reference(n) @ V[:, :k] < 0, -1.0, 1.0)
    U[:, :k] *= sg
    V[:, :k] *= sg
    with np.errstate(divide="ignore"):
        F = 1.0 / (s[None, :] ** 2 - s[:, None] ** 2)
    np.fill_diagonal(F, 0.0)
    F[k:, k:] = 0.0
    J = F * (U.T @ Ub - Ub.T @ U)
    K = F * (V.T @ Vb - Vb.T @ V)
    core = J * s[None, :] + np.diag(Sb) + s[:, None] * K
    sinv = np.zeros(n); sinv[:k] = 1.0 / s[:k]
    return U @ core @ V.T + (Ub * sinv[None, :] - U @ (U.T @ (Ub * sinv[None, :]))) @ V.T


def test_backward_exact_rank_equals_exact_svd_gradient():
    """rank(A) = l: the VJP equals the gradient of the exact truncated SVD (G2)."""
    m, n, k, l, q = 1200, 90, 8, 12, 1
    A, Om, w, GU, GV = _instance(m, n, k, l, q, 91, exact_rank=True)
    g = _gpu_grad(A, Om, k, l, q, w, GU, GV)
    ge = _exact_truncated_svd_grad(A, k, w, GU, GV)
    r = _rel(g, ge)
    flush_print(f"  rel diff vs exact truncated-SVD gradient {r:.2e}")
    assert r <= 1e-8


def test_backward_workload5_full_size():
    """100,000 x 1,000 float32, sigma_j = 1/j, k=16, l=24, q=2: vs the float64 oracle."""
    spec = sm.workload_spec(5)
    m, n, k, l, q = spec["m"], spec["n"], spec["k"], spec["l"], spec["q"]
    from synth import torch_gen
    flush_print("case workload5 generate")
    A = torch_gen.planted(m, n, spec["sigma"], 5, "cuda:0", dtype=torch.float32)
    Om = torch_gen.sketch(n, l, 5, "cuda:0")
    w = sm.gaussian(k, 5, "w")
    GU = sm.gaussian((m, k), 5, "GU")
    GV = sm.gaussian((n, k), 5, "GV")
    U, S, V, _ = T.lowrank_svd(A, k, l, q, Om)
    gA = T.lowrank_svd_backward(A, k, l, q, Om, U, S, V, dev(GU), dev(w), dev(GV))
    torch.cuda.synchronize()
    assert gA.dtype == torch.float32
    flush_print("case workload5 oracle")
    gr, _ = grad_ref.grad_ref(host(A).astype(np.float64), host(Om), k, q, w, GU, GV)
    r = _rel(host(gA).astype(np.float64), gr)
    flush_print(f"  rel diff vs oracle {r:.2e}")
    assert r <= 1e-6  # gA is rounded to float32 on output


def test_autograd_function():
    m, n, k, l, q = 800, 150, 6, 10, 2
    A, Om, w, GU, GV = _instance(m, n, k, l, q, 92)
    At = dev(A).requires_grad_(True)
    U, S, V = T.LowRankSVD.apply(At, dev(Om), k, l, q)
    L = (dev(w) * S).sum() + (dev(GU) * U).sum() + (dev(GV) * V).sum()
    L.backward()
    torch.cuda.synchronize()
    gr, _ = grad_ref.grad_ref(A, Om, k, q, w, GU, GV)
    assert _rel(host(At.grad), gr) <= 1e-9


def test_backward_trailing_plateau_is_finite():
    """A spectrum that is flat past k: the sketch lies in range(A), so the trailing singular
    values of B = Q^T A repeat (equal up to rounding).  The pairs with both indices past k
    carry zero cotangents and must not turn 1/(s_j^2 - s_i^2) into NaN."""
    m, n, k, l, q = 1200, 150, 6, 14, 1
    sigma = np.concatenate([1.0 / np.arange(1, k + 1), np.full(n - k, 0.05)])
    A = sm.planted(m, n, sigma, workload=93)
    Om = sm.sketch(n, l, 93)
    w = sm.gaussian(k, 93, "w")
    GU = sm.gaussian((m, k), 93, "GU")
    GV = sm.gaussian((n, k), 93, "GV")
    g = _gpu_grad(A, Om, k, l, q, w, GU, GV)
    assert np.all(np.isfinite(g))
    gr, _ = grad_ref.grad_ref(A, Om, k, q, w, GU, GV)
    if np.all(np.isfinite(gr)):
        assert _rel(g, gr) <= 1e-8


def test_backward_strided_outputs_and_cotangents():
    """U and V sliced from wider tensors and non-contiguous cotangents: the binding passes
    the cotangents' own row strides, so the result equals the contiguous call's."""
    m, n, k, l, q = 900, 120, 5, 10, 1
    A, Om, w, GU, GV = _instance(m, n, k, l, q, 94)
    Ad, Omd = dev(A), dev(Om)
    U, S, V, _ = T.lowrank_svd(Ad, k, l, q, Omd)
    Uw = torch.zeros(m, k + 7, dtype=torch.float64, device=Ad.device)
    Vw = torch.zeros(n, k + 3, dtype=torch.float64, device=Ad.device)
    Uw[:, :k] = U
    Vw[:, :k] = V
    gUw = torch.zeros(m, 2 * k, dtype=torch.float64, device=Ad.device)
    gUw[:, ::2] = dev(GU)
    gVt = dev(np.ascontiguousarray(GV.T)).T          # n x k, column-major view
    g1 = T.lowrank_svd_backward(Ad, k, l, q, Omd, Uw[:, :k], S, Vw[:, :k], gUw[:, ::2], dev(w),
                                gVt)
    g2 = T.lowrank_svd_backward(Ad, k, l, q, Omd, U, S, V, dev(GU), dev(w), dev(GV))
    torch.cuda.synchronize()
    assert torch.equal(g1, g2)


def test_backward_rejects_bad_sketch_and_cotangents():
    m, n, k, l, q = 300, 60, 4, 8, 1
    A, Om, w, GU, GV = _instance(m, n, k, l, q, 95)
    Ad = dev(A)
    U, S, V, _ = T.lowrank_svd(Ad, k, l, q, dev(Om))
    for bad in (dev(Om).float(), dev(Om).T.contiguous().T, dev(Om)[:, :l - 1], dev(Om).cpu()):
        with pytest.raises(ValueError):
            T.lowrank_svd_backward(Ad, k, l, q, bad, U, S, V, dev(GU), dev(w), dev(GV))
    with pytest.raises(ValueError):
        T.lowrank_svd_backward(Ad, k, l, q, dev(Om), U, S, V, dev(GU)[:, :k - 1], dev(w),
                               dev(GV))
