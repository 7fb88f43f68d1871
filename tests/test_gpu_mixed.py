"""GPU parity of the mixed-precision randomized SVD (A stored float32).

Power-step products take bfloat16 inputs, the final sketch and B = Q^T A take float32
inputs; TSQR, the small SVD and the orthonormalization stay float64.  The reference is the
float64 oracle on the exactly upcast float32 matrix with the same sketch.  Gates: the
orthonormality of U and V (<= 1e-12, spectral norm) and the spectral residual
||A - U S V^T||_2 within 1e-6 (relative to sigma_1) of the oracle's.
"""
import numpy as np
import pytest
import torch

from oracle import checks
from oracle.lowrank_ref import lowrank_ref
from synth import matrices as sm

from gpu_util import col_sin, dev, flush_print, host, ortho_gpu, residual_gpu, sigma_rel

pytestmark = pytest.mark.gpu

T = pytest.importorskip("paper_1612_08709_amd")


def _workload4_like(m, n, workload, r=None):
    sigma = np.exp(-np.arange(1, (r or min(m, n)) + 1) / 15.0)
    return sm.planted(m, n, sigma, workload=workload, noise=1e-5).astype(np.float32), sigma


def _run_mixed(A32, Om, k, q, prec):
    U, S, V, info = T.lowrank_svd(dev(A32), k, Om.shape[1], q, dev(Om), prec=prec)
    torch.cuda.synchronize()
    return host(U), host(S), host(V), info


@pytest.mark.parametrize("m,n,k,l,q", [(20000, 1500, 50, 60, 3), (3001, 517, 16, 24, 2),
                                       (5000, 640, 10, 30, 0), (4099, 333, 8, 12, 1)])
def test_mixed_vs_oracle_on_upcast(m, n, k, l, q):
    flush_print("case mixed", m, n, k, l, q)
    A32, _ = _workload4_like(m, n, 70 + l, r=min(m, n, 300))
    Om = sm.sketch(n, l, 70 + l)
    U, S, V, info = _run_mixed(A32, Om, k, q, T.PREC_MIXED)
    A64 = A32.astype(np.float64)
    Ur, Sr, Vr = lowrank_ref(A64, Om, k, q)
    assert checks.ortho_spec(U) <= 1e-12 and checks.ortho_spec(V) <= 1e-12
    e = checks.spectral_residual(A64, U, S, V, tol=1e-9)
    er = checks.spectral_residual(A64, Ur, Sr, Vr, tol=1e-9)
    flush_print(f"  residual mixed {e:.6e} oracle {er:.6e} diff {abs(e - er):.2e}; "
                f"sigma rel {sigma_rel(S, Sr):.2e}")
    assert abs(e - er) <= 1e-6 * Sr[0]
    assert sigma_rel(S, Sr) < 1e-3


def test_mixed_matches_fp64_gpu_path():
    """Same float32 A and sketch: mixed vs the all-float64 GPU path, residual within 1e-6."""
    A32, _ = _workload4_like(30000, 2000, 75, r=400)
    Om = sm.sketch(2000, 60, 75)
    Um, Sm, Vm, _ = _run_mixed(A32, Om, 50, 3, T.PREC_MIXED)
    Uf, Sf, Vf, _ = _run_mixed(A32, Om, 50, 3, T.PREC_FP64)
    A64 = A32.astype(np.float64)
    em = checks.spectral_residual(A64, Um, Sm, Vm, tol=1e-9)
    ef = checks.spectral_residual(A64, Uf, Sf, Vf, tol=1e-9)
    assert abs(em - ef) <= 1e-6 * Sf[0]
    assert checks.ortho_spec(Um) <= 1e-12 and checks.ortho_spec(Uf) <= 1e-13


def test_mixed_requires_float32_storage():
    A = torch.zeros(1000, 100, dtype=torch.float64, device="cuda:0")
    with pytest.raises(ValueError):
        T.lowrank_svd(A, 4, 8, 1, None, prec=T.PREC_MIXED)


def test_mixed_deterministic_bitwise():
    A32, _ = _workload4_like(8000, 700, 76, r=200)
    Om = dev(sm.sketch(700, 30, 76))
    Ad = dev(A32)
    r1 = [host(x) for x in T.lowrank_svd(Ad, 20, 30, 2, Om, prec=T.PREC_MIXED)[:3]]
    r2 = [host(x) for x in T.lowrank_svd(Ad, 20, 30, 2, Om, prec=T.PREC_MIXED)[:3]]
    for a, b in zip(r1, r2):
        assert np.array_equal(a, b)


def test_bf16_copy_of_a_is_bitwise_neutral():
    """The power steps reading the bfloat16 copy of A give bit-identical results to
    rounding the float32 A in every pass (TSSVD_FLAG_NO_A_COPY); odd n and ragged m."""
    A32, _ = _workload4_like(9001, 777, 78, r=250)
    Om = dev(sm.sketch(777, 36, 78))
    Ad = dev(A32)
    a = [host(x) for x in T.lowrank_svd(Ad, 24, 36, 3, Om, prec=T.PREC_MIXED)[:3]]
    b = [host(x) for x in T.lowrank_svd(Ad, 24, 36, 3, Om, prec=T.PREC_MIXED, flags=2)[:3]]
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_f32_mfma_final_flag_same_result_class():
    """The float32-MFMA final products (flag) and the default exact bf16 split agree."""
    A32, _ = _workload4_like(12000, 900, 77, r=300)
    Om = dev(sm.sketch(900, 40, 77))
    Ad = dev(A32)
    a = T.lowrank_svd(Ad, 30, 40, 2, Om, prec=T.PREC_MIXED)
    b = T.lowrank_svd(Ad, 30, 40, 2, Om, prec=T.PREC_MIXED, flags=1)
    torch.cuda.synchronize()
    A64 = A32.astype(np.float64)
    ea = checks.spectral_residual(A64, host(a[0]), host(a[1]), host(a[2]), tol=1e-9)
    eb = checks.spectral_residual(A64, host(b[0]), host(b[1]), host(b[2]), tol=1e-9)
    assert abs(ea - eb) <= 1e-6 * host(a[1])[0]
    assert sigma_rel(host(a[1]), host(b[1])) < 1e-5


def test_workload4_full_size():
    """500,000 x 8,000 float32 (16 GB), sigma_j = exp(-j/15) (j <= 600) + 1e-5 noise, k=50,
    l=60, q=3, in the launch configuration the benchmark times.  Properties that hold at
    any size: orthonormality of U and V (<= 1e-12), sigma within 1e-6 of the all-FP64 GPU
    path on the same bytes and sketch, the spectral residual within 1e-6 sigma_1 of the
    FP64 path's, and the leading sigma near the planted ones (the noise moves them by
    about ||N||_2^2 / sigma_j, ||N||_2 ~ 7e-3)."""
    from synth import torch_gen
    spec = sm.workload_spec(4)
    m, n, k, l, q = spec["m"], spec["n"], spec["k"], spec["l"], spec["q"]
    flush_print("case workload4 generate")
    A = torch_gen.planted(m, n, spec["sigma"], 4, "cuda:0", noise=spec.get("noise", 0.0),
                          dtype=torch.float32, rank=spec.get("rank"))
    Om = torch_gen.sketch(n, l, 4, "cuda:0")
    flush_print("case workload4 mixed")
    Um, Sm, Vm, _ = T.lowrank_svd(A, k, l, q, Om, prec=T.PREC_MIXED)
    flush_print("case workload4 fp64")
    Uf, Sf, Vf, _ = T.lowrank_svd(A, k, l, q, Om, prec=T.PREC_FP64)
    torch.cuda.synchronize()
    assert ortho_gpu(Um) <= 1e-12 and ortho_gpu(Vm) <= 1e-12
    assert ortho_gpu(Uf) <= 1e-13 and ortho_gpu(Vf) <= 1e-13
    sm_, sf_ = host(Sm), host(Sf)
    assert np.all(np.diff(sm_) <= 0)
    assert sigma_rel(sm_, sf_) <= 1e-6
    assert sigma_rel(sm_[:10], np.asarray(spec["sigma"])[:10]) <= 1e-3
    flush_print("case workload4 residuals")
    em = residual_gpu(A, Um, Sm, Vm)
    ef = residual_gpu(A, Uf, Sf, Vf)
    flush_print(f"  residual mixed {em:.9e} fp64 {ef:.9e} diff {abs(em - ef):.2e}")
    assert abs(em - ef) <= 1e-6 * sf_[0]
    # Algorithm 6 gives V diag(S) = A^T U exactly (A^T Q P_k = Q_B R_B P_k = Q_B W_k S_k);
    # sampled rows j of V S against FP64 dot products of column j of A with U on the host
    cols = np.sort(np.random.default_rng(4).choice(n, 12, replace=False))
    Acols = host(A[:, torch.from_numpy(cols).to(A.device)]).astype(np.float64)   # m x 12
    for name, U_, S_, V_, tol in (("mixed", Um, sm_, Vm, 1e-6), ("fp64", Uf, sf_, Vf, 1e-12)):
        ref = Acols.T @ host(U_)                                                   # 12 x k
        got = host(V_)[cols] * S_
        err = float(np.max(np.abs(got - ref))) / sf_[0]
        flush_print(f"  sampled V S vs A^T U ({name}): {err:.2e} of sigma_1")
        assert err <= tol


def test_workload4_full_size_vs_oracle():
    """500,000 x 8,000 float32 at full size against the float64 oracle run on the same bytes
    (exact upcast) with the same sketch: the mixed-precision residual ||A - U S V^T||_2 within
    1e-6 sigma_1 of the oracle's, sigma within 1e-6 relative, the all-FP64 GPU path's sigma
    within 1e-11 relative, and both orthonormal (<= 1e-12 mixed, <= 1e-13 FP64)."""
    from synth import torch_gen
    spec = sm.workload_spec(4)
    m, n, k, l, q = spec["m"], spec["n"], spec["k"], spec["l"], spec["q"]
    flush_print("case workload4 oracle: generate")
    A = torch_gen.planted(m, n, spec["sigma"], 4, "cuda:0", noise=spec.get("noise", 0.0),
                          dtype=torch.float32, rank=spec.get("rank"))
    Om = torch_gen.sketch(n, l, 4, "cuda:0")
    Um, Sm, Vm, _ = T.lowrank_svd(A, k, l, q, Om, prec=T.PREC_MIXED)
    Uf, Sf, Vf, _ = T.lowrank_svd(A, k, l, q, Om, prec=T.PREC_FP64)
    torch.cuda.synchronize()
    flush_print("case workload4 oracle: lowrank_ref on the host")
    Ur, Sr, Vr = lowrank_ref(host(A), host(Om), k, q)
    sm_, sf_ = host(Sm), host(Sf)
    flush_print(f"  sigma rel: mixed {sigma_rel(sm_, Sr):.2e}, fp64 {sigma_rel(sf_, Sr):.2e}")
    assert sigma_rel(sm_, Sr) <= 1e-6
    assert sigma_rel(sf_, Sr) <= 1e-11
    vs = col_sin(host(Vf), Vr)
    flush_print(f"  fp64 V columns vs oracle: max sin {vs.max():.2e}")
    assert vs.max() <= 1e-8
    assert ortho_gpu(Um) <= 1e-12 and ortho_gpu(Vm) <= 1e-12
    assert ortho_gpu(Uf) <= 1e-13 and ortho_gpu(Vf) <= 1e-13
    flush_print("case workload4 oracle: residuals")
    Urd, Srd, Vrd = dev(Ur), dev(Sr), dev(Vr)
    er = residual_gpu(A, Urd, Srd, Vrd)
    em = residual_gpu(A, Um, Sm, Vm)
    flush_print(f"  residual mixed {em:.9e} oracle {er:.9e} diff {abs(em - er):.2e}")
    assert abs(em - er) <= 1e-6 * Sr[0]
