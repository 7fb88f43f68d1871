"""GPU parity: lowrank_svd (Algorithm 7) through the C ABI vs the CPU oracle (same sketch)."""
import numpy as np
import pytest
import torch

from oracle import checks
from oracle.lowrank_ref import lowrank_ref
from oracle.philox import philox_normal
from synth import matrices as sm

from gpu_util import col_sin, dev, flush_print, host, sigma_rel

pytestmark = pytest.mark.gpu

T = pytest.importorskip("paper_1612_08709_amd")


def _compare(A, Om, k, q, dtype=torch.float64, s_tol=1e-11, v_tol=1e-8, **kw):
    U, S, V, info = T.lowrank_svd(dev(A, dtype), k, Om.shape[1], q, dev(Om), **kw)
    torch.cuda.synchronize()
    U, S, V = host(U), host(S), host(V)
    Aref = A.astype(np.float32).astype(np.float64) if dtype == torch.float32 else A
    Ur, Sr, Vr = lowrank_ref(Aref, Om, k, q)
    assert sigma_rel(S, Sr) < s_tol
    assert np.max(col_sin(U, Ur)) < v_tol and np.max(col_sin(V, Vr)) < v_tol
    np.testing.assert_allclose(V, Vr, atol=v_tol)
    np.testing.assert_allclose(U, Ur, atol=v_tol)
    assert checks.ortho_spec(U) < 1e-13 and checks.ortho_spec(V) < 1e-13
    return U, S, V, info


@pytest.mark.parametrize("m,n,k,l,q", [(3000, 400, 20, 30, 2), (1000, 37, 5, 8, 0),
                                       (4097, 1000, 16, 24, 2), (2500, 700, 50, 60, 3),
                                       (600, 500, 10, 10, 1), (6000, 700, 100, 100, 1)])
def test_small_vs_oracle(m, n, k, l, q):
    flush_print("case lowrank", m, n, k, l, q)
    A = sm.planted(m, n, 1.0 / np.arange(1, min(m, n) + 1), workload=50 + l)
    Om = sm.sketch(n, l, 50 + l)
    _compare(A, Om, k, q)


def test_float32_storage():
    A = sm.planted(5000, 300, 1.0 / np.arange(1, 301), workload=61)
    Om = sm.sketch(300, 24, 61)
    _compare(A, Om, 16, 2, dtype=torch.float32)


def test_exact_rank_recovers_planted_sigma():
    m, n, l, k = 8000, 600, 20, 12
    sigma = np.logspace(0, -3, l)
    A = sm.planted(m, n, sigma, workload=62)
    U, S, V, info = T.lowrank_svd(dev(A), k, l, 1, dev(sm.sketch(n, l, 62)))
    torch.cuda.synchronize()
    assert sigma_rel(host(S), sigma[:k]) < 1e-12


@pytest.mark.parametrize("q", [1, 2])
def test_rank_below_sketch_width(q):
    """rank(A) = 6 < l = 12: R of every sketch is singular, so the intermediate bases take
    the explicit Householder path; the top k <= rank triplets still match the oracle."""
    m, n, r, k, l = 3000, 300, 6, 5, 12
    A = sm.planted(m, n, np.linspace(1.0, 0.3, r), workload=64)
    Om = sm.sketch(n, l, 64)
    _compare(A, Om, k, q)


def test_ill_conditioned_sketch():
    """sigma_j = 10^(-0.45 (j-1)): sigma_16 / sigma_1 ~ 2e-7, so ||R||_F ||R^-1||_F exceeds
    the threshold of the R^-1 basis and the Householder basis is used; parity as usual."""
    m, n, k, l = 4000, 200, 8, 16
    sig = 10.0 ** (-0.45 * np.arange(n))
    A = sm.planted(m, n, sig, workload=65)
    _compare(A, sm.sketch(n, l, 65), k, 2)


def test_device_philox_sketch_matches_oracle_generator():
    """Omega = NULL: the sketch comes from Philox4x32-10 on the device (seeded)."""
    m, n, k, l, q = 3000, 500, 10, 16, 1
    A = sm.planted(m, n, 1.0 / np.arange(1, n + 1), workload=63)
    seed = 0x1234_5678_9ABC_DEF0
    U, S, V, info = T.lowrank_svd(dev(A), k, l, q, None, seed=seed)
    torch.cuda.synchronize()
    Ur, Sr, Vr = lowrank_ref(A, philox_normal(n, l, seed), k, q)
    assert sigma_rel(host(S), Sr) < 1e-10
    assert np.max(col_sin(host(V), Vr)) < 1e-7


def test_deterministic_bitwise():
    A = sm.planted(20000, 800, 1.0 / np.arange(1, 801), workload=64)
    Om = dev(sm.sketch(800, 30, 64))
    Ad = dev(A)
    r1 = [host(x) for x in T.lowrank_svd(Ad, 20, 30, 2, Om)[:3]]
    r2 = [host(x) for x in T.lowrank_svd(Ad, 20, 30, 2, Om)[:3]]
    for a, b in zip(r1, r2):
        assert np.array_equal(a, b)


def test_workload2_full_size():
    """200,000 x 2,000 FP64, sigma_j = 1/j + 1e-8 noise, k=20, l=30, q=2 (generated on the GPU)."""
    from synth import torch_gen
    spec = sm.workload_spec(2)
    m, n, k, l, q = spec["m"], spec["n"], spec["k"], spec["l"], spec["q"]
    flush_print("case workload2 generate")
    A = torch_gen.planted(m, n, spec["sigma"], 2, "cuda:0", noise=spec["noise"])
    Om = torch_gen.sketch(n, l, 2, "cuda:0")
    flush_print("case workload2 run")
    U, S, V, info = T.lowrank_svd(A, k, l, q, Om)
    torch.cuda.synchronize()
    Ah, Omh = host(A), host(Om)
    del A
    flush_print("case workload2 oracle")
    Ur, Sr, Vr = lowrank_ref(Ah, Omh, k, q)
    U, S, V = host(U), host(S), host(V)
    assert sigma_rel(S, Sr) < 1e-11
    assert np.max(col_sin(V, Vr)) < 1e-8 and np.max(col_sin(U, Ur)) < 1e-8
    assert checks.ortho_spec(U) < 1e-13 and checks.ortho_spec(V) < 1e-13
    e = checks.spectral_residual(Ah, U, S, V, iters=20)
    er = checks.spectral_residual(Ah, Ur, Sr, Vr, iters=20)
    assert abs(e - er) <= 1e-10


@pytest.mark.parametrize("mode", ["once", "auto", "twice"])
@pytest.mark.parametrize("m,n,k,l,q", [(5000, 300, 20, 40, 2), (3000, 200, 10, 12, 0)])
def test_last_basis_orthonormalization_modes(mode, m, n, k, l, q):
    """The last basis of Algorithm 5: ONCE takes the TSQR's Householder Q; AUTO and TWICE take
    Algorithm 2's two orthonormalizations as CholeskyQR passes (the second one gated in
    AUTO, always run in TWICE).  Every mode matches the oracle and returns U and V
    orthonormal to 1e-13."""
    flush_print("case lowrank last basis", mode, m, n, k, l, q)
    ortho = {"once": T.ORTHO_ONCE, "auto": T.ORTHO_AUTO, "twice": T.ORTHO_TWICE}[mode]
    A = sm.planted(m, n, 1.0 / np.arange(1, min(m, n) + 1), workload=70 + l)
    Om = sm.sketch(n, l, 70 + l)
    U, S, V, info = _compare(A, Om, k, q, ortho=ortho)
    if mode == "twice":
        assert info["reorth"] == 1
    if mode == "once":
        assert info["reorth"] == 0
