"""GPU parity of the Gram-based route (TSSVD_FLAG_GRAM): Algorithms 3 and 4 (tssvd) and
Algorithm 8 (lowrank_svd) through the C ABI vs the CPU oracle on the same inputs.

The Gram matrix squares the condition number, so inputs are planted with moderate
conditioning (kappa <= 1e2) where both sides resolve every triplet to ~1e-12; the discard
cases plant spectra that straddle sqrt(wp) with wide margins, so both sides keep the same
rank."""
import numpy as np
import pytest
import torch

from oracle import checks
from oracle.gram_ref import gram_svd_ref, lowrank_gram_ref
from synth import matrices as sm

from gpu_util import col_sin, dev, flush_print, host, sigma_rel

pytestmark = pytest.mark.gpu

T = pytest.importorskip("paper_1612_08709_amd")


def _planted(m, n, cond, workload):
    sigma = np.logspace(0, -np.log10(cond), n)
    return sm.planted(m, n, sigma, workload=workload), sigma


def _tssvd(A, dtype=torch.float64, **kw):
    U, S, V, info = T.tssvd(dev(A, dtype), flags=T.FLAG_GRAM, **kw)
    torch.cuda.synchronize()
    return host(U), host(S), host(V), info


@pytest.mark.parametrize("m,n", [(300, 5), (1000, 17), (4099, 33), (5000, 64), (3001, 65),
                                 (20000, 100)])
@pytest.mark.parametrize("ortho", [T.ORTHO_ONCE, T.ORTHO_TWICE])
def test_gram_tssvd_vs_oracle(m, n, ortho):
    flush_print("case gram tssvd", m, n, ortho)
    A, sigma = _planted(m, n, 1e2, workload=300 + n)
    U, S, V, info = _tssvd(A, ortho=ortho)
    Ur, Sr, Vr, r = gram_svd_ref(A, double=(ortho != T.ORTHO_ONCE))
    assert r == n and info["rank"] == n
    assert sigma_rel(S, Sr) < 1e-11 and sigma_rel(S, sigma) < 1e-10
    assert np.max(col_sin(U, Ur)) < 1e-9 and np.max(col_sin(V, Vr)) < 1e-9
    np.testing.assert_allclose(U, Ur, atol=1e-9)
    np.testing.assert_allclose(V, Vr, atol=1e-9)
    assert np.all(np.diff(S) <= 0)
    if ortho == T.ORTHO_TWICE:
        assert checks.ortho_spec(U) < 1e-13 and checks.ortho_spec(V) < 1e-13


def test_gram_tssvd_float32_storage():
    A, _ = _planted(6000, 40, 30.0, workload=341)
    A32 = A.astype(np.float32)
    U, S, V, info = _tssvd(A32, dtype=torch.float32, ortho=T.ORTHO_TWICE)
    Ur, Sr, Vr, _ = gram_svd_ref(A32.astype(np.float64), double=True)
    assert sigma_rel(S, Sr) < 1e-11
    assert np.max(col_sin(U, Ur)) < 1e-9 and np.max(col_sin(V, Vr)) < 1e-9


@pytest.mark.parametrize("ortho", [T.ORTHO_ONCE, T.ORTHO_TWICE])
def test_gram_tssvd_discard_at_sqrt_wp(ortho):
    """sigma = 10^0 .. 10^-9: with wp = 1e-11 (cut 3.16e-6) exactly six triplets are kept;
    the rest are zero columns with sigma = 0 on both sides."""
    sigma = 10.0 ** -np.arange(10)
    A = sm.planted(3000, 10, sigma, workload=342)
    U, S, V, info = _tssvd(A, ortho=ortho, working_precision=1e-11)
    Ur, Sr, Vr, r = gram_svd_ref(A, wp=1e-11, double=(ortho != T.ORTHO_ONCE))
    assert r == 6 and info["rank"] == 6
    np.testing.assert_allclose(S[:6], Sr[:6], rtol=1e-6)
    assert np.all(S[6:] == 0) and np.all(U[:, 6:] == 0) and np.all(V[:, 6:] == 0)
    assert np.max(col_sin(U[:, :6], Ur[:, :6])) < 1e-5
    assert np.max(col_sin(V[:, :6], Vr[:, :6])) < 1e-5


def _lowrank(A, Om, k, q, dtype=torch.float64, **kw):
    U, S, V, info = T.lowrank_svd(dev(A, dtype), k, Om.shape[1], q, dev(Om), flags=T.FLAG_GRAM,
                                  **kw)
    torch.cuda.synchronize()
    return host(U), host(S), host(V), info


@pytest.mark.parametrize("m,n,k,l,q", [(3000, 400, 20, 30, 2), (1000, 37, 5, 8, 0),
                                       (4097, 1000, 16, 24, 2), (2500, 700, 50, 60, 3),
                                       (6000, 700, 60, 100, 1)])
def test_gram_lowrank_vs_oracle(m, n, k, l, q):
    flush_print("case gram lowrank", m, n, k, l, q)
    A = sm.planted(m, n, 1.0 / np.arange(1, min(m, n) + 1), workload=350 + l)
    Om = sm.sketch(n, l, 350 + l)
    U, S, V, info = _lowrank(A, Om, k, q)
    Ur, Sr, Vr = lowrank_gram_ref(A, Om, k, q)
    assert sigma_rel(S, Sr) < 1e-10
    assert np.max(col_sin(U, Ur)) < 1e-7 and np.max(col_sin(V, Vr)) < 1e-7
    np.testing.assert_allclose(U, Ur, atol=1e-7)
    np.testing.assert_allclose(V, Vr, atol=1e-7)
    assert checks.ortho_spec(U) < 1e-13 and checks.ortho_spec(V) < 1e-13


@pytest.mark.parametrize("l,err", [(20, 4.83e-7), (10, 2.15e-7)])
def test_gram_lowrank_reproduces_printed_error(l, err):
    """Algorithm 8 on the paper's DCT test matrix (m = 10,000, n = 2,000, i = 2, wp = 1e-11):
    the printed spectral error (the first planted sigma below sqrt(wp)) and the oracle's
    kept triplets."""
    A = sm.dct_planted(10_000, 2_000, sm.paper_spectrum(l))
    Om = sm.gaussian((2_000, l), 92, "omega", 0)
    U, S, V, info = _lowrank(A, Om, l, 2, working_precision=1e-11)
    Ur, Sr, Vr = lowrank_gram_ref(A, Om, l, 2, wp=1e-11)
    r = int(np.count_nonzero(Sr))
    assert info["rank"] == r and np.count_nonzero(S) == r
    e = checks.spectral_residual(A, U, S, V, iters=20)
    assert abs(e - err) <= 0.01 * err, e
    np.testing.assert_allclose(S[:r], Sr[:r], rtol=1e-9, atol=1e-14 * Sr[0])  # eps sigma_1
    assert checks.ortho_spec(U, r) < 1e-13 and checks.ortho_spec(V, r) < 1e-13


def test_gram_lowrank_mixed_precision():
    """Mixed precision (A float32, bfloat16 power steps): residual within 1e-6 sigma_1 of the
    float64 oracle's on the upcast matrix."""
    sigma = np.exp(-np.arange(1, 301) / 15.0)
    A32 = sm.planted(20000, 1500, sigma, workload=360, noise=1e-5).astype(np.float32)
    Om = sm.sketch(1500, 60, 360)
    U, S, V, info = _lowrank(A32, Om, 50, 3, dtype=torch.float32, prec=T.PREC_MIXED)
    A64 = A32.astype(np.float64)
    Ur, Sr, Vr = lowrank_gram_ref(A64, Om, 50, 3)
    assert checks.ortho_spec(U) <= 1e-12 and checks.ortho_spec(V) <= 1e-12
    e = checks.spectral_residual(A64, U, S, V, tol=1e-9)
    er = checks.spectral_residual(A64, Ur, Sr, Vr, tol=1e-9)
    flush_print(f"  gram mixed residual {e:.6e} oracle {er:.6e}")
    assert abs(e - er) <= 1e-6 * Sr[0]
    assert sigma_rel(S, Sr) < 1e-3
