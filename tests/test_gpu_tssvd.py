"""GPU parity: tsqr and tssvd (Algorithms 1-2) through the C ABI vs the CPU oracle."""
import numpy as np
import pytest
import torch

from oracle import checks
from oracle.tssvd_ref import tssvd_ref
from synth import matrices as sm

from gpu_util import col_sin, dev, flush_print, host, sigma_rel

pytestmark = pytest.mark.gpu

T = pytest.importorskip("paper_1612_08709_amd")


def _graded(m, n, seed, cond=1e4):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((m, n)) * np.logspace(0, -np.log10(cond), n)


def _run(A64, dtype=torch.float64, **kw):
    A = dev(A64, dtype)
    U, S, V, info = T.tssvd(A, **kw)
    torch.cuda.synchronize()
    return host(U), host(S), host(V), info


def test_workload1_planted_spectrum():
    """10,000 x 20, sigma_j = 10^(-(j-1)/4): planted sigma to 1e-12 relative, U/V vs oracle."""
    spec = sm.workload_spec(1)
    A = sm.planted(spec["m"], spec["n"], spec["sigma"], workload=1)
    flush_print("case workload1", A.shape)
    U, S, V, info = _run(A)
    Ur, Sr, Vr, _ = tssvd_ref(A)
    assert sigma_rel(S, spec["sigma"]) < 1e-12
    assert sigma_rel(S, Sr) < 1e-12
    assert np.max(col_sin(U, Ur)) < 1e-9 and np.max(col_sin(V, Vr)) < 1e-9
    np.testing.assert_allclose(U, Ur, atol=1e-9)
    np.testing.assert_allclose(V, Vr, atol=1e-9)
    assert checks.ortho_spec(U) < 1e-13 and checks.ortho_spec(V) < 1e-13
    assert info["numstat"] == 0 and info["rank"] == 20


@pytest.mark.parametrize("m,n", [(1, 1), (16, 16), (17, 17), (300, 5), (257, 16), (1000, 17),
                                 (4099, 33), (5000, 64), (3001, 65), (20000, 100)])
@pytest.mark.parametrize("ortho", [T.ORTHO_ONCE, T.ORTHO_TWICE])
def test_shapes_vs_oracle(m, n, ortho):
    flush_print("case shapes", m, n, ortho)
    A = _graded(m, n, seed=m * 131 + n)
    U, S, V, info = _run(A, ortho=ortho)
    Ur, Sr, Vr, _ = tssvd_ref(A)
    assert sigma_rel(S, Sr) < 1e-12
    assert np.max(col_sin(U, Ur)) < 1e-9
    assert np.max(col_sin(V, Vr)) < 1e-9
    np.testing.assert_allclose(U, Ur, atol=1e-9)
    assert checks.ortho_spec(U) < 1e-13 and checks.ortho_spec(V) < 1e-13
    assert np.all(np.diff(S) <= 0)
    if ortho == T.ORTHO_TWICE:
        assert info["reorth"] == 1


def test_float32_storage_is_exact_upcast():
    """A stored in float32: the result is the SVD of the stored values (oracle on the upcast)."""
    A32 = _graded(6000, 40, seed=5).astype(np.float32)
    U, S, V, _ = _run(A32.astype(np.float64), dtype=torch.float32)
    Ur, Sr, Vr, _ = tssvd_ref(A32.astype(np.float64))
    assert sigma_rel(S, Sr) < 1e-12
    np.testing.assert_allclose(U, Ur, atol=1e-9)


def test_auto_mode_measures_and_skips():
    """AUTO: Householder U is orthonormal to working precision, so the second pass is skipped."""
    A = _graded(8000, 30, seed=8)
    U, S, V, info = _run(A, ortho=T.ORTHO_AUTO)
    assert 0.0 <= info["ortho"] < 1e-13 and info["reorth"] == 0
    U2, S2, V2, info2 = _run(A, ortho=T.ORTHO_AUTO, reorth_tol=1e-300)
    assert info2["reorth"] == 1
    assert sigma_rel(S2, S) < 1e-13 and np.max(col_sin(U2, U)) < 1e-10


@pytest.mark.parametrize("m,n", [(20000, 100), (30000, 48)])
def test_auto_gate_tests_the_spectral_norm(m, n):
    """The AUTO gate decides on ||U^T U - I||_2 (by Cholesky tests of (1 + tol) I - G and
    G - (1 - tol) I), not on the reported Frobenius norm: a tolerance between the two skips the
    second pass (U bitwise that of ONCE), one below the spectral norm runs it."""
    A = _graded(m, n, seed=21)
    U1, S1, V1, _ = _run(A, ortho=T.ORTHO_ONCE)
    E = U1.T @ U1 - np.eye(n)
    spec, frob = float(np.linalg.norm(E, 2)), float(np.linalg.norm(E))
    flush_print(f"case gate m={m} n={n}: ||E||_2 {spec:.2e}  ||E||_F {frob:.2e}")
    assert frob > 2.0 * spec  # room for a tolerance strictly between them
    tol = (spec * frob) ** 0.5
    U, S, V, info = _run(A, ortho=T.ORTHO_AUTO, reorth_tol=tol)
    assert info["reorth"] == 0 and info["ortho"] > tol
    assert np.array_equal(U, U1) and np.array_equal(S, S1)
    U2, S2, V2, info2 = _run(A, ortho=T.ORTHO_AUTO, reorth_tol=spec / 3.0)
    assert info2["reorth"] == 1
    assert checks.ortho_spec(U2) < 1e-13 and sigma_rel(S2, S1) < 1e-13


def test_rank_deficient_zero_columns():
    """Exactly rank-deficient input, wp = 0: the nonzero part matches; no NaN."""
    A = _graded(2000, 12, seed=9)
    A[:, 3] = 0.0
    A[:, 7] = 2.0 * A[:, 1]
    U, S, V, info = _run(A)
    Ur, Sr, Vr, _ = tssvd_ref(A)
    assert np.all(np.isfinite(U)) and np.all(np.isfinite(V))
    assert sigma_rel(S[:10], Sr[:10]) < 1e-12
    assert S[10] < 1e-14 * S[0] and S[11] < 1e-14 * S[0]
    assert info["numstat"] == 0
    live = S > 0
    assert np.all(U[:, ~live] == 0)  # an exact zero sigma has a zero left vector
    assert checks.ortho_spec(U[:, live]) < 1e-13 and checks.ortho_spec(V[:, live]) < 1e-13


def test_discard_rule_matches_oracle():
    """Working precision 1e-11: rows of R below wp |R_11| dropped, same rank as the oracle."""
    sigma = np.concatenate([np.logspace(0, -5, 9), np.full(3, 1e-15)])
    A = sm.planted(3000, 12, sigma, workload=41)
    U, S, V, info = _run(A, working_precision=1e-11)
    Ur, Sr, Vr, r = tssvd_ref(A, wp=1e-11, double=False)
    assert info["rank"] == r == 9
    assert sigma_rel(S[:r], Sr[:r]) < 1e-11
    assert np.all(S[r:] == 0) and np.all(U[:, r:] == 0) and np.all(V[:, r:] == 0)
    assert checks.ortho_spec(U, r) < 1e-13


@pytest.mark.parametrize("n,kept", [(80, 70), (64, 50)])
def test_discard_rule_wide_factors(n, kept):
    """The discard rule on the transposed Jacobi input at both kernel widths (n = 80: 64
    lane groups; n = 64: 32): `kept` planted values from 1 to 1e-5, the rest 1e-15."""
    sigma = np.concatenate([np.logspace(0, -5, kept), np.full(n - kept, 1e-15)])
    A = sm.planted(4000, n, sigma, workload=42 + n)
    U, S, V, info = _run(A, working_precision=1e-11)
    Ur, Sr, Vr, r = tssvd_ref(A, wp=1e-11, double=False)
    assert info["rank"] == r == kept
    assert sigma_rel(S[:r], Sr[:r]) < 1e-11
    assert np.max(col_sin(U[:, :r], Ur[:, :r])) < 1e-6 and np.max(col_sin(V[:, :r], Vr[:, :r])) < 1e-6
    assert np.all(S[r:] == 0) and np.all(U[:, r:] == 0) and np.all(V[:, r:] == 0)
    assert checks.ortho_spec(U, r) < 1e-13


def test_deterministic_bitwise():
    A = _graded(50000, 48, seed=11)
    a = _run(A)
    b = _run(A)
    for x, y in zip(a[:3], b[:3]):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("m,n", [(128, 128), (5000, 7), (70001, 100), (33, 33), (255, 40),
                                 (256, 48), (257, 64), (3001, 97), (20000, 113),
                                 (600001, 100), (70001, 128), (5000, 128), (4999, 64)])
def test_tsqr_factor_vs_householder(m, n):
    """R equals LAPACK's Householder R up to row signs; Q R = A; Q^T Q = I.  The shapes
    with n >= 33 run the blocked leaf (128-row blocks, 16-column panels): one partial block,
    exactly one block and one row past it, a last panel holding one real column (n = 97,
    113), and chains of several blocks per workgroup (m = 70,001 and 600,001).  m = 5000 and
    4999 end in a block of 8 and 7 rows that starts a chain, so its columns past the 8th are
    rounding residue that shrinks by the unit roundoff with each use of the 8-row space and
    squares to subnormal numbers on the way to zero (the reflector scalars must stay finite
    there)."""
    flush_print("case tsqr", m, n)
    A = _graded(m, n, seed=m + n)
    Q, R = T.tsqr(dev(A))
    torch.cuda.synchronize()
    Q, R = host(Q), host(R)
    _, Rn = np.linalg.qr(A)
    d = np.sign(np.diag(R)) * np.sign(np.diag(Rn))
    np.testing.assert_allclose(R * d[:, None], Rn, atol=1e-12 * np.abs(Rn).max())
    assert np.all(np.tril(R, -1) == 0)
    np.testing.assert_allclose(Q @ R, A, atol=1e-12 * np.abs(A).max())
    assert checks.ortho_spec(Q) < 1e-13


@pytest.mark.parametrize("m,n", [(9000, 20), (70001, 100)])
def test_tsqr_float32_input(m, n):
    A32 = _graded(m, n, seed=3).astype(np.float32)
    Q, R = T.tsqr(dev(A32))
    torch.cuda.synchronize()
    Q, R = host(Q), host(R)
    np.testing.assert_allclose(Q @ R, A32.astype(np.float64), atol=1e-12)
    assert checks.ortho_spec(Q) < 1e-13


def _workload3(dtype):
    from synth import torch_gen
    spec = sm.workload_spec(3)
    flush_print("case workload3 generate", dtype)
    A = torch_gen.planted(spec["m"], spec["n"], spec["sigma"], 3, "cuda:0", dtype=dtype)
    return spec, A


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_workload3_full_size(dtype):
    """4,000,000 x 100 (sigma log-spaced 1 .. 1e-6), stored float64 or float32, in the mode
    the benchmark times (second orthonormalization when the measured ||U^T U - I||_F exceeds
    1e-13).  Properties at full size: ||U^T U - I||_2 <= 1e-13 and ||V^T V - I||_2 <= 1e-13
    with the Gram summed pairwise, sigma against the planted values (float64 storage; float32
    rounding moves the small ones), and, for sampled rows i, U[i, :] diag(S) = A[i, :] V
    (A = U S V^T) against FP64 dot products on the host."""
    spec, A = _workload3(dtype)
    m, n = spec["m"], spec["n"]
    U, S, V, info = T.tssvd(A)
    torch.cuda.synchronize()
    from gpu_util import ortho_gpu
    ou, ov = ortho_gpu(U), ortho_gpu(V)
    s_, v_ = host(S), host(V)
    flush_print(f"  ortho U {ou:.2e} V {ov:.2e} (second pass {info['reorth']}, first-pass "
                f"||.||_F {info['ortho']:.2e}); sigma rel vs planted "
                f"{sigma_rel(s_, spec['sigma']):.2e}")
    assert ou <= 1e-13 and ov <= 1e-13
    assert np.all(np.diff(s_) <= 0)
    if dtype == torch.float64:
        assert sigma_rel(s_, spec["sigma"]) <= 1e-12
    rows = np.sort(np.random.default_rng(3).choice(m, 64, replace=False))
    idx = torch.from_numpy(rows).to(A.device)
    Arows = host(A[idx]).astype(np.float64)                                   # 64 x n
    err = float(np.max(np.abs(host(U[idx]) * s_ - Arows @ v_))) / s_[0]
    flush_print(f"  sampled U S vs A V: {err:.2e} of sigma_1")
    assert err <= 1e-13


def _angle_tol(s, c=1e-13):
    """Per-column bound on sin(angle) between computed and reference singular vectors for a
    backward error of c sigma_1: c sigma_1 / (distance from sigma_j to the other values)."""
    d = np.abs(s[:, None] - s[None, :])
    np.fill_diagonal(d, np.inf)
    return c * s[0] / d.min(axis=1)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_workload3_full_size_vs_oracle(dtype):
    """4,000,000 x 100 at full size against the oracle on the same bytes (float32 storage:
    the exact upcast): sigma to 1e-12 relative and every column of U and V within the
    perturbation bound of its singular gap (backward error 1e-13 sigma_1)."""
    spec, A = _workload3(dtype)
    U, S, V, info = T.tssvd(A)
    torch.cuda.synchronize()
    flush_print("case workload3 oracle", dtype)
    Ah = host(A).astype(np.float64)
    del A
    Ur, Sr, Vr, _ = tssvd_ref(Ah)
    del Ah
    s_ = host(S)
    tol = _angle_tol(Sr)
    su, sv = col_sin(host(U), Ur), col_sin(host(V), Vr)
    flush_print(f"  sigma rel vs oracle {sigma_rel(s_, Sr):.2e}; max sin/tol U "
                f"{np.max(su / tol):.2e} V {np.max(sv / tol):.2e}; max sin U {su.max():.2e}")
    assert sigma_rel(s_, Sr) <= 1e-12
    assert np.all(su <= tol) and np.all(sv <= tol)
