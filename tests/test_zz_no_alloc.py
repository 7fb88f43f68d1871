"""GPU: tssvd_noalloc (no workspace argument, the library's per-GPU scratch array) through
the C ABI against tssvd with a caller workspace: bitwise-equal results on two calls in a
row, the second with a smaller input, plus the oracle's singular values."""
import ctypes as C

import numpy as np
import pytest
import torch

from oracle.tssvd_ref import tssvd_ref

from gpu_util import dev, flush_print, host, sigma_rel

pytestmark = pytest.mark.gpu

T = pytest.importorskip("paper_1612_08709_amd")
N = T._native


def _graded(m, n, seed, cond=1e5):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((m, n)) * np.logspace(0, -np.log10(cond), n)


def _pair(A64, dtype, **kw):
    A = dev(A64, dtype)
    U1, S1, V1, i1 = T.tssvd(A, **kw)
    U2, S2, V2, i2 = T.tssvd_noalloc(A, **kw)
    torch.cuda.synchronize()
    return (host(U1), host(S1), host(V1), i1), (host(U2), host(S2), host(V2), i2)


@pytest.mark.parametrize("ortho", [T.ORTHO_AUTO, T.ORTHO_TWICE])
def test_noalloc_matches_tssvd_two_calls(ortho):
    # the first call fills most of the scratch array; the second, smaller one runs over
    # what the first left behind
    for (m, n, dtype, seed) in [(12000, 100, torch.float64, 11), (3001, 33, torch.float32, 12)]:
        flush_print("case tssvd_noalloc", m, n, dtype, "ortho", ortho)
        A64 = _graded(m, n, seed)
        if dtype == torch.float32:
            A64 = A64.astype(np.float32).astype(np.float64)
        (U1, S1, V1, i1), (U2, S2, V2, i2) = _pair(A64, dtype, ortho=ortho)
        assert np.array_equal(S1, S2) and np.array_equal(U1, U2) and np.array_equal(V1, V2)
        assert i1 == i2
        _, Sr, _, _ = tssvd_ref(A64)
        assert sigma_rel(S2, Sr) < 1e-12


def test_noalloc_rejects_sizes_past_the_scratch():
    lib = N.lib()
    o = N.default_opts()
    nb = C.c_size_t()
    m, n = 200000, 100
    assert lib.tssvd_workspace_bytes(m, n, N.F64, C.byref(o), C.byref(nb)) == N.OK
    assert nb.value > N.TSSVD_NOALLOC_SCRATCH_BYTES
    A = torch.empty(m, n, dtype=torch.float64, device="cuda:0")
    U = torch.empty(m, n, dtype=torch.float64, device="cuda:0")
    S = torch.empty(n, dtype=torch.float64, device="cuda:0")
    V = torch.empty(n, n, dtype=torch.float64, device="cuda:0")
    st = lib.tssvd_noalloc(C.c_void_p(A.data_ptr()), N.F64, m, n, n, C.c_void_p(U.data_ptr()), n,
                           C.c_void_p(S.data_ptr()), C.c_void_p(V.data_ptr()), n, None,
                           C.byref(o), C.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == N.E_UNSUPPORTED
    with pytest.raises(ValueError):
        T.tssvd_noalloc(A)
