"""The C ABI library: builds, loads, exports every declared symbol, validates on the host.

No compute call runs here (no GPU in this environment); every call below returns
from host-side argument validation before anything is enqueued.
"""
import ctypes as C
import math
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tssvd.h")


@pytest.fixture(scope="module")
def native():
    from paper_1612_08709_amd import _native as N
    if not os.path.exists(N.LIB_PATH):
        from paper_1612_08709_amd import build
        build.build(verbose=False)
    return N


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_abi():
    names = _declared_functions()
    for f in ("tsqr", "tssvd", "lowrank_svd", "lowrank_svd_backward", "tssvd_workspace_bytes"):
        assert f in names


def test_library_exports_every_declared_symbol(native):
    lib = native.lib()
    out = subprocess.run(["nm", "-D", "--defined-only", native.LIB_PATH], capture_output=True,
                         text=True).stdout
    exported = {ln.split()[-1] for ln in out.splitlines() if ln.strip()}
    for name in _declared_functions():
        assert name in exported, name
        assert hasattr(lib, name)
    assert set(native.EXPORTS) == set(_declared_functions())


def test_default_opts_and_strings(native):
    o = native.default_opts()
    assert o.prec == native.PREC_FP64 and o.ortho == native.ORTHO_AUTO
    assert o.working_precision == 0.0 and o.reorth_tol == 1e-13 and o.max_jacobi_sweeps == 30
    assert native.status_string(0) == "ok"
    assert "workspace" in native.status_string(2)
    assert native.lib().tssvd_version() >= 100


def test_struct_layouts_match_header(native):
    assert C.sizeof(native.Opts) == 40
    assert C.sizeof(native.Info) == 24


def test_workspace_queries_validate(native):
    lib, N = native.lib(), native
    nb = C.c_size_t()
    o = N.default_opts()
    assert lib.tssvd_workspace_bytes(1000, 20, N.F64, C.byref(o), C.byref(nb)) == N.OK
    assert nb.value > 1000 * 20 * 8
    assert lib.tssvd_workspace_bytes(10, 20, N.F64, C.byref(o), C.byref(nb)) == N.E_INVALID_ARG
    assert lib.tssvd_workspace_bytes(1000, 0, N.F64, C.byref(o), C.byref(nb)) == N.E_INVALID_ARG
    assert lib.tssvd_workspace_bytes(1000, 20, 7, C.byref(o), C.byref(nb)) == N.E_INVALID_ARG
    assert lib.tssvd_workspace_bytes(10**6, 101, N.F64, C.byref(o), C.byref(nb)) == N.E_UNSUPPORTED
    assert lib.tsqr_workspace_bytes(10**6, 128, N.F64, C.byref(nb)) == N.OK
    assert lib.tsqr_workspace_bytes(10**6, 129, N.F64, C.byref(nb)) == N.E_UNSUPPORTED
    # lowrank: 0 < k <= l < min(m, n), q >= 0
    ok = lib.lowrank_svd_workspace_bytes(2000, 500, 10, 20, 2, N.F32, C.byref(o), C.byref(nb))
    assert ok == N.OK and nb.value > 2000 * 20 * 8
    for (m, n, k, l, q) in [(2000, 500, 21, 20, 2), (2000, 500, 0, 20, 2), (2000, 20, 5, 20, 2),
                            (20, 500, 5, 20, 2), (2000, 500, 5, 20, -1)]:
        assert lib.lowrank_svd_workspace_bytes(m, n, k, l, q, N.F64, C.byref(o),
                                               C.byref(nb)) == N.E_INVALID_ARG


def test_calls_reject_bad_arguments_before_any_work(native):
    lib, N = native.lib(), native
    o = N.default_opts()
    null = C.c_void_p(0)
    fake = C.c_void_p(256)  # never dereferenced: validation fails first
    # null A
    assert lib.tssvd(null, N.F64, 100, 10, 10, fake, 10, fake, fake, 10, null, fake, 1 << 30,
                     C.byref(o), null) == N.E_INVALID_ARG
    # lda < n
    assert lib.tssvd(fake, N.F64, 100, 10, 9, fake, 10, fake, fake, 10, null, fake, 1 << 30,
                     C.byref(o), null) == N.E_INVALID_ARG
    # workspace too small
    assert lib.tssvd(fake, N.F64, 100, 10, 10, fake, 10, fake, fake, 10, null, fake, 16,
                     C.byref(o), null) == N.E_WORKSPACE
    assert lib.tssvd(fake, N.F64, 100, 10, 10, fake, 10, fake, fake, 10, null, null, 1 << 30,
                     C.byref(o), null) == N.E_WORKSPACE
    # bad option values
    bad = N.default_opts()
    bad.ortho = 9
    assert lib.tssvd(fake, N.F64, 100, 10, 10, fake, 10, fake, fake, 10, null, fake, 1 << 30,
                     C.byref(bad), null) == N.E_INVALID_ARG
    bad = N.default_opts()
    bad.working_precision = float("nan")
    assert lib.tssvd(fake, N.F64, 100, 10, 10, fake, 10, fake, fake, 10, null, fake, 1 << 30,
                     C.byref(bad), null) == N.E_INVALID_ARG
    assert lib.tsqr(fake, N.F64, 5, 10, 10, null, 10, fake, 10, fake, 1 << 30, null) == N.E_INVALID_ARG
    assert lib.lowrank_svd(fake, N.F64, 100, 50, 50, 8, 4, 1, null, fake, 8, fake, fake, 8, null,
                           fake, 1 << 30, C.byref(o), null) == N.E_INVALID_ARG
    assert lib.lowrank_svd(fake, N.F64, 100, 50, 50, 4, 8, 1, null, fake, 4, fake, fake, 4, null,
                           fake, 16, C.byref(o), null) == N.E_WORKSPACE


def test_route_flags_are_validated_on_the_host(native):
    """Flag combinations the library does not take come back before any work is enqueued."""
    lib, N = native.lib(), native
    null = C.c_void_p(0)
    fake = C.c_void_p(256)  # never dereferenced: validation fails first

    def opts(flags, wp=0.0):
        o = N.default_opts()
        o.flags, o.working_precision = flags, wp
        return o

    def lowrank(o, m=100, n=50, l=8):
        return lib.lowrank_svd(fake, N.F64, m, n, n, 4, l, 1, null, fake, 4, fake, fake, 4, null,
                               fake, 1 << 40, C.byref(o), null)

    assert lowrank(opts(N.FLAG_LU | N.FLAG_GRAM)) == N.E_INVALID_ARG
    assert lowrank(opts(N.FLAG_LU, wp=1e-11)) == N.E_UNSUPPORTED
    assert lowrank(opts(N.FLAG_LU), n=200, l=65) == N.E_UNSUPPORTED
    assert lowrank(opts(N.FLAG_LU), m=1 << 31) == N.E_UNSUPPORTED
    assert lowrank(opts(N.FLAG_MIX)) == N.E_UNSUPPORTED
    o = opts(N.FLAG_MIX | N.FLAG_GRAM)
    assert lib.tssvd(fake, N.F64, 100, 10, 10, fake, 10, fake, fake, 10, null, fake, 1 << 40,
                     C.byref(o), null) == N.E_INVALID_ARG


def test_sign_reference_constant_is_the_golden_ratio_conjugate():
    """The device source spells g = (sqrt(5)-1)/2 as a decimal literal; it must be that double."""
    src = open(os.path.join(ROOT, "paper_1612_08709_amd", "csrc", "common.h")).read()
    lit = float(re.search(r"const double g = ([0-9.]+);", src).group(1))
    assert lit == (math.sqrt(5.0) - 1.0) / 2.0


def test_python_layer_fails_loudly_without_gpu_tensors(native):
    import torch
    import paper_1612_08709_amd as T
    with pytest.raises(ValueError):
        T.tssvd(torch.zeros(10, 3, dtype=torch.float64))


def _header_constants():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    consts = {k: int(v) for k, v in re.findall(r"#define\s+TSSVD_(\w+)\s+(\d+)", text)}
    consts.update({k: int(v) for k, v in re.findall(r"\bTSSVD_(\w+)\s*=\s*(\d+)", text)})
    return consts


def _header_struct_fields(name):
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    body = re.search(r"typedef struct\s*\{([^}]*)\}\s*" + name + ";", text).group(1)
    return [re.findall(r"(\w+)\s*;", d)[0] for d in body.split(";") if d.strip()
            for d in [d + ";"]]


def test_python_constants_match_the_header():
    """Every flag, status, dtype, precision and ortho code the binding hard-codes is the
    header's value."""
    from paper_1612_08709_amd import _native as N
    h = _header_constants()
    pairs = {"FLAG_F32_MFMA_FINAL": N.FLAG_F32_MFMA_FINAL, "FLAG_NO_A_COPY": N.FLAG_NO_A_COPY,
             "FLAG_GRAM": N.FLAG_GRAM, "FLAG_LU": N.FLAG_LU, "FLAG_MIX": N.FLAG_MIX,
             "N_MAX": N.TSSVD_N_MAX, "TSQR_N_MAX": N.TSSVD_TSQR_N_MAX, "OK": N.OK,
             "E_INVALID_ARG": N.E_INVALID_ARG, "E_WORKSPACE": N.E_WORKSPACE, "E_HIP": N.E_HIP,
             "E_UNSUPPORTED": N.E_UNSUPPORTED, "F64": N.F64, "F32": N.F32,
             "PREC_FP64": N.PREC_FP64, "PREC_MIXED": N.PREC_MIXED, "ORTHO_AUTO": N.ORTHO_AUTO,
             "ORTHO_ONCE": N.ORTHO_ONCE, "ORTHO_TWICE": N.ORTHO_TWICE}
    pairs.update({k: getattr(N, k) for k in ("PROF_AX", "PROF_ATQ", "PROF_LEAF_FACTOR",
                                             "PROF_LEAF_APPLY", "PROF_AX_BF16", "PROF_ATQ_BF16",
                                             "PROF_AX_FINAL", "PROF_ATQ_FINAL", "PROF_AX_BF16C",
                                             "PROF_ATQ_BF16C")})
    for k, v in pairs.items():
        assert h[k] == v, k
    flags = [v for k, v in h.items() if k.startswith("FLAG_")]
    assert len(set(flags)) == len(flags) and all(f & (f - 1) == 0 for f in flags)


def test_python_structs_match_the_header():
    """ctypes mirrors of tssvd_opts and tssvd_info: same fields in the same order."""
    from paper_1612_08709_amd import _native as N
    assert [f for f, _ in N.Opts._fields_] == _header_struct_fields("tssvd_opts")
    assert [f for f, _ in N.Info._fields_] == _header_struct_fields("tssvd_info")


def test_sketch_and_cotangent_checks_reject_misread_layouts(native):
    """The binding passes Omega as a contiguous n x l float64 array and the cotangents with
    their own row strides; anything else would be read out of bounds by the library, so it
    is rejected (or copied) before the call."""
    import torch
    import paper_1612_08709_amd as T
    n, l = 12, 5
    ok = torch.zeros(n, l, dtype=torch.float64)
    T._check_omega(ok, n, l, "cpu")
    T._check_omega(None, n, l, "cpu")
    for bad in (ok.float(), ok.T.contiguous().T, ok[:, :l - 1], torch.zeros(n + 1, l,
                                                                              dtype=torch.float64)):
        with pytest.raises(ValueError):
            T._check_omega(bad, n, l, "cpu")
    g = torch.zeros(7, 2 * 3, dtype=torch.float32)[:, ::2]          # 7 x 3, row stride 6
    c = T._check_cotangent(g, (7, 3), "gU", "cpu")
    assert c.dtype == torch.float64 and c.is_contiguous() and c.stride(0) == 3
    assert T._check_cotangent(None, (7, 3), "gU", "cpu") is None
    with pytest.raises(ValueError):
        T._check_cotangent(torch.zeros(7, 4), (7, 3), "gU", "cpu")


def test_misaligned_workspace_is_rejected_on_the_host(native):
    """The workspace must start on 256 bytes; a misaligned one is refused before anything is
    enqueued (fake device pointers: no kernel may run)."""
    lib, N = native.lib(), native
    o = N.default_opts()
    fake = C.c_void_p(0x1000)
    nb = C.c_size_t()
    assert lib.tssvd_workspace_bytes(1000, 10, N.F64, C.byref(o), C.byref(nb)) == N.OK
    st = lib.tssvd(fake, N.F64, 1000, 10, 10, fake, 10, fake, fake, 10, None,
                   C.c_void_p(0x1010), nb.value + 256, C.byref(o), None)
    assert st == N.E_WORKSPACE
    assert lib.tsqr_workspace_bytes(1000, 10, N.F64, C.byref(nb)) == N.OK
    assert lib.tsqr(fake, N.F64, 1000, 10, 10, fake, 10, fake, 10, C.c_void_p(0x1080),
                    nb.value + 256, None) == N.E_WORKSPACE


def test_noalloc_rejects_before_touching_the_device(native):
    """tssvd_noalloc checks its arguments and the scratch limit on the host first."""
    lib, N = native.lib(), native
    o = N.default_opts()
    fake = C.c_void_p(0x1000)
    # workspace need beyond the fixed scratch array: rejected, nothing enqueued
    st = lib.tssvd_noalloc(fake, N.F64, 200000, 100, 100, fake, 100, fake, fake, 100, None,
                           C.byref(o), None)
    assert st == N.E_UNSUPPORTED
    nb = C.c_size_t()
    assert lib.tssvd_workspace_bytes(200000, 100, N.F64, C.byref(o), C.byref(nb)) == N.OK
    assert nb.value > N.TSSVD_NOALLOC_SCRATCH_BYTES
    assert lib.tssvd_noalloc(None, N.F64, 1000, 10, 10, fake, 10, fake, fake, 10, None,
                             C.byref(o), None) == N.E_INVALID_ARG
    assert lib.tssvd_noalloc(fake, N.F64, 1000, 101, 101, fake, 101, fake, fake, 101, None,
                             C.byref(o), None) == N.E_UNSUPPORTED
    text = open(HEADER).read()
    assert "#define TSSVD_NOALLOC_SCRATCH_BYTES (64u << 20)" in text
    assert N.TSSVD_NOALLOC_SCRATCH_BYTES == 64 << 20
