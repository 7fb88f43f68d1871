"""Build libtssvd.so (gfx950) from csrc/*.hip with hipcc, in-tree.

Every translation unit is compiled to an object in ``_build/`` (in parallel), then
linked into ``paper_1612_08709_amd/libtssvd.so``.  Run ``python -m
paper_1612_08709_amd.build`` or call ``build()``.
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
OUT = os.path.join(PKG, "libtssvd.so")
BUILD = os.path.join(ROOT, "_build")
ARCH = os.environ.get("TSSVD_ARCH", "gfx950")

FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    "-I", os.path.join(ROOT, "include"),
    # packed FP32 VALU forms stay off in all device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def _hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found; the HIP toolchain (ROCm) is required to build libtssvd")


def _compile(src: str, hipcc: str) -> str:
    obj = os.path.join(BUILD, os.path.splitext(os.path.basename(src))[0] + ".o")
    cmd = [hipcc, *FLAGS, "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    return obj


def build(verbose: bool = True) -> str:
    hipcc = _hipcc()
    os.makedirs(BUILD, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(lambda s: _compile(s, hipcc), srcs))
    tmp = OUT + ".tmp"
    r = subprocess.run([hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs],
                       capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, OUT)
    # throughput probes for bench.py --probe (not part of the library)
    probe_src = os.path.join(ROOT, "bench_probe.hip")
    if os.path.exists(probe_src):
        probe_out = os.path.join(BUILD, "libtssvd_probe.so")
        r = subprocess.run([hipcc, *FLAGS, "-shared", "-o", probe_out + ".tmp", probe_src],
                           capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed for {probe_src}:\n{r.stderr}")
        os.replace(probe_out + ".tmp", probe_out)
    if verbose:
        print(f"built {OUT} ({len(srcs)} sources, {ARCH})")
    return OUT


if __name__ == "__main__":
    build()
    sys.exit(0)
