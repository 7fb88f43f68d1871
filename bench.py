#!/usr/bin/env python3
"""Benchmark of the MI355X tall-skinny / randomized low-rank SVD (one GPU).

Prints ONE JSON line.  Headline: GB/s of A streamed per SVD pass for the randomized
rank-k SVD (Algorithm 7) on the 200,000 x 2,000 float64 workload (sigma_j = 1/j plus
1e-8 Gaussian noise, k=20, l=30, q=2): value = (2q+2) * bytes(A) / seconds per call,
with A resident in HBM when the timed region starts.

Also reported, in the same line:
  roofline      the dominant A-streaming kernel, timed with HIP events recorded on the
                library's stream inside the timed region (algorithmic bytes / duration)
  cpu_baseline  the float64 CPU oracle on the same matrix (host cores)
  legs          the tall-skinny SVD workloads (10,000 x 20 and 4,000,000 x 100)

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--legs w1,w3]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
METRIC = "GB/s of A streamed per SVD pass, mixed vs FP64 at ‖U*U−I‖≤1e-12"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def ortho_gpu(U):
    """||U^T U - I||_2 in float64 on the device (checker only, outside the timed region)."""
    import torch
    G = U.T @ U
    G -= torch.eye(G.shape[0], dtype=G.dtype, device=G.device)
    return float(torch.linalg.matrix_norm(G, ord=2))


def time_calls(fn, steps, warmup, prof_kinds):
    import torch
    from paper_1612_08709_amd import _native as N
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    N.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = {k: N.profile_read(k) for k in prof_kinds}
    N.profile_enable(False)
    return (t1 - t0) / steps, prof


def leg_lowrank(workload, steps, warmup, want_cpu):
    import torch
    import paper_1612_08709_amd as T
    from paper_1612_08709_amd import _native as N
    from synth import matrices as sm, torch_gen
    spec = sm.workload_spec(workload)
    m, n, k, l, q = spec["m"], spec["n"], spec["k"], spec["l"], spec["q"]
    dt = torch.float64 if spec["dtype"] == "f64" else torch.float32
    log(f"[bench] generating workload {workload}: {m} x {n} {spec['dtype']}")
    A = torch_gen.planted(m, n, spec["sigma"], workload, "cuda:0", noise=spec.get("noise", 0.0),
                          dtype=dt, rank=spec.get("rank"))
    Om = torch_gen.sketch(n, l, workload, "cuda:0")
    call = T.LowrankCall(A, k, l, q, prec=T.PREC_FP64)
    sec, prof = time_calls(lambda: call.run(Om), steps, warmup, (N.PROF_AX, N.PROF_ATQ))
    passes = 2 * q + 2
    abytes = m * n * A.element_size()
    value = passes * abytes / sec / 1e9
    U, S, V = call.run(Om)
    torch.cuda.synchronize()
    ortho_u, ortho_v = ortho_gpu(U), ortho_gpu(V)
    # dominant kernel: the family with the larger summed time
    kinds = {"gemm_ax_f64 (Y = A X)": prof[N.PROF_AX], "gemm_atq_f64 (Z = A^T Q)": prof[N.PROF_ATQ]}
    name, (tot_ms, cnt) = max(kinds.items(), key=lambda kv: kv[1][0])
    avg_s = tot_ms / max(cnt, 1) / 1e3
    # algorithmic bytes per launch: read A once, read the n x l (or m x l) operand once,
    # write the m x l (or n x l) result once
    alg_bytes = abytes + (m * l + n * l) * 8
    achieved = alg_bytes / avg_s / 1e9
    flops = 2.0 * m * n * l
    res = dict(value=value, sec=sec, passes=passes, abytes=abytes, ortho_u=ortho_u,
               ortho_v=ortho_v, A=A, Om=Om, U=U, S=S, V=V, spec=spec,
               kernel=dict(name=name, avg_ms=avg_s * 1e3, launches=cnt, alg_bytes=alg_bytes,
                           achieved_gbs=achieved, fp64_tflops=flops / avg_s / 1e12),
               kernels={kk: dict(total_ms=v[0], launches=v[1]) for kk, v in kinds.items()})
    if want_cpu:
        res["cpu"] = cpu_baseline_lowrank(A, Om, k, q, passes)
    return res


def cpu_baseline_lowrank(A, Om, k, q, passes):
    """The CPU oracle on the same bytes (float64 NumPy, all host cores)."""
    from oracle.lowrank_ref import lowrank_ref
    try:
        from threadpoolctl import threadpool_info
        threads = max([p.get("num_threads", 1) for p in threadpool_info()] or [os.cpu_count()])
    except Exception:  # pragma: no cover
        threads = os.cpu_count()
    Ah = A.cpu().numpy()
    Omh = Om.cpu().numpy()
    lowrank_ref(Ah[: min(Ah.shape[0], 20000)], Omh, k, q)  # warm-up on a slice
    times = []
    for _ in range(3):
        t0 = time.perf_counter()
        lowrank_ref(Ah, Omh, k, q)
        times.append(time.perf_counter() - t0)
    t = float(np.median(times))
    return dict(value=passes * Ah.nbytes / t / 1e9, unit="GB/s", cores=int(threads),
                kind="oracle", seconds=t,
                sample=f"full workload ({Ah.shape[0]} x {Ah.shape[1]}), median of 3 runs")


def leg_tssvd(workload, steps, warmup, dtype_name=None, m_override=None):
    import torch
    import paper_1612_08709_amd as T
    from paper_1612_08709_amd import _native as N
    from synth import matrices as sm, torch_gen
    spec = sm.workload_spec(workload)
    m, n = (m_override or spec["m"]), spec["n"]
    dname = dtype_name or spec["dtype"]
    dt = torch.float64 if dname == "f64" else torch.float32
    log(f"[bench] generating workload {workload}: {m} x {n} {dname}")
    A = torch_gen.planted(m, n, spec["sigma"], workload, "cuda:0", dtype=dt)
    o = T.make_opts(ortho=T.ORTHO_ONCE)
    nb = __import__("ctypes").c_size_t()
    lib = N.lib()
    import ctypes as C
    code = N.F64 if dt == torch.float64 else N.F32
    N.check(lib.tssvd_workspace_bytes(m, n, code, C.byref(o), C.byref(nb)), "ws")
    work = torch.empty(nb.value, dtype=torch.uint8, device="cuda:0")
    U = torch.empty(m, n, dtype=torch.float64, device="cuda:0")
    S = torch.empty(n, dtype=torch.float64, device="cuda:0")
    V = torch.empty(n, n, dtype=torch.float64, device="cuda:0")
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)

    def run():
        N.check(lib.tssvd(C.c_void_p(A.data_ptr()), code, m, n, n, C.c_void_p(U.data_ptr()), n,
                          C.c_void_p(S.data_ptr()), C.c_void_p(V.data_ptr()), n, None,
                          C.c_void_p(work.data_ptr()), nb.value, C.byref(o), stream), "tssvd")

    sec, prof = time_calls(run, steps, warmup, (N.PROF_LEAF_FACTOR, N.PROF_LEAF_APPLY))
    torch.cuda.synchronize()
    sig = torch.tensor(spec["sigma"], device="cuda:0")
    srel = float(((S - sig).abs() / sig).max()) if dt == torch.float64 else None
    abytes = m * n * A.element_size()
    lf, la = prof[N.PROF_LEAF_FACTOR], prof[N.PROF_LEAF_APPLY]
    out = dict(workload=f"tall-skinny SVD {m} x {n} {dname}", ms_per_call=sec * 1e3,
               gbs_A_per_call=abytes / sec / 1e9, ortho_U=ortho_gpu(U), sigma_rel_err=srel,
               leaf_factor_ms=lf[0] / max(lf[1], 1), leaf_apply_ms=la[0] / max(la[1], 1),
               leaf_factor_gbs=abytes / (lf[0] / max(lf[1], 1) / 1e3) / 1e9,
               leaf_factor_fp64_tflops=2.0 * m * n * n / (lf[0] / max(lf[1], 1) / 1e3) / 1e12)
    del A, U, work
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", type=int, default=2)
    ap.add_argument("--legs", default="w1,w3")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--calib-copy", action="store_true",
                    help="run one 1 GiB read + 1 GiB write elementwise kernel first (counter "
                         "calibration for the HBM traffic figures)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(this build has no multi-GPU path).", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    if args.calib_copy:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        del src, dst
    head = leg_lowrank(args.workload, args.steps, args.warmup, not args.no_cpu)
    spec = head["spec"]
    legs = {}
    for leg in [x for x in args.legs.split(",") if x]:
        try:
            if leg == "w1":
                legs["w1"] = leg_tssvd(1, max(args.steps, 20), args.warmup)
            elif leg == "w3":
                legs["w3_f64"] = leg_tssvd(3, args.steps, args.warmup, "f64")
                legs["w3_f32"] = leg_tssvd(3, args.steps, args.warmup, "f32")
        except Exception as e:  # a failing secondary leg is reported, not fatal
            legs[leg] = dict(error=repr(e))
    kern = head["kernel"]
    out = {
        "metric": METRIC,
        "value": round(head["value"], 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(head["sec"] * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"randomized rank-k SVD (Algorithm 7), {spec['m']} x {spec['n']} "
                               f"{spec['dtype']}, sigma_j = 1/j + 1e-8 noise",
                   "m": spec["m"], "n": spec["n"], "k": spec["k"], "l": spec["l"],
                   "q": spec["q"], "passes_over_A": head["passes"], "prec": "fp64"},
        "roofline": {"bound": "hbm", "achieved": round(kern["achieved_gbs"], 2),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(kern["achieved_gbs"] / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": kern["name"], "avg_ms": round(kern["avg_ms"], 4),
                     "launches": kern["launches"], "alg_bytes_per_launch": kern["alg_bytes"],
                     "fp64_tflops": round(kern["fp64_tflops"], 2),
                     "fp64_frac": round(kern["fp64_tflops"] / FP64_PEAK_TFLOPS, 4)},
        "accuracy": {"ortho_U_2norm": head["ortho_u"], "ortho_V_2norm": head["ortho_v"]},
        "kernels": head["kernels"],
        "legs": legs,
    }
    if "cpu" in head:
        out["cpu_baseline"] = head["cpu"]
    print(json.dumps(out))


if __name__ == "__main__":
    main()
