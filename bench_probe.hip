// Throughput probes for gfx950, used by `bench.py --probe` to measure the ceilings the
// library's kernels are judged against: FP64 and FP32 matrix-core (MFMA) rates, the FP64
// vector FMA rate, both at once, and HBM streaming rates for the read/write mixes of the
// passes over A.  Not part of the library.
#include <hip/hip_runtime.h>
#include <stdint.h>

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

constexpr int CH = 8;  // independent accumulator chains per wave

// CH independent v_mfma_f64_16x16x4_f64 chains per wave, `iters` rounds.
__global__ __launch_bounds__(256) void k_mfma_f64(int iters, double* out) {
  const double a = 1.0 + 1e-3 * (threadIdx.x & 63), b = 1.0 - 1e-3 * (threadIdx.x & 15);
  // the first round outside the loop: the loop then carries matrix-core results only
  f64x4 acc[CH];
#pragma unroll
  for (int c = 0; c < CH; ++c)
    acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, f64x4{0.0, 0.0, 0.0, (double)c}, 0, 0, 0);
  for (int i = 1; i < iters; ++i) {
#pragma unroll
    for (int c = 0; c < CH; ++c) acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[c], 0, 0, 0);
  }
  // keeps the chains alive (never true).  Storing the accumulators as they are, rather than
  // adding them up, lets them stay in the matrix-core registers: a sum after the loop makes
  // the compiler copy them out and back in on every round, which halves the rate measured.
  if (iters < 0) {
#pragma unroll
    for (int c = 0; c < CH; ++c)
      reinterpret_cast<f64x4*>(out)[(blockIdx.x * 256 + threadIdx.x) * CH + c] = acc[c];
  }
}

__global__ __launch_bounds__(256) void k_mfma_f32(int iters, double* out) {
  const float a = 1.0f + 1e-3f * (threadIdx.x & 63), b = 1.0f - 1e-3f * (threadIdx.x & 15);
  f32x4 acc[CH];
#pragma unroll
  for (int c = 0; c < CH; ++c)
    acc[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, f32x4{0.f, 0.f, 0.f, (float)c}, 0, 0, 0);
  for (int i = 1; i < iters; ++i) {
#pragma unroll
    for (int c = 0; c < CH; ++c) acc[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[c], 0, 0, 0);
  }
  if (iters < 0) {  // as in k_mfma_f64
#pragma unroll
    for (int c = 0; c < CH; ++c)
      reinterpret_cast<f32x4*>(out)[(blockIdx.x * 256 + threadIdx.x) * CH + c] = acc[c];
  }
}

// 2*CH independent FP64 FMA chains per lane.
__global__ __launch_bounds__(256) void k_valu_f64(int iters, double* out) {
  double x[2 * CH];
  const double m = 1.0 + 1e-9 * threadIdx.x, a = 1e-7;
#pragma unroll
  for (int c = 0; c < 2 * CH; ++c) x[c] = c;
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int c = 0; c < 2 * CH; ++c) x[c] = fma(x[c], m, a);
  }
  double s = 0.0;
#pragma unroll
  for (int c = 0; c < 2 * CH; ++c) s += x[c];
  if (s == 12345.678) out[blockIdx.x] = s;
}

// Even waves run the FP64 MFMA chains, odd waves the FP64 FMA chains (4*iters FMA
// instructions per round, about the issue time of one MFMA round).
__global__ __launch_bounds__(256) void k_mix_f64(int iters, int valu_iters, double* out) {
  const int w = threadIdx.x >> 6;
  double s = 0.0;
  if ((w & 1) == 0) {
    const double a = 1.0 + 1e-3 * (threadIdx.x & 63), b = 1.0 - 1e-3 * (threadIdx.x & 15);
    f64x4 acc[CH];
#pragma unroll
    for (int c = 0; c < CH; ++c)
      acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, f64x4{0.0, 0.0, 0.0, (double)c}, 0, 0, 0);
    for (int i = 1; i < iters; ++i) {
#pragma unroll
      for (int c = 0; c < CH; ++c) acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[c], 0, 0, 0);
    }
    if (iters < 0) {  // as in k_mfma_f64
#pragma unroll
      for (int c = 0; c < CH; ++c)
        reinterpret_cast<f64x4*>(out)[(blockIdx.x * 256 + threadIdx.x) * CH + c] = acc[c];
    }
  } else {
    double x[2 * CH];
    const double m = 1.0 + 1e-9 * threadIdx.x, a = 1e-7;
#pragma unroll
    for (int c = 0; c < 2 * CH; ++c) x[c] = c;
    for (int i = 0; i < valu_iters; ++i) {
#pragma unroll
      for (int c = 0; c < 2 * CH; ++c) x[c] = fma(x[c], m, a);
    }
#pragma unroll
    for (int c = 0; c < 2 * CH; ++c) s += x[c];
  }
  if (s == 12345.678) out[blockIdx.x] = s;
}

// Streaming read of n 16-byte vectors; one partial per workgroup.
__global__ __launch_bounds__(256) void k_read(const f32x4* __restrict__ p, int64_t n,
                                              float* __restrict__ part) {
  float s = 0.f;
  const int64_t stride = (int64_t)gridDim.x * 256;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) {
    const f32x4 v = __builtin_nontemporal_load(p + i);
    s += v[0] + v[1] + v[2] + v[3];
  }
  if (s == 12345.678f) part[blockIdx.x] = s;
}

// Read float32, write bfloat16 (truncated) of the same elements: the 2:1 read/write mix.
__global__ __launch_bounds__(256) void k_read_write_half(const f32x4* __restrict__ p, int64_t n,
                                                         u32x2* __restrict__ q) {
  const int64_t stride = (int64_t)gridDim.x * 256;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) {
    const f32x4 v = __builtin_nontemporal_load(p + i);
    u32x2 o;
    o[0] = (__float_as_uint(v[0]) >> 16) | (__float_as_uint(v[1]) & 0xFFFF0000u);
    o[1] = (__float_as_uint(v[2]) >> 16) | (__float_as_uint(v[3]) & 0xFFFF0000u);
    __builtin_nontemporal_store(o, q + i);
  }
}

// Plain copy, equal read and write bytes.
__global__ __launch_bounds__(256) void k_copy(const f32x4* __restrict__ p, int64_t n,
                                              f32x4* __restrict__ q) {
  const int64_t stride = (int64_t)gridDim.x * 256;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride)
    __builtin_nontemporal_store(__builtin_nontemporal_load(p + i), q + i);
}

extern "C" {

// kind: 0 mfma f64, 1 mfma f32, 2 valu f64, 3 mfma f64 + valu f64 (half the waves each).
// Returns flops per launch in *flops.
int probe_compute(int kind, int blocks, int iters, double* out, double* flops, void* stream) {
  hipStream_t s = (hipStream_t)stream;
  const double waves = (double)blocks * 4.0;
  switch (kind) {
    case 0:
      hipLaunchKernelGGL(k_mfma_f64, dim3(blocks), dim3(256), 0, s, iters, out);
      *flops = waves * iters * CH * 2048.0;
      break;
    case 1:
      hipLaunchKernelGGL(k_mfma_f32, dim3(blocks), dim3(256), 0, s, iters, out);
      *flops = waves * iters * CH * 2048.0;
      break;
    case 2:
      hipLaunchKernelGGL(k_valu_f64, dim3(blocks), dim3(256), 0, s, iters, out);
      *flops = waves * 64.0 * iters * 2 * CH * 2.0;
      break;
    case 3: {
      const int vi = 4 * iters;
      hipLaunchKernelGGL(k_mix_f64, dim3(blocks), dim3(256), 0, s, iters, vi, out);
      *flops = waves * 0.5 * iters * CH * 2048.0 + waves * 0.5 * 64.0 * vi * 2 * CH * 2.0;
      break;
    }
    default: return 1;
  }
  return hipGetLastError() == hipSuccess ? 0 : 3;
}

// kind: 0 read, 1 read + half-size write, 2 copy.  n16 = number of 16-byte vectors read.
int probe_stream(int kind, int blocks, const void* src, int64_t n16, void* dst, void* stream) {
  hipStream_t s = (hipStream_t)stream;
  switch (kind) {
    case 0:
      hipLaunchKernelGGL(k_read, dim3(blocks), dim3(256), 0, s, (const f32x4*)src, n16,
                         (float*)dst);
      break;
    case 1:
      hipLaunchKernelGGL(k_read_write_half, dim3(blocks), dim3(256), 0, s, (const f32x4*)src,
                         n16, (u32x2*)dst);
      break;
    case 2:
      hipLaunchKernelGGL(k_copy, dim3(blocks), dim3(256), 0, s, (const f32x4*)src, n16,
                         (f32x4*)dst);
      break;
    default: return 1;
  }
  return hipGetLastError() == hipSuccess ? 0 : 3;
}

}  // extern "C"
