// Device helpers shared by the gfx950 kernels: DPP reductions, typed loads, constants.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tsv {

// ---- lane-group reductions with data-parallel primitives (DPP), all within 16-lane rows.
// Every lane of the row ends with the bitwise-identical sum: each stage adds the same two
// operands in both partner lanes, so the result does not depend on the lane.

template <int CTRL>
__device__ __forceinline__ double dpp_d(double x) {
  int lo = __double2loint(x), hi = __double2hiint(x);
  lo = __builtin_amdgcn_update_dpp(0, lo, CTRL, 0xF, 0xF, false);
  hi = __builtin_amdgcn_update_dpp(0, hi, CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

// DPP controls: quad_perm [1,0,3,2] = 0xB1, quad_perm [2,3,0,1] = 0x4E,
// row_half_mirror = 0x141 (lane i <-> 7-i within 8), row_mirror = 0x140 (i <-> 15-i).
__device__ __forceinline__ double sum16(double x) {
  x += dpp_d<0xB1>(x);
  x += dpp_d<0x4E>(x);
  x += dpp_d<0x141>(x);
  x += dpp_d<0x140>(x);
  return x;
}

__device__ __forceinline__ double sum4(double x) {
  x += dpp_d<0xB1>(x);
  x += dpp_d<0x4E>(x);
  return x;
}

// Sum over the four 16-lane rows of a wave (lanes l, l^16, l^32, l^48) via permutes.
__device__ __forceinline__ double sum_rows4(double x) {
  const int lane = threadIdx.x & 63;
  int lo = __double2loint(x), hi = __double2hiint(x);
  int lo1 = __builtin_amdgcn_ds_bpermute(((lane ^ 16) << 2), lo);
  int hi1 = __builtin_amdgcn_ds_bpermute(((lane ^ 16) << 2), hi);
  x += __hiloint2double(hi1, lo1);
  lo = __double2loint(x); hi = __double2hiint(x);
  lo1 = __builtin_amdgcn_ds_bpermute(((lane ^ 32) << 2), lo);
  hi1 = __builtin_amdgcn_ds_bpermute(((lane ^ 32) << 2), hi);
  x += __hiloint2double(hi1, lo1);
  return x;
}

// ---- typed element loads (A may be float32 or float64; arithmetic is float64).
__device__ __forceinline__ double ld_elem(const double* p) { return *p; }
__device__ __forceinline__ double ld_elem(const float* p) { return (double)*p; }

// ---- reference vector of the output sign convention: w_i = frac((i+1) g) - 1/2.
__device__ __forceinline__ double sign_ref(int i) {
  const double g = 0.6180339887498949;  // (sqrt(5)-1)/2 rounded to double
  double t = (double)(i + 1) * g;
  return t - floor(t) - 0.5;
}

// ---- four consecutive entries of a matrix row as one register quad: a 16-byte load for float32,
// two for float64.  pin() is an empty asm statement that reads and writes the quad, so the
// float32 -> float64 conversions of one pipeline slot cannot be scheduled above it (they
// would make the wave wait for the loads of the later slots).
template <typename TA>
struct Quad;
template <>
struct Quad<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  v4 v;
  __device__ __forceinline__ void load(const float* p) { v = *reinterpret_cast<const v4*>(p); }
  __device__ __forceinline__ void zero() { v = v4{0.f, 0.f, 0.f, 0.f}; }
  __device__ __forceinline__ void pin() { asm volatile("" : "+v"(v)); }
  __device__ __forceinline__ double operator[](int s) const { return (double)v[s]; }
};
template <>
struct Quad<double> {
  typedef double v2 __attribute__((ext_vector_type(2)));
  v2 lo, hi;
  __device__ __forceinline__ void load(const double* p) {
    lo = *reinterpret_cast<const v2*>(p);
    hi = *reinterpret_cast<const v2*>(p + 2);
  }
  __device__ __forceinline__ void zero() { lo = hi = v2{0.0, 0.0}; }
  __device__ __forceinline__ void pin() { asm volatile("" : "+v"(lo), "+v"(hi)); }
  __device__ __forceinline__ double operator[](int s) const { return s < 2 ? lo[s] : hi[s - 2]; }
};

// numstat bits of tssvd_info
constexpr int NUM_NONFINITE = 1;
constexpr int NUM_NO_CONVERGENCE = 2;

}  // namespace tsv
