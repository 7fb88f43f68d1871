// LU-based tracking bases for the subspace iteration (Section 3: the intermediate
// factorizations of Algorithm 5 only carry a column space, and the lower-trapezoidal factor
// L of an LU factorization spans the same columns as Q).
//
// Pivots come from a tournament (communication-avoiding LU, Grigori-Demmel-Xiang 2011):
// every workgroup runs Gaussian elimination with partial pivoting on up to 256 candidate
// rows of Y and passes on the l rows it picked; the next level takes floor(256 / l) such
// groups per workgroup, until one workgroup remains.  Its pivot rows, as reduced at their
// step, form U (the LU factor of Y's pivot rows in pivot order), and the basis is
// L = Y U^-1 (rows in Y's order), formed by the caller with the same product that forms
// Y R^-1 for a Cholesky basis.  Any pivot order gives the same column space; partial
// pivoting keeps |L| moderate.
#include "internal.h"

#include <climits>

namespace tsv {
namespace {

constexpr int LU_THREADS = 256;

// Candidate order for the pivot search: a larger |value| wins, then a smaller row index.
// key = (bit pattern of |v|) + 1 is monotone in |v| for |v| >= 0 (NaN sorts above +inf);
// key 0 marks a lane with no candidate.
__device__ __forceinline__ bool lu_better(unsigned long long ka, int ra, unsigned long long kb,
                                          int rb) {
  return ka > kb || (ka == kb && ra < rb);
}

__device__ __forceinline__ void wave_argmax(unsigned long long& key, int& row) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const unsigned long long k2 = __shfl_xor(key, off);
    const int r2 = __shfl_xor(row, off);
    if (lu_better(k2, r2, key, row)) {
      key = k2;
      row = r2;
    }
  }
}

// One level of the tournament.  Workgroup b's candidates: rows b*256 + t of Y at the leaf
// level (cand == nullptr), else cand[b*per + t] for t < per (-1: none).  Thread t keeps its
// candidate row (l <= LM entries) in registers.  Step j: the wave argmax of |r_j|, one
// barrier, the winner of the four waves is the pivot row p; every remaining candidate
// takes f = r_j / p_j and r_c -= f p_c for c > j.  The picked rows go to out[b*l + j] in
// pivot order (-1 once the workgroup has no candidate left).
// With one workgroup (the last level) the kernel also writes T = U^-1 (l x l, row-major)
// by back substitution, thread j solving U t = e_j, and *use_q = 1 with T = I when a pivot
// is zero or T is not finite.
template <int LM>
__global__ __launch_bounds__(LU_THREADS) void k_tslu_level(
    const double* __restrict__ Y, int64_t rows, int l, int64_t ldy, const int* __restrict__ cand,
    int64_t ncand, int per, int* __restrict__ out, double* __restrict__ T,
    int* __restrict__ use_q) {
  __shared__ unsigned long long skey[2][LU_THREADS / 64];
  __shared__ int srow[2][LU_THREADS / 64];
  __shared__ double prow[2][LU_THREADS / 64][LM];
  __shared__ double Ut[LM][LM];  // last level: Ut[c][j] = U_jc
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int64_t b = blockIdx.x;
  const bool last = gridDim.x == 1;
  int row = -1;
  if (cand == nullptr) {
    const int64_t rr = b * LU_THREADS + t;
    if (rr < rows) row = (int)rr;
  } else if (t < per && b * per + t < ncand) {
    row = cand[b * per + t];
  }
  double r[LM];
  if (row >= 0) {
    const double* y = Y + (int64_t)row * ldy;
#pragma unroll
    for (int c = 0; c < LM; ++c) r[c] = (c < l) ? y[c] : 0.0;
  } else {
#pragma unroll
    for (int c = 0; c < LM; ++c) r[c] = 0.0;
  }
  if (last)
    for (int i = t; i < LM * LM; i += LU_THREADS) (&Ut[0][0])[i] = 0.0;
  bool active = row >= 0;
  bool more = true;  // uniform: some candidate is left
  // runtime loop over the steps; the register arrays are indexed only by unrolled constants
  int j = 0;
#pragma unroll 1
  for (; j < l && more; ++j) {
    const int buf = j & 1;
    double rj = 0.0;
#pragma unroll
    for (int c = 0; c < LM; ++c)
      if (c == j) rj = r[c];
    unsigned long long key =
        active ? (unsigned long long)__double_as_longlong(fabs(rj)) + 1ull : 0ull;
    int who = active ? row : INT_MAX;
    wave_argmax(key, who);
    if (active && row == who) {  // the wave's pivot candidate (rows are distinct)
      skey[buf][wave] = key;
      srow[buf][wave] = who;
#pragma unroll
      for (int c = 0; c < LM; ++c) prow[buf][wave][c] = r[c];
    } else if (lane == 0 && key == 0ull) {
      skey[buf][wave] = 0ull;
      srow[buf][wave] = INT_MAX;
    }
    __syncthreads();
    unsigned long long bk = skey[buf][0];
    int br = srow[buf][0], bw = 0;
#pragma unroll
    for (int w = 1; w < LU_THREADS / 64; ++w) {
      if (lu_better(skey[buf][w], srow[buf][w], bk, br)) {
        bk = skey[buf][w];
        br = srow[buf][w];
        bw = w;
      }
    }
    if (bk == 0ull) {
      more = false;
    } else {
      const double* pr = prow[buf][bw];
      if (last && t >= j && t < l) Ut[t][j] = pr[t];
      if (active && row == br) active = false;
      if (active) {
        const double pj = pr[j];
        const double f = (pj != 0.0) ? rj / pj : 0.0;
#pragma unroll
        for (int c = 0; c < LM; ++c) {
          const double upd = fma(-f, pr[c], r[c]);
          r[c] = (c > j) ? upd : r[c];
        }
      }
    }
    if (t == 0) out[b * l + j] = more ? br : -1;
  }
  if (t == 0)
    for (; j < l; ++j) out[b * l + j] = -1;  // fewer than l candidates in this workgroup
  if (!last) return;
  __syncthreads();  // Ut complete
  double x[LM];
#pragma unroll
  for (int i = 0; i < LM; ++i) x[i] = (i == t) ? 1.0 : 0.0;
  // column sweep: x_p = x_p / U_pp, then x_i -= U_ip x_p for i < p
#pragma unroll 1
  for (int p = l - 1; p >= 0; --p) {
    double xp = 0.0;
#pragma unroll
    for (int i = 0; i < LM; ++i)
      if (i == p) xp = x[i];
    xp = xp / Ut[p][p];
#pragma unroll
    for (int i = 0; i < LM; ++i) {
      const double upd = fma(-Ut[p][i], xp, x[i]);
      x[i] = (i < p) ? upd : ((i == p) ? xp : x[i]);
    }
  }
  double ss = 0.0;
#pragma unroll
  for (int i = 0; i < LM; ++i) ss = fma(x[i], x[i], ss);
  const int ok = (t >= l) || isfinite(ss);
  const int bad = __syncthreads_or(!ok);
  if (t < l) {
#pragma unroll
    for (int i = 0; i < LM; ++i)
      if (i < l) T[(int64_t)i * l + t] = bad ? (i == t ? 1.0 : 0.0) : x[i];
  }
  if (t == 0) *use_q = bad;
}

template <int LM>
hipError_t tslu_levels(const double* Y, int64_t rows, int l, int64_t ldy, int* idx, double* T,
                       int* use_q, hipStream_t s) {
  int64_t groups = (rows + LU_THREADS - 1) / LU_THREADS;
  int* bufA = idx;
  int* bufB = idx + groups * l;
  hipLaunchKernelGGL(k_tslu_level<LM>, dim3((unsigned)groups), dim3(LU_THREADS), 0, s, Y, rows,
                     l, ldy, nullptr, rows, LU_THREADS, bufA, T, use_q);
  const int G = LU_THREADS / l;
  const int* in = bufA;
  int* outb = bufB;
  while (groups > 1) {
    const int64_t wgs = (groups + G - 1) / G;
    hipLaunchKernelGGL(k_tslu_level<LM>, dim3((unsigned)wgs), dim3(LU_THREADS), 0, s, Y, rows, l,
                       ldy, in, groups * l, G * l, outb, T, use_q);
    groups = wgs;
    int* nxt = (outb == bufA) ? bufB : bufA;
    in = outb;
    outb = nxt;
  }
  return hipGetLastError();
}

}  // namespace

size_t lu_index_ints(int64_t rows, int l) {
  const int64_t groups = (rows + LU_THREADS - 1) / LU_THREADS;
  const int G = LU_THREADS / (l > 0 ? l : 1);
  return (size_t)(groups + (groups + G - 1) / G) * (size_t)l;
}

hipError_t lu_tracking_T(const double* Y, int64_t rows, int l, int64_t ldy, int* idx, double* T,
                         int* use_q, hipStream_t s) {
  if (l < 1 || l > LU_L_MAX || rows < l) return hipErrorInvalidValue;
  if (l <= 16) return tslu_levels<16>(Y, rows, l, ldy, idx, T, use_q, s);
  if (l <= 32) return tslu_levels<32>(Y, rows, l, ldy, idx, T, use_q, s);
  return tslu_levels<64>(Y, rows, l, ldy, idx, T, use_q, s);
}

}  // namespace tsv
