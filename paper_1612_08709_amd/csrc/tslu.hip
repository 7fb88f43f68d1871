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

namespace tsv {
namespace {

constexpr int LU_THREADS = 256;  // 512 (fan-in 8) measured slower: more waves per barrier
constexpr int LU_TBITS = 8;       // bits of a thread index
// Columns are handled in chunks of 8: a chunk past the meaningful columns is skipped, and
// a chunk's 8 pivot-row values are loaded from LDS together before its 8 updates.
constexpr int LU_CHUNK = 8;

// Pivot search key of a candidate: the bit pattern of |v| (monotone in |v|; NaN sorts above
// +inf) with its low 9 bits replaced by an "active" bit and 255 - t, so that a larger |v|
// wins, then a smaller thread index, and every key in the workgroup is distinct.  Dropping
// 9 of the 52 mantissa bits lets a value within a relative 2^-43 of the largest win, which
// leaves partial pivoting's bound |multiplier| <= 1 + 2^-43.  Key 0: no candidate.
__device__ __forceinline__ unsigned long long lu_key(double v, int t) {
  const unsigned long long bits = (unsigned long long)__double_as_longlong(fabs(v));
  constexpr unsigned long long low = (1ull << (LU_TBITS + 1)) - 1;
  return (bits & ~low) | (1ull << LU_TBITS) | (unsigned long long)(LU_THREADS - 1 - t);
}

template <int CTRL>
__device__ __forceinline__ unsigned long long dpp_max(unsigned long long key) {
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)key, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(key >> 32), CTRL, 0xF, 0xF, false);
  const unsigned long long k2 = ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo;
  return k2 > key ? k2 : key;
}

__device__ __forceinline__ unsigned long long lane_key(unsigned long long key, int lane) {
  return ((unsigned long long)(unsigned)__builtin_amdgcn_readlane((int)(key >> 32), lane) << 32) |
         (unsigned)__builtin_amdgcn_readlane((int)(unsigned)key, lane);
}

// Wave maximum of the keys, returned uniform: DPP exchanges within each row of 16 lanes
// (quad swaps, half-row mirror, row mirror), then the four row maxima by readlane.
__device__ __forceinline__ unsigned long long wave_max_key(unsigned long long key) {
  key = dpp_max<0xB1>(key);
  key = dpp_max<0x4E>(key);
  key = dpp_max<0x141>(key);
  key = dpp_max<0x140>(key);
  unsigned long long best = lane_key(key, 0);
#pragma unroll
  for (int q = 1; q < 4; ++q) {
    const unsigned long long k2 = lane_key(key, 16 * q);
    best = k2 > best ? k2 : best;
  }
  return best;
}

// One level of the tournament.  Workgroup b's candidates: rows b*256 + t of Y at the leaf
// level (cand == nullptr), else cand[b*per + t] for t < per (-1: none).  Thread t keeps its
// candidate row in registers, shifted so that r[0] is always the column of the current
// step: at step j, r[c] holds column j + c.  Step j: the wave maximum of the keys of
// |r[0]|, one barrier, the best of the four waves' candidates is the pivot row p; every
// remaining candidate takes f = r[0] / p[0] and r[c] = r[c+1] - f p[c+1] (update and shift
// in one fused multiply-add).  The pivot row leaves the candidates with its registers
// holding row j of U (shifted); after the last step each pivot thread writes its row index
// to out[b*l + j] (pivot order; -1 where the workgroup ran out of candidates).
// With one workgroup (the last level) the pivot threads also write U to LDS, and the
// kernel writes T = U^-1 (l x l, row-major), thread t solving U x = e_t by the column sweep
// from the bottom: with d[c] = b_{p-c}, x_p = d[0] / U_pp and d[c] = d[c+1] - U_{p-1-c,p} x_p.
// *use_q = 1 and T = I when a pivot is zero or x is not finite.
template <int LM>
__global__ __launch_bounds__(LU_THREADS) void k_tslu_level(
    const double* __restrict__ Y, int64_t rows, int l, int64_t ldy, const int* __restrict__ cand,
    int64_t ncand, int per, int* __restrict__ out, double* __restrict__ T,
    int* __restrict__ use_q) {
  __shared__ unsigned long long skey[2][LU_THREADS / 64];
  __shared__ double prow[2][LU_THREADS / 64][LM + 1];
  __shared__ double Ur[LM][LM];  // last level: Ur[p][c] = U_{p-1-c, p} (column p upward)
  __shared__ double Ud[LM];      // last level: U_pp
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
  if (last) {
    for (int i = t; i < LM * LM; i += LU_THREADS) (&Ur[0][0])[i] = 0.0;
    if (t < LM) Ud[t] = 0.0;
  }
  bool active = row >= 0;
  int mystep = -1;  // the step at which this thread's row became the pivot
  int j = 0;
#pragma unroll 1
  for (; j < l; ++j) {
    const int buf = j & 1;
    const unsigned long long key = active ? lu_key(r[0], t) : 0ull;
    const unsigned long long wk = wave_max_key(key);
    if (wk != 0ull && key == wk) {  // this wave's candidate (keys are distinct)
      skey[buf][wave] = wk;
      // positions 0 .. l-1-j hold columns j .. l-1; the rest is never read
#pragma unroll
      for (int cc = 0; cc < LM; cc += LU_CHUNK)
        if (cc < l - j) {
#pragma unroll
          for (int u = 0; u < LU_CHUNK; ++u) prow[buf][wave][cc + u] = r[cc + u];
        }
    } else if (lane == 0 && wk == 0ull) {
      skey[buf][wave] = 0ull;
    }
    __syncthreads();
    unsigned long long bk = skey[buf][0];
    int bw = 0;
#pragma unroll
    for (int w = 1; w < LU_THREADS / 64; ++w) {
      const unsigned long long k2 = skey[buf][w];
      if (k2 > bk) {
        bk = k2;
        bw = w;
      }
    }
    if (bk == 0ull) break;  // uniform: no candidate left
    if (key == bk) {        // the pivot row: it keeps r (= row j of U, shifted) from here on
      active = false;
      mystep = j;
    }
    if (active) {
      const double* pr = prow[buf][bw];
      const double p0 = pr[0];
      const double f = (p0 != 0.0) ? r[0] / p0 : 0.0;
      // new positions 0 .. l-2-j are meaningful; a chunk past them is skipped (its
      // registers keep stale values, which no meaningful position ever reads)
#pragma unroll
      for (int cc = 0; cc < LM; cc += LU_CHUNK) {
        if (cc < l - 1 - j) {
          double q[LU_CHUNK];
#pragma unroll
          for (int u = 0; u < LU_CHUNK; ++u) q[u] = pr[cc + u + 1];
#pragma unroll
          for (int u = 0; u < LU_CHUNK; ++u)
            r[cc + u] = fma(-f, q[u], (cc + u + 1 < LM) ? r[cc + u + 1] : 0.0);
        }
      }
    }
  }
  if (mystep >= 0) out[b * l + mystep] = row;
  if (t == 0)
    for (int jj = j; jj < l; ++jj) out[b * l + jj] = -1;  // fewer than l candidates here
  if (last && mystep >= 0) {
    // U_{s, s+k} = r[k] for the pivot row of step s
    Ud[mystep] = r[0];
#pragma unroll
    for (int k = 1; k < LM; ++k)
      if (mystep + k < l) Ur[mystep + k][k - 1] = r[k];
  }
  if (!last) return;
  __syncthreads();  // Ur, Ud complete
  double d[LM];
#pragma unroll
  for (int c = 0; c < LM; ++c) d[c] = (l - 1 - c == t) ? 1.0 : 0.0;
  int ok = 1;
#pragma unroll 1
  for (int p = l - 1; p >= 0; --p) {
    const double xp = d[0] / Ud[p];
    ok &= isfinite(xp) ? 1 : 0;
    if (t < l) T[(int64_t)p * l + t] = xp;
    const double* up = Ur[p];
#pragma unroll
    for (int cc = 0; cc < LM; cc += LU_CHUNK) {
      if (cc < p) {
        double q[LU_CHUNK];
#pragma unroll
        for (int u = 0; u < LU_CHUNK; ++u) q[u] = up[cc + u];
#pragma unroll
        for (int u = 0; u < LU_CHUNK; ++u)
          d[cc + u] = fma(-q[u], xp, (cc + u + 1 < LM) ? d[cc + u + 1] : 0.0);
      }
    }
  }
  const int bad = __syncthreads_or((t < l) && !ok);
  if (bad && t < l)
    for (int i = 0; i < l; ++i) T[(int64_t)i * l + t] = (i == t) ? 1.0 : 0.0;
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
