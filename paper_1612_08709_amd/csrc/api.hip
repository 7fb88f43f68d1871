// C ABI: argument validation, workspace planning and the stream-ordered launch sequences
// of tsqr, tssvd (Algorithms 1-2) and lowrank_svd (Algorithm 7).  No allocation, no
// host synchronization: every step is enqueued on the caller's stream.
#include <math.h>
#include <string.h>

#include "common.h"
#include "internal.h"

#include <climits>
#include <mutex>

using namespace tsv;

namespace {

constexpr int VERSION = 100;  // 0.1.0

bool bad_dtype(int32_t d) { return d != TSSVD_F64 && d != TSSVD_F32; }

tssvd_opts resolve(const tssvd_opts* o) {
  tssvd_opts r;
  tssvd_default_opts(&r);
  if (o) r = *o;
  if (r.max_jacobi_sweeps <= 0) r.max_jacobi_sweeps = 30;
  if (!(r.reorth_tol > 0.0)) r.reorth_tol = 1e-13;
  return r;
}

int check_opts(const tssvd_opts& o) {
  if (o.prec != TSSVD_PREC_FP64 && o.prec != TSSVD_PREC_MIXED) return TSSVD_E_INVALID_ARG;
  if (o.ortho < TSSVD_ORTHO_AUTO || o.ortho > TSSVD_ORTHO_TWICE) return TSSVD_E_INVALID_ARG;
  if (!isfinite(o.working_precision)) return TSSVD_E_INVALID_ARG;
  return TSSVD_OK;
}

int hip_status(hipError_t e) { return e == hipSuccess ? TSSVD_OK : TSSVD_E_HIP; }

#define TRY(expr)                               \
  do {                                          \
    hipError_t _e = (expr);                     \
    if (_e != hipSuccess) return TSSVD_E_HIP;   \
  } while (0)

// ---------------------------------------------------------------- orthonormality gate
// M = sgn (G - shift I) (k x k, packed upper triangle in LDS) positive definite?  Right-
// looking Cholesky, one barrier per step; false at the first pivot that is not positive and
// finite (the pivot is read by every thread, so all leave together).
__device__ bool gate_chol_pd(double* M, const double* __restrict__ G, int k, double sgn,
                             double shift) {
  const int tid = threadIdx.x;
  auto off = [k](int i) { return i * k - (i * (i - 1)) / 2; };
  for (int idx = tid; idx < k * k; idx += 256) {
    const int i = idx / k, j = idx - i * k;
    if (j >= i) M[off(i) + (j - i)] = sgn * (G[idx] - (i == j ? shift : 0.0));
  }
  __syncthreads();
  const int ti = tid >> 4, tj = tid & 15;
  for (int kk = 0; kk < k; ++kk) {
    const double piv = M[off(kk)];
    if (!(piv > 0.0) || !isfinite(piv)) return false;
    const double inv = 1.0 / piv;
    const double* Mk = M + off(kk) - kk;  // Mk[j] = M(kk, j)
    for (int i = kk + 1 + ti; i < k; i += 16) {
      const double f = Mk[i] * inv;
      double* Mi = M + off(i) - i;
      for (int j = i + tj; j < k; j += 16) Mi[j] = fma(-f, Mk[j], Mi[j]);
    }
    __syncthreads();
  }
  return true;
}

// G = Q^T Q (k x k, k <= TSSVD_N_MAX).  ortho = ||G - I||_F, reported (an upper bound of the
// spectral norm).  gate = 1 when the second orthonormalization must run: always for TWICE;
// for AUTO when ||G - I||_2 > tol, decided exactly: ||G - I||_2 <= tol if and only if
// (1 + tol) I - G and G - (1 - tol) I are positive semidefinite, tested (as definite) by
// Cholesky; a Frobenius norm at or below tol settles it without the factorizations.
__global__ __launch_bounds__(256) void k_ortho_gate(const double* __restrict__ G, int k, int mode,
                                                    double tol, double* __restrict__ ortho_out,
                                                    int* __restrict__ gate, tssvd_info* info) {
  __shared__ double red[256];
  __shared__ double M[TSSVD_N_MAX * (TSSVD_N_MAX + 1) / 2];
  const int tid = threadIdx.x;
  double s = 0.0;
  for (int i = tid; i < k * k; i += 256) {
    const int r = i / k, c = i - r * k;
    const double d = G[i] - (r == c ? 1.0 : 0.0);
    s = fma(d, d, s);
  }
  red[tid] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) red[tid] += red[tid + w];
    __syncthreads();
  }
  const double o = sqrt(red[0]);
  int g;
  if (mode == TSSVD_ORTHO_TWICE) {
    g = 1;
  } else if (o <= tol) {
    g = 0;
  } else {
    const bool upper = gate_chol_pd(M, G, k, -1.0, 1.0 + tol);  // (1 + tol) I - G
    __syncthreads();
    const bool lower = upper && gate_chol_pd(M, G, k, 1.0, 1.0 - tol);  // G - (1 - tol) I
    g = !(upper && lower);
  }
  if (tid == 0) {
    *ortho_out = o;
    *gate = g;
    if (info) {
      info->ortho = o;
      info->reorth = g;
    }
  }
}

// R with R^T R = G (Cholesky, R upper triangular, row-major l x l) for the Gram G = Y^T Y of
// an intermediate basis.  One workgroup of 256 threads on a 16 x 16 grid, right-looking:
// thread (ti, tj) keeps the entries G_ij, i = ti + 16a, j = tj + 16b (i <= j), in registers.
// At step k the 16 threads of row group ti = k % 16 (one 16-lane row of a wave) take the
// pivot G_kk from its owner by a lane shuffle, put the row G_k. and 1 / G_kk in a
// double-buffered LDS row and turn its own entries of row k into row k of R (G_kj /
// sqrt(G_kk)); after one barrier every thread updates its entries, G_ij -= (G_ki / G_kk) G_kj.
// R leaves the registers once, at the end, so no barrier waits on global stores.  *bad = 1
// when a pivot is not positive and finite (then R is left unspecified).
// With `dead` given (l flags, written), a pivot <= dead_tol G_kk (the squared sine of the
// angle between column k of Y and the span of the earlier columns) drops direction k: row k
// of R stays zero and there is no trailing update, so Y = Q R still holds with the dropped
// column's coefficients in column k of R, and Q has no column k; dead[k] = 1 marks it.
// With `gate` given and *gate == 0 the kernel does nothing (a step that is not taken).
template <int NB>  // NB = ceil(l / 16)
__global__ __launch_bounds__(256) void k_chol(const double* __restrict__ G, int l,
                                              double* __restrict__ R, int* __restrict__ bad,
                                              double dead_tol, int* __restrict__ dead,
                                              const int* __restrict__ gate) {
  __shared__ double rowbuf[2][16 * NB];
  __shared__ double sinv[2];
  __shared__ int sstat[2];  // 0: pivot taken, 1: direction dropped, 2: failed
  __shared__ unsigned char sdead[TSSVD_N_MAX];
  __shared__ double sdiag[TSSVD_N_MAX];  // G_kk as given, for the drop test
  if (gate && *gate == 0) return;  // uniform over the workgroup
  const int tid = threadIdx.x, ti = tid >> 4, tj = tid & 15;
  for (int i = tid; i < l; i += 256) {
    sdead[i] = 0;
    sdiag[i] = G[i * l + i];
  }
  __syncthreads();  // the zeros land before any dead flag is written
  double g[NB][NB];
#pragma unroll
  for (int a = 0; a < NB; ++a)
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const int i = ti + 16 * a, j = tj + 16 * b;
      g[a][b] = (i < l && j < l && i <= j) ? G[i * l + j] : 0.0;
    }
  int fail = 0;
#pragma unroll
  for (int ka = 0; ka < NB; ++ka) {
    for (int kr = 0; kr < 16; ++kr) {
      const int k = 16 * ka + kr;
      if (k >= l) break;  // uniform
      const int buf = k & 1;
      if (ti == kr) {  // row group of k: one 16-lane row of a wave
        const double piv = __shfl(g[ka][ka], kr, 16);
        int st = 0;
        if (dead && piv <= dead_tol * sdiag[k])
          st = 1;
        else if (!(piv > 0.0) || !isfinite(piv))
          st = 2;
        const double rd = 1.0 / sqrt(piv), inv = 1.0 / piv;
#pragma unroll
        for (int b = 0; b < NB; ++b) {
          const int j = tj + 16 * b;
          if (j < l) {
            const double v = (j >= k && st == 0) ? g[ka][b] : 0.0;
            rowbuf[buf][j] = v;
            // row k of R, kept in place until the end (zero for a dropped direction, whose
            // pivot may be 0 or negative)
            g[ka][b] = (j >= k && st == 0) ? v * rd : 0.0;
          }
        }
        if (tj == 0) {
          sinv[buf] = inv;
          sstat[buf] = st;
          if (st == 1) sdead[k] = 1;
        }
      }
      __syncthreads();
      const int st = sstat[buf];
      if (st == 2) {  // uniform
        fail = 1;
        break;
      }
      if (st == 1) continue;
      // branch-free update: the row's entries are read once, blocks a, b < ka hold rows or
      // columns before k (nothing to do), and the rest select between old and new value
      const double inv = sinv[buf];
      double ri[NB], rj[NB];
#pragma unroll
      for (int a = ka; a < NB; ++a) {
        ri[a] = rowbuf[buf][ti + 16 * a];
        rj[a] = rowbuf[buf][tj + 16 * a];
      }
#pragma unroll
      for (int a = ka; a < NB; ++a) {
        const int i = ti + 16 * a;
        const bool live = i > k && i < l;
        const double gki = ri[a] * inv;
#pragma unroll
        for (int b = a; b < NB; ++b) {
          const int j = tj + 16 * b;
          const double nv = fma(-gki, rj[b], g[a][b]);
          g[a][b] = (live && j >= i && j < l) ? nv : g[a][b];
        }
      }
    }
    if (fail) break;  // uniform
  }
  // R: the rows each thread holds, zero below the diagonal
#pragma unroll
  for (int a = 0; a < NB; ++a)
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const int i = ti + 16 * a, j = tj + 16 * b;
      if (i < l && j < l) R[i * l + j] = (i <= j) ? g[a][b] : 0.0;
    }
  __syncthreads();
  if (dead)
    for (int i = tid; i < l; i += 256) dead[i] = sdead[i];
  if (tid == 0) *bad = fail;
}

hipError_t launch_chol(const double* G, int l, double* R, int* bad, double dead_tol, int* dead,
                       const int* gate, hipStream_t s) {
  switch ((l + 15) / 16) {
    case 1: hipLaunchKernelGGL(k_chol<1>, dim3(1), dim3(256), 0, s, G, l, R, bad, dead_tol, dead, gate); break;
    case 2: hipLaunchKernelGGL(k_chol<2>, dim3(1), dim3(256), 0, s, G, l, R, bad, dead_tol, dead, gate); break;
    case 3: hipLaunchKernelGGL(k_chol<3>, dim3(1), dim3(256), 0, s, G, l, R, bad, dead_tol, dead, gate); break;
    case 4: hipLaunchKernelGGL(k_chol<4>, dim3(1), dim3(256), 0, s, G, l, R, bad, dead_tol, dead, gate); break;
    case 5: hipLaunchKernelGGL(k_chol<5>, dim3(1), dim3(256), 0, s, G, l, R, bad, dead_tol, dead, gate); break;
    case 6: hipLaunchKernelGGL(k_chol<6>, dim3(1), dim3(256), 0, s, G, l, R, bad, dead_tol, dead, gate); break;
    case 7: hipLaunchKernelGGL(k_chol<7>, dim3(1), dim3(256), 0, s, G, l, R, bad, dead_tol, dead, gate); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Rm = R with each dropped direction's column replaced by e_k (row k of R is zero): the
// nonsingular matrix whose inverse, with row k zeroed, maps Y to the kept basis.
__global__ void k_unit_dead(const double* __restrict__ R, const int* __restrict__ dead, int l,
                            double* __restrict__ Rm, const int* __restrict__ gate) {
  if (gate && *gate == 0) return;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= l * l) return;
  const int i = idx / l, j = idx - i * l;
  Rm[idx] = dead[j] ? (i == j ? 1.0 : 0.0) : R[idx];
}

// Intermediate bases of the subspace iteration (Algorithm 5 before its last step) enter
// only through products with A, and Q = Y R^-1 spans the same space as the TSQR's
// Householder Q.  With T = R^-1 the m x l basis
// need not be formed by the reverse Householder pass.  Rounding in Y R^-1 grows with
// kappa(R); when the Frobenius estimate ||R||_F ||R^-1||_F exceeds kappa_max (or R^-1 is
// not finite, e.g. for a rank-deficient sketch) the kernel sets *use_q = 1 and T = I, and
// the gated Householder apply forms Q explicitly.  With `gate` given and *gate == 0 the
// kernel does nothing.
// 1024 threads: the 16-lane group c (c += 64) solves R t = e_c bottom-up with no barrier;
// lane L keeps t_k for k = L (mod 16) in registers and the dot products are 16-lane sums.
constexpr int RINV_THREADS = 1024;
constexpr int RINV_SLOTS = (TSSVD_N_MAX + 15) / 16;

__global__ __launch_bounds__(RINV_THREADS) void k_rinv_gate(const double* __restrict__ R, int l,
                                                            double kappa_max,
                                                            double* __restrict__ T,
                                                            int* __restrict__ use_q,
                                                            const int* __restrict__ force,
                                                            const int* __restrict__ gate) {
  extern __shared__ double Rs[];  // l x l, row-major
  __shared__ double red[2][RINV_THREADS / 16];
  __shared__ int bad;
  if (gate && *gate == 0) return;  // uniform over the workgroup
  const int tid = threadIdx.x, L = tid & 15, grp = tid >> 4;
  for (int i = tid; i < l * l; i += RINV_THREADS) Rs[i] = R[i];
  __syncthreads();
  double tn = 0.0;
  for (int c = grp; c < l; c += RINV_THREADS / 16) {
    double tk[RINV_SLOTS];
#pragma unroll
    for (int q = 0; q < RINV_SLOTS; ++q) tk[q] = 0.0;
    for (int i = c; i >= 0; --i) {
      double part = 0.0;
#pragma unroll
      for (int q = 0; q < RINV_SLOTS; ++q) {
        const int k = 16 * q + L;
        if (k > i && k <= c) part = fma(Rs[i * l + k], tk[q], part);
      }
      const double ti = ((i == c ? 1.0 : 0.0) - sum16(part)) / Rs[i * l + i];
#pragma unroll
      for (int q = 0; q < RINV_SLOTS; ++q)
        if (16 * q + L == i) tk[q] = ti;
    }
#pragma unroll
    for (int q = 0; q < RINV_SLOTS; ++q) {
      const int k = 16 * q + L;
      if (k < l) T[k * l + c] = (k <= c) ? tk[q] : 0.0;
      tn = fma(tk[q], tk[q], tn);
    }
  }
  double rn = 0.0;
  for (int idx = tid; idx < l * l; idx += RINV_THREADS) rn = fma(Rs[idx], Rs[idx], rn);
  tn = sum16(tn);
  rn = sum16(rn);
  if (L == 0) {
    red[0][grp] = tn;
    red[1][grp] = rn;
  }
  __syncthreads();
  if (tid == 0) {
    double a = 0.0, b = 0.0;
    for (int g2 = 0; g2 < RINV_THREADS / 16; ++g2) {
      a += red[0][g2];
      b += red[1][g2];
    }
    const double kap = sqrt(a) * sqrt(b);
    bad = !(kap <= kappa_max) || (force && *force);  // also catches NaN / Inf
    *use_q = bad;
  }
  __syncthreads();
  if (bad)
    for (int idx = tid; idx < l * l; idx += RINV_THREADS)
      T[idx] = (idx / l == idx % l) ? 1.0 : 0.0;
}

// The same two steps for l <= LM <= 64 in one wave, with no barrier: lane j owns column j.
// Cholesky (right-looking): at step k the pivot G_kk and the row R_k. = G_k. / sqrt(G_kk)
// come from lane k and from each lane, and G_ij -= R_ki R_kj updates lane j's column, R_ki
// a broadcast read of row k, which each step writes to LDS.  A lane keeps only the entries
// i <= j of its column
// meaningful; the rest take junk that is never read.  R goes to LDS transposed, and
// T = R^-1 follows by the column sweep of back substitution on the identity (lane j solves
// R t = e_j: t_p = b_p / R_pp, then b_i -= R_ip t_p for i < p), each R_ip a broadcast LDS
// read.  The gate is the one of k_rinv_gate; *chol_bad records a failed pivot.
__device__ __forceinline__ double lane_bcast(double x, int lane) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(x);
  const unsigned lo = __builtin_amdgcn_readlane((unsigned)u, lane);
  const unsigned hi = __builtin_amdgcn_readlane((unsigned)(u >> 32), lane);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

template <int LM>
__global__ __launch_bounds__(64) void k_chol_rinv_gate(const double* __restrict__ G, int l,
                                                       double kappa_max,
                                                       double* __restrict__ T,
                                                       int* __restrict__ use_q,
                                                       int* __restrict__ chol_bad) {
  __shared__ double Rt[LM * LM];  // Rt[p * LM + i] = R_ip
  __shared__ double Rrow[LM];      // row k of R during step k
  const int j = threadIdx.x;
  double g[LM];
  // unconditional loads from clamped addresses, all issued before any is used (the empty
  // asm statements take the values where they stand, so no load is sunk into the lane
  // condition below, where it would be waited for at once), then the selection
  const int jc = j < l ? j : l - 1;
#pragma unroll
  for (int i = 0; i < LM; ++i) g[i] = G[(i < l ? i : l - 1) * l + jc];
#pragma unroll
  for (int i = 0; i < LM; ++i) asm volatile("" : "+v"(g[i]));
#pragma unroll
  for (int i = 0; i < LM; ++i) g[i] = (j < l && i <= j) ? g[i] : 0.0;
  int fail = 0;
#pragma unroll
  for (int k = 0; k < LM; ++k) {
    if (k < l && !fail) {  // uniform
      const double piv = lane_bcast(g[k], k);
      if (!(piv > 0.0) || !isfinite(piv)) {
        fail = 1;
      } else {
        g[k] *= 1.0 / sqrt(piv);  // lane j >= k: R_kj
        // row k of R through LDS: one write, then broadcast reads (no lane-to-scalar moves)
        Rrow[j] = g[k];
        __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt 0: the row is written
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int i = k + 1; i < LM; ++i) g[i] = fma(-Rrow[i], g[k], g[i]);
      }
    }
  }
  double rn = 0.0;
#pragma unroll
  for (int i = 0; i < LM; ++i) {
    const double r = (i <= j && j < l) ? g[i] : 0.0;
    Rt[j * LM + i] = r;
    rn = fma(r, r, rn);
  }
  __builtin_amdgcn_s_waitcnt(0xc07f);  // the wave's LDS writes are done (lgkmcnt 0)
  __builtin_amdgcn_wave_barrier();
  // b's identity start is formed only now (from an opaque zero taken after the writes of R),
  // so it does not hold registers during the factorization
  int zero = 0;
  asm volatile("" : "+v"(zero));
  double b[LM];
#pragma unroll
  for (int i = 0; i < LM; ++i) b[i] = (i == j + zero) ? 1.0 : 0.0;
  if (!fail) {
#pragma unroll
    for (int p = LM - 1; p >= 0; --p) {
      // keeps each step's LDS reads in that step (hoisted ahead, they had been spilled)
      asm volatile("" ::: "memory");
      if (p < l) {
        const double t = b[p] / Rt[p * LM + p];
        b[p] = t;
#pragma unroll
        for (int i = 0; i < p; ++i) b[i] = fma(-Rt[p * LM + i], t, b[i]);
      }
    }
  }
  double tn = 0.0;
#pragma unroll
  for (int i = 0; i < LM; ++i) tn = fma(b[i], b[i], tn);
  if (j >= l) tn = 0.0;
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    rn += __shfl_xor(rn, off);
    tn += __shfl_xor(tn, off);
  }
  const double kap = sqrt(rn) * sqrt(tn);
  const int bad = fail || !(kap <= kappa_max);  // also catches NaN / Inf
  if (j < l) {
#pragma unroll
    for (int i = 0; i < LM; ++i)
      if (i < l) T[i * l + j] = bad ? (i == j ? 1.0 : 0.0) : b[i];
  }
  if (j == 0) {
    *use_q = bad;
    *chol_bad = fail;
  }
}

// ---------------------------------------------------------------- Gram-based SVD
// Algorithms 3 and 4 (and the bases of Algorithm 8) share one normalization step: the
// columns of U~ = Y V get their Euclidean norms explicitly (the paper's remark on
// normalizing), norms below max(norm) sqrt(wp) are discarded, and the kept columns are
// divided by their norms.  One workgroup (n <= 256 threads): thread j owns column j.
//   sumsq  : sum_i U~_ij^2 (input)
//   nrm    : the kept norms, 0 for a discarded column (output)
//   scale  : sgn_j / nrm_j, 0 for a discarded column (output)
//   pos    : with sort != 0, the column's place when the kept norms are sorted descending
//            (ties by index) and discarded columns follow in index order; else pos_j = j
//   sgn    : with sign != 0, the sign making w^T v_j >= 0 for V's column j (the output
//            sign convention); else 1
//   rank   : number of kept columns (optional; also written to info->rank when given)
//   out_sig: when given, the kept norms at their sorted places (0 for discarded ones)
__global__ __launch_bounds__(256) void k_gram_normalize(const double* __restrict__ sumsq, int n,
                                                        double wp, const double* __restrict__ V,
                                                        int ldv, int sort, int sign,
                                                        double* __restrict__ nrm,
                                                        double* __restrict__ scale,
                                                        int* __restrict__ pos,
                                                        int* __restrict__ rank,
                                                        double* __restrict__ out_sig,
                                                        tssvd_info* __restrict__ info) {
  __shared__ double s_n[256];
  __shared__ int s_keep[256];
  const int j = threadIdx.x;
  const double v = (j < n) ? sqrt(sumsq[j]) : 0.0;
  s_n[j] = v;
  __syncthreads();
  double mx = 0.0;
  for (int i = 0; i < n; ++i) mx = fmax(mx, s_n[i]);  // same order in every thread
  const double thr = (wp > 0.0) ? mx * sqrt(wp) : 0.0;
  const int keep = (j < n) && (v > 0.0) && !(v < thr) && isfinite(v);
  s_keep[j] = keep;
  __syncthreads();
  if (j >= n) return;
  double sg = 1.0;
  if (sign) {
    double d = 0.0;
    for (int i = 0; i < n; ++i) d = fma(sign_ref(i), V[i * ldv + j], d);
    sg = (d < 0.0) ? -1.0 : 1.0;
  }
  int p = j;
  if (sort) {
    p = 0;
    if (keep) {
      for (int i = 0; i < n; ++i)
        p += s_keep[i] && (s_n[i] > v || (s_n[i] == v && i < j));
    } else {
      for (int i = 0; i < n; ++i) p += s_keep[i] || (!s_keep[i] && i < j);
    }
  }
  nrm[j] = keep ? v : 0.0;
  scale[j] = keep ? sg / v : 0.0;
  pos[j] = p;
  if (out_sig) out_sig[p] = keep ? v : 0.0;
  if (j == 0 && (rank || info)) {
    int r = 0;
    for (int i = 0; i < n; ++i) r += s_keep[i];
    if (rank) *rank = r;
    if (info) info->rank = r;
  }
}

// Y (rows x n, stride ldy) in place: column j times scale_j, moved to column pos_j.  A
// workgroup stages GN_ROWS rows in LDS.
constexpr int GN_ROWS = 8;
__global__ __launch_bounds__(256) void k_scale_permute_cols(double* __restrict__ Y, int64_t rows,
                                                            int n, int64_t ldy,
                                                            const double* __restrict__ scale,
                                                            const int* __restrict__ pos) {
  __shared__ double buf[GN_ROWS * TSSVD_N_MAX];
  const int64_t r0 = (int64_t)blockIdx.x * GN_ROWS;
  const int cnt = (int)((rows - r0 < GN_ROWS) ? rows - r0 : GN_ROWS);
  for (int idx = threadIdx.x; idx < cnt * n; idx += 256) {
    const int r = idx / n, j = idx - r * n;
    buf[r * n + pos[j]] = Y[(r0 + r) * ldy + j] * scale[j];
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < cnt * n; idx += 256) {
    const int r = idx / n, j = idx - r * n;
    Y[(r0 + r) * ldy + j] = buf[r * n + j];
  }
}

// Small n x n results of the Gram routes (one thread per output entry, fixed order):
//   mode 0: Out[i][pos_j] = V[i][j] * sgn_j with sgn_j = sign(scale_j), 0 when scale_j = 0
//           (V of Algorithm 3, sorted and signed)
//   mode 1: Out[i][j] = V[i][j] * scale_j (T = V diag(1 / norm) of an Algorithm 3 basis)
__global__ void k_gram_small(const double* __restrict__ V, int n, const double* __restrict__ scale,
                             const int* __restrict__ pos, int mode, double* __restrict__ Out,
                             int ldo) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * n) return;
  const int i = idx / n, j = idx - i * n;
  const double sc = scale[j];
  if (mode == 0)
    Out[i * ldo + pos[j]] = (sc == 0.0) ? 0.0 : ((sc < 0.0) ? -V[i * n + j] : V[i * n + j]);
  else
    Out[i * ldo + j] = V[i * n + j] * sc;
}

// R = T W^T Sigma~ V~^T of Algorithm 4 (n x n): R_ij = t_i sum_k W_ki sigma~_k V~_jk.
__global__ void k_gram_R(const double* __restrict__ t, const double* __restrict__ W,
                         const double* __restrict__ sig, const double* __restrict__ Vt, int n,
                         double* __restrict__ R) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * n) return;
  const int i = idx / n, j = idx - i * n;
  double acc = 0.0;
  for (int k = 0; k < n; ++k) acc = fma(W[k * n + i] * sig[k], Vt[j * n + k], acc);
  R[idx] = t[i] * acc;
}

// Entries past the kept rank: sigma_j = 0 and columns j of P and V zeroed (the rank
// deficient directions of R in Algorithm 4 carry rounding-level singular values).
__global__ void k_truncate_rank(const int* __restrict__ rank, double* __restrict__ S, double* P,
                                int ldp, double* V, int ldv, int n, tssvd_info* info) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  const int r = *rank;
  if (idx == 0 && info) info->rank = r;
  if (idx >= n * n) return;
  const int i = idx / n, j = idx - i * n;
  if (j < r) return;
  if (i == 0) S[j] = 0.0;
  P[i * ldp + j] = 0.0;
  V[i * ldv + j] = 0.0;
}

// T = R diag(S) (n x n), for the second orthonormalization of U = Q2 R2.
__global__ void k_scale_cols(const double* __restrict__ R, const double* __restrict__ S, int n,
                             double* __restrict__ T, const int* __restrict__ gate) {
  if (*gate == 0) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n * n) T[i] = R[i] * S[i % n];
}

// C = A B for small n x n row-major matrices (one thread per output, fixed k order).
__global__ void k_small_gemm(const double* __restrict__ A, const double* __restrict__ B, int n,
                             double* __restrict__ C, const int* __restrict__ gate) {
  if (*gate == 0) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * n) return;
  const int r = i / n, c = i - r * n;
  double s = 0.0;
  for (int t = 0; t < n; ++t) s = fma(A[r * n + t], B[t * n + c], s);
  C[i] = s;
}

// C = op(A) op(B) for n x n row-major matrices, op = transpose when ta / tb is set.
__global__ void k_small_mm(const double* __restrict__ A, int ta, const double* __restrict__ B,
                           int tb, int n, double* __restrict__ C) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * n) return;
  const int r = i / n, c = i - r * n;
  double s = 0.0;
  for (int t = 0; t < n; ++t)
    s = fma(ta ? A[t * n + r] : A[r * n + t], tb ? B[c * n + t] : B[t * n + c], s);
  C[i] = s;
}

// Omega = Q diag(sign(diag R)) for G = Q R (n x n, row-major; R the TSQR root): the Q factor
// of a Gaussian matrix with the sign correction that makes it Haar-distributed.
__global__ void k_haar_fix(const double* __restrict__ Q, const double* __restrict__ R, int n,
                           double* __restrict__ Om) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * n) return;
  const int c = i % n;
  Om[i] = R[c * n + c] < 0.0 ? -Q[i] : Q[i];
}

struct TssvdWs {
  TsqrPlan p;                      // float32 leaf plan on the mixed-precision route
  // mixed: R1 (clamped); R2 = chol(Q1^T Q1) with kept columns, its unit-modified form and
  // that form's inverse; the second pass's R2 (clamped), R3 (kept, unit-modified, inverse);
  // Rtot, Ninv, N = Ninv P; the second pass's Gram; the solve's operand tiles and partial
  // Grams
  double *Rp = nullptr, *Rc = nullptr, *Rcm = nullptr, *Ri = nullptr, *Rp2 = nullptr;
  double *R3 = nullptr, *R3m = nullptr, *R3i = nullptr, *Rtot = nullptr, *Ninv = nullptr;
  double *Nm = nullptr, *G2 = nullptr, *op = nullptr, *pcpart = nullptr;
  int* mflags = nullptr;  // mixed: [0] first Cholesky failed, [1] unused, [2] second pass,
                          // [3] second Cholesky failed
  int *mdead = nullptr, *mdead2 = nullptr;  // mixed: dropped directions per pass (n flags)
  TsqrPlan pn;                     // mixing: QR factorizations of n x n matrices
  double *Om, *Mm, *Mu, *Mv;       // mixing: Omega, R Omega^T, and the small SVD's factors
  double *Ut, *S, *Vt, *T, *P2, *S2, *W2, *V2, *G, *part, *ortho;
  double *gnrm, *gnrm2, *gscale;  // Gram route: norms of the two passes, column scales
  int* gate;
  int* gpos;  // Gram route: column places (n) and the kept rank (one more int)
  size_t bytes;
};

// The mixed-precision tall-skinny route: A stored float32, 33 <= n (the float32 blocked
// leaf), no discard rule, no mixing, not the Gram route.
bool mixed_tssvd(const tssvd_opts& o, int32_t a_dtype, int64_t n) {
  return o.prec == TSSVD_PREC_MIXED && a_dtype == TSSVD_F32 && n >= 33;
}

TssvdWs tssvd_layout(int64_t m, int n, void* work, bool mixed = false) {
  TssvdWs w;
  Carver c(work);
  w.p = tsqr_plan(m, n, 0, 0, mixed);
  tsqr_carve(w.p, c);
  if (mixed) {
    const size_t nn = (size_t)n * n;
    w.Rp = c.take<double>(nn);
    w.Rc = c.take<double>(nn);
    w.Rcm = c.take<double>(nn);
    w.Ri = c.take<double>(nn);
    w.Rp2 = c.take<double>(nn);
    w.R3 = c.take<double>(nn);
    w.R3m = c.take<double>(nn);
    w.R3i = c.take<double>(nn);
    w.Rtot = c.take<double>(nn);
    w.Ninv = c.take<double>(nn);
    w.Nm = c.take<double>(nn);
    w.G2 = c.take<double>(nn);
    w.op = c.take<double>(pc_op_elems(n));
    w.pcpart = c.take<double>((size_t)pc_grid(m) * nn);
    w.mflags = c.take<int>(4);
    w.mdead = c.take<int>((size_t)n);
    w.mdead2 = c.take<int>((size_t)n);
  }
  w.pn = tsqr_plan(n, n);
  tsqr_carve(w.pn, c);
  const size_t nn = (size_t)n * n;
  w.Om = c.take<double>(nn);
  w.Mm = c.take<double>(nn);
  w.Mu = c.take<double>(nn);
  w.Mv = c.take<double>(nn);
  w.Ut = c.take<double>(nn);
  w.S = c.take<double>(n);
  w.Vt = c.take<double>(nn);
  w.T = c.take<double>(nn);
  w.P2 = c.take<double>(nn);
  w.S2 = c.take<double>(n);
  w.W2 = c.take<double>(nn);
  w.V2 = c.take<double>(nn);
  w.G = c.take<double>(nn);
  w.part = c.take<double>(atq_partials(m, n, n));
  w.ortho = c.take<double>(1);
  w.gnrm = c.take<double>(n);
  w.gnrm2 = c.take<double>(n);
  w.gscale = c.take<double>(n);
  w.gate = c.take<int>(4);
  w.gpos = c.take<int>((size_t)n + 1);
  w.bytes = c.off + 256;
  return w;
}

// Algorithm 3 (ortho == ONCE) or Algorithm 4 on A (m x n), every step on the GPU.  The
// eigendecompositions of the Gram matrices use the one-sided Jacobi kernel: for a symmetric
// positive semidefinite matrix the SVD is the eigendecomposition, sorted descending.  The
// m x n scratch is the TSQR plan's reflector storage, which this route does not use.
hipError_t tssvd_gram(const void* A, int a_dtype, int64_t m, int ni, int64_t lda, double* U,
                      int64_t ldu, double* S, double* V, int64_t ldv, tssvd_info* info,
                      TssvdWs& w, const tssvd_opts& o, hipStream_t s) {
  const int64_t n = ni;
  const double wp = o.working_precision;
  const unsigned gs = (unsigned)((ni * ni + 255) / 256);
  const unsigned gr = (unsigned)((m + GN_ROWS - 1) / GN_ROWS);
  int* rank = w.gpos + ni;
  double* scratch = w.p.Vleaf;
  hipError_t e;
#define GTRY(x) do { e = (x); if (e != hipSuccess) return e; } while (0)
  GTRY(gram_any(A, a_dtype, lda, m, ni, w.G, ni, w.part, s));                 // B = A^* A
  GTRY(jacobi_svd(w.G, ni, ni, 0, 0.0, o.max_jacobi_sweeps, 0, w.Ut, w.S, w.Vt, info, s));
  GTRY(gemm_ax_f64(A, a_dtype, lda, m, n, w.Vt, ni, ni, U, (int)ldu, s));    // U~ = A V
  GTRY(column_sumsq(U, TSSVD_F64, m, ni, ldu, w.S2, w.part, s));
  if (o.ortho == TSSVD_ORTHO_ONCE) {
    // Algorithm 3: U = U~ Sigma^-1, sorted by sigma, output sign convention
    hipLaunchKernelGGL(k_gram_normalize, dim3(1), dim3(256), 0, s, w.S2, ni, wp, w.Vt, ni, 1,
                       1, w.gnrm, w.gscale, w.gpos, rank, S, info);
    hipLaunchKernelGGL(k_scale_permute_cols, dim3(gr), dim3(256), 0, s, U, m, ni, ldu,
                       w.gscale, w.gpos);
    hipLaunchKernelGGL(k_gram_small, dim3(gs), dim3(256), 0, s, w.Vt, ni, w.gscale, w.gpos, 0,
                       V, (int)ldv);
    return hipGetLastError();
  }
  // Algorithm 4: Y = U~ Sigma~^-1 (in U), Z = Y^* Y = W D W^*, Q~ = Y W, T = norms of Q~,
  // Q = Q~ T^-1, R = T W^* Sigma~ V~^*, R = P Sigma V^*, U = Q P.
  hipLaunchKernelGGL(k_gram_normalize, dim3(1), dim3(256), 0, s, w.S2, ni, wp, w.Vt, ni, 0, 0,
                     w.gnrm, w.gscale, w.gpos, rank, nullptr, nullptr);
  hipLaunchKernelGGL(k_scale_permute_cols, dim3(gr), dim3(256), 0, s, U, m, ni, ldu, w.gscale,
                     w.gpos);
  GTRY(gram_any(U, TSSVD_F64, ldu, m, ni, w.G, ni, w.part, s));               // Z = Y^* Y
  GTRY(jacobi_svd(w.G, ni, ni, 0, 0.0, o.max_jacobi_sweeps, 0, w.P2, w.S, w.W2, info, s));
  GTRY(gemm_ax_f64(U, TSSVD_F64, ldu, m, n, w.W2, ni, ni, scratch, ni, s));   // Q~ = Y W
  GTRY(column_sumsq(scratch, TSSVD_F64, m, ni, ni, w.S2, w.part, s));
  hipLaunchKernelGGL(k_gram_normalize, dim3(1), dim3(256), 0, s, w.S2, ni, wp, w.W2, ni, 0, 0,
                     w.gnrm2, w.gscale, w.gpos, rank, nullptr, nullptr);
  hipLaunchKernelGGL(k_scale_permute_cols, dim3(gr), dim3(256), 0, s, scratch, m, ni,
                     (int64_t)ni, w.gscale, w.gpos);                            // Q
  hipLaunchKernelGGL(k_gram_R, dim3(gs), dim3(256), 0, s, w.gnrm2, w.W2, w.gnrm, w.Vt, ni,
                     w.T);
  GTRY(jacobi_svd(w.T, ni, ni, 0, 0.0, o.max_jacobi_sweeps, 1, w.P2, w.S2, w.V2, info, s));
  hipLaunchKernelGGL(k_truncate_rank, dim3(gs), dim3(256), 0, s, rank, w.S2, w.P2, ni, w.V2,
                     ni, ni, info);
  GTRY(gemm_ax_f64(scratch, TSSVD_F64, ni, m, n, w.P2, ni, ni, U, (int)ldu, s));  // U = Q P
  GTRY(copy_matrix(w.S2, 1, ni, ni, S, ni, s));
  GTRY(copy_matrix(w.V2, n, ni, ni, V, ldv, s));
#undef GTRY
  return hipGetLastError();
}

// Attributes for the one-workgroup Cholesky and triangular inverse at l up to
// TSSVD_N_MAX (their l x l matrices exceed the default 64 KB of LDS).
hipError_t chol_rinv_attrs() {
  static bool attr_set = false;  // the attribute is per function; setting it twice is harmless
  if (attr_set) return hipSuccess;
  hipError_t e = hipFuncSetAttribute((const void*)k_rinv_gate,
                                     hipFuncAttributeMaxDynamicSharedMemorySize,
                                     160 * 1024 - 8192);
  if (e != hipSuccess) return e;
  attr_set = true;
  return hipSuccess;
}

// Mixed precision, Algorithm 2 with its first orthonormalization in float32 and its second
// in float64 (A stored float32, 33 <= n <= TSSVD_N_MAX):
//   1. TSQR of A with the blocked leaf in float32 arithmetic and the merge tree in float64:
//      A ~ Q1 R1.  Householder's backward error is ~ eps_32 ||A|| per leaf chain (measured
//      1e-6 .. 4e-6 ||A|| for 8 .. 61 blocks of 128 rows), so the float32 factors cannot
//      give a residual ||A - U S V^T|| near float64 rounding; R1 serves as a preconditioner.
//      ONCE returns this step: SVD R1 = U1~ S1 V1~^T, U = Q1 U1~ from the float32
//      reflectors (orthonormal to ~1e-6).
//   2. Q1 = A R1^-1 in float64 by a blocked triangular solve of the stored A, so that
//      A = Q1 R1 is the first factorization of Algorithm 2 (with Q1 only nearly
//      orthonormal); Q1 is written to U and G = Q1^T Q1 formed by the staged Gram kernel.
//      A = Q1 R1 to float64 rounding (times the condition of R1's 16 x 16 diagonal blocks),
//      and kappa(Q1) ~ 1 + eps_32 kappa(A) c.
//   3. Algorithm 2's second factorization Q1 = Q R2 in float64, as a Cholesky QR of Q1:
//      R2 = chol(G) (T = R2 R1 as in the algorithm).  When the
//      estimate sqrt(||G||_1) ||R2^-1||_F of kappa(R2) exceeds kPcKappa, once more on
//      Q2 = Q1 R2^-1 (a second solve, in place in U) with R3 = chol(Q2^T Q2).
//   4. SVD of R = R2 R1 (R3 R2 R1) = P S W^T by float64 Jacobi; V = W, U = Q (R^-1 P), Q the
//      last stored basis, as a row-local product in place.
// Rank deficiency: a diagonal entry of R1 below kPcClamp max|R1_ii| (a column float32 sees
// as dependent) is raised to that size, which keeps Q1 bounded.  A column of Q1 dependent on
// the earlier ones to float64 rounding (squared sine of its angle to their span at most
// kMixedDeadSine2; a zero column) is dropped: its coefficients stay in R2, and the direction
// comes out as an exact zero singular value (sigma = 0, zero column of U).  A nearly
// dependent column stays; its large kappa(R2) calls the second Cholesky pass.
// info->ortho reports ||Q1^T Q1 - I||_F and info->reorth = 1.
constexpr double kMixedDeadSine2 = 1e-24;
constexpr double kPcClamp = 0x1p-24;
constexpr double kPcKappa = 64.0;

hipError_t tssvd_mixed(const void* A, int64_t m, int ni, int64_t lda, double* U, int64_t ldu,
                       double* S, double* V, int64_t ldv, tssvd_info* info, TssvdWs& w,
                       const tssvd_opts& o, hipStream_t s, bool prof) {
  const int64_t n = ni;
  const unsigned nb = (unsigned)((ni * ni + 255) / 256);
  hipError_t e;
#define MTRY(x) do { e = (x); if (e != hipSuccess) return e; } while (0)
  MTRY(tsqr_factor(w.p, A, TSSVD_F32, lda, s, prof));
  if (o.ortho == TSSVD_ORTHO_ONCE) {
    MTRY(jacobi_svd(tsqr_root(w.p), ni, ni, 1, 0.0, o.max_jacobi_sweeps, 1, w.Vt, w.S, w.Ut,
                    info, s));
    MTRY(tsqr_apply(w.p, w.Ut, ni, U, ldu, s, prof));
    MTRY(copy_matrix(w.S, 1, ni, ni, S, ni, s));
    MTRY(copy_matrix(w.Vt, n, ni, n, V, ldv, s));
    return hipGetLastError();
  }
  MTRY(pc_trsm_gram(tsqr_root(w.p), ni, ni, kPcClamp, w.Rp, w.op, A, TSSVD_F32, lda, m, U,
                    ldu, w.pcpart, w.G, nullptr, s, false));            // Q1 -> U
  MTRY(gram_any(U, TSSVD_F64, ldu, m, ni, w.G, ni, w.part, s));        // G = Q1^T Q1
  hipLaunchKernelGGL(k_ortho_gate, dim3(1), dim3(256), 0, s, w.G, ni, (int)TSSVD_ORTHO_TWICE,
                     o.reorth_tol, w.ortho, w.gate, info);               // gate = 1
  MTRY(chol_rinv_attrs());
  const size_t lds = (size_t)ni * ni * sizeof(double);
  MTRY(launch_chol(w.G, ni, w.Rc, w.mflags, kMixedDeadSine2, w.mdead, nullptr, s));  // R2
  hipLaunchKernelGGL(k_unit_dead, dim3(nb), dim3(256), 0, s, w.Rc, w.mdead, ni, w.Rcm,
                     (const int*)nullptr);
  hipLaunchKernelGGL(k_rinv_gate, dim3(1), dim3(RINV_THREADS), lds, s, w.Rcm, ni, 1e300, w.Ri,
                     w.mflags + 1, (const int*)nullptr, (const int*)nullptr);
  MTRY(pc_kappa_flag(w.G, w.Ri, ni, kPcKappa, w.mflags + 2, s));
  // second pass Q2 = Q1 R2m^-1 with its Cholesky and inverse, every step gated on mflags[2]
  // (k_pc_combine reads none of their outputs when the flag is 0)
  const int* g2 = w.mflags + 2;
  MTRY(pc_trsm_gram(w.Rcm, ni, ni, kPcClamp, w.Rp2, w.op, U, TSSVD_F64, ldu, m, U, ldu,
                    w.pcpart, w.G2, g2, s));
  MTRY(launch_chol(w.G2, ni, w.R3, w.mflags + 3, kMixedDeadSine2, w.mdead2, g2, s));
  hipLaunchKernelGGL(k_unit_dead, dim3(nb), dim3(256), 0, s, w.R3, w.mdead2, ni, w.R3m, g2);
  hipLaunchKernelGGL(k_rinv_gate, dim3(1), dim3(RINV_THREADS), lds, s, w.R3m, ni, 1e300, w.R3i,
                     w.mflags + 1, (const int*)nullptr, g2);
  MTRY(pc_combine(w.mflags, w.Rp, w.Rc, w.Rp2, w.Ri, w.R3, w.R3i, w.mdead, w.mdead2, ni,
                  w.Rtot, w.Ninv, info, s));
  MTRY(jacobi_svd(w.Rtot, ni, ni, 1, 0.0, o.max_jacobi_sweeps, 1, w.Vt, w.S, w.Ut, info, s));
  hipLaunchKernelGGL(k_small_gemm, dim3(nb), dim3(256), 0, s, w.Ninv, w.Ut, ni, w.Nm, w.gate);
  MTRY(pc_rowmul(U, ldu, m, ni, w.Nm, ni, w.op, nullptr, s));          // U = Q Ninv P
  MTRY(copy_matrix(w.S, 1, ni, ni, S, ni, s));
  MTRY(copy_matrix(w.Vt, n, ni, n, V, ldv, s));
#undef MTRY
  return hipGetLastError();
}

}  // namespace

// The workspace must start on 256 bytes (the kernels read their packed operands from it
// with 16-byte vector loads).
static bool misaligned(const void* work) {
  return (reinterpret_cast<uintptr_t>(work) & 255) != 0;
}

extern "C" {

void tssvd_default_opts(tssvd_opts* o) {
  if (!o) return;
  memset(o, 0, sizeof(*o));
  o->prec = TSSVD_PREC_FP64;
  o->ortho = TSSVD_ORTHO_AUTO;
  o->working_precision = 0.0;
  o->reorth_tol = 1e-13;
  o->max_jacobi_sweeps = 30;
  o->seed = 0x9E3779B97F4A7C15ull;
}

const char* tssvd_status_string(int status) {
  switch (status) {
    case TSSVD_OK: return "ok";
    case TSSVD_E_INVALID_ARG: return "invalid argument";
    case TSSVD_E_WORKSPACE: return "workspace missing or too small";
    case TSSVD_E_HIP: return "HIP launch failure";
    case TSSVD_E_UNSUPPORTED: return "unsupported size or option";
    default: return "unknown status";
  }
}

int tssvd_version(void) { return VERSION; }

// ---------------------------------------------------------------- tsqr
int tsqr_workspace_bytes(int64_t m, int64_t n, int32_t a_dtype, size_t* bytes) {
  if (!bytes || bad_dtype(a_dtype) || n < 1 || m < n) return TSSVD_E_INVALID_ARG;
  if (n > TSSVD_TSQR_N_MAX) return TSSVD_E_UNSUPPORTED;
  TsqrPlan p = tsqr_plan(m, (int)n);
  Carver c(nullptr);
  tsqr_carve(p, c);
  c.take<double>((size_t)n * n);
  *bytes = c.off + 256;
  return TSSVD_OK;
}

int tsqr(const void* A, int32_t a_dtype, int64_t m, int64_t n, int64_t lda, double* Q,
         int64_t ldq, double* R, int64_t ldr, void* work, size_t work_bytes, void* stream) {
  if (!A || !R || bad_dtype(a_dtype) || n < 1 || m < n || lda < n || ldr < n ||
      (Q && ldq < n))
    return TSSVD_E_INVALID_ARG;
  if (n > TSSVD_TSQR_N_MAX) return TSSVD_E_UNSUPPORTED;
  size_t need = 0;
  tsqr_workspace_bytes(m, n, a_dtype, &need);
  if (!work || work_bytes < need || misaligned(work)) return TSSVD_E_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  TsqrPlan p = tsqr_plan(m, (int)n);
  Carver c(work);
  tsqr_carve(p, c);
  double* I = c.take<double>((size_t)n * n);
  TRY(tsqr_factor(p, A, a_dtype, lda, s));
  TRY(copy_matrix(tsqr_root(p), n, (int)n, n, R, ldr, s));
  if (Q) {
    TRY(fill_identity(I, (int)n, (int)n, s));
    TRY(tsqr_apply(p, I, (int)n, Q, ldq, s));
  }
  return TSSVD_OK;
}

// ---------------------------------------------------------------- tssvd
int tssvd_workspace_bytes(int64_t m, int64_t n, int32_t a_dtype, const tssvd_opts* opts,
                          size_t* bytes) {
  if (!bytes || bad_dtype(a_dtype) || n < 1 || m < n) return TSSVD_E_INVALID_ARG;
  if (n > TSSVD_N_MAX) return TSSVD_E_UNSUPPORTED;
  const tssvd_opts o = resolve(opts);
  *bytes = tssvd_layout(m, (int)n, nullptr, mixed_tssvd(o, a_dtype, n)).bytes;
  return TSSVD_OK;
}

}  // extern "C"

// Scratch of tssvd_noalloc: device memory in the code object, one copy per GPU, held
// until the process ends.  Host code never passes `scratch` itself to a kernel (on the
// host the name is only a stand-in); it passes the device address that
// hipGetSymbolAddress returns for the current device, looked up once per device.
static __device__ __align__(256) unsigned char scratch[TSSVD_NOALLOC_SCRATCH_BYTES];

namespace {

// The body of tssvd; prof = false keeps the measurement markers (which create HIP events
// on first use) out of the call.
int tssvd_run(const void* A, int32_t a_dtype, int64_t m, int64_t n, int64_t lda, double* U,
              int64_t ldu, double* S, double* V, int64_t ldv, tssvd_info* info, void* work,
              size_t work_bytes, const tssvd_opts* opts, void* stream, bool prof) {
  if (!A || !U || !S || !V || bad_dtype(a_dtype) || n < 1 || m < n || lda < n || ldu < n ||
      ldv < n)
    return TSSVD_E_INVALID_ARG;
  const tssvd_opts o = resolve(opts);
  if (check_opts(o) != TSSVD_OK) return TSSVD_E_INVALID_ARG;
  if (n > TSSVD_N_MAX) return TSSVD_E_UNSUPPORTED;
  const int ni = (int)n;
  const bool mixed = mixed_tssvd(o, a_dtype, n);
  if (o.prec == TSSVD_PREC_MIXED) {
    if (a_dtype != TSSVD_F32) return TSSVD_E_INVALID_ARG;
    if (!mixed || o.working_precision > 0.0 || (o.flags & (TSSVD_FLAG_MIX | TSSVD_FLAG_GRAM)))
      return TSSVD_E_UNSUPPORTED;
  }
  TssvdWs w = tssvd_layout(m, ni, work, mixed);
  if (!work || work_bytes < w.bytes || misaligned(work)) return TSSVD_E_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;

  const bool mix = (o.flags & TSSVD_FLAG_MIX) != 0;
  if (mix && (o.flags & TSSVD_FLAG_GRAM)) return TSSVD_E_INVALID_ARG;
  TRY(info_init(info, s));
  if (mixed)
    return hip_status(tssvd_mixed(A, m, ni, lda, U, ldu, S, V, ldv, info, w, o, s, prof));
  if (o.flags & TSSVD_FLAG_GRAM)
    return hip_status(tssvd_gram(A, a_dtype, m, ni, lda, U, ldu, S, V, ldv, info, w, o, s));
  // Algorithm 1: TSQR A = Q R; SVD R = U~ S V~^T (discard rule inside); U = Q U~.
  // The one-sided Jacobi runs on R^T (R^T W = P S gives R = W S P^T: U~ = W, V~ = P),
  // whose columns converge in about half the sweeps that R's need when R's columns are
  // mixed (measured 10 vs 23 sweeps for n = 100, sigma from 1 to 1e-6).
  TRY(tsqr_factor(w.p, A, a_dtype, lda, s, prof));
  const unsigned nb = (unsigned)((ni * ni + 255) / 256);
  if (!mix) {
    TRY(jacobi_svd(tsqr_root(w.p), ni, ni, 1, o.working_precision, o.max_jacobi_sweeps, 1,
                   w.Vt, w.S, w.Ut, info, s));
  } else {
    // Step (1) with the mixing moved onto R: A = Q0 R0 and R0 Omega^T = Q1 R' give
    // A Omega^T = (Q0 Q1) R', the factorization of the mixed matrix, at O(n^3) instead of a
    // pass over A.  Omega is the sign-corrected Q of an n x n Philox Gaussian (Haar).  The
    // discard rule then reads the diagonal of R'; V = Omega^T V~ and U = Q0 (Q1 U~).
    TRY(philox_sketch(w.Om, n, ni, o.seed, s));                       // G
    TRY(tsqr_factor(w.pn, w.Om, TSSVD_F64, n, s));                     // G = QG RG
    TRY(fill_identity(w.Mv, ni, ni, s));
    TRY(tsqr_apply(w.pn, w.Mv, ni, w.Mu, n, s));                       // QG
    hipLaunchKernelGGL(k_haar_fix, dim3(nb), dim3(256), 0, s, w.Mu, tsqr_root(w.pn), ni, w.Om);
    hipLaunchKernelGGL(k_small_mm, dim3(nb), dim3(256), 0, s, tsqr_root(w.p), 0, w.Om, 1, ni,
                       w.Mm);                                          // R0 Omega^T
    TRY(tsqr_factor(w.pn, w.Mm, TSSVD_F64, n, s));                     // = Q1 R'
    TRY(jacobi_svd(tsqr_root(w.pn), ni, ni, 1, o.working_precision, o.max_jacobi_sweeps, 0,
                   w.Mv, w.S, w.Mu, info, s));                         // R' = U~ S V~^T
    hipLaunchKernelGGL(k_small_mm, dim3(nb), dim3(256), 0, s, w.Om, 1, w.Mv, 0, ni, w.Vt);
    TRY(tsqr_apply(w.pn, w.Mu, ni, w.Ut, n, s));                       // Q1 U~
    TRY(sign_fix_cols(w.Vt, n, ni, ni, w.Ut, ni, ni, s));
  }
  TRY(tsqr_apply(w.p, w.Ut, ni, U, ldu, s, prof));
  TRY(copy_matrix(w.S, 1, ni, ni, S, ni, s));
  TRY(copy_matrix(w.Vt, n, ni, n, V, ldv, s));
  if (o.ortho == TSSVD_ORTHO_ONCE) return TSSVD_OK;

  // Second orthonormalization (Algorithm 2), written for U = Q2 R2:
  //   A = Q2 (R2 diag(S)) V^T,  SVD(R2 diag(S)) = P S' W^T,  U' = Q2 P, V' = V W.
  // The discard rule of Algorithm 2 step 5 tests the diagonal of R2.  Gate: always for
  // TWICE; for AUTO when ||U^T U - I||_F > reorth_tol.  The host cannot read the gate
  // without a synchronization, so the pass is always enqueued and every kernel of it
  // returns at once when the gate is 0.
  TRY(gram_any(U, TSSVD_F64, ldu, m, ni, w.G, ni, w.part, s));
  hipLaunchKernelGGL(k_ortho_gate, dim3(1), dim3(256), 0, s, w.G, ni, o.ortho, o.reorth_tol,
                     w.ortho, w.gate, info);
  TsqrPlan p2 = w.p;
  p2.gate = w.gate;
  TRY(tsqr_factor(p2, U, TSSVD_F64, ldu, s));
  hipLaunchKernelGGL(k_scale_cols, dim3((ni * ni + 255) / 256), dim3(256), 0, s,
                     tsqr_root(p2), w.S, ni, w.T, w.gate);
  TRY(jacobi_svd(w.T, ni, ni, 0, o.working_precision, o.max_jacobi_sweeps, 0, w.P2, w.S2,
                 w.W2, info, s, w.gate, tsqr_root(p2), ni));
  hipLaunchKernelGGL(k_small_gemm, dim3((ni * ni + 255) / 256), dim3(256), 0, s, w.Vt, w.W2,
                     ni, w.V2, w.gate);
  TRY(sign_fix_cols(w.V2, n, ni, ni, w.P2, ni, ni, s, w.gate));
  TRY(tsqr_apply(p2, w.P2, ni, U, ldu, s));
  TRY(copy_matrix(w.S2, 1, ni, ni, S, ni, s, w.gate));
  TRY(copy_matrix(w.V2, n, ni, n, V, ldv, s, w.gate));
  return hip_status(hipGetLastError());
}

constexpr int SCRATCH_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[SCRATCH_MAX_DEVICES] = {};

int scratch_address(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return TSSVD_E_HIP;
  if (dev < 0 || dev >= SCRATCH_MAX_DEVICES) return TSSVD_E_UNSUPPORTED;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return TSSVD_E_HIP;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return TSSVD_OK;
}

}  // namespace

extern "C" {

int tssvd(const void* A, int32_t a_dtype, int64_t m, int64_t n, int64_t lda, double* U,
          int64_t ldu, double* S, double* V, int64_t ldv, tssvd_info* info, void* work,
          size_t work_bytes, const tssvd_opts* opts, void* stream) {
  return tssvd_run(A, a_dtype, m, n, lda, U, ldu, S, V, ldv, info, work, work_bytes, opts,
                   stream, true);
}

int tssvd_noalloc(const void* A, int32_t a_dtype, int64_t m, int64_t n, int64_t lda,
                  double* U, int64_t ldu, double* S, double* V, int64_t ldv, tssvd_info* info,
                  const tssvd_opts* opts, void* stream) {
  if (!A || !U || !S || !V || bad_dtype(a_dtype) || n < 1 || m < n || lda < n || ldu < n ||
      ldv < n)
    return TSSVD_E_INVALID_ARG;
  if (n > TSSVD_N_MAX) return TSSVD_E_UNSUPPORTED;
  const bool mixed = mixed_tssvd(resolve(opts), a_dtype, n);
  if (tssvd_layout(m, (int)n, nullptr, mixed).bytes > (size_t)TSSVD_NOALLOC_SCRATCH_BYTES)
    return TSSVD_E_UNSUPPORTED;
  void* work = nullptr;
  const int st = scratch_address(&work);
  if (st != TSSVD_OK) return st;
  return tssvd_run(A, a_dtype, m, n, lda, U, ldu, S, V, ldv, info, work,
                   (size_t)TSSVD_NOALLOC_SCRATCH_BYTES, opts, stream, false);
}

}  // extern "C"

// ---------------------------------------------------------------- lowrank_svd
namespace {

struct LowrankWs {
  TsqrPlan pY, pZ;
  double *X, *Y, *Z, *Zraw, *part, *I, *P, *sig, *W, *Wk, *G, *ortho, *Tq, *Rc;
  double *gsum, *gnrm, *gscale;  // Gram route (Algorithm 8): norms and column scales
  int* gpos;                     // Gram route: column places (l) and the kept rank
  int* luidx;                    // LU tracking: tournament candidates
  void* pack;
  void* Acopy;  // bfloat16 copy of A for the mixed power steps (or null)
  int* gate;
  size_t bytes;
};

LowrankWs lowrank_layout(int64_t m, int64_t n, int k, int l, void* work, bool mixed,
                         bool acopy) {
  LowrankWs w;
  Carver c(work);
  w.pY = tsqr_plan(m, l);
  tsqr_carve(w.pY, c);
  w.pZ = tsqr_plan(n, l);
  tsqr_carve(w.pZ, c);
  w.X = c.take<double>((size_t)n * l);
  w.Y = c.take<double>((size_t)m * l);
  w.Z = c.take<double>((size_t)n * l);
  w.Zraw = c.take<double>((size_t)n * l);
  size_t np = atq_partials(m, n, l);
  const size_t np2 = atq_partials(m, l, l);
  if (np2 > np) np = np2;
  const size_t np3 = atq_partials(n, l, l);
  if (np3 > np) np = np3;
  if (mixed && mixed_partials(m, n, l) > np) np = mixed_partials(m, n, l);
  w.part = c.take<double>(np);
  w.pack = nullptr;
  if (mixed) {
    size_t pb = mixed_pack_bytes(m, l);
    if (mixed_pack_bytes(n, l) > pb) pb = mixed_pack_bytes(n, l);
    w.pack = c.take<char>(pb);
  }
  w.Acopy = acopy ? (void*)c.take<char>(bf16_copy_bytes(m, n)) : nullptr;
  const size_t ll = (size_t)l * l;
  w.I = c.take<double>(ll);
  w.P = c.take<double>(ll);
  w.sig = c.take<double>(l);
  w.W = c.take<double>(ll);
  w.Wk = c.take<double>((size_t)l * k);
  w.G = c.take<double>(ll);
  w.Tq = c.take<double>(ll);
  w.Rc = c.take<double>(ll);
  w.ortho = c.take<double>(1);
  w.gsum = c.take<double>(l);
  w.gnrm = c.take<double>(l);
  w.gscale = c.take<double>(l);
  w.gpos = c.take<int>((size_t)l + 1);
  w.luidx = c.take<int>(l <= LU_L_MAX ? lu_index_ints(m > n ? m : n, l) : 1);
  w.gate = c.take<int>(4);
  w.bytes = c.off + 256;
  return w;
}

int lowrank_check(const void* A, int32_t a_dtype, int64_t m, int64_t n, int64_t lda, int64_t k,
                  int64_t l, int64_t q) {
  if (!A || bad_dtype(a_dtype) || m < 1 || n < 1 || lda < n) return TSSVD_E_INVALID_ARG;
  if (!(0 < k && k <= l && l < m && l < n) || q < 0) return TSSVD_E_INVALID_ARG;
  if (l > TSSVD_N_MAX) return TSSVD_E_UNSUPPORTED;
  return TSSVD_OK;
}

// Discard rule of Algorithms 1-2 inside Algorithm 5 (wp > 0): the columns j of the
// Householder Q whose |R_jj| < wp |R_11| (R the TSQR root, row-major l x l) are zeroed, so
// the basis keeps only the numerically independent directions.  Gated (skipped when *gate
// == 0); *kept (optional) receives the number of kept columns.
__global__ void k_discard_cols(double* __restrict__ Y, int64_t rows, int l, int64_t ldy,
                               const double* __restrict__ R, double wp,
                               const int* __restrict__ gate, int* __restrict__ kept) {
  if (gate && *gate == 0) return;
  const double thr = wp * fabs(R[0]);
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx == 0 && kept) {
    int r = 0;
    for (int j = 0; j < l; ++j) r += !(fabs(R[j * l + j]) < thr);
    *kept = r;
  }
  if (idx >= rows * l) return;
  const int64_t i = idx / l;
  const int j = (int)(idx - i * l);
  if (fabs(R[j * l + j]) < thr) Y[i * ldy + j] = 0.0;
}

// Orthonormal basis of span(Y) by TSQR, written over Y (m x l).
// Basis of an intermediate step (rows x l, row-major): R from the Cholesky factor of the
// Gram Y^T Y (CholeskyQR), T = R^-1, Y kept.  The basis Y R^-1 loses orthogonality like
// kappa(Y)^2 eps, harmless for an intermediate step as long as kappa is moderate, so when
// the Cholesky factorization fails or ||R||_F ||R^-1||_F > 1e4 the device gate falls back to
// the TSQR of Y with the explicit Householder Q written over Y and T = I.
// Algorithm 3 on Y (rows x l, FP64, stride l) as an l x l map: T = V diag(1 / norm_j), so
// that Y T = (Y V) diag(1 / norm) is Algorithm 3's normalized left factor.  The Gram matrix
// Y^* Y is eigendecomposed by the one-sided Jacobi kernel (its SVD, for a positive
// semidefinite matrix), Y V is formed in `scratch` (rows x l) for the explicit column norms,
// and norms below max(norm) sqrt(wp) give zero columns of T.  l x l buffers: G, E (the
// eigenvectors), Ud and sd (unused Jacobi outputs).
hipError_t gram_basis(const double* Y, int64_t rows, int l, double wp, int sweeps, double* G,
                      double* E, double* Ud, double* sd, double* scratch, double* sumsq,
                      double* nrm, double* scale, int* pos, int* rank, double* T, double* part,
                      tssvd_info* info, hipStream_t s) {
  hipError_t e = gram_any(Y, TSSVD_F64, l, rows, l, G, l, part, s);            // Y^* Y
  if (e != hipSuccess) return e;
  e = jacobi_svd(G, l, l, 0, 0.0, sweeps, 0, Ud, sd, E, info, s);              // = V D V^*
  if (e != hipSuccess) return e;
  e = gemm_ax_f64(Y, TSSVD_F64, l, rows, l, E, l, l, scratch, l, s);           // Y V
  if (e != hipSuccess) return e;
  e = column_sumsq(scratch, TSSVD_F64, rows, l, l, sumsq, part, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_gram_normalize, dim3(1), dim3(256), 0, s, sumsq, l, wp, E, l, 0, 0, nrm,
                     scale, pos, rank, nullptr, nullptr);
  hipLaunchKernelGGL(k_gram_small, dim3((l * l + 255) / 256), dim3(256), 0, s, E, l, scale, pos,
                     1, T, l);
  return hipGetLastError();
}

constexpr double kKappaMax = 1e4;
// T = R^-1 for the Cholesky factor R^T R = G, with the kappa gate of k_rinv_gate (*use_q = 1
// and T = I when ||R||_F ||R^-1||_F > kmax or the factorization fails, *chol_bad = 1 for the
// latter).  Rc: l x l scratch (l > 64).
hipError_t chol_rinv(const double* G, int l, double kmax, double* T, int* use_q, int* chol_bad,
                     double* Rc, hipStream_t s) {
  hipError_t e = chol_rinv_attrs();
  if (e != hipSuccess) return e;
  if (l <= 16) {
    hipLaunchKernelGGL(k_chol_rinv_gate<16>, dim3(1), dim3(64), 0, s, G, l, kmax, T, use_q,
                       chol_bad);
  } else if (l <= 32) {
    hipLaunchKernelGGL(k_chol_rinv_gate<32>, dim3(1), dim3(64), 0, s, G, l, kmax, T, use_q,
                       chol_bad);
  } else if (l <= 64) {
    hipLaunchKernelGGL(k_chol_rinv_gate<64>, dim3(1), dim3(64), 0, s, G, l, kmax, T, use_q,
                       chol_bad);
  } else {
    e = launch_chol(G, l, Rc, chol_bad, 0.0, nullptr, nullptr, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_rinv_gate, dim3(1), dim3(RINV_THREADS), (size_t)l * l * sizeof(double),
                       s, Rc, l, kmax, T, use_q, chol_bad, (const int*)nullptr);
  }
  return hipGetLastError();
}

// With *gate == 0 (the second orthonormalization is not taken): T = I and *use_q = 0.
__global__ void k_gate_identity(const int* __restrict__ gate, double* __restrict__ T, int l,
                                int* __restrict__ use_q) {
  if (*gate != 0) return;
  for (int i = threadIdx.x; i < l * l; i += blockDim.x) T[i] = (i / l == i % l) ? 1.0 : 0.0;
  if (threadIdx.x == 0) *use_q = 0;
}

hipError_t basis_via_r(const TsqrPlan& p, double* Y, int64_t rows, int l, const double* I,
                       double* T, double* G, double* Rc, double* part, int* flags,
                       hipStream_t s, double wp = 0.0) {
  int* use_q = flags;
  int* chol_bad = flags + 1;
  // wp > 0 (the paper's discard): every basis is the TSQR's Householder Q, with the
  // discard applied on its R; kappa_max = 0 makes the device gate take that branch
  const double kmax = (wp > 0.0) ? 0.0 : kKappaMax;
  hipError_t e = gemm_atq_f64(Y, TSSVD_F64, l, rows, l, Y, l, l, G, l, part, s);  // Y^T Y
  if (e != hipSuccess) return e;
  e = chol_rinv(G, l, kmax, T, use_q, chol_bad, Rc, s);
  if (e != hipSuccess) return e;
  TsqrPlan pq = p;
  pq.gate = use_q;
  e = tsqr_factor(pq, Y, TSSVD_F64, l, s);
  if (e != hipSuccess) return e;
  e = tsqr_apply(pq, I, l, Y, l, s);
  if (e != hipSuccess || !(wp > 0.0)) return e;
  hipLaunchKernelGGL(k_discard_cols, dim3((unsigned)((rows * l + 255) / 256)), dim3(256), 0, s, Y,
                     rows, l, (int64_t)l, tsqr_root(pq), wp, use_q, nullptr);
  return hipGetLastError();
}

// Basis of an intermediate step from an LU factorization (Section 3's remark on tracking):
// T = U^-1 with U from the tournament-pivoted LU of Y, so that Y T = L (rows in Y's order).
// A singular or non-finite U sets *use_q and falls back to the TSQR's Householder Q, as
// for a rejected Cholesky basis.
hipError_t basis_via_lu(const TsqrPlan& p, double* Y, int64_t rows, int l, const double* I,
                        double* T, int* idx, int* use_q, hipStream_t s) {
  hipError_t e = lu_tracking_T(Y, rows, l, l, idx, T, use_q, s);
  if (e != hipSuccess) return e;
  TsqrPlan pq = p;
  pq.gate = use_q;
  e = tsqr_factor(pq, Y, TSSVD_F64, l, s);
  if (e != hipSuccess) return e;
  return tsqr_apply(pq, I, l, Y, l, s);
}

hipError_t orth_inplace(const TsqrPlan& p, double* Y, int l, const double* I, hipStream_t s) {
  hipError_t e = tsqr_factor(p, Y, TSSVD_F64, l, s);
  if (e != hipSuccess) return e;
  return tsqr_apply(p, I, l, Y, l, s);
}

}  // namespace

extern "C" {

int lowrank_svd_workspace_bytes(int64_t m, int64_t n, int64_t k, int64_t l, int64_t q,
                                int32_t a_dtype, const tssvd_opts* opts, size_t* bytes) {
  if (!bytes) return TSSVD_E_INVALID_ARG;
  int st = lowrank_check((const void*)1, a_dtype, m, n, n, k, l, q);
  if (st != TSSVD_OK) return st;
  const bool mixed = opts && opts->prec == TSSVD_PREC_MIXED;
  const bool acopy = mixed && q >= 1 && !(opts->flags & TSSVD_FLAG_NO_A_COPY);
  *bytes = lowrank_layout(m, n, (int)k, (int)l, nullptr, mixed, acopy).bytes;
  return TSSVD_OK;
}

int lowrank_svd(const void* A, int32_t a_dtype, int64_t m, int64_t n, int64_t lda, int64_t k,
                int64_t l, int64_t q, const double* Omega, double* U, int64_t ldu, double* S,
                double* V, int64_t ldv, tssvd_info* info, void* work, size_t work_bytes,
                const tssvd_opts* opts, void* stream) {
  int st = lowrank_check(A, a_dtype, m, n, lda, k, l, q);
  if (st != TSSVD_OK) return st;
  if (!U || !S || !V || ldu < k || ldv < k) return TSSVD_E_INVALID_ARG;
  const tssvd_opts o = resolve(opts);
  if (check_opts(o) != TSSVD_OK) return TSSVD_E_INVALID_ARG;
  const bool mixed = o.prec == TSSVD_PREC_MIXED;
  if (mixed && a_dtype != TSSVD_F32) return TSSVD_E_INVALID_ARG;
  const bool gram = (o.flags & TSSVD_FLAG_GRAM) != 0;
  const bool lu = (o.flags & TSSVD_FLAG_LU) != 0;
  const double wp = o.working_precision;  // > 0: the paper's discard rule (rank-deficient mode)
  if (lu && gram) return TSSVD_E_INVALID_ARG;
  if (o.flags & TSSVD_FLAG_MIX) return TSSVD_E_UNSUPPORTED;
  // the tournament keeps row indices as int
  if (lu && (wp > 0.0 || l > LU_L_MAX || m > INT_MAX - 1024 || n > INT_MAX - 1024))
    return TSSVD_E_UNSUPPORTED;
  const int ki = (int)k, li = (int)l;
  const bool acopy = mixed && q >= 1 && !(o.flags & TSSVD_FLAG_NO_A_COPY);
  LowrankWs w = lowrank_layout(m, n, ki, li, work, mixed, acopy);
  if (!work || work_bytes < w.bytes || misaligned(work)) return TSSVD_E_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;

  TRY(info_init(info, s));
  TRY(fill_identity(w.I, li, li, s));
  if (Omega)
    TRY(copy_matrix(Omega, n, li, l, w.X, l, s));
  else
    TRY(philox_sketch(w.X, n, li, o.seed, s));
  // Products with A.  FP64: float64 MFMA on A as stored.  MIXED: bfloat16 inputs in the
  // power steps, float32 inputs for the last sketch and for B (the operand is packed first).
  const float* A32 = static_cast<const float*>(A);
  const bool f32_final = (o.flags & TSSVD_FLAG_F32_MFMA_FINAL) != 0;
  // With the bfloat16 copy, the first power-step pass reads the float32 A and stores it
  // rounded to bfloat16; the other power-step passes read the copy (same bfloat16 values).
  bool copy_ready = false;
  auto ax = [&](const double* Xs, bool last) -> hipError_t {
    if (!mixed) return gemm_ax_f64(A, a_dtype, lda, m, n, Xs, li, li, w.Y, li, s, TSSVD_PROF_AX);
    const int kind = !last ? MIX_BF16P : (f32_final ? MIX_F32_AX : MIX_BF16X3);
    hipError_t e = pack_operand(Xs, n, li, li, kind, w.pack, s);
    if (e != hipSuccess) return e;
    if (last)
      return gemm_ax_mixed(A32, lda, m, n, w.pack, li, w.Y, li, kind, s, TSSVD_PROF_AX_FINAL);
    if (copy_ready)
      return gemm_ax_bf16c(w.Acopy, m, n, w.pack, li, w.Y, li, s, TSSVD_PROF_AX_BF16C);
    copy_ready = w.Acopy != nullptr;
    return gemm_ax_bf16p(A32, lda, m, n, w.pack, li, w.Y, li, w.Acopy, s, TSSVD_PROF_AX_BF16);
  };
  // Qs == nullptr: the operand is already packed (bfloat16, power steps)
  auto atq = [&](const double* Qs, bool last, double* Zout) -> hipError_t {
    if (!mixed)
      return gemm_atq_f64(A, a_dtype, lda, m, n, Qs, li, li, Zout, li, w.part, s,
                          TSSVD_PROF_ATQ);
    const int kind = !last ? MIX_BF16 : (f32_final ? MIX_F32_ROWS : MIX_BF16X3);
    if (Qs) {
      hipError_t e = pack_operand(Qs, m, li, li, kind, w.pack, s);
      if (e != hipSuccess) return e;
    }
    if (!last && copy_ready)
      return gemm_atq_bf16c(w.Acopy, m, n, w.pack, li, Zout, li, w.part, s,
                            TSSVD_PROF_ATQ_BF16C);
    return gemm_atq_mixed(A32, lda, m, n, w.pack, li, Zout, li, w.part, kind, s,
                          last ? TSSVD_PROF_ATQ_FINAL : TSSVD_PROF_ATQ_BF16);
  };
  // Algorithm 5: subspace iteration.  Intermediate bases: Q_j = Y R_j^-1 and
  // Q~_j = Z R~_j^-1 (or the explicit Householder Q when R is ill-conditioned).  In FP64
  // the product uses Y itself, A^* Q_j = (A^* Y) R_j^-1; in mixed precision Q_j is formed
  // first (in FP64, written straight out as bfloat16 operand fragments), because
  // bfloat16 rounding of Y's entries would be amplified by R_j^-1.
  // Algorithm 8 (TSSVD_FLAG_GRAM): the same loop with T from Algorithm 3 instead.
  int* use_q = w.gate + 1;
  int* grank = w.gpos + li;
  auto basis = [&](const TsqrPlan& p, double* Yb, int64_t rows) -> hipError_t {
    if (lu) return basis_via_lu(p, Yb, rows, li, w.I, w.Tq, w.luidx, use_q, s);
    if (!gram)
      return basis_via_r(p, Yb, rows, li, w.I, w.Tq, w.G, w.Rc, w.part, use_q, s, wp);
    return gram_basis(Yb, rows, li, o.working_precision, o.max_jacobi_sweeps, w.G, w.W, w.P,
                      w.sig, p.Vleaf, w.gsum, w.gnrm, w.gscale, w.gpos, grank, w.Tq, w.part,
                      info, s);
  };
  TRY(ax(w.X, q == 0));                                                        // A Q~_0
  for (int64_t j = 0; j < q; ++j) {
    TRY(basis(w.pY, w.Y, m));                                                  // Q_j = Y T
    if (mixed) {
      TRY(gemm_ax_f64_pack_bf16(w.Y, l, m, w.Tq, li, li, w.pack, s));         // Q_j, packed
      TRY(atq(nullptr, false, w.Z));                                           // A^* Q_j
    } else {
      TRY(atq(w.Y, false, w.Zraw));                                            // A^* Y
      TRY(gemm_ax_f64(w.Zraw, TSSVD_F64, l, n, l, w.Tq, li, li, w.Z, li, s)); // A^* Q_j
    }
    TRY(basis(w.pZ, w.Z, n));                                                  // Q~_j = Z T
    TRY(gemm_ax_f64(w.Z, TSSVD_F64, l, n, l, w.Tq, li, li, w.X, li, s));
    TRY(ax(w.X, j == q - 1));                                                  // A Q~_j
  }
  // the last basis by CholeskyQR twice (Algorithm 2 form) unless a discard rule, Algorithm 8,
  // LU tracking or a single orthonormalization (ONCE: the TSQR's Q) is asked for
  const bool cqr_last = !gram && !lu && !(wp > 0.0) && o.ortho != TSSVD_ORTHO_ONCE;
  if (gram) {
    // Algorithm 4 on the last Y: Y1 = Y T1 (Algorithm 3), then Q = Y1 T2 (Algorithm 3 on Y1);
    // the kept rank of the second pass bounds the rank of the result
    double* Y1 = w.pY.Vleaf;
    TRY(basis(w.pY, w.Y, m));
    TRY(gemm_ax_f64(w.Y, TSSVD_F64, l, m, l, w.Tq, li, li, Y1, li, s));
    TRY(gram_basis(Y1, m, li, o.working_precision, o.max_jacobi_sweeps, w.G, w.W, w.P, w.sig,
                   w.Y, w.gsum, w.gnrm, w.gscale, w.gpos, grank, w.Tq, w.part, info, s));
    TRY(gemm_ax_f64(Y1, TSSVD_F64, l, m, l, w.Tq, li, li, w.Y, li, s));      // Q
  } else if (cqr_last) {
    // Algorithm 2's two orthonormalizations on the last Y, both as CholeskyQR (each gated to
    // the TSQR like the intermediate bases): Q1 = Y R1^-1 (into Y1), G = Q1^T Q1 decides the
    // second one as in tssvd, Q = Q1 R2^-1 (T2 = I when it is not taken).  A failed second
    // Cholesky leaves T2 = I and the gated TSQR orthonormalizes Q in place.
    double* Y1 = w.pY.Vleaf;
    TRY(basis(w.pY, w.Y, m));                                                  // T1 = R1^-1
    TRY(gemm_ax_f64(w.Y, TSSVD_F64, l, m, l, w.Tq, li, li, Y1, li, s));      // Q1
    TRY(gemm_atq_f64(Y1, TSSVD_F64, l, m, l, Y1, li, li, w.G, li, w.part, s));
    hipLaunchKernelGGL(k_ortho_gate, dim3(1), dim3(256), 0, s, w.G, li, o.ortho, o.reorth_tol,
                       w.ortho, w.gate, info);
    TRY(chol_rinv(w.G, li, kKappaMax, w.Tq, use_q, use_q + 1, w.Rc, s));     // T2 = R2^-1
    hipLaunchKernelGGL(k_gate_identity, dim3(1), dim3(256), 0, s, w.gate, w.Tq, li, use_q);
    TRY(gemm_ax_f64(Y1, TSSVD_F64, l, m, l, w.Tq, li, li, w.Y, li, s));      // Q
    TsqrPlan p2 = w.pY;
    p2.gate = use_q;
    TRY(tsqr_factor(p2, w.Y, TSSVD_F64, l, s));
    TRY(tsqr_apply(p2, w.I, li, w.Y, l, s));
  } else {
    TRY(orth_inplace(w.pY, w.Y, li, w.I, s));                                  // Q
    if (wp > 0.0)
      hipLaunchKernelGGL(k_discard_cols, dim3((unsigned)((m * l + 255) / 256)), dim3(256), 0, s,
                         w.Y, m, li, l, tsqr_root(w.pY), wp, nullptr, grank);
  }
  if (!gram && !cqr_last && o.ortho != TSSVD_ORTHO_ONCE) {
    // last step orthonormalized twice (Algorithm 2 form), gated like tssvd; with the discard
    // the second pass always runs (Algorithm 2) and applies the rule again
    TRY(gemm_atq_f64(w.Y, TSSVD_F64, l, m, l, w.Y, li, li, w.G, li, w.part, s));
    hipLaunchKernelGGL(k_ortho_gate, dim3(1), dim3(256), 0, s, w.G, li,
                       wp > 0.0 ? (int)TSSVD_ORTHO_TWICE : o.ortho, o.reorth_tol, w.ortho,
                       w.gate, info);
    TsqrPlan p2 = w.pY;
    p2.gate = w.gate;
    TRY(tsqr_factor(p2, w.Y, TSSVD_F64, l, s));
    TRY(tsqr_apply(p2, w.I, li, w.Y, l, s));
    if (wp > 0.0)
      hipLaunchKernelGGL(k_discard_cols, dim3((unsigned)((m * l + 255) / 256)), dim3(256), 0, s,
                         w.Y, m, li, l, tsqr_root(p2), wp, w.gate, grank);
  }
  // Algorithm 6: B = Q^* A via B^* = A^* Q = Q_B R_B;  R_B^T = P S W^T  =>
  //   B = P S (Q_B W)^T,  U = Q P_k,  V = Q_B W_k.
  TRY(atq(w.Y, true, w.Z));                                                    // B^* = A^* Q
  TRY(tsqr_factor(w.pZ, w.Z, TSSVD_F64, l, s));
  TRY(jacobi_svd(tsqr_root(w.pZ), li, li, 1, 0.0, o.max_jacobi_sweeps, 0, w.P, w.sig, w.W,
                 info, s));
  if (gram || wp > 0.0)  // directions dropped by a discard carry rounding-level values
    hipLaunchKernelGGL(k_truncate_rank, dim3((li * li + 255) / 256), dim3(256), 0, s, grank,
                       w.sig, w.P, li, w.W, li, li, info);
  TRY(copy_matrix(w.W, l, ki, l, w.Wk, k, s));
  TRY(tsqr_apply(w.pZ, w.Wk, ki, V, ldv, s));
  TRY(sign_fix_cols(V, n, (int)ldv, ki, w.P, li, li, s));
  TRY(gemm_ax_f64(w.Y, TSSVD_F64, l, m, l, w.P, li, ki, U, (int)ldu, s));
  TRY(copy_matrix(w.sig, 1, ki, k, S, k, s));
  return hip_status(hipGetLastError());
}

// ---------------------------------------------------------------- lowrank_svd_backward
}  // extern "C"

namespace {

struct BackwardWs {
  TsqrPlan pY, pZ;
  int K2;
  // Rj, Rtj: R^-1 of each factorization (the QR layer of the reverse pass needs only that)
  double *Lcat, *Rcat, *Rj, *Rtj, *Y, *Z, *Xbar, *Qtbar, *I, *Ub, *sig, *Ws, *Wfull, *G1, *G2,
      *A1, *KB, *Kw, *Kv, *UbkT, *M, *Rinv, *K1, *K2m, *part;
  int* flags;  // basis gate: [0] the TSQR branch was taken, [1] the Cholesky failed, [2] unused
  size_t bytes;
};

BackwardWs backward_layout(int64_t m, int64_t n, int k, int l, int q, void* work) {
  BackwardWs w;
  Carver c(work);
  w.pY = tsqr_plan(m, l);
  tsqr_carve(w.pY, c);
  w.pZ = tsqr_plan(n, l);
  tsqr_carve(w.pZ, c);
  w.K2 = (2 * q + 2) * l;
  const size_t ll = (size_t)l * l;
  w.Lcat = c.take<double>((size_t)m * w.K2);
  w.Rcat = c.take<double>((size_t)n * w.K2);
  w.Rj = c.take<double>((size_t)(q + 1) * ll);
  w.Rtj = c.take<double>((size_t)(q + 1) * ll);
  w.Y = c.take<double>((size_t)m * l);
  w.Z = c.take<double>((size_t)n * l);
  w.Xbar = c.take<double>((size_t)m * l);
  w.Qtbar = c.take<double>((size_t)n * l);
  w.I = c.take<double>(ll);
  w.Ub = c.take<double>(ll);
  w.sig = c.take<double>(l);
  w.Ws = c.take<double>(ll);
  w.Wfull = c.take<double>((size_t)n * l);
  w.G1 = c.take<double>((size_t)l * k);
  w.G2 = c.take<double>((size_t)l * k);
  w.A1 = c.take<double>(ll);
  w.KB = c.take<double>(ll);
  w.Kw = c.take<double>(ll);
  w.Kv = c.take<double>((size_t)k * l);
  w.UbkT = c.take<double>((size_t)k * l);
  w.M = c.take<double>(ll);
  w.Rinv = c.take<double>(ll);
  w.K1 = c.take<double>(ll);
  w.K2m = c.take<double>(ll);
  size_t np = atq_partials(m, n, l);
  const size_t cand[3] = {atq_partials(m, l, l), atq_partials(n, l, l), atq_partials(m, l, k)};
  for (size_t x : cand)
    if (x > np) np = x;
  w.part = c.take<double>(np);
  w.flags = c.take<int>(4);
  w.bytes = c.off + 256;
  return w;
}

// Ybar = [Xbar - Qx copyltu(Xbar^T Qx)] R^-T, written to out (rows x l, stride ldo); Ri = R^-1.
hipError_t qr_back(BackwardWs& w, const double* Xbar, int64_t ldx, const double* Qx, int64_t ldq,
                   const double* Ri, int64_t rows, int l, double* out, int64_t ldo,
                   hipStream_t s) {
  hipError_t e = gemm_atq_f64(Xbar, TSSVD_F64, ldx, rows, l, Qx, (int)ldq, l, w.M, l, w.part, s);
  if (e != hipSuccess) return e;
  e = bw_qr_coef_rinv(w.M, Ri, l, w.K1, w.K2m, s);
  if (e != hipSuccess) return e;
  return rmul(Xbar, ldx, l, w.K1, Qx, ldq, l, w.K2m, rows, l, out, ldo, false, s);
}

}  // namespace

extern "C" {

int lowrank_svd_backward_workspace_bytes(int64_t m, int64_t n, int64_t k, int64_t l, int64_t q,
                                         int32_t a_dtype, const tssvd_opts* opts,
                                         size_t* bytes) {
  if (!bytes) return TSSVD_E_INVALID_ARG;
  int st = lowrank_check((const void*)1, a_dtype, m, n, n, k, l, q);
  if (st != TSSVD_OK) return st;
  (void)opts;
  *bytes = backward_layout(m, n, (int)k, (int)l, (int)q, nullptr).bytes;
  return TSSVD_OK;
}

int lowrank_svd_backward(const void* A, int32_t a_dtype, int64_t m, int64_t n, int64_t lda,
                         int64_t k, int64_t l, int64_t q, const double* Omega, const double* U,
                         int64_t ldu, const double* S, const double* V, int64_t ldv,
                         const double* gU, const double* gS, const double* gV, void* gA,
                         int64_t ldga, tssvd_info* info, void* work, size_t work_bytes,
                         const tssvd_opts* opts, void* stream) {
  int st = lowrank_check(A, a_dtype, m, n, lda, k, l, q);
  if (st != TSSVD_OK) return st;
  if (!gA || ldga < n || ldu < k || ldv < k) return TSSVD_E_INVALID_ARG;
  const tssvd_opts o = resolve(opts);
  if (check_opts(o) != TSSVD_OK) return TSSVD_E_INVALID_ARG;
  if (o.prec != TSSVD_PREC_FP64 || o.working_precision > 0.0 ||
      (o.flags & (TSSVD_FLAG_GRAM | TSSVD_FLAG_LU | TSSVD_FLAG_MIX)))
    return TSSVD_E_UNSUPPORTED;
  (void)U; (void)S; (void)V;  // the forward is recomputed from (A, Omega); see the header
  const int ki = (int)k, li = (int)l, qi = (int)q;
  BackwardWs w = backward_layout(m, n, ki, li, qi, work);
  if (!work || work_bytes < w.bytes || misaligned(work)) return TSSVD_E_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  const int K2 = w.K2;
  const size_t ll = (size_t)li * li;
  auto Lblk = [&](int b) { return w.Lcat + (size_t)b * li; };
  auto Rblk = [&](int b) { return w.Rcat + (size_t)b * li; };

  TRY(info_init(info, s));
  TRY(fill_identity(w.I, li, li, s));
  // ---- recompute the forward (Algorithm 7, one orthonormalization per factorization)
  if (Omega)
    TRY(copy_matrix(Omega, n, li, l, Rblk(1), K2, s));
  else {
    TRY(philox_sketch(w.Z, n, li, o.seed, s));
    TRY(copy_matrix(w.Z, n, li, l, Rblk(1), K2, s));
  }
  // The intermediate bases as the forward takes them (the CholeskyQR basis of Algorithm 7
  // with the device gate to the TSQR, reading 14): Q = Y T with T = R^-1, kept as the QR
  // layer's R^-1.  When the gate takes the TSQR branch, T = I, Y holds the Householder Q,
  // and R^-1 is formed from the TSQR's R by the same gated inverse kernel.
  TRY(chol_rinv_attrs());
  auto basis = [&](const TsqrPlan& p, double* Yb, int64_t rows, double* Ri,
                   double* Qout) -> hipError_t {
    hipError_t e = basis_via_r(p, Yb, rows, li, w.I, Ri, w.M, w.K1, w.part, w.flags, s);
    if (e != hipSuccess) return e;
    e = gemm_ax_f64(Yb, TSSVD_F64, l, rows, l, Ri, li, li, Qout, K2, s);  // Q = Y T
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_rinv_gate, dim3(1), dim3(RINV_THREADS), ll * sizeof(double), s,
                       tsqr_root(p), li, 1e300, Ri, w.flags + 2, (const int*)nullptr,
                       (const int*)w.flags);  // TSQR branch: R^-1 of its R (T was I)
    return hipGetLastError();
  };
  for (int j = 1; j <= qi; ++j) {
    TRY(gemm_ax_f64(A, a_dtype, lda, m, n, Rblk(j), K2, li, w.Y, li, s));
    TRY(basis(w.pY, w.Y, m, w.Rj + (j - 1) * ll, Lblk(qi + 1 + j)));         // Q_j
    TRY(gemm_atq_f64(A, a_dtype, lda, m, n, Lblk(qi + 1 + j), K2, li, w.Z, li, w.part, s));
    TRY(basis(w.pZ, w.Z, n, w.Rtj + (j - 1) * ll, Rblk(1 + j)));             // Q~_j
  }
  // the last basis by the TSQR (Algorithm 7, one orthonormalization), its R inverted
  TRY(gemm_ax_f64(A, a_dtype, lda, m, n, Rblk(1 + qi), K2, li, w.Y, li, s));
  TRY(tsqr_factor(w.pY, w.Y, TSSVD_F64, l, s));
  TRY(bw_rinv(tsqr_root(w.pY), li, w.Rj + qi * ll, s));
  TRY(tsqr_apply(w.pY, w.I, li, Lblk(0), K2, s));                          // Q
  TRY(gemm_atq_f64(A, a_dtype, lda, m, n, Lblk(0), K2, li, w.Z, li, w.part, s));  // B^T
  TRY(tsqr_factor(w.pZ, w.Z, TSSVD_F64, l, s));
  TRY(jacobi_svd(tsqr_root(w.pZ), li, li, 1, 0.0, o.max_jacobi_sweeps, 0, w.Ub, w.sig, w.Ws,
                 info, s));
  TRY(tsqr_apply(w.pZ, w.Ws, li, w.Wfull, l, s));                          // W = Q_B W~
  TRY(sign_fix_cols(w.Wfull, n, li, ki, w.Ub, li, li, s));                 // as in the forward

  // ---- SVD layer: G1 = Q^T gU, G2 = W^T gV, core coefficients, Bbar^T
  if (gU)
    TRY(gemm_atq_f64(Lblk(0), TSSVD_F64, K2, m, l, gU, (int)ldu, ki, w.G1, ki, w.part, s));
  else
    TRY(zero_fill(w.G1, (int64_t)li * ki, s));
  if (gV)
    TRY(gemm_atq_f64(w.Wfull, TSSVD_F64, l, n, l, gV, (int)ldv, ki, w.G2, ki, w.part, s));
  else
    TRY(zero_fill(w.G2, (int64_t)li * ki, s));
  TRY(bw_svd_core(w.Ub, w.sig, w.G1, w.G2, gS, li, ki, w.A1, w.KB, w.Kw, w.Kv, w.UbkT, s));
  TRY(rmul(w.Wfull, l, li, w.Kw, gV, ldv, gV ? ki : 0, w.Kv, n, li, Rblk(0), K2, false, s));
  // ---- Qbar = A Bbar^T + gU Ub_k^T, then the QR layer of the last factorization
  TRY(gemm_ax_f64(A, a_dtype, lda, m, n, Rblk(0), K2, li, w.Xbar, li, s, TSSVD_PROF_AX));
  if (gU) TRY(rmul(gU, ldu, ki, w.UbkT, nullptr, 0, 0, nullptr, m, li, w.Xbar, l, true, s));
  TRY(qr_back(w, w.Xbar, l, Lblk(0), K2, w.Rj + qi * ll, m, li, Lblk(qi + 1), K2, s));
  // ---- walk the subspace iteration backwards
  for (int j = qi; j >= 1; --j) {
    TRY(gemm_atq_f64(A, a_dtype, lda, m, n, Lblk(j + 1), K2, li, w.Qtbar, li, w.part, s,
                     TSSVD_PROF_ATQ));                                      // A^T Ybar_{j+1}
    TRY(qr_back(w, w.Qtbar, l, Rblk(1 + j), K2, w.Rtj + (j - 1) * ll, n, li, Rblk(qi + 1 + j),
                K2, s));                                                    // Zbar_j
    TRY(gemm_ax_f64(A, a_dtype, lda, m, n, Rblk(qi + 1 + j), K2, li, w.Xbar, li, s,
                    TSSVD_PROF_AX));                                        // A Zbar_j
    TRY(qr_back(w, w.Xbar, l, Lblk(qi + 1 + j), K2, w.Rj + (j - 1) * ll, m, li, Lblk(j), K2,
                s));                                                        // Ybar_j
  }
  // ---- Abar = [Q | Ybar_1..Ybar_{q+1} | Q_1..Q_q] [Bbar^T | Q~_0..Q~_q | Zbar_1..Zbar_q]^T
  TRY(gemm_nt(w.Lcat, K2, w.Rcat, K2, m, n, K2, gA, a_dtype, ldga, s));
  return hip_status(hipGetLastError());
}

// ---------------------------------------------------------------- measurement support
int tssvd_profile_enable(int on) {
  prof_enable(on != 0);
  return TSSVD_OK;
}

int tssvd_profile_read(int kind, double* total_ms, int64_t* launches) {
  if (kind < 0 || kind >= TSSVD_PROF_KINDS || !total_ms || !launches) return TSSVD_E_INVALID_ARG;
  return prof_read(kind, total_ms, launches) == hipSuccess ? TSSVD_OK : TSSVD_E_HIP;
}

}  // extern "C"
