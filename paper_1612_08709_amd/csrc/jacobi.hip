// Small dense SVD on one workgroup (gfx950): one-sided Jacobi (Hestenes) in float64.
//
// Algorithm 1 step 4 / Algorithm 2 step 7 / Algorithm 6 step 2 need the SVD of a small
// n x n factor (n <= 100).  One-sided Jacobi orthogonalizes the columns of M by plane
// rotations applied on the right, accumulating them in V:  M J1 J2 ... = U Sigma,
// V = J1 J2 ...; at convergence sigma_j = ||M e_j||, u_j = M e_j / sigma_j.  It attains
// the accuracy of a backward-stable SVD and needs only column dot products, which map
// onto 16-lane DPP reductions.
//
// Layout: M and V column-major in the 160 KB local data share (n*n doubles each).
// 16-lane groups (64 of them for n > 64, 32 for n <= 64); per round of the round-robin
// ("circle") ordering the <= 50 disjoint column pairs go to distinct groups, and a barrier
// separates rounds.
// A sweep is the n'-1 rounds (n' = n rounded up to even) that visit every pair once.
// A pair is rotated when |m_p^T m_q| > tol sqrt(|m_p|^2 |m_q|^2), tol = sqrt(n) * eps;
// iteration stops after the first sweep without rotations or at max_sweeps.
#include <float.h>

#include "common.h"
#include "internal.h"

namespace tsv {

// The three 16-lane sums of a pair (|x|^2, |y|^2, x.y) level by level, so the three DPP
// chains interleave.  Each stage adds the partner lane's value as sum16 does (same operands,
// same order, bitwise the same sums); the DPP moves take no old value (bound_ctrl, every
// source lane exists), which saves a register clear per move.
template <int CTRL>
__device__ __forceinline__ double dpp_mv(double x) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(x), CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(x), CTRL, 0xF, 0xF, true);
  return __hiloint2double(hi, lo);
}
template <int CTRL>
__device__ __forceinline__ void stage3(double& a, double& b, double& c) {
  const double pa = dpp_mv<CTRL>(a), pb = dpp_mv<CTRL>(b), pc = dpp_mv<CTRL>(c);
  a += pa;
  b += pb;
  c += pc;
}
__device__ __forceinline__ void sum16x3(double& a, double& b, double& c) {
  stage3<0xB1>(a, b, c);   // quad_perm [1,0,3,2]
  stage3<0x4E>(a, b, c);   // quad_perm [2,3,0,1]
  stage3<0x141>(a, b, c);  // row_half_mirror
  stage3<0x140>(a, b, c);  // row_mirror
}

// NT threads = NT / 16 lane groups, at least one per column pair of a round (n <= 2 NT / 16):
// 1024 for n <= 128, 512 for n <= 64, where each round's barrier then spans 8 waves, not 16.
// NPL = ceil(n / 16) entries of a column per lane: only the last of them can fall past row
// n - 1, so every other load and store is unconditional, and a lane whose last entry lies
// past the end reads row n - 1 in its place, uses zero for it and stores nothing there.
template <int NT, int NPL>
__global__ __launch_bounds__(NT) void k_jacobi(
    const double* __restrict__ M0, int ldm, int n, int transpose, double wp, int max_sweeps,
    int sign_fix, double* __restrict__ Uo, double* __restrict__ So, double* __restrict__ Vo,
    tssvd_info* __restrict__ info, const int* __restrict__ gate,
    const double* __restrict__ dsrc, int ldd) {
  if (gate && *gate == 0) return;
  extern __shared__ double smem[];
  double* M = smem;          // column c at M + c*n
  double* V = smem + n * n;  // column c at V + c*n
  __shared__ int s_rot;
  __shared__ int s_rank;
  __shared__ double s_sig[TSSVD_N_MAX];
  __shared__ int s_pos[TSSVD_N_MAX];
  __shared__ double s_sgn[TSSVD_N_MAX];
  const int tid = threadIdx.x;
  const int lane16 = tid & 15, grp = tid >> 4;

  // load (M column c, row i) = M0[i][c], or M0[c][i] for the transposed input
  for (int idx = tid; idx < n * n; idx += NT) {
    const int c = idx / n, i = idx - c * n;
    M[idx] = transpose ? M0[c * ldm + i] : M0[i * ldm + c];
    V[idx] = (c == i) ? 1.0 : 0.0;
  }
  if (tid == 0) s_rank = n;
  __syncthreads();
  // discard rule: drop row j when |D_jj| < wp |D_00|, D = dsrc (the triangular factor
  // whose diagonal decides) or M itself
  if (wp > 0.0) {
    const double thr = wp * fabs(dsrc ? dsrc[0] : M[0]);
    if (tid < n) {
      const int j = tid;
      const double djj = dsrc ? dsrc[j * ldd + j] : M[j * n + j];
      if (fabs(djj) < thr) {
        // row j of the factor: a row of M, or a column of M when M is the transpose
        if (transpose)
          for (int i = 0; i < n; ++i) M[j * n + i] = 0.0;
        else
          for (int c = 0; c < n; ++c) M[c * n + j] = 0.0;
        atomicSub(&s_rank, 1);
      }
    }
    __syncthreads();
  }

  const double tol = sqrt((double)n) * DBL_EPSILON;
  const double tol2 = tol * tol;
  const int np = (n + 1) & ~1;  // players in the circle method
  int sweep = 0;
  bool converged = (n < 2);
  while (!converged && sweep < max_sweeps) {
    if (tid == 0) s_rot = 0;
    __syncthreads();
    for (int t = 0; t < np - 1; ++t) {
      if (grp < np / 2) {
        int p, q;
        if (grp == 0) {
          p = t;
          q = np - 1;
        } else {
          // (t + grp) mod (np - 1) and (t - grp) mod (np - 1): both sums lie within one
          // period of the range (0 <= t < np - 1, 0 < grp < np / 2), so a conditional
          // subtraction or addition replaces the integer divisions
          p = t + grp;
          if (p >= np - 1) p -= np - 1;
          q = t - grp;
          if (q < 0) q += np - 1;
        }
        if (p > q) { const int tmp = p; p = q; q = tmp; }
        if (q < n) {
          double* mp = M + p * n;
          double* mq = M + q * n;
          double* vp = V + p * n;
          double* vq = V + q * n;
          const int il = lane16 + 16 * (NPL - 1);
          const bool lv = il < n;  // the last entry is a row of the matrix
          const int ilc = lv ? il : n - 1;
          // the pair's entries of M stay in registers from the dot products to the rotation
          double xr[NPL], yr[NPL], vxr[NPL], vyr[NPL];
#pragma unroll
          for (int k = 0; k < NPL; ++k) {
            const int i = (k == NPL - 1) ? ilc : lane16 + 16 * k;
            xr[k] = mp[i];
            yr[k] = mq[i];
          }
          if (!lv) {
            xr[NPL - 1] = 0.0;
            yr[NPL - 1] = 0.0;
          }
          double al = 0.0, be = 0.0, ga = 0.0;
#pragma unroll
          for (int k = 0; k < NPL; ++k) {
            al = fma(xr[k], xr[k], al);
            be = fma(yr[k], yr[k], be);
            ga = fma(xr[k], yr[k], ga);
          }
          sum16x3(al, be, ga);
          // rotate when |ga| > tol sqrt(al be), tested on squares (no square roots).
          // tan(theta) = 2 ga sign(d) / (|d| + sqrt(d^2 + 4 ga^2)), d = be - al: the smaller
          // root of t^2 + 2 zeta t - 1 = 0 with zeta = d / (2 ga), one division.
          if (ga != 0.0 && ga * ga > tol2 * al * be) {
            // V is read only for a pair that rotates (in the last sweeps most pairs do not,
            // and the rounds are bound by the local data share's traffic), in flight while
            // the rotation is computed
#pragma unroll
            for (int k = 0; k < NPL; ++k) {
              const int i = (k == NPL - 1) ? ilc : lane16 + 16 * k;
              vxr[k] = vp[i];
              vyr[k] = vq[i];
            }
            asm volatile("" ::: "memory");
            const double d = be - al;
            const double g2 = 2.0 * ga;
            const double tt = (d >= 0.0 ? g2 : -g2) / (fabs(d) + sqrt(fma(d, d, g2 * g2)));
            const double c = rsqrt(fma(tt, tt, 1.0));
            const double s = c * tt;
#pragma unroll
            for (int k = 0; k < NPL; ++k) {
              const int i = lane16 + 16 * k;
              if (k < NPL - 1 || lv) {
                mp[i] = fma(c, xr[k], -s * yr[k]);
                mq[i] = fma(s, xr[k], c * yr[k]);
                vp[i] = fma(c, vxr[k], -s * vyr[k]);
                vq[i] = fma(s, vxr[k], c * vyr[k]);
              }
            }
            if (lane16 == 0) s_rot = 1;
          }
        }
      }
      __syncthreads();

    }
    ++sweep;
    converged = (s_rot == 0);
    __syncthreads();
  }

  // singular values = column norms; sign of each pair from w^T v_j, v_j the right singular
  // vector of the factor: column j of V, or of M (normalized) when M is the transpose
  const double* sref = transpose ? M : V;
  for (int c = grp; c < n; c += NT / 16) {
    double s2 = 0.0, sw = 0.0;
    for (int i = lane16; i < n; i += 16) {
      s2 = fma(M[c * n + i], M[c * n + i], s2);
      sw = fma(sign_ref(i), sref[c * n + i], sw);
    }
    s2 = sum16(s2);
    sw = sum16(sw);
    if (lane16 == 0) {
      s_sig[c] = sqrt(s2);
      s_sgn[c] = (sign_fix && sw < 0.0) ? -1.0 : 1.0;
    }
  }
  __syncthreads();
  // descending order; ties keep the original column order
  if (tid < n) {
    const double sj = s_sig[tid];
    int pos = 0;
    for (int i = 0; i < n; ++i) {
      const double si = s_sig[i];
      pos += (si > sj) || (si == sj && i < tid);
    }
    s_pos[tid] = pos;
  }
  __syncthreads();
  const int rank = s_rank;
  for (int idx = tid; idx < n * n; idx += NT) {
    const int c = idx / n, i = idx - c * n;
    const int pos = s_pos[c];
    const double sg = s_sig[c];
    const bool keep = pos < rank && sg > 0.0;
    const double f = s_sgn[c];
    Uo[i * n + pos] = keep ? f * M[idx] / sg : 0.0;
    Vo[i * n + pos] = (pos < rank) ? f * V[idx] : 0.0;
  }
  if (tid < n) So[s_pos[tid]] = (s_pos[tid] < rank) ? s_sig[tid] : 0.0;
  if (tid == 0 && info) {
    int st = converged ? 0 : NUM_NO_CONVERGENCE;
    for (int i = 0; i < n; ++i)
      if (!isfinite(s_sig[i])) st |= NUM_NONFINITE;
    atomicOr(&info->numstat, st);
    info->rank = rank;
    info->sweeps = sweep;
  }
}

template <int NT, int NPL>
hipError_t launch_jacobi(size_t lds, const double* M, int ldm, int n, int transpose, double wp,
                         int max_sweeps, int sign_fix, double* Uo, double* So, double* Vo,
                         tssvd_info* info, hipStream_t s, const int* gate, const double* dsrc,
                         int ldd) {
  static bool attr_set = false;
  if (!attr_set) {
    const int mx = (int)(2 * TSSVD_N_MAX * TSSVD_N_MAX * sizeof(double));
    const hipError_t e = hipFuncSetAttribute((const void*)k_jacobi<NT, NPL>,
                                             hipFuncAttributeMaxDynamicSharedMemorySize, mx);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  hipLaunchKernelGGL((k_jacobi<NT, NPL>), dim3(1), dim3(NT), lds, s, M, ldm, n, transpose, wp,
                     max_sweeps, sign_fix, Uo, So, Vo, info, gate, dsrc, ldd);
  return hipGetLastError();
}

hipError_t jacobi_svd(const double* M, int ldm, int n, int transpose, double wp,
                      int max_sweeps, int sign_fix, double* Uo, double* So, double* Vo,
                      tssvd_info* info, hipStream_t s, const int* gate,
                      const double* dsrc, int ldd) {
  const size_t lds = (size_t)2 * n * n * sizeof(double);
#define TSV_JAC(NT, NPL)                                                                    \
  return launch_jacobi<NT, NPL>(lds, M, ldm, n, transpose, wp, max_sweeps, sign_fix, Uo, So, \
                                Vo, info, s, gate, dsrc, ldd)
  switch ((n + 15) / 16) {
    case 0:
    case 1: TSV_JAC(512, 1);
    case 2: TSV_JAC(512, 2);
    case 3: TSV_JAC(512, 3);
    case 4: TSV_JAC(512, 4);
    case 5: TSV_JAC(1024, 5);
    case 6: TSV_JAC(1024, 6);
    case 7: TSV_JAC(1024, 7);
    default: return hipErrorInvalidValue;
  }
#undef TSV_JAC
}

}  // namespace tsv
