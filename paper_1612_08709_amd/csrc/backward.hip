// Kernels of the reverse pass of the randomized SVD (vector-Jacobian product with the
// sketch held fixed).  The orchestration lives in api.hip; the mathematics:
//
//   SVD layer (B = Ub Sigma W^T, B^T = W Sigma Ub^T tall):  with F_ij = 1/(s_j^2 - s_i^2),
//     C   = (F o (W^T Wbar - Wbar^T W)) Sigma + diag(Sbar) + Sigma (F o (Ub^T Ubbar - Ubbar^T Ub))
//     Bbar^T = W (C - (W^T Wbar) Sigma^-1) Ub^T + Wbar Sigma^-1 Ub^T
//   QR layer (Y = Q R, R not used downstream):
//     Ybar = [Qbar - Q copyltu(Qbar^T Q)] R^-T,   copyltu(M) = tril(M) + tril(M, -1)^T
//   products:  Y = A X  ->  Abar += Ybar X^T,  Xbar = A^T Ybar
//              Z = A^T Q ->  Abar += Q Zbar^T,  Qbar = A Zbar
// Small l x l matrices (l <= 100) are handled by one-thread-per-entry kernels; the tall
// m x l updates by row kernels; the final Abar = L R^T (m x K x n) by a float64 MFMA kernel.
#include "common.h"
#include "internal.h"

namespace tsv {

typedef double f64x4 __attribute__((ext_vector_type(4)));

// A1 = Ub^T [G1, 0]   (l x l; G1 is l x k with stride k)
__global__ void k_bw_a1(const double* __restrict__ Ub, const double* __restrict__ G1, int l,
                        int k, double* __restrict__ A1) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= l * l) return;
  const int i = idx / l, j = idx - i * l;
  double s = 0.0;
  if (j < k)
    for (int t = 0; t < l; ++t) s = fma(Ub[t * l + i], G1[t * k + j], s);
  A1[idx] = s;
}

// KB = C - G2p Sigma^-1 with C as in the header; G2p = [G2, 0] (l x l), Sbar may be NULL.
__global__ void k_bw_core(const double* __restrict__ A1, const double* __restrict__ G2,
                          const double* __restrict__ sig, const double* __restrict__ Sbar, int l,
                          int k, double* __restrict__ KB) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= l * l) return;
  const int i = idx / l, j = idx - i * l;
  const double si = sig[i], sj = sig[j];
  const double g2ij = (j < k) ? G2[i * k + j] : 0.0;
  const double g2ji = (i < k) ? G2[j * k + i] : 0.0;
  double c = 0.0;
  // Pairs with both indices past k multiply zero cotangents (G1 and G2 vanish there), and
  // the trailing sketch values may repeat (exact zeros when rank(A) < l), so 1/(sj^2 - si^2)
  // is not formed for them.
  if (i != j && (i < k || j < k)) {
    const double f = 1.0 / ((sj - si) * (sj + si));
    c = f * (g2ij - g2ji) * sj + si * f * (A1[i * l + j] - A1[j * l + i]);
  } else if (i < k && Sbar) {
    c = Sbar[i];
  }
  if (j < k) c -= g2ij / sj;
  KB[idx] = c;
}

// Kw = KB Ub^T (l x l);  Kv = Sigma_k^-1 Ub_k^T (k x l);  UbkT = Ub_k^T (k x l)
__global__ void k_bw_kw(const double* __restrict__ KB, const double* __restrict__ Ub,
                        const double* __restrict__ sig, int l, int k, double* __restrict__ Kw,
                        double* __restrict__ Kv, double* __restrict__ UbkT) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < l * l) {
    const int i = idx / l, c = idx - i * l;
    double s = 0.0;
    for (int j = 0; j < l; ++j) s = fma(KB[i * l + j], Ub[c * l + j], s);
    Kw[idx] = s;
  }
  if (idx < k * l) {
    const int i = idx / l, c = idx - i * l;
    UbkT[idx] = Ub[c * l + i];
    Kv[idx] = Ub[c * l + i] / sig[i];
  }
}

// QR-layer coefficients: from M = Xbar^T Q (l x l) and R (upper, stride l):
//   K1 = R^-T,  K2 = -copyltu(M) R^-T   so that  Ybar = Xbar K1 + Q K2.
// Rinv (upper) is formed column by column by back substitution (one thread per column).
__global__ void k_bw_rinv(const double* __restrict__ R, int l, double* __restrict__ Rinv) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= l) return;
  for (int i = l - 1; i >= 0; --i) {
    double s = (i == c) ? 1.0 : 0.0;
    if (i <= c) {
      for (int t = i + 1; t <= c; ++t) s -= R[i * l + t] * Rinv[t * l + c];
      s /= R[i * l + i];
    } else {
      s = 0.0;
    }
    Rinv[i * l + c] = s;
  }
}

__global__ void k_bw_qrcoef(const double* __restrict__ M, const double* __restrict__ Rinv, int l,
                            double* __restrict__ K1, double* __restrict__ K2) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= l * l) return;
  const int i = idx / l, j = idx - i * l;
  K1[idx] = Rinv[j * l + i];  // (R^-1)^T
  double s = 0.0;
  for (int t = 0; t < l; ++t) {
    // copyltu(M)[i][t] = M[i][t] for t <= i, M[t][i] for t > i
    const double cm = (t <= i) ? M[i * l + t] : M[t * l + i];
    s = fma(cm, Rinv[j * l + t], s);  // (R^-T)[t][j] = Rinv[j][t]
  }
  K2[idx] = -s;
}

// out[r][c] = sum_t X1[r][t] K1[t][c] (+ sum_t X2[r][t] K2[t][c]) (+ out[r][c] if accum),
// r < rows, c < kout; X1 rows x k1 (stride ld1), X2 rows x k2 (stride ld2), K's dense.
__global__ void k_rmul(const double* __restrict__ X1, int64_t ld1, int k1,
                       const double* __restrict__ K1, const double* __restrict__ X2, int64_t ld2,
                       int k2, const double* __restrict__ K2, int64_t rows, int kout,
                       double* __restrict__ out, int64_t ldo, int accum) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= rows * kout) return;
  const int64_t r = idx / kout;
  const int c = (int)(idx - r * kout);
  double s = accum ? out[r * ldo + c] : 0.0;
  const double* x1 = X1 + r * ld1;
  for (int t = 0; t < k1; ++t) s = fma(x1[t], K1[t * kout + c], s);
  if (X2) {
    const double* x2 = X2 + r * ld2;
    for (int t = 0; t < k2; ++t) s = fma(x2[t], K2[t * kout + c], s);
  }
  out[r * ldo + c] = s;
}

__global__ void k_zero(double* __restrict__ p, int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = 0.0;
}

// C (m x n, A's dtype, stride ldc) = L (m x K, stride ldl) R^T (R: n x K, stride ldr), float64
// MFMA.  Wave = 32 rows x 64 columns; workgroup = 2 x 2 waves.  Both operands are contiguous
// along K, so lane (i, g) reads L[row i][k0+4g .. k0+4g+3] and R[col i][k0+4g ..] and uses
// element s in MFMA s (k-slot g <-> k0 + 4g + s).
// VEC (rows of L and R start on 16 bytes, K a multiple of 4): the main loop loads without a
// branch (rows past m and columns past n read the last valid one; those results are not
// stored) and alternates two register sets, so one step's loads are in flight during the
// other step's MFMAs; a last step of fewer than 16 (K % 16 = 4, 8 or 12) is done once with
// a lane condition.
template <typename TC, bool VEC>
__global__ __launch_bounds__(256) void k_gemm_nt(const double* __restrict__ L, int64_t ldl,
                                                 const double* __restrict__ R, int64_t ldr,
                                                 int64_t m, int64_t n, int K,
                                                 TC* __restrict__ C, int64_t ldc) {
  constexpr int TM = 2, TN = 4;
  // tile L = (row block, column block), column block fastest; workgroup IDs are dealt to
  // the 8 XCDs round-robin, so XCD x takes the contiguous tiles x*per ... and the column
  // blocks of one row block share that XCD's L2 copy of their rows of L
  const int64_t gx = (n + 127) / 128, total = gx * ((m + 63) / 64);
  const int64_t per = (total + 7) / 8;
  const int64_t tile = (int64_t)(blockIdx.x & 7) * per + (blockIdx.x >> 3);
  if (tile >= total) return;
  const int64_t rowblk = tile / gx, colblk = tile - rowblk * gx;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, g = lane >> 4;
  const int64_t rb = rowblk * 64 + (wave & 1) * 32;
  const int64_t cb = colblk * 128 + (wave >> 1) * 64;
  f64x4 acc[TM][TN];
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b) acc[a][b] = f64x4{0.0, 0.0, 0.0, 0.0};
  if constexpr (VEC) {
    const double* lp[TM];
    const double* rp[TN];
#pragma unroll
    for (int a = 0; a < TM; ++a) {
      const int64_t row = rb + 16 * a + li;
      lp[a] = L + (row < m ? row : m - 1) * ldl + 4 * g;
    }
#pragma unroll
    for (int b = 0; b < TN; ++b) {
      const int64_t col = cb + 16 * b + li;
      rp[b] = R + (col < n ? col : n - 1) * ldr + 4 * g;
    }
    auto ld = [&](int k0, Quad<double> (&x)[TM], Quad<double> (&y)[TN]) {
#pragma unroll
      for (int a = 0; a < TM; ++a) x[a].load(lp[a] + k0);
#pragma unroll
      for (int b = 0; b < TN; ++b) y[b].load(rp[b] + k0);
    };
    auto mm = [&](Quad<double> (&x)[TM], Quad<double> (&y)[TN]) {
#pragma unroll
      for (int a = 0; a < TM; ++a) x[a].pin();
#pragma unroll
      for (int b = 0; b < TN; ++b) y[b].pin();
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int a = 0; a < TM; ++a)
#pragma unroll
          for (int b = 0; b < TN; ++b)
            acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(x[a][s], y[b][s], acc[a][b], 0, 0, 0);
    };
    const int nfull = K >> 4;
    Quad<double> x0[TM], y0[TN], x1[TM], y1[TN];
    // the partial last step first (straight-line code before the loop keeps the
    // accumulators in place), with zeros in the lanes past K
    if (16 * nfull < K) {
#pragma unroll
      for (int a = 0; a < TM; ++a) x0[a].zero();
#pragma unroll
      for (int b = 0; b < TN; ++b) y0[b].zero();
      if (16 * nfull + 4 * g < K) ld(16 * nfull, x0, y0);
      mm(x0, y0);
    }
    int st = 0;
    if (nfull & 1) {
      ld(0, x0, y0);
      mm(x0, y0);
      st = 1;
    }
    if (st < nfull) {  // an even number of steps remains
      ld(16 * st, x0, y0);
      for (; st < nfull; st += 2) {
        // the empty asm statements keep each step's loads ahead of the other step's MFMAs
        ld(16 * (st + 1), x1, y1);
        asm volatile("" ::: "memory");
        mm(x0, y0);
        ld(16 * (st + 2 < nfull ? st + 2 : st + 1), x0, y0);  // the last one is not used
        asm volatile("" ::: "memory");
        mm(x1, y1);
      }
    }
  } else {
    for (int k0 = 0; k0 < K; k0 += 16) {
      double x[TM][4], y[TN][4];
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int kk = k0 + 4 * g + s;
#pragma unroll
        for (int a = 0; a < TM; ++a) {
          const int64_t row = rb + 16 * a + li;
          x[a][s] = (kk < K && row < m) ? L[row * ldl + kk] : 0.0;
        }
#pragma unroll
        for (int b = 0; b < TN; ++b) {
          const int64_t col = cb + 16 * b + li;
          y[b][s] = (kk < K && col < n) ? R[col * ldr + kk] : 0.0;
        }
      }
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int a = 0; a < TM; ++a)
#pragma unroll
          for (int b = 0; b < TN; ++b)
            acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(x[a][s], y[b][s], acc[a][b], 0, 0, 0);
    }
  }
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b) {
      const int64_t col = cb + 16 * b + li;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = rb + 16 * a + 4 * r + g;
        if (row < m && col < n) C[row * ldc + col] = (TC)acc[a][b][r];
      }
    }
}

// ---------------------------------------------------------------- launchers
static inline unsigned blocks(int64_t count) { return (unsigned)((count + 255) / 256); }

hipError_t bw_svd_core(const double* Ub, const double* sig, const double* G1, const double* G2,
                       const double* Sbar, int l, int k, double* A1, double* KB, double* Kw,
                       double* Kv, double* UbkT, hipStream_t s) {
  hipLaunchKernelGGL(k_bw_a1, dim3(blocks(l * l)), dim3(256), 0, s, Ub, G1, l, k, A1);
  hipLaunchKernelGGL(k_bw_core, dim3(blocks(l * l)), dim3(256), 0, s, A1, G2, sig, Sbar, l, k, KB);
  hipLaunchKernelGGL(k_bw_kw, dim3(blocks(l * l)), dim3(256), 0, s, KB, Ub, sig, l, k, Kw, Kv,
                     UbkT);
  return hipGetLastError();
}


hipError_t bw_rinv(const double* R, int l, double* Rinv, hipStream_t s) {
  hipLaunchKernelGGL(k_bw_rinv, dim3(1), dim3(128), 0, s, R, l, Rinv);
  return hipGetLastError();
}

hipError_t bw_qr_coef_rinv(const double* M, const double* Rinv, int l, double* K1, double* K2,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_bw_qrcoef, dim3(blocks(l * l)), dim3(256), 0, s, M, Rinv, l, K1, K2);
  return hipGetLastError();
}

hipError_t rmul(const double* X1, int64_t ld1, int k1, const double* K1, const double* X2,
                int64_t ld2, int k2, const double* K2, int64_t rows, int kout, double* out,
                int64_t ldo, bool accum, hipStream_t s) {
  // two passes of the matrix-core product Y (+)= X K when the strides fit its int arguments
  // (l <= 112 columns), else the plain kernel
  if (kout <= 112 && ldo <= INT32_MAX) {
    hipError_t e = gemm_ax_f64_acc(X1, ld1, rows, k1, K1, kout, kout, out, (int)ldo, accum, s);
    if (e != hipSuccess || !X2 || k2 <= 0) return e;
    return gemm_ax_f64_acc(X2, ld2, rows, k2, K2, kout, kout, out, (int)ldo, true, s);
  }
  hipLaunchKernelGGL(k_rmul, dim3(blocks(rows * kout)), dim3(256), 0, s, X1, ld1, k1, K1, X2,
                     ld2, k2, K2, rows, kout, out, ldo, accum ? 1 : 0);
  return hipGetLastError();
}

hipError_t zero_fill(double* p, int64_t count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero, dim3(blocks(count)), dim3(256), 0, s, p, count);
  return hipGetLastError();
}

hipError_t gemm_nt(const double* L, int64_t ldl, const double* R, int64_t ldr, int64_t m,
                   int64_t n, int K, void* C, int c_dtype, int64_t ldc, hipStream_t s) {
  const int64_t total = ((n + 127) / 128) * ((m + 63) / 64);
  dim3 grid((unsigned)(8 * ((total + 7) / 8)));
  const bool vec = (reinterpret_cast<uintptr_t>(L) & 15) == 0 &&
                   (reinterpret_cast<uintptr_t>(R) & 15) == 0 && ldl % 2 == 0 && ldr % 2 == 0 &&
                   K % 4 == 0;
  if (c_dtype == TSSVD_F64) {
    if (vec)
      hipLaunchKernelGGL((k_gemm_nt<double, true>), grid, dim3(256), 0, s, L, ldl, R, ldr, m, n,
                         K, (double*)C, ldc);
    else
      hipLaunchKernelGGL((k_gemm_nt<double, false>), grid, dim3(256), 0, s, L, ldl, R, ldr, m, n,
                         K, (double*)C, ldc);
  } else {
    if (vec)
      hipLaunchKernelGGL((k_gemm_nt<float, true>), grid, dim3(256), 0, s, L, ldl, R, ldr, m, n,
                         K, (float*)C, ldc);
    else
      hipLaunchKernelGGL((k_gemm_nt<float, false>), grid, dim3(256), 0, s, L, ldl, R, ldr, m, n,
                         K, (float*)C, ldc);
  }
  return hipGetLastError();
}

}  // namespace tsv
