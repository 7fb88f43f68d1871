// Triangular solves, Gram matrices and row-local products on gfx950 float64 matrix cores,
// for the mixed-precision tall-skinny SVD: the float32 Householder TSQR supplies R1, then
//   Q1 = A R1^-1     (blocked triangular solve in float64, A read as stored),
//   G  = Q1^T Q1     (fused into the same pass),
// and, after the Cholesky factor R2 of G, U = Q1 (R2^-1 P) by a row-local product.
// A = Q1 R1 is then the first factorization of Algorithm 2 with a Q1 that is only nearly
// orthonormal (R1 comes from a lower-precision factorization), and the algorithm's second
// factorization Q1 = Q R2 is a Cholesky QR of Q1 in float64.
//
// Matrix-core layout (v_mfma_f64_16x16x4_f64): lane (i = lane % 16, g = lane / 16) supplies
// a[i][k] and b[k][i] for k = g in each 4-deep instruction; the result register r holds
// D[4r + g][i].
//
// Triangular solve.  Row form: Q_J R_JJ = A_J - sum_{K<J} Q_K R_KJ (16-column tiles J).  It
// runs transposed, R_JJ^T Q_J^T = A_J^T - sum_K R_KJ^T Q_K^T, with the 16 rows of a wave on
// the lane index i: a Q_K^T tile in result layout is then the B operand of the next tiles
// as it stands (register s of lane group g is row 4s + g of Q_K^T).  Result row 4r + g of a
// tile stands for column sig(4r + g) = 4g + r of the tile, so a lane's four registers are
// four adjacent columns of one row of A and of Q.  The diagonal blocks are applied through
// their explicit inverses (a residual of order eps kappa(R_JJ) ||A||, not eps ||A||).
// The constant operands (-R_KJ^T and R_JJ^-T entries in that order) are packed once by
// k_pc_prep and staged in the local data share.
#include "common.h"
#include "internal.h"

namespace tsv {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ d4 mma(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Four adjacent elements of a row (a lane's share of a tile): one vector access when the
// caller has checked 16-byte alignment of the rows (VEC), else element by element.
template <bool VEC>
__device__ __forceinline__ void ld4(const float* p, bool ok, d4& v) {
  if (VEC) {
    const float4 x = ok ? *reinterpret_cast<const float4*>(p) : float4{0.f, 0.f, 0.f, 0.f};
    v[0] = x.x; v[1] = x.y; v[2] = x.z; v[3] = x.w;
  } else {
#pragma unroll
    for (int r = 0; r < 4; ++r) v[r] = ok ? (double)p[r] : 0.0;
  }
}
template <bool VEC>
__device__ __forceinline__ void ld4(const double* p, bool ok, d4& v) {
  if (VEC) {
    const double2 x0 = ok ? *reinterpret_cast<const double2*>(p) : double2{0.0, 0.0};
    const double2 x1 = ok ? *reinterpret_cast<const double2*>(p + 2) : double2{0.0, 0.0};
    v[0] = x0.x; v[1] = x0.y; v[2] = x1.x; v[3] = x1.y;
  } else {
#pragma unroll
    for (int r = 0; r < 4; ++r) v[r] = ok ? p[r] : 0.0;
  }
}
template <bool VEC>
__device__ __forceinline__ void st4(double* p, const d4& v) {
  if (VEC) {
    *reinterpret_cast<double2*>(p) = double2{v[0], v[1]};
    *reinterpret_cast<double2*>(p + 2) = double2{v[2], v[3]};
  } else {
#pragma unroll
    for (int r = 0; r < 4; ++r) p[r] = v[r];
  }
}

// column of a 16-column tile that result row x (= 4r + g) stands for
__host__ __device__ constexpr int sig(int x) { return 4 * (x & 3) + (x >> 2); }

// packed index of the tile pair (p, c), p <= c, of an nt x nt upper tile grid, and back
__host__ __device__ constexpr int upk(int p, int c, int nt) {
  return p * nt - p * (p - 1) / 2 + (c - p);
}
__device__ __forceinline__ void unpk(int t, int nt, int& p, int& c) {
  p = 0;
  while (t >= nt - p) {
    t -= nt - p;
    ++p;
  }
  c = p + t;
}

constexpr int PC_THREADS = 256;  // 4 waves, 16 rows each: 64-row chunks
constexpr int PC_CHUNK = 64;
constexpr int PC_GRID_MAX = 256;  // one workgroup per compute unit (local data share bound)

template <int NT>
constexpr int pc_pairs() { return NT * (NT + 1) / 2; }
template <int NT>
constexpr int stage_ld() { return 16 * NT + 2; }  // staging row stride (doubles)

// ---------------------------------------------------------------- operand preparation
// From R (n x n upper triangular, row-major, stride ldr; the entries below the diagonal are
// not read) to
//   Rp  = R with each diagonal entry d, |d| < tol max_i |R_ii|, replaced by
//         sign(d) tol max_i |R_ii| (by 1 when R is zero) (n x n row-major): a column that R
//         marks as (nearly) dependent then gives a bounded column of Q instead of an
//         overflow; any nonsingular Rp serves, since Q is defined as X Rp^-1,
//   Rop = the operand tiles of the triangular solve, tile pair t = upk(K, J) (K <= J), four
//         instructions s, 64 lanes: -Rp[16K + 4g + s][16J + sig(i)] for K < J and
//         Rp_JJ^-1[4g + s][sig(i)] for K = J.  Padding past n is the identity.
// One workgroup of 256 threads; dynamic shared memory: 16NT x (16NT + 1) doubles.
template <int NT>
__global__ __launch_bounds__(256) void k_pc_prep(const double* __restrict__ R, int ldr, int n,
                                                 double tol, double* __restrict__ Rp,
                                                 double* __restrict__ Rop,
                                                 const int* __restrict__ gate) {
  constexpr int NP = 16 * NT, LD = NP + 1;
  extern __shared__ double Rl[];  // NP x LD: the padded factor, then the block inverses
  __shared__ double s_thr;
  if (gate && *gate == 0) return;  // uniform over the workgroup
  const int tid = threadIdx.x;
  for (int idx = tid; idx < NP * NP; idx += 256) {
    const int i = idx / NP, j = idx - i * NP;
    double v;
    if (i < n && j < n)
      v = (j >= i) ? R[(int64_t)i * ldr + j] : 0.0;
    else
      v = (i == j) ? 1.0 : 0.0;
    Rl[i * LD + j] = v;
  }
  __syncthreads();
  if (tid == 0) {
    double mx = 0.0;
    for (int i = 0; i < n; ++i) mx = fmax(mx, fabs(Rl[i * LD + i]));
    s_thr = (mx > 0.0) ? tol * mx : 1.0;
  }
  __syncthreads();
  const double thr = s_thr;
  if (tid < n) {
    const double d = Rl[tid * LD + tid];
    if (fabs(d) < thr) Rl[tid * LD + tid] = (d < 0.0) ? -thr : thr;  // NaN stays NaN
  }
  __syncthreads();
  for (int idx = tid; idx < n * n; idx += 256) {
    const int i = idx / n, j = idx - i * n;
    Rp[idx] = Rl[i * LD + j];
  }
  // inverses of the diagonal blocks: column c of block J per thread, kept in registers
  // until every thread has read the blocks, then written over them
  double x[16];
  const int J = tid >> 4, c = tid & 15;
  if (J < NT) {
    const int o = 16 * J;
#pragma unroll
    for (int i = 0; i < 16; ++i) x[i] = 0.0;
    // back substitution R_JJ x = e_c (rows c .. 0)
    for (int i = c; i >= 0; --i) {
      double t = (i == c) ? 1.0 : 0.0;
      for (int k = i + 1; k <= c; ++k) t = fma(-Rl[(o + i) * LD + o + k], x[k], t);
      x[i] = t / Rl[(o + i) * LD + o + i];
    }
  }
  __syncthreads();  // every thread has read the diagonal blocks
  if (J < NT) {
    const int o = 16 * J;
#pragma unroll
    for (int i = 0; i < 16; ++i) Rl[(o + i) * LD + o + c] = x[i];  // block J now holds its inverse
  }
  __syncthreads();
  constexpr int NTT = pc_pairs<NT>();
  for (int idx = tid; idx < NTT * 256; idx += 256) {
    const int t = idx >> 8, s = (idx >> 6) & 3, lane = idx & 63;
    const int li = lane & 15, g = lane >> 4;
    int K, Jt;
    unpk(t, NT, K, Jt);
    const int row = 16 * K + 4 * g + s, col = 16 * Jt + sig(li);
    const double v = Rl[row * LD + col];
    Rop[idx] = (K < Jt) ? -v : v;
  }
}

// ---------------------------------------------------------------- solve + Gram
// Q = X Rp^-1 (X: m x n, float32 or float64, stride ldx; Q: float64, stride ldq; Q may be X
// itself when both are float64: every element is read and then written by the same lane) and
// this workgroup's part of Q^T Q (n x n, at part + blockIdx.x n n).  Chunks of 64 rows go to
// the workgroups in turn (chunk c to workgroup c mod gridDim.x), so each partial Gram has a
// fixed summation order.  The chunk's Q rows are staged in the local data share; each wave
// then accumulates its share of the upper tile pairs of the Gram over the 64 rows
// (contraction over rows: operands read straight from the staged rows).
template <int NT, typename TA>
__global__ __launch_bounds__(PC_THREADS, 1) void k_pc_trsm(
    const TA* X, int64_t ldx, int64_t m, int n, const double* __restrict__ Rop, double* Q,
    int64_t ldq, double* __restrict__ part, const int* __restrict__ gate) {
  if (gate && *gate == 0) return;
  constexpr int NTT = pc_pairs<NT>();
  constexpr int NPW = (NTT + 3) / 4;  // Gram tile pairs per wave
  constexpr int SLD = stage_ld<NT>();
  extern __shared__ double smem[];
  double* Rs = smem;               // NTT * 256
  double* Sb = smem + NTT * 256;   // PC_CHUNK x SLD
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, g = lane >> 4;
  for (int i = tid; i < NTT * 256; i += PC_THREADS) Rs[i] = Rop[i];
  __syncthreads();

  d4 gacc[NPW];
#pragma unroll
  for (int p = 0; p < NPW; ++p) gacc[p] = d4{0.0, 0.0, 0.0, 0.0};

  const int64_t nchunk = (m + PC_CHUNK - 1) / PC_CHUNK;
  for (int64_t ch = blockIdx.x; ch < nchunk; ch += gridDim.x) {
    const int64_t row = ch * PC_CHUNK + 16 * wave + li;
    const bool rok = row < m;
    const TA* xr = X + (rok ? row : 0) * ldx;
    d4 q[NT];
#pragma unroll
    for (int J = 0; J < NT; ++J) {
      d4 acc;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int col = 16 * J + 4 * g + r;
        acc[r] = (rok && col < n) ? (double)xr[col] : 0.0;
      }
#pragma unroll
      for (int K = 0; K < J; ++K) {
        const double* op = Rs + upk(K, J, NT) * 256 + lane;
#pragma unroll
        for (int s = 0; s < 4; ++s) acc = mma(op[64 * s], q[K][s], acc);
      }
      const double* od = Rs + upk(J, J, NT) * 256 + lane;
      d4 z = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int s = 0; s < 4; ++s) z = mma(od[64 * s], acc[s], z);
      q[J] = z;
    }
    double* qr = Q + (rok ? row : 0) * ldq;
    double* sr = Sb + (16 * wave + li) * SLD;
#pragma unroll
    for (int J = 0; J < NT; ++J)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int col = 16 * J + 4 * g + r;
        if (rok && col < n) qr[col] = q[J][r];
        sr[col] = q[J][r];
      }
    __syncthreads();
#pragma unroll
    for (int p = 0; p < NPW; ++p) {
      const int t = wave + 4 * p;
      if (t < NTT) {
        int P, C;
        unpk(t, NT, P, C);
#pragma unroll
        for (int rr = 0; rr < PC_CHUNK / 16; ++rr)
#pragma unroll
          for (int s = 0; s < 4; ++s) {
            const double* srow = Sb + (16 * rr + 4 * s + g) * SLD;
            gacc[p] = mma(srow[16 * P + li], srow[16 * C + li], gacc[p]);
          }
      }
    }
    __syncthreads();
  }
  double* pw = part + (int64_t)blockIdx.x * n * n;
#pragma unroll
  for (int p = 0; p < NPW; ++p) {
    const int t = wave + 4 * p;
    if (t < NTT) {
      int P, C;
      unpk(t, NT, P, C);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = 16 * P + 4 * r + g, j = 16 * C + li;
        if (i <= j && j < n) {  // diagonal tiles: the entry i <= j for both places
          pw[(int64_t)i * n + j] = gacc[p][r];
          pw[(int64_t)j * n + i] = gacc[p][r];
        }
      }
    }
  }
}

// The solve alone (no Gram), for callers that form Q^T Q with the staged Gram kernel: only
// the operand tiles live in the local data share, so two workgroups share a CU, and each
// wave solves two 16-row tiles whose dependent chains of matrix-core steps interleave.
// Chunks of 128 rows (4 waves x 32) go to the workgroups in turn.  Same in-place rule as
// k_pc_trsm.  Element-wise accesses (rows not 16-byte aligned or n not a multiple of 4;
// otherwise k_pc_trsm_pipe below).
template <int NT, typename TA>
__global__ __launch_bounds__(PC_THREADS, 2) void k_pc_trsm2(
    const TA* X, int64_t ldx, int64_t m, int n, const double* __restrict__ Rop, double* Q,
    int64_t ldq, const int* __restrict__ gate) {
  if (gate && *gate == 0) return;
  constexpr int NTT = pc_pairs<NT>();
  constexpr int CH = 2 * PC_CHUNK;
  extern __shared__ double smem[];
  double* Rs = smem;  // NTT * 256
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, g = lane >> 4;
  for (int i = tid; i < NTT * 256; i += PC_THREADS) Rs[i] = Rop[i];
  __syncthreads();
  const int64_t nchunk = (m + CH - 1) / CH;
  for (int64_t ch = blockIdx.x; ch < nchunk; ch += gridDim.x) {
    // the operand tiles are read per use: without this compiler barrier all of them would
    // be hoisted out of the loop into registers (and spilled)
    asm volatile("" ::: "memory");
    int64_t row[2];
    bool rok[2];
    const TA* xr[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      row[h] = ch * CH + 32 * wave + 16 * h + li;
      rok[h] = row[h] < m;
      xr[h] = X + (rok[h] ? row[h] : 0) * ldx;
    }
    d4 q[2][NT];
#pragma unroll
    for (int J = 0; J < NT; ++J) {
      d4 acc[2];
      const int c0 = 16 * J + 4 * g;
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          acc[h][r] = (rok[h] && c0 + r < n) ? (double)xr[h][c0 + r] : 0.0;
#pragma unroll
      for (int K = 0; K < J; ++K) {
        const double* op = Rs + upk(K, J, NT) * 256 + lane;
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          const double o = op[64 * s];
#pragma unroll
          for (int h = 0; h < 2; ++h) acc[h] = mma(o, q[h][K][s], acc[h]);
        }
      }
      const double* od = Rs + upk(J, J, NT) * 256 + lane;
#pragma unroll
      for (int h = 0; h < 2; ++h) q[h][J] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const double o = od[64 * s];
#pragma unroll
        for (int h = 0; h < 2; ++h) q[h][J] = mma(o, acc[h][s], q[h][J]);
      }
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      double* qr = Q + (rok[h] ? row[h] : 0) * ldq;
#pragma unroll
      for (int J = 0; J < NT; ++J) {
        const int c0 = 16 * J + 4 * g;
#pragma unroll
        for (int r = 0; r < 4; ++r)
          if (rok[h] && c0 + r < n) qr[c0 + r] = q[h][J][r];
      }
    }
  }
}

// The solve alone for 16-byte aligned rows and n a multiple of 4, pipelined: a wave takes 16
// rows per 64-row chunk (lane i: row i, four adjacent columns per tile, as above) and loads
// the rows of its next chunk, with no branch, while it solves the current one.  Rows past m
// read row m - 1 and columns past n the last four columns (their results are not stored;
// the padding of Rop is the identity).
template <int NT, typename TA>
__global__ __launch_bounds__(PC_THREADS, 2) void k_pc_trsm_pipe(
    const TA* X, int64_t ldx, int64_t m, int n, const double* __restrict__ Rop, double* Q,
    int64_t ldq, const int* __restrict__ gate) {
  if (gate && *gate == 0) return;
  constexpr int NTT = pc_pairs<NT>();
  extern __shared__ double smem[];
  double* Rs = smem;  // NTT * 256
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, g = lane >> 4;
  for (int i = tid; i < NTT * 256; i += PC_THREADS) Rs[i] = Rop[i];
  __syncthreads();
  const int64_t nchunk = (m + PC_CHUNK - 1) / PC_CHUNK;
  int64_t ch = blockIdx.x;
  if (ch >= nchunk) return;
  int cc[NT];
#pragma unroll
  for (int J = 0; J < NT; ++J) cc[J] = (16 * J + 4 * g < n) ? 16 * J + 4 * g : n - 4;
  auto ld = [&](int64_t c, Quad<TA> (&xv)[NT]) {
    const int64_t row = c * PC_CHUNK + 16 * wave + li;
    const TA* xr = X + (row < m ? row : m - 1) * ldx;
#pragma unroll
    for (int J = 0; J < NT; ++J) xv[J].load(xr + cc[J]);
  };
  auto solve = [&](int64_t c, Quad<TA> (&xv)[NT]) {
    // the operand tiles are read per use (the compiler would otherwise hoist them all out
    // of the chunk loop and spill them)
    asm volatile("" ::: "memory");
#pragma unroll
    for (int J = 0; J < NT; ++J) xv[J].pin();
    const int64_t row = c * PC_CHUNK + 16 * wave + li;
    d4 q[NT];
#pragma unroll
    for (int J = 0; J < NT; ++J) {
      d4 acc = {xv[J][0], xv[J][1], xv[J][2], xv[J][3]};
#pragma unroll
      for (int K = 0; K < J; ++K) {
        const double* op = Rs + upk(K, J, NT) * 256 + lane;
#pragma unroll
        for (int s2 = 0; s2 < 4; ++s2) acc = mma(op[64 * s2], q[K][s2], acc);
      }
      const double* od = Rs + upk(J, J, NT) * 256 + lane;
      q[J] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int s2 = 0; s2 < 4; ++s2) q[J] = mma(od[64 * s2], acc[s2], q[J]);
    }
    if (row < m) {
      double* qr = Q + row * ldq;
#pragma unroll
      for (int J = 0; J < NT; ++J)
        if (16 * J + 4 * g < n) st4<true>(qr + 16 * J + 4 * g, q[J]);
    }
  };
  Quad<TA> xa[NT], xb[NT];
  ld(ch, xa);
  for (;;) {
    const int64_t c1 = ch + gridDim.x;
    ld(c1 < nchunk ? c1 : ch, xb);  // past the end: reloaded, not used
    solve(ch, xa);
    if (c1 >= nchunk) break;
    const int64_t c2 = c1 + gridDim.x;
    ld(c2 < nchunk ? c2 : c1, xa);
    solve(c1, xb);
    if (c2 >= nchunk) break;
    ch = c2;
  }
}

// ---------------------------------------------------------------- row-local product
// X <- X N in place (X: m x n float64, stride ldx; N: n x n).  A wave loads its 16 rows (lane
// i: row i, four adjacent columns 4g .. 4g+3 of each tile as the A operand), forms each
// output tile from all of them and stores it in result layout (row 4r + g, column i), so
// every store depends on every load of the wave's rows.  Nop holds N as B operands: tile
// (K, J), instruction s, lane (i, g): N[16K + 4g + s][16J + i].
template <int NT, bool VEC>
__global__ __launch_bounds__(PC_THREADS, 1) void k_rowmul(double* X, int64_t ldx, int64_t m,
                                                          int n,
                                                          const double* __restrict__ Nop,
                                                          const int* __restrict__ gate) {
  if (gate && *gate == 0) return;
  extern __shared__ double Ns[];  // NT * NT * 256
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, g = lane >> 4;
  for (int i = tid; i < NT * NT * 256; i += PC_THREADS) Ns[i] = Nop[i];
  __syncthreads();
  const int64_t nchunk = (m + PC_CHUNK - 1) / PC_CHUNK;
  for (int64_t ch = blockIdx.x; ch < nchunk; ch += gridDim.x) {
    const int64_t r0 = ch * PC_CHUNK + 16 * wave;
    const int64_t rowa = r0 + li;
    const bool aok = rowa < m;
    const double* xa = X + (aok ? rowa : 0) * ldx;
    d4 xv[NT];
#pragma unroll
    for (int K = 0; K < NT; ++K) {
      const int c0 = 16 * K + 4 * g;
      if (VEC) {
        ld4<true>(xa + c0, aok && c0 < n, xv[K]);
      } else {
#pragma unroll
        for (int s = 0; s < 4; ++s) xv[K][s] = (aok && c0 + s < n) ? xa[c0 + s] : 0.0;
      }
    }
#pragma unroll
    for (int J = 0; J < NT; ++J) {
      d4 y = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int K = 0; K < NT; ++K) {
        const double* op = Ns + (K * NT + J) * 256 + lane;
#pragma unroll
        for (int s = 0; s < 4; ++s) y = mma(xv[K][s], op[64 * s], y);
      }
      const int col = 16 * J + li;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t rowy = r0 + 4 * r + g;
        if (rowy < m && col < n) X[rowy * ldx + col] = y[r];
      }
    }
  }
}

// The same product for 16-byte aligned rows and n a multiple of 4, pipelined: eight waves
// (one workgroup per CU, the 16 x 16-tile operand N in the local data share) and 128-row
// chunks; the rows of a wave's next chunk are loaded, with no branch, while the current
// chunk's tiles are formed.  Rows past m read row m - 1 and columns past n the last four
// columns; their results are not stored, and the padding rows of N are zero.
constexpr int RM_THREADS = 512;
constexpr int RM_CHUNK = 128;

template <int NT>
__global__ __launch_bounds__(RM_THREADS, 1) void k_rowmul_pipe(double* X, int64_t ldx,
                                                               int64_t m, int n,
                                                               const double* __restrict__ Nop,
                                                               const int* __restrict__ gate) {
  if (gate && *gate == 0) return;
  extern __shared__ double Ns[];  // NT * NT * 256
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, g = lane >> 4;
  for (int i = tid; i < NT * NT * 256; i += RM_THREADS) Ns[i] = Nop[i];
  __syncthreads();
  const int64_t nchunk = (m + RM_CHUNK - 1) / RM_CHUNK;
  int64_t ch = blockIdx.x;
  if (ch >= nchunk) return;
  int cc[NT];
#pragma unroll
  for (int K = 0; K < NT; ++K) cc[K] = (16 * K + 4 * g < n) ? 16 * K + 4 * g : n - 4;
  auto ld = [&](int64_t c, Quad<double> (&xv)[NT]) {
    const int64_t row = c * RM_CHUNK + 16 * wave + li;
    const double* xa = X + (row < m ? row : m - 1) * ldx;
#pragma unroll
    for (int K = 0; K < NT; ++K) xv[K].load(xa + cc[K]);
  };
  auto form = [&](int64_t c, Quad<double> (&xv)[NT]) {
    // the operand tiles are read per use: without the barrier the compiler would hoist all
    // of them out of the chunk loop (they do not change) and spill them
    asm volatile("" ::: "memory");
#pragma unroll
    for (int K = 0; K < NT; ++K) xv[K].pin();
    const int64_t r0 = c * RM_CHUNK + 16 * wave;
#pragma unroll
    for (int J = 0; J < NT; ++J) {
      d4 y = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int K = 0; K < NT; ++K) {
        const double* op = Ns + (K * NT + J) * 256 + lane;
#pragma unroll
        for (int s = 0; s < 4; ++s) y = mma(xv[K][s], op[64 * s], y);
      }
      const int col = 16 * J + li;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t rowy = r0 + 4 * r + g;
        if (rowy < m && col < n) X[rowy * ldx + col] = y[r];
      }
    }
  };
  Quad<double> xa[NT], xb[NT];
  ld(ch, xa);
  for (;;) {
    const int64_t c1 = ch + gridDim.x;
    ld(c1 < nchunk ? c1 : ch, xb);  // past the end: reloaded, not used
    form(ch, xa);
    if (c1 >= nchunk) break;
    const int64_t c2 = c1 + gridDim.x;
    ld(c2 < nchunk ? c2 : c1, xa);
    form(c1, xb);
    if (c2 >= nchunk) break;
    ch = c2;
  }
}

// Nop from N (n x n row-major, stride ldn; padding zero).
template <int NT>
__global__ void k_pack_rowmul(const double* __restrict__ N, int ldn, int n,
                              double* __restrict__ Nop) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= NT * NT * 256) return;
  const int tile = idx >> 8, s = (idx >> 6) & 3, lane = idx & 63;
  const int K = tile / NT, J = tile - K * NT;
  const int li = lane & 15, g = lane >> 4;
  const int row = 16 * K + 4 * g + s, col = 16 * J + li;
  Nop[idx] = (row < n && col < n) ? N[row * ldn + col] : 0.0;
}

// ---------------------------------------------------------------- small steps
// *flag = 1 when the estimate sqrt(||G||_1) ||Ri||_F of kappa_2(R), R^T R = G, Ri = R^-1,
// exceeds kmax or is not finite (||R||_2^2 = ||G||_2 <= ||G||_1; ||.||_2 <= ||.||_F).
__global__ __launch_bounds__(256) void k_kappa_flag(const double* __restrict__ G,
                                                    const double* __restrict__ Ri, int n,
                                                    double kmax, int* __restrict__ flag) {
  __shared__ double red[2][256];
  const int tid = threadIdx.x;
  double a = 0.0, b = 0.0;
  for (int j = tid; j < n; j += 256) {
    double c = 0.0;
    for (int i = 0; i < n; ++i) c += fabs(G[i * n + j]);
    a = fmax(a, c);
  }
  for (int i = tid; i < n * n; i += 256) b = fma(Ri[i], Ri[i], b);
  red[0][tid] = a;
  red[1][tid] = b;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) {
      red[0][tid] = fmax(red[0][tid], red[0][tid + w]);
      red[1][tid] += red[1][tid + w];
    }
    __syncthreads();
  }
  if (tid == 0) *flag = !(sqrt(red[0][0]) * sqrt(red[1][0]) <= kmax);
}

// The factors after one or two Cholesky passes (fl[2] selects):
//   Rtot = R2 Rp             Ninv = R2^-1     (dead flags d1)
//   Rtot = R3 R2b Rp         Ninv = R3^-1     (dead flags d2; R2b: the R2 the second solve used)
// with the rows of Rtot and of Ninv of a dropped direction zeroed.  A failed factorization
// (fl[0], or fl[3] on the second pass: a non-finite pivot) is reported as a non-finite
// result.  One workgroup; dynamic shared memory n x n doubles.
__global__ __launch_bounds__(1024) void k_pc_combine(
    const int* __restrict__ fl, const double* __restrict__ Rp, const double* __restrict__ R2,
    const double* __restrict__ R2b, const double* __restrict__ R2i,
    const double* __restrict__ R3, const double* __restrict__ R3i, const int* __restrict__ d1,
    const int* __restrict__ d2, int n, double* __restrict__ Rtot, double* __restrict__ Ninv,
    tssvd_info* __restrict__ info) {
  extern __shared__ double Tm[];  // n x n
  const int tid = threadIdx.x;
  const bool two = fl[2] != 0;
  const int* dd = two ? d2 : d1;
  // Tm = R3 R2b (upper triangular product; fixed k order) or R2
  for (int idx = tid; idx < n * n; idx += 1024) {
    const int i = idx / n, j = idx - i * n;
    double t = 0.0;
    if (two) {
      for (int k = i; k <= j; ++k) t = fma(R3[i * n + k], R2b[k * n + j], t);
    } else {
      t = R2[idx];
    }
    Tm[idx] = t;
  }
  __syncthreads();
  for (int idx = tid; idx < n * n; idx += 1024) {
    const int i = idx / n, j = idx - i * n;
    double t = 0.0;
    for (int k = i; k <= j; ++k) t = fma(Tm[i * n + k], Rp[k * n + j], t);
    Rtot[idx] = (j < i || dd[i]) ? 0.0 : t;
    Ninv[idx] = dd[i] ? 0.0 : (two ? R3i[idx] : R2i[idx]);
  }
  if (tid == 0 && info && (fl[0] || (two && fl[3]))) atomicOr(&info->numstat, NUM_NONFINITE);
}

template <int NT>
size_t trsm_lds() {
  return ((size_t)pc_pairs<NT>() * 256 + (size_t)PC_CHUNK * stage_ld<NT>()) * sizeof(double);
}

template <int NT>
hipError_t pc_launch_nt(const double* R, int ldr, int n, double tol, double* Rp, double* Rop,
                        const void* Xv, int x_dtype, int64_t ldx, int64_t m, double* Q,
                        int64_t ldq, double* part, bool gram, const int* gate, hipStream_t s) {
  static bool attr = false;
  const size_t lds2 = (size_t)pc_pairs<NT>() * 256 * sizeof(double);
  if (!attr) {
    hipError_t e = hipFuncSetAttribute((const void*)k_pc_trsm<NT, float>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)trsm_lds<NT>());
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute((const void*)k_pc_trsm<NT, double>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)trsm_lds<NT>());
    if (e != hipSuccess) return e;
    const void* k2[4] = {(const void*)k_pc_trsm2<NT, float>,
                         (const void*)k_pc_trsm_pipe<NT, float>,
                         (const void*)k_pc_trsm2<NT, double>,
                         (const void*)k_pc_trsm_pipe<NT, double>};
    for (const void* f : k2) {
      e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds2);
      if (e != hipSuccess) return e;
    }
    e = hipFuncSetAttribute((const void*)k_pc_prep<NT>,
                            hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)(16 * NT * (16 * NT + 1) * sizeof(double)));
    if (e != hipSuccess) return e;
    attr = true;
  }
  hipLaunchKernelGGL(k_pc_prep<NT>, dim3(1), dim3(256),
                     (size_t)16 * NT * (16 * NT + 1) * sizeof(double), s, R, ldr, n, tol, Rp,
                     Rop, gate);
  if (gram) {
    const int grid = pc_grid(m);
    if (x_dtype == TSSVD_F32)
      hipLaunchKernelGGL((k_pc_trsm<NT, float>), dim3(grid), dim3(PC_THREADS), trsm_lds<NT>(),
                         s, (const float*)Xv, ldx, m, n, Rop, Q, ldq, part, gate);
    else
      hipLaunchKernelGGL((k_pc_trsm<NT, double>), dim3(grid), dim3(PC_THREADS),
                         trsm_lds<NT>(), s, (const double*)Xv, ldx, m, n, Rop, Q, ldq, part,
                         gate);
  } else {
    const int64_t nch = (m + 2 * PC_CHUNK - 1) / (2 * PC_CHUNK);
    const int grid = (int)(nch < 2 * PC_GRID_MAX ? (nch > 0 ? nch : 1) : 2 * PC_GRID_MAX);
    const int64_t nch1 = (m + PC_CHUNK - 1) / PC_CHUNK;  // the pipelined kernel's chunks
    const int grid1 = (int)(nch1 < 2 * PC_GRID_MAX ? (nch1 > 0 ? nch1 : 1) : 2 * PC_GRID_MAX);
    // vector accesses when every row of X and Q starts on 16 bytes and n is whole fours
    const size_t xs = x_dtype == TSSVD_F32 ? 4 : 8;
    const bool vec = n % 4 == 0 && (reinterpret_cast<uintptr_t>(Xv) & 15) == 0 &&
                     (ldx * xs) % 16 == 0 && (reinterpret_cast<uintptr_t>(Q) & 15) == 0 &&
                     (ldq * 8) % 16 == 0;
    if (x_dtype == TSSVD_F32) {
      if (vec)
        hipLaunchKernelGGL((k_pc_trsm_pipe<NT, float>), dim3(grid1), dim3(PC_THREADS), lds2,
                           s, (const float*)Xv, ldx, m, n, Rop, Q, ldq, gate);
      else
        hipLaunchKernelGGL((k_pc_trsm2<NT, float>), dim3(grid), dim3(PC_THREADS), lds2,
                           s, (const float*)Xv, ldx, m, n, Rop, Q, ldq, gate);
    } else {
      if (vec)
        hipLaunchKernelGGL((k_pc_trsm_pipe<NT, double>), dim3(grid1), dim3(PC_THREADS), lds2,
                           s, (const double*)Xv, ldx, m, n, Rop, Q, ldq, gate);
      else
        hipLaunchKernelGGL((k_pc_trsm2<NT, double>), dim3(grid), dim3(PC_THREADS), lds2,
                           s, (const double*)Xv, ldx, m, n, Rop, Q, ldq, gate);
    }
  }
  return hipGetLastError();
}

template <int NT>
hipError_t rowmul_nt(double* X, int64_t ldx, int64_t m, int n, const double* N, int ldn,
                     double* Nop, int grid, const int* gate, hipStream_t s) {
  static bool attr = false;
  const size_t lds = (size_t)NT * NT * 256 * sizeof(double);
  if (!attr) {
    hipError_t e = hipFuncSetAttribute((const void*)k_rowmul<NT, false>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute((const void*)k_rowmul<NT, true>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    attr = true;
  }
  hipLaunchKernelGGL(k_pack_rowmul<NT>, dim3((NT * NT * 256 + 255) / 256), dim3(256), 0, s, N,
                     ldn, n, Nop);
  // vector loads when every row of X starts on 16 bytes and n is whole fours
  const bool vec = n % 4 == 0 && (reinterpret_cast<uintptr_t>(X) & 15) == 0 && ldx % 2 == 0;
  if (vec) {
    static bool attr2 = false;
    if (!attr2) {
      hipError_t e = hipFuncSetAttribute((const void*)k_rowmul_pipe<NT>,
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e != hipSuccess) return e;
      attr2 = true;
    }
    const int64_t nch = (m + RM_CHUNK - 1) / RM_CHUNK;
    const int g2 = (int)(nch < PC_GRID_MAX ? (nch > 0 ? nch : 1) : PC_GRID_MAX);
    hipLaunchKernelGGL((k_rowmul_pipe<NT>), dim3(g2), dim3(RM_THREADS), lds, s, X, ldx, m, n,
                       Nop, gate);
  } else
    hipLaunchKernelGGL((k_rowmul<NT, false>), dim3(grid), dim3(PC_THREADS), lds, s, X, ldx, m,
                       n, Nop, gate);
  return hipGetLastError();
}

}  // namespace

int pc_grid(int64_t m) {
  const int64_t nchunk = (m + PC_CHUNK - 1) / PC_CHUNK;
  return (int)(nchunk < PC_GRID_MAX ? (nchunk > 0 ? nchunk : 1) : PC_GRID_MAX);
}

size_t pc_op_elems(int n) {
  const int nt = (n + 15) / 16;
  const size_t a = (size_t)nt * (nt + 1) / 2 * 256, b = (size_t)nt * nt * 256;
  return a > b ? a : b;
}

hipError_t pc_trsm_gram(const double* R, int ldr, int n, double tol, double* Rp, double* Rop,
                        const void* X, int x_dtype, int64_t ldx, int64_t m, double* Q,
                        int64_t ldq, double* part, double* G, const int* gate, hipStream_t s,
                        bool gram) {
  hipError_t e;
  switch ((n + 15) / 16) {
    case 3: e = pc_launch_nt<3>(R, ldr, n, tol, Rp, Rop, X, x_dtype, ldx, m, Q, ldq, part, gram, gate, s); break;
    case 4: e = pc_launch_nt<4>(R, ldr, n, tol, Rp, Rop, X, x_dtype, ldx, m, Q, ldq, part, gram, gate, s); break;
    case 5: e = pc_launch_nt<5>(R, ldr, n, tol, Rp, Rop, X, x_dtype, ldx, m, Q, ldq, part, gram, gate, s); break;
    case 6: e = pc_launch_nt<6>(R, ldr, n, tol, Rp, Rop, X, x_dtype, ldx, m, Q, ldq, part, gram, gate, s); break;
    case 7: e = pc_launch_nt<7>(R, ldr, n, tol, Rp, Rop, X, x_dtype, ldx, m, Q, ldq, part, gram, gate, s); break;
    default: return hipErrorInvalidValue;
  }
  if (e != hipSuccess || !gram) return e;
  return reduce_chunks(part, pc_grid(m), n, n, G, n, s, gate);
}

hipError_t pc_rowmul(double* X, int64_t ldx, int64_t m, int n, const double* N, int ldn,
                     double* Nop, const int* gate, hipStream_t s) {
  const int grid = pc_grid(m);
  switch ((n + 15) / 16) {
    case 3: return rowmul_nt<3>(X, ldx, m, n, N, ldn, Nop, grid, gate, s);
    case 4: return rowmul_nt<4>(X, ldx, m, n, N, ldn, Nop, grid, gate, s);
    case 5: return rowmul_nt<5>(X, ldx, m, n, N, ldn, Nop, grid, gate, s);
    case 6: return rowmul_nt<6>(X, ldx, m, n, N, ldn, Nop, grid, gate, s);
    case 7: return rowmul_nt<7>(X, ldx, m, n, N, ldn, Nop, grid, gate, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t pc_kappa_flag(const double* G, const double* Ri, int n, double kmax, int* flag,
                         hipStream_t s) {
  hipLaunchKernelGGL(k_kappa_flag, dim3(1), dim3(256), 0, s, G, Ri, n, kmax, flag);
  return hipGetLastError();
}

hipError_t pc_combine(const int* fl, const double* Rp, const double* R2, const double* R2b,
                      const double* R2i, const double* R3, const double* R3i, const int* d1,
                      const int* d2, int n, double* Rtot, double* Ninv, tssvd_info* info,
                      hipStream_t s) {
  static bool attr = false;
  if (!attr) {
    hipError_t e = hipFuncSetAttribute((const void*)k_pc_combine,
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)(TSSVD_N_MAX * TSSVD_N_MAX * sizeof(double)));
    if (e != hipSuccess) return e;
    attr = true;
  }
  hipLaunchKernelGGL(k_pc_combine, dim3(1), dim3(1024), (size_t)n * n * sizeof(double), s, fl,
                     Rp, R2, R2b, R2i, R3, R3i, d1, d2, n, Rtot, Ninv, info);
  return hipGetLastError();
}

}  // namespace tsv
