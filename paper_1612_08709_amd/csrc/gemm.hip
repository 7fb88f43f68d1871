// Products with the large matrix A on gfx950 matrix cores (float64 path).
//
//   Y = A X   (m x n times n x l)   Algorithm 5 steps 2 and 9 (sketch and power steps)
//   Z = A^T Q (n x m times m x l)   Algorithm 5 step 5 and Algorithm 6 step 1 (B^* = A^* Q)
//
// Both stream A once.  They use v_mfma_f64_16x16x4_f64 (D += A(16x4) B(4x16)); per lane:
// A operand a[i = lane%16][k = lane/16], B operand b[k = lane/16][j = lane%16], result
// register r holds D[4*r + lane/16][lane%16] (measured on gfx950; the float32 16x16x4
// form instead holds D[4*(lane/16) + r][lane%16]).  The contraction index k may be mapped
// to any four values as long as A and B operands use the same map; both kernels use that
// freedom to give each lane contiguous runs of A.
//
// Z = A^T Q is split over row chunks of A ("split-K"); every (chunk, column tile) writes
// its partial n_tile x l block and a second kernel adds the chunks in chunk order, so
// the result is bitwise reproducible.  Workgroups sharing a row chunk are placed on the
// same XCD (workgroup IDs are dealt to the 8 XCDs round-robin) so the chunk of Q they
// all read stays in that XCD's L2.
#include "common.h"
#include "internal.h"

namespace tsv {

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8_t;

__device__ __forceinline__ f64x4 mfma_f64(double a, double b, f64x4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// ---------------------------------------------------------------- Y = A X
// 256 threads; wave w owns rows base + 16*(RT*w + rt) + (0..15); all NT column tiles.
// Per step of 16 along k, lane (i = lane%16, g = lane/16) loads A[row][k0+4g .. k0+4g+3]
// (one 16- or 32-byte vector when aligned) and uses element s in the s-th MFMA: k-slot g
// of MFMA s is column k0 + 4g + s.  The next step's A is loaded before this step's MFMAs.
__device__ __forceinline__ bool al16(const void* p) {
  return (reinterpret_cast<uintptr_t>(p) & 15) == 0;
}

__device__ __forceinline__ void load4(const double* p, bool full, int valid, double (&v)[4]) {
  if (full && al16(p)) {
    const double2 x0 = *reinterpret_cast<const double2*>(p);
    const double2 x1 = *reinterpret_cast<const double2*>(p + 2);
    v[0] = x0.x; v[1] = x0.y; v[2] = x1.x; v[3] = x1.y;
  } else {
#pragma unroll
    for (int s = 0; s < 4; ++s) v[s] = (s < valid) ? p[s] : 0.0;
  }
}

__device__ __forceinline__ void load4(const float* p, bool full, int valid, double (&v)[4]) {
  if (full && al16(p)) {
    const float4 x = *reinterpret_cast<const float4*>(p);
    v[0] = x.x; v[1] = x.y; v[2] = x.z; v[3] = x.w;
  } else {
#pragma unroll
    for (int s = 0; s < 4; ++s) v[s] = (s < valid) ? (double)p[s] : 0.0;
  }
}

// PACK (RT = 2, so wave w's rows are the 32-row block kb = blockIdx*4 + w): instead of
// storing Y, write the bfloat16 B-operand fragments of Y used by the mixed A^T Q kernels,
//   P[(kb*NT + nt)*64 + lane][e] = bf16(Y[32 kb + 8 (lane/16) + e][16 nt + lane%16]),
// each entry rounded once from its float64 value, exactly what packing the stored Y gives.
// The MFMA result rows 16 rt + 4 r + g of a lane become the fragment rows 8 g + e through
// a bfloat16 transpose in LDS.
//
// VEC (every row of A starts on 16 bytes and n is a multiple of 4): the main loop has no
// branch and no masked load, so the loads of the next step stay in flight while this
// step's MFMAs run (a load under a lane condition makes the compiler wait for it at the
// end of its branch).  Rows past m read row m - 1 and columns past l of X read column
// l - 1: those results are never stored.  The steps alternate between two register sets;
// a last step of fewer than 16 columns (n % 16 = 4, 8 or 12) is done once with a lane
// condition.
template <int RT, int NT, typename TA, bool PACK = false, bool VEC = false>
__global__ __launch_bounds__(256) void k_gemm_ax_f64(const TA* __restrict__ A, int64_t lda,
                                                     int64_t m, int n,
                                                     const double* __restrict__ X, int ldx,
                                                     int l, double* __restrict__ Y, int ldy,
                                                     bf16x8_t* __restrict__ P = nullptr,
                                                     int accum = 0) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, g = lane >> 4;
  const int64_t rbase = (int64_t)blockIdx.x * (64 * RT) + (int64_t)wave * (16 * RT);
  f64x4 acc[RT][NT];
#pragma unroll
  for (int rt = 0; rt < RT; ++rt)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) acc[rt][nt] = f64x4{0.0, 0.0, 0.0, 0.0};
  if constexpr (VEC) {
    const TA* ar[RT];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
      const int64_t row = rbase + 16 * rt + li;
      ar[rt] = A + (row < m ? row : m - 1) * lda + 4 * g;
    }
    int xc[NT];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) xc[nt] = (16 * nt + li < l) ? 16 * nt + li : l - 1;
    const double* xg = X + (int64_t)(4 * g) * ldx;
    auto ld = [&](int k0, Quad<TA> (&a)[RT], double (&x)[NT][4]) {
#pragma unroll
      for (int rt = 0; rt < RT; ++rt) a[rt].load(ar[rt] + k0);
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) x[nt][s] = xg[(int64_t)(k0 + s) * ldx + xc[nt]];
    };
    auto mm = [&](Quad<TA> (&a)[RT], const double (&x)[NT][4]) {
#pragma unroll
      for (int rt = 0; rt < RT; ++rt) a[rt].pin();
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int rt = 0; rt < RT; ++rt)
#pragma unroll
          for (int nt = 0; nt < NT; ++nt) acc[rt][nt] = mfma_f64(a[rt][s], x[nt][s], acc[rt][nt]);
    };
    const int nfull = n >> 4;  // whole 16-column steps
    Quad<TA> a0[RT], a1[RT];
    double x0[NT][4], x1[NT][4];
    int st = 0;
    if (nfull & 1) {
      ld(0, a0, x0);
      mm(a0, x0);
      st = 1;
    }
    if (st < nfull) {  // an even number of steps remains
      ld(16 * st, a0, x0);
      for (; st < nfull; st += 2) {
        // the empty asm statements keep each step's loads ahead of the other step's MFMAs
        // (without them the compiler moves the loads down to their uses)
        ld(16 * (st + 1), a1, x1);
        asm volatile("" ::: "memory");
        mm(a0, x0);
        ld(16 * (st + 2 < nfull ? st + 2 : st + 1), a0, x0);  // the last one is not used
        asm volatile("" ::: "memory");
        mm(a1, x1);
      }
    }
    if (16 * nfull < n) {
      const int kb = 16 * nfull + 4 * g;
#pragma unroll
      for (int rt = 0; rt < RT; ++rt) a0[rt].zero();
#pragma unroll
      for (int nt = 0; nt < NT; ++nt)
#pragma unroll
        for (int s = 0; s < 4; ++s) x0[nt][s] = 0.0;
      if (kb < n) {
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) a0[rt].load(ar[rt] + 16 * nfull);
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
          for (int nt = 0; nt < NT; ++nt)
            x0[nt][s] = xg[(int64_t)(16 * nfull + s) * ldx + xc[nt]];
      }
      mm(a0, x0);
    }
  } else {
    const TA* arow[RT];
    bool rok[RT];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
      const int64_t row = rbase + 16 * rt + li;
      rok[rt] = row < m;
      arow[rt] = A + (rok[rt] ? row : 0) * lda;
    }
    auto load_a = [&](int k0, double (&a)[RT][4]) {
      const int kb = k0 + 4 * g;
      const int valid = n - kb;
#pragma unroll
      for (int rt = 0; rt < RT; ++rt) {
        if (rok[rt] && valid > 0) {
          load4(arow[rt] + kb, valid >= 4, valid, a[rt]);
        } else {
#pragma unroll
          for (int s = 0; s < 4; ++s) a[rt][s] = 0.0;
        }
      }
    };
    double a[RT][4];
    load_a(0, a);
    for (int k0 = 0; k0 < n; k0 += 16) {
      double an[RT][4], x[NT][4];
      const int kn = (k0 + 16 < n) ? k0 + 16 : k0;
      load_a(kn, an);
      const int kb = k0 + 4 * g;
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int kk = kb + s;
        const bool kok = kk < n;
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
          const int col = 16 * nt + li;
          x[nt][s] = (kok && col < l) ? X[(int64_t)kk * ldx + col] : 0.0;
        }
      }
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int rt = 0; rt < RT; ++rt)
#pragma unroll
          for (int nt = 0; nt < NT; ++nt) acc[rt][nt] = mfma_f64(a[rt][s], x[nt][s], acc[rt][nt]);
#pragma unroll
      for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int s = 0; s < 4; ++s) a[rt][s] = an[rt][s];
    }
  }
  if constexpr (PACK) {
    static_assert(RT == 2, "one 32-row block per wave");
    // qs[wave][nt][col i][row 0..31]: a lane's eight fragment rows are 16 contiguous bytes
    __shared__ __attribute__((aligned(16))) __bf16 qs[4][NT][16][32];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
      for (int nt = 0; nt < NT; ++nt)
#pragma unroll
        for (int r = 0; r < 4; ++r) qs[wave][nt][li][16 * rt + 4 * r + g] = (__bf16)acc[rt][nt][r];
    __syncthreads();
    if (rbase < m) {
      const int64_t kb = rbase >> 5;
#pragma unroll
      for (int nt = 0; nt < NT; ++nt)
        P[(kb * NT + nt) * 64 + lane] = *reinterpret_cast<const bf16x8_t*>(&qs[wave][nt][li][8 * g]);
    }
    return;
  }
#pragma unroll
  for (int rt = 0; rt < RT; ++rt)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      const int col = 16 * nt + li;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = rbase + 16 * rt + 4 * r + g;
        if (row < m && col < l)
          Y[row * ldy + col] = accum ? Y[row * ldy + col] + acc[rt][nt][r] : acc[rt][nt][r];
      }
    }
}

// The branch-free main loop of k_gemm_ax_f64 applies when every row of A starts on 16 bytes
// and the contraction length is a multiple of 4.
template <typename TA>
static bool ax_vec(const TA* A, int64_t lda, int64_t n) {
  return (reinterpret_cast<uintptr_t>(A) & 15) == 0 && (lda * (int64_t)sizeof(TA)) % 16 == 0 &&
         n % 4 == 0;
}

template <int NT>
static void launch_ax_pack(const double* Y, int64_t ldy, int64_t m, const double* T, int ldt,
                           int l, void* P, hipStream_t s) {
  constexpr int RT = 2;
  const int64_t grid = (m + 64 * RT - 1) / (64 * RT);
  if (ax_vec(Y, ldy, l))
    hipLaunchKernelGGL((k_gemm_ax_f64<RT, NT, double, true, true>), dim3((unsigned)grid),
                       dim3(256), 0, s, Y, ldy, m, l, T, ldt, l, (double*)nullptr, 0,
                       (bf16x8_t*)P);
  else
    hipLaunchKernelGGL((k_gemm_ax_f64<RT, NT, double, true>), dim3((unsigned)grid), dim3(256),
                       0, s, Y, ldy, m, l, T, ldt, l, (double*)nullptr, 0, (bf16x8_t*)P);
}

hipError_t gemm_ax_f64_pack_bf16(const double* Y, int64_t ldy, int64_t m, const double* T,
                                 int ldt, int l, void* P, hipStream_t s) {
  switch ((l + 15) / 16) {
    case 1: launch_ax_pack<1>(Y, ldy, m, T, ldt, l, P, s); break;
    case 2: launch_ax_pack<2>(Y, ldy, m, T, ldt, l, P, s); break;
    case 3: launch_ax_pack<3>(Y, ldy, m, T, ldt, l, P, s); break;
    case 4: launch_ax_pack<4>(Y, ldy, m, T, ldt, l, P, s); break;
    case 5: launch_ax_pack<5>(Y, ldy, m, T, ldt, l, P, s); break;
    case 6: launch_ax_pack<6>(Y, ldy, m, T, ldt, l, P, s); break;
    case 7: launch_ax_pack<7>(Y, ldy, m, T, ldt, l, P, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int NT, typename TA>
static void launch_ax(const TA* A, int64_t lda, int64_t m, int64_t n, const double* X,
                      int ldx, int l, double* Y, int ldy, int accum, hipStream_t s) {
  constexpr int RT = 2;
  const int64_t grid = (m + 64 * RT - 1) / (64 * RT);
  if (ax_vec(A, lda, n))
    hipLaunchKernelGGL((k_gemm_ax_f64<RT, NT, TA, false, true>), dim3((unsigned)grid),
                       dim3(256), 0, s, A, lda, m, (int)n, X, ldx, l, Y, ldy, nullptr, accum);
  else
    hipLaunchKernelGGL((k_gemm_ax_f64<RT, NT, TA>), dim3((unsigned)grid), dim3(256), 0, s, A,
                       lda, m, (int)n, X, ldx, l, Y, ldy, nullptr, accum);
}

template <typename TA>
static hipError_t ax_dispatch(const TA* A, int64_t lda, int64_t m, int64_t n, const double* X,
                              int ldx, int l, double* Y, int ldy, int accum, hipStream_t s) {
  const int nt = (l + 15) / 16;
  switch (nt) {
    case 1: launch_ax<1>(A, lda, m, n, X, ldx, l, Y, ldy, accum, s); break;
    case 2: launch_ax<2>(A, lda, m, n, X, ldx, l, Y, ldy, accum, s); break;
    case 3: launch_ax<3>(A, lda, m, n, X, ldx, l, Y, ldy, accum, s); break;
    case 4: launch_ax<4>(A, lda, m, n, X, ldx, l, Y, ldy, accum, s); break;
    case 5: launch_ax<5>(A, lda, m, n, X, ldx, l, Y, ldy, accum, s); break;
    case 6: launch_ax<6>(A, lda, m, n, X, ldx, l, Y, ldy, accum, s); break;
    case 7: launch_ax<7>(A, lda, m, n, X, ldx, l, Y, ldy, accum, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t gemm_ax_f64(const void* A, int a_dtype, int64_t lda, int64_t m, int64_t n,
                       const double* X, int ldx, int l, double* Y, int ldy, hipStream_t s,
                       int prof) {
  prof_begin(prof, s);
  hipError_t e = (a_dtype == TSSVD_F64)
                     ? ax_dispatch((const double*)A, lda, m, n, X, ldx, l, Y, ldy, 0, s)
                     : ax_dispatch((const float*)A, lda, m, n, X, ldx, l, Y, ldy, 0, s);
  prof_end(prof, s);
  return e;
}

hipError_t gemm_ax_f64_acc(const double* A, int64_t lda, int64_t m, int64_t n, const double* X,
                           int ldx, int l, double* Y, int ldy, bool accum, hipStream_t s) {
  return ax_dispatch(A, lda, m, n, X, ldx, l, Y, ldy, accum ? 1 : 0, s);
}

// ---------------------------------------------------------------- Z = A^T Q
// Workgroup = (row chunk, 256-column tile); wave w owns columns c0 + 64w .. c0 + 64w + 63.
// Output rows of the MFMA are columns of A: tile mt (0..3) covers columns cw + 4*i + mt
// (i = 0..15), so lane (i, g) reads the four contiguous values A[row][cw+4i .. cw+4i+3].
// The contraction runs over rows: in one MFMA, k-slot g is row r + g.
constexpr int ATQ_COLS = 256;

// VEC (every row of A starts on 16 bytes and n is a multiple of 4): the whole four-row
// groups of the chunk run through a ring of ATQ_DEPTH groups in flight with no branch and
// no masked load (as in k_gemm_ax_f64); columns past n read columns n - 4 .. n - 1 and
// columns past l of Q read column l - 1, and those results are never stored.  The last
// partial group is done once with a lane condition.
constexpr int ATQ_DEPTH = 4;

template <int NT, typename TA, bool RS, typename TQ = double, bool VEC = false>
__global__ __launch_bounds__(256) void k_gemm_atq_f64(const TA* __restrict__ A, int64_t lda,
                                                      int64_t m, int n,
                                                      const TQ* __restrict__ Q, int ldq,
                                                      int l, int ncol, int nchunk,
                                                      int64_t chunk_rows,
                                                      double* __restrict__ part) {
  // RS (n <= 64, one column tile of one wave): every wave takes a row chunk of its own
  constexpr bool rowsplit = RS;
  const int total = rowsplit ? (nchunk + 3) / 4 : ncol * nchunk;
  const int per = (total + 7) / 8;
  const int L = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
  if (L >= total) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int chunk = rowsplit ? 4 * L + wave : L / ncol;
  const int ct = rowsplit ? 0 : L - chunk * ncol;
  if (chunk >= nchunk) return;
  const int li = lane & 15, g = lane >> 4;
  const int cw = rowsplit ? 0 : ct * ATQ_COLS + 64 * wave;
  if (cw >= n) return;
  const int64_t r0 = (int64_t)chunk * chunk_rows;
  const int64_t r1 = (r0 + chunk_rows < m) ? r0 + chunk_rows : m;
  f64x4 acc[4][NT];
#pragma unroll
  for (int mt = 0; mt < 4; ++mt)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = f64x4{0.0, 0.0, 0.0, 0.0};
  const int cb = cw + 4 * li;
  if constexpr (VEC) {
    const TA* ap = A + (r0 + g) * lda + (cb < n ? cb : n - 4);
    int qc[NT];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) qc[nt] = (16 * nt + li < l) ? 16 * nt + li : l - 1;
    const TQ* qp = Q + (r0 + g) * ldq;
    auto ld = [&](int64_t grp, Quad<TA>& a, double (&q)[NT]) {
      a.load(ap + 4 * grp * lda);
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) q[nt] = (double)qp[4 * grp * ldq + qc[nt]];
    };
    auto mm = [&](Quad<TA>& a, const double (&q)[NT]) {
      a.pin();
#pragma unroll
      for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = mfma_f64(a[mt], q[nt], acc[mt][nt]);
    };
    const int64_t nfull = (r1 - r0) >> 2;                 // whole four-row groups
    const int64_t nring = nfull / ATQ_DEPTH * ATQ_DEPTH;  // those run through the ring
    Quad<TA> a[ATQ_DEPTH];
    double q[ATQ_DEPTH][NT];
    // first the groups after the ring: at most ATQ_DEPTH, the last possibly partial; rows
    // past the chunk give zeros.  (Straight-line code before the loop: with MFMAs after
    // the loop the compiler copies the accumulators in and out of it on every iteration.)
#pragma unroll
    for (int t = 0; t < ATQ_DEPTH; ++t) {
      const int64_t gi = nring + t;
      a[t].zero();
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) q[t][nt] = 0.0;
      if (r0 + 4 * gi + g < r1) ld(gi, a[t], q[t]);
      mm(a[t], q[t]);
    }
    if (nring > 0) {
#pragma unroll
      for (int d = 0; d < ATQ_DEPTH; ++d) {
        ld(d, a[d], q[d]);
        asm volatile("" ::: "memory");  // the same load order as in the loop
      }
      for (int64_t gb = 0; gb < nring; gb += ATQ_DEPTH) {
#pragma unroll
        for (int d = 0; d < ATQ_DEPTH; ++d) {
          mm(a[d], q[d]);
          const int64_t nx = gb + ATQ_DEPTH + d;
          ld(nx < nring ? nx : gb + d, a[d], q[d]);  // past the ring: reloaded, not used
          // keeps the loads ahead of the next groups' MFMAs (the compiler would otherwise
          // move them down to their uses)
          asm volatile("" ::: "memory");
        }
      }
    }
  } else {
    const int cvalid = n - cb;
    auto load = [&](int64_t rq, double (&a)[4], double (&q)[NT]) {
      const int64_t row = rq + g;
      const bool rok = row < r1;
      const int64_t rr = rok ? row : r0;
      if (rok && cvalid > 0) {
        load4(A + rr * lda + cb, cvalid >= 4, cvalid, a);
      } else {
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) a[mt] = 0.0;
      }
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        const int col = 16 * nt + li;
        q[nt] = (rok && col < l) ? (double)Q[rr * ldq + col] : 0.0;
      }
    };
    double a[4], q[NT];
    load(r0, a, q);
    for (int64_t rq = r0; rq < r1; rq += 4) {
      double an[4], qn[NT];
      load((rq + 4 < r1) ? rq + 4 : rq, an, qn);
#pragma unroll
      for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = mfma_f64(a[mt], q[nt], acc[mt][nt]);
#pragma unroll
      for (int mt = 0; mt < 4; ++mt) a[mt] = an[mt];
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) q[nt] = qn[nt];
    }
  }
  double* P = part + (int64_t)chunk * n * l;
#pragma unroll
  for (int mt = 0; mt < 4; ++mt)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      const int col = 16 * nt + li;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = 4 * r + g;          // MFMA output row
        const int c = cw + 4 * i + mt;    // column of A
        if (c < n && col < l) P[(int64_t)c * l + col] = acc[mt][nt][r];
      }
    }
}

__global__ void k_reduce_chunks_strided(const double* __restrict__ part, int nchunk,
                                        int64_t count, int64_t stride, double* __restrict__ Z,
                                        int l, int ldz, const int* __restrict__ gate) {
  if (gate && *gate == 0) return;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= count) return;
  double s = 0.0;
  for (int c = 0; c < nchunk; ++c) s += part[(int64_t)c * stride + idx];
  const int64_t row = idx / l;
  const int col = (int)(idx - row * l);
  Z[row * ldz + col] = s;
}

__global__ void k_reduce_chunks(const double* __restrict__ part, int nchunk, int64_t count,
                                double* __restrict__ Z, int l, int ldz,
                                const int* __restrict__ gate) {
  if (gate && *gate == 0) return;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= count) return;
  // chunk order is fixed (bitwise reproducible); the loads of eight chunks are issued
  // before their additions so the latency of one does not serialize the next
  double s = 0.0;
  int c = 0;
  for (; c + 8 <= nchunk; c += 8) {
    double v[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = part[(int64_t)(c + j) * count + idx];
#pragma unroll
    for (int j = 0; j < 8; ++j) s += v[j];
  }
  for (; c < nchunk; ++c) s += part[(int64_t)c * count + idx];
  const int64_t row = idx / l;
  const int col = (int)(idx - row * l);
  Z[row * ldz + col] = s;
}

static void atq_grid(int64_t m, int64_t n, int& ncol, int& nchunk, int64_t& chunk_rows) {
  ncol = (int)((n + ATQ_COLS - 1) / ATQ_COLS);
  // n <= 64: one wave per row chunk (see the kernel), so ask for four chunks per workgroup
  int64_t want = n <= 64 ? 4096 : (1024 + ncol - 1) / ncol;
  const int64_t maxc = n <= 64 ? (m + 63) / 64 : (m + 255) / 256;
  if (want > maxc) want = maxc;
  if (want < 1) want = 1;
  chunk_rows = (m + want - 1) / want;
  chunk_rows = (chunk_rows + 15) / 16 * 16;
  nchunk = (int)((m + chunk_rows - 1) / chunk_rows);
}

size_t atq_partials(int64_t m, int64_t n, int l) {
  int ncol, nchunk;
  int64_t cr;
  atq_grid(m, n, ncol, nchunk, cr);
  return (size_t)nchunk * n * l;
}

template <int NT, typename TA, typename TQ = double>
static void launch_atq(const TA* A, int64_t lda, int64_t m, int64_t n, const TQ* Q, int ldq,
                       int l, double* part, hipStream_t s) {
  int ncol, nchunk;
  int64_t cr;
  atq_grid(m, n, ncol, nchunk, cr);
  const int total = n <= 64 ? (nchunk + 3) / 4 : ncol * nchunk;
  const int grid = ((total + 7) / 8) * 8;
  const bool vec = ax_vec(A, lda, n);
  if (n <= 64)
    hipLaunchKernelGGL((k_gemm_atq_f64<NT, TA, true, TQ>), dim3(grid), dim3(256), 0, s, A, lda, m,
                       (int)n, Q, ldq, l, ncol, nchunk, cr, part);
  else if (vec)
    hipLaunchKernelGGL((k_gemm_atq_f64<NT, TA, false, TQ, true>), dim3(grid), dim3(256), 0, s, A,
                       lda, m, (int)n, Q, ldq, l, ncol, nchunk, cr, part);
  else
    hipLaunchKernelGGL((k_gemm_atq_f64<NT, TA, false, TQ>), dim3(grid), dim3(256), 0, s, A, lda, m,
                       (int)n, Q, ldq, l, ncol, nchunk, cr, part);
}

template <typename TA, typename TQ = double>
static hipError_t atq_dispatch(const TA* A, int64_t lda, int64_t m, int64_t n, const TQ* Q,
                               int ldq, int l, double* part, hipStream_t s) {
  switch ((l + 15) / 16) {
    case 1: launch_atq<1, TA, TQ>(A, lda, m, n, Q, ldq, l, part, s); break;
    case 2: launch_atq<2, TA, TQ>(A, lda, m, n, Q, ldq, l, part, s); break;
    case 3: launch_atq<3, TA, TQ>(A, lda, m, n, Q, ldq, l, part, s); break;
    case 4: launch_atq<4, TA, TQ>(A, lda, m, n, Q, ldq, l, part, s); break;
    case 5: launch_atq<5, TA, TQ>(A, lda, m, n, Q, ldq, l, part, s); break;
    case 6: launch_atq<6, TA, TQ>(A, lda, m, n, Q, ldq, l, part, s); break;
    case 7: launch_atq<7, TA, TQ>(A, lda, m, n, Q, ldq, l, part, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------- G = Y^T Y
// Gram of a tall FP64 matrix with l <= 16*NT <= 64 columns (the bases of the power steps,
// the orthonormality checks).  Tile (ti, tj) of G is the product of Y's column tiles ti
// and tj, so one load serves both operands: per group of four rows, lane (i, g) loads
// Y[row0 + g][16t + i] (t < NT), the A operand of tile t (a[i][k = g]) and its B operand
// (b[k = g][j = i]) at once.  Only the tiles ti <= tj are formed.  Workgroup c takes rows
// [c*chunk, (c+1)*chunk); its wave w the four-row groups w, w+4, ...; the four waves'
// sums are added in a fixed order through LDS and the workgroup writes its partial Gram
// with both (i, j) and (j, i) set from the entry i <= j, so every partial, and the reduced
// G, is exactly symmetric.
constexpr int GRAM_WG_MAX = 512;
constexpr int GRAM_DEPTH = 4;  // four-row groups in flight per wave

template <int NT, typename TY = double>
__global__ __launch_bounds__(256) void k_gram_f64(const TY* __restrict__ Y, int64_t rows,
                                                  int l, int ldy, int64_t chunk,
                                                  double* __restrict__ part) {
  constexpr int NTILE = NT * (NT + 1) / 2;
  __shared__ double red[2][NTILE * 4 * 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, g = lane >> 4;
  const int64_t r0 = (int64_t)blockIdx.x * chunk;
  const int64_t r1 = (r0 + chunk < rows) ? r0 + chunk : rows;
  f64x4 acc[NTILE];
#pragma unroll
  for (int t = 0; t < NTILE; ++t) acc[t] = f64x4{0.0, 0.0, 0.0, 0.0};
  auto load = [&](int64_t grp, double (&y)[NT]) {
    const int64_t row = r0 + 4 * grp + g;
    const bool ok = row < r1;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const int col = 16 * t + li;
      y[t] = (ok && col < l) ? (double)Y[row * ldy + col] : 0.0;
    }
  };
  const int64_t ngrp = (r1 - r0 + 3) / 4;  // four-row groups of the chunk (r1 > r0)
  double y[GRAM_DEPTH][NT];
#pragma unroll
  for (int d = 0; d < GRAM_DEPTH; ++d) load(wave + 4 * d, y[d]);
  for (int64_t gb = wave; gb < ngrp; gb += 4 * GRAM_DEPTH) {
#pragma unroll
    for (int d = 0; d < GRAM_DEPTH; ++d) {
      int t = 0;
#pragma unroll
      for (int ti = 0; ti < NT; ++ti)
#pragma unroll
        for (int tj = ti; tj < NT; ++tj, ++t) acc[t] = mfma_f64(y[d][ti], y[d][tj], acc[t]);
      // groups past the chunk load zeros (their rows fail the row test)
      load(gb + 4 * (d + GRAM_DEPTH), y[d]);
    }
  }
  // fixed-order sum of the four waves: (w0 + w2) + (w1 + w3)
  auto put = [&](int slot) {
#pragma unroll
    for (int t = 0; t < NTILE; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) red[slot][(t * 4 + r) * 64 + lane] = acc[t][r];
  };
  auto add = [&](int slot) {
#pragma unroll
    for (int t = 0; t < NTILE; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[t][r] += red[slot][(t * 4 + r) * 64 + lane];
  };
  if (wave >= 2) put(wave - 2);
  __syncthreads();
  if (wave < 2) add(wave);
  __syncthreads();
  if (wave == 1) put(0);
  __syncthreads();
  if (wave != 0) return;
  add(0);
  double* P = part + (int64_t)blockIdx.x * l * l;
  int t = 0;
#pragma unroll
  for (int ti = 0; ti < NT; ++ti)
#pragma unroll
    for (int tj = ti; tj < NT; ++tj, ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = 16 * ti + 4 * r + g, j = 16 * tj + li;
        if (i <= j && j < l) {
          P[(int64_t)i * l + j] = acc[t][r];
          P[(int64_t)j * l + i] = acc[t][r];
        }
      }
}

// 65 <= l <= 16*NT <= 128: the NT(NT+1)/2 tiles are dealt to the four waves (tile t to wave
// t % 4), and every wave sums its tiles over all rows of the workgroup's chunk, so no
// cross-wave sum is needed and a wave holds at most ceil(NTILE/4) accumulator tiles.  Each
// wave loads every four-row group itself (the other waves' loads of it hit the L1).
template <int NT, int W, typename TY>
__device__ __forceinline__ void gram_wave_tiles(const TY* __restrict__ Y, int64_t r0, int64_t r1,
                                                int l, int ldy, double* __restrict__ P) {
  constexpr int NTILE = NT * (NT + 1) / 2;
  constexpr int PER = (NTILE - W + 3) / 4;  // tiles W, W+4, ...
  const int lane = threadIdx.x & 63, li = lane & 15, g = lane >> 4;
  // tile number -> (ti, tj), ti <= tj, in the order of k_gram_f64
  auto tile_i = [](int t) constexpr {
    int ti = 0;
    while (t >= NT - ti) { t -= NT - ti; ++ti; }
    return ti;
  };
  auto tile_j = [](int t) constexpr {
    int ti = 0;
    while (t >= NT - ti) { t -= NT - ti; ++ti; }
    return ti + t;
  };
  f64x4 acc[PER > 0 ? PER : 1];
#pragma unroll
  for (int q = 0; q < PER; ++q) acc[q] = f64x4{0.0, 0.0, 0.0, 0.0};
  auto load = [&](int64_t grp, double (&y)[NT]) {
    const int64_t row = r0 + 4 * grp + g;
    const bool ok = row < r1;
    const TY* yr = Y + (ok ? row : r0) * ldy;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const int col = 16 * t + li;
      const double v = (double)yr[col < l ? col : l - 1];
      y[t] = (ok && col < l) ? v : 0.0;
    }
  };
  const int64_t ngrp = (r1 - r0 + 3) / 4;
  double y0[NT], y1[NT];
  load(0, y0);
  load(1, y1);
  for (int64_t gb = 0; gb < ngrp; gb += 2) {
#pragma unroll
    for (int q = 0; q < PER; ++q)
      acc[q] = mfma_f64(y0[tile_i(W + 4 * q)], y0[tile_j(W + 4 * q)], acc[q]);
    load(gb + 2, y0);  // groups past the chunk load zeros
#pragma unroll
    for (int q = 0; q < PER; ++q)
      acc[q] = mfma_f64(y1[tile_i(W + 4 * q)], y1[tile_j(W + 4 * q)], acc[q]);
    load(gb + 3, y1);
  }
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int ti = tile_i(W + 4 * q), tj = tile_j(W + 4 * q);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = 16 * ti + 4 * r + g, j = 16 * tj + li;
      if (i <= j && j < l) {
        P[(int64_t)i * l + j] = acc[q][r];
        P[(int64_t)j * l + i] = acc[q][r];
      }
    }
  }
}

template <int NT, typename TY = double>
__global__ __launch_bounds__(256) void k_gram_f64w(const TY* __restrict__ Y, int64_t rows,
                                                   int l, int ldy, int64_t chunk,
                                                   double* __restrict__ part) {
  const int wave = threadIdx.x >> 6;
  const int64_t r0 = (int64_t)blockIdx.x * chunk;
  const int64_t r1 = (r0 + chunk < rows) ? r0 + chunk : rows;
  double* P = part + (int64_t)blockIdx.x * l * l;
  switch (wave) {
    case 0: gram_wave_tiles<NT, 0>(Y, r0, r1, l, ldy, P); break;
    case 1: gram_wave_tiles<NT, 1>(Y, r0, r1, l, ldy, P); break;
    case 2: gram_wave_tiles<NT, 2>(Y, r0, r1, l, ldy, P); break;
    default: gram_wave_tiles<NT, 3>(Y, r0, r1, l, ldy, P); break;
  }
}

// 33 <= l <= 16*NT <= 128, staged: 64-row chunks go to the workgroups in turn (chunk c to
// workgroup c mod gridDim.x, a fixed order per partial).  A chunk is loaded four rows per
// pass, 64 consecutive threads per row (coalesced), into registers while the previous chunk
// is summed, then stored to the local data share (padding columns as zeros).  Each wave sums
// its share of the NT(NT+1)/2 tile pairs over the 64 rows, both operands read from the
// staged rows (contraction over rows: lane (i, g) supplies row 4q + g of tile columns i).
constexpr int GS_CH = 64;
template <int NT>
constexpr int gs_ld() { return 16 * NT + 2; }
template <int NT>
constexpr size_t gs_lds() { return (size_t)GS_CH * gs_ld<NT>() * sizeof(double); }

template <int NT, typename TY>
__global__ __launch_bounds__(256, 2) void k_gram_staged(const TY* __restrict__ Y, int64_t rows,
                                                        int l, int ldy,
                                                        double* __restrict__ part) {
  constexpr int NTT = NT * (NT + 1) / 2;
  constexpr int NPW = (NTT + 3) / 4;
  constexpr int SLD = gs_ld<NT>();
  constexpr int CPR = (16 * NT + 63) / 64;  // 64-column slices per row
  constexpr int PASSES = GS_CH / 4;         // four rows per pass, 64 threads per row
  extern __shared__ double Sb[];  // GS_CH x SLD
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, g = lane >> 4;
  // thread t stages row 4 pass + t / 64, columns t % 64 + 64 c (padding past l: zeros)
  const int prow = tid >> 6, pcol = tid & 63;
  const int64_t nch = (rows + GS_CH - 1) / GS_CH;
  double pre[PASSES][CPR];
  auto load = [&](int64_t ch) {
    const int64_t r0 = ch * GS_CH + prow;
#pragma unroll
    for (int ps = 0; ps < PASSES; ++ps) {
      const int64_t row = r0 + 4 * ps;
      const TY* yr = Y + (row < rows ? row : 0) * (int64_t)ldy;
#pragma unroll
      for (int c = 0; c < CPR; ++c) {
        const int col = pcol + 64 * c;
        pre[ps][c] = (row < rows && col < l) ? (double)yr[col] : 0.0;
      }
    }
  };
  f64x4 acc[NPW];
#pragma unroll
  for (int p = 0; p < NPW; ++p) acc[p] = f64x4{0.0, 0.0, 0.0, 0.0};
  int tp[NPW], tq[NPW];
#pragma unroll
  for (int p = 0; p < NPW; ++p) {
    int t = wave + 4 * p, a = 0;
    if (t >= NTT) t = 0;  // unused slot (not summed)
    while (t >= NT - a) {
      t -= NT - a;
      ++a;
    }
    tp[p] = a;
    tq[p] = a + t;
  }
  if (blockIdx.x < nch) load(blockIdx.x);
  for (int64_t ch = blockIdx.x; ch < nch; ch += gridDim.x) {
    __syncthreads();  // the previous chunk's sums have read the staged rows
#pragma unroll
    for (int ps = 0; ps < PASSES; ++ps)
#pragma unroll
      for (int c = 0; c < CPR; ++c) {
        const int col = pcol + 64 * c;
        if (col < 16 * NT) Sb[(4 * ps + prow) * SLD + col] = pre[ps][c];
      }
    __syncthreads();
    if (ch + gridDim.x < nch) load(ch + gridDim.x);
#pragma unroll
    for (int p = 0; p < NPW; ++p) {
      if (wave + 4 * p < NTT) {
        const int ci = 16 * tp[p] + li, cj = 16 * tq[p] + li;
#pragma unroll
        for (int q = 0; q < GS_CH / 4; ++q) {
          const double* srow = Sb + (4 * q + g) * SLD;
          acc[p] = mfma_f64(srow[ci], srow[cj], acc[p]);
        }
      }
    }
  }
  double* P = part + (int64_t)blockIdx.x * l * l;
#pragma unroll
  for (int p = 0; p < NPW; ++p) {
    if (wave + 4 * p < NTT) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = 16 * tp[p] + 4 * r + g, j = 16 * tq[p] + li;
        if (i <= j && j < l) {  // diagonal tiles: the entry i <= j for both places
          P[(int64_t)i * l + j] = acc[p][r];
          P[(int64_t)j * l + i] = acc[p][r];
        }
      }
    }
  }
}

template <int NT, typename TY>
static hipError_t launch_gram_staged(const TY* Y, int64_t rows, int l, int ldy, int nwg,
                                     double* part, hipStream_t s) {
  static bool attr = false;
  if (!attr) {
    hipError_t e = hipFuncSetAttribute((const void*)k_gram_staged<NT, TY>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)gs_lds<NT>());
    if (e != hipSuccess) return e;
    attr = true;
  }
  hipLaunchKernelGGL((k_gram_staged<NT, TY>), dim3(nwg), dim3(256), gs_lds<NT>(), s, Y, rows, l,
                     ldy, part);
  return hipGetLastError();
}

// Workgroups (row chunks) of the Gram kernels.  Never more chunks than the A^T Q kernels
// use for the same shape (atq_grid: ceil(rows/64) up to l = 64, ceil(rows/256) beyond), so
// the partials fit in the atq_partials(rows, l, l) doubles callers provide.
static int gram_grid(int64_t rows, int l, int64_t& chunk) {
  int64_t want = l <= 64 ? (rows + 63) / 64 : (rows + 255) / 256;
  if (want > GRAM_WG_MAX) want = GRAM_WG_MAX;
  chunk = (rows + want - 1) / want;
  chunk = (chunk + 15) / 16 * 16;
  return (int)((rows + chunk - 1) / chunk);
}

template <typename TY>
static hipError_t gram_f64(const TY* Y, int64_t rows, int l, int ldy, double* G, int ldg,
                           double* part, hipStream_t s) {
  if (l >= 33) {
    // staged kernel: at most 512 workgroups and never more than the partials callers
    // provide (the A^T Q chunk count for this shape)
    int ncol, nck;
    int64_t cr;
    atq_grid(rows, l, ncol, nck, cr);
    const int64_t nch = (rows + GS_CH - 1) / GS_CH;
    int64_t nwg = nch < 512 ? nch : 512;
    if (nwg > nck) nwg = nck;
    if (nwg < 1) nwg = 1;
    hipError_t e;
    switch ((l + 15) / 16) {
      case 3: e = launch_gram_staged<3>(Y, rows, l, ldy, (int)nwg, part, s); break;
      case 4: e = launch_gram_staged<4>(Y, rows, l, ldy, (int)nwg, part, s); break;
      case 5: e = launch_gram_staged<5>(Y, rows, l, ldy, (int)nwg, part, s); break;
      case 6: e = launch_gram_staged<6>(Y, rows, l, ldy, (int)nwg, part, s); break;
      case 7: e = launch_gram_staged<7>(Y, rows, l, ldy, (int)nwg, part, s); break;
      case 8: e = launch_gram_staged<8>(Y, rows, l, ldy, (int)nwg, part, s); break;
      default: return hipErrorInvalidValue;
    }
    if (e != hipSuccess) return e;
    return reduce_chunks(part, (int)nwg, l, l, G, ldg, s);
  }
  int64_t chunk;
  const int nwg = gram_grid(rows, l, chunk);
  switch ((l + 15) / 16) {
    case 1: hipLaunchKernelGGL((k_gram_f64<1, TY>), dim3(nwg), dim3(256), 0, s, Y, rows, l, ldy, chunk, part); break;
    case 2: hipLaunchKernelGGL((k_gram_f64<2, TY>), dim3(nwg), dim3(256), 0, s, Y, rows, l, ldy, chunk, part); break;
    case 3: hipLaunchKernelGGL((k_gram_f64<3, TY>), dim3(nwg), dim3(256), 0, s, Y, rows, l, ldy, chunk, part); break;
    case 4: hipLaunchKernelGGL((k_gram_f64<4, TY>), dim3(nwg), dim3(256), 0, s, Y, rows, l, ldy, chunk, part); break;
    case 5: hipLaunchKernelGGL((k_gram_f64w<5, TY>), dim3(nwg), dim3(256), 0, s, Y, rows, l, ldy, chunk, part); break;
    case 6: hipLaunchKernelGGL((k_gram_f64w<6, TY>), dim3(nwg), dim3(256), 0, s, Y, rows, l, ldy, chunk, part); break;
    case 7: hipLaunchKernelGGL((k_gram_f64w<7, TY>), dim3(nwg), dim3(256), 0, s, Y, rows, l, ldy, chunk, part); break;
    case 8: hipLaunchKernelGGL((k_gram_f64w<8, TY>), dim3(nwg), dim3(256), 0, s, Y, rows, l, ldy, chunk, part); break;
    default: return hipErrorInvalidValue;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return reduce_chunks(part, nwg, l, l, G, ldg, s);
}

// ---------------------------------------------------------------- column sums of squares
// out[j] = sum_i Y[i][j]^2 (Y rows x l, stride ldy, l <= 256): workgroup c sums rows
// [c*chunk, (c+1)*chunk) in order, thread j its column (consecutive threads read
// consecutive columns of a row), and the chunks are added in a fixed order.
template <typename TY>
__global__ __launch_bounds__(256) void k_colsq(const TY* __restrict__ Y, int64_t rows, int l,
                                               int64_t ldy, int64_t chunk,
                                               double* __restrict__ part) {
  const int j = threadIdx.x;
  if (j >= l) return;
  const int64_t r0 = (int64_t)blockIdx.x * chunk;
  const int64_t r1 = (r0 + chunk < rows) ? r0 + chunk : rows;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};  // four interleaved running sums, added in order
  int64_t r = r0;
  for (; r + 4 <= r1; r += 4) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const double y = (double)Y[(r + u) * ldy + j];
      acc[u] = fma(y, y, acc[u]);
    }
  }
  for (; r < r1; ++r) {
    const double y = (double)Y[r * ldy + j];
    acc[0] = fma(y, y, acc[0]);
  }
  part[(int64_t)blockIdx.x * l + j] = (acc[0] + acc[1]) + (acc[2] + acc[3]);
}

hipError_t column_sumsq(const void* Y, int y_dtype, int64_t rows, int l, int64_t ldy, double* out,
                        double* part, hipStream_t s) {
  if (l < 1 || l > 256) return hipErrorInvalidValue;
  int64_t want = (rows + 255) / 256;
  if (want > GRAM_WG_MAX) want = GRAM_WG_MAX;
  if (want < 1) want = 1;
  const int64_t chunk = (rows + want - 1) / want;
  const int nwg = (int)((rows + chunk - 1) / chunk);
  if (y_dtype == TSSVD_F64)
    hipLaunchKernelGGL((k_colsq<double>), dim3(nwg), dim3(256), 0, s, (const double*)Y, rows, l,
                       ldy, chunk, part);
  else
    hipLaunchKernelGGL((k_colsq<float>), dim3(nwg), dim3(256), 0, s, (const float*)Y, rows, l,
                       ldy, chunk, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return reduce_chunks(part, nwg, 1, l, out, l, s);
}

size_t column_sumsq_partials(int64_t rows, int l) {
  int64_t want = (rows + 255) / 256;
  if (want > GRAM_WG_MAX) want = GRAM_WG_MAX;
  if (want < 1) want = 1;
  return (size_t)want * l;
}

// G = Y^T Y (l x l) for a tall Y of either storage type: the Gram kernel for l <= 64, the
// split-K A^T Q kernel with Q = Y otherwise.  `part` holds atq_partials(rows, l, l) doubles.
hipError_t gram_any(const void* Y, int y_dtype, int64_t ldy, int64_t rows, int l, double* G,
                    int ldg, double* part, hipStream_t s) {
  if (l <= 128)
    return (y_dtype == TSSVD_F64)
               ? gram_f64((const double*)Y, rows, l, (int)ldy, G, ldg, part, s)
               : gram_f64((const float*)Y, rows, l, (int)ldy, G, ldg, part, s);
  hipError_t e = (y_dtype == TSSVD_F64)
                     ? atq_dispatch((const double*)Y, ldy, rows, l, (const double*)Y, (int)ldy,
                                    l, part, s)
                     : atq_dispatch((const float*)Y, ldy, rows, l, (const float*)Y, (int)ldy, l,
                                    part, s);
  if (e != hipSuccess) return e;
  int ncol, nchunk;
  int64_t cr;
  atq_grid(rows, l, ncol, nchunk, cr);
  return reduce_chunks(part, nchunk, l, l, G, ldg, s);
}

hipError_t gemm_atq_f64(const void* A, int a_dtype, int64_t lda, int64_t m, int64_t n,
                        const double* Q, int ldq, int l, double* Z, int ldz, double* part,
                        hipStream_t s, int prof) {
  if (a_dtype == TSSVD_F64 && A == (const void*)Q && lda == ldq && n == l && l <= 128 && m > 0)
    return gram_f64(Q, m, l, ldq, Z, ldz, part, s);  // partials fit: nwg <= atq chunks
  prof_begin(prof, s);
  hipError_t e = (a_dtype == TSSVD_F64)
                     ? atq_dispatch((const double*)A, lda, m, n, Q, ldq, l, part, s)
                     : atq_dispatch((const float*)A, lda, m, n, Q, ldq, l, part, s);
  prof_end(prof, s);
  if (e != hipSuccess) return e;
  int ncol, nchunk;
  int64_t cr;
  atq_grid(m, n, ncol, nchunk, cr);
  return reduce_chunks(part, nchunk, n, l, Z, ldz, s);
}

// First level for many chunks: group gi adds chunks gi*G .. gi*G + G - 1 (in order) and
// stores the sum over chunk gi*G's slot, which only this group reads.
__global__ void k_reduce_groups(double* __restrict__ part, int nchunk, int64_t count, int G,
                                const int* __restrict__ gate) {
  if (gate && *gate == 0) return;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= count) return;
  const int c0 = blockIdx.y * G;
  const int c1 = (c0 + G < nchunk) ? c0 + G : nchunk;
  double s = 0.0;
  int c = c0;
  for (; c + 8 <= c1; c += 8) {
    double v[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = part[(int64_t)(c + j) * count + idx];
#pragma unroll
    for (int j = 0; j < 8; ++j) s += v[j];
  }
  for (; c < c1; ++c) s += part[(int64_t)c * count + idx];
  part[(int64_t)c0 * count + idx] = s;
}

hipError_t reduce_chunks(const double* part, int nchunk, int64_t n, int l, double* Z, int ldz,
                         hipStream_t s, const int* gate) {
  const int64_t count = n * (int64_t)l;
  if (nchunk > 64 && count < (1 << 16)) {
    // few outputs, many chunks (Grams of tall matrices): two fixed-order levels, so the
    // sums run on many threads instead of one long chain per output
    const int G = (nchunk + 63) / 64;
    const int ng = (nchunk + G - 1) / G;
    hipLaunchKernelGGL(k_reduce_groups, dim3((unsigned)((count + 255) / 256), ng), dim3(256), 0,
                       s, const_cast<double*>(part), nchunk, count, G, gate);
    hipLaunchKernelGGL(k_reduce_chunks_strided, dim3((unsigned)((count + 255) / 256)),
                       dim3(256), 0, s, part, ng, count, (int64_t)G * count, Z, l, ldz, gate);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_reduce_chunks, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s,
                     part, nchunk, count, Z, l, ldz, gate);
  return hipGetLastError();
}

}  // namespace tsv
