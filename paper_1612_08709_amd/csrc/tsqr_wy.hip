// Blocked (compact WY) TSQR leaf for 33 <= n <= 128 on gfx950 matrix cores, in float64 or
// (for the first orthonormalization of the mixed-precision tall-skinny SVD) float32
// arithmetic.
//
// Method (Algorithm 1 step 2; Section 2's reduction): a workgroup walks its row blocks A_t
// (128 rows) in order, carrying the triangular factor R of the rows seen so far, and
// factors the stacked matrix [R; A_t] by Householder reflectors.  Reflector j touches row j
// of R and the block rows only, so its vector is y_j = [e_j; v_j] and it is stored as the
// block part v_j.  The n reflectors are taken 16 at a time (a panel p of columns
// 16p .. 16p+15): the panel's reflectors are formed one column at a time, then they are
// applied to the other columns at once in compact WY form,
//   H_{16p} ... H_{16p+15} = I - Y_p T_p Y_p^T   (T_p 16 x 16 upper triangular),
// as two products on the matrix cores: W = Y_p^T X (a contraction over the block rows)
// and X -= Y_p (T_p^T W).  The same contraction against the panels already done gives
// Z_cp = V_c^T V_p (c < p); with the T_p these determine the block's whole reflector product
// Q_t = I - Y T Y^T, T = [T_c, T_cp; 0, T_p], T_cp = -T_c Z_cp T_p (the usual forward
// accumulation), which the apply pass uses without forming T.
//
// Apply pass (U = Q [S; 0] for a seed S from the merge tree): Q_t [S; 0] = [S - W; -V W]
// with W = T S, and W is found panel by panel from the last one back,
//   W_p = T_p (S_p - sum_{q > p} Z_pq W_q)
// (each W_q is subtracted from the sums of the earlier panels as soon as it is formed),
// so each block costs a small n x n x k recurrence plus one 128 x n x k product that
// writes the block's rows of U; the seed of the block before is S - W.
//
// Matrix-core layout (v_mfma_f64_16x16x4_f64 and v_mfma_f32_16x16x4_f32, measured): lane
// (i = lane%16, g = lane/16); A operand a[i][k=g], B operand b[k=g][j=i].  The result
// register r holds D[row(r, g)][i] with row(r, g) = 4r + g in float64 and 4g + r in
// float32.  A 16 x 16 tile "in result layout" is held as 4 registers per lane.  A
// contraction over the rows of two such tiles needs no data movement: in the s-th
// instruction lane (i, g) supplies its register s of both (row(s, g)).  Tiles read as A
// operands from memory are stored "operand-permuted": row i keeps column row(s, g) at
// position 4g + s, so a lane loads its four k values as one vector.
#include <cstddef>
#include <type_traits>

#include "common.h"
#include "internal.h"

namespace tsv {

namespace {

constexpr int WB = 128;       // rows per block
constexpr int WWAVES = 4;     // waves per workgroup, 32 rows (two 16-row tiles) each
constexpr int WTHREADS = 64 * WWAVES;

// ---- per compute type: matrix-core instruction and its register layout
template <typename CT>
struct Wy;

template <>
struct Wy<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 mma(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // row of the tile held by result register r of lane group g
  static __host__ __device__ constexpr int row(int r, int g) { return 4 * r + g; }
  // register and lane group holding row j
  static __host__ __device__ constexpr int reg_of(int j) { return j >> 2; }
  static __host__ __device__ constexpr int grp_of(int j) { return j & 3; }
};

template <>
struct Wy<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 mma(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __host__ __device__ constexpr int row(int r, int g) { return 4 * g + r; }
  static __host__ __device__ constexpr int reg_of(int j) { return j & 3; }
  static __host__ __device__ constexpr int grp_of(int j) { return j >> 2; }
};

// operand-permuted position of column k within its 16-column group: column row(s, g) at 4g+s
template <typename CT>
__host__ __device__ constexpr int opos(int k) {
  return 4 * Wy<CT>::grp_of(k) + Wy<CT>::reg_of(k);
}

// ---- cross-lane moves on 32-bit words, and their float64 (two-word) forms
// x + x[lane ^ 16] and x + x[lane ^ 32], through the row-swap instructions: after the swap
// the two registers hold the values of both rows of each pair, and their sum has the same
// operand order in both rows, so the partner lanes get bitwise-equal sums.
__device__ __forceinline__ float pair_sum16(float x) {
  const unsigned u = __float_as_uint(x);
  const auto a = __builtin_amdgcn_permlane16_swap(u, u, false, false);
  return __uint_as_float(a[0]) + __uint_as_float(a[1]);
}
__device__ __forceinline__ float pair_sum32(float x) {
  const unsigned u = __float_as_uint(x);
  const auto a = __builtin_amdgcn_permlane32_swap(u, u, false, false);
  return __uint_as_float(a[0]) + __uint_as_float(a[1]);
}
__device__ __forceinline__ double pair_sum16(double x) {
  const unsigned lo = (unsigned)__double2loint(x), hi = (unsigned)__double2hiint(x);
  const auto a = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
  const auto b = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
  return __hiloint2double((int)b[0], (int)a[0]) + __hiloint2double((int)b[1], (int)a[1]);
}
__device__ __forceinline__ double pair_sum32(double x) {
  const unsigned lo = (unsigned)__double2loint(x), hi = (unsigned)__double2hiint(x);
  const auto a = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
  const auto b = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
  return __hiloint2double((int)b[0], (int)a[0]) + __hiloint2double((int)b[1], (int)a[1]);
}

// Row G (lanes 16G .. 16G+15) of x copied to all four 16-lane rows, lane by lane.
template <int G>
__device__ __forceinline__ unsigned row_to_all_u(unsigned x) {
  const auto a = __builtin_amdgcn_permlane16_swap(x, x, false, false);  // rows (0,0,2,2) | (1,1,3,3)
  const unsigned y = (G & 1) ? a[1] : a[0];
  const auto b = __builtin_amdgcn_permlane32_swap(y, y, false, false);  // halves (lo,lo) | (hi,hi)
  return (G & 2) ? b[1] : b[0];
}
template <int G>
__device__ __forceinline__ float row_to_all(float x) {
  return __uint_as_float(row_to_all_u<G>(__float_as_uint(x)));
}
template <int G>
__device__ __forceinline__ double row_to_all(double x) {
  return __hiloint2double((int)row_to_all_u<G>((unsigned)__double2hiint(x)),
                          (int)row_to_all_u<G>((unsigned)__double2loint(x)));
}

// x from lane j of this lane's 16-lane row (DPP row broadcast).
template <int J>
__device__ __forceinline__ float row_bcast(float x) {
  return __int_as_float(
      __builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x150 + J, 0xF, 0xF, false));
}
template <int J>
__device__ __forceinline__ double row_bcast(double x) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), 0x150 + J, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), 0x150 + J, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

// Reflector of (alpha, x) with ||x||^2 = s: beta = -sign(alpha) sqrt(alpha^2 + s),
// tau = (beta - alpha) / beta, scale = 1 / (alpha - beta) (v = scale x); s = 0 gives the
// identity (tau = 0, beta = alpha, scale = 0).  Written with the hardware reciprocal square
// root and reciprocal, each refined by Newton steps (two in float64, one in float32;
// relative error a few units in the last place), and |beta - alpha| = |alpha| + nrm, so
// tau = (|alpha| + nrm) / nrm; the operands of rsq and rcp stay finite and non-zero.
__device__ __forceinline__ void householder(double alpha, double s, double& beta, double& tau,
                                            double& scale) {
  const double q = fma(alpha, alpha, s);
  const bool live = s > 0.0 && q > 0.0;
  // below 2^-900 the argument is scaled by 2^900 (exactly), so the hardware reciprocal
  // square root never sees a subnormal (a column that is zero up to rounding)
  const bool tiny = q < 0x1p-900;
  const double qq = live ? (tiny ? q * 0x1p900 : q) : 1.0;
  double rs = __builtin_amdgcn_rsq(qq);
  rs = rs * fma(-0.5 * qq * rs, rs, 1.5);
  rs = rs * fma(-0.5 * qq * rs, rs, 1.5);
  const double nrm = tiny ? (qq * rs) * 0x1p-450 : qq * rs;
  rs = tiny ? rs * 0x1p450 : rs;
  const double gam = fabs(alpha) + nrm;  // |alpha - beta|
  double rg = __builtin_amdgcn_rcp(gam);
  rg = rg * fma(-gam, rg, 2.0);
  rg = rg * fma(-gam, rg, 2.0);
  const double b = alpha >= 0.0 ? -nrm : nrm;
  beta = live ? b : alpha;
  tau = live ? gam * rs : 0.0;
  scale = live ? (alpha >= 0.0 ? rg : -rg) : 0.0;
}
__device__ __forceinline__ void householder(float alpha, float s, float& beta, float& tau,
                                            float& scale) {
  const float q = fmaf(alpha, alpha, s);
  const bool live = s > 0.0f && q > 0.0f;
  // below 2^-100 scaled by 2^100 (exactly): a column that is zero up to float32 rounding
  // (a block with fewer rows than columns leaves such columns) can square to a subnormal
  const bool tiny = q < 0x1p-100f;
  const float qq = live ? (tiny ? q * 0x1p100f : q) : 1.0f;
  float rs = __builtin_amdgcn_rsqf(qq);
  rs = rs * fmaf(-0.5f * qq * rs, rs, 1.5f);
  const float nrm = tiny ? (qq * rs) * 0x1p-50f : qq * rs;
  rs = tiny ? rs * 0x1p50f : rs;
  const float gam = fabsf(alpha) + nrm;
  float rg = __builtin_amdgcn_rcpf(gam);
  rg = rg * fmaf(-gam, rg, 2.0f);
  const float b = alpha >= 0.0f ? -nrm : nrm;
  beta = live ? b : alpha;
  tau = live ? gam * rs : 0.0f;
  scale = live ? (alpha >= 0.0f ? rg : -rg) : 0.0f;
}

// f(integral_constant<int, I>) for I = B .. E-1, at compile time
template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}

// Four adjacent elements from a 16-byte aligned address, as vector loads.
__device__ __forceinline__ void load4_aligned(const double* p, double (&v)[4]) {
  const double2 a = *reinterpret_cast<const double2*>(p);
  const double2 b = *reinterpret_cast<const double2*>(p + 2);
  v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y;
}
__device__ __forceinline__ void load4_aligned(const float* p, float (&v)[4]) {
  const float4 a = *reinterpret_cast<const float4*>(p);
  v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
}

// Index of the upper tile (p, c), p <= c, in the packed tile list of an NT x NT grid.
__host__ __device__ constexpr int utile(int p, int c, int nt) { return p * nt - p * (p - 1) / 2 + (c - p); }
// Index of the strictly upper pair (c, q), c < q.
__host__ __device__ constexpr int upair(int c, int q, int nt) { return c * nt - c * (c + 1) / 2 + (q - c - 1); }

// Column tiles per contraction round (partials staged in the local data share).  With
// float64 and n <= 112 the shared state stays under 80 KB, so two workgroups share a CU and
// each hides the other's barrier waits and block loads; in float32 (half the registers and
// shared state) four do.
template <int NT>
constexpr int wch() { return NT <= 4 ? NT - 1 : 2; }

template <typename CT, int NT>
struct WyShared {
  CT R[NT * (NT + 1) / 2][4][64];  // carried factor, upper tiles in result layout
  CT part[WWAVES][wch<NT>()][4][64];  // per-wave partial contractions (V transposes first)
  CT Wbr[wch<NT>()][4][64];        // -T_p^T W of the round's tiles
  CT slot[2][WWAVES][16];          // per-wave partial column dots (panel steps)
  CT ZT[16][16];                   // v_k^T v_j (k < j) of the panel, then T_p (row-major)
  CT tau[16];                      // directly after ZT (read as ZT[16][0..15])
};

}  // namespace

template <typename CT, int NT>
size_t wy_factor_lds() { return sizeof(WyShared<CT, NT>); }

// One leaf chain per workgroup: blocks [blockIdx.x*bpw, ...).  Outputs per block: V
// (128 x 16NT, operand-permuted rows), T_p (NT tiles, operand-permuted), Z_cp (pairs c < p,
// operand-permuted), all in the compute type; per workgroup the final R (n x n row-major,
// zero below the diagonal, float64).
template <typename CT, int NT, typename TA>
__global__ __launch_bounds__(WTHREADS, sizeof(CT) == 4 ? 4 : 2) void k_wy_factor(
    const TA* __restrict__ A, int64_t lda, int64_t m, int n, int bpw, int64_t nblocks,
    CT* __restrict__ Vg, CT* __restrict__ Tg, CT* __restrict__ Zg, double* __restrict__ Rw,
    const int* __restrict__ gate) {
  using L = Wy<CT>;
  using v4 = typename L::v4;
  if (gate && *gate == 0) return;
  extern __shared__ __attribute__((aligned(16))) char wy_smem[];
  WyShared<CT, NT>& sh = *reinterpret_cast<WyShared<CT, NT>*>(wy_smem);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, g = lane >> 4;
  constexpr int NTT = NT * (NT + 1) / 2;
  constexpr int NPAIR = NT * (NT - 1) / 2;
  constexpr int LDV = 16 * NT;
  constexpr int WCH = wch<NT>();
  static_assert(WCH * 256 >= 512, "a wave's part[] area must hold its two 16 x 16 tiles");
  const CT zero = CT(0), one = CT(1);

  for (int i = tid; i < NTT * 256; i += WTHREADS) (&sh.R[0][0][0])[i] = zero;
  __syncthreads();

  const int64_t b0 = (int64_t)blockIdx.x * bpw;
  const int64_t b1 = (b0 + bpw < nblocks) ? b0 + bpw : nblocks;
  for (int64_t blk = b0; blk < b1; ++blk) {
    // ---- load the block: a[rt][c][r] = A[row0 + 32 wave + 16 rt + row(r, g)][16 c + li]
    CT a[2][NT][4];
    const int64_t rbase = blk * WB + 32 * wave;
    {
      // the last tile is the only one that can pass n (NT = ceil(n / 16)); its lanes past n
      // read column n-1 and are zeroed, rows past m read row m-1 and are zeroed
      const int lastc = 16 * (NT - 1) + li < n ? 16 * (NT - 1) + li : n - 1;
      const bool lastok = 16 * (NT - 1) + li < n;
#pragma unroll
      for (int rt = 0; rt < 2; ++rt)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t row = rbase + 16 * rt + L::row(r, g);
          const bool rok = row < m;
          const TA* ar = A + (rok ? row : m - 1) * lda;
#pragma unroll
          for (int c = 0; c < NT - 1; ++c) a[rt][c][r] = (CT)ar[16 * c + li];
          a[rt][NT - 1][r] = lastok ? (CT)ar[lastc] : zero;
          if (!rok) {
#pragma unroll
            for (int c = 0; c < NT; ++c) a[rt][c][r] = zero;
          }
        }
    }
    CT* Vb = Vg + blk * (int64_t)WB * LDV;
    CT* Tb = Tg + blk * (int64_t)NT * 256;
    CT* Zb = Zg + blk * (int64_t)(NPAIR > 0 ? NPAIR : 1) * 256;

    for (int p = 0; p < NT && 16 * p < n; ++p) {
      // ---- panel p: copy its tiles out of a[][][]
      CT pa[2][4];
#pragma unroll
      for (int rt = 0; rt < 2; ++rt)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          CT v = zero;
#pragma unroll
          for (int c = 0; c < NT; ++c) v = (c == p) ? a[rt][c][r] : v;
          pa[rt][r] = v;
        }
      // the panel's diagonal R tile in result layout, updated identically in every wave
      CT rd[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) rd[r] = sh.R[utile(p, p, NT)][r][lane];

      static_for<0, 16>([&](auto jc) {
        constexpr int j = decltype(jc)::value;
        if (16 * p + j >= n) return;  // uniform: every later column is past n too
        // column j of the panel, broadcast to the 16 lanes of each row
        CT xj[2][4];
#pragma unroll
        for (int rt = 0; rt < 2; ++rt)
#pragma unroll
          for (int r = 0; r < 4; ++r) xj[rt][r] = row_bcast<j>(pa[rt][r]);
        CT d0 = zero, d1 = zero;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          d0 = fma(xj[0][r], pa[0][r], d0);
          d1 = fma(xj[1][r], pa[1][r], d1);
        }
        const CT d = pair_sum32(pair_sum16(d0 + d1));
        if (g == 0) sh.slot[j & 1][wave][li] = d;
        constexpr int jr = L::reg_of(j), jg = L::grp_of(j);
        const CT Rj = row_to_all<jg>(rd[jr]);  // R[16p+j][16p+li]
        __syncthreads();
        // D(li) = sum over the block rows of x_j * x_li (fixed order)
        const CT D = (sh.slot[j & 1][0][li] + sh.slot[j & 1][1][li]) +
                     (sh.slot[j & 1][2][li] + sh.slot[j & 1][3][li]);
        const CT Dj = row_bcast<j>(D);
        const CT alpha = row_bcast<j>(Rj);
        CT tau, beta, scale;
        householder(alpha, Dj, beta, tau, scale);
        // x_li -= tau (y_j^T x_li) y_j for li > j; column j becomes v_j = scale x_j
        const CT w = tau * fma(D, scale, Rj);
        const CT c1 = (li == j) ? scale : one;
        const CT c2 = (li > j) ? -w * scale : zero;
#pragma unroll
        for (int rt = 0; rt < 2; ++rt)
#pragma unroll
          for (int r = 0; r < 4; ++r) pa[rt][r] = fma(c2, xj[rt][r], pa[rt][r] * c1);
        if (g == jg) rd[jr] = (li == j) ? beta : (li > j ? Rj - w : Rj);
        if (wave == 0 && g == 0) {
          sh.ZT[li][j] = scale * D;  // v_li^T v_j, used for li < j
          if (li == j) sh.tau[j] = tau;
        }
      });
      // ---- panel done: V_p into a[][][]
#pragma unroll
      for (int rt = 0; rt < 2; ++rt)
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
          for (int c = 0; c < NT; ++c) a[rt][c][r] = (c == p) ? pa[rt][r] : a[rt][c][r];
      if (wave == 0) {
        // diagonal R tile back; T_p over ZT by the forward recurrence
        //   T[i][j] = -tau_j sum_{i<=k<j} T[i][k] (v_k^T v_j),  T[j][j] = tau_j
        // (lane li computes row li); columns past n were never stepped and are zero.
        const int nj = n - 16 * p < 16 ? n - 16 * p : 16;
#pragma unroll
        for (int r = 0; r < 4; ++r) sh.R[utile(p, p, NT)][r][lane] = rd[r];
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        // float64: ZT and tau through a base address held in a vector register, so the reads
        // below use constant offsets (with the constant shared-memory addresses the compiler
        // builds every one of the 136 addresses separately, out of spilled scalars).  In
        // float32 the register pressure elsewhere is such that this measured slower.
        using Sh = WyShared<CT, NT>;
        static_assert(offsetof(Sh, tau) == offsetof(Sh, ZT) + 256 * sizeof(CT),
                      "tau must follow ZT");
        const CT* zt = &sh.ZT[0][0];
        if constexpr (sizeof(CT) == 8) asm volatile("" : "+v"(zt));
        CT trow[16];
#pragma unroll
        for (int j = 0; j < 16; ++j) {
          CT t = zero;
#pragma unroll
          for (int k = 0; k < j; ++k) t = fma(trow[k], zt[16 * k + j], t);
          const CT tj = zt[256 + j];  // tau follows ZT
          trow[j] = (j >= nj) ? zero : (li < j) ? -tj * t : (li == j ? tj : zero);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        if (g == 0) {
#pragma unroll
          for (int k = 0; k < 16; ++k) {
            sh.ZT[li][k] = trow[k];
            Tb[(int64_t)p * 256 + li * 16 + opos<CT>(k)] = trow[k];
          }
        }
      }
      // ---- V_p transposed to the operand layout through this wave's part[] area (16 x 16
      // tiles, column index XOR-swizzled by the row), then stored
      CT vt[2][4];
      {
        CT* buf = &sh.part[wave][0][0][0];
#pragma unroll
        for (int rt = 0; rt < 2; ++rt)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int row = L::row(r, g);
            buf[rt * 256 + row * 16 + (li ^ row)] = pa[rt][r];
          }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
        for (int rt = 0; rt < 2; ++rt)
#pragma unroll
          for (int s = 0; s < 4; ++s) vt[rt][s] = buf[rt * 256 + li * 16 + (L::row(s, g) ^ li)];
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        __builtin_amdgcn_wave_barrier();
      }
#pragma unroll
      for (int rt = 0; rt < 2; ++rt) {
        CT* vr = Vb + (int64_t)(32 * wave + 16 * rt + li) * LDV + 16 * p + 4 * g;
#pragma unroll
        for (int s = 0; s < 4; ++s) vr[s] = vt[rt][s];
      }

      // ---- contractions W = V_p^T X_c (c != p) in rounds of WCH tiles; each round ends
      // with the update X_c += V_p (-T_p^T W_c) of its trailing tiles
      int slot_i = 0;
#pragma unroll
      for (int c = 0; c < NT; ++c) {
        if (c == p) continue;
        const int k = slot_i % WCH;
        {
          v4 acc = {zero, zero, zero, zero};
#pragma unroll
          for (int rt = 0; rt < 2; ++rt)
#pragma unroll
            for (int s = 0; s < 4; ++s) acc = L::mma(pa[rt][s], a[rt][c][s], acc);
#pragma unroll
          for (int r = 0; r < 4; ++r) sh.part[wave][k][r][lane] = acc[r];
        }
        ++slot_i;
        const bool last = (c == NT - 1) || (c == NT - 2 && p == NT - 1);
        if (k == WCH - 1 || last) {
          const int nk = k + 1;            // tiles in this round
          const int first = slot_i - nk;   // index (among c != p) of the round's first tile
          __syncthreads();
          if (wave < nk) {
            const int sidx = first + wave;
            const int cc = sidx < p ? sidx : sidx + 1;  // the tile it stands for
            v4 sum;
#pragma unroll
            for (int r = 0; r < 4; ++r)
              sum[r] = (sh.part[0][wave][r][lane] + sh.part[1][wave][r][lane]) +
                       (sh.part[2][wave][r][lane] + sh.part[3][wave][r][lane]);
            if (cc > p) {
              // W = R_pc + V_p^T X_c;  W' = T_p^T W;  R_pc -= W';  Wbr = -W'
              const int ti = utile(p, cc, NT);
#pragma unroll
              for (int r = 0; r < 4; ++r) sum[r] += sh.R[ti][r][lane];
              v4 wp = {zero, zero, zero, zero};
#pragma unroll
              for (int s = 0; s < 4; ++s) wp = L::mma(sh.ZT[L::row(s, g)][li], sum[s], wp);
#pragma unroll
              for (int r = 0; r < 4; ++r) {
                sh.R[ti][r][lane] -= wp[r];
                sh.Wbr[wave][r][lane] = -wp[r];
              }
            } else {
              // sum = V_p^T V_cc = Z_{cc,p}^T: Z[li][row(r, g)] is register r, stored at the
              // operand-permuted position 4g + r of row li
              CT* zt = Zb + (int64_t)upair(cc, p, NT) * 256 + li * 16 + 4 * g;
#pragma unroll
              for (int r = 0; r < 4; ++r) zt[r] = sum[r];
            }
          }
          __syncthreads();
#pragma unroll
          for (int c2 = 0; c2 < NT; ++c2) {
            if (c2 <= p) continue;
            const int s2 = c2 - 1;  // index of c2 among c != p (c2 > p)
            if (s2 < first || s2 >= slot_i) continue;
            CT wb[4];
#pragma unroll
            for (int s = 0; s < 4; ++s) wb[s] = sh.Wbr[s2 - first][s][lane];
#pragma unroll
            for (int rt = 0; rt < 2; ++rt) {
              v4 acc = {a[rt][c2][0], a[rt][c2][1], a[rt][c2][2], a[rt][c2][3]};
#pragma unroll
              for (int s = 0; s < 4; ++s) acc = L::mma(vt[rt][s], wb[s], acc);
#pragma unroll
              for (int r = 0; r < 4; ++r) a[rt][c2][r] = acc[r];
            }
          }
        }
      }
    }
  }
  __syncthreads();
  // ---- the chain's R, row-major n x n, float64
  double* Ro = Rw + (int64_t)blockIdx.x * n * n;
  for (int i = tid; i < n * n; i += WTHREADS) {
    const int row = i / n, col = i - row * n;
    double v = 0.0;
    if (col >= row) {
      const int p = row >> 4, c = col >> 4, rr = row & 15, cc = col & 15;
      v = (double)sh.R[utile(p, c, NT)][L::reg_of(rr)][cc + 16 * L::grp_of(rr)];
    }
    Ro[i] = v;
  }
}

// Apply: one workgroup of 8 waves per leaf chain, blocks from the chain's last to its
// first.  The seed S (n x k, k <= n, row-major, float64) of the chain comes from the merge
// tree.  Per block, two phases:
//   1. W = T S by the panel recurrence W_p = T_p (S_p - sum_{q>p} Z_pq W_q): wave c
//      (c < ceil(k/16)) takes output columns 16c .. 16c+15 and keeps its seed tiles in
//      registers (S <- S - W afterwards).  A W tile in result layout is, lane for lane, the
//      B operand of the product below, so it goes to the local data share as it stands.
//   2. The block's rows of U = -V W: wave t takes rows 16t .. 16t+15 (each row of V read
//      once, as A operands) and all output tiles, W read from the local data share.
// The wave's V rows are loaded before phase 1, so their latency hides behind it.  With ZS
// (when it fits) the block's T_p and Z_cp tiles are staged in the local data share too:
// the next block's are copied in at the end of phase 2, so the recurrence reads no global
// memory.
constexpr int WA_WAVES = WB / 16;  // 8: one row tile per wave in phase 2
template <typename CT, int NT>
constexpr size_t wa_lds(bool zs) {
  return ((size_t)NT * NT + (zs ? (size_t)NT * (NT + 1) / 2 : 0)) * 256 * sizeof(CT);
}
template <typename CT, int NT>
constexpr bool wa_zs() { return wa_lds<CT, NT>(true) <= 160 * 1024; }

template <typename CT, int NT, typename OT, bool ZS>
__global__ __launch_bounds__(64 * WA_WAVES) void k_wy_apply(
    const CT* __restrict__ Vg, const CT* __restrict__ Tg, const CT* __restrict__ Zg,
    const double* __restrict__ Sw, int n, int k, int bpw, int64_t nblocks, int64_t m,
    OT* __restrict__ out, int64_t ldo, const int* __restrict__ gate) {
  using L = Wy<CT>;
  using v4 = typename L::v4;
  if (gate && *gate == 0) return;
  constexpr int NPAIR = NT * (NT - 1) / 2;
  constexpr int NZT = NPAIR + NT;  // staged tiles: the Z_cp pairs, then T_0 .. T_{NT-1}
  extern __shared__ __attribute__((aligned(16))) char wa_smem[];
  // [q][J][s][lane] = W[16q + row(s, g)][16J + i]
  CT* Wl = reinterpret_cast<CT*>(wa_smem);
  CT* ZTl = Wl + NT * NT * 256;  // ZS: the block's Z_cp then T_p tiles (global layout)
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, g = lane >> 4;
  constexpr int LDV = 16 * NT;
  const CT zero = CT(0);
  const int np = (n + 15) >> 4;   // panels in use
  const int ncw = (k + 15) >> 4;  // output column tiles (<= np)
  const bool cwave = wave < ncw;
  const int col = 16 * wave + li;
  // seed tile q of a column wave, result layout: s[q][r] = S[16q + row(r, g)][col]
  CT s[NT][4];
  const double* S = Sw + (int64_t)blockIdx.x * n * k;
#pragma unroll
  for (int q = 0; q < NT; ++q)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = 16 * q + L::row(r, g);
      s[q][r] = (cwave && col < k && row < n) ? (CT)S[(int64_t)row * k + col] : zero;
    }
  const int64_t b0 = (int64_t)blockIdx.x * bpw;
  const int64_t b1 = (b0 + bpw < nblocks) ? b0 + bpw : nblocks;
  // ZS: the next block's tiles are loaded into registers at the start of a block and put
  // into the local data share after its phase 2 (one memory latency per block, hidden
  // behind the block's work, instead of one per staged element)
  constexpr int ZPT = (NZT * 256 + 64 * WA_WAVES - 1) / (64 * WA_WAVES);
  CT zreg[ZS ? ZPT : 1];
  auto fetch_zt = [&](int64_t blk) {
    const CT* Zb = Zg + blk * (int64_t)(NPAIR > 0 ? NPAIR : 1) * 256;
    const CT* Tb = Tg + blk * (int64_t)NT * 256;
#pragma unroll
    for (int u = 0; u < ZPT; ++u) {
      int i = tid + 64 * WA_WAVES * u;
      i = i < NZT * 256 ? i : NZT * 256 - 1;
      zreg[u] = *((i < NPAIR * 256) ? Zb + i : Tb + (i - NPAIR * 256));
    }
  };
  auto put_zt = [&]() {
#pragma unroll
    for (int u = 0; u < ZPT; ++u) {
      const int i = tid + 64 * WA_WAVES * u;
      if (i < NZT * 256) ZTl[i] = zreg[u];
    }
  };
  if constexpr (ZS) {
    if (b1 > b0) {
      fetch_zt(b1 - 1);
      put_zt();
    }
    __syncthreads();
  }
  // every load so far has landed: the compiler's wait counts inside the block loop then
  // track only that loop's own loads (otherwise the seed loads above, on the path that skips
  // the staging, make it wait for each block's V rows before phase 1)
  __builtin_amdgcn_s_waitcnt(0);
  for (int64_t blk = b1 - 1; blk >= b0; --blk) {
    const CT* Vb = Vg + blk * (int64_t)WB * LDV;
    const CT* Zb = ZS ? ZTl : Zg + blk * (int64_t)(NPAIR > 0 ? NPAIR : 1) * 256;
    const CT* Tb = ZS ? ZTl + NPAIR * 256 : Tg + blk * (int64_t)NT * 256;
    // this wave's rows of V (phase 2), as A operands: row 16 wave + i, 16-column group q.
    // All NT groups are loaded, with no condition (a row holds 16 NT elements); groups
    // q >= np are never used.  Then the next block's staged tiles, after them: waiting for
    // these rows in phase 2 does not wait for those.
    CT va[NT][4];
    {
      // rows of V are 16-byte aligned (the workspace is, and a row is 16 NT elements)
      const CT* vr = Vb + (int64_t)(16 * wave + li) * LDV + 4 * g;
#pragma unroll
      for (int q = 0; q < NT; ++q) load4_aligned(vr + 16 * q, va[q]);
    }
    if constexpr (ZS) fetch_zt(blk > b0 ? blk - 1 : blk);  // no branch: the last is unused
    // ---- phase 1: W = T S, last panel first.  Each W_q, once formed, is pushed at once into
    // the sums of the panels before it (acc_q' -= Z_q'q W_q, independent accumulators), so
    // the dependent chain is one panel's T product and one Z product per step instead of
    // all of a panel's Z products.  Tiles of W past the panels in use are never read.
    if (cwave) {
      CT ac[NT][4];
#pragma unroll
      for (int q = 0; q < NT; ++q)
#pragma unroll
        for (int r = 0; r < 4; ++r) ac[q][r] = s[q][r];
#pragma unroll
      for (int q = NT - 1; q >= 0; --q) {
        if (q >= np) continue;
        const CT* tr = Tb + q * 256 + li * 16 + 4 * g;
        v4 wv = {zero, zero, zero, zero};
#pragma unroll
        for (int t = 0; t < 4; ++t) wv = L::mma(tr[t], ac[q][t], wv);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          Wl[((q * NT + wave) * 4 + r) * 64 + lane] = wv[r];
          s[q][r] -= wv[r];
        }
#pragma unroll
        for (int q2 = 0; q2 < q; ++q2) {
          const CT* zr = Zb + upair(q2, q, NT) * 256 + li * 16 + 4 * g;
          v4 a = {ac[q2][0], ac[q2][1], ac[q2][2], ac[q2][3]};
#pragma unroll
          for (int t = 0; t < 4; ++t) a = L::mma(-zr[t], wv[t], a);
#pragma unroll
          for (int r = 0; r < 4; ++r) ac[q2][r] = a[r];
        }
      }
    }
    __syncthreads();
    // ---- phase 2: rows 16 wave .. 16 wave + 15 of U = -V W
    const int64_t row0 = blk * WB + 16 * wave;
    if (row0 < m) {
      // unrolled (a loop here would make the compiler wait for the staged tiles' loads too,
      // at its entry)
#pragma unroll
      for (int J = 0; J < NT; ++J) {
        if (J >= ncw) break;
        v4 u = {zero, zero, zero, zero};
#pragma unroll
        for (int q = 0; q < NT; ++q) {
          if (q >= np) continue;
          const CT* wl = Wl + (q * NT + J) * 256 + lane;
#pragma unroll
          for (int t = 0; t < 4; ++t) u = L::mma(va[q][t], wl[64 * t], u);
        }
        const int c = 16 * J + li;
        if (c < k) {
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int64_t row = row0 + L::row(r, g);
            if (row < m) out[row * ldo + c] = (OT)(-u[r]);
          }
        }
      }
    }
    if constexpr (ZS) {
      if (blk > b0) put_zt();  // phase 1 of this block has read the staged tiles
    }
    __syncthreads();  // before the next block's phase 1 reads them and overwrites W
  }
}

// ------------------------------------------------------------------------- host side

size_t wy_block_elems(int nt) {
  return (size_t)WB * 16 * nt + (size_t)nt * 256 + (size_t)(nt > 1 ? nt * (nt - 1) / 2 : 1) * 256;
}

template <typename CT, int NT>
static hipError_t wy_factor_launch(const TsqrPlan& p, const void* A, int a_dtype, int64_t lda,
                                   hipStream_t s) {
  const size_t lds = wy_factor_lds<CT, NT>();
  static bool attr[2] = {false, false};
  const int di = a_dtype == TSSVD_F64 ? 0 : 1;
  if (!attr[di]) {
    hipError_t e = (di == 0)
        ? hipFuncSetAttribute((const void*)k_wy_factor<CT, NT, double>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds)
        : hipFuncSetAttribute((const void*)k_wy_factor<CT, NT, float>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    attr[di] = true;
  }
  CT* V = (CT*)p.Vwy;
  CT* T = (CT*)p.Twy;
  CT* Z = (CT*)p.Zwy;
  if (a_dtype == TSSVD_F64)
    hipLaunchKernelGGL((k_wy_factor<CT, NT, double>), dim3(p.W), dim3(WTHREADS), lds, s,
                       (const double*)A, lda, p.m, p.n, p.bpw, p.nblocks, V, T, Z, p.Rlev[0],
                       p.gate);
  else
    hipLaunchKernelGGL((k_wy_factor<CT, NT, float>), dim3(p.W), dim3(WTHREADS), lds, s,
                       (const float*)A, lda, p.m, p.n, p.bpw, p.nblocks, V, T, Z, p.Rlev[0],
                       p.gate);
  return hipGetLastError();
}

template <typename CT, int NT, typename OT>
static hipError_t wy_apply_launch(const TsqrPlan& p, const double* S0, int k, OT* out,
                                  int64_t ldo, hipStream_t s) {
  constexpr bool ZS = wa_zs<CT, NT>();
  const size_t lds = wa_lds<CT, NT>(ZS);
  static bool attr = false;
  if (!attr) {
    hipError_t e = hipFuncSetAttribute((const void*)k_wy_apply<CT, NT, OT, ZS>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    attr = true;
  }
  hipLaunchKernelGGL((k_wy_apply<CT, NT, OT, ZS>), dim3(p.W), dim3(64 * WA_WAVES), lds, s,
                     (const CT*)p.Vwy, (const CT*)p.Twy, (const CT*)p.Zwy, S0, p.n, k,
                     p.bpw, p.nblocks, p.m, out, ldo, p.gate);
  return hipGetLastError();
}

template <typename CT>
static hipError_t wy_factor_ct(const TsqrPlan& p, const void* A, int a_dtype, int64_t lda,
                               hipStream_t s) {
  switch (p.ntw) {
    case 3: return wy_factor_launch<CT, 3>(p, A, a_dtype, lda, s);
    case 4: return wy_factor_launch<CT, 4>(p, A, a_dtype, lda, s);
    case 5: return wy_factor_launch<CT, 5>(p, A, a_dtype, lda, s);
    case 6: return wy_factor_launch<CT, 6>(p, A, a_dtype, lda, s);
    case 7: return wy_factor_launch<CT, 7>(p, A, a_dtype, lda, s);
    case 8: return wy_factor_launch<CT, 8>(p, A, a_dtype, lda, s);
    default: return hipErrorInvalidValue;
  }
}

template <typename CT, typename OT>
static hipError_t wy_apply_ct(const TsqrPlan& p, const double* S0, int k, OT* out, int64_t ldo,
                              hipStream_t s) {
  if (k < 1 || k > 16 * p.ntw) return hipErrorInvalidValue;  // W holds ntw x ntw tiles
  switch (p.ntw) {
    case 3: return wy_apply_launch<CT, 3>(p, S0, k, out, ldo, s);
    case 4: return wy_apply_launch<CT, 4>(p, S0, k, out, ldo, s);
    case 5: return wy_apply_launch<CT, 5>(p, S0, k, out, ldo, s);
    case 6: return wy_apply_launch<CT, 6>(p, S0, k, out, ldo, s);
    case 7: return wy_apply_launch<CT, 7>(p, S0, k, out, ldo, s);
    case 8: return wy_apply_launch<CT, 8>(p, S0, k, out, ldo, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t wy_factor(const TsqrPlan& p, const void* A, int a_dtype, int64_t lda, hipStream_t s) {
  return p.wyf32 ? wy_factor_ct<float>(p, A, a_dtype, lda, s)
                 : wy_factor_ct<double>(p, A, a_dtype, lda, s);
}

hipError_t wy_apply(const TsqrPlan& p, const double* S0, int k, double* out, int64_t ldo,
                    hipStream_t s) {
  return p.wyf32 ? wy_apply_ct<float>(p, S0, k, out, ldo, s)
                 : wy_apply_ct<double>(p, S0, k, out, ldo, s);
}

}  // namespace tsv
