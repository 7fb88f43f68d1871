// Blocked (compact WY) TSQR leaf for 33 <= n <= 128 on gfx950 FP64 matrix cores.
//
// Method (Algorithm 1 step 2; Section 2's reduction): a workgroup walks its row blocks A_t
// (256 rows) in order, carrying the triangular factor R of the rows seen so far, and
// factors the stacked matrix [R; A_t] by Householder reflectors.  Reflector j touches row j
// of R and the block rows only, so its vector is y_j = [e_j; v_j] and it is stored as the
// block part v_j.  The n reflectors are taken 16 at a time (a panel p of columns
// 16p .. 16p+15): the panel's reflectors are formed one column at a time, then they are
// applied to the other columns at once in compact WY form,
//   H_{16p} ... H_{16p+15} = I - Y_p T_p Y_p^T   (T_p 16 x 16 upper triangular),
// as two products on the matrix cores: W = Y_p^T X (a contraction over the 256 block rows)
// and X -= Y_p (T_p^T W).  The same contraction against the panels already done gives
// Z_cp = V_c^T V_p (c < p); with the T_p these determine the block's whole reflector product
// Q_t = I - Y T Y^T, T = [T_c, T_cp; 0, T_p], T_cp = -T_c Z_cp T_p (the usual forward
// accumulation), which the apply pass uses without forming T.
//
// Apply pass (U = Q [S; 0] for a seed S from the merge tree): Q_t [S; 0] = [S - W; -V W]
// with W = T S, and W is found panel by panel from the last one back,
//   W_p = T_p (S_p - sum_{q > p} Z_pq W_q),
// so each block costs a small n x n x k recurrence plus one 256 x n x k product that
// writes the block's rows of U; the seed of the block before is S - W.
//
// Matrix-core layout (v_mfma_f64_16x16x4_f64, measured): lane (i = lane%16, g = lane/16);
// A operand a[i][k=g], B operand b[k=g][j=i]; result register r holds D[4r+g][i].  A
// 16 x 16 tile "in result layout" is held as 4 registers per lane, register r = row 4r+g,
// column i.  A contraction over the rows of two such tiles needs no data movement: in the
// s-th instruction lane (i, g) supplies row 4s+g of both.  Tiles read as A operands from
// memory are stored "operand-permuted": row i keeps its 16 entries at positions 4g+s for
// column 4s+g, so a lane loads its four k values as one 32-byte vector.
#include <type_traits>

#include "common.h"
#include "internal.h"

namespace tsv {

namespace {

typedef double f64x4 __attribute__((ext_vector_type(4)));

constexpr int WB = 128;       // rows per block
constexpr int WWAVES = 4;     // waves per workgroup, 32 rows (two 16-row tiles) each
constexpr int WTHREADS = 64 * WWAVES;

__device__ __forceinline__ f64x4 mfma64(double a, double b, f64x4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ double shfl_d(double x, int src_lane) {
  const int addr = src_lane << 2;
  const int lo = __builtin_amdgcn_ds_bpermute(addr, __double2loint(x));
  const int hi = __builtin_amdgcn_ds_bpermute(addr, __double2hiint(x));
  return __hiloint2double(hi, lo);
}

// x + x[lane ^ 16] and x + x[lane ^ 32], through the row-swap instructions: after the swap
// the two registers hold the values of both rows of each pair, and their sum has the same
// operand order in both rows, so the partner lanes get bitwise-equal sums.
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
__device__ __forceinline__ double row_to_all(double x) {
  return __hiloint2double((int)row_to_all_u<G>((unsigned)__double2hiint(x)),
                          (int)row_to_all_u<G>((unsigned)__double2loint(x)));
}

// x from lane j of this lane's 16-lane row (DPP row broadcast).
template <int J>
__device__ __forceinline__ double row_bcast(double x) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), 0x150 + J, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), 0x150 + J, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

// Reflector of (alpha, x) with ||x||^2 = s: beta = -sign(alpha) sqrt(alpha^2 + s),
// tau = (beta - alpha) / beta, scale = 1 / (alpha - beta) (v = scale x); s = 0 gives the
// identity (tau = 0, beta = alpha, scale = 0).  Written with the hardware reciprocal square
// root and reciprocal, each refined by two Newton steps (relative error a few units in the
// last place), and |beta - alpha| = |alpha| + nrm, so tau = (|alpha| + nrm) / nrm; the
// operands of the rsq and rcp stay finite and non-zero for any finite input.
__device__ __forceinline__ void householder(double alpha, double s, double& beta, double& tau,
                                            double& scale) {
  const bool live = s > 0.0;
  const double q = fma(alpha, alpha, s);
  const double qq = live ? q : 1.0;
  double rs = __builtin_amdgcn_rsq(qq);
  rs = rs * fma(-0.5 * qq * rs, rs, 1.5);
  rs = rs * fma(-0.5 * qq * rs, rs, 1.5);
  const double nrm = qq * rs;
  const double gam = fabs(alpha) + nrm;  // |alpha - beta|
  double rg = __builtin_amdgcn_rcp(gam);
  rg = rg * fma(-gam, rg, 2.0);
  rg = rg * fma(-gam, rg, 2.0);
  const double b = alpha >= 0.0 ? -nrm : nrm;
  beta = live ? b : alpha;
  tau = live ? gam * rs : 0.0;
  scale = live ? (alpha >= 0.0 ? rg : -rg) : 0.0;
}

// f(integral_constant<int, I>) for I = B .. E-1, at compile time
template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}

// Index of the upper tile (p, c), p <= c, in the packed tile list of an NT x NT grid.
__host__ __device__ constexpr int utile(int p, int c, int nt) { return p * nt - p * (p - 1) / 2 + (c - p); }
// Index of the strictly upper pair (c, q), c < q.
__host__ __device__ constexpr int upair(int c, int q, int nt) { return c * nt - c * (c + 1) / 2 + (q - c - 1); }
// operand-permuted position of column k within its 16-column group
__host__ __device__ constexpr int opos(int k) { return 4 * (k & 3) + (k >> 2); }

// Column tiles per contraction round (partials staged in the local data share).  With
// n <= 112 the shared state stays under 80 KB, so two workgroups share a CU and each hides
// the other's barrier waits and block loads.
template <int NT>
constexpr int wch() { return NT <= 4 ? NT - 1 : 2; }

template <int NT>
struct WyShared {
  double R[NT * (NT + 1) / 2][4][64];  // carried factor, upper tiles in result layout
  double part[WWAVES][wch<NT>()][4][64];  // per-wave partial contractions (V transposes first)
  double Wbr[wch<NT>()][4][64];        // -T_p^T W of the round's tiles
  double slot[2][WWAVES][16];          // per-wave partial column dots (panel steps)
  double ZT[16][16];                   // v_k^T v_j (k < j) of the panel, then T_p (row-major)
  double tau[16];
};

}  // namespace

template <int NT>
size_t wy_factor_lds() { return sizeof(WyShared<NT>); }

// One leaf chain per workgroup: blocks [blockIdx.x*bpw, ...).  Outputs per block: V
// (128 x 16NT, operand-permuted rows), T_p (NT tiles, operand-permuted), Z_cp (pairs c < p,
// operand-permuted); per workgroup the final R (n x n row-major, zero below the diagonal).
template <int NT, typename TA>
__global__ __launch_bounds__(WTHREADS, 2) void k_wy_factor(
    const TA* __restrict__ A, int64_t lda, int64_t m, int n, int bpw, int64_t nblocks,
    double* __restrict__ Vg, double* __restrict__ Tg, double* __restrict__ Zg,
    double* __restrict__ Rw, const int* __restrict__ gate) {
  if (gate && *gate == 0) return;
  extern __shared__ __attribute__((aligned(16))) char wy_smem[];
  WyShared<NT>& sh = *reinterpret_cast<WyShared<NT>*>(wy_smem);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, g = lane >> 4;
  constexpr int NTT = NT * (NT + 1) / 2;
  constexpr int NPAIR = NT * (NT - 1) / 2;
  constexpr int LDV = 16 * NT;
  constexpr int WCH = wch<NT>();
  static_assert(WCH * 256 >= 512, "a wave's part[] area must hold its two 16 x 16 tiles");

  for (int i = tid; i < NTT * 256; i += WTHREADS) (&sh.R[0][0][0])[i] = 0.0;
  __syncthreads();

  const int64_t b0 = (int64_t)blockIdx.x * bpw;
  const int64_t b1 = (b0 + bpw < nblocks) ? b0 + bpw : nblocks;
  for (int64_t blk = b0; blk < b1; ++blk) {
    // ---- load the block: a[rt][c][r] = A[row0 + 32 wave + 16 rt + 4 r + g][16 c + li]
    double a[2][NT][4];
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
          const int64_t row = rbase + 16 * rt + 4 * r + g;
          const bool rok = row < m;
          const TA* ar = A + (rok ? row : m - 1) * lda;
#pragma unroll
          for (int c = 0; c < NT - 1; ++c) a[rt][c][r] = (double)ar[16 * c + li];
          a[rt][NT - 1][r] = lastok ? (double)ar[lastc] : 0.0;
          if (!rok) {
#pragma unroll
            for (int c = 0; c < NT; ++c) a[rt][c][r] = 0.0;
          }
        }
    }
    double* Vb = Vg + blk * (int64_t)WB * LDV;
    double* Tb = Tg + blk * (int64_t)NT * 256;
    double* Zb = Zg + blk * (int64_t)(NPAIR > 0 ? NPAIR : 1) * 256;

    for (int p = 0; p < NT && 16 * p < n; ++p) {
      // ---- panel p: copy its tiles out of a[][][]
      double pa[2][4];
#pragma unroll
      for (int rt = 0; rt < 2; ++rt)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          double v = 0.0;
#pragma unroll
          for (int c = 0; c < NT; ++c) v = (c == p) ? a[rt][c][r] : v;
          pa[rt][r] = v;
        }
      // the panel's diagonal R tile in result layout (register r: row 4r+g, column li),
      // updated identically in every wave
      double rd[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) rd[r] = sh.R[utile(p, p, NT)][r][lane];

      static_for<0, 16>([&](auto jc) {
        constexpr int j = decltype(jc)::value;
        if (16 * p + j >= n) return;  // uniform: every later column is past n too
        // column j of the panel, broadcast to the 16 lanes of each row
        double xj[2][4];
#pragma unroll
        for (int rt = 0; rt < 2; ++rt)
#pragma unroll
          for (int r = 0; r < 4; ++r) xj[rt][r] = row_bcast<j>(pa[rt][r]);
        double d0 = 0.0, d1 = 0.0;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          d0 = fma(xj[0][r], pa[0][r], d0);
          d1 = fma(xj[1][r], pa[1][r], d1);
        }
        const double d = pair_sum32(pair_sum16(d0 + d1));
        if (g == 0) sh.slot[j & 1][wave][li] = d;
        constexpr int jr = j >> 2, jg = j & 3;
        const double Rj = row_to_all<jg>(rd[jr]);  // R[16p+j][16p+li]
        __syncthreads();
        // D(li) = sum over the block rows of x_j * x_li (fixed order)
        const double D = (sh.slot[j & 1][0][li] + sh.slot[j & 1][1][li]) +
                         (sh.slot[j & 1][2][li] + sh.slot[j & 1][3][li]);
        const double Dj = row_bcast<j>(D);
        const double alpha = row_bcast<j>(Rj);
        double tau, beta, scale;
        householder(alpha, Dj, beta, tau, scale);
        // x_li -= tau (y_j^T x_li) y_j for li > j; column j becomes v_j = scale x_j
        const double w = tau * fma(D, scale, Rj);
        const double c1 = (li == j) ? scale : 1.0;
        const double c2 = (li > j) ? -w * scale : 0.0;
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
        // diagonal R tile back; T_p over ZT in place by the forward recurrence
        //   T[i][j] = -tau_j sum_{i<=k<j} T[i][k] (v_k^T v_j),  T[j][j] = tau_j,
        // column by column (all reads of a column before its writes); columns past n were
        // never stepped and are zero.
        const int nj = n - 16 * p < 16 ? n - 16 * p : 16;
#pragma unroll
        for (int r = 0; r < 4; ++r) sh.R[utile(p, p, NT)][r][lane] = rd[r];
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        double trow[16];
#pragma unroll
        for (int j = 0; j < 16; ++j) {
          double t = 0.0;
#pragma unroll
          for (int k = 0; k < j; ++k) t = fma(trow[k], sh.ZT[k][j], t);
          const double tj = sh.tau[j];
          trow[j] = (j >= nj) ? 0.0 : (li < j) ? -tj * t : (li == j ? tj : 0.0);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        if (g == 0) {
#pragma unroll
          for (int k = 0; k < 16; ++k) {
            sh.ZT[li][k] = trow[k];
            Tb[(int64_t)p * 256 + li * 16 + opos(k)] = trow[k];
          }
        }
      }
      // ---- V_p transposed to the operand layout through this wave's part[] area (16 x 16
      // tiles, column index XOR-swizzled by the row), then stored
      double vt[2][4];
      {
        double* buf = &sh.part[wave][0][0][0];
#pragma unroll
        for (int rt = 0; rt < 2; ++rt)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int row = 4 * r + g;
            buf[rt * 256 + row * 16 + (li ^ row)] = pa[rt][r];
          }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
        for (int rt = 0; rt < 2; ++rt)
#pragma unroll
          for (int s = 0; s < 4; ++s) vt[rt][s] = buf[rt * 256 + li * 16 + ((4 * s + g) ^ li)];
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        __builtin_amdgcn_wave_barrier();
      }
#pragma unroll
      for (int rt = 0; rt < 2; ++rt) {
        double* vr = Vb + (int64_t)(32 * wave + 16 * rt + li) * LDV + 16 * p + 4 * g;
        *reinterpret_cast<double2*>(vr) = double2{vt[rt][0], vt[rt][1]};
        *reinterpret_cast<double2*>(vr + 2) = double2{vt[rt][2], vt[rt][3]};
      }

      // ---- contractions W = V_p^T X_c (c != p) in rounds of WCH tiles; each round ends
      // with the update X_c += V_p (-T_p^T W_c) of its trailing tiles
      int slot_i = 0;
#pragma unroll
      for (int c = 0; c < NT; ++c) {
        if (c == p) continue;
        const int k = slot_i % WCH;
        {
          f64x4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
          for (int rt = 0; rt < 2; ++rt)
#pragma unroll
            for (int s = 0; s < 4; ++s) acc = mfma64(pa[rt][s], a[rt][c][s], acc);
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
            f64x4 sum = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int r = 0; r < 4; ++r)
              sum[r] = (sh.part[0][wave][r][lane] + sh.part[1][wave][r][lane]) +
                       (sh.part[2][wave][r][lane] + sh.part[3][wave][r][lane]);
            if (cc > p) {
              // W = R_pc + V_p^T X_c;  W' = T_p^T W;  R_pc -= W';  Wbr = -W'
              const int ti = utile(p, cc, NT);
#pragma unroll
              for (int r = 0; r < 4; ++r) sum[r] += sh.R[ti][r][lane];
              f64x4 wp = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
              for (int s = 0; s < 4; ++s) wp = mfma64(sh.ZT[4 * s + g][li], sum[s], wp);
#pragma unroll
              for (int r = 0; r < 4; ++r) {
                sh.R[ti][r][lane] -= wp[r];
                sh.Wbr[wave][r][lane] = -wp[r];
              }
            } else {
              // sum = V_p^T V_cc = Z_{cc,p}^T: Z[li][4r+g] is register r; store row li
              double* zt = Zb + (int64_t)upair(cc, p, NT) * 256 + li * 16;
#pragma unroll
              for (int r = 0; r < 4; ++r) zt[opos(4 * r + g)] = sum[r];
            }
          }
          __syncthreads();
#pragma unroll
          for (int c2 = 0; c2 < NT; ++c2) {
            if (c2 <= p) continue;
            const int s2 = c2 - 1;  // index of c2 among c != p (c2 > p)
            if (s2 < first || s2 >= slot_i) continue;
            double wb[4];
#pragma unroll
            for (int s = 0; s < 4; ++s) wb[s] = sh.Wbr[s2 - first][s][lane];
#pragma unroll
            for (int rt = 0; rt < 2; ++rt) {
              f64x4 acc = {a[rt][c2][0], a[rt][c2][1], a[rt][c2][2], a[rt][c2][3]};
#pragma unroll
              for (int s = 0; s < 4; ++s) acc = mfma64(vt[rt][s], wb[s], acc);
#pragma unroll
              for (int r = 0; r < 4; ++r) a[rt][c2][r] = acc[r];
            }
          }
        }
      }
    }
    // panels past n (n < 16 NT) do not exist: NT = ceil(n / 16)
  }
  __syncthreads();
  // ---- the chain's R, row-major n x n
  double* Ro = Rw + (int64_t)blockIdx.x * n * n;
  for (int i = tid; i < n * n; i += WTHREADS) {
    const int row = i / n, col = i - row * n;
    double v = 0.0;
    if (col >= row) {
      const int p = row >> 4, c = col >> 4, rr = row & 15, cc = col & 15;
      // result layout: register (rr >> 2), lane (cc + 16 (rr & 3))
      v = sh.R[utile(p, c, NT)][rr >> 2][cc + 16 * (rr & 3)];
    }
    Ro[i] = v;
  }
}

// Apply: one workgroup per leaf chain, one wave per 16-column tile of the output (k
// columns).  The seed S (n x k, row-major) of the chain comes from the merge tree.
template <int NT>
__global__ __launch_bounds__(64 * 8) void k_wy_apply(
    const double* __restrict__ Vg, const double* __restrict__ Tg, const double* __restrict__ Zg,
    const double* __restrict__ Sw, int n, int k, int bpw, int64_t nblocks, int64_t m,
    double* __restrict__ out, int64_t ldo, const int* __restrict__ gate) {
  if (gate && *gate == 0) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, g = lane >> 4;
  constexpr int NPAIR = NT * (NT - 1) / 2;
  constexpr int LDV = 16 * NT;
  const int np = (n + 15) >> 4;  // panels in use
  const int col = 16 * wave + li;
  const bool cok = col < k;
  // seed tile q, result layout: s[q][r] = S[16q + 4r + g][col]
  double s[NT][4];
  const double* S = Sw + (int64_t)blockIdx.x * n * k;
#pragma unroll
  for (int q = 0; q < NT; ++q)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = 16 * q + 4 * r + g;
      s[q][r] = (cok && row < n) ? S[(int64_t)row * k + col] : 0.0;
    }
  const int64_t b0 = (int64_t)blockIdx.x * bpw;
  const int64_t b1 = (b0 + bpw < nblocks) ? b0 + bpw : nblocks;
  for (int64_t blk = b1 - 1; blk >= b0; --blk) {
    const double* Vb = Vg + blk * (int64_t)WB * LDV;
    const double* Tb = Tg + blk * (int64_t)NT * 256;
    const double* Zb = Zg + blk * (int64_t)(NPAIR > 0 ? NPAIR : 1) * 256;
    // W_p = T_p (S_p - sum_{q>p} Z_pq W_q), last panel first
    double wq[NT][4];
#pragma unroll
    for (int q = NT - 1; q >= 0; --q) {
      if (q >= np) {
#pragma unroll
        for (int r = 0; r < 4; ++r) wq[q][r] = 0.0;
        continue;
      }
      f64x4 acc = {s[q][0], s[q][1], s[q][2], s[q][3]};
#pragma unroll
      for (int q2 = q + 1; q2 < NT; ++q2) {
        if (q2 >= np) continue;
        const double* zr = Zb + (int64_t)upair(q, q2, NT) * 256 + li * 16 + 4 * g;
        const double2 z0 = *reinterpret_cast<const double2*>(zr);
        const double2 z1 = *reinterpret_cast<const double2*>(zr + 2);
        acc = mfma64(-z0.x, wq[q2][0], acc);
        acc = mfma64(-z0.y, wq[q2][1], acc);
        acc = mfma64(-z1.x, wq[q2][2], acc);
        acc = mfma64(-z1.y, wq[q2][3], acc);
      }
      const double* tr = Tb + (int64_t)q * 256 + li * 16 + 4 * g;
      const double2 t0 = *reinterpret_cast<const double2*>(tr);
      const double2 t1 = *reinterpret_cast<const double2*>(tr + 2);
      f64x4 wv = {0.0, 0.0, 0.0, 0.0};
      wv = mfma64(t0.x, acc[0], wv);
      wv = mfma64(t0.y, acc[1], wv);
      wv = mfma64(t1.x, acc[2], wv);
      wv = mfma64(t1.y, acc[3], wv);
#pragma unroll
      for (int r = 0; r < 4; ++r) wq[q][r] = wv[r];
    }
    // rows of U: -V W, 16 rows per tile
    for (int rt = 0; rt < WB / 16; ++rt) {
      const int64_t row0 = blk * WB + 16 * rt;
      if (row0 >= m) break;
      f64x4 u = {0.0, 0.0, 0.0, 0.0};
      const double* vr = Vb + (int64_t)(16 * rt + li) * LDV + 4 * g;
#pragma unroll
      for (int q = 0; q < NT; ++q) {
        if (q >= np) continue;
        const double2 v0 = *reinterpret_cast<const double2*>(vr + 16 * q);
        const double2 v1 = *reinterpret_cast<const double2*>(vr + 16 * q + 2);
        u = mfma64(v0.x, wq[q][0], u);
        u = mfma64(v0.y, wq[q][1], u);
        u = mfma64(v1.x, wq[q][2], u);
        u = mfma64(v1.y, wq[q][3], u);
      }
      if (cok) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t row = row0 + 4 * r + g;
          if (row < m) out[row * ldo + col] = -u[r];
        }
      }
    }
#pragma unroll
    for (int q = 0; q < NT; ++q)
#pragma unroll
      for (int r = 0; r < 4; ++r) s[q][r] -= wq[q][r];
  }
}

// ------------------------------------------------------------------------- host side

size_t wy_block_doubles(int nt) {
  return (size_t)WB * 16 * nt + (size_t)nt * 256 + (size_t)(nt > 1 ? nt * (nt - 1) / 2 : 1) * 256;
}

template <int NT>
static hipError_t wy_factor_launch(const TsqrPlan& p, const void* A, int a_dtype, int64_t lda,
                                   hipStream_t s) {
  const size_t lds = wy_factor_lds<NT>();
  static bool attr[2] = {false, false};
  const int di = a_dtype == TSSVD_F64 ? 0 : 1;
  if (!attr[di]) {
    hipError_t e = (di == 0)
        ? hipFuncSetAttribute((const void*)k_wy_factor<NT, double>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds)
        : hipFuncSetAttribute((const void*)k_wy_factor<NT, float>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    attr[di] = true;
  }
  if (a_dtype == TSSVD_F64)
    hipLaunchKernelGGL((k_wy_factor<NT, double>), dim3(p.W), dim3(WTHREADS), lds, s,
                       (const double*)A, lda, p.m, p.n, p.bpw, p.nblocks, p.Vwy, p.Twy, p.Zwy,
                       p.Rlev[0], p.gate);
  else
    hipLaunchKernelGGL((k_wy_factor<NT, float>), dim3(p.W), dim3(WTHREADS), lds, s,
                       (const float*)A, lda, p.m, p.n, p.bpw, p.nblocks, p.Vwy, p.Twy, p.Zwy,
                       p.Rlev[0], p.gate);
  return hipGetLastError();
}

template <int NT>
static hipError_t wy_apply_launch(const TsqrPlan& p, int k, double* out, int64_t ldo,
                                  hipStream_t s) {
  const int waves = (k + 15) / 16;
  hipLaunchKernelGGL((k_wy_apply<NT>), dim3(p.W), dim3(64 * waves), 0, s, p.Vwy, p.Twy, p.Zwy,
                     p.Slev[0], p.n, k, p.bpw, p.nblocks, p.m, out, ldo, p.gate);
  return hipGetLastError();
}

hipError_t wy_factor(const TsqrPlan& p, const void* A, int a_dtype, int64_t lda, hipStream_t s) {
  switch (p.ntw) {
    case 3: return wy_factor_launch<3>(p, A, a_dtype, lda, s);
    case 4: return wy_factor_launch<4>(p, A, a_dtype, lda, s);
    case 5: return wy_factor_launch<5>(p, A, a_dtype, lda, s);
    case 6: return wy_factor_launch<6>(p, A, a_dtype, lda, s);
    case 7: return wy_factor_launch<7>(p, A, a_dtype, lda, s);
    case 8: return wy_factor_launch<8>(p, A, a_dtype, lda, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t wy_apply(const TsqrPlan& p, int k, double* out, int64_t ldo, hipStream_t s) {
  if (k < 1 || k > 128) return hipErrorInvalidValue;
  switch (p.ntw) {
    case 3: return wy_apply_launch<3>(p, k, out, ldo, s);
    case 4: return wy_apply_launch<4>(p, k, out, ldo, s);
    case 5: return wy_apply_launch<5>(p, k, out, ldo, s);
    case 6: return wy_apply_launch<6>(p, k, out, ldo, s);
    case 7: return wy_apply_launch<7>(p, k, out, ldo, s);
    case 8: return wy_apply_launch<8>(p, k, out, ldo, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace tsv
