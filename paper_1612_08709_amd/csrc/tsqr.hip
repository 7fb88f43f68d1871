// TSQR for gfx950: structured Householder QR of row blocks, a fixed binary merge tree,
// and the reverse application of the stored reflectors that forms Q explicitly.
//
// Method (Algorithm 1 step 2; Section 2's tree "reduction"): a workgroup walks its row
// blocks A_t in order, carrying the triangular factor R of everything seen so far, and
// factors the stacked matrix [R; A_t].  Reflector j acts on row j of R and on the block
// rows only (R is upper triangular), so it is stored as its block part v_j plus tau_j:
//   H_j = I - tau_j [e_j; v_j][e_j; v_j]^T,   H_{n-1} ... H_0 [R; A_t] = [R'; 0].
// The per-workgroup factors are merged by a tree with the same step: a node's carry is its
// first child's R and its block stacks the next G children's R factors (G = B / n), so
// the tree has fan-in G + 1 and few levels.  Q [S; 0] is formed top-down: every merge node
// maps its seed S to the seeds of its children, and every leaf workgroup maps its seed to
// its rows of Q by walking its blocks backwards.
//
// Register layout (256 threads): thread (rg, cg), rg = lane & 15 ("row group", one
// 16-lane DPP row), cg = (lane >> 4) + 4 * wave (column group, 0..15).  A block of
// B = 16*NR rows and n <= 16*NC columns lives in registers: thread (rg, cg) holds rows
// rg + 16 r (r < NR) and columns cg + 16 c (c < NC).  Dot products over the block rows
// are NR fused multiply-adds per thread plus a 4-stage DPP reduction inside the 16-lane
// row, so no shared memory and no barrier is needed for them.
#include "common.h"
#include "internal.h"

namespace tsv {

__device__ __forceinline__ int ts_rg() { return threadIdx.x & 15; }
__device__ __forceinline__ int ts_cg() { return ((threadIdx.x & 63) >> 4) + 4 * (threadIdx.x >> 6); }

// Packed upper-triangular storage of an n x n R: row j begins at j*n - j*(j-1)/2.
__device__ __forceinline__ int tri_off(int j, int n) { return j * n - ((j * (j - 1)) >> 1); }
__device__ __forceinline__ int tri_idx(int j, int c, int n) { return tri_off(j, n) + (c - j); }
__host__ __device__ __forceinline__ int tri_size(int n) { return n * (n + 1) / 2; }

// Structured Householder QR of [R (packed, LDS); a (block in registers)].
// On return R holds the new factor, a holds the reflector tails v_j in column j, and
// tau_lds[j] the scalars.  LAPACK sign convention: beta = -sign(alpha) * ||(alpha, x)||,
// tau = (beta - alpha) / beta, v = x / (alpha - beta); a zero tail gives H_j = I.
template <int NC, int NR>
__device__ __forceinline__ void factor_block(double (&a)[NR][NC], double* Rs, int n,
                                             double* vbuf, double* tau_lds) {
  const int rg = ts_rg(), cg = ts_cg();
  constexpr int B = 16 * NR;
#pragma unroll
  for (int jc = 0; jc < NC; ++jc) {
    for (int jr = 0; jr < 16; ++jr) {
      const int j = 16 * jc + jr;
      if (j >= n) break;
      double* vb = vbuf + (j & 1) * B;
      const int rj = tri_off(j, n) - j;  // R[j][c] = Rs[rj + c]
      if (cg == jr) {
        double s = 0.0;
#pragma unroll
        for (int r = 0; r < NR; ++r) s = fma(a[r][jc], a[r][jc], s);
        s = sum16(s);
        const double alpha = Rs[rj + j];
        double tau = 0.0, beta = alpha, scale = 0.0;
        if (s > 0.0) {
          const double nrm = sqrt(fma(alpha, alpha, s));
          beta = (alpha >= 0.0) ? -nrm : nrm;
          tau = (beta - alpha) / beta;
          scale = 1.0 / (alpha - beta);
        }
#pragma unroll
        for (int r = 0; r < NR; ++r) {
          a[r][jc] *= scale;
          vb[rg + 16 * r] = a[r][jc];
        }
        if (rg == 0) {
          tau_lds[j] = tau;
          Rs[rj + j] = beta;
        }
      }
      __syncthreads();
      const double tau = tau_lds[j];
      if (tau != 0.0) {
        double v[NR];
#pragma unroll
        for (int r = 0; r < NR; ++r) v[r] = vb[rg + 16 * r];
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          if (c < jc) continue;
          const int col = cg + 16 * c;
          if ((c == jc && cg <= jr) || col >= n) continue;
          double d = 0.0;
#pragma unroll
          for (int r = 0; r < NR; ++r) d = fma(v[r], a[r][c], d);
          const double rjc = Rs[rj + col];
          d = (sum16(d) + rjc) * tau;
#pragma unroll
          for (int r = 0; r < NR; ++r) a[r][c] = fma(-d, v[r], a[r][c]);
          if (rg == 0) Rs[rj + col] = rjc - d;
        }
      }
    }
  }
}

// y <- H_0 H_1 ... H_{n-1} applied to [S; y] (reverse order), S (n x k, row stride k) in
// LDS.  Column col of S and y is touched only by the 16-lane row that owns it, so no
// barrier is needed; the reflector column for step j-1 is fetched while step j computes.
template <int NC, int NR>
__device__ __forceinline__ void apply_block_reverse(double (&y)[NR][NC], double* Ss,
                                                    const double* __restrict__ Vb,
                                                    const double* __restrict__ taub, int n,
                                                    int k) {
  const int rg = ts_rg(), cg = ts_cg();
  constexpr int B = 16 * NR;
  double vn[NR];
  double taun = taub[n - 1];
#pragma unroll
  for (int r = 0; r < NR; ++r) vn[r] = Vb[(int64_t)(n - 1) * B + rg + 16 * r];
  for (int j = n - 1; j >= 0; --j) {
    double v[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) v[r] = vn[r];
    const double tau = taun;
    if (j > 0) {
      taun = taub[j - 1];
#pragma unroll
      for (int r = 0; r < NR; ++r) vn[r] = Vb[(int64_t)(j - 1) * B + rg + 16 * r];
    }
    if (tau == 0.0) continue;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const int col = cg + 16 * c;
      if (col >= k) continue;
      double d = 0.0;
#pragma unroll
      for (int r = 0; r < NR; ++r) d = fma(v[r], y[r][c], d);
      const double sj = Ss[j * k + col];
      d = (sum16(d) + sj) * tau;
#pragma unroll
      for (int r = 0; r < NR; ++r) y[r][c] = fma(-d, v[r], y[r][c]);
      if (rg == 0) Ss[j * k + col] = sj - d;
    }
  }
}

// ------------------------------------------------------------------------- kernels

template <int NC, int NR, typename TA>
__global__ __launch_bounds__(256) void k_leaf_factor(const TA* __restrict__ A, int64_t lda,
                                                     int64_t m, int n, int bpw,
                                                     int64_t nblocks, double* __restrict__ Vw,
                                                     double* __restrict__ tauw,
                                                     double* __restrict__ Rw,
                                                     const int* __restrict__ gate) {
  if (gate && *gate == 0) return;
  extern __shared__ double smem[];
  constexpr int B = 16 * NR;
  const int ts = tri_size(n);
  double* Rs = smem;
  double* vbuf = Rs + ts;
  double* tl = vbuf + 2 * B;
  const int tid = threadIdx.x, rg = ts_rg(), cg = ts_cg();
  for (int i = tid; i < ts; i += 256) Rs[i] = 0.0;
  __syncthreads();
  const int64_t b0 = (int64_t)blockIdx.x * bpw;
  const int64_t b1 = (b0 + bpw < nblocks) ? b0 + bpw : nblocks;
  for (int64_t blk = b0; blk < b1; ++blk) {
    const int64_t row0 = blk * B;
    double a[NR][NC];
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const int64_t row = row0 + rg + 16 * r;
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        const int col = cg + 16 * c;
        a[r][c] = (row < m && col < n) ? ld_elem(A + row * lda + col) : 0.0;
      }
    }
    factor_block<NC, NR>(a, Rs, n, vbuf, tl);
    double* Vb = Vw + blk * (int64_t)n * B;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const int col = cg + 16 * c;
      if (col < n) {
#pragma unroll
        for (int r = 0; r < NR; ++r) Vb[(int64_t)col * B + rg + 16 * r] = a[r][c];
      }
    }
    __syncthreads();
    for (int j = tid; j < n; j += 256) tauw[blk * n + j] = tl[j];
    __syncthreads();
  }
  double* Ro = Rw + (int64_t)blockIdx.x * n * n;
  for (int i = tid; i < n * n; i += 256) {
    const int r = i / n, c = i - r * n;
    Ro[i] = (c >= r) ? Rs[tri_idx(r, c, n)] : 0.0;
  }
}

// One merge node per workgroup.  Node i takes the fan = G + 1 factors first = i*fan ...:
// the first is the carry R (LDS), the next G are stacked at row offsets 0, n, 2n, ... of
// one block of B = 16*NR rows (G = B / n), so one structured factorization merges them
// all: [R_0; R_1; ...; R_G] -> R.  Missing children are zero rows; a node with no child
// beyond the first copies R_0 and records tau = 0 (identity) for the apply pass.
template <int NC, int NR>
__global__ __launch_bounds__(256) void k_tree_factor(const double* __restrict__ Rin, int nin,
                                                     int n, int G, double* __restrict__ Rout,
                                                     double* __restrict__ Vt,
                                                     double* __restrict__ taut,
                                                     const int* __restrict__ gate) {
  if (gate && *gate == 0) return;
  extern __shared__ double smem[];
  constexpr int B = 16 * NR;
  const int ts = tri_size(n);
  double* Rs = smem;
  double* vbuf = Rs + ts;
  double* tl = vbuf + 2 * B;
  const int tid = threadIdx.x, rg = ts_rg(), cg = ts_cg();
  const int node = blockIdx.x;
  const int64_t first = (int64_t)node * (G + 1);
  const double* R0 = Rin + first * n * n;
  double* Ro = Rout + (int64_t)node * n * n;
  if (first + 1 >= nin) {
    for (int i = tid; i < n * n; i += 256) Ro[i] = R0[i];
    for (int j = tid; j < n; j += 256) taut[(int64_t)node * n + j] = 0.0;
    return;
  }
  for (int i = tid; i < n * n; i += 256) {
    const int r = i / n, c = i - r * n;
    if (c >= r) Rs[tri_idx(r, c, n)] = R0[i];
  }
  double a[NR][NC];
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    const int row = rg + 16 * r;
    const int ch = row / n, lr = row - ch * n;  // child 1 + ch, its row lr
    const bool live = ch < G && first + 1 + ch < nin;
    const double* Rc = Rin + (first + 1 + ch) * n * n + (int64_t)lr * n;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const int col = cg + 16 * c;
      a[r][c] = (live && col < n) ? Rc[col] : 0.0;
    }
  }
  __syncthreads();
  factor_block<NC, NR>(a, Rs, n, vbuf, tl);
  double* Vb = Vt + (int64_t)node * n * B;
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const int col = cg + 16 * c;
    if (col < n) {
#pragma unroll
      for (int r = 0; r < NR; ++r) Vb[(int64_t)col * B + rg + 16 * r] = a[r][c];
    }
  }
  __syncthreads();
  for (int j = tid; j < n; j += 256) taut[(int64_t)node * n + j] = tl[j];
  for (int i = tid; i < n * n; i += 256) {
    const int r = i / n, c = i - r * n;
    Ro[i] = (c >= r) ? Rs[tri_idx(r, c, n)] : 0.0;
  }
}

// Seeds of one tree level from the level above: node seed S (n x k) -> the seeds of its
// children, [S_0; S_1; ...; S_G] = H_0 ... H_{n-1} [S; 0] with S_i at block rows
// (i-1)*n ... i*n-1 for i >= 1.
template <int NC, int NR>
__global__ __launch_bounds__(256) void k_tree_apply(const double* __restrict__ Sin,
                                                    int nchild, int n, int k, int G,
                                                    const double* __restrict__ Vt,
                                                    const double* __restrict__ taut,
                                                    double* __restrict__ Sout,
                                                    const int* __restrict__ gate) {
  if (gate && *gate == 0) return;
  extern __shared__ double smem[];
  constexpr int B = 16 * NR;
  double* Ss = smem;
  const int tid = threadIdx.x, rg = ts_rg(), cg = ts_cg();
  const int node = blockIdx.x;
  const int64_t first = (int64_t)node * (G + 1);
  const bool merged = first + 1 < nchild;
  const double* S = Sin + (int64_t)node * n * k;
  for (int i = tid; i < n * k; i += 256) Ss[i] = S[i];
  __syncthreads();
  double y[NR][NC];
#pragma unroll
  for (int r = 0; r < NR; ++r)
#pragma unroll
    for (int c = 0; c < NC; ++c) y[r][c] = 0.0;
  if (merged)
    apply_block_reverse<NC, NR>(y, Ss, Vt + (int64_t)node * n * B, taut + (int64_t)node * n,
                                n, k);
  __syncthreads();
  double* S0 = Sout + first * n * k;
  for (int i = tid; i < n * k; i += 256) S0[i] = Ss[i];
  if (merged) {
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const int row = rg + 16 * r;
      const int ch = row / n, lr = row - ch * n;
      if (ch < G && first + 1 + ch < nchild) {
        double* Sc = Sout + (first + 1 + ch) * n * k + (int64_t)lr * k;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          const int col = cg + 16 * c;
          if (col < k) Sc[col] = y[r][c];
        }
      }
    }
  }
}

// Rows of Q S for one leaf workgroup: walk its blocks backwards.
template <int NC, int NR>
__global__ __launch_bounds__(256) void k_leaf_apply(const double* __restrict__ Vw,
                                                    const double* __restrict__ tauw,
                                                    const double* __restrict__ Sw, int n,
                                                    int k, int bpw, int64_t nblocks,
                                                    int64_t m, double* __restrict__ out,
                                                    int64_t ldo, const int* __restrict__ gate) {
  if (gate && *gate == 0) return;
  extern __shared__ double smem[];
  constexpr int B = 16 * NR;
  double* Ss = smem;
  const int tid = threadIdx.x, rg = ts_rg(), cg = ts_cg();
  const double* S = Sw + (int64_t)blockIdx.x * n * k;
  for (int i = tid; i < n * k; i += 256) Ss[i] = S[i];
  __syncthreads();
  const int64_t b0 = (int64_t)blockIdx.x * bpw;
  const int64_t b1 = (b0 + bpw < nblocks) ? b0 + bpw : nblocks;
  for (int64_t blk = b1 - 1; blk >= b0; --blk) {
    double y[NR][NC];
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
      for (int c = 0; c < NC; ++c) y[r][c] = 0.0;
    apply_block_reverse<NC, NR>(y, Ss, Vw + blk * (int64_t)n * B, tauw + blk * n, n, k);
    const int64_t row0 = blk * B;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const int64_t row = row0 + rg + 16 * r;
      if (row < m) {
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          const int col = cg + 16 * c;
          if (col < k) out[row * ldo + col] = y[r][c];
        }
      }
    }
  }
}

// ------------------------------------------------------------------------- host side

// Column tile: thread (rg, cg) owns columns cg + 16c, c < NC.  Leaf blocks have B = 16*NR
// rows; merge nodes use blocks of BT = 16*TNR rows.
static void pick_tile(int n, int& nc, int& nr, int& tnr) {
  if (n <= 16) { nc = 1; nr = 16; tnr = 16; }
  else if (n <= 32) { nc = 2; nr = 16; tnr = 16; }
  else if (n <= 64) { nc = 4; nr = 16; tnr = 16; }
  else { nc = 8; nr = 8; tnr = 8; }
}

TsqrPlan tsqr_plan(int64_t m, int n, int nr, int wtarget, bool leaf_f32) {
  TsqrPlan p;
  p.m = m;
  p.n = n;
  pick_tile(n, p.nc, p.nr, p.tnr);
  if ((nr == 8 || nr == 16) && p.nc <= 4) p.nr = nr;
  p.B = 16 * p.nr;
  p.BT = 16 * p.tnr;
  // n >= 33: blocked leaf on the matrix cores, 128-row blocks, 256-thread workgroups, two
  // per CU (one for n > 112, whose carried factor needs more of the local data share).
  if (n >= 33 && n <= 128) {
    p.ntw = (n + 15) / 16;
    p.B = 128;
    p.wyf32 = leaf_f32;
  }
  p.nblocks = (m + p.B - 1) / p.B;
  // About as many leaf workgroups as can be resident at once (two per CU for the wide
  // tiles and the float64 blocked leaf, four for the float32 blocked leaf and the narrow
  // tiles): fewer would idle CUs, more would only deepen the merge tree.
  const int64_t target = wtarget > 0 ? wtarget
                         : p.ntw ? (p.wyf32 ? 1024 : p.ntw <= 7 ? 512 : 256)
                                 : (p.nc >= 4) ? 512 : 1024;
  int64_t W = p.nblocks < target ? p.nblocks : target;
  p.bpw = (int)((p.nblocks + W - 1) / W);
  p.W = (int)((p.nblocks + p.bpw - 1) / p.bpw);
  // merge nodes stack G = BT / n child factors in one block: fan-in G + 1
  p.G = p.BT / n;
  p.cnt.clear();
  p.cnt.push_back(p.W);
  while (p.cnt.back() > 1) p.cnt.push_back((p.cnt.back() + p.G) / (p.G + 1));
  return p;
}

void tsqr_carve(TsqrPlan& p, Carver& c) {
  const int n = p.n;
  if (p.ntw) {
    const int nt = p.ntw;
    const size_t nv = (size_t)p.nblocks * p.B * 16 * nt;
    const size_t ntt = (size_t)p.nblocks * nt * 256;
    const size_t nz = (size_t)p.nblocks * (nt > 1 ? nt * (nt - 1) / 2 : 1) * 256;
    if (p.wyf32) {
      p.Vwy = c.take<float>(nv);
      p.Twy = c.take<float>(ntt);
      p.Zwy = c.take<float>(nz);
      p.Vleaf = nullptr;  // no float64 m x n scratch in a float32 plan
    } else {
      p.Vwy = c.take<double>(nv);
      p.Twy = c.take<double>(ntt);
      p.Zwy = c.take<double>(nz);
      p.Vleaf = (double*)p.Vwy;
    }
    p.tauleaf = nullptr;
  } else {
    p.Vleaf = c.take<double>((size_t)p.nblocks * n * p.B);
    p.tauleaf = c.take<double>((size_t)p.nblocks * n);
  }
  const int L = (int)p.cnt.size();
  p.Rlev.assign(L, nullptr);
  p.Slev.assign(L, nullptr);
  p.Vtree.assign(L > 1 ? L - 1 : 0, nullptr);
  p.tautree.assign(L > 1 ? L - 1 : 0, nullptr);
  for (int l = 0; l < L; ++l) {
    p.Rlev[l] = c.take<double>((size_t)p.cnt[l] * n * n);
    p.Slev[l] = c.take<double>((size_t)p.cnt[l] * n * n);
  }
  for (int l = 0; l + 1 < L; ++l) {
    p.Vtree[l] = c.take<double>((size_t)p.cnt[l + 1] * n * p.BT);
    p.tautree[l] = c.take<double>((size_t)p.cnt[l + 1] * n);
  }
}

double* tsqr_root(const TsqrPlan& p) { return p.Rlev.back(); }

template <int NC, int NR, int TNR>
static hipError_t factor_impl(const TsqrPlan& p, const void* A, int a_dtype, int64_t lda,
                              hipStream_t s, bool prof) {
  const int n = p.n;
  const size_t lds = (size_t)(tri_size(n) + 2 * 16 * NR + n) * sizeof(double);
  if (prof) prof_begin(TSSVD_PROF_LEAF_FACTOR, s);
  if (p.ntw) {
    hipError_t e = wy_factor(p, A, a_dtype, lda, s);
    if (e != hipSuccess) return e;
  } else if (a_dtype == TSSVD_F64)
    hipLaunchKernelGGL((k_leaf_factor<NC, NR, double>), dim3(p.W), dim3(256), lds, s,
                       (const double*)A, lda, p.m, n, p.bpw, p.nblocks, p.Vleaf, p.tauleaf,
                       p.Rlev[0], p.gate);
  else
    hipLaunchKernelGGL((k_leaf_factor<NC, NR, float>), dim3(p.W), dim3(256), lds, s,
                       (const float*)A, lda, p.m, n, p.bpw, p.nblocks, p.Vleaf, p.tauleaf,
                       p.Rlev[0], p.gate);
  if (prof) prof_end(TSSVD_PROF_LEAF_FACTOR, s);
  const size_t lds_t = (size_t)(tri_size(n) + 2 * 16 * TNR + n) * sizeof(double);
  for (size_t l = 0; l + 1 < p.cnt.size(); ++l)
    hipLaunchKernelGGL((k_tree_factor<NC, TNR>), dim3(p.cnt[l + 1]), dim3(256), lds_t, s,
                       p.Rlev[l], p.cnt[l], n, p.G, p.Rlev[l + 1], p.Vtree[l], p.tautree[l],
                       p.gate);
  return hipGetLastError();
}

template <int NC, int NR, int TNR>
static hipError_t apply_impl(const TsqrPlan& p, const double* S, int k, double* out,
                             int64_t ldo, hipStream_t s, bool prof) {
  const int n = p.n;
  const int L = (int)p.cnt.size();
  // the root's seed is S itself (n x k, stride k, the layout of every level's seeds)
  auto seed = [&](int lev) -> const double* { return lev == L - 1 ? S : p.Slev[lev]; };
  const size_t lds = (size_t)n * k * sizeof(double);
  for (int l = L - 2; l >= 0; --l)
    hipLaunchKernelGGL((k_tree_apply<NC, TNR>), dim3(p.cnt[l + 1]), dim3(256), lds, s,
                       seed(l + 1), p.cnt[l], n, k, p.G, p.Vtree[l], p.tautree[l],
                       p.Slev[l], p.gate);
  if (prof) prof_begin(TSSVD_PROF_LEAF_APPLY, s);
  if (p.ntw) {
    const hipError_t e = wy_apply(p, seed(0), k, out, ldo, s);
    if (e != hipSuccess) return e;
  } else {
    hipLaunchKernelGGL((k_leaf_apply<NC, NR>), dim3(p.W), dim3(256), lds, s, p.Vleaf,
                       p.tauleaf, seed(0), n, k, p.bpw, p.nblocks, p.m, out, ldo, p.gate);
  }
  if (prof) prof_end(TSSVD_PROF_LEAF_APPLY, s);
  return hipGetLastError();
}

hipError_t tsqr_factor(const TsqrPlan& p, const void* A, int a_dtype, int64_t lda,
                       hipStream_t s, bool prof) {
  switch (p.nc * 100 + p.nr) {
    case 116: return factor_impl<1, 16, 16>(p, A, a_dtype, lda, s, prof);
    case 108: return factor_impl<1, 8, 16>(p, A, a_dtype, lda, s, prof);
    case 216: return factor_impl<2, 16, 16>(p, A, a_dtype, lda, s, prof);
    case 208: return factor_impl<2, 8, 16>(p, A, a_dtype, lda, s, prof);
    case 416: return factor_impl<4, 16, 16>(p, A, a_dtype, lda, s, prof);
    case 408: return factor_impl<4, 8, 16>(p, A, a_dtype, lda, s, prof);
    case 808: return factor_impl<8, 8, 8>(p, A, a_dtype, lda, s, prof);
    default: return hipErrorInvalidValue;
  }
}

hipError_t tsqr_apply(const TsqrPlan& p, const double* S, int k, double* out, int64_t ldo,
                      hipStream_t s, bool prof) {
  switch (p.nc * 100 + p.nr) {
    case 116: return apply_impl<1, 16, 16>(p, S, k, out, ldo, s, prof);
    case 108: return apply_impl<1, 8, 16>(p, S, k, out, ldo, s, prof);
    case 216: return apply_impl<2, 16, 16>(p, S, k, out, ldo, s, prof);
    case 208: return apply_impl<2, 8, 16>(p, S, k, out, ldo, s, prof);
    case 416: return apply_impl<4, 16, 16>(p, S, k, out, ldo, s, prof);
    case 408: return apply_impl<4, 8, 16>(p, S, k, out, ldo, s, prof);
    case 808: return apply_impl<8, 8, 8>(p, S, k, out, ldo, s, prof);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace tsv
