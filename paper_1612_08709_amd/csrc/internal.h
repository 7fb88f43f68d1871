// Host-side launchers shared between the kernel translation units and the C ABI layer.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <vector>

#include "../../include/tssvd.h"

namespace tsv {

// ------------------------------------------------------------------ workspace carving
struct Carver {
  char* base;
  size_t off = 0;
  explicit Carver(void* b) : base(static_cast<char*>(b)) {}
  template <typename T>
  T* take(size_t count) {
    off = (off + 255) & ~size_t(255);
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
};

// ------------------------------------------------------------------ TSQR
// Row blocks of B = 16*NR rows; each leaf workgroup reduces `bpw` consecutive blocks.
struct TsqrPlan {
  int64_t m = 0;
  int n = 0;
  int nc = 0, nr = 0, B = 0;  // leaf column tile, leaf rows per thread, leaf block rows
  int tnr = 0, BT = 0;        // merge-node rows per thread and block rows
  int64_t nblocks = 0;
  int W = 0;             // leaf workgroups
  int bpw = 0;           // blocks per leaf workgroup
  int G = 0;             // child factors stacked per merge block (fan-in G + 1)
  std::vector<int> cnt;  // cnt[0] = W, cnt[L+1] = ceil(cnt[L]/(G+1)), last = 1
  // workspace regions (filled by carve)
  double* Vleaf = nullptr;  // nblocks * n * B   reflector tails, column-major per block
  double* tauleaf = nullptr;  // nblocks * n
  std::vector<double*> Rlev;  // per level: cnt[L] * n * n
  std::vector<double*> Vtree; // per level L (merges producing level L+1): cnt[L+1] * n * BT
  std::vector<double*> tautree;
  std::vector<double*> Slev;  // seeds per level: cnt[L] * n * n
  // When non-NULL, every kernel of the plan returns at once if *gate == 0 (device flag).
  const int* gate = nullptr;
  // Blocked leaf (33 <= n <= 128): ntw = 16-column tiles, 256-row blocks; per block the
  // reflector tails V (256 x 16 ntw), the panel factors T_p and the products Z_cp = V_c^T V_p.
  // Vleaf then points at Vwy (callers use it as m x n scratch) and tauleaf is unused.
  int ntw = 0;
  bool wyf32 = false;  // blocked leaf in float32 arithmetic and storage (V, T_p, Z_cp)
  void* Vwy = nullptr;
  void* Twy = nullptr;
  void* Zwy = nullptr;
};

// nr (8 or 16, narrow tiles only) and wtarget (leaf workgroups) override the defaults.
// leaf_f32: the blocked leaf (33 <= n <= 128) computes in float32 (wyf32); the merge tree
// stays float64.  For n < 33 the flag is ignored (check p.wyf32).
TsqrPlan tsqr_plan(int64_t m, int n, int nr = 0, int wtarget = 0, bool leaf_f32 = false);
void tsqr_carve(TsqrPlan& p, Carver& c);
// Factor: leaf blocks + tree.  After it, root R (n x n, upper, row-major) is tsqr_root(p).
hipError_t tsqr_factor(const TsqrPlan& p, const void* A, int a_dtype, int64_t lda,
                       hipStream_t s, bool prof = false);
double* tsqr_root(const TsqrPlan& p);
// Apply: Q [S; 0] for a root seed S (n x k, row-major, stride k, device), written to
// out (m x k, stride ldo).  S is copied first, so it may live anywhere.
hipError_t tsqr_apply(const TsqrPlan& p, const double* S, int k, double* out, int64_t ldo,
                      hipStream_t s, bool prof = false);

// Blocked leaf kernels (csrc/tsqr_wy.hip), used by tsqr_factor / tsqr_apply when ntw > 0.
hipError_t wy_factor(const TsqrPlan& p, const void* A, int a_dtype, int64_t lda, hipStream_t s);
hipError_t wy_apply(const TsqrPlan& p, const double* S0, int k, double* out, int64_t ldo,
                    hipStream_t s);
// elements of storage per block: V, the ntw panel factors T_p and the Z_cp pairs
size_t wy_block_elems(int ntw);

// ------------------------------------------------------------------ small SVD (Jacobi)
// SVD of M (n x n row-major, stride ldm; its transpose when transpose != 0):
//   M = Uo diag(So) Vo^T, columns sorted by descending singular value.
// wp > 0 zeroes the rows j with |M_jj| < wp |M_00| first (discard rule) and zeroes the
// triplets past the kept rank; the diagonal tested is that of dsrc (stride ldd) when
// given, else M's.  sign_fix orients pairs so that w^T v_j >= 0.
hipError_t jacobi_svd(const double* M, int ldm, int n, int transpose, double wp,
                      int max_sweeps, int sign_fix, double* Uo, double* So, double* Vo,
                      tssvd_info* info, hipStream_t s, const int* gate = nullptr,
                      const double* dsrc = nullptr, int ldd = 0);

// ------------------------------------------------------------------ products with A
// Y (m x l, stride ldy) = A (m x n) X (n x l, stride ldx), float64 accumulation.
hipError_t gemm_ax_f64(const void* A, int a_dtype, int64_t lda, int64_t m, int64_t n,
                       const double* X, int ldx, int l, double* Y, int ldy, hipStream_t s,
                       int prof = -1);
// The same for float64 A with Y += A X when accum (Y read before it is written).
hipError_t gemm_ax_f64_acc(const double* A, int64_t lda, int64_t m, int64_t n, const double* X,
                           int ldx, int l, double* Y, int ldy, bool accum, hipStream_t s);
// Z (n x l, stride ldz) = A^T (n x m) Q (m x l, stride ldq).  Split over row chunks into
// `part` (size atq_partials(m, n, l) doubles), reduced in a fixed order.
size_t atq_partials(int64_t m, int64_t n, int l);
hipError_t gemm_atq_f64(const void* A, int a_dtype, int64_t lda, int64_t m, int64_t n,
                        const double* Q, int ldq, int l, double* Z, int ldz, double* part,
                        hipStream_t s, int prof = -1);

// Q = Y T (Y m x l float64, T l x l) written as the bfloat16 fragments of Q that
// pack_operand(Q, m, l, l, MIX_BF16, P) produces (bitwise the same), Q never stored.
hipError_t gemm_ax_f64_pack_bf16(const double* Y, int64_t ldy, int64_t m, const double* T,
                                 int ldt, int l, void* P, hipStream_t s);
// G = Y^T Y (l x l, FP64) of a tall Y stored as float64 or float32 (y_dtype); `part` holds
// atq_partials(rows, l, l) doubles.  Fixed summation order.
hipError_t gram_any(const void* Y, int y_dtype, int64_t ldy, int64_t rows, int l, double* G,
                    int ldg, double* part, hipStream_t s);
// out[j] = sum_i Y[i][j]^2 for a tall Y (l <= 256); `part` holds column_sumsq_partials doubles.
hipError_t column_sumsq(const void* Y, int y_dtype, int64_t rows, int l, int64_t ldy, double* out,
                        double* part, hipStream_t s);
size_t column_sumsq_partials(int64_t rows, int l);

// ------------------------------------------------------------------ LU tracking bases
// T = U^-1 for the tournament-pivoted LU factor U of Y (rows x l, float64, row-major,
// stride ldy, rows >= l, l <= LU_L_MAX), so that Y T spans range(Y); *use_q (device) = 1
// and T = I when U is singular or not finite.  idx: lu_index_ints(rows, l) ints.
constexpr int LU_L_MAX = 64;
size_t lu_index_ints(int64_t rows, int l);
hipError_t lu_tracking_T(const double* Y, int64_t rows, int l, int64_t ldy, int* idx, double* T,
                         int* use_q, hipStream_t s);
hipError_t reduce_chunks(const double* part, int nchunk, int64_t n, int l, double* Z, int ldz,
                         hipStream_t s, const int* gate = nullptr);

// Mixed precision (A stored float32).  kind: operand packing / MFMA flavour.
constexpr int MIX_BF16 = 0;    // bfloat16 inputs, float32 accumulation
constexpr int MIX_F32_AX = 1;  // float32 inputs, packed for Y = A X
constexpr int MIX_F32_ROWS = 2;  // float32 inputs, padded rows for Z = A^T Q
constexpr int MIX_BF16X3 = 3;  // float32-accurate inputs as three exact bfloat16 pieces
constexpr int MIX_BF16P = 4;   // bfloat16, k paired in 64-column groups (first pass with copy)
size_t mixed_partials(int64_t m, int64_t n, int l);
size_t mixed_pack_bytes(int64_t K, int l);
// Pack the K x l float64 operand S (stride lds) for the kernels below.
hipError_t pack_operand(const double* S, int64_t K, int l, int lds, int kind, void* P,
                        hipStream_t s);
// Y (m x l) = A X with X packed as MIX_BF16 or MIX_F32_AX.
hipError_t gemm_ax_mixed(const float* A, int64_t lda, int64_t m, int64_t n, const void* Xp,
                         int l, double* Y, int ldy, int kind, hipStream_t s, int prof = -1);
// Power-step Y = A X from the float32 A, bfloat16 inputs, X packed as MIX_BF16P; with
// Acopy non-null it also stores the bfloat16 copy of A (first pass).
hipError_t gemm_ax_bf16p(const float* A, int64_t lda, int64_t m, int64_t n, const void* Xp,
                         int l, double* Y, int ldy, void* Acopy, hipStream_t s, int prof = -1);
// bfloat16 copy of A: row-major m x bf16_copy_ld(n) (n rounded up to 64, zero-padded).
int64_t bf16_copy_ld(int64_t n);
size_t bf16_copy_bytes(int64_t m, int64_t n);
// Y = A X (X packed as MIX_BF16P) and Z = A^T Q (Q packed as MIX_BF16) reading the copy.
hipError_t gemm_ax_bf16c(const void* Ac, int64_t m, int64_t n, const void* Xp, int l, double* Y,
                         int ldy, hipStream_t s, int prof = -1);
hipError_t gemm_atq_bf16c(const void* Ac, int64_t m, int64_t n, const void* Qp, int l,
                          double* Z, int ldz, double* part, hipStream_t s, int prof = -1);
// Z (n x l) = A^T Q with Q packed as MIX_BF16 or MIX_F32_ROWS (kind MIX_F32_ROWS selects
// the float32 kernel).
hipError_t gemm_atq_mixed(const float* A, int64_t lda, int64_t m, int64_t n, const void* Qp,
                          int l, double* Z, int ldz, double* part, int kind, hipStream_t s,
                          int prof = -1);

// ------------------------------------------------------------------ preconditioned Cholesky QR
// (csrc/precond.hip; 33 <= n <= 112)
// Rp = R with diagonal entries below tol max|R_ii| raised to that size; Q = X Rp^-1 (X m x n
// float32 or float64, stride ldx; Q float64, stride ldq, may be X itself for float64) and
// G = Q^T Q (n x n).  Rop: pc_op_elems(n) doubles; part: pc_grid(m) n n doubles.  With a
// gate, every kernel (preparation, solve, reduction) does its work only if *gate != 0.
int pc_grid(int64_t m);
size_t pc_op_elems(int n);
// gram = false: the solve only (Q written, G and part untouched).
hipError_t pc_trsm_gram(const double* R, int ldr, int n, double tol, double* Rp, double* Rop,
                        const void* X, int x_dtype, int64_t ldx, int64_t m, double* Q,
                        int64_t ldq, double* part, double* G, const int* gate, hipStream_t s,
                        bool gram = true);
// X <- X N in place (X m x n float64, stride ldx; N n x n, stride ldn); Nop: pc_op_elems(n).
hipError_t pc_rowmul(double* X, int64_t ldx, int64_t m, int n, const double* N, int ldn,
                     double* Nop, const int* gate, hipStream_t s);
// *flag = 1 when sqrt(||G||_1) ||Ri||_F > kmax (an upper bound of kappa_2 of G's Cholesky
// factor, Ri its inverse) or not finite.
hipError_t pc_kappa_flag(const double* G, const double* Ri, int n, double kmax, int* flag,
                         hipStream_t s);
// fl[2] != 0: Rtot = R3 R2b Rp, Ninv = R3^-1; else Rtot = R2 Rp, Ninv = R2^-1; rows of a
// dropped direction (flags d2, resp. d1) zeroed in both; fl[0] / fl[3] (failed Cholesky
// factorizations) set NUM_NONFINITE in info.
hipError_t pc_combine(const int* fl, const double* Rp, const double* R2, const double* R2b,
                      const double* R2i, const double* R3, const double* R3i, const int* d1,
                      const int* d2, int n, double* Rtot, double* Ninv, tssvd_info* info,
                      hipStream_t s);

// ------------------------------------------------------------------ reverse pass
hipError_t bw_svd_core(const double* Ub, const double* sig, const double* G1, const double* G2,
                       const double* Sbar, int l, int k, double* A1, double* KB, double* Kw,
                       double* Kv, double* UbkT, hipStream_t s);
// Rinv = R^-1 (upper triangular l x l, stride l; back substitution, one thread per column).
hipError_t bw_rinv(const double* R, int l, double* Rinv, hipStream_t s);
// The same from R^-1 (upper triangular, stride l) already formed.
hipError_t bw_qr_coef_rinv(const double* M, const double* Rinv, int l, double* K1, double* K2,
                           hipStream_t s);
hipError_t rmul(const double* X1, int64_t ld1, int k1, const double* K1, const double* X2,
                int64_t ld2, int k2, const double* K2, int64_t rows, int kout, double* out,
                int64_t ldo, bool accum, hipStream_t s);
hipError_t zero_fill(double* p, int64_t count, hipStream_t s);
hipError_t gemm_nt(const double* L, int64_t ldl, const double* R, int64_t ldr, int64_t m,
                   int64_t n, int K, void* C, int c_dtype, int64_t ldc, hipStream_t s);

// ------------------------------------------------------------------ misc
hipError_t fill_identity(double* S, int n, int k, hipStream_t s);
hipError_t philox_sketch(double* X, int64_t n, int l, uint64_t seed, hipStream_t s);
// Orient columns of V (n x k) so that w^T v_j >= 0; flip the same columns of P (rows x k,
// stride ldp) and of V.
hipError_t sign_fix_cols(double* V, int64_t n, int ldv, int k, double* P, int prow, int ldp,
                         hipStream_t s, const int* gate = nullptr);
hipError_t copy_matrix(const double* src, int64_t rows, int cols, int64_t lds, double* dst,
                       int64_t ldd, hipStream_t s, const int* gate = nullptr);
hipError_t info_init(tssvd_info* info, hipStream_t s);

// measurement markers (no-ops unless tssvd_profile_enable(1) was called); kind < 0 = none
void prof_begin(int kind, hipStream_t s);
void prof_end(int kind, hipStream_t s);
void prof_enable(bool on);
hipError_t prof_read(int kind, double* total_ms, int64_t* launches);

}  // namespace tsv
