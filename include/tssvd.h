/*
 * tssvd.h — C ABI of the MI355X (gfx950) tall-skinny and randomized low-rank SVD library.
 *
 * Method: Li, Kluger, Tygert, "Randomized algorithms for distributed computation of
 * principal component analysis and singular value decomposition".
 *   - tsqr / tssvd      : Algorithms 1 and 2 (Section 2): Householder TSQR reduced up a
 *                         binary tree, SVD of the small triangular factor, U = Q U~,
 *                         optional second orthonormalization.
 *   - lowrank_svd       : Algorithm 7 (Section 3) = Algorithm 5 (randomized subspace
 *                         iteration) feeding Algorithm 6 (direct SVD of B = Q^* A).
 *   - lowrank_svd_backward : vector-Jacobian product of lowrank_svd with the sketch held
 *                         fixed (not in the paper; the reverse mode of the same forward).
 *
 * Conventions shared by every entry point
 *   - Matrices are row-major.  "ld" arguments are row strides in elements (ld >= columns).
 *   - Every matrix/vector pointer is a DEVICE pointer owned by the caller.  The library
 *     never allocates device or host memory and never synchronizes the stream: all work
 *     is enqueued on `stream` (a hipStream_t; NULL = the legacy default stream).
 *   - Scratch memory is the caller's `work` buffer (device, 256-byte aligned, else
 *     TSSVD_E_WORKSPACE), sized by the matching *_workspace_bytes query.  Its contents are
 *     undefined on return.
 *   - Inputs A may be float64 or float32 (a_dtype).  Outputs U, S, V are float64.
 *   - Return value: a tssvd_status for errors detectable on the host (checked before
 *     any work is enqueued; nothing is enqueued on error).  Numerical conditions found
 *     on the device are written to the optional device record `info`.
 *   - Singular values are descending and non-negative.  Sign convention: each pair
 *     (u_j, v_j) is oriented so that w^T v_j >= 0 with w_i = frac((i+1) g) - 1/2,
 *     g = (sqrt(5)-1)/2, i = 0..n-1.  Triplets past the numerical rank (discard rule,
 *     working_precision > 0) have sigma = 0 and zero columns in U and V.  With
 *     working_precision = 0 a singular value that comes out exactly 0 (an exactly
 *     rank-deficient A) has a zero column in U: A does not determine that direction.
 *   - Results are bitwise reproducible for identical inputs, options and sizes (fixed
 *     reduction orders, no floating-point atomics).
 *   - Calls that share a `work` buffer must be ordered on one stream.
 */
#ifndef TSSVD_H
#define TSSVD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Largest column count handled by tssvd and largest sketch width l for lowrank_svd.
 * The small SVD keeps both n x n factors in the 160 KB local data share of one CU. */
#define TSSVD_N_MAX 100
/* Largest column count handled by tsqr alone. */
#define TSSVD_TSQR_N_MAX 128

typedef enum {
  TSSVD_OK = 0,
  TSSVD_E_INVALID_ARG = 1,   /* null pointer, bad size, ld too small, k > l, ...        */
  TSSVD_E_WORKSPACE = 2,     /* work == NULL or work_bytes below the query's answer     */
  TSSVD_E_HIP = 3,           /* a HIP launch failed                                     */
  TSSVD_E_UNSUPPORTED = 4    /* size or option outside what this build implements      */
} tssvd_status;

typedef enum { TSSVD_F64 = 0, TSSVD_F32 = 1 } tssvd_dtype;

typedef enum {
  TSSVD_PREC_FP64 = 0,       /* every product and factorization in float64              */
  TSSVD_PREC_MIXED = 1       /* Requires a_dtype == TSSVD_F32 (else
                                TSSVD_E_INVALID_ARG).  lowrank_svd: power-iteration
                                products in bfloat16 with float32 accumulation; final
                                sketch and B products with float32-exact inputs (three
                                bfloat16 pieces per value) and float32 accumulation;
                                TSQR, small SVD and the second orthonormalization in
                                float64.  tssvd (33 <= n; no discard rule, mixing or
                                Gram route, else TSSVD_E_UNSUPPORTED): Algorithm 2 with
                                its first factorization A = Q1 R1 from a float32 TSQR
                                (leaf reflectors and their matrix-core products in
                                float32, merge tree in float64) whose Q1 is formed as
                                A R1^-1 by a float64 triangular solve, and its second
                                Q1 = Q R2 as a float64 Cholesky QR (repeated once when
                                R2 is ill-conditioned); T = R2 R1 = P S W^T, U = Q P.
                                ONCE returns U = Q1~ U1~ from the float32 Householder
                                reflectors (orthonormal to ~1e-6).  A direction that
                                is exactly dependent (to float64 rounding) comes out as
                                sigma = 0 with a zero column of U.                     */
} tssvd_prec;

typedef enum {
  TSSVD_ORTHO_AUTO = 0,      /* run the second orthonormalization only if
                                ||U^T U - I||_2 > reorth_tol (decided exactly from the
                                Gram matrix G: (1 + tol) I - G and G - (1 - tol) I both
                                pass a Cholesky factorization, or ||G - I||_F <= tol)  */
  TSSVD_ORTHO_ONCE = 1,      /* Algorithm 1: one orthonormalization                     */
  TSSVD_ORTHO_TWICE = 2      /* Algorithm 2: always orthonormalize twice                */
} tssvd_ortho;

typedef struct {
  int32_t prec;              /* tssvd_prec                                               */
  int32_t ortho;             /* tssvd_ortho (tssvd, and the last step of Algorithm 5)    */
  double working_precision;  /* discard rule of Algorithms 1-2: rows of R with
                                |R_jj| < wp |R_11| are dropped; <= 0 disables (default)  */
  double reorth_tol;         /* TSSVD_ORTHO_AUTO threshold (default 1e-13)               */
  int32_t max_jacobi_sweeps; /* cap on one-sided Jacobi sweeps in the small SVD (30)     */
  int32_t flags;             /* TSSVD_FLAG_* bits (default 0)                            */
  uint64_t seed;             /* Philox4x32-10 key used when lowrank_svd gets Omega==NULL */
} tssvd_opts;

/* Mixed mode: run the final sketch and B products on float32 matrix cores instead of the
 * default exact three-way bfloat16 split of the float32 inputs (same float32-input result,
 * float32 accumulation either way). */
#define TSSVD_FLAG_F32_MFMA_FINAL 1
/* Mixed precision, q >= 1: do not keep a bfloat16 copy of A for the power steps.  By
 * default the first pass over A also stores A rounded to bfloat16 (m x n rounded up to 32
 * columns, 2 bytes each, inside the workspace) and the other power-step passes read that
 * copy instead of the float32 A: half the bytes, bit-identical products.  With this flag
 * the workspace is smaller by that amount and every pass reads the float32 A. */
#define TSSVD_FLAG_NO_A_COPY 2
/* Gram-based route (Section 2's second method, with the explicit column normalization of
 * the paper's remark on normalizing).  tssvd: Algorithm 3 when ortho == TSSVD_ORTHO_ONCE,
 * else Algorithm 4 (always two passes): B = A^* A, eigendecomposition B = V D V^*,
 * U~ = A V, sigma = column norms of U~, columns with sigma < max(sigma) sqrt(wp) dropped
 * (wp = working_precision), U = U~ Sigma^-1; Algorithm 4 repeats the pass on U and forms
 * U, Sigma, V from the SVD of R = T W^* Sigma~ V~^*.  lowrank_svd: Algorithm 8 (Algorithm 5
 * with its intermediate bases from Algorithm 3 and its last from Algorithm 4, then
 * Algorithm 6); working_precision > 0 is allowed with this flag.  Triplets past the kept
 * rank come back as zero columns with sigma = 0 and info->rank reports the rank.  The Gram
 * matrix squares the condition number: singular values below ~sqrt(eps) sigma_1 are not
 * resolved (the paper's trade of accuracy for one pass). */
#define TSSVD_FLAG_GRAM 4
/* lowrank_svd: LU-based subspace tracking (Section 3's remark on the power iterations).
 * The intermediate bases of Algorithm 5 are L = Y U^-1 from an LU factorization of Y with
 * tournament pivoting (Gaussian elimination with partial pivoting on groups of rows, the
 * picked rows competing again up a tree) instead of an orthonormal Q; they span the same
 * columns.  The last step keeps Algorithm 2's double orthonormalization, so the result is
 * that of Algorithm 7 up to rounding.  A singular pivot block falls back to the Householder
 * Q for that step.  Requires l <= 64, working_precision <= 0 and m, n < 2^31 - 1024
 * (TSSVD_E_UNSUPPORTED otherwise); TSSVD_FLAG_GRAM with it is TSSVD_E_INVALID_ARG.  Other entry points ignore
 * the flag, except lowrank_svd_backward, which rejects it. */
#define TSSVD_FLAG_LU 8
/* tssvd: Algorithm 1 step (1), the random orthogonal mixing of the Remark on randomness,
 * which makes the discard rule (working_precision > 0) reveal the rank whatever the order
 * of A's columns.  Omega (n x n) is the Q factor of an n x n matrix of Philox4x32-10
 * normals keyed by opts->seed (the lowrank_svd sketch layout), with the column signs that
 * make diag(R) positive (Haar-distributed).  It is applied to the triangular factor:
 * A = Q0 R0, R0 Omega^T = Q1 R', so A Omega^T = (Q0 Q1) R'; the rule reads the diagonal of
 * R', V = Omega^T V~, U = Q0 Q1 U~.  The second pass of Algorithm 2 is unmixed.  With
 * TSSVD_FLAG_GRAM it is TSSVD_E_INVALID_ARG; lowrank_svd and lowrank_svd_backward reject
 * it (TSSVD_E_UNSUPPORTED). */
#define TSSVD_FLAG_MIX 16

/* Device-side record written (when non-NULL) at the end of every call. */
typedef struct {
  int32_t numstat;           /* bit 0: non-finite value met; bit 1: Jacobi sweep cap hit */
  int32_t rank;              /* number of kept singular triplets                          */
  int32_t sweeps;            /* Jacobi sweeps used by the last small SVD                  */
  int32_t reorth;            /* 1 if a second orthonormalization pass ran                 */
  double ortho;              /* ||Q^T Q - I||_F of the orthonormal factor before the
                                conditional second pass (an upper bound of the spectral
                                norm the AUTO gate tests); -1 when not measured          */
} tssvd_info;

void tssvd_default_opts(tssvd_opts* opts);
const char* tssvd_status_string(int status);
/* Library version as major*10000 + minor*100 + patch. */
int tssvd_version(void);

/* ---------------------------------------------------------------------------------------
 * tsqr — Algorithm 1 step 2: A = Q R for a tall m x n matrix (m >= n, 1 <= n <= 128).
 * Row blocks of A are reduced by structured Householder QR, the per-block R factors are
 * merged pairwise up a fixed binary tree, and Q is formed explicitly by applying the
 * stored reflectors to [I; 0] when Q != NULL.
 *   A   : m x n, a_dtype, stride lda           (read)
 *   Q   : m x n float64, stride ldq, or NULL    (written)
 *   R   : n x n float64 upper triangular, stride ldr (written; strict lower part zeroed)
 * The diagonal of R may be negative (Householder convention beta = -sign(alpha) ||x||).
 * ------------------------------------------------------------------------------------- */
int tsqr_workspace_bytes(int64_t m, int64_t n, int32_t a_dtype, size_t* bytes);
int tsqr(const void* A, int32_t a_dtype, int64_t m, int64_t n, int64_t lda,
         double* Q, int64_t ldq, double* R, int64_t ldr,
         void* work, size_t work_bytes, void* stream);

/* ---------------------------------------------------------------------------------------
 * tssvd — thin SVD of a tall-skinny A (Algorithms 1 and 2): A = U diag(S) V^T.
 *   A : m x n (m >= n, 1 <= n <= TSSVD_N_MAX), a_dtype, stride lda   (read)
 *   U : m x n float64, stride ldu                                     (written)
 *   S : n float64                                                     (written)
 *   V : n x n float64, stride ldv                                     (written)
 *   info : optional device tssvd_info                                 (written)
 * opts == NULL means tssvd_default_opts.
 * ------------------------------------------------------------------------------------- */
int tssvd_workspace_bytes(int64_t m, int64_t n, int32_t a_dtype, const tssvd_opts* opts,
                          size_t* bytes);
int tssvd(const void* A, int32_t a_dtype, int64_t m, int64_t n, int64_t lda,
          double* U, int64_t ldu, double* S, double* V, int64_t ldv,
          tssvd_info* info, void* work, size_t work_bytes, const tssvd_opts* opts,
          void* stream);

/* ---------------------------------------------------------------------------------------
 * tssvd_noalloc — tssvd without a workspace argument, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, options, results and errors as tssvd; the scratch memory is
 * a fixed array of TSSVD_NOALLOC_SCRATCH_BYTES inside the library's code object, one per
 * GPU, held from its first use until the process ends.  The call allocates nothing and
 * does not record measurement events.
 *   - Sizes whose tssvd_workspace_bytes exceeds TSSVD_NOALLOC_SCRATCH_BYTES return
 *     TSSVD_E_UNSUPPORTED (nothing is enqueued).  In this version n = 100 fits
 *     m <= 13,056 rows, n = 64 fits m <= 31,872 and n = 20 fits m <= 303,040.
 *   - The array belongs to the current device (hipGetDevice) of the calling thread;
 *     `stream` must be a stream of that device.  Its address is looked up on the first
 *     call on each device.
 *   - Every call on one GPU shares that GPU's array and leaves its contents behind: calls
 *     that may overlap on one GPU (different streams, or different host threads without
 *     ordering) race and must be serialized by the caller.
 * ------------------------------------------------------------------------------------- */
#define TSSVD_NOALLOC_SCRATCH_BYTES (64u << 20)
int tssvd_noalloc(const void* A, int32_t a_dtype, int64_t m, int64_t n, int64_t lda,
                  double* U, int64_t ldu, double* S, double* V, int64_t ldv,
                  tssvd_info* info, const tssvd_opts* opts, void* stream);

/* ---------------------------------------------------------------------------------------
 * lowrank_svd — rank-k approximation A ~ U diag(S) V^T by Algorithm 7 with sketch width
 * l and q power iterations (the paper's i): 2q+2 passes over A.
 *   A     : m x n, a_dtype, stride lda.  Requires 0 < k <= l < min(m, n), l <= TSSVD_N_MAX,
 *           q >= 0, and the sketched dimension n >= l.
 *   Omega : n x l float64 row-major (stride l) Gaussian sketch, or NULL to draw it on the
 *           device with Philox4x32-10 keyed by opts->seed (layout: entries in row-major
 *           order, four per counter value t, counter (t mod 2^32, t div 2^32, 0, 0), key
 *           (seed mod 2^32, seed div 2^32), Box-Muller on (u0,u1), (u2,u3) with
 *           u = (x + 1/2) 2^-32).
 *   U : m x k float64 (ldu), S : k float64, V : n x k float64 (ldv)     (written)
 * opts->working_precision > 0 is the paper's rank-deficient mode: every basis of Algorithm
 * 5 is the TSQR's Householder Q with the columns whose |R_jj| < wp |R_11| dropped (set to
 * zero), and the last basis is orthonormalized twice with the rule applied after each pass.
 * Triplets past the kept rank come back as zero columns with S = 0; info->rank is the rank.
 * Otherwise (wp = 0, ortho AUTO or TWICE) the last basis takes Algorithm 2's two
 * orthonormalizations as CholeskyQR, each with a device gate to the Householder TSQR
 * (non-positive pivot or ||R||_F ||R^-1||_F > 1e4), the second decided by opts->ortho and
 * reorth_tol as in tssvd; with ORTHO_ONCE it is the TSQR's Householder Q.
 * With TSSVD_FLAG_GRAM the call runs Algorithm 8 instead (see the flag).
 * ------------------------------------------------------------------------------------- */
int lowrank_svd_workspace_bytes(int64_t m, int64_t n, int64_t k, int64_t l, int64_t q,
                                int32_t a_dtype, const tssvd_opts* opts, size_t* bytes);
int lowrank_svd(const void* A, int32_t a_dtype, int64_t m, int64_t n, int64_t lda,
                int64_t k, int64_t l, int64_t q, const double* Omega,
                double* U, int64_t ldu, double* S, double* V, int64_t ldv,
                tssvd_info* info, void* work, size_t work_bytes, const tssvd_opts* opts,
                void* stream);

/* ---------------------------------------------------------------------------------------
 * lowrank_svd_backward — dL/dA for a scalar loss L(U, S, V) of lowrank_svd's outputs,
 * given the cotangents gU = dL/dU (m x k, stride ldu), gS = dL/dS (k), gV = dL/dV
 * (n x k, stride ldv); any of the three may be NULL (zero).  The derivative is that of the
 * implemented forward map with Omega held fixed (Omega == NULL: the Philox sketch of
 * opts->seed).  The forward is recomputed from (A, Omega) inside the call with one
 * orthonormalization per factorization (a second pass on an orthonormal factor has
 * identity derivative): the intermediate bases as lowrank_svd forms them (CholeskyQR,
 * with the device gate to the TSQR), the last one by the TSQR; U, S, V must therefore
 * come from lowrank_svd on the same A, Omega, k,
 * l, q and options; they are not read.  2q+2 passes over A recompute the forward, 2q+1
 * passes and one m x (2q+2)l x n product form gA.
 *   gA : m x n, a_dtype, stride ldga (written)
 * Requires opts->prec == TSSVD_PREC_FP64, working_precision <= 0 and none of
 * TSSVD_FLAG_GRAM, TSSVD_FLAG_LU, TSSVD_FLAG_MIX (TSSVD_E_UNSUPPORTED otherwise).
 * ------------------------------------------------------------------------------------- */
int lowrank_svd_backward_workspace_bytes(int64_t m, int64_t n, int64_t k, int64_t l,
                                         int64_t q, int32_t a_dtype, const tssvd_opts* opts,
                                         size_t* bytes);
int lowrank_svd_backward(const void* A, int32_t a_dtype, int64_t m, int64_t n, int64_t lda,
                         int64_t k, int64_t l, int64_t q, const double* Omega,
                         const double* U, int64_t ldu, const double* S, const double* V,
                         int64_t ldv, const double* gU, const double* gS, const double* gV,
                         void* gA, int64_t ldga, tssvd_info* info, void* work,
                         size_t work_bytes, const tssvd_opts* opts, void* stream);

/* ---------------------------------------------------------------------------------------
 * Measurement support.  While enabled, HIP events are recorded on the call's stream right
 * before and after every launch of the kernels that stream A (one kind per kernel family);
 * tssvd_profile_read waits for the recorded events and returns the summed durations.
 * Disabled (the default) it costs nothing.  Event objects are host-side HIP resources,
 * created on first use and reused; no device memory is allocated.
 * ------------------------------------------------------------------------------------- */
enum {
  TSSVD_PROF_AX = 0,           /* Y = A X passes over A, float64 products                 */
  TSSVD_PROF_ATQ = 1,          /* Z = A^T Q passes over A, float64 (before the reduce)    */
  TSSVD_PROF_LEAF_FACTOR = 2,  /* TSQR leaf factorization (reads the tall matrix)         */
  TSSVD_PROF_LEAF_APPLY = 3,   /* TSQR leaf application (writes the tall factor)          */
  TSSVD_PROF_AX_BF16 = 4,      /* Y = A X, bfloat16 inputs (mixed power steps)            */
  TSSVD_PROF_ATQ_BF16 = 5,     /* Z = A^T Q, bfloat16 inputs (mixed power steps)          */
  TSSVD_PROF_AX_FINAL = 6,     /* Y = A X, float32-exact inputs (mixed final sketch)      */
  TSSVD_PROF_ATQ_FINAL = 7,    /* Z = A^T Q, float32-exact inputs (mixed B = Q^T A)       */
  TSSVD_PROF_AX_BF16C = 8,     /* Y = A X reading the bfloat16 copy of A (mixed)          */
  TSSVD_PROF_ATQ_BF16C = 9,    /* Z = A^T Q reading the bfloat16 copy of A (mixed)        */
  TSSVD_PROF_KINDS = 10
};
int tssvd_profile_enable(int on);      /* on != 0: start recording (counters reset)      */
int tssvd_profile_read(int kind, double* total_ms, int64_t* launches);

#ifdef __cplusplus
}
#endif
#endif /* TSSVD_H */
