// Mixed-precision products with a float32-stored A on gfx950 matrix cores.
//
//   power steps (Algorithm 5 steps 2, 5 and 7 before the last):  bfloat16 inputs (round to
//   nearest even, converted in registers), float32 accumulation, v_mfma_f32_16x16x32_bf16;
//   final sketch (Algorithm 5 step 9) and B^* = A^* Q (Algorithm 6 step 1): float32 inputs
//   and accumulation, v_mfma_f32_16x16x4_f32.
// Results are written in float64; A^T Q partials over row chunks are reduced in float64 in
// chunk order (same reduction kernel as the float64 path).
//
// Operand layouts (measured on gfx950):
//   16x16x32 bf16: A operand lane l holds row l%16, k = 8*(l/16) + e (e < 8); B operand
//                  column l%16, k = 8*(l/16) + e; result register r = D[4*(l/16)+r][l%16].
//   16x16x4 f32:   A operand row l%16, k = l/16; B operand k = l/16, column l%16;
//                  result register r = D[4*(l/16)+r][l%16].
// A is read straight into fragments: for Y = A X a lane reads 8 (bf16) or 4 (f32)
// consecutive columns of one row; for Z = A^T Q a lane reads 4 consecutive columns of 8
// (bf16) or 1 (f32) rows and the four result tiles interleave those columns (tile e holds
// columns c + 4i + e), so no transposition through shared memory is needed.  The small
// operand (X or Q) is packed beforehand into the exact per-lane fragment order.
#include "common.h"
#include "internal.h"

namespace tsv {

#ifndef AXF_RT
#define AXF_RT 4
#endif
#ifndef AXC_RT
#define AXC_RT 4
#endif

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f32x4 mfma_bf16(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f32x4 mfma_f32(float a, float b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// ---------------------------------------------------------------- operand packing
// bf16 B-operand fragments of a K x l float64 matrix S (stride lds), each entry rounded
// once from its float64 value to the nearest bfloat16 (ties to even):
//   P[(kb*NT + nt)*64 + lane][e] = S[32 kb + 8 (lane/16) + e][16 nt + lane%16]  (0 outside)
__global__ void k_pack_bf16(const double* __restrict__ S, int64_t K, int l, int lds, int NT,
                            int64_t nkb, bf16x8* __restrict__ P) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= nkb * NT * 64) return;
  const int lane = (int)(idx & 63);
  const int64_t t = idx >> 6;
  const int nt = (int)(t % NT);
  const int64_t kb = t / NT;
  const int col = 16 * nt + (lane & 15);
  const int64_t k0 = 32 * kb + 8 * (lane >> 4);
  bf16x8 v;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const int64_t k = k0 + e;
    v[e] = (__bf16)((k < K && col < l) ? S[k * lds + col] : 0.0);
  }
  P[idx] = v;
}

// Paired layout for the first pass with the copy: in each 64-row group kg, lane (i, g)
// of MFMA j in {0, 1} takes rows 64 kg + 16 g + 8 j + e, so a lane's A values for the two
// MFMAs are 16 consecutive columns:
//   P[((kg*2 + j)*NT + nt)*64 + lane][e] = S[64 kg + 16 (lane/16) + 8 j + e][16 nt + lane%16]
__global__ void k_pack_bf16p(const double* __restrict__ S, int64_t K, int l, int lds, int NT,
                             int64_t ng, bf16x8* __restrict__ P) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= ng * 2 * NT * 64) return;
  const int lane = (int)(idx & 63);
  const int64_t t = idx >> 6;
  const int nt = (int)(t % NT);
  const int64_t kj = t / NT;  // kg * 2 + j
  const int col = 16 * nt + (lane & 15);
  const int64_t k0 = 64 * (kj >> 1) + 16 * (lane >> 4) + 8 * (kj & 1);
  bf16x8 v;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const int64_t k = k0 + e;
    v[e] = (__bf16)((k < K && col < l) ? S[k * lds + col] : 0.0);
  }
  P[idx] = v;
}

// f32 B-operand fragments for Y = A X:  P[((kb*NT + nt)*64 + lane)*4 + s] =
//   S[16 kb + 4 (lane/16) + s][16 nt + lane%16]
__global__ void k_pack_f32_ax(const double* __restrict__ S, int64_t K, int l, int lds, int NT,
                              int64_t nkb, float* __restrict__ P) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= nkb * NT * 64) return;
  const int lane = (int)(idx & 63);
  const int64_t t = idx >> 6;
  const int nt = (int)(t % NT);
  const int64_t kb = t / NT;
  const int col = 16 * nt + (lane & 15);
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const int64_t k = 16 * kb + 4 * (lane >> 4) + s;
    P[idx * 4 + s] = (k < K && col < l) ? (float)S[k * lds + col] : 0.0f;
  }
}

// f32 rows of Q padded to L = 16 NT columns and to whole row quads: P[r*L + c]
__global__ void k_pack_f32_rows(const double* __restrict__ S, int64_t K, int l, int lds, int L,
                                int64_t Kpad, float* __restrict__ P) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= Kpad * L) return;
  const int64_t r = idx / L;
  const int c = (int)(idx - r * L);
  P[idx] = (r < K && c < l) ? (float)S[r * lds + c] : 0.0f;
}

// Exact three-way bfloat16 split of float32 values, a pair at a time: x = x1 + x2 + x3,
// each piece the nearest bfloat16 of what is left (a float32 significand has 24 bits =
// 3 x 8).  The pieces come as packed bfloat16 pairs (low half = x0): one packed
// round-to-nearest-even conversion per piece and pair; a piece is widened back to float32
// with a shift (low half) or a mask (high half), both exact.
typedef float f32x2v __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2v __attribute__((ext_vector_type(2)));
typedef unsigned u32x4v __attribute__((ext_vector_type(4)));
__device__ __forceinline__ unsigned cvt_pk_bf16(float x0, float x1) {
  return __builtin_bit_cast(unsigned, __builtin_convertvector(f32x2v{x0, x1}, bf16x2v));
}
__device__ __forceinline__ float bf16_lo(unsigned w) { return __uint_as_float(w << 16); }
__device__ __forceinline__ float bf16_hi(unsigned w) { return __uint_as_float(w & 0xffff0000u); }

template <int PIECES>
__device__ __forceinline__ void split_pk(float x0, float x1, unsigned (&w)[PIECES]) {
  w[0] = cvt_pk_bf16(x0, x1);
  if (PIECES == 3) {
    const float r0 = x0 - bf16_lo(w[0]), r1 = x1 - bf16_hi(w[0]);
    w[1 % PIECES] = cvt_pk_bf16(r0, r1);
    w[2 % PIECES] = cvt_pk_bf16(r0 - bf16_lo(w[1 % PIECES]), r1 - bf16_hi(w[1 % PIECES]));
  }
}

// Three bfloat16 pieces of the float64 operand, each the nearest bfloat16 of what is left
// (x = x1 + x2 + x3 + O(2^-24 |x|)): P[piece * nfrag + frag] (piece 0..2).
__global__ void k_pack_bf16x3(const double* __restrict__ S, int64_t K, int l, int lds, int NT,
                              int64_t nkb, bf16x8* __restrict__ P) {
  const int64_t nfrag = nkb * NT * 64;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= nfrag) return;
  const int lane = (int)(idx & 63);
  const int64_t t = idx >> 6;
  const int nt = (int)(t % NT);
  const int64_t kb = t / NT;
  const int col = 16 * nt + (lane & 15);
  const int64_t k0 = 32 * kb + 8 * (lane >> 4);
  bf16x8 v1, v2, v3;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const int64_t k = k0 + e;
    const double x = (k < K && col < l) ? S[k * lds + col] : 0.0;
    const __bf16 x1 = (__bf16)x;
    const double r1 = x - (double)x1;
    const __bf16 x2 = (__bf16)r1;
    const double r2 = r1 - (double)x2;
    v1[e] = x1;
    v2[e] = x2;
    v3[e] = (__bf16)r2;
  }
  P[idx] = v1;
  P[nfrag + idx] = v2;
  P[2 * nfrag + idx] = v3;
}

__device__ __forceinline__ bool aligned16(const void* p) {
  return (reinterpret_cast<uintptr_t>(p) & 15) == 0;
}

// ---------------------------------------------------------------- Y = A X, bf16
// PIECES = 1: bfloat16 inputs.  PIECES = 3: A and X split exactly into three bfloat16
// pieces; the six products a1x1 + a1x2 + a2x1 + a2x2 + a1x3 + a3x1 (all terms down to
// relative weight 2^-24) give float32-input accuracy at bfloat16 matrix-core rate.
//
// Wave w owns rows base + 16*(RT*w + rt) + (0..15).  Per step of 32 along k, lane
// (i = lane%16, g = lane/16) reads A[row][32kb + 8g .. 32kb + 8g + 7] (two 16-byte loads
// when VEC: A 16-byte aligned and lda a multiple of 4).  The main loop runs over the full
// steps with no bounds tests (rows past m read row m-1 and are not stored); a ragged last
// step reads with tests.  The A and X fragments of step kb+1 are loaded before the
// products of step kb.
//
// The products, smallest first into every accumulator (the same order per accumulator
// either way); PMAJOR (product-major) keeps consecutive matrix-core instructions
// independent, which suits Y = A X, while A^T Q runs faster tile-major.
template <int R, int NT, int PIECES, bool PMAJOR>
__device__ __forceinline__ void mfma_pieces(const bf16x8 (&a)[PIECES][R],
                                            const bf16x8 (&b)[PIECES][NT],
                                            f32x4 (&acc)[R][NT]) {
  constexpr int np = PIECES == 3 ? 6 : 1;
  // product q: piece pa(q) of A times piece pb(q) of the other operand
  auto pa = [](int q) { return (q == 0 ? 2 : q == 2 || q == 3 ? 1 : 0) % PIECES; };
  auto pb = [](int q) { return (q == 1 ? 2 : q == 2 || q == 4 ? 1 : 0) % PIECES; };
  if (PMAJOR) {
#pragma unroll
    for (int q = 6 - np; q < 6; ++q)
#pragma unroll
      for (int r = 0; r < R; ++r)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
          acc[r][nt] = mfma_bf16(a[pa(q)][r], b[pb(q)][nt], acc[r][nt]);
  } else {
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int nt = 0; nt < NT; ++nt)
#pragma unroll
        for (int q = 6 - np; q < 6; ++q)
          acc[r][nt] = mfma_bf16(a[pa(q)][r], b[pb(q)][nt], acc[r][nt]);
  }
}

template <int R, int PIECES>
__device__ __forceinline__ void to_pieces_rows(const float (&v)[R][8], bf16x8 (&a)[PIECES][R]) {
  if (PIECES == 1) {
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int e = 0; e < 8; ++e) a[0][r][e] = (__bf16)v[r][e];
    return;
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    unsigned w[4][PIECES];
#pragma unroll
    for (int q = 0; q < 4; ++q) split_pk<PIECES>(v[r][2 * q], v[r][2 * q + 1], w[q]);
#pragma unroll
    for (int pc = 0; pc < PIECES; ++pc)
      a[pc][r] = __builtin_bit_cast(bf16x8, u32x4v{w[0][pc], w[1][pc], w[2][pc], w[3][pc]});
  }
}

template <int RT, int NT, int PIECES, bool VEC>
__global__ __launch_bounds__(256) void k_ax_bf16(const float* __restrict__ A, int64_t lda,
                                                 int64_t m, int n,
                                                 const bf16x8* __restrict__ Xp, int64_t nfrag,
                                                 int l, double* __restrict__ Y, int ldy) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, g = lane >> 4;
  const int64_t rbase = (int64_t)blockIdx.x * (64 * RT) + (int64_t)wave * (16 * RT);
  f32x4 acc[RT][NT];
#pragma unroll
  for (int rt = 0; rt < RT; ++rt)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) acc[rt][nt] = f32x4{0.f, 0.f, 0.f, 0.f};
  const float* arow[RT];
#pragma unroll
  for (int rt = 0; rt < RT; ++rt) {
    const int64_t row = rbase + 16 * rt + li;
    arow[rt] = A + (row < m ? row : m - 1) * lda + 8 * g;
  }
  const bf16x8* xp = Xp + lane;
  auto load_a = [&](int kb, float (&v)[RT][8]) {
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
      const float* p = arow[rt] + 32 * kb;
      if (VEC) {
        const float4 x0 = *reinterpret_cast<const float4*>(p);
        const float4 x1 = *reinterpret_cast<const float4*>(p + 4);
        v[rt][0] = x0.x; v[rt][1] = x0.y; v[rt][2] = x0.z; v[rt][3] = x0.w;
        v[rt][4] = x1.x; v[rt][5] = x1.y; v[rt][6] = x1.z; v[rt][7] = x1.w;
      } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) v[rt][e] = p[e];
      }
    }
  };
  auto load_b = [&](int kb, bf16x8 (&b)[PIECES][NT]) {
#pragma unroll
    for (int pc = 0; pc < PIECES; ++pc)
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) b[pc][nt] = xp[pc * nfrag + ((int64_t)kb * NT + nt) * 64];
  };
  // One piece: X fragments are shared by the four waves: a step's NT*64 fragments are loaded
  // once per workgroup (each thread its share, with the step's A), stored to LDS slot
  // kb & 1 when the step comes up and read back by every wave after a barrier.  Slot s is
  // rewritten only after the next step's barrier, which every wave reaches after its reads.
  constexpr int FS = NT * 64;            // fragments per piece and step
  constexpr int FR = PIECES * FS;        // per step
  constexpr int FPT = (FR + 255) / 256;  // loaded per thread
  __shared__ bf16x8 xs[2][FR];
  const int tid = threadIdx.x;
  auto load_x = [&](int kb, bf16x8 (&x)[FPT]) {
#pragma unroll
    for (int u = 0; u < FPT; ++u) {
      const int f = tid + 256 * u;
      if (FR % 256 == 0 || f < FR) {
        const int pc = f / FS;
        x[u] = Xp[pc * nfrag + (int64_t)kb * FS + (f - pc * FS)];
      }
    }
  };
  auto stage = [&](int slot, const bf16x8 (&x)[FPT], bf16x8 (&b)[PIECES][NT]) {
#pragma unroll
    for (int u = 0; u < FPT; ++u) {
      const int f = tid + 256 * u;
      if (FR % 256 == 0 || f < FR) xs[slot][f] = x[u];
    }
    __syncthreads();
#pragma unroll
    for (int pc = 0; pc < PIECES; ++pc)
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) b[pc][nt] = xs[slot][pc * FS + nt * 64 + lane];
  };
  // Two register sets, two steps in flight: the products of step kb run while the loads of
  // step kb+1 are outstanding.  Step kb+2's A and X shares are loaded into step kb's
  // registers as soon as A is split into pieces and the shares are in LDS (scheduling
  // barriers keep the compiler from hoisting loads above the products, which would make the
  // wait for one step also wait for the next).  Steps past the last are clamped to it (a
  // harmless reload).
  const int nfull = n >> 5;
  if constexpr (PIECES == 1) {
    if (nfull > 0) {
      float v0[RT][8], v1[RT][8];
      bf16x8 x0[FPT], x1[FPT];
      const int last = nfull - 1;
      load_a(0, v0);
      load_x(0, x0);
      load_a(last < 1 ? last : 1, v1);
      load_x(last < 1 ? last : 1, x1);
      bf16x8 a[PIECES][RT], b[PIECES][NT];
      int kb = 0;
      for (; kb + 2 <= nfull; kb += 2) {
        stage(0, x0, b);
        to_pieces_rows<RT, PIECES>(v0, a);
        __builtin_amdgcn_sched_barrier(0);
        const int k2 = (kb + 2 < last) ? kb + 2 : last;
        load_a(k2, v0);
        load_x(k2, x0);
        __builtin_amdgcn_sched_barrier(0);
        mfma_pieces<RT, NT, PIECES, true>(a, b, acc);
        __builtin_amdgcn_sched_barrier(0);
        stage(1, x1, b);
        to_pieces_rows<RT, PIECES>(v1, a);
        __builtin_amdgcn_sched_barrier(0);
        const int k3 = (kb + 3 < last) ? kb + 3 : last;
        load_a(k3, v1);
        load_x(k3, x1);
        __builtin_amdgcn_sched_barrier(0);
        mfma_pieces<RT, NT, PIECES, true>(a, b, acc);
        __builtin_amdgcn_sched_barrier(0);
      }
      if (kb < nfull) {
        stage(0, x0, b);
        to_pieces_rows<RT, PIECES>(v0, a);
        mfma_pieces<RT, NT, PIECES, true>(a, b, acc);
      }
    }
  } else if (nfull > 0) {
    // three pieces (occupancy 1, long steps): each wave loads its own X fragments, which
    // measured faster than a barrier per step
    float v0[RT][8], v1[RT][8];
    bf16x8 b0[PIECES][NT], b1[PIECES][NT];
    const int last = nfull - 1;
    load_a(0, v0);
    load_b(0, b0);
    load_a(last < 1 ? last : 1, v1);
    load_b(last < 1 ? last : 1, b1);
    bf16x8 a[PIECES][RT];
    int kb = 0;
    for (; kb + 2 <= nfull; kb += 2) {
      to_pieces_rows<RT, PIECES>(v0, a);
      __builtin_amdgcn_sched_barrier(0);
      const int k2 = (kb + 2 < last) ? kb + 2 : last;
      load_a(k2, v0);
      __builtin_amdgcn_sched_barrier(0);
      mfma_pieces<RT, NT, PIECES, true>(a, b0, acc);
      __builtin_amdgcn_sched_barrier(0);
      load_b(k2, b0);
      __builtin_amdgcn_sched_barrier(0);
      to_pieces_rows<RT, PIECES>(v1, a);
      __builtin_amdgcn_sched_barrier(0);
      const int k3 = (kb + 3 < last) ? kb + 3 : last;
      load_a(k3, v1);
      __builtin_amdgcn_sched_barrier(0);
      mfma_pieces<RT, NT, PIECES, true>(a, b1, acc);
      __builtin_amdgcn_sched_barrier(0);
      load_b(k3, b1);
      __builtin_amdgcn_sched_barrier(0);
    }
    if (kb < nfull) {
      to_pieces_rows<RT, PIECES>(v0, a);
      mfma_pieces<RT, NT, PIECES, true>(a, b0, acc);
    }
  }
  if ((nfull << 5) < n) {
    // ragged last step: columns past n read as 0 (the packed X rows there are 0 as well)
    const int k0 = (nfull << 5) + 8 * g;
    float v[RT][8];
    bf16x8 b[PIECES][NT];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
      for (int e = 0; e < 8; ++e) v[rt][e] = (k0 + e < n) ? arow[rt][32 * nfull + e] : 0.f;
    load_b(nfull, b);
    bf16x8 a[PIECES][RT];
    to_pieces_rows<RT, PIECES>(v, a);
    mfma_pieces<RT, NT, PIECES, true>(a, b, acc);
  }
#pragma unroll
  for (int rt = 0; rt < RT; ++rt)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      const int col = 16 * nt + li;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = rbase + 16 * rt + 4 * g + r;
        if (row < m && col < l) Y[row * ldy + col] = (double)acc[rt][nt][r];
      }
    }
}

// ---------------------------------------------------------------- Y = A X, f32
template <int RT, int NT>
__global__ __launch_bounds__(256) void k_ax_f32(const float* __restrict__ A, int64_t lda,
                                                int64_t m, int n, const float* __restrict__ Xp,
                                                int l, double* __restrict__ Y, int ldy) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, g = lane >> 4;
  const int64_t rbase = (int64_t)blockIdx.x * (64 * RT) + (int64_t)wave * (16 * RT);
  f32x4 acc[RT][NT];
#pragma unroll
  for (int rt = 0; rt < RT; ++rt)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) acc[rt][nt] = f32x4{0.f, 0.f, 0.f, 0.f};
  const float* arow[RT];
  bool rok[RT];
#pragma unroll
  for (int rt = 0; rt < RT; ++rt) {
    const int64_t row = rbase + 16 * rt + li;
    rok[rt] = row < m;
    arow[rt] = A + (rok[rt] ? row : 0) * lda;
  }
  const int nkb = (n + 15) / 16;
  for (int kb = 0; kb < nkb; ++kb) {
    const int k0 = 16 * kb + 4 * g;
    float a[RT][4];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
      const float* p = arow[rt] + k0;
      if (rok[rt] && k0 + 4 <= n && aligned16(p)) {
        const float4 x = *reinterpret_cast<const float4*>(p);
        a[rt][0] = x.x; a[rt][1] = x.y; a[rt][2] = x.z; a[rt][3] = x.w;
      } else {
#pragma unroll
        for (int s = 0; s < 4; ++s) a[rt][s] = (rok[rt] && k0 + s < n) ? p[s] : 0.0f;
      }
    }
    float4 b[NT];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt)
      b[nt] = reinterpret_cast<const float4*>(Xp)[((int64_t)kb * NT + nt) * 64 + lane];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        acc[rt][nt] = mfma_f32(a[rt][0], b[nt].x, acc[rt][nt]);
        acc[rt][nt] = mfma_f32(a[rt][1], b[nt].y, acc[rt][nt]);
        acc[rt][nt] = mfma_f32(a[rt][2], b[nt].z, acc[rt][nt]);
        acc[rt][nt] = mfma_f32(a[rt][3], b[nt].w, acc[rt][nt]);
      }
  }
#pragma unroll
  for (int rt = 0; rt < RT; ++rt)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      const int col = 16 * nt + li;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = rbase + 16 * rt + 4 * g + r;
        if (row < m && col < l) Y[row * ldy + col] = (double)acc[rt][nt][r];
      }
    }
}

// ---------------------------------------------------------------- Z = A^T Q, bf16 / f32
// Workgroup = (row chunk, 256-column tile), wave w owns 64 columns cw = c0 + 64 w.
constexpr int MX_COLS = 256;
#ifndef AX_RT
#define AX_RT 4
#endif
#ifndef AX_RT3
#define AX_RT3 8  // rows per wave 128: halves the fragment bytes per byte of A (occupancy 1 either way)
#endif

__device__ __forceinline__ void mx_tile(int total, int ncol, int& chunk, int& ct, bool& ok) {
  const int per = (total + 7) / 8;
  const int L = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
  ok = L < total;
  chunk = ok ? L / ncol : 0;
  ct = ok ? L - chunk * ncol : 0;
}

// Z = A^T Q with bfloat16 pieces.  Per step of 32 rows, lane (i, g) reads the four
// columns cb = cw + 4i .. cb+3 of rows rb + 8g + t (t < 8); MFMA tile e takes column
// cb + e, k-slot (g, t) row rb + 8g + t.  Full steps run without bounds tests when FC;
// the ragged last rows of the matrix are tested.
template <int PIECES>
__device__ __forceinline__ void to_pieces_cols(const float (&v)[8][4], bf16x8 (&a)[PIECES][4]) {
  if (PIECES == 1) {
#pragma unroll
    for (int t = 0; t < 8; ++t)
#pragma unroll
      for (int e = 0; e < 4; ++e) a[0][e][t] = (__bf16)v[t][e];
    return;
  }
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    unsigned w[4][PIECES];
#pragma unroll
    for (int q = 0; q < 4; ++q) split_pk<PIECES>(v[2 * q][e], v[2 * q + 1][e], w[q]);
#pragma unroll
    for (int pc = 0; pc < PIECES; ++pc)
      a[pc][e] = __builtin_bit_cast(bf16x8, u32x4v{w[0][pc], w[1][pc], w[2][pc], w[3][pc]});
  }
}

// Each wave loads its own Q fragments (three pieces: occupancy 1 and long steps, where a
// barrier per step measured slower).
template <int NT, int PIECES, bool FC>
__device__ __forceinline__ void atq_rows_own(const float* __restrict__ A, int64_t lda, int n,
                                         int cb, int g, int64_t r0, int64_t r1,
                                         const bf16x8* __restrict__ qp, int64_t nfrag,
                                         f32x4 (&acc)[4][NT]) {
  auto load_a = [&](int64_t rb, float (&v)[8][4]) {
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const float* p = A + (rb + 8 * g + t) * lda + cb;
      if (FC) {
        const float4 x = *reinterpret_cast<const float4*>(p);
        v[t][0] = x.x; v[t][1] = x.y; v[t][2] = x.z; v[t][3] = x.w;
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) v[t][e] = (cb + e < n) ? p[e] : 0.f;
      }
    }
  };
  auto load_b = [&](int64_t rb, bf16x8 (&b)[PIECES][NT]) {
    const int64_t kb = rb >> 5;
#pragma unroll
    for (int pc = 0; pc < PIECES; ++pc)
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) b[pc][nt] = qp[pc * nfrag + (kb * NT + nt) * 64];
  };
  const int64_t rfull = r0 + (((r1 - r0) >> 5) << 5);
  if (rfull > r0) {
    // two register sets, two steps in flight (as in Y = A X)
    float v0[8][4], v1[8][4];
    bf16x8 b0[PIECES][NT], b1[PIECES][NT];
    const int64_t last = rfull - 32;
    load_a(r0, v0);
    load_b(r0, b0);
    const int64_t r1st = (r0 + 32 < last) ? r0 + 32 : last;
    load_a(r1st, v1);
    load_b(r1st, b1);
    bf16x8 a[PIECES][4];
    int64_t rb = r0;
    for (; rb + 64 <= rfull; rb += 64) {
      to_pieces_cols<PIECES>(v0, a);
      __builtin_amdgcn_sched_barrier(0);
      const int64_t r2 = (rb + 64 < last) ? rb + 64 : last;
      load_a(r2, v0);
      __builtin_amdgcn_sched_barrier(0);
      mfma_pieces<4, NT, PIECES, false>(a, b0, acc);
      __builtin_amdgcn_sched_barrier(0);
      load_b(r2, b0);
      __builtin_amdgcn_sched_barrier(0);
      to_pieces_cols<PIECES>(v1, a);
      __builtin_amdgcn_sched_barrier(0);
      const int64_t r3 = (rb + 96 < last) ? rb + 96 : last;
      load_a(r3, v1);
      __builtin_amdgcn_sched_barrier(0);
      mfma_pieces<4, NT, PIECES, false>(a, b1, acc);
      __builtin_amdgcn_sched_barrier(0);
      load_b(r3, b1);
      __builtin_amdgcn_sched_barrier(0);
    }
    if (rb < rfull) {
      to_pieces_cols<PIECES>(v0, a);
      mfma_pieces<4, NT, PIECES, false>(a, b0, acc);
    }
  }
  if (rfull < r1) {
    // ragged last rows (only the chunk that ends at m): rows past r1 read as 0
    float v[8][4];
    bf16x8 b[PIECES][NT];
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int64_t row = rfull + 8 * g + t;
      const float* p = A + row * lda + cb;
#pragma unroll
      for (int e = 0; e < 4; ++e) v[t][e] = (row < r1 && cb + e < n) ? p[e] : 0.f;
    }
    load_b(rfull, b);
    bf16x8 a[PIECES][4];
    to_pieces_cols<PIECES>(v, a);
    mfma_pieces<4, NT, PIECES, false>(a, b, acc);
  }
}

// One piece: the Q fragments of a 32-row step (NT*64) are shared by the four waves through
// a two-slot LDS ring as in Y = A X, so all four waves run the loop; a wave with wact false
// (its columns lie past n) loads no A.
template <int NT, int PIECES, bool FC>
__device__ __forceinline__ void atq_rows(const float* __restrict__ A, int64_t lda, int n,
                                         int cb, int g, bool wact, int64_t r0, int64_t r1,
                                         const bf16x8* __restrict__ Qp, int64_t nfrag,
                                         bf16x8 (*qs)[PIECES * NT * 64], f32x4 (&acc)[4][NT]) {
  static_assert(PIECES == 1, "three pieces use atq_rows_own");
  constexpr int FS = NT * 64;
  constexpr int FR = PIECES * FS;
  constexpr int FPT = (FR + 255) / 256;
  const int tid = threadIdx.x, lane = tid & 63;
  auto load_a = [&](int64_t rb, float (&v)[8][4]) {
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const float* p = A + (rb + 8 * g + t) * lda + cb;
      if (FC) {
        float4 x = make_float4(0.f, 0.f, 0.f, 0.f);
        if (wact) x = *reinterpret_cast<const float4*>(p);
        v[t][0] = x.x; v[t][1] = x.y; v[t][2] = x.z; v[t][3] = x.w;
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) v[t][e] = (wact && cb + e < n) ? p[e] : 0.f;
      }
    }
  };
  auto load_x = [&](int64_t rb, bf16x8 (&x)[FPT]) {
    const int64_t kb = rb >> 5;
#pragma unroll
    for (int u = 0; u < FPT; ++u) {
      const int f = tid + 256 * u;
      if (FR % 256 == 0 || f < FR) {
        const int pc = f / FS;
        x[u] = Qp[pc * nfrag + kb * FS + (f - pc * FS)];
      }
    }
  };
  auto stage = [&](int slot, const bf16x8 (&x)[FPT], bf16x8 (&b)[PIECES][NT]) {
#pragma unroll
    for (int u = 0; u < FPT; ++u) {
      const int f = tid + 256 * u;
      if (FR % 256 == 0 || f < FR) qs[slot][f] = x[u];
    }
    __syncthreads();
#pragma unroll
    for (int pc = 0; pc < PIECES; ++pc)
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) b[pc][nt] = qs[slot][pc * FS + nt * 64 + lane];
  };
  // Order of the sums (the same in the kernel that reads the bfloat16 copy of A, so the two
  // agree bit for bit): the ragged last rows first (only the chunk that ends at m; rows past
  // r1 read as 0, and with no ragged rows the step is all zeros), then the whole 32-row
  // steps in order, an odd one first on its own.  All MFMAs before the paired loop: MFMAs
  // after it make the compiler copy the accumulators in and out on every iteration.
  const int64_t rfull = r0 + (((r1 - r0) >> 5) << 5);
  {
    float v[8][4];
    bf16x8 b[PIECES][NT];
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int64_t row = rfull + 8 * g + t;
      const float* p = A + row * lda + cb;
#pragma unroll
      for (int e = 0; e < 4; ++e) v[t][e] = (wact && row < r1 && cb + e < n) ? p[e] : 0.f;
    }
    const int64_t kb = rfull < r1 ? rfull >> 5 : 0;
#pragma unroll
    for (int pc = 0; pc < PIECES; ++pc)
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) b[pc][nt] = Qp[pc * nfrag + kb * FS + nt * 64 + lane];
    bf16x8 a[PIECES][4];
    to_pieces_cols<PIECES>(v, a);
    mfma_pieces<4, NT, PIECES, false>(a, b, acc);
  }
  const int64_t nsteps = (rfull - r0) >> 5;
  {
    float v[8][4];
    bf16x8 x[FPT], b[PIECES][NT], a[PIECES][4];
    if (nsteps & 1) {
      load_a(r0, v);
      load_x(r0, x);
    } else {
#pragma unroll
      for (int t = 0; t < 8; ++t)
#pragma unroll
        for (int e = 0; e < 4; ++e) v[t][e] = 0.f;
#pragma unroll
      for (int u = 0; u < FPT; ++u) x[u] = __builtin_bit_cast(bf16x8, u32x4v{0u, 0u, 0u, 0u});
    }
    stage(1, x, b);  // slot 1: the loop's first barrier comes before its next write
    to_pieces_cols<PIECES>(v, a);
    mfma_pieces<4, NT, PIECES, false>(a, b, acc);
  }
  if (nsteps > 1) {
    // two register sets, two steps in flight (as in Y = A X)
    float v0[8][4], v1[8][4];
    bf16x8 x0[FPT], x1[FPT];
    const int64_t last = rfull - 32;
    const int64_t rs = r0 + 32 * (nsteps & 1);  // first step of the pairs
    load_a(rs, v0);
    load_x(rs, x0);
    __builtin_amdgcn_sched_barrier(0);  // the same load order as in the loop
    load_a(rs + 32, v1);
    load_x(rs + 32, x1);
    __builtin_amdgcn_sched_barrier(0);
    bf16x8 a[PIECES][4], b[PIECES][NT];
    for (int64_t rb = rs; rb + 64 <= rfull; rb += 64) {
      stage(0, x0, b);
      to_pieces_cols<PIECES>(v0, a);
      __builtin_amdgcn_sched_barrier(0);
      const int64_t r2 = (rb + 64 < last) ? rb + 64 : last;
      load_a(r2, v0);
      load_x(r2, x0);
      __builtin_amdgcn_sched_barrier(0);
      mfma_pieces<4, NT, PIECES, false>(a, b, acc);
      __builtin_amdgcn_sched_barrier(0);
      stage(1, x1, b);
      to_pieces_cols<PIECES>(v1, a);
      __builtin_amdgcn_sched_barrier(0);
      const int64_t r3 = (rb + 96 < last) ? rb + 96 : last;
      load_a(r3, v1);
      load_x(r3, x1);
      __builtin_amdgcn_sched_barrier(0);
      mfma_pieces<4, NT, PIECES, false>(a, b, acc);
      __builtin_amdgcn_sched_barrier(0);
    }
  }
}

// FC: every wave's 64 columns lie inside A and rows are 16-byte aligned (n a multiple of
// 64, A 16-byte aligned, lda a multiple of 4); otherwise every load is tested.
template <int NT, int PIECES, bool FC>
__global__ __launch_bounds__(256) void k_atq_bf16(const float* __restrict__ A, int64_t lda,
                                                  int64_t m, int n,
                                                  const bf16x8* __restrict__ Qp, int64_t nfrag,
                                                  int l, int ncol, int nchunk, int64_t chunk_rows,
                                                  double* __restrict__ part) {
  int chunk, ct;
  bool ok;
  mx_tile(ncol * nchunk, ncol, chunk, ct, ok);
  if (!ok) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, g = lane >> 4;
  const int cw = ct * MX_COLS + 64 * wave;
  const bool wact = cw < n;
  const int64_t r0 = (int64_t)chunk * chunk_rows;  // chunk_rows is a multiple of 32
  const int64_t r1 = (r0 + chunk_rows < m) ? r0 + chunk_rows : m;
  const int cb = cw + 4 * li;
  __shared__ bf16x8 qs[2][PIECES == 1 ? NT * 64 : 1];
  f32x4 acc[4][NT];
#pragma unroll
  for (int e = 0; e < 4; ++e)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) acc[e][nt] = f32x4{0.f, 0.f, 0.f, 0.f};
  if constexpr (PIECES == 1) {
    atq_rows<NT, PIECES, FC>(A, lda, n, cb, g, wact, r0, r1, Qp, nfrag, qs, acc);
    if (!wact) return;
  } else {
    if (!wact) return;
    atq_rows_own<NT, PIECES, FC>(A, lda, n, cb, g, r0, r1, Qp + lane, nfrag, acc);
  }
  double* P = part + (int64_t)chunk * n * l;
#pragma unroll
  for (int e = 0; e < 4; ++e)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      const int col = 16 * nt + li;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int c = cw + 4 * (4 * g + r) + e;
        if (c < n && col < l) P[(int64_t)c * l + col] = (double)acc[e][nt][r];
      }
    }
}

template <int NT>
__global__ __launch_bounds__(256) void k_atq_f32(const float* __restrict__ A, int64_t lda,
                                                 int64_t m, int n, const float* __restrict__ Qf,
                                                 int l, int ncol, int nchunk,
                                                 int64_t chunk_rows, double* __restrict__ part) {
  int chunk, ct;
  bool ok;
  mx_tile(ncol * nchunk, ncol, chunk, ct, ok);
  if (!ok) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, g = lane >> 4;
  const int cw = ct * MX_COLS + 64 * wave;
  if (cw >= n) return;
  constexpr int L = 16 * NT;
  const int64_t r0 = (int64_t)chunk * chunk_rows;
  const int64_t r1 = (r0 + chunk_rows < m) ? r0 + chunk_rows : m;
  const int cb = cw + 4 * li;
  const bool cvec = (cb + 4 <= n);
  f32x4 acc[4][NT];
#pragma unroll
  for (int e = 0; e < 4; ++e)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) acc[e][nt] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int64_t rq = r0; rq < r1; rq += 4) {
    const int64_t row = rq + g;
    const float* p = A + row * lda + cb;
    float v0 = 0.f, v1 = 0.f, v2 = 0.f, v3 = 0.f;
    if (row < r1) {
      if (cvec && aligned16(p)) {
        const float4 x = *reinterpret_cast<const float4*>(p);
        v0 = x.x; v1 = x.y; v2 = x.z; v3 = x.w;
      } else {
        v0 = (cb + 0 < n) ? p[0] : 0.f;
        v1 = (cb + 1 < n) ? p[1] : 0.f;
        v2 = (cb + 2 < n) ? p[2] : 0.f;
        v3 = (cb + 3 < n) ? p[3] : 0.f;
      }
    }
    float b[NT];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) b[nt] = Qf[row * L + 16 * nt + li];  // rows padded
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      acc[0][nt] = mfma_f32(v0, b[nt], acc[0][nt]);
      acc[1][nt] = mfma_f32(v1, b[nt], acc[1][nt]);
      acc[2][nt] = mfma_f32(v2, b[nt], acc[2][nt]);
      acc[3][nt] = mfma_f32(v3, b[nt], acc[3][nt]);
    }
  }
  double* P = part + (int64_t)chunk * n * l;
#pragma unroll
  for (int e = 0; e < 4; ++e)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      const int col = 16 * nt + li;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int c = cw + 4 * (4 * g + r) + e;
        if (c < n && col < l) P[(int64_t)c * l + col] = (double)acc[e][nt][r];
      }
    }
}

// ---------------------------------------------------------------- bfloat16 copy of A
// The power steps round A to bfloat16 in every pass.  The first pass can store the rounded
// values once (row-major, leading dimension ldc = n rounded up to 64, zero-padded), and
// the later power steps then stream that copy: half the bytes, bit-identical products.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// Power-step Y = A X from the float32 A with the paired k layout (X packed as MIX_BF16P):
// per 64-column group a lane reads 16 consecutive floats of each of its rows (four 16-byte
// loads, 256 bytes per row across the four lane groups) and rounds them to bfloat16 for
// two MFMAs.  With CW (first pass) it also stores those 32 bytes to the copy (128
// contiguous bytes per row): long runs in both directions.
template <int RT, int NT, bool VEC, bool CW>
__global__ __launch_bounds__(256) void k_ax_bf16p(const float* __restrict__ A, int64_t lda,
                                                  int64_t m, int n,
                                                  const bf16x8* __restrict__ Xp, int l,
                                                  double* __restrict__ Y, int ldy,
                                                  bf16x8* __restrict__ Ac, int64_t ldc8) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, g = lane >> 4;
  const int64_t rbase = (int64_t)blockIdx.x * (64 * RT) + (int64_t)wave * (16 * RT);
  f32x4 acc[RT][NT];
#pragma unroll
  for (int rt = 0; rt < RT; ++rt)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) acc[rt][nt] = f32x4{0.f, 0.f, 0.f, 0.f};
  const float* arow[RT];
  bf16x8* crow[RT];
#pragma unroll
  for (int rt = 0; rt < RT; ++rt) {
    const int64_t row = rbase + 16 * rt + li;
    arow[rt] = A + (row < m ? row : m - 1) * lda + 16 * g;
    crow[rt] = (CW && row < m) ? Ac + row * ldc8 + 2 * g : nullptr;
  }
  const bf16x8* xp = Xp + lane;
  auto load_a = [&](int kg, float (&v)[RT][16]) {
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
      const float* p = arow[rt] + 64 * kg;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        if (VEC) {
          const float4 x = *reinterpret_cast<const float4*>(p + 4 * q);
          v[rt][4 * q] = x.x; v[rt][4 * q + 1] = x.y; v[rt][4 * q + 2] = x.z; v[rt][4 * q + 3] = x.w;
        } else {
#pragma unroll
          for (int e = 0; e < 4; ++e) v[rt][4 * q + e] = p[4 * q + e];
        }
      }
    }
  };
  auto load_b = [&](int kg, bf16x8 (&b)[2][NT]) {
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) b[j][nt] = xp[((int64_t)(2 * kg + j) * NT + nt) * 64];
  };
  auto products = [&](const float (&v)[RT][16], const bf16x8 (&b)[2][NT], int kg) {
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
      bf16x8 a[2];
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int e = 0; e < 8; ++e) a[j][e] = (__bf16)v[rt][8 * j + e];
      if (CW && crow[rt]) {
        crow[rt][8 * kg] = a[0];
        crow[rt][8 * kg + 1] = a[1];
      }
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) acc[rt][nt] = mfma_bf16(a[j], b[j][nt], acc[rt][nt]);
    }
  };
  // X fragments of a group (2*NT*64, contiguous) are shared by the four waves through a
  // two-slot LDS ring, as in k_ax_bf16c.
  constexpr int FR = 2 * NT * 64;
  constexpr int FPT = (FR + 255) / 256;
  __shared__ bf16x8 xs[2][FR];
  const int tid = threadIdx.x;
  auto load_x = [&](int kg, bf16x8 (&x)[FPT]) {
    const bf16x8* src = Xp + (int64_t)kg * FR;
#pragma unroll
    for (int u = 0; u < FPT; ++u)
      if (FR % 256 == 0 || tid + 256 * u < FR) x[u] = src[tid + 256 * u];
  };
  auto stage = [&](int slot, const bf16x8 (&x)[FPT], bf16x8 (&b)[2][NT]) {
#pragma unroll
    for (int u = 0; u < FPT; ++u)
      if (FR % 256 == 0 || tid + 256 * u < FR) xs[slot][tid + 256 * u] = x[u];
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) b[j][nt] = xs[slot][(j * NT + nt) * 64 + lane];
  };
  const int nfull = n >> 6;
  if (nfull > 0) {
    float v0[RT][16], v1[RT][16];
    bf16x8 x0[FPT], x1[FPT], b[2][NT];
    const int last = nfull - 1;
    load_a(0, v0);
    load_x(0, x0);
    load_a(last < 1 ? last : 1, v1);
    load_x(last < 1 ? last : 1, x1);
    int kg = 0;
    for (; kg + 2 <= nfull; kg += 2) {
      stage(0, x0, b);
      products(v0, b, kg);
      __builtin_amdgcn_sched_barrier(0);
      const int k2 = (kg + 2 < last) ? kg + 2 : last;
      load_a(k2, v0);
      load_x(k2, x0);
      __builtin_amdgcn_sched_barrier(0);
      stage(1, x1, b);
      products(v1, b, kg + 1);
      __builtin_amdgcn_sched_barrier(0);
      const int k3 = (kg + 3 < last) ? kg + 3 : last;
      load_a(k3, v1);
      load_x(k3, x1);
      __builtin_amdgcn_sched_barrier(0);
    }
    if (kg < nfull) {
      stage(0, x0, b);
      products(v0, b, kg);
    }
  }
  if ((nfull << 6) < n) {
    // ragged last group: columns past n read as 0 (zero padding of the copy, zero X rows)
    const int k0 = (nfull << 6) + 16 * g;
    float v[RT][16];
    bf16x8 b[2][NT];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
      for (int e = 0; e < 16; ++e) v[rt][e] = (k0 + e < n) ? arow[rt][64 * nfull + e] : 0.f;
    load_b(nfull, b);
    products(v, b, nfull);
  }
#pragma unroll
  for (int rt = 0; rt < RT; ++rt)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      const int col = 16 * nt + li;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = rbase + 16 * rt + 4 * g + r;
        if (row < m && col < l) Y[row * ldy + col] = (double)acc[rt][nt][r];
      }
    }
}

// Y = A X from the copy, paired k layout (X packed as MIX_BF16P): per 64-column group a
// lane reads its 16 consecutive values of a row as two adjacent 16-byte fragments, used by
// the two MFMAs as they are; same products in the same order as k_ax_bf16p, so the result
// is bitwise that of rounding the float32 A in the pass.  Rows past m read row m-1.
//
// The four waves need the same X fragments, so a group's fragments (2*NT*64, contiguous in
// Xp) are read from memory once per workgroup: thread t loads fragments t, t + 256, ... of
// group kg + 2 while group kg computes, and stores them to LDS slot kg & 1 when group kg + 2
// comes up; after a barrier every wave reads its B operands there.  Slot s is rewritten
// only after the barrier of the next group, which every wave reaches after its reads of s.
template <int RT, int NT>
__global__ __launch_bounds__(256) void k_ax_bf16c(const bf16x8* __restrict__ Ac, int64_t ldc8,
                                                  int64_t m, int ngroups,
                                                  const bf16x8* __restrict__ Xp, int l,
                                                  double* __restrict__ Y, int ldy) {
  constexpr int FR = 2 * NT * 64;         // X fragments per group
  constexpr int FPT = (FR + 255) / 256;   // loaded per thread
  __shared__ bf16x8 xs[2][FR];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, g = lane >> 4;
  const int64_t rbase = (int64_t)blockIdx.x * (64 * RT) + (int64_t)wave * (16 * RT);
  f32x4 acc[RT][NT];
#pragma unroll
  for (int rt = 0; rt < RT; ++rt)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) acc[rt][nt] = f32x4{0.f, 0.f, 0.f, 0.f};
  const bf16x8* arow[RT];
#pragma unroll
  for (int rt = 0; rt < RT; ++rt) {
    const int64_t row = rbase + 16 * rt + li;
    arow[rt] = Ac + (row < m ? row : m - 1) * ldc8 + 2 * g;
  }
  auto load = [&](int kg, bf16x8 (&a)[2][RT], bf16x8 (&x)[FPT]) {
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int rt = 0; rt < RT; ++rt) a[j][rt] = arow[rt][8 * kg + j];
    const bf16x8* src = Xp + (int64_t)kg * FR;
#pragma unroll
    for (int u = 0; u < FPT; ++u)
      if (FR % 256 == 0 || tid + 256 * u < FR) x[u] = src[tid + 256 * u];
  };
  auto products = [&](int slot, const bf16x8 (&a)[2][RT], const bf16x8 (&x)[FPT]) {
#pragma unroll
    for (int u = 0; u < FPT; ++u)
      if (FR % 256 == 0 || tid + 256 * u < FR) xs[slot][tid + 256 * u] = x[u];
    __syncthreads();
    bf16x8 b[2][NT];
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) b[j][nt] = xs[slot][(j * NT + nt) * 64 + lane];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) acc[rt][nt] = mfma_bf16(a[j][rt], b[j][nt], acc[rt][nt]);
  };
  // two register sets, two groups in flight (as in k_ax_bf16).  An odd group count does its
  // first group alone, before the loop (through LDS slot 1, which the loop's first barrier
  // protects): MFMAs after the loop would make the compiler copy the accumulators in and
  // out of it on every iteration.
  bf16x8 a0[2][RT], a1[2][RT], x0[FPT], x1[FPT];
  const int last = ngroups - 1;
  int kg = 0;
  if (ngroups & 1) {
    load(0, a0, x0);
    products(1, a0, x0);
    kg = 1;
  }
  load(kg < last ? kg : last, a0, x0);
  __builtin_amdgcn_sched_barrier(0);  // the same load order as in the loop
  load(kg + 1 < last ? kg + 1 : last, a1, x1);
  __builtin_amdgcn_sched_barrier(0);
  for (; kg + 2 <= ngroups; kg += 2) {
    products(0, a0, x0);
    __builtin_amdgcn_sched_barrier(0);
    load((kg + 2 < last) ? kg + 2 : last, a0, x0);
    __builtin_amdgcn_sched_barrier(0);
    products(1, a1, x1);
    __builtin_amdgcn_sched_barrier(0);
    load((kg + 3 < last) ? kg + 3 : last, a1, x1);
    __builtin_amdgcn_sched_barrier(0);
  }
#pragma unroll
  for (int rt = 0; rt < RT; ++rt)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      const int col = 16 * nt + li;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = rbase + 16 * rt + 4 * g + r;
        if (row < m && col < l) Y[row * ldy + col] = (double)acc[rt][nt][r];
      }
    }
}

// Z = A^T Q from the copy: lane (i, g) reads 4 columns (8 bytes) of rows rb + 8g + t and
// regroups them into the four MFMA fragments (tile e takes column cb + e), as k_atq_bf16.
template <int NT>
__device__ __forceinline__ void atqc_products(const uint2 (&v)[8], const bf16x8 (&b)[NT],
                                              f32x4 (&acc)[4][NT]) {
  bf16x8 a[4];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    u32x4 lo, hi;  // tiles 2h (low halves) and 2h+1 (high halves), rows t in pairs
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const unsigned x0 = h ? v[2 * j].y : v[2 * j].x;
      const unsigned x1 = h ? v[2 * j + 1].y : v[2 * j + 1].x;
      lo[j] = (x0 & 0xFFFFu) | (x1 << 16);
      hi[j] = (x0 >> 16) | (x1 & 0xFFFF0000u);
    }
    a[2 * h] = __builtin_bit_cast(bf16x8, lo);
    a[2 * h + 1] = __builtin_bit_cast(bf16x8, hi);
  }
#pragma unroll
  for (int e = 0; e < 4; ++e)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) acc[e][nt] = mfma_bf16(a[e], b[nt], acc[e][nt]);
}

// The Q fragments of a 32-row step (NT*64, contiguous) are shared by the four waves through
// LDS as in k_ax_bf16c, two steps per barrier, so every wave takes part in the loop; a
// wave whose columns lie past n reads no A (zeros) and stores nothing.
// At most two waves per SIMD: with the loads unconditional the kernel fits three, which
// measured slower on the 500,000 x 8,000 power steps (more streams in flight per channel).
template <int NT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 2))) void k_atq_bf16c(const __bf16* __restrict__ Ac, int64_t ldc,
                                                   int64_t m, int n,
                                                   const bf16x8* __restrict__ Qp, int l,
                                                   int ncol, int nchunk, int64_t chunk_rows,
                                                   double* __restrict__ part) {
  constexpr int FR = NT * 64;             // Q fragments per step
  constexpr int FPT = (FR + 255) / 256;   // loaded per thread
  __shared__ bf16x8 qs[2][2][FR];
  int chunk, ct;
  bool ok;
  mx_tile(ncol * nchunk, ncol, chunk, ct, ok);
  if (!ok) return;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, g = lane >> 4;
  const int cw = ct * MX_COLS + 64 * wave;
  const bool wact = cw < n;
  const int64_t r0 = (int64_t)chunk * chunk_rows;  // chunk_rows is a multiple of 32
  const int64_t r1 = (r0 + chunk_rows < m) ? r0 + chunk_rows : m;
  // lanes past the padded row read its last four entries: their columns are past n, and
  // results for columns past n are never stored (no lane condition on the loads)
  const int cb = cw + 4 * li;
  const int cbc = cb < ldc ? cb : ldc - 4;  // ldc is a multiple of 32
  f32x4 acc[4][NT];
#pragma unroll
  for (int e = 0; e < 4; ++e)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) acc[e][nt] = f32x4{0.f, 0.f, 0.f, 0.f};
  const bf16x8* qp = Qp + lane;
  // Q shares first: waiting for a step's shares then does not wait for its A
  auto load = [&](int64_t rb, uint2 (&v)[8], bf16x8 (&x)[FPT]) {
    const bf16x8* src = Qp + (rb >> 5) * FR;
#pragma unroll
    for (int u = 0; u < FPT; ++u)
      if (FR % 256 == 0 || tid + 256 * u < FR) x[u] = src[tid + 256 * u];
#pragma unroll
    for (int t = 0; t < 8; ++t)
      v[t] = *reinterpret_cast<const uint2*>(Ac + (rb + 8 * g + t) * ldc + cbc);
  };
  // both steps of a 64-row pair are staged together: one barrier per pair
  auto stage = [&](int slot, const bf16x8 (&x0)[FPT], const bf16x8 (&x1)[FPT]) {
#pragma unroll
    for (int u = 0; u < FPT; ++u)
      if (FR % 256 == 0 || tid + 256 * u < FR) {
        qs[slot][0][tid + 256 * u] = x0[u];
        qs[slot][1][tid + 256 * u] = x1[u];
      }
    __syncthreads();
  };
  auto products = [&](int slot, int h, const uint2 (&v)[8]) {
    bf16x8 b[NT];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) b[nt] = qs[slot][h][nt * 64 + lane];
    atqc_products<NT>(v, b, acc);
  };
  // The order of the sums is that of atq_rows (which rounds the float32 A to bfloat16 on
  // the fly), so both give the same bits: everything outside the paired loop first, as
  // straight-line MFMAs (MFMAs after the loop would make the compiler copy the
  // accumulators in and out of it on every iteration):
  //  * the ragged last rows (only the chunk that ends at m), rows past r1 read as 0;
  //  * with an odd number of whole 32-row steps, the first step alone (through LDS slot 1,
  //    which the loop's first barrier protects); with an even number a step of zeros.
  const int64_t rfull = r0 + (((r1 - r0) >> 5) << 5);
  {
    uint2 v[8];
    bf16x8 b[NT];
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int64_t row = rfull + 8 * g + t;
      v[t] = (row < r1 && wact) ? *reinterpret_cast<const uint2*>(Ac + row * ldc + cbc)
                                : make_uint2(0u, 0u);
    }
    const int64_t kb = rfull < r1 ? rfull >> 5 : 0;
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) b[nt] = qp[(kb * NT + nt) * 64];
    atqc_products<NT>(v, b, acc);
  }
  const int64_t nsteps = (rfull - r0) >> 5;
  {
    uint2 v[8];
    bf16x8 x[FPT];
    if (nsteps & 1) {
      load(r0, v, x);
    } else {
#pragma unroll
      for (int t = 0; t < 8; ++t) v[t] = make_uint2(0u, 0u);
#pragma unroll
      for (int u = 0; u < FPT; ++u) x[u] = __builtin_bit_cast(bf16x8, u32x4{0u, 0u, 0u, 0u});
    }
    stage(1, x, x);
    products(1, 0, v);
  }
  if (nsteps > 1) {
    uint2 v0[8], v1[8];
    bf16x8 x0[FPT], x1[FPT];
    const int64_t last = rfull - 32;
    const int64_t rs = r0 + 32 * (nsteps & 1);  // first step of the pairs
    load(rs, v0, x0);
    __builtin_amdgcn_sched_barrier(0);  // the same load order as in the loop
    load(rs + 32, v1, x1);
    __builtin_amdgcn_sched_barrier(0);
    int slot = 0;
    for (int64_t rb = rs; rb + 64 <= rfull; rb += 64) {
      stage(slot, x0, x1);
      products(slot, 0, v0);
      __builtin_amdgcn_sched_barrier(0);
      load((rb + 64 < last) ? rb + 64 : last, v0, x0);
      __builtin_amdgcn_sched_barrier(0);
      products(slot, 1, v1);
      __builtin_amdgcn_sched_barrier(0);
      load((rb + 96 < last) ? rb + 96 : last, v1, x1);
      __builtin_amdgcn_sched_barrier(0);
      slot ^= 1;
    }
  }
  if (!wact) return;
  double* P = part + (int64_t)chunk * n * l;
#pragma unroll
  for (int e = 0; e < 4; ++e)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      const int col = 16 * nt + li;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int c = cw + 4 * (4 * g + r) + e;
        if (c < n && col < l) P[(int64_t)c * l + col] = (double)acc[e][nt][r];
      }
    }
}

// ---------------------------------------------------------------- host side
static void mx_grid(int64_t m, int64_t n, int& ncol, int& nchunk, int64_t& chunk_rows) {
  ncol = (int)((n + MX_COLS - 1) / MX_COLS);
  int64_t want = (1024 + ncol - 1) / ncol;
  const int64_t maxc = (m + 255) / 256;
  if (want > maxc) want = maxc;
  if (want < 1) want = 1;
  chunk_rows = (m + want - 1) / want;
  chunk_rows = (chunk_rows + 31) / 32 * 32;
  nchunk = (int)((m + chunk_rows - 1) / chunk_rows);
}

size_t mixed_partials(int64_t m, int64_t n, int l) {
  int ncol, nchunk;
  int64_t cr;
  mx_grid(m, n, ncol, nchunk, cr);
  return (size_t)nchunk * n * l;
}

size_t mixed_pack_bytes(int64_t K, int l) {
  const int NT = (l + 15) / 16;
  const int64_t Kpad = (K + 31) / 32 * 32;
  return (size_t)Kpad * 16 * NT * 6;  // the largest packing: three bfloat16 pieces
}

hipError_t pack_operand(const double* S, int64_t K, int l, int lds, int kind, void* P,
                        hipStream_t s) {
  const int NT = (l + 15) / 16;
  if (kind == MIX_BF16) {
    const int64_t nkb = (K + 31) / 32;
    const int64_t tot = nkb * NT * 64;
    hipLaunchKernelGGL(k_pack_bf16, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, S, K,
                       l, lds, NT, nkb, (bf16x8*)P);
  } else if (kind == MIX_BF16P) {
    const int64_t ng = (K + 63) / 64;
    const int64_t tot = ng * 2 * NT * 64;
    hipLaunchKernelGGL(k_pack_bf16p, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, S,
                       K, l, lds, NT, ng, (bf16x8*)P);
  } else if (kind == MIX_BF16X3) {
    const int64_t nkb = (K + 31) / 32;
    const int64_t tot = nkb * NT * 64;
    hipLaunchKernelGGL(k_pack_bf16x3, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, S,
                       K, l, lds, NT, nkb, (bf16x8*)P);
  } else if (kind == MIX_F32_AX) {
    const int64_t nkb = (K + 15) / 16;
    const int64_t tot = nkb * NT * 64;
    hipLaunchKernelGGL(k_pack_f32_ax, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, S,
                       K, l, lds, NT, nkb, (float*)P);
  } else {
    const int64_t Kpad = (K + 31) / 32 * 32;
    const int64_t tot = Kpad * 16 * NT;
    hipLaunchKernelGGL(k_pack_f32_rows, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, S,
                       K, l, lds, 16 * NT, Kpad, (float*)P);
  }
  return hipGetLastError();
}

template <int NT>
static void launch_ax_mixed(const float* A, int64_t lda, int64_t m, int64_t n, const void* Xp,
                            int l, double* Y, int ldy, int kind, hipStream_t s) {
  constexpr int RT = AX_RT;
  const unsigned grid = (unsigned)((m + 64 * RT - 1) / (64 * RT));
  const bool vec = (reinterpret_cast<uintptr_t>(A) & 15) == 0 && (lda & 3) == 0;
  const int64_t nfrag = (int64_t)((n + 31) / 32) * NT * 64;
  if (kind == MIX_F32_AX) {
    constexpr int RT2 = 2;
    hipLaunchKernelGGL((k_ax_f32<RT2, NT>), dim3((unsigned)((m + 64 * RT2 - 1) / (64 * RT2))),
                       dim3(256), 0, s, A, lda, m, (int)n, (const float*)Xp, l, Y, ldy);
  } else if (kind == MIX_BF16) {
    if (vec)
      hipLaunchKernelGGL((k_ax_bf16<RT, NT, 1, true>), dim3(grid), dim3(256), 0, s, A, lda, m,
                         (int)n, (const bf16x8*)Xp, nfrag, l, Y, ldy);
    else
      hipLaunchKernelGGL((k_ax_bf16<RT, NT, 1, false>), dim3(grid), dim3(256), 0, s, A, lda, m,
                         (int)n, (const bf16x8*)Xp, nfrag, l, Y, ldy);
  } else {
    constexpr int RT3 = AX_RT3;
    const unsigned grid3 = (unsigned)((m + 64 * RT3 - 1) / (64 * RT3));
    if (vec)
      hipLaunchKernelGGL((k_ax_bf16<RT3, NT, 3, true>), dim3(grid3), dim3(256), 0, s, A, lda, m,
                         (int)n, (const bf16x8*)Xp, nfrag, l, Y, ldy);
    else
      hipLaunchKernelGGL((k_ax_bf16<RT3, NT, 3, false>), dim3(grid3), dim3(256), 0, s, A, lda,
                         m, (int)n, (const bf16x8*)Xp, nfrag, l, Y, ldy);
  }
}

hipError_t gemm_ax_mixed(const float* A, int64_t lda, int64_t m, int64_t n, const void* Xp,
                         int l, double* Y, int ldy, int kind, hipStream_t s, int prof) {
  prof_begin(prof, s);
  switch ((l + 15) / 16) {
    case 1: launch_ax_mixed<1>(A, lda, m, n, Xp, l, Y, ldy, kind, s); break;
    case 2: launch_ax_mixed<2>(A, lda, m, n, Xp, l, Y, ldy, kind, s); break;
    case 3: launch_ax_mixed<3>(A, lda, m, n, Xp, l, Y, ldy, kind, s); break;
    case 4: launch_ax_mixed<4>(A, lda, m, n, Xp, l, Y, ldy, kind, s); break;
    case 5: launch_ax_mixed<5>(A, lda, m, n, Xp, l, Y, ldy, kind, s); break;
    case 6: launch_ax_mixed<6>(A, lda, m, n, Xp, l, Y, ldy, kind, s); break;
    case 7: launch_ax_mixed<7>(A, lda, m, n, Xp, l, Y, ldy, kind, s); break;
    default: return hipErrorInvalidValue;
  }
  prof_end(prof, s);
  return hipGetLastError();
}

template <int NT>
static void launch_atq_mixed(const float* A, int64_t lda, int64_t m, int64_t n, const void* Qp,
                             int l, double* part, int kind, hipStream_t s) {
  int ncol, nchunk;
  int64_t cr;
  mx_grid(m, n, ncol, nchunk, cr);
  const int total = ncol * nchunk;
  const int grid = ((total + 7) / 8) * 8;
  const int64_t nfrag = ((m + 31) / 32) * NT * 64;
  const bool vec =
      (reinterpret_cast<uintptr_t>(A) & 15) == 0 && (lda & 3) == 0 && (n & 63) == 0;
  if (kind == MIX_BF16) {
    if (vec)
      hipLaunchKernelGGL((k_atq_bf16<NT, 1, true>), dim3(grid), dim3(256), 0, s, A, lda, m,
                         (int)n, (const bf16x8*)Qp, nfrag, l, ncol, nchunk, cr, part);
    else
      hipLaunchKernelGGL((k_atq_bf16<NT, 1, false>), dim3(grid), dim3(256), 0, s, A, lda, m,
                         (int)n, (const bf16x8*)Qp, nfrag, l, ncol, nchunk, cr, part);
  } else if (kind == MIX_BF16X3) {
    if (vec)
      hipLaunchKernelGGL((k_atq_bf16<NT, 3, true>), dim3(grid), dim3(256), 0, s, A, lda, m,
                         (int)n, (const bf16x8*)Qp, nfrag, l, ncol, nchunk, cr, part);
    else
      hipLaunchKernelGGL((k_atq_bf16<NT, 3, false>), dim3(grid), dim3(256), 0, s, A, lda, m,
                         (int)n, (const bf16x8*)Qp, nfrag, l, ncol, nchunk, cr, part);
  } else {
    hipLaunchKernelGGL((k_atq_f32<NT>), dim3(grid), dim3(256), 0, s, A, lda, m, (int)n,
                       (const float*)Qp, l, ncol, nchunk, cr, part);
  }
}

hipError_t gemm_atq_mixed(const float* A, int64_t lda, int64_t m, int64_t n, const void* Qp,
                          int l, double* Z, int ldz, double* part, int kind, hipStream_t s,
                          int prof) {
  prof_begin(prof, s);
  switch ((l + 15) / 16) {
    case 1: launch_atq_mixed<1>(A, lda, m, n, Qp, l, part, kind, s); break;
    case 2: launch_atq_mixed<2>(A, lda, m, n, Qp, l, part, kind, s); break;
    case 3: launch_atq_mixed<3>(A, lda, m, n, Qp, l, part, kind, s); break;
    case 4: launch_atq_mixed<4>(A, lda, m, n, Qp, l, part, kind, s); break;
    case 5: launch_atq_mixed<5>(A, lda, m, n, Qp, l, part, kind, s); break;
    case 6: launch_atq_mixed<6>(A, lda, m, n, Qp, l, part, kind, s); break;
    case 7: launch_atq_mixed<7>(A, lda, m, n, Qp, l, part, kind, s); break;
    default: return hipErrorInvalidValue;
  }
  prof_end(prof, s);
  int ncol, nchunk;
  int64_t cr;
  mx_grid(m, n, ncol, nchunk, cr);
  return reduce_chunks(part, nchunk, n, l, Z, ldz, s);
}

int64_t bf16_copy_ld(int64_t n) { return (n + 63) / 64 * 64; }

size_t bf16_copy_bytes(int64_t m, int64_t n) { return (size_t)m * bf16_copy_ld(n) * 2; }

template <int NT>
static void launch_ax_bf16c(const void* Ac, int64_t m, int64_t n, const void* Xp, int l,
                            double* Y, int ldy, hipStream_t s) {
  constexpr int RT = AXC_RT;
  const unsigned grid = (unsigned)((m + 64 * RT - 1) / (64 * RT));
  const int64_t ldc = bf16_copy_ld(n);
  hipLaunchKernelGGL((k_ax_bf16c<RT, NT>), dim3(grid), dim3(256), 0, s, (const bf16x8*)Ac,
                     ldc / 8, m, (int)(ldc / 64), (const bf16x8*)Xp, l, Y, ldy);
}

hipError_t gemm_ax_bf16c(const void* Ac, int64_t m, int64_t n, const void* Xp, int l, double* Y,
                         int ldy, hipStream_t s, int prof) {
  prof_begin(prof, s);
  switch ((l + 15) / 16) {
    case 1: launch_ax_bf16c<1>(Ac, m, n, Xp, l, Y, ldy, s); break;
    case 2: launch_ax_bf16c<2>(Ac, m, n, Xp, l, Y, ldy, s); break;
    case 3: launch_ax_bf16c<3>(Ac, m, n, Xp, l, Y, ldy, s); break;
    case 4: launch_ax_bf16c<4>(Ac, m, n, Xp, l, Y, ldy, s); break;
    case 5: launch_ax_bf16c<5>(Ac, m, n, Xp, l, Y, ldy, s); break;
    case 6: launch_ax_bf16c<6>(Ac, m, n, Xp, l, Y, ldy, s); break;
    case 7: launch_ax_bf16c<7>(Ac, m, n, Xp, l, Y, ldy, s); break;
    default: return hipErrorInvalidValue;
  }
  prof_end(prof, s);
  return hipGetLastError();
}

template <int NT>
static void launch_atq_bf16c(const void* Ac, int64_t m, int64_t n, const void* Qp, int l,
                             double* part, hipStream_t s) {
  int ncol, nchunk;
  int64_t cr;
  mx_grid(m, n, ncol, nchunk, cr);
  const int total = ncol * nchunk;
  const int grid = ((total + 7) / 8) * 8;
  hipLaunchKernelGGL((k_atq_bf16c<NT>), dim3(grid), dim3(256), 0, s, (const __bf16*)Ac,
                     bf16_copy_ld(n), m, (int)n, (const bf16x8*)Qp, l, ncol, nchunk, cr, part);
}

hipError_t gemm_atq_bf16c(const void* Ac, int64_t m, int64_t n, const void* Qp, int l,
                          double* Z, int ldz, double* part, hipStream_t s, int prof) {
  prof_begin(prof, s);
  switch ((l + 15) / 16) {
    case 1: launch_atq_bf16c<1>(Ac, m, n, Qp, l, part, s); break;
    case 2: launch_atq_bf16c<2>(Ac, m, n, Qp, l, part, s); break;
    case 3: launch_atq_bf16c<3>(Ac, m, n, Qp, l, part, s); break;
    case 4: launch_atq_bf16c<4>(Ac, m, n, Qp, l, part, s); break;
    case 5: launch_atq_bf16c<5>(Ac, m, n, Qp, l, part, s); break;
    case 6: launch_atq_bf16c<6>(Ac, m, n, Qp, l, part, s); break;
    case 7: launch_atq_bf16c<7>(Ac, m, n, Qp, l, part, s); break;
    default: return hipErrorInvalidValue;
  }
  prof_end(prof, s);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  int ncol, nchunk;
  int64_t cr;
  mx_grid(m, n, ncol, nchunk, cr);
  return reduce_chunks(part, nchunk, n, l, Z, ldz, s);
}

template <int NT>
static void launch_ax_bf16p(const float* A, int64_t lda, int64_t m, int64_t n, const void* Xp,
                            int l, double* Y, int ldy, void* Ac, hipStream_t s) {
  constexpr int RT = AXF_RT;
  const unsigned grid = (unsigned)((m + 64 * RT - 1) / (64 * RT));
  const bool vec = (reinterpret_cast<uintptr_t>(A) & 15) == 0 && (lda & 3) == 0;
  const int64_t ldc8 = bf16_copy_ld(n) / 8;
  if (vec && Ac)
    hipLaunchKernelGGL((k_ax_bf16p<RT, NT, true, true>), dim3(grid), dim3(256), 0, s, A, lda,
                       m, (int)n, (const bf16x8*)Xp, l, Y, ldy, (bf16x8*)Ac, ldc8);
  else if (Ac)
    hipLaunchKernelGGL((k_ax_bf16p<RT, NT, false, true>), dim3(grid), dim3(256), 0, s, A, lda,
                       m, (int)n, (const bf16x8*)Xp, l, Y, ldy, (bf16x8*)Ac, ldc8);
  else if (vec)
    hipLaunchKernelGGL((k_ax_bf16p<RT, NT, true, false>), dim3(grid), dim3(256), 0, s, A, lda,
                       m, (int)n, (const bf16x8*)Xp, l, Y, ldy, nullptr, ldc8);
  else
    hipLaunchKernelGGL((k_ax_bf16p<RT, NT, false, false>), dim3(grid), dim3(256), 0, s, A, lda,
                       m, (int)n, (const bf16x8*)Xp, l, Y, ldy, nullptr, ldc8);
}

hipError_t gemm_ax_bf16p(const float* A, int64_t lda, int64_t m, int64_t n, const void* Xp,
                         int l, double* Y, int ldy, void* Acopy, hipStream_t s, int prof) {
  prof_begin(prof, s);
  switch ((l + 15) / 16) {
    case 1: launch_ax_bf16p<1>(A, lda, m, n, Xp, l, Y, ldy, Acopy, s); break;
    case 2: launch_ax_bf16p<2>(A, lda, m, n, Xp, l, Y, ldy, Acopy, s); break;
    case 3: launch_ax_bf16p<3>(A, lda, m, n, Xp, l, Y, ldy, Acopy, s); break;
    case 4: launch_ax_bf16p<4>(A, lda, m, n, Xp, l, Y, ldy, Acopy, s); break;
    case 5: launch_ax_bf16p<5>(A, lda, m, n, Xp, l, Y, ldy, Acopy, s); break;
    case 6: launch_ax_bf16p<6>(A, lda, m, n, Xp, l, Y, ldy, Acopy, s); break;
    case 7: launch_ax_bf16p<7>(A, lda, m, n, Xp, l, Y, ldy, Acopy, s); break;
    default: return hipErrorInvalidValue;
  }
  prof_end(prof, s);
  return hipGetLastError();
}

}  // namespace tsv
