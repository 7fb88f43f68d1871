// Small helper kernels: identity seeds, the Philox sketch, the output sign convention,
// strided copies, the orthonormality measure and the device-side call record.
#include "common.h"
#include "internal.h"

namespace tsv {

__global__ void k_fill_identity(double* S, int n, int k) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < n * k) {
    const int r = idx / k, c = idx - r * k;
    S[idx] = (r == c) ? 1.0 : 0.0;
  }
}

hipError_t fill_identity(double* S, int n, int k, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_identity, dim3((n * k + 255) / 256), dim3(256), 0, s, S, n, k);
  return hipGetLastError();
}

// ---- Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) and Box-Muller normals.
__device__ __forceinline__ void philox_round(uint32_t& c0, uint32_t& c1, uint32_t& c2,
                                             uint32_t& c3, uint32_t k0, uint32_t k1) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t hi0 = __umulhi(M0, c0), lo0 = M0 * c0;
  const uint32_t hi1 = __umulhi(M1, c2), lo1 = M1 * c2;
  const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
  c0 = n0;
  c1 = lo1;
  c2 = n2;
  c3 = lo0;
}

__global__ void k_philox_sketch(double* X, int64_t total, uint32_t key0, uint32_t key1) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (4 * t >= total) return;
  uint32_t c0 = (uint32_t)(t & 0xFFFFFFFFll), c1 = (uint32_t)(t >> 32), c2 = 0, c3 = 0;
  uint32_t k0 = key0, k1 = key1;
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    philox_round(c0, c1, c2, c3, k0, k1);
  }
  const double u0 = ((double)c0 + 0.5) * 0x1p-32, u1 = ((double)c1 + 0.5) * 0x1p-32;
  const double u2 = ((double)c2 + 0.5) * 0x1p-32, u3 = ((double)c3 + 0.5) * 0x1p-32;
  const double r0 = sqrt(-2.0 * log(u0)), r1 = sqrt(-2.0 * log(u2));
  double s0, co0, s1, co1;
  sincospi(2.0 * u1, &s0, &co0);
  sincospi(2.0 * u3, &s1, &co1);
  const double z[4] = {r0 * co0, r0 * s0, r1 * co1, r1 * s1};
  for (int i = 0; i < 4; ++i)
    if (4 * t + i < total) X[4 * t + i] = z[i];
}

hipError_t philox_sketch(double* X, int64_t n, int l, uint64_t seed, hipStream_t s) {
  const int64_t total = n * (int64_t)l;
  const int64_t nt = (total + 3) / 4;
  hipLaunchKernelGGL(k_philox_sketch, dim3((unsigned)((nt + 255) / 256)), dim3(256), 0, s, X,
                     total, (uint32_t)(seed & 0xFFFFFFFFull), (uint32_t)(seed >> 32));
  return hipGetLastError();
}

// ---- sign convention: one workgroup per column; fixed-order reduction of w^T v_j.
__global__ __launch_bounds__(256) void k_sign_fix(double* V, int64_t n, int ldv, double* P,
                                                  int prow, int ldp, const int* gate) {
  if (gate && *gate == 0) return;
  __shared__ double red[256];
  const int j = blockIdx.x, tid = threadIdx.x;
  double s = 0.0;
  for (int64_t i = tid; i < n; i += 256) s = fma(sign_ref((int)i), V[i * ldv + j], s);
  red[tid] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) red[tid] += red[tid + w];
    __syncthreads();
  }
  if (red[0] < 0.0) {
    for (int64_t i = tid; i < n; i += 256) V[i * ldv + j] = -V[i * ldv + j];
    if (P)
      for (int i = tid; i < prow; i += 256) P[(int64_t)i * ldp + j] = -P[(int64_t)i * ldp + j];
  }
}

hipError_t sign_fix_cols(double* V, int64_t n, int ldv, int k, double* P, int prow, int ldp,
                         hipStream_t s, const int* gate) {
  hipLaunchKernelGGL(k_sign_fix, dim3(k), dim3(256), 0, s, V, n, ldv, P, prow, ldp, gate);
  return hipGetLastError();
}

__global__ void k_copy(const double* __restrict__ src, int64_t rows, int cols, int64_t lds,
                       double* __restrict__ dst, int64_t ldd, const int* gate) {
  if (gate && *gate == 0) return;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= rows * cols) return;
  const int64_t r = idx / cols;
  const int c = (int)(idx - r * cols);
  dst[r * ldd + c] = src[r * lds + c];
}

hipError_t copy_matrix(const double* src, int64_t rows, int cols, int64_t lds, double* dst,
                       int64_t ldd, hipStream_t s, const int* gate) {
  const int64_t tot = rows * cols;
  if (tot == 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, src, rows,
                     cols, lds, dst, ldd, gate);
  return hipGetLastError();
}

__global__ void k_info_init(tssvd_info* info) {
  if (threadIdx.x == 0) {
    info->numstat = 0;
    info->rank = 0;
    info->sweeps = 0;
    info->reorth = 0;
    info->ortho = -1.0;
  }
}

hipError_t info_init(tssvd_info* info, hipStream_t s) {
  if (!info) return hipSuccess;
  hipLaunchKernelGGL(k_info_init, dim3(1), dim3(64), 0, s, info);
  return hipGetLastError();
}

}  // namespace tsv

// ---- measurement markers: pairs of HIP events around kernels that stream A.
#include <mutex>
#include <vector>

namespace tsv {
namespace {
struct ProfKind {
  std::vector<hipEvent_t> b, e;
  size_t used = 0;
  bool open = false;
};
std::mutex g_prof_mu;
bool g_prof_on = false;
ProfKind g_prof[TSSVD_PROF_KINDS];
}  // namespace

void prof_enable(bool on) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  g_prof_on = on;
  for (auto& k : g_prof) {
    k.used = 0;
    k.open = false;
  }
}

void prof_begin(int kind, hipStream_t s) {
  if (kind < 0 || kind >= TSSVD_PROF_KINDS) return;
  std::lock_guard<std::mutex> lk(g_prof_mu);
  if (!g_prof_on) return;
  ProfKind& k = g_prof[kind];
  if (k.used == k.b.size()) {
    hipEvent_t b, e;
    if (hipEventCreate(&b) != hipSuccess) return;
    if (hipEventCreate(&e) != hipSuccess) return;
    k.b.push_back(b);
    k.e.push_back(e);
  }
  if (hipEventRecord(k.b[k.used], s) == hipSuccess) k.open = true;
}

void prof_end(int kind, hipStream_t s) {
  if (kind < 0 || kind >= TSSVD_PROF_KINDS) return;
  std::lock_guard<std::mutex> lk(g_prof_mu);
  ProfKind& k = g_prof[kind];
  if (!g_prof_on || !k.open) return;
  if (hipEventRecord(k.e[k.used], s) == hipSuccess) ++k.used;
  k.open = false;
}

hipError_t prof_read(int kind, double* total_ms, int64_t* launches) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  ProfKind& k = g_prof[kind];
  double tot = 0.0;
  for (size_t i = 0; i < k.used; ++i) {
    hipError_t e = hipEventSynchronize(k.e[i]);
    if (e != hipSuccess) return e;
    float ms = 0.f;
    e = hipEventElapsedTime(&ms, k.b[i], k.e[i]);
    if (e != hipSuccess) return e;
    tot += ms;
  }
  *total_ms = tot;
  *launches = (int64_t)k.used;
  return hipSuccess;
}

}  // namespace tsv
