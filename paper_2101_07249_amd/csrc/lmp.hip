// Spectral-LMP application to one vector (Section 3.2, eq. spectral_LMP_factor in
// closed form): y = x + U diag(dcoef) U^T x, dcoef = theta^{-1/2} - 1.
//
// Two passes over U (n_A x k, column-major), each HBM-bound:
//   lmp_gemv_t: t = dcoef .* (U^T x)   -- chunk partials, then a fixed-order sum
//   lmp_gemv_n: y = x + U t
// U^T x: a workgroup owns 32 columns and a long run of rows, each thread keeps 32
// accumulators and reduces once.  x + U t: a thread owns 2 rows and streams the
// columns 8 at a time (16 independent loads in flight).
#include "wc4d_internal.h"

namespace wc4d {

constexpr int kLT = 256;  // threads per block
constexpr int kLE = 2;    // rows per thread (x + U t pass)
constexpr int kLC = 8;    // columns per group (x + U t pass)
constexpr int kLRows = kLT * kLE;
constexpr int kTG = 32;   // columns per workgroup (U^T x pass)
constexpr int kTU = 1;    // row unroll (U^T x pass)

static inline long long lmp_chunks(long long nA) { return (nA + kLRows - 1) / kLRows; }

// U^T x: grid (column groups of kTG) x (row splits); about 512 workgroups (measured:
// 32 columns x 1 row per thread streams U at ~90% of the plain-read rate on MI355X,
// 16 columns x 2 rows at ~60%).
static inline int lmp_t_splits(long long nA, int k) {
  const int ncg = (k + kTG - 1) / kTG;
  long long sp = (512 + ncg - 1) / ncg;
  const long long maxs = (nA + 4095) / 4096;  // at least 4096 rows per split
  if (sp > maxs) sp = maxs;
  return sp < 1 ? 1 : (int)sp;
}

size_t lmp_gemv_ws_doubles(long long nA, int k) { return (size_t)lmp_t_splits(nA, k) * k + k; }
size_t lmp_gemv_t_offset(long long nA, int k) { return (size_t)lmp_t_splits(nA, k) * k; }

// Partial sums of columns [c0, c0 + kTG) over rows [rb, re): each thread runs down
// its rows with kTG accumulators; one block reduction at the end.
template <typename T>
__global__ __launch_bounds__(kLT) void k_lmp_gemv_t_partial(long long nA, int k, long long rows_per,
                                                            const T* __restrict__ U, long long ldu,
                                                            const double* __restrict__ x,
                                                            double* __restrict__ part,
                                                            const int* __restrict__ skip) {
  __shared__ double sh[kLT / 64][kTG];
  if (skip != nullptr && *skip != 0) return;
  const int c0 = blockIdx.x * kTG;
  const int split = blockIdx.y;
  const long long rb = (long long)split * rows_per;
  long long re = rb + rows_per;
  if (re > nA) re = nA;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const T* Uc[kTG];
#pragma unroll
  for (int c = 0; c < kTG; ++c) Uc[c] = U + (size_t)(c0 + c < k ? c0 + c : 0) * ldu;
  double acc[kTG];
#pragma unroll
  for (int c = 0; c < kTG; ++c) acc[c] = 0.0;
  for (long long r = rb + threadIdx.x; r < re; r += (long long)kLT * kTU) {
    double xv[kTU];
    bool ok[kTU];
#pragma unroll
    for (int u = 0; u < kTU; ++u) {
      const long long rr = r + (long long)u * kLT;
      ok[u] = rr < re;
      xv[u] = ok[u] ? x[rr] : 0.0;
    }
#pragma unroll
    for (int c = 0; c < kTG; ++c) {
#pragma unroll
      for (int u = 0; u < kTU; ++u) {
        const long long rr = r + (long long)u * kLT;
        if (ok[u]) acc[c] += (double)Uc[c][rr] * xv[u];
      }
    }
  }
#pragma unroll
  for (int c = 0; c < kTG; ++c) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc[c] += __shfl_down(acc[c], o, 64);
  }
  if (lane == 0) {
#pragma unroll
    for (int c = 0; c < kTG; ++c) sh[wave][c] = acc[c];
  }
  __syncthreads();
  if (threadIdx.x < kTG && c0 + (int)threadIdx.x < k) {
    double sum = 0.0;
#pragma unroll
    for (int w = 0; w < kLT / 64; ++w) sum += sh[w][threadIdx.x];
    part[(size_t)split * k + c0 + threadIdx.x] = sum;
  }
}

__global__ void k_lmp_gemv_t_final(int splits, int k, const double* __restrict__ part,
                                   const double* __restrict__ dcoef, double* __restrict__ t,
                                   const int* __restrict__ skip) {
  if (skip != nullptr && *skip != 0) return;
  // one wavefront per column: lanes stride the splits, then a fixed-order tree
  const int c = blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (c >= k) return;
  double s = 0.0;
  for (int b = lane; b < splits; b += 64) s += part[(size_t)b * k + c];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
  if (lane == 0) t[c] = (dcoef != nullptr) ? dcoef[c] * s : s;
}

// 4 consecutive rows per thread: one 16-byte (float) or two 16-byte (double) loads per
// column; requires ldu % 4 == 0 (U is allocated that way) and 16-byte aligned x, y.
template <typename T>
static __device__ inline void load4(const T* p, double (&v)[4]);
template <>
__device__ inline void load4<float>(const float* p, double (&v)[4]) {
  const float4 f = *reinterpret_cast<const float4*>(p);
  v[0] = f.x; v[1] = f.y; v[2] = f.z; v[3] = f.w;
}
template <>
__device__ inline void load4<double>(const double* p, double (&v)[4]) {
  const double2 a = *reinterpret_cast<const double2*>(p);
  const double2 b = *reinterpret_cast<const double2*>(p + 2);
  v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y;
}

template <typename T>
__global__ __launch_bounds__(kLT) void k_lmp_gemv_n(long long nA, int k, const T* __restrict__ U,
                                                    long long ldu, const double* __restrict__ t,
                                                    const double* __restrict__ x,
                                                    double* __restrict__ y,
                                                    const int* __restrict__ skip) {
  extern __shared__ double ts[];
  if (skip != nullptr && *skip != 0) return;
  for (int c = threadIdx.x; c < k; c += kLT) ts[c] = t[c];
  __syncthreads();
  const long long r0 = ((long long)blockIdx.x * kLT + threadIdx.x) * 4;
  if (r0 >= nA) return;
  const bool full = r0 + 4 <= nA;
  double acc[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) acc[e] = (r0 + e < nA) ? x[r0 + e] : 0.0;
  for (int c0 = 0; c0 < k; c0 += kLC) {
    double u[kLC][4];
#pragma unroll
    for (int c = 0; c < kLC; ++c) {
      if (c0 + c < k && full) {
        load4<T>(U + (size_t)(c0 + c) * ldu + r0, u[c]);
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e)
          u[c][e] = (c0 + c < k && r0 + e < nA) ? (double)U[(size_t)(c0 + c) * ldu + r0 + e] : 0.0;
      }
    }
#pragma unroll
    for (int c = 0; c < kLC; ++c) {
      const double tc = (c0 + c < k) ? ts[c0 + c] : 0.0;
#pragma unroll
      for (int e = 0; e < 4; ++e) acc[e] += u[c][e] * tc;
    }
  }
#pragma unroll
  for (int e = 0; e < 4; ++e)
    if (r0 + e < nA) y[r0 + e] = acc[e];
}

hipError_t lmp_gemv_t(long long nA, int k, const void* U, bool u32, long long ldu,
                      const double* dcoef, const double* x, double* ws, const int* skip,
                      hipStream_t s, double* tout) {
  const int sp = lmp_t_splits(nA, k);
  long long rows_per = (nA + sp - 1) / sp;
  double* part = ws;
  double* t = (tout != nullptr) ? tout : ws + (size_t)sp * k;
  dim3 grid((k + kTG - 1) / kTG, sp);
  if (u32)
    hipLaunchKernelGGL(k_lmp_gemv_t_partial<float>, grid, dim3(kLT), 0, s, nA, k, rows_per,
                       (const float*)U, ldu, x, part, skip);
  else
    hipLaunchKernelGGL(k_lmp_gemv_t_partial<double>, grid, dim3(kLT), 0, s, nA, k, rows_per,
                       (const double*)U, ldu, x, part, skip);
  hipLaunchKernelGGL(k_lmp_gemv_t_final, dim3((k + 3) / 4), dim3(256), 0, s, sp, k, part, dcoef, t,
                     skip);
  return hipGetLastError();
}

hipError_t lmp_gemv_n(long long nA, int k, const void* U, bool u32, long long ldu, const double* x,
                      double* y, const double* ws, const int* skip, hipStream_t s) {
  if (ldu % 4 != 0) return hipErrorInvalidValue;
  const long long nch = (nA + 4LL * kLT - 1) / (4LL * kLT);
  const double* t = ws + (size_t)lmp_t_splits(nA, k) * k;
  if (u32)
    hipLaunchKernelGGL(k_lmp_gemv_n<float>, dim3((unsigned)nch), dim3(kLT), sizeof(double) * k, s, nA,
                       k, (const float*)U, ldu, t, x, y, skip);
  else
    hipLaunchKernelGGL(k_lmp_gemv_n<double>, dim3((unsigned)nch), dim3(kLT), sizeof(double) * k, s,
                       nA, k, (const double*)U, ldu, t, x, y, skip);
  return hipGetLastError();
}

}  // namespace wc4d
