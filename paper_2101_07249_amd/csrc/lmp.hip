// Spectral-LMP application to one vector (Section 3.2, eq. spectral_LMP_factor in
// closed form): y = x + U diag(dcoef) U^T x, dcoef = theta^{-1/2} - 1.
//
// Two passes over U (n_A x k), each HBM-bound:
//   lmp_gemv_t: t = dcoef .* (U^T x)   -- chunk partials, then a fixed-order sum
//   lmp_gemv_n: y = x + U t
// Float64 U is column-major (leading dimension ldu).  U^T x: a workgroup owns 32
// columns and a long run of rows, each thread keeps 32 accumulators and reduces once.
// x + U t: a thread owns 4 rows and streams the columns 8 at a time.
//
// The float32 or float16 copy the PCG streams is panel-major instead: panel p holds rows
// [256 p, 256 p + 256) of all k columns, column-major with leading dimension 256, at
// offset 256 k p, and rows at or past n_A are zero.  A workgroup working on one panel
// reads one contiguous block (1 KB or 512 bytes per column).  The float16 copy scales
// each column by a power of two (exact), undone in the coefficients the passes apply.
// Measured on MI355X at n_A = 413,696, k = 251 over the float32 copy (isolated): U^T x
// 73 us (5.7 TB/s) and the fused PCG pass 78 us (5.5 TB/s), against 77 us and 144 us for
// the same passes over a column-major copy (a plain read of the 415 MB runs at 6.3 TB/s);
// over the float16 copy inside the PCG: U^T x 45 us, the fused pass 41 us.
#include "wc4d_internal.h"

#include <climits>

namespace wc4d {

constexpr int kLT = 256;  // threads per block
constexpr int kLC = 8;    // columns per group (x + U t pass)
constexpr int kTG = 32;   // columns per workgroup (U^T x pass)
constexpr int kTU = 1;    // row unroll (U^T x pass)

size_t lmp_panel_elems(long long nA, int k) { return (size_t)lmp_panels(nA) * kPanel * k; }

// U^T x over the float32 panels: grid (column groups of kPG) x (splits of pan_per
// consecutive panels); about 1024 workgroups.
constexpr int kPG = 16;
static inline long long pan_t_per(long long nA, int k) {
  const long long np = lmp_panels(nA);
  const int ncg = (k + kPG - 1) / kPG;
  long long sp = (1024 + ncg - 1) / ncg;
  if (sp > np) sp = np;
  if (sp < 1) sp = 1;
  return (np + sp - 1) / sp;
}
static inline int pan_t_splits(long long nA, int k) {
  const long long per = pan_t_per(nA, k);
  return (int)((lmp_panels(nA) + per - 1) / per);
}

// Row-owning float16 pass: panels per workgroup.  At most 404 workgroups (1.6 per CU, and at
// most 1024: one dot partial each) so that the whole grid is resident at once at the
// kernel's occupancy (3 waves per SIMD); at n_A = 413,696 (1,616 panels) 4 panels each.
static inline long long rows_pan_per(long long nA) {
  const long long np = lmp_panels(nA);
  long long per = (np + 403) / 404;
  if (per < (np + 1023) / 1024) per = (np + 1023) / 1024;
  return per < 1 ? 1 : per;
}
static inline int rows_grid(long long nA) {
  const long long per = rows_pan_per(nA);
  return (int)((lmp_panels(nA) + per - 1) / per);
}

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

// partials of either layout, then t
static inline int t_splits_max(long long nA, int k) {
  return std::max(std::max(lmp_t_splits(nA, k), pan_t_splits(nA, k)), rows_grid(nA));
}
size_t lmp_gemv_ws_doubles(long long nA, int k) { return (size_t)t_splits_max(nA, k) * k + k; }
size_t lmp_gemv_t_offset(long long nA, int k) { return (size_t)t_splits_max(nA, k) * k; }

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
    acc[c] = wave_sum_d(acc[c]);
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

// Partial (split b, column c) at part[b sb + c sc]: (sb, sc) = (k, 1) for the split-major
// partials, (1, splits) for the column-major ones of the row-owning float16 pass.
__device__ __forceinline__ void gemv_t_final_body(int bid, int splits, int k, const double* __restrict__ part,
                                                  const double* __restrict__ dcoef, double* __restrict__ t,
                                                  const int* __restrict__ skip, long long sb, long long sc) {
  if (skip != nullptr && *skip != 0) return;
  // one wavefront per column: lanes stride the splits, then a fixed-order tree
  const int c = bid * (blockDim.x / 64) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (c >= k) return;
  // eight loads in flight per lane, then added in split order
  double s = 0.0;
  for (int b0 = lane; b0 < splits; b0 += 64 * 8) {
    double v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int b = b0 + 64 * q;
      v[q] = b < splits ? part[(size_t)b * sb + (size_t)c * sc] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < 8; ++q)
      if (b0 + 64 * q < splits) s += v[q];
  }
  s = wave_sum_d(s);
  if (lane == 0) t[c] = (dcoef != nullptr) ? dcoef[c] * s : s;
}

__global__ void k_lmp_gemv_t_final(int splits, int k, const double* __restrict__ part,
                                   const double* __restrict__ dcoef, double* __restrict__ t,
                                   const int* __restrict__ skip, long long sb, long long sc) {
  gemv_t_final_body(blockIdx.x, splits, k, part, dcoef, t, skip, sb, sc);
}

// Two such sums in one launch (workgroups [0, nb) the first, [nb, 2 nb) the second), each
// with its own partials, output and skip flag; same split count and strides.
__global__ void k_lmp_gemv_t_final2(int nb, int splits, int k, const double* __restrict__ part1,
                                    double* __restrict__ t1, const int* __restrict__ skip1,
                                    const double* __restrict__ part2, double* __restrict__ t2,
                                    const int* __restrict__ skip2, long long sb, long long sc) {
  if ((int)blockIdx.x < nb)
    gemv_t_final_body(blockIdx.x, splits, k, part1, nullptr, t1, skip1, sb, sc);
  else
    gemv_t_final_body(blockIdx.x - nb, splits, k, part2, nullptr, t2, skip2, sb, sc);
}

// 4 consecutive rows per thread: two 16-byte loads per column; requires ldu % 4 == 0
// (U is allocated that way) and 16-byte aligned x, y.
template <typename T>
static __device__ inline void load4(const T* p, double (&v)[4]);
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


// ------------------------------------------------ panel copies

// P = panels of (float)U; Uround (optional, column-major with ldu) = (double)(float)U,
// the values the passes over P see.
__global__ void k_lmp_to_panels(const double* __restrict__ U, long long ldu, long long nA, int k,
                                long long npan, float* __restrict__ P, double* __restrict__ Uround) {
  const long long total = npan * kPanel * k;
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (long long)gridDim.x * blockDim.x) {
    const long long rr = t % kPanel, c = (t / kPanel) % k, pn = t / ((long long)kPanel * k);
    const long long i = pn * kPanel + rr;
    const float v = i < nA ? (float)U[c * ldu + i] : 0.0f;
    P[t] = v;
    if (Uround != nullptr && i < nA) Uround[c * ldu + i] = (double)v;
  }
}

hipError_t lmp_to_panels(float* P, const double* U, long long ldu, long long nA, int k,
                         double* Uround, hipStream_t s) {
  hipLaunchKernelGGL(k_lmp_to_panels, dim3(4096), dim3(256), 0, s, U, ldu, nA, k, lmp_panels(nA), P,
                     Uround);
  return hipGetLastError();
}

// cexp[c] = ilogb(max_i |U_ic|) - 14 (0 for a zero column): cexp starts at INT_MIN, each
// workgroup of a (column, row slab) grid raises it to its slab's exponent (ilogb is monotonic,
// so the largest slab exponent is the column's), then zero columns get 0.
__global__ void k_lmp_col_exp_init(int k, int* __restrict__ cexp) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c < k) cexp[c] = INT_MIN;
}

__global__ __launch_bounds__(256) void k_lmp_col_exp_slab(const double* __restrict__ U, long long ldu, long long nA,
                                                          long long rows, int* __restrict__ cexp) {
  __shared__ double sh[4];
  const int c = blockIdx.x;
  const long long rb = (long long)blockIdx.y * rows;
  const long long re = rb + rows < nA ? rb + rows : nA;
  double m = 0.0;
  for (long long i = rb + threadIdx.x; i < re; i += 256) m = fmax(m, fabs(U[c * ldu + i]));
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    m = fmax(fmax(sh[0], sh[1]), fmax(sh[2], sh[3]));
    if (m > 0.0) atomicMax(&cexp[c], ilogb(m) - 14);
  }
}

__global__ void k_lmp_col_exp_fix(int k, int* __restrict__ cexp) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c < k && cexp[c] == INT_MIN) cexp[c] = 0;
}

__global__ void k_lmp_to_panels16(const double* __restrict__ U, long long ldu, long long nA, int k,
                                  long long npan, const int* __restrict__ cexp, _Float16* __restrict__ P,
                                  double* __restrict__ Uround) {
  const long long total = npan * kPanel * k;
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (long long)gridDim.x * blockDim.x) {
    const long long rr = t % kPanel, c = (t / kPanel) % k, pn = t / ((long long)kPanel * k);
    const long long i = pn * kPanel + rr;
    const int e = cexp[c];
    const _Float16 h = i < nA ? (_Float16)ldexp(U[c * ldu + i], -e) : (_Float16)0.0f;
    P[t] = h;
    if (Uround != nullptr && i < nA) Uround[c * ldu + i] = ldexp((double)h, e);
  }
}

hipError_t lmp_to_panels16(_Float16* P, int* cexp, const double* U, long long ldu, long long nA, int k,
                           double* Uround, hipStream_t s) {
  constexpr int kSlabs = 16;
  const long long rows = (nA + kSlabs - 1) / kSlabs;
  hipLaunchKernelGGL(k_lmp_col_exp_init, dim3((k + 255) / 256), dim3(256), 0, s, k, cexp);
  hipLaunchKernelGGL(k_lmp_col_exp_slab, dim3(k, kSlabs), dim3(256), 0, s, U, ldu, nA, rows, cexp);
  hipLaunchKernelGGL(k_lmp_col_exp_fix, dim3((k + 255) / 256), dim3(256), 0, s, k, cexp);
  hipLaunchKernelGGL(k_lmp_to_panels16, dim3(4096), dim3(256), 0, s, U, ldu, nA, k, lmp_panels(nA), cexp, P,
                     Uround);
  return hipGetLastError();
}

// out[0] = ||GU - I||_F, out[1] = min(0, min_i dcoef_i): one workgroup.
__global__ __launch_bounds__(256) void k_lmp_copy_check(int k, const double* __restrict__ GU,
                                                        const double* __restrict__ dcoef, double* __restrict__ out) {
  __shared__ double sa[256], sb[256];
  double a = 0.0, b = 0.0;
  for (long long t = threadIdx.x; t < (long long)k * k; t += 256) {
    const long long i = t % k, j = t / k;
    const double v = GU[t] - (i == j ? 1.0 : 0.0);
    a += v * v;
  }
  for (int i = threadIdx.x; i < k; i += 256) b = fmin(b, dcoef[i]);
  sa[threadIdx.x] = a;
  sb[threadIdx.x] = b;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      sa[threadIdx.x] += sa[threadIdx.x + w];
      sb[threadIdx.x] = fmin(sb[threadIdx.x], sb[threadIdx.x + w]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = sqrt(sa[0]);
    out[1] = sb[0];
  }
}

hipError_t lmp_copy_check(int k, const double* GU, const double* dcoef, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_lmp_copy_check, dim3(1), dim3(256), 0, s, k, GU, dcoef, out);
  return hipGetLastError();
}

// Partial sums of columns [c0, c0 + kPG) over panels [pb, pe): thread = one row of the
// panel (the 256 threads read 1 KB per column), kPG accumulators, one block reduction.
// With pdot (PCG): the column-group-0 workgroups also sum pdot . x over their panels into
// dotpart[split].
__global__ __launch_bounds__(kPanel) void k_lmp_pan_t_partial(long long nA, int k, long long pan_per,
                                                              const float* __restrict__ P,
                                                              const double* __restrict__ x,
                                                              double* __restrict__ part,
                                                              const int* __restrict__ skip,
                                                              const double* __restrict__ pdot,
                                                              double* __restrict__ dotpart) {
  __shared__ double sh[kPanel / 64][kPG];
  __shared__ double shd[kPanel / 64];
  if (skip != nullptr && *skip != 0) return;
  const bool dot = pdot != nullptr && blockIdx.x == 0;
  double dv = 0.0;
  const int c0 = blockIdx.x * kPG;
  const int split = blockIdx.y;
  const long long np = lmp_panels(nA);
  const long long pb = (long long)split * pan_per;
  long long pe = pb + pan_per;
  if (pe > np) pe = np;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int col[kPG];
#pragma unroll
  for (int c = 0; c < kPG; ++c) col[c] = (c0 + c < k ? c0 + c : 0) * kPanel;
  double acc[kPG];
#pragma unroll
  for (int c = 0; c < kPG; ++c) acc[c] = 0.0;
  for (long long pn = pb; pn < pe; ++pn) {
    const long long i = pn * kPanel + threadIdx.x;
    const double xv = i < nA ? x[i] : 0.0;
    if (dot && i < nA) dv += pdot[i] * xv;
    const float* Pp = P + (size_t)pn * kPanel * k + threadIdx.x;
#pragma unroll
    for (int c = 0; c < kPG; ++c) acc[c] += (double)Pp[col[c]] * xv;
  }
  if (dot) {
    dv = wave_sum_d(dv);
    if (lane == 0) shd[wave] = dv;
  }
#pragma unroll
  for (int c = 0; c < kPG; ++c) {
    acc[c] = wave_sum_d(acc[c]);
  }
  if (lane == 0) {
#pragma unroll
    for (int c = 0; c < kPG; ++c) sh[wave][c] = acc[c];
  }
  __syncthreads();
  if (threadIdx.x < kPG && c0 + (int)threadIdx.x < k) {
    double sum = 0.0;
#pragma unroll
    for (int w = 0; w < kPanel / 64; ++w) sum += sh[w][threadIdx.x];
    part[(size_t)split * k + c0 + threadIdx.x] = sum;
  }
  if (dot && threadIdx.x == 0) {
    double sum = 0.0;
#pragma unroll
    for (int w = 0; w < kPanel / 64; ++w) sum += shd[w];
    dotpart[split] = sum;
  }
}

// U^T x over the float16 copy with x read once: workgroup b owns panels [b per, b per + per)
// and all columns.  x of up to kXP panels at a time is staged in LDS; then, chunk by chunk of
// 64 columns, lane l of half-wave g (g = 2 wave + lane / 32) holds rows 8 (l % 32) .. + 7 of
// each staged panel (one 16-byte load per column) for columns cc + g + 8 j, j < 8.  A 3-step
// butterfly and a 2-step sum across the half-wave leave column cc + g + 8 ((l % 32) / 4)'s
// sum in lanes with l % 4 = 0, which add it to the workgroup's column totals in LDS; the
// totals go out column-major (part[c G + b], G workgroups) scaled back by 2^cexp[c].  With
// pdot (PCG) every workgroup also sums pdot . x over its rows into dotpart[b].  Used with
// JC = 4 columns per half-wave per chunk (8 converted columns per lane would take all the
// registers: the compiler converts a chunk's halves to double before its FMAs) and QU = 2
// panels' loads in flight (inside the PCG at C3: 44.9 us per pass with its final sum against
// 47.5 us for one panel at a time; 4 panels 45.8 us).  Inside the
// PCG at n_A = 413,696, k = 251: 45.2 us with 4 panels per workgroup, against 53.1 us for 16
// columns x 2 rows per thread (x re-read by every column group); JC = 2 with 2 panels
// each ran 46.3 us, shapes whose grid is not resident at once 55-60 us.
// The body takes its workgroup's index bid among nblk workgroups of the pass, so that a
// launch can also carry other work in workgroups past nblk.
constexpr int kXP = 4;
template <int JC, int QU>
__device__ __forceinline__ void pan_t16_rows_body(int bid, int nblk, long long nA, int k, long long pan_per,
                                                  const _Float16* __restrict__ P, const int* __restrict__ cexp,
                                                  const double* __restrict__ x, double* __restrict__ part,
                                                  const int* __restrict__ skip, const double* __restrict__ pdot,
                                                  double* __restrict__ dotpart) {
  typedef _Float16 h8 __attribute__((ext_vector_type(8)));
  constexpr int CW = 8 * JC;        // columns per chunk
  constexpr int LPC = 32 / JC;      // lanes that end up holding one column's sum
  __shared__ double xs[kXP][kPanel];
  __shared__ double tsum[512];
  __shared__ double shd[kPanel / 64];
  if (skip != nullptr && *skip != 0) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = 2 * wave + (lane >> 5), l32 = lane & 31, r8 = 8 * l32;
  const long long np = lmp_panels(nA);
  const long long pb = (long long)bid * pan_per;
  long long pe = pb + pan_per;
  if (pe > np) pe = np;
  for (int c = threadIdx.x; c < k; c += kPanel) tsum[c] = 0.0;
  double dv = 0.0;
  for (long long g0 = pb; g0 < pe; g0 += kXP) {
    const int ng = (int)(pe - g0 < kXP ? pe - g0 : kXP);
    __syncthreads();  // previous group's reads of xs (and the tsum clear) are done
    for (int q = 0; q < ng; ++q) {
      const long long i = (g0 + q) * kPanel + threadIdx.x;
      const double xv = i < nA ? x[i] : 0.0;
      xs[q][threadIdx.x] = xv;
      if (pdot != nullptr && i < nA) dv += pdot[i] * xv;
    }
    __syncthreads();
#pragma unroll 1
    for (int cc = 0; cc < k; cc += CW) {
      double aj[JC];
#pragma unroll
      for (int j = 0; j < JC; ++j) aj[j] = 0.0;
#pragma unroll 1
      for (int q0 = 0; q0 < ng; q0 += QU) {
        // QU panels' loads in flight before their products; columns past k read column
        // k - 1 (their sums are never written out), panels past ng are skipped
        h8 u[QU][JC];
#pragma unroll
        for (int qq = 0; qq < QU; ++qq) {
          if (q0 + qq < ng) {
            const _Float16* Pp = P + (size_t)(g0 + q0 + qq) * kPanel * k + r8;
#pragma unroll
            for (int j = 0; j < JC; ++j) {
              const int c = min(cc + g + 8 * j, k - 1);
              u[qq][j] = *reinterpret_cast<const h8*>(Pp + (size_t)c * kPanel);
            }
          }
        }
#pragma unroll
        for (int qq = 0; qq < QU; ++qq) {
          if (q0 + qq < ng) {
            double xr[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) xr[e] = xs[q0 + qq][r8 + e];
#pragma unroll
            for (int j = 0; j < JC; ++j) {
              double a = 0.0;
#pragma unroll
              for (int e = 0; e < 8; ++e) a += (double)(float)u[qq][j][e] * xr[e];
              aj[j] += a;
            }
          }
        }
      }
      // butterfly from width 16 down: a lane keeps the lower (bit clear) or upper half of its
      // remaining sums and adds the partner's copy; then the lanes sharing a column add up
#pragma unroll
      for (int w = 16, nv = JC; nv > 1; w >>= 1, nv >>= 1) {
        const bool hi = (l32 & w) != 0;
#pragma unroll
        for (int t = 0; t < nv / 2; ++t) {
          const double send = hi ? aj[t] : aj[t + nv / 2];
          const double keep = hi ? aj[t + nv / 2] : aj[t];
          aj[t] = keep + __shfl_xor(send, w, 64);
        }
      }
#pragma unroll
      for (int w = LPC / 2; w > 0; w >>= 1) aj[0] += __shfl_xor(aj[0], w, 64);
      const int c = cc + g + 8 * (l32 / LPC);
      if (l32 % LPC == 0 && c < k) tsum[c] += aj[0];
    }
  }
  __syncthreads();
  for (int c = threadIdx.x; c < k; c += kPanel) part[(size_t)c * nblk + bid] = ldexp(tsum[c], cexp[c]);
  if (pdot != nullptr) {
    dv = wave_sum_d(dv);
    if (lane == 0) shd[wave] = dv;
    __syncthreads();
    if (threadIdx.x == 0) dotpart[bid] = (shd[0] + shd[1]) + (shd[2] + shd[3]);
  }
}

template <int JC, int QU>
__global__ __launch_bounds__(kPanel) void k_lmp_pan_t16_rows(long long nA, int k, long long pan_per,
                                                             const _Float16* __restrict__ P,
                                                             const int* __restrict__ cexp,
                                                             const double* __restrict__ x,
                                                             double* __restrict__ part,
                                                             const int* __restrict__ skip,
                                                             const double* __restrict__ pdot,
                                                             double* __restrict__ dotpart) {
  pan_t16_rows_body<JC, QU>(blockIdx.x, gridDim.x, nA, k, pan_per, P, cexp, x, part, skip, pdot, dotpart);
}

// The end of a fused PCG iteration in one launch: workgroups [0, G) form the partials of
// U^T r over the float16 panels when the iteration's beta kernel asked for a refresh of
// u = U^T r (*no_refresh == 0; they return at once otherwise), the rest update p = z + beta p
// (nothing once the solve is done).  r is not written and p not read by the pass.
template <int JC, int QU>
__global__ __launch_bounds__(kPanel) void k_update_p_refresh16(const PcgState* __restrict__ st, double* __restrict__ p,
                                                               const double* __restrict__ z, long long nA, int k,
                                                               long long pan_per, int G,
                                                               const _Float16* __restrict__ P,
                                                               const int* __restrict__ cexp,
                                                               const double* __restrict__ r,
                                                               double* __restrict__ rpart) {
  if ((int)blockIdx.x < G) {
    pan_t16_rows_body<JC, QU>(blockIdx.x, G, nA, k, pan_per, P, cexp, r, rpart, &st->no_refresh, nullptr, nullptr);
    return;
  }
  if (st->done) return;
  const double beta = st->beta;
  const long long stride = (long long)(gridDim.x - G) * kPanel;
  for (long long i = (long long)(blockIdx.x - G) * kPanel + threadIdx.x; i < nA; i += stride) p[i] = z[i] + beta * p[i];
}

// y = x + U t over panels: wave w of a 256-thread block takes columns w, w + 4, ...
// (CU in flight: 2 float32 columns of 16-byte loads, 4 float16 columns of 8-byte loads), a
// lane holds 4 rows of the panel; the four waves' sums meet in LDS.
template <typename T, int CU>
__global__ __launch_bounds__(kPanel) void k_lmp_pan_n(long long nA, int k, const T* __restrict__ P,
                                                      const int* __restrict__ cexp,
                                                      const double* __restrict__ t,
                                                      const double* __restrict__ x,
                                                      double* __restrict__ y,
                                                      const int* __restrict__ skip) {
  extern __shared__ double sm[];
  double* ts = sm;           // k coefficients (times 2^cexp for float16)
  double* red = sm + k;      // [4 waves][256 rows]
  if (skip != nullptr && *skip != 0) return;
  for (int c = threadIdx.x; c < k; c += kPanel) ts[c] = cexp != nullptr ? ldexp(t[c], cexp[c]) : t[c];
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const long long np = lmp_panels(nA);
  for (long long pn = blockIdx.x; pn < np; pn += gridDim.x) {
    const T* Pp = P + (size_t)pn * kPanel * k + 4 * lane;
    double a[4] = {0.0, 0.0, 0.0, 0.0};
    for (int c0 = wave; c0 < k; c0 += 4 * CU) {
      float4 u[CU];
      double tc[CU];
#pragma unroll
      for (int j = 0; j < CU; ++j) {
        const int c = c0 + 4 * j;
        u[j] = c < k ? pan_ld4(Pp + (size_t)c * kPanel) : make_float4(0.f, 0.f, 0.f, 0.f);
        tc[j] = c < k ? ts[c] : 0.0;
      }
#pragma unroll
      for (int j = 0; j < CU; ++j) {
        a[0] += u[j].x * tc[j]; a[1] += u[j].y * tc[j]; a[2] += u[j].z * tc[j]; a[3] += u[j].w * tc[j];
      }
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) red[wave * kPanel + 4 * lane + e] = a[e];
    __syncthreads();
    const long long i = pn * kPanel + threadIdx.x;
    if (i < nA) {
      const int q = threadIdx.x;
      y[i] = x[i] + ((red[q] + red[kPanel + q]) + (red[2 * kPanel + q] + red[3 * kPanel + q]));
    }
    __syncthreads();
  }
}

int lmp_pan_t_splits(long long nA, int k, LmpFmt fmt) {
  return fmt == LMP_P16 ? rows_grid(nA) : pan_t_splits(nA, k);
}

// partials of U^T x over the panel copy (either precision); returns the split count and the
// partials' strides (split, column)
static int launch_pan_t_partial(long long nA, int k, const LmpU& U, const double* x, double* part,
                                const int* skip, const double* pdot, double* dotpart, hipStream_t s,
                                long long* sb, long long* sc) {
  if (U.fmt == LMP_P16) {
    const int G = rows_grid(nA);
    hipLaunchKernelGGL((k_lmp_pan_t16_rows<4, 2>), dim3(G), dim3(kPanel), 0, s, nA, k, rows_pan_per(nA),
                       (const _Float16*)U.p, U.cexp, x, part, skip, pdot, dotpart);
    *sb = 1;
    *sc = G;
    return G;
  }
  const int sp = pan_t_splits(nA, k);
  hipLaunchKernelGGL(k_lmp_pan_t_partial, dim3((k + kPG - 1) / kPG, sp), dim3(kPanel), 0, s, nA, k,
                     pan_t_per(nA, k), (const float*)U.p, x, part, skip, pdot, dotpart);
  *sb = k;
  *sc = 1;
  return sp;
}

hipError_t lmp_pan_t_partials(long long nA, int k, const LmpU& U, const double* x, const double* pdot,
                              double* ws, double* dotpart, const int* skip, hipStream_t s) {
  if (U.fmt == LMP_F64) return hipErrorInvalidValue;
  long long sb, sc;
  const int sp = launch_pan_t_partial(nA, k, U, x, ws, skip, pdot, dotpart, s, &sb, &sc);
  hipLaunchKernelGGL(k_lmp_gemv_t_final, dim3((k + 3) / 4), dim3(256), 0, s, sp, k, ws, nullptr,
                     ws + lmp_gemv_t_offset(nA, k), skip, sb, sc);
  return hipGetLastError();
}

hipError_t lmp_pan16_t_partials_refresh(long long nA, int k, const LmpU& U, const double* x, const double* pdot,
                                        double* ws, double* dotpart, const int* skip, const double* rpart,
                                        double* u, const int* no_refresh, hipStream_t s) {
  if (U.fmt != LMP_P16) return hipErrorInvalidValue;
  long long sb, sc;
  const int sp = launch_pan_t_partial(nA, k, U, x, ws, skip, pdot, dotpart, s, &sb, &sc);
  const int nb = (k + 3) / 4;
  hipLaunchKernelGGL(k_lmp_gemv_t_final2, dim3(2 * nb), dim3(256), 0, s, nb, sp, k, ws,
                     ws + lmp_gemv_t_offset(nA, k), skip, rpart, u, no_refresh, sb, sc);
  return hipGetLastError();
}

size_t lmp_pan16_refresh_doubles(long long nA, int k) { return (size_t)rows_grid(nA) * k; }

hipError_t pcg_update_p_refresh16(const PcgState* st, double* p, const double* z, long long nA, int k,
                                  const LmpU& U, const double* r, double* rpart, hipStream_t s) {
  if (U.fmt != LMP_P16) return hipErrorInvalidValue;
  const int G = rows_grid(nA);
  hipLaunchKernelGGL((k_update_p_refresh16<4, 2>), dim3(G + 2048), dim3(kPanel), 0, s, st, p, z, nA, k,
                     rows_pan_per(nA), G, (const _Float16*)U.p, U.cexp, r, rpart);
  return hipGetLastError();
}

// blocks for a pass over all panels: ceil(np / per) with per = ceil(np / 1024)
int lmp_panel_grid(long long nA) {
  const long long np = lmp_panels(nA);
  const long long per = (np + 1023) / 1024;
  return (int)((np + per - 1) / per);
}

hipError_t lmp_gemv_t(long long nA, int k, const LmpU& U, const double* dcoef, const double* x, double* ws,
                      const int* skip, hipStream_t s, double* tout) {
  double* part = ws;
  double* t = (tout != nullptr) ? tout : ws + lmp_gemv_t_offset(nA, k);
  int sp;
  long long sb = k, sc = 1;
  if (U.fmt != LMP_F64) {
    sp = launch_pan_t_partial(nA, k, U, x, part, skip, nullptr, nullptr, s, &sb, &sc);
  } else {
    sp = lmp_t_splits(nA, k);
    const long long rows_per = (nA + sp - 1) / sp;
    hipLaunchKernelGGL(k_lmp_gemv_t_partial<double>, dim3((k + kTG - 1) / kTG, sp), dim3(kLT), 0, s, nA,
                       k, rows_per, (const double*)U.p, U.ldu, x, part, skip);
  }
  hipLaunchKernelGGL(k_lmp_gemv_t_final, dim3((k + 3) / 4), dim3(256), 0, s, sp, k, part, dcoef, t,
                     skip, sb, sc);
  return hipGetLastError();
}

hipError_t lmp_gemv_n(long long nA, int k, const LmpU& U, const double* x, double* y, const double* ws,
                      const int* skip, hipStream_t s) {
  const double* t = ws + lmp_gemv_t_offset(nA, k);
  const size_t lds = sizeof(double) * (k + 4 * kPanel);
  if (U.fmt == LMP_P16) {
    hipLaunchKernelGGL((k_lmp_pan_n<_Float16, 4>), dim3(lmp_panel_grid(nA)), dim3(kPanel), lds, s, nA, k,
                       (const _Float16*)U.p, U.cexp, t, x, y, skip);
    return hipGetLastError();
  }
  if (U.fmt == LMP_P32) {
    hipLaunchKernelGGL((k_lmp_pan_n<float, 2>), dim3(lmp_panel_grid(nA)), dim3(kPanel), lds, s, nA, k,
                       (const float*)U.p, (const int*)nullptr, t, x, y, skip);
    return hipGetLastError();
  }
  if (U.ldu % 4 != 0) return hipErrorInvalidValue;
  const long long nch = (nA + 4LL * kLT - 1) / (4LL * kLT);
  hipLaunchKernelGGL(k_lmp_gemv_n<double>, dim3((unsigned)nch), dim3(kLT), sizeof(double) * k, s,
                       nA, k, (const double*)U.p, U.ldu, t, x, y, skip);
  return hipGetLastError();
}

}  // namespace wc4d
