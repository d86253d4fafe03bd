// Few-column products Y = S X with S fixed (the D^{1/2} product of one vector over all its
// time levels, S = Q^{1/2}) on the int8 matrix cores, by an error-free splitting of both
// operands into int8 slices (the Ozaki scheme: Ozaki, Ogita, Oishi and Rump, "Error-free
// transformations of matrix multiplication by using fast routines of matrix multiplication
// and its applications", Numer. Algorithms 59, 2012; its integer form as in Ootomo, Ozaki and
// Yokota, "DGEMM on integer matrix multiplication unit", IJHPCA 2024).
//
// Row i of S is written as 2^{e_i} sum_{t=1..6} a_t 2^{-7t} with integer digits |a_t| <= 127
// (e_i = floor(log2 max_k |S_ik|) + 1, so |S_ik| 2^{-e_i} < 1, truncated after 42 bits), and
// column j of X likewise with exponent f_j and digits b_u.  Then
//     (S X)_ij ~= 2^{e_i + f_j} sum_{t + u <= 7} 2^{-7 (t + u)} sum_k a_t(i, k) b_u(k, j),
// where every inner sum is an exact int32 product on v_mfma_i32_16x16x64_i8 (|sum| <= 6 K 127^2
// < 2^31 for K <= 8192 per split).  The 21 pairs with t + u <= 7 are kept; the others and the
// truncation leave an error of a few K 2^{-42} relative to max_k |S_ik| max_k |X_kj|: about
// 2e-11 of a column's largest entry for n = 4096 (a CPU model of the same arithmetic), against
// 1e-16 for float64 arithmetic.  Each output's levels t + u = 2..7 keep their own int32
// accumulator and are combined in float64 at the end, so the result does not depend on the
// launch shape beyond the split-K sum (fixed order).
//
// Layouts (fragment-major: every MFMA operand is one contiguous 1 KB piece, lane l's 16
// bytes at l * 16).  Slices of S: int8 [kOzS][nR / 16][nK / 64][1024], the piece (t, rb, ks)
// holding rows 16 rb + l % 16 and K 64 ks + 16 (l / 16) .. + 16 (nR, nK: n rounded up to 64,
// zero padded); row exponents int [nR].  Slices of X: int8 [kOzS][Lp / 16][nK / 64][1024], the
// piece (u, cb, ks) holding columns 16 cb + l % 16 (Lp = L rounded up to 112); column
// exponents int [Lp].  Split-K partials: float64 [splits][Lp][n].
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "wc4d_internal.h"

namespace wc4d {
namespace {

constexpr int kOzS = 6;          // slices per operand
constexpr int kOzBits = 7;       // bits per digit
constexpr int kOzCB = 7;         // 16-column blocks per launch chunk (112 columns)
constexpr int kOzLP = 16 * kOzCB;
constexpr int kOzLev = 2 * kOzS - (kOzS - 1) - 1;  // levels t + u = 2..kOzS + 1

typedef int v4i __attribute__((ext_vector_type(4)));

// exponent e with |v| < 2^e for the largest magnitude v of a row or column (0 for zeros)
__device__ inline int oz_exponent(double vmax) {
  if (!(vmax > 0.0)) return 0;
  int e;
  (void)frexp(vmax, &e);  // vmax = f 2^e, f in [0.5, 1)
  return e;
}

// the kOzS digits of v 2^{-e} (|v| < 2^e), truncated toward zero after 7 kOzS bits
__device__ inline void oz_digits(double v, int e, signed char (&d)[kOzS]) {
  const double a = ldexp(fabs(v), kOzS * kOzBits - e);  // < 2^(7 kOzS), exact
  unsigned long long m = (unsigned long long)a;         // truncation
  const bool neg = v < 0.0;
#pragma unroll
  for (int t = kOzS - 1; t >= 0; --t) {
    const int dig = (int)(m & 127ull);
    m >>= kOzBits;
    d[t] = (signed char)(neg ? -dig : dig);
  }
}

// ---- slices of S (once): per-row exponents, then 64 x 64 tiles through LDS
__global__ __launch_bounds__(256) void k_oz_row_exp(const double* __restrict__ S, long long lds, int n,
                                                     int* __restrict__ es) {
  __shared__ double red[4][64];
  const int i = blockIdx.x * 64 + (threadIdx.x & 63), part = threadIdx.x >> 6;
  double mx = 0.0;
  if (i < n)
    for (int k = part; k < n; k += 4) mx = fmax(mx, fabs(S[(long long)k * lds + i]));
  red[part][threadIdx.x & 63] = mx;
  __syncthreads();
  if (part == 0) {
    const double m = fmax(fmax(red[0][threadIdx.x], red[1][threadIdx.x]), fmax(red[2][threadIdx.x], red[3][threadIdx.x]));
    es[i] = (i < n) ? oz_exponent(m) : 0;
  }
}

__global__ __launch_bounds__(256) void k_oz_split_rows(const double* __restrict__ S, long long lds, int n, int nR,
                                                       int nK, const int* __restrict__ es, signed char* __restrict__ Ss) {
  __shared__ double tile[64][65];  // [k][i]
  const int i0 = blockIdx.x * 64, k0 = blockIdx.y * 64;
  for (int q = threadIdx.x; q < 64 * 64; q += 256) {
    const int ii = q & 63, kk = q >> 6;
    const int i = i0 + ii, k = k0 + kk;
    tile[kk][ii] = (i < n && k < n) ? S[(long long)k * lds + i] : 0.0;
  }
  __syncthreads();
  // thread: row ii = tid / 4, 16 consecutive k at 16 (tid % 4): one lane's piece of a fragment
  const int ii = threadIdx.x >> 2, kq = (threadIdx.x & 3) * 16;
  const int e = es[i0 + ii];
  const int nRB = nR / 16, nKS = nK / 64, rb = (i0 + ii) >> 4, fl = ((i0 + ii) & 15) + 16 * (threadIdx.x & 3);
  signed char out[kOzS][16];
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    signed char d[kOzS];
    oz_digits(tile[kq + j][ii], e, d);
#pragma unroll
    for (int t = 0; t < kOzS; ++t) out[t][j] = d[t];
  }
#pragma unroll
  for (int t = 0; t < kOzS; ++t) {
    v4i w;
    __builtin_memcpy(&w, out[t], 16);
    *reinterpret_cast<v4i*>(Ss + (((size_t)t * nRB + rb) * nKS + k0 / 64) * 1024 + fl * 16) = w;
  }
}

// ---- slices of X (per call): one workgroup of 1024 threads per column (zero past L); each
// thread holds four consecutive k of the column in registers (looping for n > 4096), so the
// column is read once for its largest magnitude and sliced from registers
__global__ __launch_bounds__(1024) void k_oz_split_cols(const double* __restrict__ X, long long ldc, int n, int L,
                                                        int nK, int Lpad, signed char* __restrict__ Xs,
                                                        int* __restrict__ fs, const int* __restrict__ skip) {
  if (skip != nullptr && *skip != 0) return;
  __shared__ double red[16];
  const int j = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const double* x = X + (long long)j * ldc;
  const bool live = j < L;
  double mx = 0.0;
  for (int k = 4 * tid; k < n; k += 4096)
    if (live) {
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (k + q < n) mx = fmax(mx, fabs(x[k + q]));
    }
  for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o));
  if (lane == 0) red[wave] = mx;
  __syncthreads();
  double m = red[0];
#pragma unroll
  for (int w = 1; w < 16; ++w) m = fmax(m, red[w]);
  const int f = oz_exponent(m);
  if (tid == 0) fs[j] = live ? f : 0;
  for (int k0 = 4 * tid; k0 < nK; k0 += 4096) {
    signed char out[kOzS][4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int k = k0 + q;
      signed char d[kOzS];
      oz_digits((live && k < n) ? x[k] : 0.0, f, d);
#pragma unroll
      for (int t = 0; t < kOzS; ++t) out[t][q] = d[t];
    }
    const int fl = (j & 15) + 16 * ((k0 & 63) >> 4);
#pragma unroll
    for (int t = 0; t < kOzS; ++t) {
      int w;
      __builtin_memcpy(&w, out[t], 4);
      *reinterpret_cast<int*>(Xs + (((size_t)t * (Lpad / 16) + (j >> 4)) * (nK / 64) + k0 / 64) * 1024 + fl * 16 +
                              (k0 & 15)) = w;
    }
  }
}

// ---- the product: workgroup = 64 rows x 112 columns x one K range; 16 waves: wave w takes
// rows 16 (w & 3) .. + 16 and the column blocks {2 (w >> 2), 2 (w >> 2) + 1} of the 7 (the last
// group only block 6).  Each K step's operands, the X pieces (kOzS slices x 7 column blocks)
// and the S pieces (kOzS slices x 4 row groups), are copied global -> LDS by the load-to-LDS
// instruction (no registers) one step ahead, double buffered (wave w copies pieces w, w + 16,
// ...); every wave waits for all of its loads before the barrier that hands the buffer over,
// so no ordering of memory operations is assumed.  Four waves per SIMD hide what one step
// ahead does not.
template <int NSTEP>
__global__ __launch_bounds__(1024, 1) void k_oz_gemm(const signed char* __restrict__ Ss, const int* __restrict__ es,
                                                    const signed char* __restrict__ Xs,
                                                    const int* __restrict__ fs, int n, int nR, int nK, int Lpad,
                                                    int kchunk, double* __restrict__ P,
                                                    const int* __restrict__ skip) {
  if (skip != nullptr && *skip != 0) return;
  constexpr int kFrag = 1024;
  constexpr int kXP = kOzS * kOzCB, kSP = kOzS * 4, kPieces = kXP + kSP;  // pieces per step
  constexpr int kStage = kPieces * kFrag;
  extern __shared__ __align__(16) signed char xl[];  // [2][kPieces][1024]: X pieces, then S pieces
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int rg = wave & 3, cg = wave >> 2;
  const int cb0 = 2 * cg, ncb = cg < 3 ? 2 : 1;
  const int i0 = blockIdx.x * 64 + 16 * rg;
  const int split = blockIdx.y, chunk = blockIdx.z;
  const int nKS = nK / 64, nRB = nR / 16, nCB = Lpad / 16;
  const int ksb = split * (kchunk / 64), kse = min(nKS, ksb + kchunk / 64);
  const int col0 = chunk * kOzLP;
  // piece p of step ks: p < kXP: X (slice p / 7, block p % 7); else S (slice q / 4, row
  // group q % 4), q = p - kXP
  constexpr int kFull = kPieces / 16;  // pieces every wave copies; the first kPieces % 16 waves one more
  auto load_step = [&](int ks, int stage) {
#pragma unroll
    for (int j = 0; j <= kFull; ++j) {
      const int p = wave + 16 * j;
      if (j == kFull && p >= kPieces) break;
      const signed char* src;
      if (p < kXP) {
        const int u = p / kOzCB, cb = p - u * kOzCB;
        src = Xs + (((size_t)u * nCB + chunk * kOzCB + cb) * nKS + ks) * kFrag;
      } else {
        const int q = p - kXP, t = q >> 2, r = q & 3;
        src = Ss + (((size_t)t * nRB + blockIdx.x * 4 + r) * nKS + ks) * kFrag;
      }
      __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)(src + lane * 16),
                                       (__attribute__((address_space(3))) void*)(xl + stage * kStage + p * kFrag),
                                       16, 0, 0);
    }
  };
  v4i acc[2][kOzLev];
#pragma unroll
  for (int b = 0; b < 2; ++b)
#pragma unroll
    for (int l = 0; l < kOzLev; ++l) acc[b][l] = v4i{0, 0, 0, 0};
  auto step = [&](int ks) {
    const int stage = (ks - ksb) & 1;
    // all of this wave's copies (this step's operands) and LDS reads (the previous step's)
    // done, then the barrier hands the buffers over; the empty asm statements keep the
    // compiler from moving memory accesses across it
    __builtin_amdgcn_s_waitcnt(0);
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
    load_step(min(ks + 1, kse - 1), stage ^ 1);
    const signed char* base = xl + stage * kStage + lane * 16;
    v4i sa[kOzS];
#pragma unroll
    for (int t = 0; t < kOzS; ++t) sa[t] = *reinterpret_cast<const v4i*>(base + (kXP + 4 * t + rg) * kFrag);
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      if (b < ncb) {
        v4i xv[kOzS];
#pragma unroll
        for (int u = 0; u < kOzS; ++u) xv[u] = *reinterpret_cast<const v4i*>(base + (u * kOzCB + cb0 + b) * kFrag);
#pragma unroll
        for (int t = 0; t < kOzS; ++t)
#pragma unroll
          for (int u = 0; u < kOzS; ++u)
            if (t + u <= kOzS - 1)
              acc[b][t + u] = __builtin_amdgcn_mfma_i32_16x16x64_i8(sa[t], xv[u], acc[b][t + u], 0, 0, 0);
      }
    }
  };
  if (ksb < kse) {
    load_step(ksb, 0);
    if (NSTEP > 0) {
#pragma unroll
      for (int i = 0; i < NSTEP; ++i) step(ksb + i);
    } else {
      for (int ks = ksb; ks < kse; ++ks) step(ks);
    }
    __builtin_amdgcn_s_waitcnt(0);  // the unused copies of the last step
  }
  // combine the levels in float64: level l (digit pair t + u = l + 2) weighs 2^{-7 (l + 2)}
#pragma unroll
  for (int b = 0; b < 2; ++b) {
    if (b >= ncb) continue;
    const int c = col0 + 16 * (cb0 + b) + (lane & 15);
    const int f = fs[c];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = i0 + 4 * (lane >> 4) + r;
      double v = 0.0;
#pragma unroll
      for (int l = kOzLev - 1; l >= 0; --l) v = v * 0x1p-7 + (double)acc[b][l][r];
      v = ldexp(v, es[i] + f - 2 * kOzBits);
      if (i < n) P[((size_t)split * Lpad + c) * n + i] = v;
    }
  }
}

// Y(:, j) = E(:, j) + sc_j sum_s P[s](:, j), sc_0 = scale0, else 1 (fixed order)
__global__ void k_oz_reduce(const double* __restrict__ P, int splits, int n, int L, int Lpad, long long ldc,
                            double scale0, const double* __restrict__ E, double* __restrict__ Y,
                            const int* __restrict__ skip) {
  if (skip != nullptr && *skip != 0) return;
  const long long total = (long long)n * L;
  for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < total;
       q += (long long)gridDim.x * blockDim.x) {
    const int j = (int)(q / n), i = (int)(q - (long long)j * n);
    double v = 0.0;
    for (int s = 0; s < splits; ++s) v += P[((size_t)s * Lpad + j) * n + i];
    if (j == 0) v *= scale0;
    const long long o = (long long)j * ldc + i;
    Y[o] = (E != nullptr ? E[o] : 0.0) + v;
  }
}

// two buffers of one K step's pieces: X (kOzS x 7) and S (kOzS x 4), 1 KB each
size_t oz_gemm_lds() { return (size_t)2 * (kOzS * kOzCB + kOzS * 4) * 1024; }

}  // namespace

size_t oz_slices_bytes(int n) {
  const size_t nR = (size_t)(n + 63) / 64 * 64;
  return (size_t)kOzS * nR * nR;
}

int oz_padded(int n) { return (n + 63) / 64 * 64; }

int oz_lpad(int L) { return (L + kOzLP - 1) / kOzLP * kOzLP; }

size_t oz_xs_bytes(int n, int L) { return (size_t)kOzS * oz_lpad(L) * oz_padded(n); }

int oz_splits(int n, int L) {
  const int tiles = oz_padded(n) / 64, chunks = oz_lpad(L) / kOzLP, ksteps = oz_padded(n) / 64;
  int sp = std::max(1, (256 + tiles * chunks - 1) / (tiles * chunks));
  sp = std::min(sp, ksteps);
  // at most 8192 of K per split (int32 range of the accumulators)
  const int kchunk_steps = (ksteps + sp - 1) / sp;
  if (kchunk_steps * 64 > 8192) sp = (ksteps + 127) / 128;
  return sp;
}

size_t oz_partials_doubles(int n, int L) { return (size_t)oz_splits(n, L) * oz_lpad(L) * n; }

hipError_t oz_split_matrix(const double* S, long long lds, int n, signed char* Ss, int* es, hipStream_t s) {
  const int nR = oz_padded(n);
  hipLaunchKernelGGL(k_oz_row_exp, dim3(nR / 64), dim3(256), 0, s, S, lds, n, es);
  hipLaunchKernelGGL(k_oz_split_rows, dim3(nR / 64, nR / 64), dim3(256), 0, s, S, lds, n, nR, nR, es, Ss);
  return hipGetLastError();
}

hipError_t oz_gemm(int n, int L, const signed char* Ss, const int* es, const double* X, long long ldc,
                   double scale0, const double* E, double* Y, signed char* Xs, int* fs, double* P,
                   const int* skip, hipStream_t s) {
  const int nR = oz_padded(n), nK = nR, Lpad = oz_lpad(L);
  const int splits = oz_splits(n, L);
  const int ksteps = nK / 64;
  const int kchunk = (ksteps + splits - 1) / splits * 64;
  hipLaunchKernelGGL(k_oz_split_cols, dim3(Lpad), dim3(1024), 0, s, X, ldc, n, L, nK, Lpad, Xs, fs, skip);
  const size_t lds = oz_gemm_lds();
  const dim3 ggrid(nR / 64, splits, Lpad / kOzLP);
  if (kchunk == 16 * 64 && ksteps % 16 == 0)
    hipLaunchKernelGGL(k_oz_gemm<16>, ggrid, dim3(1024), lds, s, Ss, es, Xs, fs, n, nR, nK, Lpad, kchunk, P, skip);
  else
    hipLaunchKernelGGL(k_oz_gemm<0>, ggrid, dim3(1024), lds, s, Ss, es, Xs, fs, n, nR, nK, Lpad, kchunk, P, skip);
  const long long total = (long long)n * L;
  const int grid = (int)std::min<long long>((total + 255) / 256, 2048);
  hipLaunchKernelGGL(k_oz_reduce, dim3(grid), dim3(256), 0, s, P, splits, n, L, Lpad, ldc, scale0, E, Y, skip);
  return hipGetLastError();
}

hipError_t oz_set_lds_limit() {
  const size_t lds = oz_gemm_lds();
  hipError_t e = hipFuncSetAttribute((const void*)k_oz_gemm<0>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void*)k_oz_gemm<16>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  return e;
}

}  // namespace wc4d
