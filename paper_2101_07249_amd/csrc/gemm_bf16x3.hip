// Split-precision GEMM for the D^{1/2} products of the sketch block applies:
// C = alpha S X [+ E] with float64 inputs and outputs, computed as
//   S_hi X_hi + S_hi X_lo + S_lo X_hi,   S = S_hi + S_lo, X = X_hi + X_lo (bfloat16 pairs),
// on v_mfma_f32_16x16x32_bf16 with float32 accumulation.  The dropped S_lo X_lo term
// and the bfloat16 rounding of the low parts are O(2^-16) relative; the float32 sum
// over K adds O(sqrt(K) 2^-24).
//
// Two kernels for each form.  The LDS-tiled ones (k_gemm_bf16x3, k_gemm_fp16x3): S is
// pre-split once (split_bf16_rows, split_f16_rows) into two row-major arrays (row i holds
// S(i, 0..K-1) contiguously), so an MFMA operand row is one 16-byte load, and X is split
// while it is staged into LDS.  The fragment-major one (k_gemm_x3_frag, products with many
// 256 x 256 tiles such as the sketch block's all-level product): both operands are pre-split
// into 1 KB MFMA operand pieces that are copied global -> LDS without passing through
// registers (layout below).  Both form the same three products in the same K order, so they
// give the same bits.
//
// The float16 form (gemm_fp16x3) has 11 significant bits per part instead of 8 but a
// narrow exponent range, so both operands are scaled by powers of two: row i of S by
// 2^-eS_i and column j of X by 2^-eX_j, chosen so the row's / column's largest magnitude
// lands in [2^14, 2^15).  With S = 2^eS (Sh + Sl) and X likewise (Sl, Xl the float16
// rounding residuals),
//   S X ~ 2^(eS + eX) (Sh Xh + Sh Xl + Sl Xh)
// in one float32 accumulator; the dropped Sl Xl term is O(2^-22) relative.  A residual is
// subnormal only for an element more than 2^17 below its row's / column's largest, whose
// share of the product is below 2^-17, so the loss stays below 2^-28 relative.  The
// column exponents of X come from a pre-pass (k_col_exponents).
//
// v_mfma_f32_16x16x32_bf16 lane layout (wave64): operand a = A[l%16][8(l/16) + e],
// operand b = B[8(l/16) + e][l%16] (e = 0..7), result register r = D[4(l/16) + r][l%16].
// As in gemm_f64 the product is formed transposed (MFMA rows = columns t of C), so a
// lane's results are 4 consecutive columns of one row and the 16 lanes sharing l/16
// store 16 consecutive rows of a column.
#include <cstdlib>
#include <cstring>

#include "wc4d_internal.h"

namespace wc4d {

typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));

static __device__ inline f4 mfma_bf16(bf8 a, bf8 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

static __device__ inline void split2(double x, __bf16& hi, __bf16& lo) {
  hi = (__bf16)(float)x;
  lo = (__bf16)(float)(x - (double)(float)hi);
}

// Shi/Slo (row-major, ld K): S(i, k) for i < M, k < K from column-major S (lds).
__global__ void k_split_bf16_rows(int M, int K, const double* __restrict__ S, long long lds,
                                  __bf16* __restrict__ Shi, __bf16* __restrict__ Slo) {
  const long long tot = (long long)M * K;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < tot;
       e += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(e / K), k = (int)(e % K);
    __bf16 h, l;
    split2(S[(size_t)i + (size_t)k * lds], h, l);
    Shi[e] = h;
    Slo[e] = l;
  }
}

hipError_t split_bf16_rows(int M, int K, const double* S, long long lds, __bf16* Shi, __bf16* Slo,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_split_bf16_rows, dim3(2048), dim3(256), 0, s, M, K, S, lds, Shi, Slo);
  return hipGetLastError();
}

// Power-of-two exponent e with max |v| 2^-e in [2^14, 2^15) (0 for an all-zero set).
static __device__ inline int scale_exponent(double amax) {
  if (!(amax > 0.0)) return 0;
  return ilogb(amax) - 14;
}

static __device__ inline void split_f16(double x, int e, _Float16& hi, _Float16& lo) {
  const double y = ldexp(x, -e);
  hi = (_Float16)y;
  lo = (_Float16)(y - (double)hi);
}

// Row exponents of S and its float16 parts (row-major, ld K): one workgroup per row.
__global__ __launch_bounds__(256) void k_split_f16_rows(int M, int K, const double* __restrict__ S, long long lds,
                                                         _Float16* __restrict__ Shi, _Float16* __restrict__ Slo,
                                                         int* __restrict__ rowexp) {
  __shared__ double sh[256];
  for (int i = blockIdx.x; i < M; i += gridDim.x) {
    double m = 0.0;
    for (int k = threadIdx.x; k < K; k += 256) m = fmax(m, fabs(S[(size_t)i + (size_t)k * lds]));
    sh[threadIdx.x] = m;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + w]);
      __syncthreads();
    }
    const int e = scale_exponent(sh[0]);
    __syncthreads();
    if (threadIdx.x == 0) rowexp[i] = e;
    for (int k = threadIdx.x; k < K; k += 256) {
      _Float16 h, l;
      split_f16(S[(size_t)i + (size_t)k * lds], e, h, l);
      Shi[(size_t)i * K + k] = h;
      Slo[(size_t)i * K + k] = l;
    }
  }
}

hipError_t split_f16_rows(int M, int K, const double* S, long long lds, _Float16* Shi, _Float16* Slo, int* rowexp,
                          hipStream_t s) {
  hipLaunchKernelGGL(k_split_f16_rows, dim3(M < 2048 ? M : 2048), dim3(256), 0, s, M, K, S, lds, Shi, Slo, rowexp);
  return hipGetLastError();
}

// Column exponents of X (K rows, columns through bmap): one workgroup per column.
__global__ __launch_bounds__(256) void k_col_exponents(int ncol, int K, const double* __restrict__ B, ColMap bmap,
                                                        int* __restrict__ colexp) {
  __shared__ double sh[256];
  for (int j = blockIdx.x; j < ncol; j += gridDim.x) {
    const double* x = B + bmap.off(j);
    double m = 0.0;
    for (int k = threadIdx.x; k < K; k += 256) m = fmax(m, fabs(x[k]));
    sh[threadIdx.x] = m;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + w]);
      __syncthreads();
    }
    if (threadIdx.x == 0) colexp[j] = scale_exponent(sh[0]);
    __syncthreads();
  }
}

constexpr int XBM = 128, XBN = 128, XBK = 32;  // XBM: the float16 form's rows
constexpr int XPK = XBK + 8;  // LDS row pitch in bf16 (80 bytes)

// Tile: 64 WR rows (i) x XBN columns (j) of C; 2 WR waves as WR (i) x 2 (j), each 64 x 64.
// Loaders: two threads per S row (16 k each), NT / XBN threads per X column (KX k each).
// WR = 4 halves the number of row blocks that each re-read all of X.
template <int WR>
__global__ __launch_bounds__(128 * WR) void k_gemm_bf16x3(int M, int ncol, int K, double alpha,
                                                          const __bf16* __restrict__ Shi,
                                                          const __bf16* __restrict__ Slo,
                                                          const double* __restrict__ B, ColMap bmap,
                                                          double* __restrict__ C, ColMap cmap,
                                                          const double* __restrict__ E, ColMap emap) {
  constexpr int BM = 64 * WR, NT = 128 * WR, TPC = NT / XBN, KX = XBK / TPC;
  static_assert(KX % 8 == 0, "whole bf16x8 vectors per X loader thread");
  __shared__ __attribute__((aligned(16))) __bf16 Sh[BM][XPK], Sl[BM][XPK];
  __shared__ __attribute__((aligned(16))) __bf16 Xh[XBN][XPK], Xl[XBN][XPK];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int i0 = blockIdx.x * BM, j0 = blockIdx.y * XBN;
  const int wi0 = (wave % WR) * 64, wj0 = (wave / WR) * 64;
  f4 acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = f4{0.f, 0.f, 0.f, 0.f};

  const int lr = tid >> 1, lh = (tid & 1) * 16;           // S loader
  const int xc = tid / TPC, xk = (tid % TPC) * KX;        // X loader
  const bool srow_ok = (i0 + lr) < M;
  const __bf16* shp = Shi + (size_t)(srow_ok ? i0 + lr : 0) * K;
  const __bf16* slp = Slo + (size_t)(srow_ok ? i0 + lr : 0) * K;
  const bool xcol_ok = (j0 + xc) < ncol;
  const double* xp = B + (xcol_ok ? bmap.off(j0 + xc) : 0);
  bf8 rsh[2], rsl[2];
  double rx[KX];
  // 16-byte loads when the row / column start is aligned and the slab is inside K
  const bool svec = (K % 8) == 0;
  const bool xvec = ((reinterpret_cast<uintptr_t>(xp) & 15) == 0);
  auto gload = [&](int k0) {
    const int kb = k0 + lh;
    if (svec && kb + 16 <= K) {
#pragma unroll
      for (int v = 0; v < 2; ++v) {
        rsh[v] = srow_ok ? *reinterpret_cast<const bf8*>(shp + kb + 8 * v) : bf8{};
        rsl[v] = srow_ok ? *reinterpret_cast<const bf8*>(slp + kb + 8 * v) : bf8{};
      }
    } else {
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const bool ok = srow_ok && (kb + e) < K;
        rsh[e / 8][e % 8] = ok ? shp[kb + e] : (__bf16)0.f;
        rsl[e / 8][e % 8] = ok ? slp[kb + e] : (__bf16)0.f;
      }
    }
    const int xb = k0 + xk;
    if (xvec && xb + KX <= K) {
#pragma unroll
      for (int v = 0; v < KX / 2; ++v) {
        const double2 d2 = xcol_ok ? *reinterpret_cast<const double2*>(xp + xb + 2 * v) : double2{0.0, 0.0};
        rx[2 * v] = d2.x;
        rx[2 * v + 1] = d2.y;
      }
    } else {
#pragma unroll
      for (int e = 0; e < KX; ++e) rx[e] = (xcol_ok && (xb + e) < K) ? xp[xb + e] : 0.0;
    }
  };
  gload(0);
  for (int k0 = 0; k0 < K; k0 += XBK) {
    __syncthreads();
    *reinterpret_cast<bf8*>(&Sh[lr][lh]) = rsh[0];
    *reinterpret_cast<bf8*>(&Sh[lr][lh + 8]) = rsh[1];
    *reinterpret_cast<bf8*>(&Sl[lr][lh]) = rsl[0];
    *reinterpret_cast<bf8*>(&Sl[lr][lh + 8]) = rsl[1];
#pragma unroll
    for (int v = 0; v < KX / 8; ++v) {
      bf8 h0, l0;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        __bf16 h, l;
        split2(rx[8 * v + e], h, l);
        h0[e] = h;
        l0[e] = l;
      }
      *reinterpret_cast<bf8*>(&Xh[xc][xk + 8 * v]) = h0;
      *reinterpret_cast<bf8*>(&Xl[xc][xk + 8 * v]) = l0;
    }
    __syncthreads();
    if (k0 + XBK < K) gload(k0 + XBK);
    const int kk = 8 * (lane >> 4);
    bf8 xh[4], xl[4], sh[4], sl[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const int j = wj0 + a * 16 + (lane & 15);
      xh[a] = *reinterpret_cast<const bf8*>(&Xh[j][kk]);
      xl[a] = *reinterpret_cast<const bf8*>(&Xl[j][kk]);
    }
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int i = wi0 + b * 16 + (lane & 15);
      sh[b] = *reinterpret_cast<const bf8*>(&Sh[i][kk]);
      sl[b] = *reinterpret_cast<const bf8*>(&Sl[i][kk]);
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        acc[a][b] = mfma_bf16(xh[a], sh[b], acc[a][b]);
        acc[a][b] = mfma_bf16(xl[a], sh[b], acc[a][b]);
        acc[a][b] = mfma_bf16(xh[a], sl[b], acc[a][b]);
      }
  }
  // acc[a][b][r] = C[i = i0 + wi0 + 16 b + l%16][j = j0 + wj0 + 16 a + 4 (l/16) + r]
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int j = j0 + wj0 + a * 16 + 4 * (lane >> 4) + r;
      if (j >= ncol) continue;
      const long long co = cmap.off(j);
      const long long eo = (E != nullptr) ? emap.off(j) : 0;
      const double sc = alpha * cmap.colscale(j);
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int i = i0 + wi0 + b * 16 + (lane & 15);
        if (i < M) {
          double v = sc * (double)acc[a][b][r];
          if (E != nullptr) v += E[eo + i];
          C[co + i] = v;
        }
      }
    }
}

typedef _Float16 h8 __attribute__((ext_vector_type(8)));

static __device__ inline f4 mfma_f16(h8 a, h8 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
}

// Same tiling as k_gemm_bf16x3, with the row and column exponents applied in the epilogue.
__global__ __launch_bounds__(256) void k_gemm_fp16x3(int M, int ncol, int K, double alpha,
                                                     const _Float16* __restrict__ Shi,
                                                     const _Float16* __restrict__ Slo,
                                                     const int* __restrict__ rowexp,
                                                     const double* __restrict__ B, ColMap bmap,
                                                     const int* __restrict__ colexp,
                                                     double* __restrict__ C, ColMap cmap,
                                                     const double* __restrict__ E, ColMap emap) {
  __shared__ __attribute__((aligned(16))) _Float16 Sh[XBM][XPK], Sl[XBM][XPK];
  __shared__ __attribute__((aligned(16))) _Float16 Xh[XBN][XPK], Xl[XBN][XPK];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int i0 = blockIdx.x * XBM, j0 = blockIdx.y * XBN;
  const int wi0 = (wave & 1) * 64, wj0 = (wave >> 1) * 64;
  f4 acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = f4{0.f, 0.f, 0.f, 0.f};
  const int lr = tid >> 1, lh = (tid & 1) * 16;
  const bool srow_ok = (i0 + lr) < M;
  const _Float16* shp = Shi + (size_t)(srow_ok ? i0 + lr : 0) * K;
  const _Float16* slp = Slo + (size_t)(srow_ok ? i0 + lr : 0) * K;
  const bool xcol_ok = (j0 + lr) < ncol;
  const double* xp = B + (xcol_ok ? bmap.off(j0 + lr) : 0);
  const int xe = xcol_ok ? colexp[j0 + lr] : 0;
  h8 rsh[2], rsl[2];
  double rx[16];
  const bool svec = (K % 8) == 0;
  const bool xvec = ((reinterpret_cast<uintptr_t>(xp) & 15) == 0);
  auto gload = [&](int k0) {
    const int kb = k0 + lh;
    if (svec && kb + 16 <= K) {
#pragma unroll
      for (int v = 0; v < 2; ++v) {
        rsh[v] = srow_ok ? *reinterpret_cast<const h8*>(shp + kb + 8 * v) : h8{};
        rsl[v] = srow_ok ? *reinterpret_cast<const h8*>(slp + kb + 8 * v) : h8{};
      }
    } else {
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const bool ok = srow_ok && (kb + e) < K;
        rsh[e / 8][e % 8] = ok ? shp[kb + e] : (_Float16)0.f;
        rsl[e / 8][e % 8] = ok ? slp[kb + e] : (_Float16)0.f;
      }
    }
    if (xvec && kb + 16 <= K) {
#pragma unroll
      for (int v = 0; v < 8; ++v) {
        const double2 d2 = xcol_ok ? *reinterpret_cast<const double2*>(xp + kb + 2 * v) : double2{0.0, 0.0};
        rx[2 * v] = d2.x;
        rx[2 * v + 1] = d2.y;
      }
    } else {
#pragma unroll
      for (int e = 0; e < 16; ++e) rx[e] = (xcol_ok && (kb + e) < K) ? xp[kb + e] : 0.0;
    }
  };
  gload(0);
  for (int k0 = 0; k0 < K; k0 += XBK) {
    __syncthreads();
    *reinterpret_cast<h8*>(&Sh[lr][lh]) = rsh[0];
    *reinterpret_cast<h8*>(&Sh[lr][lh + 8]) = rsh[1];
    *reinterpret_cast<h8*>(&Sl[lr][lh]) = rsl[0];
    *reinterpret_cast<h8*>(&Sl[lr][lh + 8]) = rsl[1];
    {
      h8 h0, h1, l0, l1;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        _Float16 h, l;
        split_f16(rx[e], xe, h, l);
        h0[e] = h;
        l0[e] = l;
        split_f16(rx[8 + e], xe, h, l);
        h1[e] = h;
        l1[e] = l;
      }
      *reinterpret_cast<h8*>(&Xh[lr][lh]) = h0;
      *reinterpret_cast<h8*>(&Xh[lr][lh + 8]) = h1;
      *reinterpret_cast<h8*>(&Xl[lr][lh]) = l0;
      *reinterpret_cast<h8*>(&Xl[lr][lh + 8]) = l1;
    }
    __syncthreads();
    if (k0 + XBK < K) gload(k0 + XBK);
    const int kk = 8 * (lane >> 4);
    h8 xh[4], xl[4], sh[4], sl[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const int j = wj0 + a * 16 + (lane & 15);
      xh[a] = *reinterpret_cast<const h8*>(&Xh[j][kk]);
      xl[a] = *reinterpret_cast<const h8*>(&Xl[j][kk]);
    }
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int i = wi0 + b * 16 + (lane & 15);
      sh[b] = *reinterpret_cast<const h8*>(&Sh[i][kk]);
      sl[b] = *reinterpret_cast<const h8*>(&Sl[i][kk]);
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        acc[a][b] = mfma_f16(xh[a], sh[b], acc[a][b]);
        acc[a][b] = mfma_f16(xl[a], sh[b], acc[a][b]);
        acc[a][b] = mfma_f16(xh[a], sl[b], acc[a][b]);
      }
  }
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int j = j0 + wj0 + a * 16 + 4 * (lane >> 4) + r;
      if (j >= ncol) continue;
      const long long co = cmap.off(j);
      const long long eo = (E != nullptr) ? emap.off(j) : 0;
      const int ej = colexp[j];
      const double sc = alpha * cmap.colscale(j);
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int i = i0 + wi0 + b * 16 + (lane & 15);
        if (i < M) {
          double v = sc * ldexp((double)acc[a][b][r], rowexp[i] + ej);
          if (E != nullptr) v += E[eo + i];
          C[co + i] = v;
        }
      }
    }
}

hipError_t gemm_fp16x3(int M, int ncol, int K, double alpha, const _Float16* Shi, const _Float16* Slo,
                       const int* rowexp, const double* B, ColMap bmap, int* colexp, double* C, ColMap cmap,
                       const double* E, ColMap emap, hipStream_t s) {
  if (M <= 0 || ncol <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_col_exponents, dim3(ncol < 4096 ? ncol : 4096), dim3(256), 0, s, ncol, K, B, bmap, colexp);
  dim3 grid((M + XBM - 1) / XBM, (ncol + XBN - 1) / XBN);
  hipLaunchKernelGGL(k_gemm_fp16x3, grid, dim3(256), 0, s, M, ncol, K, alpha, Shi, Slo, rowexp, B, bmap, colexp, C,
                     cmap, E, emap);
  return hipGetLastError();
}

hipError_t gemm_bf16x3(int M, int ncol, int K, double alpha, const __bf16* Shi, const __bf16* Slo,
                       const double* B, ColMap bmap, double* C, ColMap cmap, const double* E,
                       ColMap emap, hipStream_t s) {
  if (M <= 0 || ncol <= 0) return hipSuccess;
  const long long cb = (ncol + XBN - 1) / XBN;
  // 256-row tiles (one 8-wave workgroup per CU) once the grid still holds 1024 of them
  // (measured at 4096 x 25,856 x 4096: 5.7 ms against 6.0 ms per call for 128-row tiles)
  if ((long long)((M + 255) / 256) * cb >= 1024) {
    dim3 grid((M + 255) / 256, (unsigned)cb);
    hipLaunchKernelGGL(k_gemm_bf16x3<4>, grid, dim3(512), 0, s, M, ncol, K, alpha, Shi, Slo, B, bmap, C, cmap, E,
                       emap);
  } else {
    dim3 grid((M + 127) / 128, (unsigned)cb);
    hipLaunchKernelGGL(k_gemm_bf16x3<2>, grid, dim3(256), 0, s, M, ncol, K, alpha, Shi, Slo, B, bmap, C, cmap, E,
                       emap);
  }
  return hipGetLastError();
}


// ---- fragment-major form for large products (the sketch block's all-level D^{1/2} product).
// Both operands are split (S once per problem, X per call) into bf16 hi/lo parts, or for the
// float16 form into scaled float16 hi/lo parts with the row / column exponents above, stored as
// 1 KB pieces in the MFMA operand order: piece (kb, blk, part) holds the 16 rows (columns of X)
// 16 blk .. + 16 and K 32 kb .. + 32, lane l's 8 values (row 16 blk + l % 16, K 32 kb + 8 (l / 16)
// + e) at 8 l; pieces ordered [kb][blk][part], rows / columns padded with zeros to a multiple
// of 256 and K to a multiple of 32.  The product then copies whole pieces global -> LDS with
// the load-to-LDS instruction (no registers, no LDS writes by the waves) and every lane's
// operand read is one conflict-free 16-byte LDS load.
constexpr int kFT = 256;  // tile rows and columns
constexpr int kFP = 512;  // 16-bit values per piece
constexpr int kFStage = 64 * kFP;  // one K step: 16 row blocks x 2 parts, then 16 column blocks x 2 parts

// the two 16-bit forms: element and operand types, the MFMA, and the hi/lo split (the
// float16 form scales by 2^-e first)
template <bool F16> struct Frag;
template <> struct Frag<false> {
  typedef __bf16 E;
  typedef bf8 V;
  static __device__ inline f4 mfma(V a, V b, f4 c) { return mfma_bf16(a, b, c); }
  static __device__ inline void split(double x, int, E& h, E& l) { split2(x, h, l); }
};
template <> struct Frag<true> {
  typedef _Float16 E;
  typedef h8 V;
  static __device__ inline f4 mfma(V a, V b, f4 c) { return mfma_f16(a, b, c); }
  static __device__ inline void split(double x, int e, E& h, E& l) { split_f16(x, e, h, l); }
};

// A(r, k) = XCOL ? A[amap.off(r) + k] : A[r + k lda], for r < R, k < K; zero outside.  exps
// (float16 form): the exponent of each r.
template <bool XCOL, bool F16>
__global__ __launch_bounds__(256) void k_split_frag(int R, int K, int nB, int nKB, const double* __restrict__ A,
                                                    long long lda, ColMap amap, const int* __restrict__ exps,
                                                    typename Frag<F16>::E* __restrict__ F) {
  typedef typename Frag<F16>::E Et;
  typedef typename Frag<F16>::V Vt;
  const long long tot = (long long)nB * nKB * 64;
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < tot;
       t += (long long)gridDim.x * blockDim.x) {
    const long long P = t >> 6;
    const int lane = (int)(t & 63);
    const int blk = (int)(P / nKB), kb = (int)(P - (long long)blk * nKB);
    const int r = 16 * blk + (lane & 15), k0 = 32 * kb + 8 * (lane >> 4);
    double v[8];
    int ex = 0;
    if (r < R) {
      if (F16) ex = exps[r];
      if (XCOL) {
        const double* col = A + amap.off(r);
        if (k0 + 8 <= K && (reinterpret_cast<uintptr_t>(col + k0) & 15) == 0) {
#pragma unroll
          for (int e = 0; e < 8; e += 2) {
            const double2 d2 = *reinterpret_cast<const double2*>(col + k0 + e);
            v[e] = d2.x;
            v[e + 1] = d2.y;
          }
        } else {
#pragma unroll
          for (int e = 0; e < 8; ++e) v[e] = (k0 + e < K) ? col[k0 + e] : 0.0;
        }
      } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) v[e] = (k0 + e < K) ? A[(size_t)r + (size_t)(k0 + e) * lda] : 0.0;
      }
    } else {
#pragma unroll
      for (int e = 0; e < 8; ++e) v[e] = 0.0;
    }
    Vt h, l;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      Et a, b;
      Frag<F16>::split(v[e], ex, a, b);
      h[e] = a;
      l[e] = b;
    }
    Et* dst = F + ((size_t)kb * nB + blk) * 2 * kFP + (size_t)lane * 8;
    *reinterpret_cast<Vt*>(dst) = h;
    *reinterpret_cast<Vt*>(dst + kFP) = l;
  }
}

// The product on fragment-major parts: one workgroup per 256 x 256 tile of C (rows of S x
// columns of X), 8 waves, wave w computing rows 64 (w & 3) .. + 64 and columns 128 (w >> 2) ..
// + 128 (4 x 8 blocks of 16 x 16, three MFMAs each per K step of 32).  Each K step's 64 pieces
// (64 KB) are copied into LDS one step ahead, double buffered; every wave waits for all of its
// copies and LDS reads before the barrier that hands a buffer over, so no ordering between
// memory operations is assumed.  Tiles are ordered so that the workgroups one XCD runs at a
// time share 4 row tiles (S) and a run of column tiles (X) in that XCD's L2.  The float16 form
// scales each output by 2^(rowexp_i + colexp_j).
template <bool F16>
__global__ __launch_bounds__(512, 1) void k_gemm_x3_frag(int M, int ncol, int nKB, int nRT, int nCT, double alpha,
                                                        const typename Frag<F16>::E* __restrict__ Sf,
                                                        const typename Frag<F16>::E* __restrict__ Xf,
                                                        const int* __restrict__ rowexp,
                                                        const int* __restrict__ colexp, double* __restrict__ C,
                                                        ColMap cmap, const double* __restrict__ E, ColMap emap) {
  typedef typename Frag<F16>::E Et;
  typedef typename Frag<F16>::V Vt;
  extern __shared__ __align__(16) char flb[];  // [2][64][kFP] 16-bit values
  Et* fl = reinterpret_cast<Et*>(flb);
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  // workgroup w runs on XCD w % 8: give each XCD a contiguous range of the tile order
  const int G = gridDim.x, wg = blockIdx.x;
  const int q8 = G >> 3, r8 = G & 7, xcd = wg & 7, loc = wg >> 3;
  const int L = (xcd < r8) ? xcd * (q8 + 1) + loc : r8 * (q8 + 1) + (xcd - r8) * q8 + loc;
  // tile order: groups of (up to) 4 row tiles, column tiles within a group
  const int GR = nRT < 4 ? nRT : 4;
  const int g = L / (GR * nCT), rem = L - g * GR * nCT;
  const int gs = (nRT - g * GR) < GR ? (nRT - g * GR) : GR;
  const int rt = g * GR + rem % gs, ct = rem / gs;
  const int nRB = 16 * nRT, nCB = 16 * nCT;
  const int wr = wave & 3, wc = wave >> 2;
  auto load_step = [&](int kb, int stage) {
#pragma unroll
    for (int jj = 0; jj < 8; ++jj) {
      const int pc = wave + 8 * jj;  // jj < 4: S pieces (row block pc / 2, part pc % 2); else X
      const Et* src = jj < 4 ? Sf + (((size_t)kb * nRB + 16 * rt + (pc >> 1)) * 2 + (pc & 1)) * kFP
                             : Xf + (((size_t)kb * nCB + 16 * ct + ((pc - 32) >> 1)) * 2 + (pc & 1)) * kFP;
      __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)(src + lane * 8),
                                       (__attribute__((address_space(3))) void*)(fl + (stage * 64 + pc) * kFP), 16,
                                       0, 0);
    }
  };
  f4 acc[8][4];
#pragma unroll
  for (int a = 0; a < 8; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = f4{0.f, 0.f, 0.f, 0.f};
  load_step(0, 0);
  for (int kb = 0; kb < nKB; ++kb) {
    const int stage = kb & 1;
    // this wave's copies of step kb and its LDS reads of step kb - 1 done, then the barrier
    // hands the buffers over; the empty asm statements keep memory accesses on their side
    __builtin_amdgcn_s_waitcnt(0);
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
    if (kb + 1 < nKB) load_step(kb + 1, stage ^ 1);
    const Et* base = fl + stage * kFStage + lane * 8;
    Vt sh[4], sl[4], xh[8], xl[8];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      sh[b] = *reinterpret_cast<const Vt*>(base + (2 * (4 * wr + b)) * kFP);
      sl[b] = *reinterpret_cast<const Vt*>(base + (2 * (4 * wr + b) + 1) * kFP);
    }
#pragma unroll
    for (int a = 0; a < 8; ++a) {
      const int px = 32 + 2 * (8 * wc + a);
      xh[a] = *reinterpret_cast<const Vt*>(base + px * kFP);
      xl[a] = *reinterpret_cast<const Vt*>(base + (px + 1) * kFP);
    }
#pragma unroll
    for (int a = 0; a < 8; ++a) {
#pragma unroll
      for (int b = 0; b < 4; ++b) acc[a][b] = Frag<F16>::mfma(xh[a], sh[b], acc[a][b]);
#pragma unroll
      for (int b = 0; b < 4; ++b) acc[a][b] = Frag<F16>::mfma(xl[a], sh[b], acc[a][b]);
#pragma unroll
      for (int b = 0; b < 4; ++b) acc[a][b] = Frag<F16>::mfma(xh[a], sl[b], acc[a][b]);
    }
    // instruction order: the S pieces and the first X pair, then the 12 MFMAs of each X pair
    // with the next pair's two LDS reads issued halfway (measured 2.02 ms per C3 product
    // against 2.26 ms when every pair's reads wait just before its MFMAs)
    __builtin_amdgcn_sched_group_barrier(0x100, 10, 0);
#pragma unroll
    for (int a = 0; a < 7; ++a) {
      __builtin_amdgcn_sched_group_barrier(0x008, 6, 0);
      __builtin_amdgcn_sched_group_barrier(0x100, 2, 0);
      __builtin_amdgcn_sched_group_barrier(0x008, 6, 0);
    }
    __builtin_amdgcn_sched_group_barrier(0x008, 12, 0);
  }
  // acc[a][b][r] = C[i = rt 256 + 64 wr + 16 b + l % 16][j = ct 256 + 128 wc + 16 a + 4 (l / 16) + r]
  const int i0 = rt * kFT + 64 * wr, j0 = ct * kFT + 128 * wc;
#pragma unroll
  for (int a = 0; a < 8; ++a)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int j = j0 + a * 16 + 4 * (lane >> 4) + r;
      if (j >= ncol) continue;
      const long long co = cmap.off(j);
      const long long eo = (E != nullptr) ? emap.off(j) : 0;
      const double sc = alpha * cmap.colscale(j);
      const int ej = F16 ? colexp[j] : 0;
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int i = i0 + b * 16 + (lane & 15);
        if (i < M) {
          double v = (double)acc[a][b][r];
          if (F16) v = ldexp(v, rowexp[i] + ej);
          v *= sc;
          if (E != nullptr) v += E[eo + i];
          C[co + i] = v;
        }
      }
    }
}

static int frag_tiles(int R) { return (R + kFT - 1) / kFT; }

size_t bf16_frag_elems(int R, int K) {
  return (size_t)frag_tiles(R) * kFT * (size_t)((K + 31) / 32) * 32 * 2;
}

bool split_use_frag(int M, int ncol) {
  const char* env = getenv("WC4D_SPLIT_GEMM_KERNEL");
  if (env != nullptr && strcmp(env, "frag") == 0) return true;
  if (env != nullptr && strcmp(env, "tiled") == 0) return false;
  // enough 256 x 256 tiles for two rounds of the 256 CUs (at one workgroup per CU)
  return (long long)frag_tiles(M) * frag_tiles(ncol) >= 512;
}

hipError_t split_bf16_frag_rows(int M, int K, const double* S, long long lds, __bf16* F, hipStream_t s) {
  const int nB = 16 * frag_tiles(M), nKB = (K + 31) / 32;
  hipLaunchKernelGGL((k_split_frag<false, false>), dim3(2048), dim3(256), 0, s, M, K, nB, nKB, S, lds, plain_cols(0),
                     nullptr, F);
  return hipGetLastError();
}

hipError_t split_f16_frag_rows(int M, int K, const double* S, long long lds, const int* rowexp, _Float16* F,
                               hipStream_t s) {
  const int nB = 16 * frag_tiles(M), nKB = (K + 31) / 32;
  hipLaunchKernelGGL((k_split_frag<false, true>), dim3(2048), dim3(256), 0, s, M, K, nB, nKB, S, lds, plain_cols(0),
                     rowexp, F);
  return hipGetLastError();
}

hipError_t split_frag_set_lds_limit() {
  hipError_t e = hipFuncSetAttribute((const void*)k_gemm_x3_frag<false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     2 * kFStage * 2);
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void*)k_gemm_x3_frag<true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            2 * kFStage * 2);
  return e;
}

hipError_t gemm_bf16x3_frag(int M, int ncol, int K, double alpha, const __bf16* Sf, const double* B, ColMap bmap,
                            __bf16* Xf, double* C, ColMap cmap, const double* E, ColMap emap, hipStream_t s) {
  if (M <= 0 || ncol <= 0) return hipSuccess;
  const int nRT = frag_tiles(M), nCT = frag_tiles(ncol), nKB = (K + 31) / 32;
  hipLaunchKernelGGL((k_split_frag<true, false>), dim3(4096), dim3(256), 0, s, ncol, K, 16 * nCT, nKB, B, 0LL, bmap,
                     nullptr, Xf);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_gemm_x3_frag<false>, dim3(nRT * nCT), dim3(512), 2 * kFStage * 2, s, M, ncol, nKB, nRT, nCT,
                     alpha, Sf, Xf, nullptr, nullptr, C, cmap, E, emap);
  return hipGetLastError();
}

hipError_t gemm_fp16x3_frag(int M, int ncol, int K, double alpha, const _Float16* Sf, const int* rowexp,
                            const double* B, ColMap bmap, int* colexp, _Float16* Xf, double* C, ColMap cmap,
                            const double* E, ColMap emap, hipStream_t s) {
  if (M <= 0 || ncol <= 0) return hipSuccess;
  const int nRT = frag_tiles(M), nCT = frag_tiles(ncol), nKB = (K + 31) / 32;
  hipLaunchKernelGGL(k_col_exponents, dim3(ncol < 4096 ? ncol : 4096), dim3(256), 0, s, ncol, K, B, bmap, colexp);
  hipLaunchKernelGGL((k_split_frag<true, true>), dim3(4096), dim3(256), 0, s, ncol, K, 16 * nCT, nKB, B, 0LL, bmap,
                     colexp, Xf);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_gemm_x3_frag<true>, dim3(nRT * nCT), dim3(512), 2 * kFStage * 2, s, M, ncol, nKB, nRT, nCT,
                     alpha, Sf, Xf, rowexp, colexp, C, cmap, E, emap);
  return hipGetLastError();
}

}  // namespace wc4d
