// float64 MFMA GEMMs for gfx950.
//
// gemm_f64:  C(:, t) = alpha * A * B(:, t) [+ E(:, t)]  -- the D^{1/2} products
//            (A = B^{1/2} or Q^{1/2}, B = the time levels of a block of vectors),
//            the tall-skinny products Y R^{-1}, Z W and the LMP's U * T.
// gram_f64:  G = X^T Y for tall X, Y (Gram matrices of CholeskyQR2, K = Z^T A Z,
//            the LMP's U^T X), deterministic split-K.
//
// v_mfma_f64_16x16x4_f64 lane layout (wave64): operand a = A[l%16][l/16],
// operand b = B[l/16][l%16], result register r = D[l/16 + 4r][l%16].
// gemm_f64 runs the MFMA on the transposed product (rows of the MFMA are the
// columns t of C), so the 16 lanes that share l/16 hold 16 consecutive rows of
// one column of C and store 128 contiguous bytes.
#include "wc4d_internal.h"

#include <algorithm>

namespace wc4d {

typedef double d4 __attribute__((ext_vector_type(4)));

static __device__ inline d4 mfma16x16x4(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Tile BM (rows of C) x BN (columns of C), K step BK, 256 threads = WGI x WGJ waves.
// SPLIT: blockIdx.z takes K range [z kchunk, (z+1) kchunk) and writes its partial
// tile to ws + z M ncol (plain M x ncol); k_gemm_splitk_reduce finishes.
template <int BM, int BN, int BK, int WGI, int WGJ, bool SPLIT>
__global__ __launch_bounds__(256) void k_gemm_f64(int M, int ncol, int K, double alpha,
                                                  const double* __restrict__ A, long long lda,
                                                  const double* __restrict__ B, ColMap bmap,
                                                  double* __restrict__ C, ColMap cmap,
                                                  const double* __restrict__ E, ColMap emap,
                                                  const int* __restrict__ skip, int kchunk,
                                                  double* __restrict__ ws) {
  static_assert(WGI * WGJ == 4, "4 waves");
  constexpr int WI = BM / WGI, WJ = BN / WGJ;
  constexpr int TI = WI / 16, TJ = WJ / 16;
  static_assert(TI >= 1 && TJ >= 1, "wave tile >= 16x16");
  constexpr int NA = BM * BK / 256;
  constexpr int NB = BN * BK / 256;
  static_assert(NA >= 1 && NB >= 1, "tile too small for 256 threads");
  constexpr int PA = BM + 4, PB = BN + 4;
  __shared__ double As[BK][PA];
  __shared__ double Bs[BK][PB];

  if (skip != nullptr && *skip != 0) return;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int i0 = blockIdx.x * BM;
  const int j0 = blockIdx.y * BN;
  const int wi0 = (wave % WGI) * WI;
  const int wj0 = (wave / WGI) * WJ;
  const int kbeg = SPLIT ? blockIdx.z * kchunk : 0;
  const int kend0 = SPLIT ? min(K, kbeg + kchunk) : K;
  const int kend = bmap.upper ? min(kend0, j0 + BN) : kend0;  // upper triangular B: zeros below

  d4 acc[TJ][TI];
#pragma unroll
  for (int a = 0; a < TJ; ++a)
#pragma unroll
    for (int b = 0; b < TI; ++b) acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};

  long long boff[NB];
  bool bval[NB];
#pragma unroll
  for (int e = 0; e < NB; ++e) {
    const int j = (tid + 256 * e) / BK;
    bval[e] = (j0 + j) < ncol;
    boff[e] = bval[e] ? bmap.off(j0 + j) : 0;
  }
  double ra[NA], rb[NB];
  auto gload = [&](int k0) {
#pragma unroll
    for (int e = 0; e < NA; ++e) {
      const int idx = tid + 256 * e;
      const int gi = i0 + idx % BM, gk = k0 + idx / BM;
      ra[e] = (gi < M && gk < kend) ? A[(long long)gi + (long long)gk * lda] : 0.0;
    }
#pragma unroll
    for (int e = 0; e < NB; ++e) {
      const int gk = k0 + (tid + 256 * e) % BK;
      rb[e] = (bval[e] && gk < kend) ? B[boff[e] + gk] : 0.0;
    }
  };
  gload(kbeg);
  for (int k0 = kbeg; k0 < kend; k0 += BK) {
    __syncthreads();
#pragma unroll
    for (int e = 0; e < NA; ++e) {
      const int idx = tid + 256 * e;
      As[idx / BM][idx % BM] = ra[e];
    }
#pragma unroll
    for (int e = 0; e < NB; ++e) {
      const int idx = tid + 256 * e;
      Bs[idx % BK][idx / BK] = rb[e];
    }
    __syncthreads();
    if (k0 + BK < kend) gload(k0 + BK);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      const int kr = kk + (lane >> 4);
      double av[TJ], bv[TI];
#pragma unroll
      for (int a = 0; a < TJ; ++a) av[a] = Bs[kr][wj0 + a * 16 + (lane & 15)];
#pragma unroll
      for (int b = 0; b < TI; ++b) bv[b] = As[kr][wi0 + b * 16 + (lane & 15)];
#pragma unroll
      for (int a = 0; a < TJ; ++a)
#pragma unroll
        for (int b = 0; b < TI; ++b) acc[a][b] = mfma16x16x4(av[a], bv[b], acc[a][b]);
    }
  }
#pragma unroll
  for (int a = 0; a < TJ; ++a) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int j = j0 + wj0 + a * 16 + (lane >> 4) + 4 * r;
      if (j >= ncol) continue;
      if (SPLIT) {
        double* wz = ws + (size_t)blockIdx.z * M * ncol + (size_t)j * M;
#pragma unroll
        for (int b = 0; b < TI; ++b) {
          const int i = i0 + wi0 + b * 16 + (lane & 15);
          if (i < M) wz[i] = acc[a][b][r];
        }
        continue;
      }
      const long long co = cmap.off(j);
      const long long eo = (E != nullptr) ? emap.off(j) : 0;
      const double aj = alpha * cmap.colscale(j);
#pragma unroll
      for (int b = 0; b < TI; ++b) {
        const int i = i0 + wi0 + b * 16 + (lane & 15);
        if (i < M) {
          double v = aj * acc[a][b][r];
          if (E != nullptr) v += E[eo + i];
          C[co + i] = v;
        }
      }
    }
  }
}

__global__ void k_gemm_splitk_reduce(int M, int ncol, int splits, double alpha,
                                     const double* __restrict__ ws, double* __restrict__ C,
                                     ColMap cmap, const double* __restrict__ E, ColMap emap,
                                     const int* __restrict__ skip) {
  if (skip != nullptr && *skip != 0) return;
  const int j = blockIdx.y;
  const long long co = cmap.off(j);
  const long long eo = (E != nullptr) ? emap.off(j) : 0;
  const double aj = alpha * cmap.colscale(j);
  const size_t plane = (size_t)M * ncol;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < M; i += gridDim.x * blockDim.x) {
    double v = 0.0;
    for (int z = 0; z < splits; ++z) v += ws[z * plane + (size_t)j * M + i];
    v *= aj;
    if (E != nullptr) v += E[eo + i];
    C[co + i] = v;
  }
}

// Split-K variant for few columns (ncol <= BN) in which each wave owns 16 rows of A:
// a wave's A fragments (MFMA operand layout) come straight from global memory one K step
// ahead, only the B tile (shared by the 4 waves) is staged in LDS, double-buffered, so a
// K step needs one barrier and the next step's loads are in flight during the MFMAs.
template <int BN, int BK>
__global__ __launch_bounds__(256) void k_gemm_f64_pa(int M, int ncol, int K, const double* __restrict__ A,
                                                     long long lda, const double* __restrict__ B, ColMap bmap,
                                                     int kchunk, double* __restrict__ ws,
                                                     const int* __restrict__ skip) {
  constexpr int BM = 64, TJ = BN / 16, KS = BK / 4;
  constexpr int NB = BN * BK / 256;
  static_assert(BN % 16 == 0 && (BN * BK) % 256 == 0 && BK % 4 == 0, "tile shape");
  constexpr int PB = BN + 4;
  __shared__ double Bs[2][BK][PB];
  if (skip != nullptr && *skip != 0) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int i0 = blockIdx.x * BM;
  const int kbeg = blockIdx.z * kchunk;
  const int kend = min(K, kbeg + kchunk);
  // this lane's A row and the K offset of its MFMA operand within a 4-step
  const int ai = i0 + wave * 16 + (lane & 15);
  const bool arow = ai < M;
  const double* Ar = A + (arow ? ai : 0);
  const int ak = lane >> 4;
  d4 acc[TJ];
#pragma unroll
  for (int a = 0; a < TJ; ++a) acc[a] = d4{0.0, 0.0, 0.0, 0.0};
  long long boff[NB];
  bool bval[NB];
#pragma unroll
  for (int e = 0; e < NB; ++e) {
    const int j = (tid + 256 * e) / BK;
    bval[e] = j < ncol;
    boff[e] = bval[e] ? bmap.off(j) : 0;
  }
  double ra[KS], rb[NB];
  auto load_a = [&](int k0, double (&v)[KS]) {
#pragma unroll
    for (int q = 0; q < KS; ++q) {
      const int gk = k0 + 4 * q + ak;
      v[q] = (arow && gk < kend) ? Ar[(long long)gk * lda] : 0.0;
    }
  };
  auto load_b = [&](int k0) {
#pragma unroll
    for (int e = 0; e < NB; ++e) {
      const int gk = k0 + (tid + 256 * e) % BK;
      rb[e] = (bval[e] && gk < kend) ? B[boff[e] + gk] : 0.0;
    }
  };
  auto store_b = [&](int buf) {
#pragma unroll
    for (int e = 0; e < NB; ++e) {
      const int idx = tid + 256 * e;
      Bs[buf][idx % BK][idx / BK] = rb[e];
    }
  };
  load_b(kbeg);
  load_a(kbeg, ra);
  store_b(0);
  __syncthreads();
  int buf = 0;
  for (int k0 = kbeg; k0 < kend; k0 += BK) {
    const bool more = k0 + BK < kend;
    double na[KS];
    if (more) {
      load_b(k0 + BK);
      load_a(k0 + BK, na);
    }
#pragma unroll
    for (int q = 0; q < KS; ++q) {
      const int kr = 4 * q + ak;
      double av[TJ];
#pragma unroll
      for (int a = 0; a < TJ; ++a) av[a] = Bs[buf][kr][a * 16 + (lane & 15)];
#pragma unroll
      for (int a = 0; a < TJ; ++a) acc[a] = mfma16x16x4(av[a], ra[q], acc[a]);
    }
    if (more) {
      store_b(buf ^ 1);
#pragma unroll
      for (int q = 0; q < KS; ++q) ra[q] = na[q];
    }
    __syncthreads();
    buf ^= 1;
  }
  double* wz = ws + (size_t)blockIdx.z * M * ncol;
#pragma unroll
  for (int a = 0; a < TJ; ++a) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int j = a * 16 + (lane >> 4) + 4 * r;
      if (j < ncol && arow) wz[(size_t)j * M + ai] = acc[a][r];
    }
  }
}

template <int BN, int BK>
static hipError_t launch_gemm_split_pa(int M, int ncol, int K, int splits, double alpha, const double* A,
                                       long long lda, const double* B, ColMap bmap, double* C, ColMap cmap,
                                       const double* E, ColMap emap, const int* skip, double* ws,
                                       hipStream_t s) {
  int kchunk = (K + splits - 1) / splits;
  kchunk = (kchunk + BK - 1) / BK * BK;
  splits = (K + kchunk - 1) / kchunk;
  dim3 grid((M + 63) / 64, 1, splits);
  hipLaunchKernelGGL((k_gemm_f64_pa<BN, BK>), grid, dim3(256), 0, s, M, ncol, K, A, lda, B, bmap, kchunk, ws,
                     skip);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  dim3 rg((M + 255) / 256 < 64 ? (M + 255) / 256 : 64, ncol);
  hipLaunchKernelGGL(k_gemm_splitk_reduce, rg, dim3(256), 0, s, M, ncol, splits, alpha, ws, C, cmap, E, emap,
                     skip);
  return hipGetLastError();
}

template <int BM, int BN, int BK, int WGI, int WGJ>
static hipError_t launch_gemm(int M, int ncol, int K, double alpha, const double* A, long long lda,
                              const double* B, ColMap bmap, double* C, ColMap cmap,
                              const double* E, ColMap emap, const int* skip, hipStream_t s) {
  dim3 grid((M + BM - 1) / BM, (ncol + BN - 1) / BN);
  hipLaunchKernelGGL((k_gemm_f64<BM, BN, BK, WGI, WGJ, false>), grid, dim3(256), 0, s, M, ncol, K,
                     alpha, A, lda, B, bmap, C, cmap, E, emap, skip, K, nullptr);
  return hipGetLastError();
}

template <int BM, int BN, int BK, int WGI, int WGJ>
static hipError_t launch_gemm_split(int M, int ncol, int K, int splits, double alpha,
                                    const double* A, long long lda, const double* B, ColMap bmap,
                                    double* C, ColMap cmap, const double* E, ColMap emap,
                                    const int* skip, double* ws, hipStream_t s) {
  int kchunk = (K + splits - 1) / splits;
  kchunk = (kchunk + BK - 1) / BK * BK;
  splits = (K + kchunk - 1) / kchunk;
  dim3 grid((M + BM - 1) / BM, (ncol + BN - 1) / BN, splits);
  hipLaunchKernelGGL((k_gemm_f64<BM, BN, BK, WGI, WGJ, true>), grid, dim3(256), 0, s, M, ncol, K,
                     alpha, A, lda, B, bmap, C, cmap, E, emap, skip, kchunk, ws);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  dim3 rg((M + 255) / 256 < 64 ? (M + 255) / 256 : 64, ncol);
  hipLaunchKernelGGL(k_gemm_splitk_reduce, rg, dim3(256), 0, s, M, ncol, splits, alpha, ws, C, cmap,
                     E, emap, skip);
  return hipGetLastError();
}

// Split count for a split-K launch of `bn`-wide column tiles (0: not possible).
static long long split_count(int M, int ncol, int K, int bn, size_t ws_doubles, int want) {
  const long long t = (long long)((M + 63) / 64) * (long long)((ncol + bn - 1) / bn);
  long long splits = want > 0 ? want : (512 + t - 1) / t;
  splits = std::min<long long>(splits, K / 256);
  while (splits > 1 && (size_t)splits * M * ncol > ws_doubles) --splits;
  return splits >= 2 ? splits : 0;
}

bool gemm_tile_feasible(int tile, int M, int ncol, int K, const double* ws, size_t ws_doubles) {
  switch (tile) {
    case GEMM_AUTO: return true;
    case GEMM_SPLIT_64x16: return ws != nullptr && ncol <= 16 && split_count(M, ncol, K, 16, ws_doubles, 0) > 0;
    case GEMM_SPLIT_64x112:
    case GEMM_SPLIT_64x112_PA: return ws != nullptr && ncol <= 112 && split_count(M, ncol, K, 112, ws_doubles, 0) > 0;
    case GEMM_128x16: case GEMM_128x128: case GEMM_64x64: case GEMM_32x32: return true;
    default: return false;
  }
}

hipError_t gemm_f64_tile(int tile, int splits, int M, int ncol, int K, double alpha, const double* A,
                         long long lda, const double* B, ColMap bmap, double* C, ColMap cmap, const double* E,
                         ColMap emap, const int* skip, hipStream_t s, double* ws, size_t ws_doubles) {
  if (M <= 0 || ncol <= 0) return hipSuccess;
  auto tiles = [&](int bm, int bn) {
    return (long long)((M + bm - 1) / bm) * (long long)((ncol + bn - 1) / bn);
  };
  if (tile == GEMM_AUTO) {
    // Few output columns and a long K: split K so the launch fills the chip.
    if (ws != nullptr && ncol <= 112 && K >= 512 &&
        split_count(M, ncol, K, ncol <= 16 ? 16 : 112, ws_doubles, 0) > 0)
      tile = ncol <= 16 ? GEMM_SPLIT_64x16 : GEMM_SPLIT_64x112;
    else if (ncol <= 16)
      tile = GEMM_128x16;
    else if (tiles(128, 128) >= 1024)
      tile = GEMM_128x128;
    else if (tiles(64, 64) >= 1024)
      tile = GEMM_64x64;
    else
      tile = GEMM_32x32;
  }
  if (!gemm_tile_feasible(tile, M, ncol, K, ws, ws_doubles)) return hipErrorInvalidValue;
  switch (tile) {
    case GEMM_SPLIT_64x16: {
      const long long sp = split_count(M, ncol, K, 16, ws_doubles, splits);
      return launch_gemm_split<64, 16, 32, 4, 1>(M, ncol, K, (int)sp, alpha, A, lda, B, bmap, C, cmap, E, emap,
                                                 skip, ws, s);
    }
    case GEMM_SPLIT_64x112: {
      const long long sp = split_count(M, ncol, K, 112, ws_doubles, splits);
      return launch_gemm_split<64, 112, 32, 4, 1>(M, ncol, K, (int)sp, alpha, A, lda, B, bmap, C, cmap, E,
                                                  emap, skip, ws, s);
    }
    case GEMM_SPLIT_64x112_PA: {
      const long long sp = split_count(M, ncol, K, 112, ws_doubles, splits);
      return launch_gemm_split_pa<112, 32>(M, ncol, K, (int)sp, alpha, A, lda, B, bmap, C, cmap, E, emap, skip, ws,
                                           s);
    }
    case GEMM_128x16:
      return launch_gemm<128, 16, 16, 4, 1>(M, ncol, K, alpha, A, lda, B, bmap, C, cmap, E, emap, skip, s);
    case GEMM_128x128:
      return launch_gemm<128, 128, 16, 2, 2>(M, ncol, K, alpha, A, lda, B, bmap, C, cmap, E, emap, skip, s);
    case GEMM_64x64:
      return launch_gemm<64, 64, 16, 2, 2>(M, ncol, K, alpha, A, lda, B, bmap, C, cmap, E, emap, skip, s);
    default:
      return launch_gemm<32, 32, 16, 2, 2>(M, ncol, K, alpha, A, lda, B, bmap, C, cmap, E, emap, skip, s);
  }
}

hipError_t gemm_f64(int M, int ncol, int K, double alpha, const double* A, long long lda,
                    const double* B, ColMap bmap, double* C, ColMap cmap, const double* E,
                    ColMap emap, const int* skip, hipStream_t s, double* ws, size_t ws_doubles) {
  return gemm_f64_tile(GEMM_AUTO, 0, M, ncol, K, alpha, A, lda, B, bmap, C, cmap, E, emap, skip, s, ws,
                       ws_doubles);
}

// ----------------------------------------------- two-segment few-column product
// Y = S1 X1 (columns t < n1) and S2 X2 (columns t < n2) in one split-K launch: the
// D^{1/2} product of one or two vectors (S1 = Q^{1/2} on the N later time levels,
// S2 = B^{1/2} on time level 0).  blockIdx.z < z1 works on segment 1, the rest on
// segment 2; MFMA column tiles past a segment's column count are skipped, so the
// B^{1/2} segment costs a matrix-vector product.  k_dsqrt2_reduce sums the K splits
// of both segments in a fixed order and applies the epilogue.
struct Seg {
  const double* A;
  ColMap bmap, cmap, emap;
  int ncol;
  int splits;
  int kchunk;
  size_t wsoff;  // doubles
};

constexpr int SBN = 112;

// SBM rows x SBN columns per workgroup, K staged SBK at a time; 4 waves each own SBM / 4
// rows (SBM / 64 MFMA row blocks) and all SBN columns.
template <int SBM, int SBK>
__global__ __launch_bounds__(256) void k_dsqrt2(int M, int K, long long lda, const double* __restrict__ B,
                                                Seg s1, Seg s2, double* __restrict__ ws,
                                                const int* __restrict__ skip) {
  constexpr int WI = SBM / 4, RB = WI / 16, WJ = SBN;
  constexpr int TJ = WJ / 16;
  constexpr int NA = SBM * SBK / 256, NB = SBN * SBK / 256;
  __shared__ double As[SBK][SBM + 4];
  __shared__ double Bs[SBK][SBN + 4];
  if (skip != nullptr && *skip != 0) return;
  const bool first = (int)blockIdx.z < s1.splits;
  const Seg& sg = first ? s1 : s2;
  const int z = first ? blockIdx.z : blockIdx.z - s1.splits;
  const int ncol = sg.ncol;
  const double* __restrict__ A = sg.A;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int i0 = blockIdx.x * SBM;
  const int wi0 = wave * WI;
  const int kbeg = z * sg.kchunk;
  const int kend = min(K, kbeg + sg.kchunk);
  d4 acc[RB][TJ];
#pragma unroll
  for (int r = 0; r < RB; ++r)
#pragma unroll
    for (int a = 0; a < TJ; ++a) acc[r][a] = d4{0.0, 0.0, 0.0, 0.0};
  long long boff[NB];
  bool bval[NB];
#pragma unroll
  for (int e = 0; e < NB; ++e) {
    const int j = (tid + 256 * e) / SBK;
    bval[e] = j < ncol;
    boff[e] = bval[e] ? sg.bmap.off(j) : 0;
  }
  double ra[NA], rb[NB];
  auto gload = [&](int k0) {
#pragma unroll
    for (int e = 0; e < NA; ++e) {
      const int idx = tid + 256 * e;
      const int gi = i0 + idx % SBM, gk = k0 + idx / SBM;
      ra[e] = (gi < M && gk < kend) ? A[(long long)gi + (long long)gk * lda] : 0.0;
    }
#pragma unroll
    for (int e = 0; e < NB; ++e) {
      const int gk = k0 + (tid + 256 * e) % SBK;
      rb[e] = (bval[e] && gk < kend) ? B[boff[e] + gk] : 0.0;
    }
  };
  gload(kbeg);
  for (int k0 = kbeg; k0 < kend; k0 += SBK) {
    __syncthreads();
#pragma unroll
    for (int e = 0; e < NA; ++e) {
      const int idx = tid + 256 * e;
      As[idx / SBM][idx % SBM] = ra[e];
    }
#pragma unroll
    for (int e = 0; e < NB; ++e) {
      const int idx = tid + 256 * e;
      Bs[idx % SBK][idx / SBK] = rb[e];
    }
    __syncthreads();
    if (k0 + SBK < kend) gload(k0 + SBK);
#pragma unroll
    for (int kk = 0; kk < SBK; kk += 4) {
      const int kr = kk + (lane >> 4);
      double bv[RB];
#pragma unroll
      for (int r = 0; r < RB; ++r) bv[r] = As[kr][wi0 + 16 * r + (lane & 15)];
#pragma unroll
      for (int a = 0; a < TJ; ++a) {
        if (a * 16 < ncol) {
          const double xv = Bs[kr][a * 16 + (lane & 15)];
#pragma unroll
          for (int r = 0; r < RB; ++r) acc[r][a] = mfma16x16x4(xv, bv[r], acc[r][a]);
        }
      }
    }
  }
  double* wz = ws + sg.wsoff + (size_t)z * M * ncol;
#pragma unroll
  for (int r = 0; r < RB; ++r)
#pragma unroll
    for (int a = 0; a < TJ; ++a) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int j = a * 16 + (lane >> 4) + 4 * q;
        const int i = i0 + wi0 + 16 * r + (lane & 15);
        if (j < ncol && i < M) wz[(size_t)j * M + i] = acc[r][a][q];
      }
    }
}

__global__ void k_dsqrt2_reduce(int M, Seg s1, Seg s2, double alpha, const double* __restrict__ ws,
                                double* __restrict__ C, const double* __restrict__ E,
                                const int* __restrict__ skip) {
  if (skip != nullptr && *skip != 0) return;
  const bool first = (int)blockIdx.y < s1.ncol;
  const Seg& sg = first ? s1 : s2;
  const int j = first ? blockIdx.y : blockIdx.y - s1.ncol;
  const long long co = sg.cmap.off(j);
  const long long eo = (E != nullptr) ? sg.emap.off(j) : 0;
  const double aj = alpha * sg.cmap.colscale(j);
  const size_t plane = (size_t)M * sg.ncol;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < M; i += gridDim.x * blockDim.x) {
    double v = 0.0;
    for (int zz = 0; zz < sg.splits; ++zz) v += ws[sg.wsoff + zz * plane + (size_t)j * M + i];
    v *= aj;
    if (E != nullptr) v += E[eo + i];
    C[co + i] = v;
  }
}

static int dsqrt2_rows(int variant) { return variant == 0 ? 64 : 128; }

// K splits of a two-segment launch: the request (or enough to give ~512 workgroups per
// segment), at most K / 256, and no more than ws holds (0 when even 1 split does not fit).
static int dsqrt2_splits(int variant, int splits, int M, int n1, int n2, int K, size_t ws_doubles) {
  const int tiles = (M + dsqrt2_rows(variant) - 1) / dsqrt2_rows(variant);
  int sp = splits > 0 ? splits : (512 + tiles - 1) / tiles;
  sp = std::max(1, std::min(sp, std::max(1, K / 256)));
  while (sp > 1 && (size_t)sp * M * (n1 + n2) > ws_doubles) --sp;
  return ((size_t)sp * M * (n1 + n2) <= ws_doubles) ? sp : 0;
}

size_t dsqrt2_ws_doubles(int M, int n1, int n2, int K) {
  const int tiles = (M + 63) / 64;
  const int sp = std::max(1, std::min((512 + tiles - 1) / tiles, K / 256));
  return (size_t)sp * M * (n1 + n2);
}

bool dsqrt2_feasible(int variant, int splits, int M, int n1, int n2, int K, size_t ws_doubles) {
  if (variant < 0 || variant >= DSQRT2_NVARIANTS || n1 > SBN || n2 > SBN || n1 < 1 || n2 < 0) return false;
  const int sp = dsqrt2_splits(variant, splits, M, n1, n2, K, ws_doubles);
  return sp > 0 && (splits <= 0 || sp == splits);
}

hipError_t dsqrt2_f64_v(int variant, int splits, int M, int K, const double* B, double* C, const double* E,
                        const double* A1, ColMap b1, ColMap c1, ColMap e1, int n1, const double* A2, ColMap b2,
                        ColMap c2, ColMap e2, int n2, const int* skip, double* ws, size_t ws_doubles,
                        hipStream_t s) {
  if (!dsqrt2_feasible(variant, splits, M, n1, n2, K, ws_doubles)) return hipErrorInvalidValue;
  int sp = dsqrt2_splits(variant, splits, M, n1, n2, K, ws_doubles);
  const int sbk = variant == 1 ? 16 : 32;
  int kchunk = (K + sp - 1) / sp;
  kchunk = (kchunk + sbk - 1) / sbk * sbk;
  sp = (K + kchunk - 1) / kchunk;
  Seg s1{A1, b1, c1, e1, n1, sp, kchunk, 0};
  Seg s2{A2, b2, c2, e2, n2, sp, kchunk, (size_t)sp * M * n1};
  const int rows = dsqrt2_rows(variant);
  const dim3 grid((M + rows - 1) / rows, 1, (n2 > 0 ? 2 : 1) * sp);  // n2 = 0: one segment
  if (variant == 0)
    hipLaunchKernelGGL((k_dsqrt2<64, 32>), grid, dim3(256), 0, s, M, K, (long long)M, B, s1, s2, ws, skip);
  else if (variant == 1)
    hipLaunchKernelGGL((k_dsqrt2<128, 16>), grid, dim3(256), 0, s, M, K, (long long)M, B, s1, s2, ws, skip);
  else
    hipLaunchKernelGGL((k_dsqrt2<128, 32>), grid, dim3(256), 0, s, M, K, (long long)M, B, s1, s2, ws, skip);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  dim3 rg((M + 255) / 256 < 64 ? (M + 255) / 256 : 64, n1 + n2);
  hipLaunchKernelGGL(k_dsqrt2_reduce, rg, dim3(256), 0, s, M, s1, s2, 1.0, ws, C, E, skip);
  return hipGetLastError();
}

hipError_t dsqrt2_f64(int M, int K, const double* B, double* C, const double* E, const double* A1,
                      ColMap b1, ColMap c1, ColMap e1, int n1, const double* A2, ColMap b2, ColMap c2,
                      ColMap e2, int n2, const int* skip, double* ws, size_t ws_doubles, hipStream_t s) {
  return dsqrt2_f64_v(0, 0, M, K, B, C, E, A1, b1, c1, e1, n1, A2, b2, c2, e2, n2, skip, ws, ws_doubles, s);
}

// ------------------------------------------------------------------ Gram

constexpr int GT = 64;   // output tile
constexpr int GBK = 16;  // K step

static int gram_splits(int m1, int m2, long long K) {
  const long long tiles = (long long)((m1 + GT - 1) / GT) * ((m2 + GT - 1) / GT);
  long long want = (2048 + tiles - 1) / tiles;          // aim for ~2048 workgroups
  long long maxs = (K + 255) / 256;                      // at least 256 rows per split
  long long sp = want < maxs ? want : maxs;
  if (sp < 1) sp = 1;
  return (int)sp;
}

size_t gram_ws_doubles(int m1, int m2, long long K) {
  return (size_t)gram_splits(m1, m2, K) * (size_t)m1 * (size_t)m2;
}

// Partial G over rows [kb, ke) of one split, tile (blockIdx.x, blockIdx.y); with sym (X = Y,
// G symmetric) blockIdx.x numbers the tiles on and above the diagonal instead.
__global__ __launch_bounds__(256) void k_gram_partial(int m1, int m2, long long K, long long kchunk,
                                                      const double* __restrict__ X, ColMap xmap,
                                                      const double* __restrict__ Y, ColMap ymap,
                                                      double* __restrict__ ws,
                                                      const int* __restrict__ skip, int sym) {
  constexpr int NL = GT * GBK / 256;  // 4 loads per operand per thread
  __shared__ double Xs[GBK][GT + 4];
  __shared__ double Ys[GBK][GT + 4];
  if (skip != nullptr && *skip != 0) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  int ti = blockIdx.x, tj = blockIdx.y;
  if (sym) {  // row ti of the upper triangle holds T - ti tiles
    const int T = (m1 + GT - 1) / GT;
    int rem = blockIdx.x;
    ti = 0;
    while (rem >= T - ti) {
      rem -= T - ti;
      ++ti;
    }
    tj = ti + rem;
  }
  const int i0 = ti * GT, j0 = tj * GT;
  const int split = blockIdx.z;
  const long long kb = (long long)split * kchunk;
  long long ke = kb + kchunk;
  if (ke > K) ke = K;
  const int wi0 = (wave & 1) * 32, wj0 = (wave >> 1) * 32;
  d4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};
  long long xo[NL], yo[NL];
  bool xv[NL], yv[NL];
#pragma unroll
  for (int e = 0; e < NL; ++e) {
    const int c = (tid + 256 * e) / GBK;
    xv[e] = (i0 + c) < m1;
    yv[e] = (j0 + c) < m2;
    xo[e] = xv[e] ? xmap.off(i0 + c) : 0;
    yo[e] = yv[e] ? ymap.off(j0 + c) : 0;
  }
  double rx[NL], ry[NL];
  auto gload = [&](long long k0) {
#pragma unroll
    for (int e = 0; e < NL; ++e) {
      const long long gk = k0 + (tid + 256 * e) % GBK;
      rx[e] = (xv[e] && gk < ke) ? X[xo[e] + gk] : 0.0;
      ry[e] = (yv[e] && gk < ke) ? Y[yo[e] + gk] : 0.0;
    }
  };
  if (kb < ke) gload(kb);
  for (long long k0 = kb; k0 < ke; k0 += GBK) {
    __syncthreads();
#pragma unroll
    for (int e = 0; e < NL; ++e) {
      const int idx = tid + 256 * e;
      Xs[idx % GBK][idx / GBK] = rx[e];
      Ys[idx % GBK][idx / GBK] = ry[e];
    }
    __syncthreads();
    if (k0 + GBK < ke) gload(k0 + GBK);
#pragma unroll
    for (int kk = 0; kk < GBK; kk += 4) {
      const int kr = kk + (lane >> 4);
      double av[2], bv[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) av[a] = Xs[kr][wi0 + a * 16 + (lane & 15)];
#pragma unroll
      for (int b = 0; b < 2; ++b) bv[b] = Ys[kr][wj0 + b * 16 + (lane & 15)];
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = mfma16x16x4(av[a], bv[b], acc[a][b]);
    }
  }
  double* out = ws + (size_t)split * m1 * m2;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = i0 + wi0 + a * 16 + (lane >> 4) + 4 * r;
        const int j = j0 + wj0 + b * 16 + (lane & 15);
        if (i < m1 && j < m2) out[(size_t)i + (size_t)j * m1] = acc[a][b][r];
      }
}

__global__ void k_gram_reduce(int m1, int m2, int splits, const double* __restrict__ ws,
                              double* __restrict__ G, int ldg, const int* __restrict__ skip, int sym) {
  if (skip != nullptr && *skip != 0) return;
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long tot = (long long)m1 * m2;
  if (e >= tot) return;
  const int i = (int)(e % m1), j = (int)(e / m1);
  // symmetric: an entry below the diagonal tiles is its mirror image's (the same products in
  // the same order, so the same bits as computing it)
  const long long src = (sym && i / GT > j / GT) ? (long long)j + (long long)i * m1 : e;
  double sum = 0.0;
  for (int sp = 0; sp < splits; ++sp) sum += ws[(size_t)sp * tot + src];
  G[(size_t)i + (size_t)j * ldg] = sum;
}

hipError_t gram_f64(int m1, int m2, long long K, const double* X, ColMap xmap, const double* Y,
                    ColMap ymap, double* G, int ldg, double* ws, const int* skip, hipStream_t s) {
  if (m1 <= 0 || m2 <= 0) return hipSuccess;
  const int sp = gram_splits(m1, m2, K);
  long long kchunk = (K + sp - 1) / sp;
  kchunk = (kchunk + GBK - 1) / GBK * GBK;
  // X^T X: only the tiles on and above the diagonal (a Nystrom build at n_A = 413,696, m = 256:
  // 41 against 44 ms, the same bits)
  const int sym = (X == Y && m1 == m2 && xmap.ld == ymap.ld && xmap.per == ymap.per && xmap.base == ymap.base &&
                   xmap.stride == ymap.stride)
                      ? 1
                      : 0;
  const int T1 = (m1 + GT - 1) / GT;
  dim3 grid(sym ? T1 * (T1 + 1) / 2 : T1, sym ? 1 : (m2 + GT - 1) / GT, sp);
  hipLaunchKernelGGL(k_gram_partial, grid, dim3(256), 0, s, m1, m2, K, kchunk, X, xmap, Y, ymap,
                     ws, skip, sym);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const long long tot = (long long)m1 * m2;
  hipLaunchKernelGGL(k_gram_reduce, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, m1, m2,
                     sp, ws, G, ldg, skip, sym);
  return hipGetLastError();
}

}  // namespace wc4d
