// Small dense float64 linear algebra on the device, for the m x m problems of the
// randomised eigendecompositions (m = sketch width <= 512): Cholesky (CholeskyQR2
// and Algorithm 4's E2 = C^T C), triangular inverse, small products and the
// symmetric eigenproblem (Algorithm 2's EVD, Algorithms 3 and 5).
#include <mutex>

#include "wc4d_internal.h"

#include <cmath>

namespace wc4d {

// ------------------------------------------------------------------ Cholesky
// Right-looking, one workgroup, matrix in global memory (L2 resident).  A pivot
// that falls to m * eps of its original diagonal (or below) counts as failure:
// the Gram matrix is numerically singular and CholeskyQR would not orthonormalise.
__global__ __launch_bounds__(1024) void k_chol_upper(int m, double* __restrict__ G, int ldg,
                                                     int* __restrict__ status) {
  __shared__ double s_piv;
  __shared__ int s_bad;
  __shared__ double s_diag0[512];
  const int tid = threadIdx.x, nt = blockDim.x;
  if (tid == 0) s_bad = 0;
  for (int k = tid; k < m; k += nt) s_diag0[k] = G[k + (size_t)k * ldg];
  __syncthreads();
  const double floor_rel = (double)m * 2.220446049250313e-16;
  for (int k = 0; k < m; ++k) {
    if (tid == 0) {
      const double d = G[k + (size_t)k * ldg];
      if (!(d > floor_rel * s_diag0[k]) || !isfinite(d)) {
        s_bad = 1;
        s_piv = 1.0;
      } else {
        s_piv = sqrt(d);
      }
    }
    __syncthreads();
    if (s_bad) break;
    const double piv = s_piv;
    // row k of R: R(k, j) = G(k, j) / R(k, k), j >= k
    for (int j = k + tid; j < m; j += nt) {
      const double v = (j == k) ? piv : G[k + (size_t)j * ldg] / piv;
      G[k + (size_t)j * ldg] = v;
    }
    __syncthreads();
    // trailing update of the upper triangle: G(i, j) -= R(k, i) R(k, j), k < i <= j.
    // Columns j are spread over the threads (several threads per column when there are
    // fewer columns than threads), each walking a strided share of rows i <= j.
    const int w = m - k - 1;
    if (w > 0) {
      const int tpc = max(1, nt / w);            // threads per column
      const int col = tid / tpc, sub = tid % tpc;
      for (int jj = col; jj < w; jj += nt / tpc) {
        const int j = k + 1 + jj;
        const double rkj = G[k + (size_t)j * ldg];
        double* gcol = G + (size_t)j * ldg;
        for (int i = k + 1 + sub; i <= j; i += tpc) gcol[i] -= G[k + (size_t)i * ldg] * rkj;
      }
    }
    __syncthreads();
  }
  if (s_bad) {
    if (tid == 0) *status = 1;
    return;
  }
  // zero the strict lower triangle
  const long long tot = (long long)m * m;
  for (long long e = tid; e < tot; e += nt) {
    const int i = (int)(e % m), j = (int)(e / m);
    if (i > j) G[i + (size_t)j * ldg] = 0.0;
  }
}

// The same factorisation blocked by 32 columns (still one workgroup): block row J of R
// (32 rows, columns c0 .. m) is factored in LDS (pivot, row scaling, and the update of the
// block's later rows, one step per column), written back, and then the trailing upper
// triangle takes the block's rank-32 update in 4 x 4 register tiles with the k terms in
// ascending order.  Every element therefore sees the same sequence of floating-point
// updates as in the kernel above; only the number of barriers per column changes.
constexpr int kCBK = 32;   // block width
__global__ __launch_bounds__(1024) void k_chol_upper_blk(int m, double* __restrict__ G, int ldg,
                                                         int* __restrict__ status) {
  extern __shared__ double sR[];   // kCBK x m: row r of the block row at sR[r m + j]
  __shared__ double s_diag0[512];
  __shared__ double s_piv;
  __shared__ int s_bad;
  const int tid = threadIdx.x, nt = blockDim.x;
  if (tid == 0) s_bad = 0;
  for (int k = tid; k < m; k += nt) s_diag0[k] = G[k + (size_t)k * ldg];
  __syncthreads();
  const double floor_rel = (double)m * 2.220446049250313e-16;
  for (int c0 = 0; c0 < m; c0 += kCBK) {
    const int bw = min(kCBK, m - c0), w = m - c0;
    // block row J of the current matrix (upper part)
    for (int e = tid; e < bw * w; e += nt) {
      const int r = e / w, j = c0 + e % w;
      sR[r * m + j] = (j >= c0 + r) ? G[(c0 + r) + (size_t)j * ldg] : 0.0;
    }
    __syncthreads();
    for (int kk = 0; kk < bw; ++kk) {
      const int k = c0 + kk;
      double* rk = sR + kk * m;
      if (tid == 0) {
        const double d = rk[k];
        if (!(d > floor_rel * s_diag0[k]) || !isfinite(d)) {
          s_bad = 1;
          s_piv = 1.0;
        } else {
          s_piv = sqrt(d);
        }
      }
      __syncthreads();
      if (s_bad) break;
      const double piv = s_piv;
      for (int j = k + tid; j < m; j += nt) rk[j] = (j == k) ? piv : rk[j] / piv;
      __syncthreads();
      // the block's later rows: G(i, j) -= R(k, i) R(k, j), k < i < c0 + bw, j >= i
      const int rows = bw - kk - 1;
      for (int e = tid; e < rows * w; e += nt) {
        const int r = kk + 1 + e / w, j = c0 + e % w;
        if (j >= c0 + r) sR[r * m + j] -= rk[c0 + r] * rk[j];
      }
      __syncthreads();
    }
    if (s_bad) break;
    // R's block row back to G
    for (int e = tid; e < bw * w; e += nt) {
      const int r = e / w, j = c0 + e % w;
      if (j >= c0 + r) G[(c0 + r) + (size_t)j * ldg] = sR[r * m + j];
    }
    // trailing update of rows and columns >= c1 (upper triangle), 4 x 4 tiles
    const int c1 = c0 + bw, wt = m - c1;
    if (wt > 0) {
      const int ntl = (wt + 3) / 4;
      for (int t = tid; t < ntl * ntl; t += nt) {
        const int ti = t / ntl, tj = t % ntl;
        if (ti > tj) continue;
        const int i0 = c1 + 4 * ti, j0 = c1 + 4 * tj;
        double acc[4][4];
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            const int i = i0 + r, j = j0 + c;
            acc[r][c] = (i < m && j < m && i <= j) ? G[i + (size_t)j * ldg] : 0.0;
          }
        for (int kk = 0; kk < bw; ++kk) {
          const double* rk = sR + kk * m;
          double ri[4], rj[4];
#pragma unroll
          for (int r = 0; r < 4; ++r) ri[r] = (i0 + r < m) ? rk[i0 + r] : 0.0;
#pragma unroll
          for (int c = 0; c < 4; ++c) rj[c] = (j0 + c < m) ? rk[j0 + c] : 0.0;
#pragma unroll
          for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int c = 0; c < 4; ++c) acc[r][c] -= ri[r] * rj[c];
        }
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            const int i = i0 + r, j = j0 + c;
            if (i < m && j < m && i <= j) G[i + (size_t)j * ldg] = acc[r][c];
          }
      }
    }
    __syncthreads();
  }
  if (s_bad) {
    if (tid == 0) *status = 1;
    return;
  }
  const long long tot = (long long)m * m;
  for (long long e = tid; e < tot; e += nt) {
    const int i = (int)(e % m), j = (int)(e / m);
    if (i > j) G[i + (size_t)j * ldg] = 0.0;
  }
}

hipError_t chol_upper(int m, double* G, int ldg, int* status, hipStream_t s) {
  if (m > 512) return hipErrorInvalidValue;
  const size_t lds = sizeof(double) * kCBK * (size_t)m;  // <= 128 KB
  static std::once_flag once;
  static hipError_t attr = hipSuccess;
  std::call_once(once, [] {
    attr = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_chol_upper_blk),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)(sizeof(double) * kCBK * 512));
  });
  if (attr == hipSuccess) {
    hipLaunchKernelGGL(k_chol_upper_blk, dim3(1), dim3(1024), lds, s, m, G, ldg, status);
  } else {
    hipLaunchKernelGGL(k_chol_upper, dim3(1), dim3(1024), 0, s, m, G, ldg, status);
  }
  return hipGetLastError();
}

// ------------------------------------------------------- triangular inverse
// Column j of X = R^{-1} solves R x = e_j by column-oriented back substitution;
// one wavefront per column, the column held in registers (lane l owns rows
// l, l + 64, ...).
template <int RPL>
__global__ __launch_bounds__(64) void k_tri_inv_upper(int m, const double* __restrict__ R, int ldr,
                                                      double* __restrict__ X, int ldi) {
  const int j = blockIdx.x;
  const int lane = threadIdx.x;
  double x[RPL];
#pragma unroll
  for (int t = 0; t < RPL; ++t) x[t] = (lane + 64 * t == j) ? 1.0 : 0.0;
  for (int i = j; i >= 0; --i) {
    // x_i /= R_ii (owner lane), broadcast, then x_l -= R_li x_i for l < i
    const int own = i & 63, slot = i >> 6;
    double xi = 0.0;
#pragma unroll
    for (int t = 0; t < RPL; ++t)
      if (t == slot) xi = x[t];
    xi = __shfl(xi, own, 64);
    xi /= R[i + (size_t)i * ldr];
#pragma unroll
    for (int t = 0; t < RPL; ++t) {
      const int l = lane + 64 * t;
      if (l == i) x[t] = xi;
      else if (l < i) x[t] -= R[l + (size_t)i * ldr] * xi;
    }
  }
#pragma unroll
  for (int t = 0; t < RPL; ++t) {
    const int l = lane + 64 * t;
    if (l < m) X[l + (size_t)j * ldi] = (l <= j) ? x[t] : 0.0;
  }
}

hipError_t tri_inv_upper(int m, const double* R, int ldr, double* Rinv, int ldi, hipStream_t s) {
  if (m <= 64) hipLaunchKernelGGL(k_tri_inv_upper<1>, dim3(m), dim3(64), 0, s, m, R, ldr, Rinv, ldi);
  else if (m <= 128) hipLaunchKernelGGL(k_tri_inv_upper<2>, dim3(m), dim3(64), 0, s, m, R, ldr, Rinv, ldi);
  else if (m <= 256) hipLaunchKernelGGL(k_tri_inv_upper<4>, dim3(m), dim3(64), 0, s, m, R, ldr, Rinv, ldi);
  else if (m <= 512) hipLaunchKernelGGL(k_tri_inv_upper<8>, dim3(m), dim3(64), 0, s, m, R, ldr, Rinv, ldi);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

// ------------------------------------------------------------- small GEMM
__global__ void k_small_gemm(int M, int N, int K, double alpha, const double* __restrict__ A,
                             int lda, int tA, const double* __restrict__ B, int ldb, int tB,
                             double* __restrict__ C, int ldc) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (i >= M) return;
  double acc = 0.0;
  for (int k = 0; k < K; ++k) {
    const double a = tA ? A[k + (size_t)i * lda] : A[i + (size_t)k * lda];
    const double b = tB ? B[j + (size_t)k * ldb] : B[k + (size_t)j * ldb];
    acc += a * b;
  }
  C[i + (size_t)j * ldc] = alpha * acc;
}

hipError_t small_gemm(int M, int N, int K, double alpha, const double* A, int lda, int tA,
                      const double* B, int ldb, int tB, double* C, int ldc, hipStream_t s) {
  if (M <= 0 || N <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_small_gemm, dim3((M + 127) / 128, N), dim3(128), 0, s, M, N, K, alpha, A,
                     lda, tA, B, ldb, tB, C, ldc);
  return hipGetLastError();
}

// ------------------------------------------------------------ Jacobi EVD
// Round-robin (circle) pairing: round r pairs 2 h players into h disjoint pairs,
// player 0 fixed; over rounds 0 .. 2h - 2 every pair meets once.

static __device__ inline void rr_pair(int r, int k, int mp, int& p, int& q) {
  const int c = mp - 1;
  int a, b;
  if (k == 0) {
    a = 0;
    b = 1 + (r + mp - 2) % c;
  } else {
    a = 1 + (r + k - 1) % c;
    b = 1 + (r + mp - 2 - k) % c;
  }
  p = a < b ? a : b;
  q = a < b ? b : a;
}

// One-sided (Hestenes) block Jacobi for the SPD m x m matrices of the randomised
// methods: find orthogonal V with W = K V having orthogonal columns; then
// K v_i = ||w_i|| v_i.  Columns are split into nblk blocks of bs; in each block
// round workgroup g takes the block pair (P, Q) of the round-robin schedule, holds
// those 2 bs columns of W and V in LDS and rotates every pair among them (2 bs - 1
// local rounds, one pair per wavefront).  A sweep is nblk - 1 block rounds; the
// iteration stops after a sweep without rotations.  Rotation of columns (a, b)
// with alpha = |a|^2, beta = |b|^2, gamma = a.b: zeta = (beta - alpha) / (2 gamma),
// t = sign(zeta) / (|zeta| + sqrt(1 + zeta^2)), c = 1 / sqrt(1 + t^2), s = c t,
// a <- c a - s b, b <- s a + c b, which makes the pair orthogonal.
constexpr int kOJT = 1024;

struct OjCfg {
  int bs, nblk;
};

static OjCfg oj_cfg(int m) {
  OjCfg c;
  // 8 columns per block (4 bs m doubles of LDS): at m = 256, 16 block pairs per round with
  // 15 local rounds each build the Nystrom LMP 2.6 ms faster than 8 pairs of 16 columns with
  // 31 local rounds (the rotations' float64 arithmetic is the work; more pairs spread it)
  c.bs = 8;
  c.nblk = (m + c.bs - 1) / c.bs;
  if (c.nblk < 2) c.nblk = 2;
  c.nblk += c.nblk & 1;
  return c;
}

__global__ __launch_bounds__(kOJT) void k_oj_init(int m, double* __restrict__ K, int ldk,
                                                  double* __restrict__ V, int ldv, int* ctrl, int sym) {
  for (long long e = threadIdx.x; e < (long long)m * m; e += kOJT) {
    const int i = (int)(e % m), j = (int)(e / m);
    if (sym && i < j) {
      const double v = 0.5 * (K[i + (size_t)j * ldk] + K[j + (size_t)i * ldk]);
      K[i + (size_t)j * ldk] = v;
      K[j + (size_t)i * ldk] = v;
    }
    V[i + (size_t)j * ldv] = (i == j) ? 1.0 : 0.0;
  }
  if (threadIdx.x == 0) {
    ctrl[0] = 0;  // converged
    ctrl[1] = 0;  // rotations in the current sweep
  }
}

// MR = rows per lane (m <= 64 MR).
template <int MR>
__global__ __launch_bounds__(kOJT) void k_oj_round(int m, int bs, int nblk, int r,
                                                   double* __restrict__ W, int ldw,
                                                   double* __restrict__ V, int ldv, int* ctrl,
                                                   double tol) {
  extern __shared__ double lds[];
  if (ctrl[0]) return;
  int P, Q;
  rr_pair(r, blockIdx.x, nblk, P, Q);
  const int nloc = 2 * bs;
  double* Ws = lds;
  double* Vs = lds + (size_t)nloc * m;
  auto gcol = [&](int c) { return c < bs ? P * bs + c : Q * bs + (c - bs); };
  for (long long e = threadIdx.x; e < (long long)nloc * m; e += kOJT) {
    const int c = (int)(e / m), i = (int)(e % m);
    const int gc = gcol(c);
    Ws[e] = gc < m ? W[i + (size_t)gc * ldw] : 0.0;
    Vs[e] = gc < m ? V[i + (size_t)gc * ldv] : 0.0;
  }
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  int rot = 0;
  for (int lr = 0; lr < nloc - 1; ++lr) {
    if (wave < bs) {
      int a, b;
      rr_pair(lr, wave, nloc, a, b);
      if (gcol(a) < m && gcol(b) < m) {
        double* wa_p = Ws + (size_t)a * m;
        double* wb_p = Ws + (size_t)b * m;
        double wa[MR], wb[MR];
        double al = 0.0, be = 0.0, ga = 0.0;
#pragma unroll
        for (int t = 0; t < MR; ++t) {
          const int i = lane + 64 * t;
          wa[t] = i < m ? wa_p[i] : 0.0;
          wb[t] = i < m ? wb_p[i] : 0.0;
          al += wa[t] * wa[t];
          be += wb[t] * wb[t];
          ga += wa[t] * wb[t];
        }
        al = wave_sum_d(al);
        be = wave_sum_d(be);
        ga = wave_sum_d(ga);
        if (ga != 0.0 && ga * ga > tol * tol * (al * be)) {  // |ga| > tol sqrt(al be)
          const double zeta = (be - al) / (2.0 * ga);
          const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
          const double c = 1.0 / sqrt(1.0 + t * t), sn = c * t;
          double* va_p = Vs + (size_t)a * m;
          double* vb_p = Vs + (size_t)b * m;
#pragma unroll
          for (int q = 0; q < MR; ++q) {
            const int i = lane + 64 * q;
            if (i < m) {
              wa_p[i] = c * wa[q] - sn * wb[q];
              wb_p[i] = sn * wa[q] + c * wb[q];
              const double va = va_p[i], vb = vb_p[i];
              va_p[i] = c * va - sn * vb;
              vb_p[i] = sn * va + c * vb;
            }
          }
          ++rot;
        }
      }
    }
    __syncthreads();
  }
  for (long long e = threadIdx.x; e < (long long)nloc * m; e += kOJT) {
    const int c = (int)(e / m), i = (int)(e % m);
    const int gc = gcol(c);
    if (gc < m) {
      W[i + (size_t)gc * ldw] = Ws[e];
      V[i + (size_t)gc * ldv] = Vs[e];
    }
  }
  if (lane == 0 && rot > 0) atomicAdd(&ctrl[1], rot);
}

__global__ void k_oj_sweep_end(int* ctrl) {
  if (threadIdx.x != 0 || ctrl[0]) return;
  if (ctrl[1] == 0) ctrl[0] = 1;
  ctrl[1] = 0;
}

// eigenvalues = column norms of W, sorted decreasing (stable), vectors = columns of V
// with the largest-magnitude entry made positive; W is reused as scratch.
__global__ __launch_bounds__(kOJT) void k_oj_finish(int m, double* __restrict__ W, int ldw,
                                                    double* __restrict__ V, int ldv,
                                                    double* __restrict__ lam) {
  __shared__ double nrm[512];
  __shared__ int rank_of[512];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int c = wave; c < m; c += kOJT / 64) {
    double s = 0.0;
    for (int i = lane; i < m; i += 64) s += W[i + (size_t)c * ldw] * W[i + (size_t)c * ldw];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if (lane == 0) nrm[c] = sqrt(s);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < m; i += kOJT) {
    const double li = nrm[i];
    int rk = 0;
    for (int j = 0; j < m; ++j) {
      const double lj = nrm[j];
      if (lj > li || (lj == li && j < i)) ++rk;
    }
    rank_of[i] = rk;
    lam[rk] = li;
  }
  __syncthreads();
  for (int c = wave; c < m; c += kOJT / 64) {
    double best = -1.0, sv = 1.0;
    for (int i = lane; i < m; i += 64) {
      const double v = V[i + (size_t)c * ldv];
      if (fabs(v) > best) {
        best = fabs(v);
        sv = v;
      }
    }
    // lowest index wins ties, so the choice is deterministic
    int bidx = lane;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const double ob = __shfl_xor(best, o, 64);
      const double os = __shfl_xor(sv, o, 64);
      const int oi = __shfl_xor(bidx, o, 64);
      if (ob > best || (ob == best && oi < bidx)) {
        best = ob;
        sv = os;
        bidx = oi;
      }
    }
    const double sg = sv < 0.0 ? -1.0 : 1.0;
    const int dst = rank_of[c];
    for (int i = lane; i < m; i += 64) W[i + (size_t)dst * ldw] = sg * V[i + (size_t)c * ldv];
  }
  __syncthreads();
  for (long long e = threadIdx.x; e < (long long)m * m; e += kOJT) {
    const int i = (int)(e % m), j = (int)(e / m);
    V[i + (size_t)j * ldv] = W[i + (size_t)j * ldw];
  }
}

__global__ void k_shift_diag_trace(int m, double* __restrict__ G, int ldg, double c) {
  __shared__ double sh[256];
  double acc = 0.0;
  for (int i = threadIdx.x; i < m; i += 256) acc += G[i + (size_t)i * ldg];
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  const double sft = c * sh[0];
  for (int i = threadIdx.x; i < m; i += 256) G[i + (size_t)i * ldg] += sft;
}

__global__ void k_diag_accumulate(int m, const double* __restrict__ R, int ldr, double* __restrict__ d,
                                  int first) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < m; i += gridDim.x * blockDim.x) {
    const double r = fabs(R[i + (size_t)i * ldr]);
    d[i] = first ? r : d[i] * r;
  }
}

hipError_t diag_accumulate(int m, const double* R, int ldr, double* d, bool first, hipStream_t s) {
  hipLaunchKernelGGL(k_diag_accumulate, dim3((m + 255) / 256), dim3(256), 0, s, m, R, ldr, d, first ? 1 : 0);
  return hipGetLastError();
}

__global__ void k_rank_check(int m, const double* __restrict__ d, double tol, int* __restrict__ status) {
  __shared__ double smin[256], smax[256];
  double lo = INFINITY, hi = 0.0;
  bool bad = false;
  for (int i = threadIdx.x; i < m; i += 256) {
    const double v = d[i];
    if (!isfinite(v)) bad = true;
    lo = fmin(lo, v);
    hi = fmax(hi, v);
  }
  smin[threadIdx.x] = bad ? -1.0 : lo;
  smax[threadIdx.x] = hi;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      smin[threadIdx.x] = fmin(smin[threadIdx.x], smin[threadIdx.x + w]);
      smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + w]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0 && (smin[0] < 0.0 || !(smin[0] >= tol * smax[0]))) *status = 2;
}

hipError_t rank_check(int m, const double* d, double tol, int* status, hipStream_t s) {
  hipLaunchKernelGGL(k_rank_check, dim3(1), dim3(256), 0, s, m, d, tol, status);
  return hipGetLastError();
}

hipError_t shift_diag_trace(int m, double* G, int ldg, double c, hipStream_t s) {
  hipLaunchKernelGGL(k_shift_diag_trace, dim3(1), dim3(256), 0, s, m, G, ldg, c);
  return hipGetLastError();
}

hipError_t jacobi_evd(int m, double* K, int ldk, double* lam, double* V, int ldv, int* ctrl,
                      hipStream_t s, bool sym, const EvdPoll* poll) {
  if (m > 512 || m < 1) return hipErrorInvalidValue;
  const OjCfg c = oj_cfg(m);
  const size_t lds = sizeof(double) * 4 * (size_t)c.bs * m;
  static std::once_flag attr_once;
  std::call_once(attr_once, [] {
    (void)hipFuncSetAttribute((const void*)k_oj_round<4>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)(sizeof(double) * 4 * 16 * 256));
    (void)hipFuncSetAttribute((const void*)k_oj_round<8>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)(sizeof(double) * 4 * 8 * 512));
  });
  const double tol = sqrt((double)m) * 2.220446049250313e-16;
  hipLaunchKernelGGL(k_oj_init, dim3(1), dim3(kOJT), 0, s, m, K, ldk, V, ldv, ctrl, sym ? 1 : 0);
  const int max_sweeps = 20;
  for (int sw = 0; sw < max_sweeps; ++sw) {
    if (poll != nullptr && sw >= 2) {
      // the flag copied after sweep sw - 2; sweep sw - 1 keeps the device busy meanwhile
      const hipError_t e = hipEventSynchronize(poll->ev[sw & 1]);
      if (e != hipSuccess) return e;
      if (*poll->host[sw & 1] != 0) break;
    }
    for (int r = 0; r < c.nblk - 1; ++r) {
      if (m <= 256)
        hipLaunchKernelGGL(k_oj_round<4>, dim3(c.nblk / 2), dim3(kOJT), lds, s, m, c.bs, c.nblk, r, K, ldk, V, ldv,
                           ctrl, tol);
      else
        hipLaunchKernelGGL(k_oj_round<8>, dim3(c.nblk / 2), dim3(kOJT), lds, s, m, c.bs, c.nblk, r, K, ldk, V, ldv,
                           ctrl, tol);
    }
    hipLaunchKernelGGL(k_oj_sweep_end, dim3(1), dim3(64), 0, s, ctrl);
    if (poll != nullptr) {
      hipError_t e = hipMemcpyAsync(poll->host[sw & 1], ctrl, sizeof(int), hipMemcpyDeviceToHost, s);
      if (e == hipSuccess) e = hipEventRecord(poll->ev[sw & 1], s);
      if (e != hipSuccess) return e;
    }
  }
  hipLaunchKernelGGL(k_oj_finish, dim3(1), dim3(kOJT), 0, s, m, K, ldk, V, ldv, lam);
  return hipGetLastError();
}

__global__ void k_ritz_finish(int k, const double* __restrict__ lam, int mode,
                              double* __restrict__ theta, double* __restrict__ dcoef) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= k) return;
  double t = lam[i];
  if (mode == 1) t = sqrt(t > 0.0 ? t : 0.0);
  if (mode == 2) t = t * t;
  theta[i] = t;
  dcoef[i] = 1.0 / sqrt(t) - 1.0;
}

__global__ void k_transpose_small(int m, const double* __restrict__ A, int lda, double* __restrict__ B, int ldb) {
  const int i = blockIdx.x * 16 + (threadIdx.x & 15), j = blockIdx.y * 16 + (threadIdx.x >> 4);
  if (i < m && j < m) B[j + (size_t)i * ldb] = A[i + (size_t)j * lda];
}

hipError_t transpose_small(int m, const double* A, int lda, double* B, int ldb, hipStream_t s) {
  hipLaunchKernelGGL(k_transpose_small, dim3((m + 15) / 16, (m + 15) / 16), dim3(256), 0, s, m, A, lda, B, ldb);
  return hipGetLastError();
}

hipError_t ritz_finish(int k, const double* lam, int mode, double* theta, double* dcoef,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_ritz_finish, dim3((k + 255) / 256), dim3(256), 0, s, k, lam, mode, theta,
                     dcoef);
  return hipGetLastError();
}

}  // namespace wc4d
