// Small dense float64 linear algebra on the device, for the m x m problems of the
// randomised eigendecompositions (m = sketch width <= 512): Cholesky (CholeskyQR2
// and Algorithm 4's E2 = C^T C), triangular inverse, small products and the
// symmetric eigenproblem (Algorithm 2's EVD, Algorithms 3 and 5).
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
    // trailing update of the upper triangle: G(i, j) -= R(k, i) R(k, j), k < i <= j
    const int w = m - k - 1;
    const long long tot = (long long)w * w;
    for (long long e = tid; e < tot; e += nt) {
      const int i = k + 1 + (int)(e % w), j = k + 1 + (int)(e / w);
      if (i <= j) G[i + (size_t)j * ldg] -= G[k + (size_t)i * ldg] * G[k + (size_t)j * ldg];
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

hipError_t chol_upper(int m, double* G, int ldg, int* status, hipStream_t s) {
  if (m > 512) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_chol_upper, dim3(1), dim3(1024), 0, s, m, G, ldg, status);
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
// Cyclic Jacobi with the round-robin (circle) ordering: each round rotates m'/2
// disjoint index pairs at once (m' = m rounded up to even; the extra index is a
// dummy).  A rotation J = [[c, s], [-s, c]] on (p, q) zeroes a_pq of J^T A J
// (Golub and Van Loan's symmetric Schur step).  All 2x2 blocks of a round are
// updated independently, upper blocks only, mirrored to keep A exactly symmetric.
// A pair is skipped when |a_pq| <= tol sqrt(|a_pp a_qq|); a sweep without a
// rotation ends the iteration.
constexpr int kJacMaxPairs = 256;  // m <= 512

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

__global__ __launch_bounds__(1024) void k_jacobi(int m, double* __restrict__ A, int lda,
                                                 double* __restrict__ V, int ldv,
                                                 double* __restrict__ lam, int max_sweeps,
                                                 double tol) {
  __shared__ double sc[kJacMaxPairs], ss[kJacMaxPairs];
  __shared__ int sp[kJacMaxPairs], sq[kJacMaxPairs];
  __shared__ int s_rot;
  __shared__ int rank_of[2 * kJacMaxPairs];
  const int tid = threadIdx.x, nt = blockDim.x;
  const int mp = (m + 1) & ~1;
  const int np = mp / 2;
  // symmetrise and set V = I
  for (long long e = tid; e < (long long)m * m; e += nt) {
    const int i = (int)(e % m), j = (int)(e / m);
    if (i < j) {
      const double v = 0.5 * (A[i + (size_t)j * lda] + A[j + (size_t)i * lda]);
      A[i + (size_t)j * lda] = v;
      A[j + (size_t)i * lda] = v;
    }
    V[i + (size_t)j * ldv] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int sweep = 0; sweep < max_sweeps; ++sweep) {
    if (tid == 0) s_rot = 0;
    __syncthreads();
    for (int r = 0; r < mp - 1; ++r) {
      // rotation parameters of this round's pairs
      for (int k = tid; k < np; k += nt) {
        int p, q;
        rr_pair(r, k, mp, p, q);
        double c = 1.0, s = 0.0;
        if (q < m) {
          const double app = A[p + (size_t)p * lda], aqq = A[q + (size_t)q * lda];
          const double apq = A[p + (size_t)q * lda];
          if (fabs(apq) > tol * sqrt(fabs(app * aqq)) && apq != 0.0) {
            const double tau = (aqq - app) / (2.0 * apq);
            const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + t * t);
            s = t * c;
            atomicAdd(&s_rot, 1);
          }
        }
        sc[k] = c;
        ss[k] = s;
        sp[k] = p;
        sq[k] = q;
      }
      __syncthreads();
      // 2x2 blocks (P, Q) with P <= Q: B = J_P^T A_PQ J_Q
      const int nblk = np * (np + 1) / 2;
      for (int e = tid; e < nblk; e += nt) {
        // decode e -> (P, Q), P <= Q, row-major over the upper triangle
        int P = (int)((sqrt(8.0 * e + 1.0) - 1.0) * 0.5);
        while ((P + 1) * (P + 2) / 2 <= e) ++P;
        while (P * (P + 1) / 2 > e) --P;
        const int Qi = e - P * (P + 1) / 2;  // 0..P
        const int a = Qi, b = P;              // pair a <= pair b
        const double ca = sc[a], sa = ss[a], cb = sc[b], sb = ss[b];
        if (sa == 0.0 && sb == 0.0) continue;
        const int p = sp[a], q = sq[a], u = sp[b], v = sq[b];
        if (a == b) {
          if (q >= m) continue;
          const double app = A[p + (size_t)p * lda], aqq = A[q + (size_t)q * lda];
          const double apq = A[p + (size_t)q * lda];
          const double t = sa / ca;
          A[p + (size_t)p * lda] = app - t * apq;
          A[q + (size_t)q * lda] = aqq + t * apq;
          A[p + (size_t)q * lda] = 0.0;
          A[q + (size_t)p * lda] = 0.0;
          continue;
        }
        // rows {p, q} (pair a), columns {u, v} (pair b); dummy index >= m is absent
        const bool hq = q < m, hv = v < m;
        const double x_pu = A[p + (size_t)u * lda];
        const double x_pv = hv ? A[p + (size_t)v * lda] : 0.0;
        const double x_qu = hq ? A[q + (size_t)u * lda] : 0.0;
        const double x_qv = (hq && hv) ? A[q + (size_t)v * lda] : 0.0;
        // rows: J_a^T
        const double r_pu = ca * x_pu - sa * x_qu, r_qu = sa * x_pu + ca * x_qu;
        const double r_pv = ca * x_pv - sa * x_qv, r_qv = sa * x_pv + ca * x_qv;
        // columns: J_b
        const double y_pu = cb * r_pu - sb * r_pv, y_pv = sb * r_pu + cb * r_pv;
        const double y_qu = cb * r_qu - sb * r_qv, y_qv = sb * r_qu + cb * r_qv;
        A[p + (size_t)u * lda] = y_pu;
        A[u + (size_t)p * lda] = y_pu;
        if (hv) {
          A[p + (size_t)v * lda] = y_pv;
          A[v + (size_t)p * lda] = y_pv;
        }
        if (hq) {
          A[q + (size_t)u * lda] = y_qu;
          A[u + (size_t)q * lda] = y_qu;
        }
        if (hq && hv) {
          A[q + (size_t)v * lda] = y_qv;
          A[v + (size_t)q * lda] = y_qv;
        }
      }
      // V <- V J: columns p, q of every rotated pair
      for (long long e = tid; e < (long long)m * np; e += nt) {
        const int i = (int)(e % m), k = (int)(e / m);
        const double s = ss[k];
        if (s == 0.0) continue;
        const double c = sc[k];
        const int p = sp[k], q = sq[k];
        const double vp = V[i + (size_t)p * ldv], vq = V[i + (size_t)q * ldv];
        V[i + (size_t)p * ldv] = c * vp - s * vq;
        V[i + (size_t)q * ldv] = s * vp + c * vq;
      }
      __syncthreads();
    }
    if (s_rot == 0) break;
    __syncthreads();
  }
  // sort decreasing (stable by index) and normalise signs
  __syncthreads();
  for (int i = tid; i < m; i += nt) {
    const double li = A[i + (size_t)i * lda];
    int rk = 0;
    for (int j = 0; j < m; ++j) {
      const double lj = A[j + (size_t)j * lda];
      if (lj > li || (lj == li && j < i)) ++rk;
    }
    rank_of[i] = rk;
    lam[rk] = li;
  }
  __syncthreads();
  // write sorted vectors into A's storage (A is no longer needed), then copy to V
  for (int i = tid; i < m; i += nt) {
    // sign: largest-magnitude entry positive
    double best = 0.0;
    int bi = 0;
    for (int r2 = 0; r2 < m; ++r2) {
      const double v = fabs(V[r2 + (size_t)i * ldv]);
      if (v > best) {
        best = v;
        bi = r2;
      }
    }
    const double sg = V[bi + (size_t)i * ldv] < 0.0 ? -1.0 : 1.0;
    const int dst = rank_of[i];
    for (int r2 = 0; r2 < m; ++r2) A[r2 + (size_t)dst * lda] = sg * V[r2 + (size_t)i * ldv];
  }
  __syncthreads();
  for (long long e = tid; e < (long long)m * m; e += nt) {
    const int i = (int)(e % m), j = (int)(e / m);
    V[i + (size_t)j * ldv] = A[i + (size_t)j * lda];
  }
}

hipError_t jacobi_evd(int m, double* K, int ldk, double* lam, double* V, int ldv, hipStream_t s) {
  if (m > 2 * kJacMaxPairs) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_jacobi, dim3(1), dim3(1024), 0, s, m, K, ldk, V, ldv, lam, 60, 1e-15);
  return hipGetLastError();
}

__global__ void k_ritz_finish(int k, const double* __restrict__ lam, int mode,
                              double* __restrict__ theta, double* __restrict__ dcoef) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= k) return;
  double t = lam[i];
  if (mode == 1) t = sqrt(t > 0.0 ? t : 0.0);
  theta[i] = t;
  dcoef[i] = 1.0 / sqrt(t) - 1.0;
}

hipError_t ritz_finish(int k, const double* lam, int mode, double* theta, double* dcoef,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_ritz_finish, dim3((k + 255) / 256), dim3(256), 0, s, k, lam, mode, theta,
                     dcoef);
  return hipGetLastError();
}

}  // namespace wc4d
