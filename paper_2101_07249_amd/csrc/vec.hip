// Vector kernels of split preconditioned CG (Section 3.1, Algorithm 1) with the
// scalar recurrences kept on the device, plus small helpers.
//
// Reductions are deterministic: a fixed grid of kRB blocks writes one partial per
// block (grid-stride order fixed by n), and a single-block kernel sums the
// partials in index order.  Every kernel returns at once when the solve is done.
#include <algorithm>

#include "wc4d_internal.h"

#include <cmath>

namespace wc4d {

constexpr int kRB = 1024;   // reduction blocks
constexpr int kRT = 256;    // threads per reduction block

size_t pcg_red_doubles() { return (size_t)kRB * 4; }

static __device__ inline double block_sum(double v, double* sh) {
  // wavefront reduction then across the 4 waves of a 256-thread block
  v = wave_sum_d(v);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wave] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0) {
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += sh[w];
  }
  return t;  // valid in thread 0
}

// Sum of kRB partials red[q*kRB ...] in index order (one 256-thread block).
static __device__ inline double final_sum(const double* red, double* sh) {
  double v = 0.0;
  for (int b = threadIdx.x; b < kRB; b += blockDim.x) v += red[b];
  return block_sum(v, sh);
}

// --------------------------------------------------------------- init
__global__ __launch_bounds__(kRT) void k_dot2_partial(const double* __restrict__ a,
                                                      const double* __restrict__ b, long long n,
                                                      double* __restrict__ red) {
  __shared__ double sh[16];
  double v0 = 0.0, v1 = 0.0;
  for (long long i = (long long)blockIdx.x * kRT + threadIdx.x; i < n; i += (long long)kRB * kRT) {
    v0 += a[i] * a[i];
    v1 += b[i] * b[i];
  }
  const double t0 = block_sum(v0, sh);
  const double t1 = block_sum(v1, sh);
  if (threadIdx.x == 0) {
    red[blockIdx.x] = t0;
    red[kRB + blockIdx.x] = t1;
  }
}

__global__ __launch_bounds__(kRT) void k_pcg_init_final(PcgState* st, const double* __restrict__ red,
                                                        double tol, int maxit, int criterion) {
  __shared__ double sh[16];
  const double bb = final_sum(red, sh);
  const double rr = final_sum(red + kRB, sh);
  if (threadIdx.x == 0) {
    st->bnorm2 = bb;
    st->rr = rr;
    st->r0norm2 = rr;
    st->rr_new = rr;
    st->tol = tol;
    st->maxit = maxit;
    st->criterion = criterion;
    st->iter = 0;
    st->status = 0;
    st->alpha = 0.0;
    st->beta = 0.0;
    st->ss = 0.0;
    st->xbs = 0.0;
    // nothing to do for b = 0 (x = 0 solves it); r_0 = 0 means x_0 already solves it
    st->done = (bb == 0.0 || rr == 0.0) ? 1 : 0;
    st->rr_ref = rr;
    st->last_refresh = 0;
    st->no_refresh = 1;
  }
}

hipError_t pcg_kernels_init(PcgState* st, const double* b, const double* s0, const double* r0,
                            long long nA, double tol, int maxit, int criterion, double* red,
                            hipStream_t s) {
  (void)s0;
  hipLaunchKernelGGL(k_dot2_partial, dim3(kRB), dim3(kRT), 0, s, b, r0, nA, red);
  hipLaunchKernelGGL(k_pcg_init_final, dim3(1), dim3(kRT), 0, s, st, red, tol, maxit, criterion);
  return hipGetLastError();
}

// --------------------------------------------------------------- alpha
__global__ __launch_bounds__(kRT) void k_dot_partial(const PcgState* __restrict__ st,
                                                     const double* __restrict__ a,
                                                     const double* __restrict__ b, long long n,
                                                     double* __restrict__ red) {
  __shared__ double sh[16];
  if (st->done) return;
  double v = 0.0;
  for (long long i = (long long)blockIdx.x * kRT + threadIdx.x; i < n; i += (long long)kRB * kRT)
    v += a[i] * b[i];
  const double t = block_sum(v, sh);
  if (threadIdx.x == 0) red[blockIdx.x] = t;
}

__global__ __launch_bounds__(kRT) void k_alpha_final(PcgState* st, const double* __restrict__ red) {
  __shared__ double sh[16];
  if (st->done) return;
  const double pap = final_sum(red, sh);
  if (threadIdx.x == 0) {
    st->pAp = pap;
    if (!(pap > 0.0) || !isfinite(pap)) {
      st->status = WC4D_EBREAKDOWN;
      st->done = 1;
      st->no_refresh = 1;
    } else {
      st->alpha = st->rr / pap;
    }
  }
}

hipError_t pcg_dot_alpha(PcgState* st, const double* p, const double* Ap, long long nA,
                         double* red, hipStream_t s) {
  hipLaunchKernelGGL(k_dot_partial, dim3(kRB), dim3(kRT), 0, s, st, p, Ap, nA, red);
  hipLaunchKernelGGL(k_alpha_final, dim3(1), dim3(kRT), 0, s, st, red);
  return hipGetLastError();
}

// ------------------------------------------------- x, s updates (+ partials)
// x += alpha p; s -= alpha Ap; partials of s.s and x.(b + s) into red[0..2 kRB).
__global__ __launch_bounds__(kRT) void k_update_xs(const PcgState* __restrict__ st,
                                                   double* __restrict__ x, double* __restrict__ sr,
                                                   const double* __restrict__ b,
                                                   const double* __restrict__ p,
                                                   const double* __restrict__ Ap, long long n,
                                                   double* __restrict__ red) {
  __shared__ double sh[16];
  if (st->done) return;
  const double alpha = st->alpha;
  double vs = 0.0, vj = 0.0;
  for (long long i = (long long)blockIdx.x * kRT + threadIdx.x; i < n; i += (long long)kRB * kRT) {
    const double xi = x[i] + alpha * p[i];
    const double si = sr[i] - alpha * Ap[i];
    x[i] = xi;
    sr[i] = si;
    vs += si * si;
    vj += xi * (b[i] + si);
  }
  const double t0 = block_sum(vs, sh);
  const double t1 = block_sum(vj, sh);
  if (threadIdx.x == 0) {
    red[blockIdx.x] = t0;
    red[kRB + blockIdx.x] = t1;
  }
}

hipError_t pcg_update_xs(PcgState* st, double* x, double* sres, const double* b, const double* p,
                         const double* Ap, long long nA, double* red, hipStream_t s) {
  hipLaunchKernelGGL(k_update_xs, dim3(kRB), dim3(kRT), 0, s, st, x, sres, b, p, Ap, nA, red);
  return hipGetLastError();
}

// ---------------------------------------------- r update, beta, convergence
__global__ __launch_bounds__(kRT) void k_update_r(const PcgState* __restrict__ st,
                                                  double* __restrict__ r,
                                                  const double* __restrict__ w, long long n,
                                                  double* __restrict__ red) {
  __shared__ double sh[16];
  if (st->done) return;
  const double alpha = st->alpha;
  double v = 0.0;
  for (long long i = (long long)blockIdx.x * kRT + threadIdx.x; i < n; i += (long long)kRB * kRT) {
    const double ri = r[i] - alpha * w[i];
    r[i] = ri;
    v += ri * ri;
  }
  const double t = block_sum(v, sh);
  if (threadIdx.x == 0) red[2 * kRB + blockIdx.x] = t;
}

// The three sums of kRB partials in one pass: every thread's loads of all three are in
// flight together, and one pair of barriers combines the wavefronts (each sum in the same
// order as final_sum's).
static __device__ inline void final_sum3(const double* red, double* sh, double& s0, double& s1, double& s2) {
  // a block of kRT threads (the loop's trip count is then known, so all loads are in flight)
  double v0 = 0.0, v1 = 0.0, v2 = 0.0;
#pragma unroll
  for (int b = threadIdx.x; b < kRB; b += kRT) {
    v0 += red[b];
    v1 += red[kRB + b];
    v2 += red[2 * kRB + b];
  }
  v0 = wave_sum_d(v0);
  v1 = wave_sum_d(v1);
  v2 = wave_sum_d(v2);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = kRT / 64;
  __syncthreads();
  if (lane == 0) {
    sh[wave] = v0;
    sh[nw + wave] = v1;
    sh[2 * nw + wave] = v2;
  }
  __syncthreads();
  s0 = s1 = s2 = 0.0;
  if (threadIdx.x == 0) {
    for (int w = 0; w < nw; ++w) s0 += sh[w];
    for (int w = 0; w < nw; ++w) s1 += sh[nw + w];
    for (int w = 0; w < nw; ++w) s2 += sh[2 * nw + w];
  }
}

__global__ __launch_bounds__(kRT) void k_beta_final(PcgState* st, const double* __restrict__ red,
                                                    double* __restrict__ hist) {
  __shared__ double sh[3 * (kRT / 64)];
  if (st->done) return;
  double ss, xbs, rr;
  final_sum3(red, sh, ss, xbs, rr);
  if (threadIdx.x == 0) {
    const int it = st->iter + 1;
    st->iter = it;
    st->ss = ss;
    st->xbs = xbs;
    st->beta = rr / st->rr;
    st->rr_new = rr;
    st->rr = rr;
    const double rt = sqrt(ss / st->bnorm2);
    const double rp = sqrt(rr / st->r0norm2);
    if (hist != nullptr) {
      hist[it - 1] = rt;
      hist[st->maxit + it - 1] = rp;
      hist[2 * st->maxit + it - 1] = -0.5 * xbs;
      hist[3 * st->maxit + it - 1] = st->alpha;   // CG coefficients (Section 3.4's T_j)
      hist[4 * st->maxit + it - 1] = st->beta;
    }
    const double crit = (st->criterion == WC4D_RES_TRUE) ? rt : rp;
    if (!isfinite(crit)) {
      st->status = WC4D_EBREAKDOWN;
      st->done = 1;
    } else if (crit <= st->tol) {
      st->status = WC4D_OK;
      st->done = 1;
    } else if (it >= st->maxit) {
      st->status = WC4D_ENOCONV;
      st->done = 1;
    }
    // fused variant: recompute u = U^T r exactly once r.r has dropped by 100x since the
    // last refresh (or after 50 steps), since the recursion's absolute rounding error does
    // not shrink with u
    const bool go = !st->done && (rr < 1e-2 * st->rr_ref || it - st->last_refresh >= 50);
    st->no_refresh = go ? 0 : 1;
    if (go) {
      st->rr_ref = rr;
      st->last_refresh = it;
    }
  }
}

// Preconditioned CG with a preconditioner function (the Ritz-LMP): the numerator of alpha
// and beta is r^T z, and r is the true residual s itself.
__global__ __launch_bounds__(kRT) void k_init_std_partial(const double* __restrict__ b, const double* __restrict__ s0,
                                                          const double* __restrict__ z0, long long n,
                                                          double* __restrict__ red) {
  __shared__ double sh[16];
  double vb = 0.0, vz = 0.0, vs = 0.0;
  for (long long i = (long long)blockIdx.x * kRT + threadIdx.x; i < n; i += (long long)kRB * kRT) {
    vb += b[i] * b[i];
    vz += s0[i] * z0[i];
    vs += s0[i] * s0[i];
  }
  const double t0 = block_sum(vb, sh);
  const double t1 = block_sum(vz, sh);
  const double t2 = block_sum(vs, sh);
  if (threadIdx.x == 0) {
    red[blockIdx.x] = t0;
    red[kRB + blockIdx.x] = t1;
    red[2 * kRB + blockIdx.x] = t2;
  }
}

__global__ __launch_bounds__(kRT) void k_init_std_final(PcgState* st, const double* __restrict__ red, double tol,
                                                        int maxit, int criterion) {
  __shared__ double sh[16];
  const double bb = final_sum(red, sh);
  const double rz = final_sum(red + kRB, sh);
  const double ss = final_sum(red + 2 * kRB, sh);
  if (threadIdx.x == 0) {
    st->bnorm2 = bb;
    st->rr = rz;
    st->r0norm2 = rz;
    st->rr_new = rz;
    st->ss = ss;
    st->tol = tol;
    st->maxit = maxit;
    st->criterion = criterion;
    st->iter = 0;
    st->status = 0;
    st->alpha = 0.0;
    st->beta = 0.0;
    st->xbs = 0.0;
    st->done = (bb == 0.0 || ss == 0.0) ? 1 : 0;
    st->rr_ref = rz;
    st->last_refresh = 0;
    st->no_refresh = 1;
  }
}

hipError_t pcg_kernels_init_std(PcgState* st, const double* b, const double* s0, const double* z0, long long nA,
                                double tol, int maxit, int criterion, double* red, hipStream_t s) {
  hipLaunchKernelGGL(k_init_std_partial, dim3(kRB), dim3(kRT), 0, s, b, s0, z0, nA, red);
  hipLaunchKernelGGL(k_init_std_final, dim3(1), dim3(kRT), 0, s, st, red, tol, maxit, criterion);
  return hipGetLastError();
}

// partials of a.b into the third reduction slot (the one k_beta_final reads as r^T z)
hipError_t pcg_dot_rz(PcgState* st, const double* a, const double* b, long long nA, double* red, hipStream_t s) {
  hipLaunchKernelGGL(k_dot_partial, dim3(kRB), dim3(kRT), 0, s, st, a, b, nA, red + 2 * kRB);
  return hipGetLastError();
}

hipError_t pcg_beta_final(PcgState* st, double* red, double* hist, hipStream_t s) {
  hipLaunchKernelGGL(k_beta_final, dim3(1), dim3(kRT), 0, s, st, red, hist);
  return hipGetLastError();
}

__global__ void k_neg_inv(const double* __restrict__ th, double* __restrict__ out, int k) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < k) out[i] = -1.0 / th[i];
}

hipError_t vec_neg_inv(const double* theta, double* out, int k, hipStream_t s) {
  hipLaunchKernelGGL(k_neg_inv, dim3((k + 255) / 256), dim3(256), 0, s, theta, out, k);
  return hipGetLastError();
}

__global__ void k_sub_small(double* __restrict__ a, const double* __restrict__ b, int k, const int* skip) {
  if (skip != nullptr && *skip != 0) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < k) a[i] -= b[i];
}

hipError_t vec_sub_small(double* a, const double* b, int k, const int* skip, hipStream_t s) {
  hipLaunchKernelGGL(k_sub_small, dim3((k + 255) / 256), dim3(256), 0, s, a, b, k, skip);
  return hipGetLastError();
}

__global__ void k_copy_skip(double* __restrict__ y, const double* __restrict__ x, long long n, const int* skip) {
  if (skip != nullptr && *skip != 0) return;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    y[i] = x[i];
}

hipError_t vec_copy_skip(double* y, const double* x, long long n, const int* skip, hipStream_t s) {
  hipLaunchKernelGGL(k_copy_skip, dim3((unsigned)std::min<long long>((n + 255) / 256, 2048)), dim3(256), 0, s, y, x,
                     n, skip);
  return hipGetLastError();
}

hipError_t pcg_update_r(PcgState* st, double* r, const double* w, long long nA, double* red,
                        double* hist, hipStream_t s) {
  hipLaunchKernelGGL(k_update_r, dim3(kRB), dim3(kRT), 0, s, st, r, w, nA, red);
  hipLaunchKernelGGL(k_beta_final, dim3(1), dim3(kRT), 0, s, st, red, hist);
  return hipGetLastError();
}

hipError_t pcg_update_r_only(PcgState* st, double* r, const double* w, long long nA, double* red, hipStream_t s) {
  hipLaunchKernelGGL(k_update_r, dim3(kRB), dim3(kRT), 0, s, st, r, w, nA, red);
  return hipGetLastError();
}

// y = x - F t over j columns of F (ldf; no alignment assumed), t staged in LDS; with
// red != null also the partials of y^T y into the slot k_beta_final reads as r^T r.
__global__ __launch_bounds__(kRT) void k_reorth_sub(const PcgState* __restrict__ st, int j,
                                                    const double* __restrict__ F, long long ldf,
                                                    const double* __restrict__ t,
                                                    const double* __restrict__ x, double* __restrict__ y,
                                                    long long n, double* __restrict__ red) {
  __shared__ double ts[512];
  __shared__ double sh[16];
  if (st->done) return;
  for (int c = threadIdx.x; c < j; c += kRT) ts[c] = t[c];
  __syncthreads();
  double v = 0.0;
  for (long long i = (long long)blockIdx.x * kRT + threadIdx.x; i < n; i += (long long)kRB * kRT) {
    double acc = x[i];
    for (int c = 0; c < j; ++c) acc -= F[(long long)c * ldf + i] * ts[c];
    y[i] = acc;
    v += acc * acc;
  }
  if (red == nullptr) return;
  const double tt = block_sum(v, sh);
  if (threadIdx.x == 0) red[2 * kRB + blockIdx.x] = tt;
}

hipError_t pcg_reorth_sub(const PcgState* st, int j, const double* F, long long ldf, const double* t,
                          const double* x, double* y, long long nA, double* red, hipStream_t s) {
  if (j < 1 || j > 512) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_reorth_sub, dim3(kRB), dim3(kRT), 0, s, st, j, F, ldf, t, x, y, nA, red);
  return hipGetLastError();
}

// p = z + beta p
__global__ void k_update_p(const PcgState* __restrict__ st, double* __restrict__ p,
                           const double* __restrict__ z, long long n) {
  if (st->done) return;
  const double beta = st->beta;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    p[i] = z[i] + beta * p[i];
}

// Lanczos vector f_j = (-1)^j r_j / ||r_j|| into column j of F when iteration j has run
// (st->iter == j; j = 0 is the initial residual).
__global__ void k_lanczos_col(const PcgState* __restrict__ st, int j, const double* __restrict__ r,
                              double* __restrict__ F, long long ldf, long long n) {
  if (st->iter != j || !(st->rr > 0.0)) return;
  const double sc = ((j & 1) ? -1.0 : 1.0) / sqrt(st->rr);
  double* f = F + (long long)j * ldf;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    f[i] = sc * r[i];
}

hipError_t pcg_lanczos_col(const PcgState* st, int j, const double* r, double* F, long long ldf, long long nA,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_lanczos_col, dim3(1024), dim3(256), 0, s, st, j, r, F, ldf, nA);
  return hipGetLastError();
}

hipError_t pcg_update_p(PcgState* st, double* p, const double* z, long long nA, hipStream_t s) {
  hipLaunchKernelGGL(k_update_p, dim3(2048), dim3(256), 0, s, st, p, z, nA);
  return hipGetLastError();
}

// ------------------------------------------------------------ helpers
__global__ void k_to_f32(float* __restrict__ y, const double* __restrict__ x, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    y[i] = (float)x[i];
}
__global__ void k_to_f64(double* __restrict__ y, const float* __restrict__ x, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    y[i] = (double)x[i];
}
hipError_t vec_to_f32(float* y, const double* x, long long n, hipStream_t s) {
  hipLaunchKernelGGL(k_to_f32, dim3(2048), dim3(256), 0, s, y, x, n);
  return hipGetLastError();
}
hipError_t vec_to_f64(double* y, const float* x, long long n, hipStream_t s) {
  hipLaunchKernelGGL(k_to_f64, dim3(2048), dim3(256), 0, s, y, x, n);
  return hipGetLastError();
}

__global__ void k_copy(double* __restrict__ y, const double* __restrict__ x, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    y[i] = x[i];
}

hipError_t vec_copy(double* y, const double* x, long long n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy, dim3(2048), dim3(256), 0, s, y, x, n);
  return hipGetLastError();
}

__global__ void k_fill(double* __restrict__ y, double v, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    y[i] = v;
}

hipError_t vec_fill(double* y, double v, long long n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill, dim3(2048), dim3(256), 0, s, y, v, n);
  return hipGetLastError();
}

__global__ void k_scale_rows(double* __restrict__ T, int k, int m, int ldt,
                             const double* __restrict__ dcoef, const int* __restrict__ skip) {
  if (skip != nullptr && *skip != 0) return;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= k * m) return;
  const int i = e % k, j = e / k;
  T[i + (size_t)j * ldt] *= dcoef[i];
}

hipError_t vec_scale_rows(double* T, int k, int m, int ldt, const double* dcoef, const int* skip,
                          hipStream_t s) {
  if (k * m <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_scale_rows, dim3((k * m + 255) / 256), dim3(256), 0, s, T, k, m, ldt, dcoef,
                     skip);
  return hipGetLastError();
}

__global__ void k_stash_innov(const double* __restrict__ d, const double* __restrict__ rinv,
                              double* __restrict__ st, int q) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < q) st[k] = d[k] * rinv[k];
}

hipError_t stash_from_innov(const double* d, const double* rinv, double* stash, int q,
                            hipStream_t s) {
  if (q <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_stash_innov, dim3((q + 255) / 256), dim3(256), 0, s, d, rinv, stash, q);
  return hipGetLastError();
}

// s_0 = b - A x_0 (the A x_0 product is skipped when x_0 = 0: flag set by init)
__global__ void k_s0(const double* __restrict__ b, const double* __restrict__ Ax,
                     const int* __restrict__ xzero, double* __restrict__ s0, long long n) {
  const bool z = *xzero != 0;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    s0[i] = z ? b[i] : b[i] - Ax[i];
}

__global__ __launch_bounds__(kRT) void k_norm_partial(const double* __restrict__ x, long long n,
                                                      double* __restrict__ red) {
  __shared__ double sh[16];
  double v = 0.0;
  for (long long i = (long long)blockIdx.x * kRT + threadIdx.x; i < n; i += (long long)kRB * kRT)
    v += x[i] * x[i];
  const double t = block_sum(v, sh);
  if (threadIdx.x == 0) red[blockIdx.x] = t;
}

__global__ __launch_bounds__(kRT) void k_zero_flag(const double* __restrict__ red,
                                                   int* __restrict__ flag) {
  __shared__ double sh[16];
  const double t = final_sum(red, sh);
  if (threadIdx.x == 0) *flag = (t == 0.0) ? 1 : 0;
}

hipError_t pcg_x0_zero_flag(const double* x, long long n, double* red, int* flag, hipStream_t s) {
  hipLaunchKernelGGL(k_norm_partial, dim3(kRB), dim3(kRT), 0, s, x, n, red);
  hipLaunchKernelGGL(k_zero_flag, dim3(1), dim3(kRT), 0, s, red, flag);
  return hipGetLastError();
}

hipError_t pcg_s0(const double* b, const double* Ax, const int* xzero, double* s0, long long n,
                  hipStream_t s) {
  hipLaunchKernelGGL(k_s0, dim3(2048), dim3(256), 0, s, b, Ax, xzero, s0, n);
  return hipGetLastError();
}

// 2-D block copy Y(:, c) = X(:, c), rows < rows.
__global__ void k_copy2d(double* __restrict__ Y, long long ldy, const double* __restrict__ X,
                         long long ldx, long long rows, int cols) {
  const int c = blockIdx.y;
  if (c >= cols) return;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < rows;
       i += (long long)gridDim.x * blockDim.x)
    Y[i + c * ldy] = X[i + c * ldx];
}

hipError_t block_copy(double* Y, long long ldy, const double* X, long long ldx, long long rows,
                      int cols, hipStream_t s) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy2d, dim3(256, cols), dim3(256), 0, s, Y, ldy, X, ldx, rows, cols);
  return hipGetLastError();
}

// ------------------------------------------------ fused LMP inside PCG
// With u = U^T r kept as a k-vector, one PCG iteration needs U^T (A p) (one pass
// over U) and one pass producing both w = C A p and z = C r_new:
//   t = U^T Ap,  d1 = dcoef .* t,  w = Ap + U d1,  r_new = r - alpha w,
//   u_new = U^T r_new = u - alpha (t + (U^T U) d1),  d2 = dcoef .* u_new,
//   z = r_new + U d2.
// k_pcg_lmp_coeffs forms d1, d2 and u_new (one workgroup).
// 64 rows per 256-thread block, 4 threads per row splitting the k-long dot product.
__global__ __launch_bounds__(256) void k_pcg_lmp_coeffs(const PcgState* __restrict__ st, int k,
                                                        const double* __restrict__ t,
                                                        const double* __restrict__ dcoef,
                                                        const double* __restrict__ GU,
                                                        double* __restrict__ u,
                                                        double* __restrict__ d12) {
  extern __shared__ double sd1[];
  if (st->done) return;
  const double alpha = st->alpha;
  for (int c = threadIdx.x; c < k; c += blockDim.x) sd1[c] = dcoef[c] * t[c];
  __syncthreads();
  const int c = blockIdx.x * 64 + (threadIdx.x >> 2), sub = threadIdx.x & 3;
  double g = 0.0;
  if (c < k) {
#pragma unroll 4
    for (int j = sub; j < k; j += 4) g += GU[c + (size_t)j * k] * sd1[j];
  }
  g += __shfl_xor(g, 1, 64);
  g += __shfl_xor(g, 2, 64);
  if (c < k && sub == 0) {
    const double un = u[c] - alpha * (t[c] + g);
    u[c] = un;
    d12[c] = sd1[c];
    d12[k + c] = dcoef[c] * un;
  }
}

hipError_t pcg_lmp_coeffs(const PcgState* st, int k, const double* t, const double* dcoef,
                          const double* GU, double* u, double* d12, hipStream_t s) {
  hipLaunchKernelGGL(k_pcg_lmp_coeffs, dim3((k + 63) / 64), dim3(256), sizeof(double) * k, s, st, k,
                     t, dcoef, GU, u, d12);
  return hipGetLastError();
}

// Dual pass: r <- r - alpha (Ap + U d1), z = r + U d2, partials of r.r into red[2 kRB ..).
// Column-major float64 U: 4 consecutive rows per thread, 16-byte loads (ldu % 4 == 0).
constexpr int kDC = 16;  // columns per group
template <typename T>
static __device__ inline void ld4(const T* p, double (&v)[4]);
template <>
__device__ inline void ld4<double>(const double* p, double (&v)[4]) {
  const double2 a = *reinterpret_cast<const double2*>(p);
  const double2 b = *reinterpret_cast<const double2*>(p + 2);
  v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y;
}

template <typename T>
__global__ __launch_bounds__(kRT) void k_pcg_lmp_dual(const PcgState* __restrict__ st, long long nA,
                                                      int k, const T* __restrict__ U, long long ldu,
                                                      const double* __restrict__ d12,
                                                      const double* __restrict__ Ap,
                                                      double* __restrict__ r, double* __restrict__ z,
                                                      double* __restrict__ red) {
  extern __shared__ double sd[];
  __shared__ double sh[16];
  if (st->done) return;
  const double alpha = st->alpha;
  for (int c = threadIdx.x; c < 2 * k; c += kRT) sd[c] = d12[c];
  __syncthreads();
  double vsum = 0.0;
  const long long chunk = (long long)kRT * 4;
  for (long long rb = (long long)blockIdx.x * chunk; rb < nA; rb += (long long)kRB * chunk) {
    const long long r0 = rb + 4LL * threadIdx.x;
    const bool full = r0 + 4 <= nA;
    double aw[4] = {0.0, 0.0, 0.0, 0.0}, az[4] = {0.0, 0.0, 0.0, 0.0};
    for (int c0 = 0; c0 < k; c0 += kDC) {
      double uv[kDC][4];
#pragma unroll
      for (int c = 0; c < kDC; ++c) {
        if (c0 + c < k && full) {
          ld4<T>(U + (size_t)(c0 + c) * ldu + r0, uv[c]);
        } else {
#pragma unroll
          for (int e = 0; e < 4; ++e)
            uv[c][e] = (c0 + c < k && r0 + e < nA) ? (double)U[(size_t)(c0 + c) * ldu + r0 + e] : 0.0;
        }
      }
#pragma unroll
      for (int c = 0; c < kDC; ++c) {
        const double t1 = (c0 + c < k) ? sd[c0 + c] : 0.0;
        const double t2 = (c0 + c < k) ? sd[k + c0 + c] : 0.0;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          aw[e] += uv[c][e] * t1;
          az[e] += uv[c][e] * t2;
        }
      }
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      if (r0 + e < nA) {
        const long long i = r0 + e;
        const double rn = r[i] - alpha * (Ap[i] + aw[e]);
        r[i] = rn;
        z[i] = rn + az[e];
        vsum += rn * rn;
      }
    }
  }
  const double tot = block_sum(vsum, sh);
  if (threadIdx.x == 0) red[2 * kRB + blockIdx.x] = tot;
}


// ------------------------------- fused LMP inside PCG, panel copy of U

// Row i of the dual pass: r -= alpha (Ap + w), z = r + zz, x += alpha p, s -= alpha Ap
// (the true residual), with the partials of r.r, s.s and x.(b + s).
static __device__ inline void pcg_dual_row(long long i, double alpha, double w, double zz,
                                           const double* __restrict__ Ap, double* __restrict__ r,
                                           double* __restrict__ z, double* __restrict__ x,
                                           double* __restrict__ sr, const double* __restrict__ b,
                                           const double* __restrict__ p, double& vsum, double& vs,
                                           double& vj) {
  const double api = Ap[i];
  const double rn = r[i] - alpha * (api + w);
  r[i] = rn;
  z[i] = rn + zz;
  vsum += rn * rn;
  const double xi = x[i] + alpha * p[i];
  const double si = sr[i] - alpha * api;
  x[i] = xi;
  sr[i] = si;
  vs += si * si;
  vj += xi * (b[i] + si);
}

// After the U^T Ap pass and the fixed-order sum of its partials into t: p.Ap from that
// pass's partials (every block sums them in the same order, block 0 records pAp and
// alpha), d1 = dcoef .* t, and for 8 rows c per block (32 threads each)
// u_c <- u_c - alpha (t_c + (GU d1)_c) with GU's row c (GU = U^T U is symmetric),
// d12 = [d1, dcoef .* u].
constexpr int kCR = 8;  // rows of u per block
__global__ __launch_bounds__(kRT) void k_pcg_coeffs_pan(PcgState* __restrict__ st, int k, int sp,
                                                        const double* __restrict__ tv,
                                                        const double* __restrict__ dotpart,
                                                        const double* __restrict__ dcoef,
                                                        const double* __restrict__ GU,
                                                        double* __restrict__ u,
                                                        double* __restrict__ d12) {
  extern __shared__ double sm[];
  double* sd1 = sm;       // d1 (k)
  double* stv = sm + k;   // t (k)
  __shared__ double sh[16];
  __shared__ double s_alpha;
  __shared__ int s_done;
  // block 0 may set done during this kernel: each block reads it once
  if (threadIdx.x == 0) s_done = st->done;
  __syncthreads();
  if (s_done) return;
  // loads that do not wait for alpha first: t and d1 = dcoef .* t into LDS, this thread's
  // entries of its GU row; then p.Ap from the pass's partials
  for (int c = threadIdx.x; c < k; c += kRT) {
    const double t = tv[c];
    stv[c] = t;
    sd1[c] = dcoef[c] * t;
  }
  const int c = blockIdx.x * kCR + (threadIdx.x >> 5), sub = threadIdx.x & 31;
  constexpr int kGH = 16;  // GU entries held per thread (k <= 512)
  double gr[kGH];
#pragma unroll
  for (int q = 0; q < kGH; ++q) {
    const int j = sub + 32 * q;
    gr[q] = (c < k && j < k) ? GU[(size_t)c * k + j] : 0.0;
  }
  // sp <= kRB partials: all of a thread's loads in flight, then added in order
  double pv[kRB / kRT];
#pragma unroll
  for (int q = 0; q < kRB / kRT; ++q) {
    const int b = threadIdx.x + kRT * q;
    pv[q] = b < sp ? dotpart[b] : 0.0;
  }
  double v = 0.0;
#pragma unroll
  for (int q = 0; q < kRB / kRT; ++q)
    if (threadIdx.x + kRT * q < sp) v += pv[q];
  const double pap = block_sum(v, sh);
  if (threadIdx.x == 0) {
    const bool ok = pap > 0.0 && isfinite(pap);
    s_alpha = ok ? st->rr / pap : 0.0;
    if (blockIdx.x == 0) {
      st->pAp = pap;
      if (ok) {
        st->alpha = s_alpha;
      } else {
        st->status = WC4D_EBREAKDOWN;
        st->done = 1;
        st->no_refresh = 1;
      }
    }
    if (!ok) s_alpha = -1.0;  // flag: nothing more to do
  }
  __syncthreads();
  const double alpha = s_alpha;
  if (alpha < 0.0) return;
  double g = 0.0;
  if (c < k) {
#pragma unroll
    for (int q = 0; q < kGH; ++q) {
      const int j = sub + 32 * q;
      if (j < k) g += gr[q] * sd1[j];
    }
  }
#pragma unroll
  for (int o = 16; o > 0; o >>= 1) g += __shfl_xor(g, o, 64);
  if (c < k && sub == 0) {
    const double un = u[c] - alpha * (stv[c] + g);
    u[c] = un;
    d12[c] = sd1[c];
    d12[k + c] = dcoef[c] * un;
  }
}

hipError_t pcg_lmp_coeffs_pan(PcgState* st, int k, int sp, const double* t, const double* red,
                              const double* dcoef, const double* GU, double* u, double* d12,
                              hipStream_t s) {
  if (sp > kRB) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_pcg_coeffs_pan, dim3((k + kCR - 1) / kCR), dim3(kRT), sizeof(double) * 2 * k, s, st,
                     k, sp, t, red + 3 * kRB, dcoef, GU, u, d12);
  return hipGetLastError();
}

double* pcg_dot_slots(double* red) { return red + 3 * kRB; }

// Dual pass over the float32 panel copy of U: wave w of a 256-thread block takes
// columns w, w + 4, ... (two in flight), a lane holds 4 rows of the panel, and the four
// waves' sums of U d1 and U d2 meet in LDS; thread q then updates row q of the panel.
// Blocks own panels blockIdx.x, + gridDim.x, ...; block 0 clears the r.r partial slots
// of blocks that do not exist (gridDim.x .. kRB).
__global__ __launch_bounds__(kRT) void k_pcg_lmp_dual_pan(const PcgState* __restrict__ st,
                                                          long long nA, int k,
                                                          const float* __restrict__ P,
                                                          const double* __restrict__ d12,
                                                          const double* __restrict__ Ap,
                                                          double* __restrict__ r,
                                                          double* __restrict__ z,
                                                          double* __restrict__ red,
                                                          double* __restrict__ x,
                                                          double* __restrict__ sr,
                                                          const double* __restrict__ b,
                                                          const double* __restrict__ p) {
  extern __shared__ double sm[];
  double* sd = sm;             // d1 (k), d2 (k)
  double* rw = sm + 2 * k;     // [4 waves][2][kPanel rows]
  __shared__ double sh[16];
  if (st->done) return;
  const double alpha = st->alpha;
  for (int c = threadIdx.x; c < 2 * k; c += kRT) sd[c] = d12[c];
  if (blockIdx.x == 0)
    for (int q = (int)gridDim.x + threadIdx.x; q < kRB; q += kRT) {
      red[q] = 0.0;
      red[kRB + q] = 0.0;
      red[2 * kRB + q] = 0.0;
    }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const long long np = lmp_panels(nA);
  double vsum = 0.0, vs = 0.0, vj = 0.0;
  for (long long pn = blockIdx.x; pn < np; pn += gridDim.x) {
    const float* Pp = P + (size_t)pn * kPanel * k + 4 * lane;
    double aw[4] = {0.0, 0.0, 0.0, 0.0}, az[4] = {0.0, 0.0, 0.0, 0.0};
    for (int c0 = wave; c0 < k; c0 += 8) {
      const int c1 = c0 + 4;
      const float4 u0 = *reinterpret_cast<const float4*>(Pp + (size_t)c0 * kPanel);
      const float4 u1 = c1 < k ? *reinterpret_cast<const float4*>(Pp + (size_t)c1 * kPanel)
                               : make_float4(0.f, 0.f, 0.f, 0.f);
      const double a0 = sd[c0], b0 = sd[k + c0];
      const double a1 = c1 < k ? sd[c1] : 0.0, b1 = c1 < k ? sd[k + c1] : 0.0;
      aw[0] += u0.x * a0; aw[1] += u0.y * a0; aw[2] += u0.z * a0; aw[3] += u0.w * a0;
      az[0] += u0.x * b0; az[1] += u0.y * b0; az[2] += u0.z * b0; az[3] += u0.w * b0;
      aw[0] += u1.x * a1; aw[1] += u1.y * a1; aw[2] += u1.z * a1; aw[3] += u1.w * a1;
      az[0] += u1.x * b1; az[1] += u1.y * b1; az[2] += u1.z * b1; az[3] += u1.w * b1;
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      rw[(2 * wave) * kPanel + 4 * lane + e] = aw[e];
      rw[(2 * wave + 1) * kPanel + 4 * lane + e] = az[e];
    }
    __syncthreads();
    const int q = threadIdx.x;
    const long long i = pn * kPanel + q;
    if (i < nA) {
      const double w = (rw[q] + rw[2 * kPanel + q]) + (rw[4 * kPanel + q] + rw[6 * kPanel + q]);
      const double zz = (rw[kPanel + q] + rw[3 * kPanel + q]) + (rw[5 * kPanel + q] + rw[7 * kPanel + q]);
      pcg_dual_row(i, alpha, w, zz, Ap, r, z, x, sr, b, p, vsum, vs, vj);
    }
    __syncthreads();
  }
  const double t0 = block_sum(vs, sh);
  const double t1 = block_sum(vj, sh);
  const double t2 = block_sum(vsum, sh);
  if (threadIdx.x == 0) {
    red[blockIdx.x] = t0;
    red[kRB + blockIdx.x] = t1;
    red[2 * kRB + blockIdx.x] = t2;
  }
}

// The same over the float16 copy: a lane holds 8 rows (one 16-byte load per column), a
// half-wave covers a panel column, so the 8 half-waves g = 2 wave + lane / 32 take columns
// g, g + 8, ... (two in flight); their sums meet in LDS.  A column's coefficients carry
// its 2^cexp.  (Measured at n_A = 413,696, k = 251: 42 us, against 53 us for 4 rows per
// lane.)
__global__ __launch_bounds__(kRT) void k_pcg_lmp_dual_pan16(const PcgState* __restrict__ st,
                                                            long long nA, int k,
                                                            const _Float16* __restrict__ P,
                                                            const int* __restrict__ cexp,
                                                            const double* __restrict__ d12,
                                                            const double* __restrict__ Ap,
                                                            double* __restrict__ r,
                                                            double* __restrict__ z,
                                                            double* __restrict__ red,
                                                            double* __restrict__ x,
                                                            double* __restrict__ sr,
                                                            const double* __restrict__ b,
                                                            const double* __restrict__ p) {
  typedef _Float16 h8 __attribute__((ext_vector_type(8)));
  extern __shared__ double sm[];
  double* sd = sm;             // d1 (k), d2 (k), times 2^cexp
  double* rw = sm + 2 * k;     // [8 half-waves][2][kPanel rows]
  __shared__ double sh[16];
  if (st->done) return;
  const double alpha = st->alpha;
  for (int c = threadIdx.x; c < 2 * k; c += kRT) sd[c] = ldexp(d12[c], cexp[c < k ? c : c - k]);
  if (blockIdx.x == 0)
    for (int q = (int)gridDim.x + threadIdx.x; q < kRB; q += kRT) {
      red[q] = 0.0;
      red[kRB + q] = 0.0;
      red[2 * kRB + q] = 0.0;
    }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = 2 * wave + (lane >> 5), r8 = 8 * (lane & 31);
  const long long np = lmp_panels(nA);
  double vsum = 0.0, vs = 0.0, vj = 0.0;
  for (long long pn = blockIdx.x; pn < np; pn += gridDim.x) {
    const _Float16* Pp = P + (size_t)pn * kPanel * k + r8;
    double aw[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0}, az[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int c0 = g; c0 < k; c0 += 16) {
      const int c1 = c0 + 8;
      const h8 u0 = *reinterpret_cast<const h8*>(Pp + (size_t)c0 * kPanel);
      const h8 u1 = c1 < k ? *reinterpret_cast<const h8*>(Pp + (size_t)c1 * kPanel) : h8{};
      const double a0 = sd[c0], b0 = sd[k + c0];
      const double a1 = c1 < k ? sd[c1] : 0.0, b1 = c1 < k ? sd[k + c1] : 0.0;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const double v0 = (double)(float)u0[e], v1 = (double)(float)u1[e];
        aw[e] += v0 * a0;
        az[e] += v0 * b0;
        aw[e] += v1 * a1;
        az[e] += v1 * b1;
      }
    }
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      rw[(2 * g) * kPanel + r8 + e] = aw[e];
      rw[(2 * g + 1) * kPanel + r8 + e] = az[e];
    }
    __syncthreads();
    const int q = threadIdx.x;
    const long long i = pn * kPanel + q;
    if (i < nA) {
      const double* w0 = rw + q;
      const double w = ((w0[0] + w0[2 * kPanel]) + (w0[4 * kPanel] + w0[6 * kPanel])) +
                       ((w0[8 * kPanel] + w0[10 * kPanel]) + (w0[12 * kPanel] + w0[14 * kPanel]));
      const double zz = ((w0[kPanel] + w0[3 * kPanel]) + (w0[5 * kPanel] + w0[7 * kPanel])) +
                        ((w0[9 * kPanel] + w0[11 * kPanel]) + (w0[13 * kPanel] + w0[15 * kPanel]));
      pcg_dual_row(i, alpha, w, zz, Ap, r, z, x, sr, b, p, vsum, vs, vj);
    }
    __syncthreads();
  }
  const double t0 = block_sum(vs, sh);
  const double t1 = block_sum(vj, sh);
  const double t2 = block_sum(vsum, sh);
  if (threadIdx.x == 0) {
    red[blockIdx.x] = t0;
    red[kRB + blockIdx.x] = t1;
    red[2 * kRB + blockIdx.x] = t2;
  }
}


hipError_t pcg_lmp_dual(PcgState* st, long long nA, int k, const double* U, long long ldu,
                        const double* d12, const double* Ap, double* r, double* z, double* red,
                        double* hist, hipStream_t s) {
  if (ldu % 4 != 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_pcg_lmp_dual<double>, dim3(kRB), dim3(kRT), sizeof(double) * 2 * k, s, st, nA, k,
                     U, ldu, d12, Ap, r, z, red);
  hipLaunchKernelGGL(k_beta_final, dim3(1), dim3(kRT), 0, s, st, red, hist);
  return hipGetLastError();
}

hipError_t pcg_lmp_dual_pan(PcgState* st, long long nA, int k, const LmpU& U, const double* d12,
                            const double* Ap, double* r, double* z, double* x, double* sres,
                            const double* b, const double* p, double* red, double* hist, hipStream_t s) {
  static_assert(kPanel == kRT, "one thread per panel row in the row update");
  const int grid = lmp_panel_grid(nA);
  if (grid > kRB) return hipErrorInvalidValue;  // one partial slot per block
  if (U.fmt == LMP_P16)
    hipLaunchKernelGGL(k_pcg_lmp_dual_pan16, dim3(grid), dim3(kRT), sizeof(double) * (2 * k + 16 * kPanel), s, st,
                       nA, k, (const _Float16*)U.p, U.cexp, d12, Ap, r, z, red, x, sres, b, p);
  else if (U.fmt == LMP_P32)
    hipLaunchKernelGGL(k_pcg_lmp_dual_pan, dim3(grid), dim3(kRT), sizeof(double) * (2 * k + 8 * kPanel), s, st,
                       nA, k, (const float*)U.p, d12, Ap, r, z, red, x, sres, b, p);
  else
    return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_beta_final, dim3(1), dim3(kRT), 0, s, st, red, hist);
  return hipGetLastError();
}

}  // namespace wc4d
