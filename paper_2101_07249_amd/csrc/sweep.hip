// Tangent-linear (L^{-1}) and adjoint (L^{-T}) sweeps over the assimilation window
// (Section 2.1: x_0 = p_0, x_{i+1} = M_i x_i + p_{i+1}; transposed: w_N = z_N,
// w_i = z_i + M_i^T w_{i+1}), with the direct-observation term H^T R^{-1} H fused in.
//
// Each workgroup owns `cpb` columns of the block for the whole window.  A column's
// state lives in LDS (two n-long buffers, for the neighbour exchange of the
// stencil); each thread owns points j = lt, lt + tpc, ... (coalesced) and keeps the
// next step's forcing p_{i+1} (or z_i) in registers, loaded one step ahead.
// HBM traffic per column: the n_A forcing values in, the q stash values out
// (forward); the q stash values in, the n_A outputs out (adjoint).
#include <algorithm>
#include <vector>

#include "wc4d_internal.h"

namespace wc4d {

// ------------------------------------------------------------- model steps

struct AdvDiffOps {
  static constexpr int kTmp = 0;  // extra per-column LDS buffers
  static constexpr bool kStages = false;
};
struct L96Ops {
  static constexpr int kTmp = 2;
  static constexpr bool kStages = true;
};

static __device__ inline int wrap(int j, int n) { return j < 0 ? j + n : (j >= n ? j - n : j); }

// Jacobian of the L96 tendency at y applied to u, at point j (u, y in LDS):
// (u_{j+1} - u_{j-2}) y_{j-1} + (y_{j+1} - y_{j-2}) u_{j-1} - u_j.
static __device__ inline double l96_jac(const double* y, const double* u, int j, int n) {
  const int m2 = wrap(j - 2, n), m1 = wrap(j - 1, n), p1 = wrap(j + 1, n);
  return (u[p1] - u[m2]) * y[m1] + (y[p1] - y[m2]) * u[m1] - u[j];
}
// Its transpose: y_{j-2} a_{j-1} - y_{j+1} a_{j+2} + (y_{j+2} - y_{j-1}) a_{j+1} - a_j.
static __device__ inline double l96_jacT(const double* y, const double* a, int j, int n) {
  const int m2 = wrap(j - 2, n), m1 = wrap(j - 1, n), p1 = wrap(j + 1, n), p2 = wrap(j + 2, n);
  return y[m2] * a[m1] - y[p1] * a[p2] + (y[p2] - y[m1]) * a[p1] - a[j];
}

// Observations of one time level, prefetched: up to kOB entries per thread
// (k = kb + lt + o tpc); entries beyond that are read directly.  Two slots: a level of every
// 4th point of n = 4096 has 1024 observations for the 1024 threads of a column, and the
// adjoint holding fewer registers streams faster (4.8 against 4.6 TB/s with four slots).
constexpr int kOB = 2;

struct ObsBuf {
  int kb, ke;
  int idx[kOB];
  double val[kOB];  // forward: 1 / R_kk; adjoint: the stash value
};

// Forward: the list of time t (indices and 1/R); beyond N it is empty.
static __device__ inline void obs_load_fwd(const SweepModel& md, const int* s_off, int t, int N,
                                           int lt, int tpc, ObsBuf& ob) {
  ob.kb = (t <= N) ? s_off[t] : 0;
  ob.ke = (t <= N) ? s_off[t + 1] : 0;
#pragma unroll
  for (int o = 0; o < kOB; ++o) {
    const int k = ob.kb + lt + o * tpc;
    const bool v = k < ob.ke;
    ob.idx[o] = v ? md.obs_idx[k] : 0;
    ob.val[o] = v ? md.obs_rinv[k] : 0.0;
  }
}
// stash[k] = rinv[k] x[idx[k]]
static __device__ inline void obs_gather(const SweepModel& md, const ObsBuf& ob, const double* x,
                                         double* st, int lt, int tpc) {
#pragma unroll
  for (int o = 0; o < kOB; ++o) {
    const int k = ob.kb + lt + o * tpc;
    if (k < ob.ke) st[k] = ob.val[o] * x[ob.idx[o]];
  }
  for (int k = ob.kb + lt + kOB * tpc; k < ob.ke; k += tpc) st[k] = md.obs_rinv[k] * x[md.obs_idx[k]];
}
// Adjoint: indices and stash values of time t (t >= 0).
static __device__ inline void obs_load_bwd(const SweepModel& md, const int* s_off, int t,
                                           const double* st, int lt, int tpc, ObsBuf& ob) {
  ob.kb = (t >= 0) ? s_off[t] : 0;
  ob.ke = (t >= 0) ? s_off[t + 1] : 0;
#pragma unroll
  for (int o = 0; o < kOB; ++o) {
    const int k = ob.kb + lt + o * tpc;
    const bool v = k < ob.ke;
    ob.idx[o] = v ? md.obs_idx[k] : 0;
    ob.val[o] = v ? st[k] : 0.0;
  }
}
// w[idx[k]] += stash[k] (H^T); indices within one time level are distinct.
static __device__ inline void obs_scatter(const SweepModel& md, const ObsBuf& ob, double* w,
                                          const double* st, int lt, int tpc) {
#pragma unroll
  for (int o = 0; o < kOB; ++o) {
    const int k = ob.kb + lt + o * tpc;
    if (k < ob.ke) w[ob.idx[o]] += ob.val[o];
  }
  for (int k = ob.kb + lt + kOB * tpc; k < ob.ke; k += tpc) w[md.obs_idx[k]] += st[k];
}

// --------------------------------------------------------------- forward

// Tangent-linear step x_{i+1} = M_i x_i + p_{i+1}: reads cur (LDS), returns xn.
template <class Ops, int PPT>
static __device__ inline void tl_step(const SweepModel& md, int i, const double* cur, double* ys,
                                      double* t1, double* t2, const double (&pf)[PPT],
                                      double (&xn)[PPT], int lt, int tpc) {
  const int n = md.n;
  if constexpr (!Ops::kStages) {
#pragma unroll
    for (int e = 0; e < PPT; ++e) {
      const int j = lt + e * tpc;
      if (j < n) {
        const int jm = j == 0 ? n - 1 : j - 1, jp = j == n - 1 ? 0 : j + 1;
        xn[e] = md.ca * cur[jm] + md.cb * cur[j] + md.cc * cur[jp] + pf[e];
      }
    }
  } else {
    // RK4 tangent-linear step at trajectory point x_i (stage inputs y1..y4).
    const double dt = md.dt;
    const double* st = md.stages + (size_t)i * 4 * n;
    for (int idx = threadIdx.x; idx < 4 * n; idx += blockDim.x) ys[idx] = st[idx];
    __syncthreads();
    double dx[PPT], d1[PPT], d2[PPT], d3[PPT];
#pragma unroll
    for (int e = 0; e < PPT; ++e) {
      const int j = lt + e * tpc;
      if (j < n) {
        dx[e] = cur[j];
        d1[e] = l96_jac(ys, cur, j, n);
        t1[j] = dx[e] + 0.5 * dt * d1[e];
      }
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < PPT; ++e) {
      const int j = lt + e * tpc;
      if (j < n) {
        d2[e] = l96_jac(ys + n, t1, j, n);
        t2[j] = dx[e] + 0.5 * dt * d2[e];
      }
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < PPT; ++e) {
      const int j = lt + e * tpc;
      if (j < n) {
        d3[e] = l96_jac(ys + 2 * n, t2, j, n);
        t1[j] = dx[e] + dt * d3[e];
      }
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < PPT; ++e) {
      const int j = lt + e * tpc;
      if (j < n) {
        const double d4v = l96_jac(ys + 3 * n, t1, j, n);
        xn[e] = dx[e] + (dt / 6.0) * (d1[e] + 2.0 * d2[e] + 2.0 * d3[e] + d4v) + pf[e];
      }
    }
  }
}

// Adjoint step w_i = M_i^T w_{i+1} + z_i (z_i dense part only): reads cur, returns wn.
template <class Ops, int PPT>
static __device__ inline void adj_step(const SweepModel& md, int i, const double* cur, double* ys,
                                       double* t1, double* t2, const double (&zf)[PPT],
                                       double (&wn)[PPT], int lt, int tpc) {
  const int n = md.n;
  if constexpr (!Ops::kStages) {
#pragma unroll
    for (int e = 0; e < PPT; ++e) {
      const int j = lt + e * tpc;
      if (j < n) {
        const int jm = j == 0 ? n - 1 : j - 1, jp = j == n - 1 ? 0 : j + 1;
        // (M^T w)_j = ca w_{j+1} + cb w_j + cc w_{j-1}
        wn[e] = md.ca * cur[jp] + md.cb * cur[j] + md.cc * cur[jm] + zf[e];
      }
    }
  } else {
    // Reverse-mode sweep through the RK4 stages of the step from x_i.
    const double dt = md.dt;
    const double* st = md.stages + (size_t)i * 4 * n;
    for (int idx = threadIdx.x; idx < 4 * n; idx += blockDim.x) ys[idx] = st[idx];
    __syncthreads();
    double a[PPT], ax[PPT];
#pragma unroll
    for (int e = 0; e < PPT; ++e) {
      const int j = lt + e * tpc;
      if (j < n) {
        a[e] = cur[j];
        const double u4 = (dt / 6.0) * l96_jacT(ys + 3 * n, cur, j, n);
        ax[e] = a[e] + u4;
        t1[j] = (dt / 3.0) * a[e] + dt * u4;
      }
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < PPT; ++e) {
      const int j = lt + e * tpc;
      if (j < n) {
        const double u3 = l96_jacT(ys + 2 * n, t1, j, n);
        ax[e] += u3;
        t2[j] = (dt / 3.0) * a[e] + 0.5 * dt * u3;
      }
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < PPT; ++e) {
      const int j = lt + e * tpc;
      if (j < n) {
        const double u2 = l96_jacT(ys + n, t2, j, n);
        ax[e] += u2;
        t1[j] = (dt / 6.0) * a[e] + 0.5 * dt * u2;
      }
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < PPT; ++e) {
      const int j = lt + e * tpc;
      if (j < n) wn[e] = ax[e] + l96_jacT(ys, t1, j, n) + zf[e];
    }
  }
}

template <int PPT>
static __device__ inline void load_level(const double* base, int lev, int last, int n, int lt,
                                         int tpc, bool act, double (&f)[PPT]) {
#pragma unroll
  for (int e = 0; e < PPT; ++e) {
    const int j = lt + e * tpc;
    f[e] = (act && j < n && lev >= 0 && lev <= last) ? base[(size_t)lev * n + j] : 0.0;
  }
}

// LDS layout: [4n stage inputs (L96)] [cpb x (2 + kTmp) n state buffers] [N+2 ints]
template <class Ops>
static __device__ inline int* lds_obs_offsets(double* lds, int n, int cpb) {
  return reinterpret_cast<int*>(lds + (Ops::kStages ? 4 * n : 0) + (size_t)cpb * (2 + Ops::kTmp) * n);
}

template <class Ops, int PPT>
__global__ __launch_bounds__(Ops::kStages == 0 && PPT <= 4 ? 1024 : 512) void k_sweep_fwd(SweepModel md, const double* __restrict__ P,
                                                   long long ldp, int m, double* __restrict__ stash,
                                                   long long ldst, double* __restrict__ Xout,
                                                   long long ldx, const int* __restrict__ skip,
                                                   int cpb) {
  extern __shared__ double lds[];
  if (skip != nullptr && *skip != 0) return;
  const int n = md.n, N = md.N;
  const int tpc = blockDim.x / cpb;
  const int lc = threadIdx.x / tpc, lt = threadIdx.x % tpc;
  const int col = blockIdx.x * cpb + lc;
  const bool act = col < m;
  const bool obs = act && stash != nullptr;
  double* ys = lds;
  double* base = lds + (Ops::kStages ? 4 * n : 0) + (size_t)lc * (2 + Ops::kTmp) * n;
  double* b0 = base;
  double* b1 = base + n;
  double* t1 = base + 2 * n;
  double* t2 = base + 3 * n;
  int* s_off = lds_obs_offsets<Ops>(lds, n, cpb);
  for (int t = threadIdx.x; t < N + 2; t += blockDim.x) s_off[t] = md.obs_off[t];
  const double* Pc = P + (size_t)(act ? col : 0) * ldp;
  double* St = stash + (size_t)(act ? col : 0) * ldst;
  double* Xc = Xout + (size_t)(act ? col : 0) * ldx;

  double fa[PPT], fb[PPT], xn[PPT];
  load_level<PPT>(Pc, 0, N, n, lt, tpc, act, xn);
#pragma unroll
  for (int e = 0; e < PPT; ++e) {
    const int j = lt + e * tpc;
    if (j < n) {
      b0[j] = xn[e];
      if (act && Xout != nullptr) Xc[j] = xn[e];
    }
  }
  load_level<PPT>(Pc, 1, N, n, lt, tpc, act, fa);
  load_level<PPT>(Pc, 2, N, n, lt, tpc, act, fb);
  __syncthreads();
  ObsBuf oa, ob;
  obs_load_fwd(md, s_off, 0, N, lt, tpc, oa);
  if (obs) obs_gather(md, oa, b0, St, lt, tpc);
  obs_load_fwd(md, s_off, 1, N, lt, tpc, oa);
  obs_load_fwd(md, s_off, 2, N, lt, tpc, ob);

  // two steps per trip so every prefetch buffer is consumed in place
  for (int i = 0; i < N; i += 2) {
    tl_step<Ops, PPT>(md, i, b0, ys, t1, t2, fa, xn, lt, tpc);
    load_level<PPT>(Pc, i + 3, N, n, lt, tpc, act, fa);
#pragma unroll
    for (int e = 0; e < PPT; ++e) {
      const int j = lt + e * tpc;
      if (j < n) {
        b1[j] = xn[e];
        if (act && Xout != nullptr) Xc[(size_t)(i + 1) * n + j] = xn[e];
      }
    }
    __syncthreads();
    if (obs) obs_gather(md, oa, b1, St, lt, tpc);
    obs_load_fwd(md, s_off, i + 3, N, lt, tpc, oa);
    if (i + 1 >= N) break;
    tl_step<Ops, PPT>(md, i + 1, b1, ys, t1, t2, fb, xn, lt, tpc);
    load_level<PPT>(Pc, i + 4, N, n, lt, tpc, act, fb);
#pragma unroll
    for (int e = 0; e < PPT; ++e) {
      const int j = lt + e * tpc;
      if (j < n) {
        b0[j] = xn[e];
        if (act && Xout != nullptr) Xc[(size_t)(i + 2) * n + j] = xn[e];
      }
    }
    __syncthreads();
    if (obs) obs_gather(md, ob, b0, St, lt, tpc);
    obs_load_fwd(md, s_off, i + 4, N, lt, tpc, ob);
  }
}

// --------------------------------------------------------------- adjoint

template <class Ops, int PPT>
__global__ __launch_bounds__(Ops::kStages == 0 && PPT <= 4 ? 1024 : 512) void k_sweep_bwd(SweepModel md, const double* __restrict__ stash,
                                                   long long ldst, const double* __restrict__ Z,
                                                   long long ldz, int m, double* __restrict__ W,
                                                   long long ldw, const int* __restrict__ skip,
                                                   int cpb) {
  extern __shared__ double lds[];
  if (skip != nullptr && *skip != 0) return;
  const int n = md.n, N = md.N;
  const int tpc = blockDim.x / cpb;
  const int lc = threadIdx.x / tpc, lt = threadIdx.x % tpc;
  const int col = blockIdx.x * cpb + lc;
  const bool act = col < m;
  const bool dense = (stash == nullptr);
  const bool obs = act && !dense;
  double* ys = lds;
  double* base = lds + (Ops::kStages ? 4 * n : 0) + (size_t)lc * (2 + Ops::kTmp) * n;
  double* b0 = base;
  double* b1 = base + n;
  double* t1 = base + 2 * n;
  double* t2 = base + 3 * n;
  int* s_off = lds_obs_offsets<Ops>(lds, n, cpb);
  for (int t = threadIdx.x; t < N + 2; t += blockDim.x) s_off[t] = md.obs_off[t];
  const double* St = dense ? nullptr : stash + (size_t)(act ? col : 0) * ldst;
  const double* Zc = dense ? Z + (size_t)(act ? col : 0) * ldz : nullptr;
  double* Wc = W + (size_t)(act ? col : 0) * ldw;

  // w_N = z_N
  double za[PPT], zb[PPT], wn[PPT];
  load_level<PPT>(Zc, N, N, n, lt, tpc, act && dense, wn);
#pragma unroll
  for (int e = 0; e < PPT; ++e) {
    const int j = lt + e * tpc;
    if (j < n) b0[j] = wn[e];
  }
  load_level<PPT>(Zc, N - 1, N, n, lt, tpc, act && dense, za);
  load_level<PPT>(Zc, N - 2, N, n, lt, tpc, act && dense, zb);
  __syncthreads();
  ObsBuf oa, ob;
  if (obs) {
    obs_load_bwd(md, s_off, N, St, lt, tpc, oa);
    obs_scatter(md, oa, b0, St, lt, tpc);
    obs_load_bwd(md, s_off, N - 1, St, lt, tpc, oa);
    obs_load_bwd(md, s_off, N - 2, St, lt, tpc, ob);
  }
  __syncthreads();
#pragma unroll
  for (int e = 0; e < PPT; ++e) {
    const int j = lt + e * tpc;
    if (act && j < n) Wc[(size_t)N * n + j] = b0[j];
  }

  for (int i = N - 1; i >= 0; i -= 2) {
    adj_step<Ops, PPT>(md, i, b0, ys, t1, t2, za, wn, lt, tpc);
    load_level<PPT>(Zc, i - 2, N, n, lt, tpc, act && dense, za);
#pragma unroll
    for (int e = 0; e < PPT; ++e) {
      const int j = lt + e * tpc;
      if (j < n) b1[j] = wn[e];
    }
    __syncthreads();
    if (obs) {
      obs_scatter(md, oa, b1, St, lt, tpc);
      obs_load_bwd(md, s_off, i - 2, St, lt, tpc, oa);
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < PPT; ++e) {
      const int j = lt + e * tpc;
      if (act && j < n) Wc[(size_t)i * n + j] = b1[j];
    }
    if (i - 1 < 0) break;
    adj_step<Ops, PPT>(md, i - 1, b1, ys, t1, t2, zb, wn, lt, tpc);
    load_level<PPT>(Zc, i - 3, N, n, lt, tpc, act && dense, zb);
#pragma unroll
    for (int e = 0; e < PPT; ++e) {
      const int j = lt + e * tpc;
      if (j < n) b0[j] = wn[e];
    }
    __syncthreads();
    if (obs) {
      obs_scatter(md, ob, b0, St, lt, tpc);
      obs_load_bwd(md, s_off, i - 3, St, lt, tpc, ob);
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < PPT; ++e) {
      const int j = lt + e * tpc;
      if (act && j < n) Wc[(size_t)(i - 1) * n + j] = b0[j];
    }
  }
}

// ------------------------------------------- single-vector Lorenz-96 sweeps
// For one column the N RK4 steps are a chain of dependent stencil updates on n points.
// One wavefront owns the whole state: lane l holds the PPT contiguous points
// [l PPT, (l + 1) PPT) in registers (n = 64 PPT); neighbour values of the state and the
// stage increments come from the adjacent lanes by shuffles (periodic: lane 0 and lane
// 63 are neighbours), so a step needs no workgroup barrier for them.  The RK4 stage
// inputs y1..y4 of the next step are loaded into registers (coalesced) while the
// current step computes, then parked in a padded LDS double buffer from which each
// lane reads its chunk and halo.  Observations use an n-double LDS buffer.
constexpr int kVL = 64;

template <int PPT>
static __device__ inline int vpad(int j) {
  return j + j / PPT;  // one spare double per chunk spreads the lanes over the banks
}

// u at chunk offsets -2..PPT+1 from the lane's registers and its neighbours'.
template <int PPT>
struct Halo {
  double m2, m1, p1, p2;
};

template <int PPT>
static __device__ inline Halo<PPT> halo(const double (&u)[PPT], int lane) {
  const int lp = (lane + kVL - 1) & (kVL - 1), ln = (lane + 1) & (kVL - 1);
  Halo<PPT> h;
  h.m2 = __shfl(u[PPT - 2], lp);
  h.m1 = __shfl(u[PPT - 1], lp);
  h.p1 = __shfl(u[0], ln);
  h.p2 = __shfl(u[1], ln);
  return h;
}

template <int PPT>
static __device__ inline double at(const double (&u)[PPT], const Halo<PPT>& h, int e) {
  // e in [-2, PPT + 1]; resolved at compile time after unrolling
  return e == -2 ? h.m2 : e == -1 ? h.m1 : e == PPT ? h.p1 : e == PPT + 1 ? h.p2 : u[e];
}

// y of one stage over the chunk and a 2-point halo on each side: yv[e + 2], e in [-2, PPT + 1].
template <int PPT>
static __device__ inline void load_y(const double* ysb, int n, int j0, double (&yv)[PPT + 4]) {
#pragma unroll
  for (int e = -2; e < PPT + 2; ++e) {
    int j = j0 + e;
    j = j < 0 ? j + n : (j >= n ? j - n : j);
    yv[e + 2] = ysb[vpad<PPT>(j)];
  }
}

// d = J(y) u at the lane's points: (u_{j+1} - u_{j-2}) y_{j-1} + (y_{j+1} - y_{j-2}) u_{j-1} - u_j.
template <int PPT>
static __device__ inline void jac_v(const double (&yv)[PPT + 4], const double (&u)[PPT], int lane,
                                    double (&d)[PPT]) {
  const Halo<PPT> h = halo<PPT>(u, lane);
#pragma unroll
  for (int e = 0; e < PPT; ++e)
    d[e] = (at<PPT>(u, h, e + 1) - at<PPT>(u, h, e - 2)) * yv[e + 1] +
           (yv[e + 3] - yv[e]) * at<PPT>(u, h, e - 1) - u[e];
}

// d = J(y)^T a: y_{j-2} a_{j-1} - y_{j+1} a_{j+2} + (y_{j+2} - y_{j-1}) a_{j+1} - a_j.
template <int PPT>
static __device__ inline void jacT_v(const double (&yv)[PPT + 4], const double (&a)[PPT], int lane,
                                     double (&d)[PPT]) {
  const Halo<PPT> h = halo<PPT>(a, lane);
#pragma unroll
  for (int e = 0; e < PPT; ++e)
    d[e] = yv[e] * at<PPT>(a, h, e - 1) - yv[e + 3] * at<PPT>(a, h, e + 2) +
           (yv[e + 4] - yv[e + 1]) * at<PPT>(a, h, e + 1) - a[e];
}

template <int PPT>
size_t l96v_lds_bytes(int n) {
  // two stage-input buffers (4 padded levels each), the observation buffer, the transpose buffer
  return sizeof(double) * ((size_t)9 * (n + n / PPT) + n);
}

// Chunk layout (lane l holds points l PPT + e) <-> coalesced layout (lane l holds l + 64 q),
// through the padded LDS buffer tr: global loads and stores then cover 64 consecutive
// doubles per instruction.
template <int PPT>
static __device__ inline void to_chunk(double* tr, int lane, const double (&co)[PPT], double (&ch)[PPT]) {
  __syncthreads();
#pragma unroll
  for (int q = 0; q < PPT; ++q) tr[vpad<PPT>(lane + kVL * q)] = co[q];
  __syncthreads();
#pragma unroll
  for (int e = 0; e < PPT; ++e) ch[e] = tr[vpad<PPT>(lane * PPT + e)];
}

template <int PPT>
static __device__ inline void to_coalesced(double* tr, int lane, const double (&ch)[PPT], double (&co)[PPT]) {
  __syncthreads();
#pragma unroll
  for (int e = 0; e < PPT; ++e) tr[vpad<PPT>(lane * PPT + e)] = ch[e];
  __syncthreads();
#pragma unroll
  for (int q = 0; q < PPT; ++q) co[q] = tr[vpad<PPT>(lane + kVL * q)];
}

// One stage (s) of step i's inputs: entries lane + 64 q, q < PPT, of level s.
template <int PPT>
static __device__ inline void pfs_load(const double* stages, int i, int s, int n, int lane, double (&pf)[PPT]) {
  const double* src = stages + (size_t)i * 4 * n + (size_t)s * n;
#pragma unroll
  for (int q = 0; q < PPT; ++q) pf[q] = src[lane + kVL * q];
}

template <int PPT>
static __device__ inline void pfs_store(double* ysb, int s, int n, int lane, const double (&pf)[PPT]) {
  double* dst = ysb + (size_t)s * (n + n / PPT);
#pragma unroll
  for (int q = 0; q < PPT; ++q) dst[vpad<PPT>(lane + kVL * q)] = pf[q];
}

template <int PPT>
__global__ __launch_bounds__(64) void k_l96v_fwd(SweepModel md, const double* __restrict__ P,
                                                 double* __restrict__ stash, double* __restrict__ Xout,
                                                 const int* __restrict__ skip) {
  extern __shared__ double vlds[];
  if (skip != nullptr && *skip != 0) return;
  const int n = md.n, N = md.N, lane = threadIdx.x;
  const int sp = n + n / PPT;
  double* ysb[2] = {vlds, vlds + 4 * sp};
  double* xs = vlds + 8 * sp;
  double* tr = xs + n;
  const double dt = md.dt;
  double x[PPT], pn[PPT], co[PPT], pf[PPT];
#pragma unroll
  for (int q = 0; q < PPT; ++q) co[q] = P[lane + kVL * q];
  to_chunk<PPT>(tr, lane, co, x);
  auto store_x = [&](int lev) {
    if (Xout == nullptr) return;
    to_coalesced<PPT>(tr, lane, x, co);
#pragma unroll
    for (int q = 0; q < PPT; ++q) Xout[(size_t)lev * n + lane + kVL * q] = co[q];
  };
  auto gather = [&](int lev) {
    const int kb = md.obs_off[lev], ke = md.obs_off[lev + 1];
    if (stash == nullptr || kb == ke) return;
    __syncthreads();
#pragma unroll
    for (int e = 0; e < PPT; ++e) xs[lane * PPT + e] = x[e];
    __syncthreads();
    for (int k = kb + lane; k < ke; k += kVL) stash[k] = md.obs_rinv[k] * xs[md.obs_idx[k]];
  };
  store_x(0);
  gather(0);
  for (int st = 0; st < 4 && N > 0; ++st) {
    pfs_load<PPT>(md.stages, 0, st, n, lane, pf);
    pfs_store<PPT>(ysb[0], st, n, lane, pf);
  }
  __syncthreads();
  const int j0 = lane * PPT;
  for (int i = 0; i < N; ++i) {
    const double* yb = ysb[i & 1];
    double* ynext = ysb[(i + 1) & 1];
    const bool more = i + 1 < N;
#pragma unroll
    for (int q = 0; q < PPT; ++q) co[q] = P[(size_t)(i + 1) * n + lane + kVL * q];
    double yv[PPT + 4], d[PPT], t[PPT], acc[PPT];
    if (more) pfs_load<PPT>(md.stages, i + 1, 0, n, lane, pf);
    load_y<PPT>(yb, n, j0, yv);
    jac_v<PPT>(yv, x, lane, d);
#pragma unroll
    for (int e = 0; e < PPT; ++e) {
      acc[e] = d[e];
      t[e] = x[e] + 0.5 * dt * d[e];
    }
    if (more) {
      pfs_store<PPT>(ynext, 0, n, lane, pf);
      pfs_load<PPT>(md.stages, i + 1, 1, n, lane, pf);
    }
    load_y<PPT>(yb + sp, n, j0, yv);
    jac_v<PPT>(yv, t, lane, d);
#pragma unroll
    for (int e = 0; e < PPT; ++e) {
      acc[e] += 2.0 * d[e];
      t[e] = x[e] + 0.5 * dt * d[e];
    }
    if (more) {
      pfs_store<PPT>(ynext, 1, n, lane, pf);
      pfs_load<PPT>(md.stages, i + 1, 2, n, lane, pf);
    }
    load_y<PPT>(yb + 2 * sp, n, j0, yv);
    jac_v<PPT>(yv, t, lane, d);
#pragma unroll
    for (int e = 0; e < PPT; ++e) {
      acc[e] += 2.0 * d[e];
      t[e] = x[e] + dt * d[e];
    }
    if (more) {
      pfs_store<PPT>(ynext, 2, n, lane, pf);
      pfs_load<PPT>(md.stages, i + 1, 3, n, lane, pf);
    }
    load_y<PPT>(yb + 3 * sp, n, j0, yv);
    jac_v<PPT>(yv, t, lane, d);
    if (more) pfs_store<PPT>(ynext, 3, n, lane, pf);
    to_chunk<PPT>(tr, lane, co, pn);
#pragma unroll
    for (int e = 0; e < PPT; ++e) x[e] = x[e] + (dt / 6.0) * (acc[e] + d[e]) + pn[e];
    store_x(i + 1);
    gather(i + 1);
    __syncthreads();
  }
}

template <int PPT>
__global__ __launch_bounds__(64) void k_l96v_bwd(SweepModel md, const double* __restrict__ stash,
                                                 const double* __restrict__ Z, double* __restrict__ W,
                                                 const int* __restrict__ skip) {
  extern __shared__ double vlds[];
  if (skip != nullptr && *skip != 0) return;
  const int n = md.n, N = md.N, lane = threadIdx.x, j0 = lane * PPT;
  const int sp = n + n / PPT;
  double* ysb[2] = {vlds, vlds + 4 * sp};
  double* xs = vlds + 8 * sp;
  double* tr = xs + n;
  const double dt = md.dt;
  double w[PPT], co[PPT], pf[PPT];
  // z_i added into w: dense rows of Z, or H_i^T stash_i scattered through LDS
  auto add_z = [&](int lev) {
    if (stash == nullptr) {
#pragma unroll
      for (int q = 0; q < PPT; ++q) co[q] = Z[(size_t)lev * n + lane + kVL * q];
      __syncthreads();
#pragma unroll
      for (int q = 0; q < PPT; ++q) tr[vpad<PPT>(lane + kVL * q)] = co[q];
      __syncthreads();
#pragma unroll
      for (int e = 0; e < PPT; ++e) w[e] += tr[vpad<PPT>(j0 + e)];
      return;
    }
    const int kb = md.obs_off[lev], ke = md.obs_off[lev + 1];
    if (kb == ke) return;
    __syncthreads();
#pragma unroll
    for (int e = 0; e < PPT; ++e) xs[j0 + e] = 0.0;
    __syncthreads();
    for (int k = kb + lane; k < ke; k += kVL) xs[md.obs_idx[k]] = stash[k];
    __syncthreads();
#pragma unroll
    for (int e = 0; e < PPT; ++e) w[e] += xs[j0 + e];
  };
  auto store_w = [&](int lev) {
    __syncthreads();
#pragma unroll
    for (int e = 0; e < PPT; ++e) tr[vpad<PPT>(j0 + e)] = w[e];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < PPT; ++q) W[(size_t)lev * n + lane + kVL * q] = tr[vpad<PPT>(lane + kVL * q)];
  };
#pragma unroll
  for (int e = 0; e < PPT; ++e) w[e] = 0.0;
  add_z(N);
  store_w(N);
  for (int st = 0; st < 4 && N > 0; ++st) {
    pfs_load<PPT>(md.stages, N - 1, st, n, lane, pf);
    pfs_store<PPT>(ysb[(N - 1) & 1], st, n, lane, pf);
  }
  __syncthreads();
  for (int i = N - 1; i >= 0; --i) {
    const double* yb = ysb[i & 1];
    double* ynext = ysb[(i - 1) & 1];
    const bool more = i > 0;
    double yv[PPT + 4], u[PPT], ax[PPT], t[PPT];
    if (more) pfs_load<PPT>(md.stages, i - 1, 3, n, lane, pf);
    load_y<PPT>(yb + 3 * sp, n, j0, yv);
    jacT_v<PPT>(yv, w, lane, u);
#pragma unroll
    for (int e = 0; e < PPT; ++e) {
      u[e] *= dt / 6.0;
      ax[e] = w[e] + u[e];
      t[e] = (dt / 3.0) * w[e] + dt * u[e];
    }
    if (more) {
      pfs_store<PPT>(ynext, 3, n, lane, pf);
      pfs_load<PPT>(md.stages, i - 1, 2, n, lane, pf);
    }
    load_y<PPT>(yb + 2 * sp, n, j0, yv);
    jacT_v<PPT>(yv, t, lane, u);
#pragma unroll
    for (int e = 0; e < PPT; ++e) {
      ax[e] += u[e];
      t[e] = (dt / 3.0) * w[e] + 0.5 * dt * u[e];
    }
    if (more) {
      pfs_store<PPT>(ynext, 2, n, lane, pf);
      pfs_load<PPT>(md.stages, i - 1, 1, n, lane, pf);
    }
    load_y<PPT>(yb + sp, n, j0, yv);
    jacT_v<PPT>(yv, t, lane, u);
#pragma unroll
    for (int e = 0; e < PPT; ++e) {
      ax[e] += u[e];
      t[e] = (dt / 6.0) * w[e] + 0.5 * dt * u[e];
    }
    if (more) {
      pfs_store<PPT>(ynext, 1, n, lane, pf);
      pfs_load<PPT>(md.stages, i - 1, 0, n, lane, pf);
    }
    load_y<PPT>(yb, n, j0, yv);
    jacT_v<PPT>(yv, t, lane, u);
    if (more) pfs_store<PPT>(ynext, 0, n, lane, pf);
#pragma unroll
    for (int e = 0; e < PPT; ++e) w[e] = ax[e] + u[e];
    add_z(i);
    store_w(i);
    __syncthreads();
  }
}

// PPT for a single-vector Lorenz-96 sweep (0: not applicable).
static int l96v_ppt(const SweepModel& md, int m) {
  if (md.kind != 1 || m != 1 || md.n % kVL != 0) return 0;
  const int ppt = md.n / kVL;
  return (ppt == 4 || ppt == 8 || ppt == 16) ? ppt : 0;
}

template <int PPT>
static hipError_t l96v_fwd_launch(const SweepModel& md, const double* P, double* stash, double* Xout,
                                  const int* skip, hipStream_t s) {
  const size_t lds = l96v_lds_bytes<PPT>(md.n);
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_l96v_fwd<PPT>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_l96v_fwd<PPT>, dim3(1), dim3(kVL), lds, s, md, P, stash, Xout, skip);
  return hipGetLastError();
}

template <int PPT>
static hipError_t l96v_bwd_launch(const SweepModel& md, const double* stash, const double* Z, double* W,
                                  const int* skip, hipStream_t s) {
  const size_t lds = l96v_lds_bytes<PPT>(md.n);
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_l96v_bwd<PPT>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_l96v_bwd<PPT>, dim3(1), dim3(kVL), lds, s, md, stash, Z, W, skip);
  return hipGetLastError();
}

// ------------------------------------ single-wave trapezoids (advection-diffusion)
// For one or a few columns the window's N sequential steps over the whole domain are
// latency-bound.  The stencil has radius 1, so a wavefront can own W points [j0, j0 + W)
// and run all N steps on the extended range [j0 - N, j0 + W + N) (periodic indices;
// n >= E = 64 PE, so no point appears twice): after s steps only the outer s points on
// each side are wrong, so the owned points are exact at every level, and wavefronts
// never communicate.  Lane l holds the PE contiguous local points [l PE, (l + 1) PE) in
// registers and takes its neighbours' edge points through DPP wavefront shifts, so a
// step needs no barrier.
//
// A step must not wait on memory: loads (and, on this architecture, stores) retire in
// order through one counter, so any load whose address depends on another load, or a
// store-heavy step, drains the prefetch queue.  Hence the forcing rows are prefetched TD
// steps ahead in a register ring; the observations a wavefront touches come from
// fixed-slot lists built at finalize (no offsets to chase: slot s of (wavefront b,
// level t) at ((b (N+1) + t) kTS + s), entry {k, local point l, 1 / R_kk}, l < 0 for an
// empty slot); the adjoint reads its entries 2 TD steps and their stash values TD steps
// ahead; and the adjoint's output rows leave through LDS as coalesced stores.
constexpr int kTW = 64;            // one wavefront per workgroup
constexpr int kTOW = 2;            // entry slots per lane per (wavefront, level)
constexpr int kTS = kTW * kTOW;    // entry slots per (wavefront, level)

bool tw_setup(int n, int N, const std::vector<int>& off, const std::vector<int>& idx,
              const std::vector<double>& rinv, int* pe, int* W, std::vector<TwEntry>& ent) {
  // 4 or 8 points per lane (16 would leave the step's registers spilling into AGPRs).  A
  // step is bound by one wavefront's instruction issue, so fewer points per lane run each
  // step faster on more wavefronts, at the price of redundant halo points: 4 points per
  // lane while the owned width W is at least an eighth of the range (at n = 4096, N = 100:
  // 74 wavefronts; the forward and adjoint sweeps of the PCG took 15.4 and 14.3 ms per
  // inner loop against 19.4 and 18.9 ms with 8 points on 14), 8 points while W is at least
  // a quarter
  int q = 4;
  for (; q <= 8; q *= 2) {
    const int E = kTW * q, w = E - 2 * N;
    if (w > 0 && (q == 4 ? 8 : 4) * w >= E && n >= E) break;
  }
  if (q > 8 || off[N + 1] == 0) return false;
  const int E = kTW * q, Wd = E - 2 * N, nb = (n + Wd - 1) / Wd;
  ent.assign((size_t)nb * (N + 1) * kTS, TwEntry{0, -1, 0.0});
  for (int b = 0; b < nb; ++b) {
    const int j0 = b * Wd, Wc = std::min(Wd, n - j0), Ec = Wc + 2 * N, g0 = j0 - N;
    for (int t = 0; t <= N; ++t) {
      TwEntry* slot = ent.data() + ((size_t)b * (N + 1) + t) * kTS;
      int c = 0;
      for (int k = off[t]; k < off[t + 1]; ++k) {
        int l = (idx[k] - g0) % n;
        if (l < 0) l += n;
        if (l >= Ec) continue;
        if (c == kTS) return false;  // denser than the slots: the general kernels take it
        slot[c++] = TwEntry{k, l, rinv[k]};
      }
    }
  }
  *pe = q;
  *W = Wd;
  return true;
}

// v of lane - 1 (lane 0 keeps its own) and of lane + 1 (lane 63 keeps its own): DPP
// wavefront shifts (wave_shr:1, wave_shl:1), one per 32-bit half.  The kept edge values
// only reach points outside the trapezoid.
static __device__ inline double from_lower_lane(double v) {
  const int lo = __double2loint(v), hi = __double2hiint(v);
  return __hiloint2double(__builtin_amdgcn_update_dpp(hi, hi, 0x138, 0xf, 0xf, false),
                          __builtin_amdgcn_update_dpp(lo, lo, 0x138, 0xf, 0xf, false));
}
static __device__ inline double from_upper_lane(double v) {
  const int lo = __double2loint(v), hi = __double2hiint(v);
  return __hiloint2double(__builtin_amdgcn_update_dpp(hi, hi, 0x130, 0xf, 0xf, false),
                          __builtin_amdgcn_update_dpp(lo, lo, 0x130, 0xf, 0xf, false));
}

// A lane's local points: byte offsets of their global indices within a level, and which
// of them the wavefront owns.  Points past the extended range (last wavefront) and rows
// past the last level are loaded anyway: they hold finite data of other points and,
// like the trapezoid's edges, never reach an owned point.
template <int PE>
struct TwGeom {
  unsigned off8[PE];
  bool own[PE];
  int N, Wc, j0;
  __device__ TwGeom(int n, int N_, int W, int lane) : N(N_) {
    j0 = blockIdx.x * W;
    Wc = min(W, n - j0);
    const int g0 = j0 - N;
#pragma unroll
    for (int e = 0; e < PE; ++e) {
      const int l = lane * PE + e;
      int j = g0 + l;  // in [-N, n + E): one wrap at most
      j = j < 0 ? j + n : (j >= n ? j - n : j);
      off8[e] = 8u * (unsigned)j;
      own[e] = l >= N && l < N + Wc;
    }
  }
  __device__ bool owned(int l) const { return l >= N && l < N + Wc; }
  // v = row lev (clamped to [0, last]) of the n-long rows at base, at this lane's points
  __device__ void load(const double* base, int lev, int last, int n, double (&v)[PE]) const {
    lev = lev < 0 ? 0 : (lev > last ? last : lev);
    const char* row = reinterpret_cast<const char*>(base + (size_t)lev * n);
#pragma unroll
    for (int e = 0; e < PE; ++e) v[e] = *reinterpret_cast<const double*>(row + off8[e]);
  }
  __device__ void store(double* base, int lev, int n, const double (&v)[PE]) const {
    char* row = reinterpret_cast<char*>(base + (size_t)lev * n);
#pragma unroll
    for (int e = 0; e < PE; ++e)
      if (own[e]) *reinterpret_cast<double*>(row + off8[e]) = v[e];
  }
};

// the kTOW entry slots of (wavefront, level t) this lane reads (t clamped to [0, N])
static __device__ inline const TwEntry* tw_slots(const SweepModel& md, int t) {
  t = t < 0 ? 0 : (t > md.N ? md.N : t);
  return md.tw_e + ((size_t)blockIdx.x * (md.N + 1) + t) * kTS + threadIdx.x;
}

// WX: also write every x_t (owned points) to Xout.  The step count of the main loop is a
// multiple of TD with no per-step guards and every memory operation of a step is issued
// unconditionally (the stash store of a slot the wavefront does not own goes to a dummy
// double), so the compiler can keep the ring's loads in flight across the loop's back edge.
// The single-wave sweeps hand values between lanes through LDS.  A workgroup is one
// wavefront and a wavefront's LDS operations complete in issue order, so a wave-level
// code-motion barrier is enough (a workgroup barrier would also make the wave wait for
// every LDS operation in flight).
static __device__ inline void lds_order() { __builtin_amdgcn_wave_barrier(); }

template <int PE, int TD, bool WX>
__global__ __launch_bounds__(kTW) void k_sweep_fwd_w(SweepModel md, const double* __restrict__ P,
                                                     long long ldp, double* __restrict__ stash,
                                                     long long ldst, double* __restrict__ Xout,
                                                     long long ldx, const int* __restrict__ skip) {
  __shared__ double xs[kTW * PE];
  if (skip != nullptr && *skip != 0) return;
  const int n = md.n, N = md.N, lane = threadIdx.x;
  const TwGeom<PE> g(n, N, md.tw_W, lane);
  const double* Pc = P + (size_t)blockIdx.y * ldp;
  double* St = stash + (size_t)blockIdx.y * ldst;
  double* Xc = WX ? Xout + (size_t)blockIdx.y * ldx : nullptr;
  double x[PE], f[TD][PE];
  TwEntry ob[TD][kTOW];
  auto load_obs = [&](int t, TwEntry (&o)[kTOW]) {
    const TwEntry* sl = tw_slots(md, t);
#pragma unroll
    for (int r = 0; r < kTOW; ++r) o[r] = sl[kTW * r];
  };
  // level t's outputs: stash_k = x_j / R_kk for owned observations (and owned points of x)
  auto emit = [&](int t, const TwEntry (&o)[kTOW]) {
    if (WX) g.store(Xc, t, n, x);
#pragma unroll
    for (int e = 0; e < PE; ++e) xs[lane * PE + e] = x[e];
    lds_order();
#pragma unroll
    for (int r = 0; r < kTOW; ++r) {
      const bool own = g.owned(o[r].l);
      double* dst = own ? St + o[r].k : md.tw_dummy;
      *dst = o[r].v * xs[own ? o[r].l : 0];
    }
    lds_order();
  };
  auto step = [&](int i, double (&fu)[PE], TwEntry (&ou)[kTOW]) {
    const double xm = from_lower_lane(x[PE - 1]), xp = from_upper_lane(x[0]);
    double nx[PE];
#pragma unroll
    for (int e = 0; e < PE; ++e) {
      const double left = e > 0 ? x[e - 1] : xm, right = e + 1 < PE ? x[e + 1] : xp;
      nx[e] = md.ca * left + md.cb * x[e] + md.cc * right + fu[e];
    }
#pragma unroll
    for (int e = 0; e < PE; ++e) x[e] = nx[e];
    g.load(Pc, i + 1 + TD, N, n, fu);
    emit(i + 1, ou);
    load_obs(i + 1 + TD, ou);
  };
  g.load(Pc, 0, N, n, x);
#pragma unroll
  for (int u = 0; u < TD; ++u) g.load(Pc, u + 1, N, n, f[u]);
  {
    TwEntry o0[kTOW];
    load_obs(0, o0);
    emit(0, o0);
  }
#pragma unroll
  for (int u = 0; u < TD; ++u) load_obs(u + 1, ob[u]);
  const int full = N - N % TD;
  for (int i = 0; i < full; i += TD) {
#pragma unroll
    for (int u = 0; u < TD; ++u) step(i + u, f[u], ob[u]);
  }
#pragma unroll
  for (int u = 0; u < TD; ++u)
    if (full + u < N) step(full + u, f[u], ob[u]);
}

// Adjoint from the stash (z_t = H_t^T stash_t); a dense adjoint forcing takes the
// general kernel.
// DIRECT (n and N even, the output columns 16-byte aligned with even ldw): a lane stores
// its owned point pairs straight from registers (pairs outside the owned run go to
// md.tw_dummy), and the H^T stash scatter buffer is cleared after it is read, so a level
// costs one LDS round trip.  Otherwise the owned run is staged through LDS.
template <int PE, int TD, bool DIRECT>
__global__ __launch_bounds__(kTW) void k_sweep_bwd_w(SweepModel md, const double* __restrict__ stash,
                                                     long long ldst, double* __restrict__ Wout,
                                                     long long ldw, const int* __restrict__ skip) {
  __shared__ double xs[kTW * PE];
  if (skip != nullptr && *skip != 0) return;
  const int n = md.n, N = md.N, lane = threadIdx.x;
  const TwGeom<PE> g(n, N, md.tw_W, lane);
  const double* St = stash + (size_t)blockIdx.y * ldst;
  double* Wc = Wout + (size_t)blockIdx.y * ldw;
  // n even: every wavefront's owned run starts at an even index (W is even) in a row that
  // starts at an even index, so with a 16-byte aligned column the stores can be 16 bytes
  // wide (and the owned count g.Wc is even)
  const bool vec2 = (n & 1) == 0 && (reinterpret_cast<uintptr_t>(Wc) & 15) == 0;
  // entries {k, l} of the level 2 TD steps ahead, values (l, stash_k) of the level TD steps
  // ahead.  Levels below 0 read level 0's slots (no step consumes them).  Nothing may touch
  // a loaded register before its use, or the step would wait for it: the entries stay
  // int2 pairs as loaded.
  int2 ent[TD][kTOW];
  int bl[TD][kTOW];
  double bv[TD][kTOW];
  auto load_ent = [&](int t, int2 (&o)[kTOW]) {
    const TwEntry* sl = tw_slots(md, t);
#pragma unroll
    for (int r = 0; r < kTOW; ++r) o[r] = *reinterpret_cast<const int2*>(sl + kTW * r);
  };
  // empty slots hold k = 0, a valid stash entry (q >= 1): every load is issued, so the
  // number of memory operations per step is fixed
  auto load_val = [&](const int2 (&o)[kTOW], int (&ol)[kTOW], double (&v)[kTOW]) {
#pragma unroll
    for (int r = 0; r < kTOW; ++r) {
      ol[r] = o[r].y;
      v[r] = St[o[r].x];
    }
  };
  double w[PE];
  // H_t^T stash_t added over the extended range, then the owned points of level t written
  // out through LDS, 64 (n odd) or 128 (n even) consecutive doubles per store instruction
  auto finish = [&](int t, const int (&ol)[kTOW], const double (&v)[kTOW]) {
    if (DIRECT) {
#pragma unroll
      for (int r = 0; r < kTOW; ++r)
        if (ol[r] >= 0) xs[ol[r]] = v[r];
      lds_order();
#pragma unroll
      for (int e = 0; e < PE; ++e) {
        w[e] += xs[lane * PE + e];
        xs[lane * PE + e] = 0.0;  // read before cleared (in-order LDS), clean for the next level
      }
      lds_order();
#pragma unroll
      for (int q = 0; q < PE / 2; ++q) {
        const int l = lane * PE + 2 * q;  // extended index of the pair; owned ones map to j0 + l - N
        const bool own = l >= N && l + 2 <= N + g.Wc;
        double* dst = own ? Wc + ((size_t)t * n + g.j0 + (l - N)) : md.tw_dummy;
        *reinterpret_cast<double2*>(dst) = make_double2(w[2 * q], w[2 * q + 1]);
      }
      return;
    }
#pragma unroll
    for (int e = 0; e < PE; ++e) xs[lane * PE + e] = 0.0;
    lds_order();
#pragma unroll
    for (int r = 0; r < kTOW; ++r)
      if (ol[r] >= 0) xs[ol[r]] = v[r];
    lds_order();
#pragma unroll
    for (int e = 0; e < PE; ++e) {
      w[e] += xs[lane * PE + e];
      xs[lane * PE + e] = w[e];
    }
    lds_order();
    // a fixed number of unconditional stores (W <= 64 PE): lanes past the owned range
    // repeat the last segment with the same values
    double* row = Wc + (size_t)t * n + g.j0;
    const double* src = xs + N;
    if (vec2) {
#pragma unroll
      for (int it = 0; it < PE / 2; ++it) {
        const int c = min(2 * lane + 2 * kTW * it, g.Wc - 2);
        *reinterpret_cast<double2*>(row + c) = make_double2(src[c], src[c + 1]);
      }
    } else {
#pragma unroll
      for (int it = 0; it < PE; ++it) {
        const int c = min(lane + kTW * it, g.Wc - 1);
        row[c] = src[c];
      }
    }
    lds_order();
  };
#pragma unroll
  for (int e = 0; e < PE; ++e) w[e] = 0.0;
  if (DIRECT) {
#pragma unroll
    for (int e = 0; e < PE; ++e) xs[lane * PE + e] = 0.0;
    lds_order();
  }
  {
    int2 e0[kTOW];
    int ol[kTOW];
    double v0[kTOW];
    load_ent(N, e0);
    load_val(e0, ol, v0);
    finish(N, ol, v0);
  }
#pragma unroll
  for (int u = 0; u < TD; ++u) {
    int2 e0[kTOW];
    load_ent(N - 1 - u, e0);
    load_val(e0, bl[u], bv[u]);
    load_ent(N - 1 - u - TD, ent[u]);
  }
  auto step = [&](int i, int2 (&eu)[kTOW], int (&lu)[kTOW], double (&vu)[kTOW]) {
    const double wm = from_lower_lane(w[PE - 1]), wp = from_upper_lane(w[0]);
    double nw[PE];
#pragma unroll
    for (int e = 0; e < PE; ++e) {
      const double left = e > 0 ? w[e - 1] : wm, right = e + 1 < PE ? w[e + 1] : wp;
      nw[e] = md.ca * right + md.cb * w[e] + md.cc * left;
    }
#pragma unroll
    for (int e = 0; e < PE; ++e) w[e] = nw[e];
    finish(i, lu, vu);
    load_val(eu, lu, vu);
    load_ent(i - 2 * TD, eu);
  };
  // full trips of TD steps without guards (levels N-1 down to N % TD), then the rest
  const int rest = N % TD;
  for (int i0 = N - 1; i0 >= rest; i0 -= TD) {
#pragma unroll
    for (int u = 0; u < TD; ++u) step(i0 - u, ent[u], bl[u], bv[u]);
  }
#pragma unroll
  for (int u = 0; u < TD; ++u)
    if (u < rest) step(rest - 1 - u, ent[u], bl[u], bv[u]);
}

// --------------------------------------------------------------- launch

struct SweepCfg {
  int tpc, ppt, cpb;
};

static SweepCfg sweep_cfg(int n, int kind) {
  SweepCfg c;
  if (n <= 64) {
    c.tpc = 64;
  } else if (n <= (kind == 1 ? 1024 : 2048)) {
    c.tpc = 256;  // Lorenz-96 keeps <= 4 points per thread to stay in registers
  } else if (kind == 0 && n <= 4096) {
    // advection-diffusion, 4 points per thread: 1024 threads per column (at n = 4096, m = 256:
    // 4.73 / 4.6 TB/s forward / adjoint against 4.6 / 4.2 TB/s with 512 threads of 8 points)
    c.tpc = 1024;
  } else {
    c.tpc = 512;  // n <= 8192 (16 points per thread); larger n is rejected at setup
  }
  int ppt = (n + c.tpc - 1) / c.tpc;
  int p2 = 1;
  while (p2 < ppt) p2 <<= 1;
  c.ppt = p2;
  c.cpb = (c.tpc == 64) ? 4 : 1;
  return c;
}

static size_t sweep_lds_bytes(const SweepModel& md, const SweepCfg& c) {
  const int per = 2 + (md.kind == 1 ? 2 : 0);
  return sizeof(double) * ((md.kind == 1 ? 4 * (size_t)md.n : 0) + (size_t)c.cpb * per * md.n) +
         sizeof(int) * ((size_t)md.N + 2);
}

#define WC4D_SWEEP_DISPATCH(KERNEL, OPS, ...)                                                   \
  switch (c.ppt) {                                                                               \
    case 1: hipLaunchKernelGGL((KERNEL<OPS, 1>), grid, block, lds, s, __VA_ARGS__); break;      \
    case 2: hipLaunchKernelGGL((KERNEL<OPS, 2>), grid, block, lds, s, __VA_ARGS__); break;      \
    case 4: hipLaunchKernelGGL((KERNEL<OPS, 4>), grid, block, lds, s, __VA_ARGS__); break;      \
    case 8: hipLaunchKernelGGL((KERNEL<OPS, 8>), grid, block, lds, s, __VA_ARGS__); break;      \
    case 16: hipLaunchKernelGGL((KERNEL<OPS, 16>), grid, block, lds, s, __VA_ARGS__); break;    \
    default: return hipErrorInvalidValue;                                                        \
  }

hipError_t sweep_fwd(const SweepModel& md, const double* P, long long ldp, int m, double* stash,
                     long long ldst, double* Xout, long long ldx, const int* skip, hipStream_t s) {
  if (m <= 0) return hipSuccess;
  switch (l96v_ppt(md, m)) {
    case 4: return l96v_fwd_launch<4>(md, P, stash, Xout, skip, s);
    case 8: return l96v_fwd_launch<8>(md, P, stash, Xout, skip, s);
    case 16: return l96v_fwd_launch<16>(md, P, stash, Xout, skip, s);
    default: break;
  }
  if (md.kind == 0 && m <= 8 && md.tw_pe > 0 && stash != nullptr) {
    dim3 grid((md.n + md.tw_W - 1) / md.tw_W, m);
#define WC4D_TW_FWD(PE, TD)                                                                        \
  if (Xout != nullptr)                                                                             \
    hipLaunchKernelGGL((k_sweep_fwd_w<PE, TD, true>), grid, dim3(kTW), 0, s, md, P, ldp, stash, ldst, \
                       Xout, ldx, skip);                                                           \
  else                                                                                             \
    hipLaunchKernelGGL((k_sweep_fwd_w<PE, TD, false>), grid, dim3(kTW), 0, s, md, P, ldp, stash,     \
                       ldst, Xout, ldx, skip);
    if (md.tw_pe == 4) {
      WC4D_TW_FWD(4, 8)
    } else if (md.tw_pe == 8) {
      WC4D_TW_FWD(8, 8)
    } else {
      return hipErrorInvalidValue;
    }
#undef WC4D_TW_FWD
    return hipGetLastError();
  }
  const SweepCfg c = sweep_cfg(md.n, md.kind);
  const size_t lds = sweep_lds_bytes(md, c);
  dim3 grid((m + c.cpb - 1) / c.cpb), block(c.tpc * c.cpb);
  if (md.kind == 0) {
    WC4D_SWEEP_DISPATCH(k_sweep_fwd, AdvDiffOps, md, P, ldp, m, stash, ldst, Xout, ldx, skip, c.cpb)
  } else {
    WC4D_SWEEP_DISPATCH(k_sweep_fwd, L96Ops, md, P, ldp, m, stash, ldst, Xout, ldx, skip, c.cpb)
  }
  return hipGetLastError();
}

hipError_t sweep_bwd(const SweepModel& md, const double* stash, long long ldst, const double* Z,
                     long long ldz, int m, double* W, long long ldw, const int* skip,
                     hipStream_t s) {
  if (m <= 0) return hipSuccess;
  switch (l96v_ppt(md, m)) {
    case 4: return l96v_bwd_launch<4>(md, stash, Z, W, skip, s);
    case 8: return l96v_bwd_launch<8>(md, stash, Z, W, skip, s);
    case 16: return l96v_bwd_launch<16>(md, stash, Z, W, skip, s);
    default: break;
  }
  if (md.kind == 0 && m <= 8 && md.tw_pe > 0 && stash != nullptr) {
    dim3 grid((md.n + md.tw_W - 1) / md.tw_W, m);
    const bool direct = (md.n & 1) == 0 && (md.N & 1) == 0 && (ldw & 1) == 0 &&
                        (reinterpret_cast<uintptr_t>(W) & 15) == 0;
    if (md.tw_pe == 4 && direct)
      hipLaunchKernelGGL((k_sweep_bwd_w<4, 8, true>), grid, dim3(kTW), 0, s, md, stash, ldst, W, ldw, skip);
    else if (md.tw_pe == 4)
      hipLaunchKernelGGL((k_sweep_bwd_w<4, 8, false>), grid, dim3(kTW), 0, s, md, stash, ldst, W, ldw, skip);
    else if (md.tw_pe == 8 && direct)
      hipLaunchKernelGGL((k_sweep_bwd_w<8, 8, true>), grid, dim3(kTW), 0, s, md, stash, ldst, W, ldw, skip);
    else if (md.tw_pe == 8)
      hipLaunchKernelGGL((k_sweep_bwd_w<8, 8, false>), grid, dim3(kTW), 0, s, md, stash, ldst, W, ldw, skip);
    else
      return hipErrorInvalidValue;
    return hipGetLastError();
  }
  const SweepCfg c = sweep_cfg(md.n, md.kind);
  const size_t lds = sweep_lds_bytes(md, c);
  dim3 grid((m + c.cpb - 1) / c.cpb), block(c.tpc * c.cpb);
  if (md.kind == 0) {
    WC4D_SWEEP_DISPATCH(k_sweep_bwd, AdvDiffOps, md, stash, ldst, Z, ldz, m, W, ldw, skip, c.cpb)
  } else {
    WC4D_SWEEP_DISPATCH(k_sweep_bwd, L96Ops, md, stash, ldst, Z, ldz, m, W, ldw, skip, c.cpb)
  }
  return hipGetLastError();
}

size_t sweep_lds_required(const SweepModel& md) {
  if (md.n > 8192) return (size_t)-1;
  return sweep_lds_bytes(md, sweep_cfg(md.n, md.kind));
}

}  // namespace wc4d
