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

// Observation stash of time level i: stash[k] = rinv[k] * x[idx[k]].
static __device__ inline void obs_gather(const SweepModel& md, int i, const double* x, double* st,
                                         int lt, int tpc) {
  const int kb = md.obs_off[i], ke = md.obs_off[i + 1];
  for (int k = kb + lt; k < ke; k += tpc) st[k] = md.obs_rinv[k] * x[md.obs_idx[k]];
}
// Scatter-add of the stash (H_i^T); indices within one time level are distinct.
static __device__ inline void obs_scatter(const SweepModel& md, int i, double* w, const double* st,
                                          int lt, int tpc) {
  const int kb = md.obs_off[i], ke = md.obs_off[i + 1];
  for (int k = kb + lt; k < ke; k += tpc) w[md.obs_idx[k]] += st[k];
}

// --------------------------------------------------------------- forward

template <class Ops, int PPT>
__global__ __launch_bounds__(512) void k_sweep_fwd(SweepModel md, const double* __restrict__ P,
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
  double* ys = lds;                                       // 4 n stage inputs (L96)
  double* base = lds + (Ops::kStages ? 4 * n : 0) + (size_t)lc * (2 + Ops::kTmp) * n;
  double* b0 = base;
  double* b1 = base + n;
  double* t1 = base + 2 * n;
  double* t2 = base + 3 * n;
  const double* Pc = P + (size_t)(act ? col : 0) * ldp;
  double* St = stash + (size_t)(act ? col : 0) * ldst;
  double* Xc = Xout + (size_t)(act ? col : 0) * ldx;

  double pc[PPT], pn[PPT];
#pragma unroll
  for (int e = 0; e < PPT; ++e) {
    const int j = lt + e * tpc;
    pc[e] = (act && j < n) ? Pc[j] : 0.0;
    pn[e] = (act && j < n && N >= 1) ? Pc[(size_t)n + j] : 0.0;
  }
#pragma unroll
  for (int e = 0; e < PPT; ++e) {
    const int j = lt + e * tpc;
    if (j < n) {
      b0[j] = pc[e];
      if (act && Xout != nullptr) Xc[j] = pc[e];
    }
  }
  __syncthreads();
  if (act && stash != nullptr) obs_gather(md, 0, b0, St, lt, tpc);

  for (int i = 0; i < N; ++i) {
    double* cur = (i & 1) ? b1 : b0;
    double* nxt = (i & 1) ? b0 : b1;
#pragma unroll
    for (int e = 0; e < PPT; ++e) pc[e] = pn[e];
    if (i + 2 <= N) {
#pragma unroll
      for (int e = 0; e < PPT; ++e) {
        const int j = lt + e * tpc;
        pn[e] = (act && j < n) ? Pc[(size_t)(i + 2) * n + j] : 0.0;
      }
    }
    double xn[PPT];
    if constexpr (!Ops::kStages) {
#pragma unroll
      for (int e = 0; e < PPT; ++e) {
        const int j = lt + e * tpc;
        if (j < n) {
          const int jm = j == 0 ? n - 1 : j - 1, jp = j == n - 1 ? 0 : j + 1;
          xn[e] = md.ca * cur[jm] + md.cb * cur[j] + md.cc * cur[jp] + pc[e];
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
          xn[e] = dx[e] + (dt / 6.0) * (d1[e] + 2.0 * d2[e] + 2.0 * d3[e] + d4v) + pc[e];
        }
      }
    }
#pragma unroll
    for (int e = 0; e < PPT; ++e) {
      const int j = lt + e * tpc;
      if (j < n) {
        nxt[j] = xn[e];
        if (act && Xout != nullptr) Xc[(size_t)(i + 1) * n + j] = xn[e];
      }
    }
    __syncthreads();
    if (act && stash != nullptr) obs_gather(md, i + 1, nxt, St, lt, tpc);
  }
}

// --------------------------------------------------------------- adjoint

template <class Ops, int PPT>
__global__ __launch_bounds__(512) void k_sweep_bwd(SweepModel md, const double* __restrict__ stash,
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
  double* ys = lds;
  double* base = lds + (Ops::kStages ? 4 * n : 0) + (size_t)lc * (2 + Ops::kTmp) * n;
  double* b0 = base;
  double* b1 = base + n;
  double* t1 = base + 2 * n;
  double* t2 = base + 3 * n;
  const double* St = dense ? nullptr : stash + (size_t)(act ? col : 0) * ldst;
  const double* Zc = dense ? Z + (size_t)(act ? col : 0) * ldz : nullptr;
  double* Wc = W + (size_t)(act ? col : 0) * ldw;

  // w_N = z_N
  double zc[PPT], zn[PPT];
#pragma unroll
  for (int e = 0; e < PPT; ++e) {
    const int j = lt + e * tpc;
    zc[e] = (dense && act && j < n) ? Zc[(size_t)N * n + j] : 0.0;
    zn[e] = (dense && act && j < n && N >= 1) ? Zc[(size_t)(N - 1) * n + j] : 0.0;
    if (j < n) b0[j] = zc[e];
  }
  __syncthreads();
  if (!dense) {
    if (act) obs_scatter(md, N, b0, St, lt, tpc);
    __syncthreads();
  }
#pragma unroll
  for (int e = 0; e < PPT; ++e) {
    const int j = lt + e * tpc;
    if (act && j < n) Wc[(size_t)N * n + j] = b0[j];
  }

  int par = 0;
  for (int i = N - 1; i >= 0; --i, par ^= 1) {
    double* cur = par ? b1 : b0;
    double* nxt = par ? b0 : b1;
#pragma unroll
    for (int e = 0; e < PPT; ++e) zc[e] = zn[e];
    if (dense && i >= 1) {
#pragma unroll
      for (int e = 0; e < PPT; ++e) {
        const int j = lt + e * tpc;
        zn[e] = (act && j < n) ? Zc[(size_t)(i - 1) * n + j] : 0.0;
      }
    }
    double wn[PPT];
    if constexpr (!Ops::kStages) {
#pragma unroll
      for (int e = 0; e < PPT; ++e) {
        const int j = lt + e * tpc;
        if (j < n) {
          const int jm = j == 0 ? n - 1 : j - 1, jp = j == n - 1 ? 0 : j + 1;
          // (M^T w)_j = ca w_{j+1} + cb w_j + cc w_{j-1}
          wn[e] = md.ca * cur[jp] + md.cb * cur[j] + md.cc * cur[jm] + zc[e];
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
        if (j < n) wn[e] = ax[e] + l96_jacT(ys, t1, j, n) + zc[e];
      }
    }
#pragma unroll
    for (int e = 0; e < PPT; ++e) {
      const int j = lt + e * tpc;
      if (j < n) nxt[j] = wn[e];
    }
    __syncthreads();
    if (!dense) {
      if (act) obs_scatter(md, i, nxt, St, lt, tpc);
      __syncthreads();
    }
#pragma unroll
    for (int e = 0; e < PPT; ++e) {
      const int j = lt + e * tpc;
      if (act && j < n) Wc[(size_t)i * n + j] = nxt[j];
    }
  }
}

// --------------------------------------------------------------- launch

struct SweepCfg {
  int tpc, ppt, cpb;
};

static SweepCfg sweep_cfg(int n, int kind) {
  SweepCfg c;
  if (n <= 64) {
    c.tpc = 64;
  } else if (n <= (kind == 1 ? 1024 : 4096)) {
    c.tpc = 256;  // Lorenz-96 keeps <= 4 points per thread to stay in registers
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
  return sizeof(double) * ((md.kind == 1 ? 4 * (size_t)md.n : 0) + (size_t)c.cpb * per * md.n);
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
