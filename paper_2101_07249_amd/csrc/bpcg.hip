// Many inner loops in one persistent launch: split PCG (Section 3.1, Algorithm 1) with
// the spectral LMP of each problem (Section 3.2, eq. spectral_LMP_factor) on the first-
// level preconditioned Hessian (Section 2.2, eq. forcing_1stlvl_prec) of each of a batch
// of advection-diffusion problems of uneven size.
//
// One grid of workgroups (a few per compute unit) drains a device work queue.  A queue
// entry is one item of one phase of one problem's iteration:
//   C1  rows   u = U^T s0                      (start: r0 = C s0, p0 = C r0)
//   C2  rows   r0 = s0 + U (d .* u)
//   C3  rows   u = U^T r0
//   C4  rows   p0 = r0 + U (d .* u); the first dot products
//   D1  tiles  W = D^{1/2} p                   (64 rows of B^{1/2} / Q^{1/2} x 64 levels)
//   FW  one    forward sweep x_0 = W_0, x_{i+1} = M x_i + W_{i+1}; stash = R^{-1} H x
//   BW  one    adjoint sweep w_N = z_N, w_i = z_i + M^T w_{i+1}, z = H^T stash; W = w
//   D2  tiles  Ap = p + D^{1/2} W
//   T   rows   t = U^T Ap, u = U^T r, p.Ap
//   UP  rows   x += a p, s -= a Ap, r -= a (Ap + U d1), z = r + U d2, r.r, s.s, x.(b + s)
//   P   rows   p = z + b p
// with d = theta^{-1/2} - 1, d1 = d .* t and d2 = d .* (u - a (t + U^T U d1)) = d .* U^T r_new,
// so C^T A p = Ap + U d1 and C r_new = r_new + U d2 (C = C^T): each iteration streams U once
// for its products with U^T and once for its products with U.
//
// Items of one phase run on any workgroups in any order; the workgroup that finishes a
// phase's last item (a per-problem counter) reduces the phase's partial sums in a fixed
// order (deterministic), updates the problem's scalars and enqueues the next phase.  The
// queue is a ring of tickets with per-slot sequence numbers: a producer waits for its slot
// to be free, writes the entry and publishes it; a consumer waits for its ticket to be
// published, reads it and frees the slot for the ticket one ring later.  Workgroups take
// tickets in order, and every published ticket is held by a running workgroup, so items
// keep flowing until no problem is left; then every waiting workgroup sees the count of
// problems left reach zero and returns.  Every wait also gives up after a wall-clock limit
// and raises an error flag that all waits check, so the grid always drains.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <mutex>
#include <numeric>
#include <thread>
#include <vector>

#include "abi_common.h"

namespace wc4d {
namespace {

constexpr int kBT = 256;          // threads per workgroup
constexpr int kRows = 4096;       // rows per row item
constexpr int kTM = 64;           // rows of S per product tile
constexpr int kTN = 64;           // time levels per product tile
constexpr int kTK = 32;           // K step of a product tile
constexpr int kMaxK = 64;         // largest k_r the row phases hold in LDS
constexpr int kMaxPts = 32;       // sweep points per thread (n <= 8192)
constexpr unsigned kRing = 1u << 16;  // queue entries (power of two)

enum Phase { PH_C1 = 0, PH_C2, PH_C3, PH_C4, PH_D1, PH_FW, PH_BW, PH_D2, PH_T, PH_UP, PH_P, PH_NPHASE };

// The phase that follows each phase while the problem goes on (after C4 and UP the problem
// may finish instead; after P the next iteration starts).
__host__ __device__ constexpr int next_phase(int ph) {
  switch (ph) {
    case PH_C1: return PH_C2;
    case PH_C2: return PH_C3;
    case PH_C3: return PH_C4;
    case PH_C4: return PH_D1;
    case PH_D1: return PH_FW;
    case PH_FW: return PH_BW;
    case PH_BW: return PH_D2;
    case PH_D2: return PH_T;
    case PH_T: return PH_UP;
    case PH_UP: return PH_P;
    case PH_P: return PH_D1;
    default: return -1;
  }
}

struct BpDesc {
  int n, N, q, k;
  long long nA;
  double ca, cb, cc;          // stencil: (M x)_j = ca x_{j-1} + cb x_j + cc x_{j+1}, periodic
  const double* Bs;           // B^{1/2}, n x n column-major (symmetric)
  const double* Qs;           // Q^{1/2}
  int scaledB;                // B^{1/2} = bscale Q^{1/2}: one product over all levels
  double bscale;
  const int* slot;            // n_A: observation index at (level, point), -1 where unobserved
  const double* rinv;         // q: 1 / R_kk
  const double* U;            // n_A x k column-major (ldu)
  long long ldu;
  const double* dcoef;        // k: theta^{-1/2} - 1
  const double* GU;           // k x k: U^T U
  const double* b;
  double* x;
  double *s, *r, *z, *p, *Ap, *W, *stash;
  double* part;               // row partials: nchunk x kPartStride
  double* d12;                // 2 k
  int nchunk;                 // row items
  int tiles_m, tiles_n;       // product tiles
  double tol;
  int maxit, criterion;
};
constexpr int kPartStride = 2 * kMaxK + 4;

struct BpState {
  double rr, r0norm2, bnorm2, ss, xbs, pAp, alpha, beta;
  int iter, done, status, pending;
};

struct BpItem {
  int p, phase, item, iter;
};

struct BpQueue {
  unsigned long long head, tail;
  int problems_left, error;
  long long items_done;
  unsigned long long busy[PH_NPHASE + 1];  // wall-clock ticks spent in items of each phase (+ transitions)
  unsigned long long count[PH_NPHASE + 1];
};

struct BpArgs {
  const BpDesc* D;
  BpState* S;
  BpItem* items;
  unsigned long long* seq;
  BpQueue* Q;
  long long wait_ticks;  // wall-clock limit of one wait (100 MHz ticks)
  int sweep_f32;
};

typedef double d4 __attribute__((ext_vector_type(4)));

__device__ inline unsigned long long now_ticks() { return __builtin_amdgcn_s_memrealtime(); }

// device-scope (agent) fences: acquire invalidates this CU's caches of other workgroups'
// data, release writes this workgroup's data back to where other XCDs see it
__device__ inline void fence_acq() { __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent"); }
__device__ inline void fence_rel() { __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent"); }

// Loads and stores through global-address-space pointers.  The item functions are not
// inlined into the kernel (each keeps its own register allocation) and their pointers come
// from the descriptors in memory, so plain pointers would compile to flat accesses, which
// also count against the LDS wait counter and stall every LDS read behind global loads.
typedef double dv2 __attribute__((ext_vector_type(2)));
typedef const __attribute__((address_space(1))) double gdouble;
typedef const __attribute__((address_space(1))) dv2 gdv2;
typedef const __attribute__((address_space(1))) int gint;
__device__ inline double gld(const double* p) { return *(gdouble*)p; }
__device__ inline dv2 gld2(const double* p) { return *(gdv2*)p; }
__device__ inline int gldi(const int* p) { return *(gint*)p; }
__device__ inline void gst(double* p, double v) { *(__attribute__((address_space(1))) double*)p = v; }
// LDS through local-address-space pointers (the item functions receive LDS as plain pointers)
template <class T>
__device__ inline T sld(const T* p) {
  return *(const __attribute__((address_space(3))) T*)p;
}
template <class T>
__device__ inline void sst(T* p, T v) {
  *(__attribute__((address_space(3))) T*)p = v;
}

// back off between polls: 8, 16, ..., 128 sleeps of 8 x 64 cycles
__device__ inline void backoff(int& b) {
  for (int z = 0; z < b; ++z) __builtin_amdgcn_s_sleep(8);
  if (b < 16) b *= 2;
}

template <class T>
__device__ inline T ld_acq(T* p) {
  return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
template <class T>
__device__ inline T ld_rlx(T* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class T>
__device__ inline void st_rel(T* p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// Sums of Q values over the workgroup (every thread passes Q values); thread 0 receives
// them in out[0..Q) (fixed order: deterministic).  red: 4 Q doubles of LDS.
template <int Q>
__device__ inline void block_sums(const double (&v)[Q], double* red, double (&out)[Q]) {
  const int wave = threadIdx.x >> 6;
  double w[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) w[q] = wave_sum_d(v[q]);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) {
#pragma unroll
    for (int q = 0; q < Q; ++q) red[wave * Q + q] = w[q];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < Q; ++q) out[q] = (red[q] + red[Q + q]) + (red[2 * Q + q] + red[3 * Q + q]);
  }
  __syncthreads();
}

// ------------------------------------------------------------------ products
// Y(:, lev) = alpha_lev S X(:, lev) [+ E(:, lev)] for the 64 rows [64 rt, 64 rt + 64) and
// the levels [l0, l0 + nl) of one product tile; S is n x n column-major.  float64 MFMA on
// the transposed product (as in gemm_f64.hip): lanes sharing l/16 hold 16 consecutive rows
// of one output column.  lds: 2 x kTK x 68 doubles.
__device__ __noinline__ void product_tile(const double* __restrict__ S, int n, int rt, int l0, int nl, double scale0,
                             const double* __restrict__ X, const double* __restrict__ E, double* __restrict__ Y,
                             double* lds) {
  constexpr int PA = kTM + 4, PB = kTN + 4;
  double* As = lds;              // [kTK][PA]
  double* Bs = lds + kTK * PA;   // [kTK][PB]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int i0 = rt * kTM;
  const int wi0 = (wave & 1) * 32, wj0 = (wave >> 1) * 32;
  d4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};
  constexpr int kLd = kTK * kTM / kBT;  // elements of each operand per thread and K step
  static_assert(kTM == 64 && kTN == 64 && kLd * kBT == kTK * kTM, "product tile shape");
  double ra[kLd], rb[kLd];
  auto gload = [&](int k0) {
#pragma unroll
    for (int e = 0; e < kLd; ++e) {
      const int idx = tid + kBT * e;
      const int gi = i0 + (idx & 63), gk = k0 + (idx >> 6);
      ra[e] = (gi < n && gk < n) ? gld(S + (long long)gi + (long long)gk * n) : 0.0;
      const int j = idx / kTK, kk = k0 + idx % kTK;
      rb[e] = (j < nl && kk < n) ? gld(X + (long long)(l0 + j) * n + kk) : 0.0;
    }
  };
  gload(0);
  for (int k0 = 0; k0 < n; k0 += kTK) {
    __syncthreads();
#pragma unroll
    for (int e = 0; e < kLd; ++e) {
      const int idx = tid + kBT * e;
      sst(As + (idx >> 6) * PA + (idx & 63), ra[e]);
      sst(Bs + (idx % kTK) * PB + idx / kTK, rb[e]);
    }
    __syncthreads();
    if (k0 + kTK < n) gload(k0 + kTK);
#pragma unroll
    for (int kk = 0; kk < kTK; kk += 4) {
      const int kr = kk + (lane >> 4);
      double av[2], bv[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) av[a] = sld(Bs + kr * PB + wj0 + a * 16 + (lane & 15));
#pragma unroll
      for (int b = 0; b < 2; ++b) bv[b] = sld(As + kr * PA + wi0 + b * 16 + (lane & 15));
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], acc[a][b], 0, 0, 0);
    }
  }
#pragma unroll
  for (int a = 0; a < 2; ++a) {
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) {
      const int j = wj0 + a * 16 + (lane >> 4) + 4 * rr;
      if (j >= nl) continue;
      const int lev = l0 + j;
      const double sc = (lev == 0) ? scale0 : 1.0;
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const int i = i0 + wi0 + b * 16 + (lane & 15);
        if (i < n) {
          const long long o = (long long)lev * n + i;
          double v = sc * acc[a][b][rr];
          if (E != nullptr) v += gld(E + o);
          gst(Y + o, v);
        }
      }
    }
  }
  __syncthreads();  // LDS reuse by the next item
}

// product tile `item` of Y = D^{1/2} X [+ E]
__device__ void dsqrt_item(const BpDesc& d, int item, const double* X, const double* E, double* Y, double* lds) {
  const int rt = item % d.tiles_m, g = item / d.tiles_m;
  if (d.scaledB) {
    const int l0 = g * kTN;
    product_tile(d.Qs, d.n, rt, l0, min(kTN, d.N + 1 - l0), d.bscale, X, E, Y, lds);
  } else if (g == 0) {
    product_tile(d.Bs, d.n, rt, 0, 1, 1.0, X, E, Y, lds);
  } else {
    const int l0 = 1 + (g - 1) * kTN;
    product_tile(d.Qs, d.n, rt, l0, min(kTN, d.N + 1 - l0), 1.0, X, E, Y, lds);
  }
}

// -------------------------------------------------------------------- sweeps
// One workgroup runs a whole sweep; thread t owns points j = t + 256 e (coalesced level
// reads), neighbours come through LDS.  T: float64, or float32 for the reduced-precision
// sweep option (state and stencil in float32; inputs and outputs float64).
template <class T>
__device__ __noinline__ void sweep_fwd_item(const BpDesc& d, T* xs) {
  const int n = d.n, N = d.N, t = threadIdx.x;
  const int E = (n + kBT - 1) / kBT;
  const T ca = (T)d.ca, cb = (T)d.cb, cc = (T)d.cc;
  T xr[kMaxPts];
#pragma unroll
  for (int e = 0; e < kMaxPts; ++e) {
    const int j = t + kBT * e;
    xr[e] = (e < E && j < n) ? (T)gld(d.W + j) : (T)0;
  }
  for (int i = 0;; ++i) {
    // observations of level i: stash = R^{-1} H x_i
#pragma unroll
    for (int e = 0; e < kMaxPts; ++e) {
      const int j = t + kBT * e;
      if (e < E && j < n) {
        const int k = gldi(d.slot + (long long)i * n + j);
        if (k >= 0) gst(d.stash + k, gld(d.rinv + k) * (double)xr[e]);
      }
    }
    if (i == N) break;
#pragma unroll
    for (int e = 0; e < kMaxPts; ++e) {
      const int j = t + kBT * e;
      if (e < E && j < n) sst(xs + j, xr[e]);
    }
    __syncthreads();
    const double* Wn = d.W + (long long)(i + 1) * n;
#pragma unroll
    for (int e = 0; e < kMaxPts; ++e) {
      const int j = t + kBT * e;
      if (e < E && j < n) {
        const int jm = j == 0 ? n - 1 : j - 1, jp = j == n - 1 ? 0 : j + 1;
        xr[e] = ca * sld(xs + jm) + cb * xr[e] + cc * sld(xs + jp) + (T)gld(Wn + j);
      }
    }
    __syncthreads();
  }
}

template <class T>
__device__ __noinline__ void sweep_bwd_item(const BpDesc& d, T* xs) {
  const int n = d.n, N = d.N, t = threadIdx.x;
  const int E = (n + kBT - 1) / kBT;
  const T ca = (T)d.ca, cb = (T)d.cb, cc = (T)d.cc;
  T wr[kMaxPts];
  // w_N = z_N
#pragma unroll
  for (int e = 0; e < kMaxPts; ++e) {
    const int j = t + kBT * e;
    T v = (T)0;
    if (e < E && j < n) {
      const int k = gldi(d.slot + (long long)N * n + j);
      if (k >= 0) v = (T)gld(d.stash + k);
      gst(d.W + (long long)N * n + j, (double)v);
    }
    wr[e] = v;
  }
  for (int i = N - 1; i >= 0; --i) {
#pragma unroll
    for (int e = 0; e < kMaxPts; ++e) {
      const int j = t + kBT * e;
      if (e < E && j < n) sst(xs + j, wr[e]);
    }
    __syncthreads();
    const long long lo = (long long)i * n;
#pragma unroll
    for (int e = 0; e < kMaxPts; ++e) {
      const int j = t + kBT * e;
      if (e < E && j < n) {
        const int jm = j == 0 ? n - 1 : j - 1, jp = j == n - 1 ? 0 : j + 1;
        const int k = gldi(d.slot + lo + j);
        const T z = k >= 0 ? (T)gld(d.stash + k) : (T)0;
        wr[e] = z + ca * sld(xs + jp) + cb * wr[e] + cc * sld(xs + jm);
        gst(d.W + lo + j, (double)wr[e]);
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------- row phases
// The row phases stream U (n_A x k, ldu % 4 == 0, 16-byte aligned): each thread takes 4
// consecutive rows per step and loads them as two 16-byte pieces per column, 8 columns at a
// time, so that a workgroup keeps 16 KB of U loads in flight instead of one row per thread.


// rows [i, i + 4) of column q of U; FULL: all four exist, else zeros past r1
template <bool FULL>
__device__ inline void u_load4(const BpDesc& d, long long i, int q, long long r1, double (&u)[4]) {
  const double* up = d.U + i + (long long)q * d.ldu;
  if (FULL) {
    const dv2 a = gld2(up);
    const dv2 b = gld2(up + 2);
    u[0] = a.x;
    u[1] = a.y;
    u[2] = b.x;
    u[3] = b.y;
  } else {
#pragma unroll
    for (int e = 0; e < 4; ++e) u[e] = (i + e < r1) ? gld(up + e) : 0.0;
  }
}

template <bool FULL>
__device__ inline void v_load4(const double* v, long long i, long long r1, double (&o)[4]) {
#pragma unroll
  for (int e = 0; e < 4; ++e) o[e] = (FULL || i + e < r1) ? gld(v + i + e) : 0.0;
}

// one quad of rows of U^T a and U^T b over the 8 columns [c0, c0 + 8) (columns past k read
// as zero)
template <bool FULL>
__device__ inline void ut_quad(const BpDesc& d, long long i, long long r1, int c0, const double* a,
                               const double* bvec, double (&ta)[8], double (&tb)[8]) {
  double av[4], bv[4] = {0.0, 0.0, 0.0, 0.0};
  v_load4<FULL>(a, i, r1, av);
  if (bvec) v_load4<FULL>(bvec, i, r1, bv);
  double u[8][4];
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    if (c0 + q < d.k) {
      u_load4<FULL>(d, i, c0 + q, r1, u[q]);
    } else {
#pragma unroll
      for (int e = 0; e < 4; ++e) u[q][e] = 0.0;
    }
  }
#pragma unroll
  for (int q = 0; q < 8; ++q) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      ta[q] += u[q][e] * av[e];
      tb[q] += u[q][e] * bv[e];
    }
  }
}

// Partials of U^T a (columns 0..k), U^T b (k..2k, when b != null) and dot(a2, b2) over the
// rows of item `c`: written to part[c * kPartStride + ...].  Whole quads of rows in the
// loop; the one thread whose quad crosses r1 takes it after the loop.
__device__ __noinline__ void ut_rows(const BpDesc& d, int c, const double* a, const double* bvec, const double* da,
                                     const double* db, double* red) {
  const long long r0 = (long long)c * kRows, r1 = min(d.nA, r0 + kRows);
  double* out = d.part + (long long)c * kPartStride;
#pragma unroll 1
  for (int c0 = 0; c0 < d.k; c0 += 8) {
    double ta[8], tb[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) ta[q] = tb[q] = 0.0;
    long long i = r0 + 4LL * threadIdx.x;
#pragma unroll 1
    for (; i + 4 <= r1; i += 4LL * kBT) ut_quad<true>(d, i, r1, c0, a, bvec, ta, tb);
    if (i < r1) ut_quad<false>(d, i, r1, c0, a, bvec, ta, tb);
    double sa[8], sb[8];
    block_sums<8>(ta, red, sa);
    if (bvec) block_sums<8>(tb, red, sb);
    if (threadIdx.x == 0) {
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        if (c0 + q < d.k) {
          out[c0 + q] = sa[q];
          if (bvec) out[d.k + c0 + q] = sb[q];
        }
      }
    }
  }
  if (da != nullptr) {
    double v[1] = {0.0}, sv[1];
    for (long long i = r0 + threadIdx.x; i < r1; i += kBT) v[0] += gld(da + i) * gld(db + i);
    block_sums<1>(v, red, sv);
    if (threadIdx.x == 0) out[2 * d.k] = sv[0];
  }
}

// the U coefficient sums of the UP phase for one quad of rows: u1 = U coef[0..k),
// u2 = U coef[k..2k)
template <bool FULL>
__device__ inline void up_quad(const BpDesc& d, long long i, long long r1, const double* coef, double (&u1)[4],
                               double (&u2)[4]) {
  const int k = d.k;
  int q = 0;
#pragma unroll 1
  for (; q + 8 <= k; q += 8) {
    double u[8][4];
#pragma unroll
    for (int j = 0; j < 8; ++j) u_load4<FULL>(d, i, q + j, r1, u[j]);
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const double c1 = sld(coef + q + j), c2 = sld(coef + k + q + j);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        u1[e] += u[j][e] * c1;
        u2[e] += u[j][e] * c2;
      }
    }
  }
#pragma unroll 1
  for (; q < k; ++q) {
    double u[4];
    u_load4<FULL>(d, i, q, r1, u);
    const double c1 = sld(coef + q), c2 = sld(coef + k + q);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      u1[e] += u[e] * c1;
      u2[e] += u[e] * c2;
    }
  }
}

// y = a + U coef over the rows of item c (coef: k doubles in LDS)
__device__ inline double u_row(const BpDesc& d, long long i, const double* coef) {
  double v = 0.0;
  for (int q = 0; q < d.k; ++q) v += d.U[i + (long long)q * d.ldu] * coef[q];
  return v;
}

__device__ __noinline__ void row_item(const BpDesc& d, BpState& st, int phase, int c, double* lds) {
  double* red = lds;        // 32 doubles
  double* coef = lds + 32;  // 2 k doubles
  const long long r0 = (long long)c * kRows, r1 = min(d.nA, r0 + kRows);
  double* out = d.part + (long long)c * kPartStride;
  if (phase == PH_C1) {
    ut_rows(d, c, d.s, nullptr, nullptr, nullptr, red);
    return;
  }
  if (phase == PH_C3) {
    ut_rows(d, c, d.r, nullptr, nullptr, nullptr, red);
    return;
  }
  if (phase == PH_T) {
    ut_rows(d, c, d.Ap, d.r, d.p, d.Ap, red);
    return;
  }
  if (phase == PH_C2 || phase == PH_C4) {
    for (int q = threadIdx.x; q < d.k; q += kBT) coef[q] = d.d12[d.k + q];
    __syncthreads();
    const double* src = phase == PH_C2 ? d.s : d.r;
    double* dst = phase == PH_C2 ? d.r : d.p;
    double bb = 0.0, ss = 0.0, rr = 0.0, xbs = 0.0;
    for (long long i = r0 + threadIdx.x; i < r1; i += kBT) {
      dst[i] = src[i] + u_row(d, i, coef);
      if (phase == PH_C4) {
        const double bi = d.b[i], si = d.s[i], ri = d.r[i];
        bb += bi * bi;
        ss += si * si;
        rr += ri * ri;
        xbs += d.x[i] * (bi + si);
      }
    }
    if (phase == PH_C4) {
      const double v[4] = {bb, ss, rr, xbs};
      double sv[4];
      block_sums<4>(v, red, sv);
      if (threadIdx.x == 0) {
        out[0] = sv[0];
        out[1] = sv[1];
        out[2] = sv[2];
        out[3] = sv[3];
      }
    }
    __syncthreads();
    return;
  }
  if (phase == PH_UP) {
    for (int q = threadIdx.x; q < 2 * d.k; q += kBT) coef[q] = d.d12[q];
    __syncthreads();
    const double al = st.alpha;
    double rr = 0.0, ss = 0.0, xbs = 0.0;
#pragma unroll 1
    for (long long i = r0 + 4LL * threadIdx.x; i < r1; i += 4LL * kBT) {
      double u1[4] = {0.0, 0.0, 0.0, 0.0}, u2[4] = {0.0, 0.0, 0.0, 0.0};
      if (i + 4 <= r1) {
        up_quad<true>(d, i, r1, coef, u1, u2);
      } else {
        up_quad<false>(d, i, r1, coef, u1, u2);
      }
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const long long ie = i + e;
        if (ie >= r1) continue;
        const double a = gld(d.Ap + ie);
        const double rn = gld(d.r + ie) - al * (a + u1[e]);
        gst(d.r + ie, rn);
        gst(d.z + ie, rn + u2[e]);
        const double xi = gld(d.x + ie) + al * gld(d.p + ie);
        const double si = gld(d.s + ie) - al * a;
        gst(d.x + ie, xi);
        gst(d.s + ie, si);
        rr += rn * rn;
        ss += si * si;
        xbs += xi * (gld(d.b + ie) + si);
      }
    }
    const double v[3] = {rr, ss, xbs};
    double sv[3];
    block_sums<3>(v, red, sv);
    if (threadIdx.x == 0) {
      out[0] = sv[0];
      out[1] = sv[1];
      out[2] = sv[2];
    }
    __syncthreads();
    return;
  }
  if (phase == PH_P) {
    const double be = st.beta;
    long long i = r0 + 4LL * threadIdx.x;
#pragma unroll 1
    for (; i + 4 <= r1; i += 4LL * kBT) {
      double z4[4], p4[4];
      v_load4<true>(d.z, i, r1, z4);
      v_load4<true>(d.p, i, r1, p4);
#pragma unroll
      for (int e = 0; e < 4; ++e) gst(d.p + i + e, z4[e] + be * p4[e]);
    }
    for (; i < r1; ++i) gst(d.p + i, gld(d.z + i) + be * gld(d.p + i));
    return;
  }
}

// ------------------------------------------------------------------ the queue
__device__ int phase_items(const BpDesc& d, int phase) {
  switch (phase) {
    case PH_D1:
    case PH_D2: return d.tiles_m * d.tiles_n;
    case PH_FW:
    case PH_BW: return 1;
    default: return d.nchunk;
  }
}

// Enqueue the items of `phase` of problem p (whole workgroup).  Returns false on a wait
// that ran out of time (the error flag is then set).
__device__ __noinline__ bool enqueue(const BpArgs& A, int p, int phase, int iter, int* sh) {
  const BpDesc& d = A.D[p];
  const int cnt = phase_items(d, phase);
  if (threadIdx.x == 0) {
    sh[3] = 1;
    __hip_atomic_store(&A.S[p].pending, cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const unsigned long long t0 =
        __hip_atomic_fetch_add(&A.Q->tail, (unsigned long long)cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    sh[0] = (int)(t0 & 0x7fffffff);
    sh[1] = (int)(t0 >> 31);
  }
  __syncthreads();
  const unsigned long long t0 = ((unsigned long long)(unsigned)sh[1] << 31) | (unsigned long long)(unsigned)sh[0];
  __syncthreads();
  bool ok = true;
  for (int j = threadIdx.x; j < cnt; j += kBT) {
    const unsigned long long ticket = t0 + j;
    const unsigned slot = (unsigned)(ticket & (kRing - 1));
    const unsigned long long start = now_ticks();
    int bo = 1;
    while (ld_rlx(&A.seq[slot]) != ticket) {
      if (ld_rlx(&A.Q->error) != 0 || now_ticks() - start > (unsigned long long)A.wait_ticks) {
        __hip_atomic_store(&A.Q->error, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        ok = false;
        break;
      }
      backoff(bo);
    }
    if (!ok) break;
    fence_acq();
    A.items[slot] = BpItem{p, phase, j, iter};
    st_rel(&A.seq[slot], ticket + 1);
  }
  if (!ok) sh[3] = 0;
  __syncthreads();
  const bool all_ok = sh[3] != 0;
  __syncthreads();
  return all_ok;  // the same in every thread
}

__device__ void finish_problem(const BpArgs& A, int p, int status) {
  if (threadIdx.x == 0) {
    A.S[p].status = status;
    A.S[p].done = 1;
    __hip_atomic_fetch_add(&A.Q->problems_left, -1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// sum over the row items' partials, entry e (fixed order: deterministic)
__device__ double sum_parts(const BpDesc& d, int e) {
  double v = 0.0;
  for (int c = 0; c < d.nchunk; ++c) v += d.part[(long long)c * kPartStride + e];
  return v;
}

__device__ bool converged(const BpDesc& d, const BpState& st) {
  const double t2 = d.tol * d.tol;
  return d.criterion == WC4D_RES_TRUE ? st.ss <= t2 * st.bnorm2 : st.rr <= t2 * st.r0norm2;
}

// The work after the last item of a phase (whole workgroup; one problem).
__device__ __noinline__ bool transition(const BpArgs& A, int p, int phase, int iter, double* lds, int* sh) {
  const BpDesc& d = A.D[p];
  BpState& st = A.S[p];
  const int k = d.k;
  switch (phase) {
    case PH_C1:
    case PH_C3: {
      // coefficients d .* (U^T v) for the expansion that follows
      for (int q = threadIdx.x; q < k; q += kBT) d.d12[k + q] = d.dcoef[q] * sum_parts(d, q);
      __syncthreads();
      return enqueue(A, p, next_phase(phase), iter, sh);
    }
    case PH_C4: {
      if (threadIdx.x == 0) {
        st.bnorm2 = sum_parts(d, 0);
        st.ss = sum_parts(d, 1);
        st.rr = sum_parts(d, 2);
        st.xbs = sum_parts(d, 3);
        st.r0norm2 = st.rr;
        st.iter = 0;
        sh[2] = (st.bnorm2 == 0.0 || converged(d, st)) ? 1 : 0;
      }
      __syncthreads();
      if (sh[2]) {
        finish_problem(A, p, WC4D_OK);
        return true;
      }
      return enqueue(A, p, next_phase(phase), 1, sh);
    }
    case PH_C2:
    case PH_D1:
    case PH_FW:
    case PH_BW:
    case PH_D2: return enqueue(A, p, next_phase(phase), iter, sh);
    case PH_T: {
      double* tv = lds + 32;   // k: t = U^T Ap
      double* d1 = tv + kMaxK; // k
      if (threadIdx.x == 0) {
        const double pAp = sum_parts(d, 2 * k);
        st.pAp = pAp;
        st.alpha = st.rr / pAp;
        sh[2] = (pAp > 0.0 && isfinite(pAp) && isfinite(st.alpha)) ? 0 : 1;
      }
      for (int q = threadIdx.x; q < k; q += kBT) {
        tv[q] = sum_parts(d, q);
        d1[q] = d.dcoef[q] * tv[q];
      }
      __syncthreads();
      if (sh[2]) {
        finish_problem(A, p, WC4D_EBREAKDOWN);
        return true;
      }
      const double al = st.alpha;
      for (int q = threadIdx.x; q < k; q += kBT) {
        // U^T r_new = U^T r - alpha (t + U^T U d1)
        double g = 0.0;
        for (int c = 0; c < k; ++c) g += d.GU[q + (long long)c * k] * d1[c];
        const double un = sum_parts(d, k + q) - al * (tv[q] + g);
        d.d12[q] = d1[q];
        d.d12[k + q] = d.dcoef[q] * un;
      }
      __syncthreads();
      return enqueue(A, p, next_phase(phase), iter, sh);
    }
    case PH_UP: {
      if (threadIdx.x == 0) {
        const double rr = sum_parts(d, 0);
        st.beta = rr / st.rr;
        st.rr = rr;
        st.ss = sum_parts(d, 1);
        st.xbs = sum_parts(d, 2);
        st.iter = iter;
        int code = -1;
        if (!isfinite(rr) || !isfinite(st.ss)) code = WC4D_EBREAKDOWN;
        else if (converged(d, st)) code = WC4D_OK;
        else if (iter >= d.maxit) code = WC4D_ENOCONV;
        sh[2] = code;
      }
      __syncthreads();
      const int code = sh[2];
      __syncthreads();
      if (code != -1) {
        finish_problem(A, p, code);
        return true;
      }
      return enqueue(A, p, next_phase(phase), iter, sh);
    }
    case PH_P: return enqueue(A, p, next_phase(phase), iter + 1, sh);
    default:
      // no such phase: stop every workgroup
      if (threadIdx.x == 0) __hip_atomic_store(&A.Q->error, 3, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return false;
  }
}

__global__ __launch_bounds__(kBT, 2) void k_bpcg(BpArgs A) {
  extern __shared__ double lds[];
  __shared__ int sh[8];
  __shared__ BpItem cur;
  for (;;) {
    if (threadIdx.x == 0) {
      int got = 0;
      const unsigned long long ticket =
          __hip_atomic_fetch_add(&A.Q->head, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const unsigned slot = (unsigned)(ticket & (kRing - 1));
      const unsigned long long start = now_ticks();
      int bo = 1;
      for (;;) {
        // spin with coherent relaxed loads (no cache invalidation per poll), acquire once seen
        if (ld_rlx(&A.seq[slot]) == ticket + 1) {
          fence_acq();
          cur = A.items[slot];
          st_rel(&A.seq[slot], ticket + kRing);
          got = 1;
          break;
        }
        if (ld_rlx(&A.Q->problems_left) <= 0 || ld_rlx(&A.Q->error) != 0) break;
        if (now_ticks() - start > (unsigned long long)A.wait_ticks) {
          __hip_atomic_store(&A.Q->error, 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          break;
        }
        backoff(bo);
      }
      sh[0] = got;
    }
    __syncthreads();
    const int got = sh[0];
    const BpItem it = cur;
    __syncthreads();
    if (!got) return;
    fence_acq();  // every thread: the item's inputs were written by other workgroups
    const unsigned long long t_item = now_ticks();
    const BpDesc& d = A.D[it.p];
    switch (it.phase) {
      case PH_D1: dsqrt_item(d, it.item, d.p, nullptr, d.W, lds); break;
      case PH_D2: dsqrt_item(d, it.item, d.W, d.p, d.Ap, lds); break;
      case PH_FW:
        if (A.sweep_f32) sweep_fwd_item<float>(d, (float*)lds);
        else sweep_fwd_item<double>(d, lds);
        break;
      case PH_BW:
        if (A.sweep_f32) sweep_bwd_item<float>(d, (float*)lds);
        else sweep_bwd_item<double>(d, lds);
        break;
      default: row_item(d, A.S[it.p], it.phase, it.item, lds); break;
    }
    fence_rel();  // every thread: this item's writes, device-wide
    __syncthreads();
    if (threadIdx.x == 0) {
      // the last item of the phase acquires everyone's writes
      const int old = __hip_atomic_fetch_add(&A.S[it.p].pending, -1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
      sh[1] = (old == 1);
      __hip_atomic_fetch_add(&A.Q->items_done, 1ll, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_fetch_add(&A.Q->busy[it.phase], now_ticks() - t_item, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_fetch_add(&A.Q->count[it.phase], 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
    const int last = sh[1];
    __syncthreads();
    if (last) {
      const unsigned long long t_tr = now_ticks();
      fence_acq();
      const bool ok = transition(A, it.p, it.phase, it.iter, lds, sh);
      fence_rel();
      __syncthreads();
      if (threadIdx.x == 0) {
        __hip_atomic_fetch_add(&A.Q->busy[PH_NPHASE], now_ticks() - t_tr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_add(&A.Q->count[PH_NPHASE], 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      if (!ok) return;
    }
  }
}

__global__ void k_sub(double* __restrict__ s, const double* __restrict__ b, const double* __restrict__ a,
                      long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) s[i] = b[i] - a[i];
}

size_t bpcg_lds_bytes() {
  const size_t prod = sizeof(double) * 2 * kTK * (kTM + 4);
  const size_t sweep = sizeof(double) * 8192;
  const size_t rows = sizeof(double) * (32 + 2 * kMaxK);
  return std::max(prod, std::max(sweep, rows));
}

}  // namespace
}  // namespace wc4d

// ------------------------------------------------------------------- host side
using namespace wc4d;

namespace {

// per-phase profile of the last persistent launch (see wc4d_batch_persistent_profile)
std::mutex g_prof_mu;
double g_prof_ms[PH_NPHASE + 2] = {0};
long long g_prof_count[PH_NPHASE + 2] = {0};

struct Arena {
  double* base = nullptr;
  int* slot = nullptr;
  double* rinv = nullptr;
};

}  // namespace

extern "C" int wc4d_batch_solve_persistent(wc4d_problem* ps, int count, int method, int k_r, int l,
                                           const double* const* G, unsigned long long seed, const double* const* b,
                                           double* const* x, const wc4d_pcg_opts* opts, int flags,
                                           wc4d_pcg_info* infos, int* status, double* kernel_ms) {
  if (ps == nullptr || count < 1 || b == nullptr || x == nullptr || opts == nullptr || infos == nullptr ||
      status == nullptr || k_r < 1 || k_r > kMaxK || l < 0 || (flags & ~WC4D_BATCH_SWEEP_FP32) != 0)
    return WC4D_EINVAL;
  if (opts->maxit < 1 || !(opts->tol >= 0.0) ||
      (opts->criterion != WC4D_RES_TRUE && opts->criterion != WC4D_RES_PRECOND))
    return WC4D_EINVAL;
  int device = -1;
  for (int i = 0; i < count; ++i) {
    wc4d_problem p = ps[i];
    if (!is_state_ok(p) || b[i] == nullptr || x[i] == nullptr) return WC4D_EINVAL;
    if (p->strong) return fail(p, WC4D_EINVAL, "persistent batch: weak-constraint problems only");
    if (device < 0) device = p->device;
    if (p->device != device) return fail(p, WC4D_EINVAL, "batch problems must share one device");
    if (p->model != 0 || p->n > 8192)
      return fail(p, WC4D_EINVAL, "the persistent batch takes advection-diffusion problems with n <= 8192");
    for (int j = 0; j < i; ++j)
      if (ps[j] == p) return fail(p, WC4D_EINVAL, "a problem appears twice in the batch");
  }
  DevGuard guard(device);
  const int m = k_r + l;
  long long queue_need = 0;
  for (int i = 0; i < count; ++i) {
    wc4d_problem p = ps[i];
    if (m > p->nA) return fail(p, WC4D_EINVAL, "sketch wider than the problem");
    if (p->prec & (WC4D_PREC_LMP_FP32 | WC4D_PREC_LMP_FP16))
      return fail(p, WC4D_EINVAL, "the persistent batch streams the float64 U: finalize without LMP copy flags");
    // at most one phase of each problem is in the queue at a time; its largest phase must
    // fit with the ring at most half full, so that a producer never waits on an unread slot
    const long long tiles = (long long)((p->n + kTM - 1) / kTM) * (p->scaledB ? (p->N + kTN) / kTN : 1 + (p->N + kTN - 1) / kTN);
    const long long rows = (p->nA + kRows - 1) / kRows;
    queue_need += std::max(tiles, rows);
  }
  if (queue_need > (long long)(kRing / 2))
    return fail(ps[0], WC4D_EINVAL, "batch too large for the work queue");
  for (int i = 0; i < count; ++i) status[i] = WC4D_OK;
  // the caller's b and x may still be being written on its streams
  {
    const hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return fail(ps[0], WC4D_EHIP, hipGetErrorString(e));
  }

  // ---- LMP builds and s_0 = b - A x_0 with the single-problem kernels, largest first,
  // a few host threads with a stream each
  std::vector<int> order(count);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int c) {
    return (double)ps[a]->n * ps[a]->n * (ps[a]->N + 1.0) > (double)ps[c]->n * ps[c]->n * (ps[c]->N + 1.0);
  });
  std::vector<wc4d_lmp> lmps(count, nullptr);
  std::vector<Arena> arenas(count);
  std::vector<BpDesc> desc(count);
  const long long chunk = kRows;
  int setup_rc = WC4D_OK;
  std::mutex mu;
  std::atomic<int> next{0};
  auto setup = [&]() {
    (void)hipSetDevice(device);
    hipStream_t st = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
      std::lock_guard<std::mutex> lk(mu);
      setup_rc = WC4D_EHIP;
      return;
    }
    for (int oi = next.fetch_add(1); oi < count; oi = next.fetch_add(1)) {
      const int i = order[oi];
      wc4d_problem p = ps[i];
      int rc = wc4d_lmp_build(p, method, k_r, l, G ? G[i] : nullptr, seed + (unsigned long long)i, &lmps[i], st);
      const long long nA = p->nA;
      const int nchunk = (int)((nA + chunk - 1) / chunk);
      Arena& ar = arenas[i];
      const size_t vec_doubles = (size_t)6 * nA + (size_t)std::max(p->q, 1) + (size_t)nchunk * kPartStride +
                                 2 * kMaxK;
      if (rc == WC4D_OK) rc = dev_alloc(p, &ar.base, vec_doubles);
      if (rc == WC4D_OK) rc = dev_alloc(p, &ar.slot, (size_t)nA);
      if (rc == WC4D_OK) rc = dev_alloc(p, &ar.rinv, (size_t)std::max(p->q, 1));
      if (rc == WC4D_OK) {
        // observation slot map and 1/R in stacking order
        std::vector<int> slot((size_t)nA, -1);
        std::vector<double> rinv((size_t)std::max(p->q, 1), 0.0);
        int kk = 0;
        for (int lev = 0; lev <= p->N; ++lev) {
          const auto& idx = p->obs_idx[lev];
          const auto& rd = p->obs_r[lev];
          for (size_t a = 0; a < idx.size(); ++a, ++kk) {
            slot[(size_t)lev * p->n + idx[a]] = kk;
            rinv[kk] = 1.0 / rd[a];
          }
        }
        hipError_t e = hipMemcpyAsync(ar.slot, slot.data(), sizeof(int) * nA, hipMemcpyHostToDevice, st);
        if (e == hipSuccess)
          e = hipMemcpyAsync(ar.rinv, rinv.data(), sizeof(double) * rinv.size(), hipMemcpyHostToDevice, st);
        BpDesc& d = desc[i];
        d.n = p->n;
        d.N = p->N;
        d.q = p->q;
        d.k = k_r;
        d.nA = nA;
        d.ca = p->c + p->r;
        d.cb = 1.0 - p->c - 2.0 * p->r;
        d.cc = p->r;
        d.Bs = p->dB;
        d.Qs = p->dQ;
        d.scaledB = p->scaledB ? 1 : 0;
        d.bscale = p->bScale;
        d.slot = ar.slot;
        d.rinv = ar.rinv;
        d.U = lmps[i]->U;
        d.ldu = lmps[i]->ldu;
        d.dcoef = lmps[i]->dcoef;
        d.GU = lmps[i]->GU;
        d.b = b[i];
        d.x = x[i];
        double* v = ar.base;
        d.s = v;
        d.r = v + nA;
        d.z = v + 2 * nA;
        d.p = v + 3 * nA;
        d.Ap = v + 4 * nA;
        d.W = v + 5 * nA;
        d.stash = v + 6 * nA;
        d.part = d.stash + std::max(p->q, 1);
        d.d12 = d.part + (size_t)nchunk * kPartStride;
        d.nchunk = nchunk;
        d.tiles_m = (p->n + kTM - 1) / kTM;
        d.tiles_n = d.scaledB ? (p->N + 1 + kTN - 1) / kTN : 1 + (p->N + kTN - 1) / kTN;
        d.tol = opts->tol;
        d.maxit = opts->maxit;
        d.criterion = opts->criterion;
        // s_0 = b - A x_0 (float64 operator)
        if (e == hipSuccess && ensure_block(p, 1) == WC4D_OK) {
          rc = apply_A_core(p, x[i], nA, d.Ap, nA, 1, nullptr, st);
          if (rc == WC4D_OK) {
            hipLaunchKernelGGL(k_sub, dim3((unsigned)((nA + 255) / 256)), dim3(256), 0, st, d.s, b[i], d.Ap, nA);
            e = hipGetLastError();
          }
        } else if (e == hipSuccess) {
          rc = WC4D_ENOMEM;
        }
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (rc == WC4D_OK && e != hipSuccess) rc = fail(p, WC4D_EHIP, hipGetErrorString(e));
      }
      if (rc != WC4D_OK) {
        std::lock_guard<std::mutex> lk(mu);
        status[i] = rc;
        if (setup_rc == WC4D_OK) setup_rc = rc;
      }
    }
    (void)hipStreamSynchronize(st);
    (void)hipStreamDestroy(st);
  };
  {
    const int nw = std::min(4, count);
    std::vector<std::thread> pool;
    for (int w = 0; w < nw; ++w) pool.emplace_back(setup);
    for (auto& t : pool) t.join();
  }
  auto cleanup = [&]() {
    for (int i = 0; i < count; ++i) {
      dev_free(&arenas[i].base);
      dev_free(&arenas[i].slot);
      dev_free(&arenas[i].rinv);
      if (lmps[i]) wc4d_lmp_destroy(lmps[i]);
    }
  };
  if (setup_rc != WC4D_OK) {
    cleanup();
    return setup_rc;
  }

  // ---- queue, states, descriptors; the first phase of every problem, largest first
  wc4d_problem p0 = ps[order[0]];
  BpDesc* dD = nullptr;
  BpState* dS = nullptr;
  BpItem* dItems = nullptr;
  unsigned long long* dSeq = nullptr;
  BpQueue* dQ = nullptr;
  auto free_all = [&]() {
    dev_free(&dD);
    dev_free(&dS);
    dev_free(&dItems);
    dev_free(&dSeq);
    dev_free(&dQ);
    cleanup();
  };
  int rc = dev_alloc(p0, &dD, (size_t)count);
  if (rc == WC4D_OK) rc = dev_alloc(p0, &dS, (size_t)count);
  if (rc == WC4D_OK) rc = dev_alloc(p0, &dItems, (size_t)kRing);
  if (rc == WC4D_OK) rc = dev_alloc(p0, &dSeq, (size_t)kRing);
  if (rc == WC4D_OK) rc = dev_alloc(p0, &dQ, 1);
  if (rc != WC4D_OK) {
    free_all();
    return rc;
  }
  auto bail = [&](const char* what, hipError_t e) {
    free_all();
    const std::string msg = std::string("persistent batch: ") + what + ": " + hipGetErrorString(e);
    for (int i = 0; i < count; ++i) fail(ps[i], WC4D_EHIP, msg);
    return WC4D_EHIP;
  };
#define BPCHK(call)                                \
  do {                                             \
    const hipError_t e_ = (call);                  \
    if (e_ != hipSuccess) return bail(#call, e_);  \
  } while (0)
  for (int i = 0; i < count; ++i)
    if (desc[i].ldu % 4 != 0 || (reinterpret_cast<uintptr_t>(desc[i].U) & 15) != 0) {
      free_all();
      return fail(ps[i], WC4D_EINVAL, "persistent batch: U must have ldu % 4 == 0 and 16-byte alignment");
    }
  std::vector<BpState> hS(count);
  std::vector<BpItem> hItems(kRing);
  std::vector<unsigned long long> hSeq(kRing);
  for (unsigned t = 0; t < kRing; ++t) hSeq[t] = t;
  unsigned long long tail = 0;
  for (int oi = 0; oi < count; ++oi) {
    const int i = order[oi];
    std::memset(&hS[i], 0, sizeof(BpState));
    hS[i].pending = desc[i].nchunk;
    for (int c = 0; c < desc[i].nchunk; ++c, ++tail) {
      if (tail >= kRing) {
        free_all();
        return fail(p0, WC4D_EINVAL, "batch too large for the work queue");
      }
      hItems[tail] = BpItem{i, PH_C1, c, 0};
      hSeq[tail] = tail + 1;
    }
  }
  BpQueue hQ{};
  hQ.head = 0;
  hQ.tail = tail;
  hQ.problems_left = count;
  BPCHK(hipMemcpy(dD, desc.data(), sizeof(BpDesc) * count, hipMemcpyHostToDevice));
  BPCHK(hipMemcpy(dS, hS.data(), sizeof(BpState) * count, hipMemcpyHostToDevice));
  BPCHK(hipMemcpy(dItems, hItems.data(), sizeof(BpItem) * kRing, hipMemcpyHostToDevice));
  BPCHK(hipMemcpy(dSeq, hSeq.data(), sizeof(unsigned long long) * kRing, hipMemcpyHostToDevice));
  BPCHK(hipMemcpy(dQ, &hQ, sizeof(BpQueue), hipMemcpyHostToDevice));

  // ---- one persistent launch: as many workgroups as can be resident (at most 2 per CU)
  const size_t lds = bpcg_lds_bytes();
  static std::once_flag attr_once;
  std::call_once(attr_once, [&] {
    (void)hipFuncSetAttribute((const void*)k_bpcg, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  });
  int cus = 0, per_cu = 0;
  BPCHK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device));
  BPCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_bpcg, kBT, lds));
  per_cu = std::max(1, std::min(per_cu, 2));
  // the device's constant wall clock (kHz) sets the wait limit: 20 s per wait
  int clock_khz = 0;
  if (hipDeviceGetAttribute(&clock_khz, hipDeviceAttributeWallClockRate, device) != hipSuccess || clock_khz <= 0)
    clock_khz = 100000;
  BpArgs args{dD, dS, dItems, dSeq, dQ, 20ll * 1000 * clock_khz, (flags & WC4D_BATCH_SWEEP_FP32) ? 1 : 0};
  hipEvent_t e0 = nullptr, e1 = nullptr;
  BPCHK(hipEventCreate(&e0));
  BPCHK(hipEventCreate(&e1));
  BPCHK(hipEventRecord(e0, nullptr));
  hipLaunchKernelGGL(k_bpcg, dim3(cus * per_cu), dim3(kBT), lds, nullptr, args);
  hipError_t le = hipGetLastError();
  BPCHK(hipEventRecord(e1, nullptr));
  hipError_t se = hipEventSynchronize(e1);
  float ms = 0.f;
  if (se == hipSuccess) (void)hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (le != hipSuccess || se != hipSuccess) {
    free_all();
    const std::string msg = std::string("persistent batch launch (") + std::to_string(cus * per_cu) +
                            " workgroups, " + std::to_string(lds) + " bytes of LDS): " +
                            hipGetErrorString(le != hipSuccess ? le : se);
    for (int i = 0; i < count; ++i) fail(ps[i], WC4D_EHIP, msg);
    return WC4D_EHIP;
  }
  if (kernel_ms) *kernel_ms = ms;
  BPCHK(hipMemcpy(&hQ, dQ, sizeof(BpQueue), hipMemcpyDeviceToHost));
  {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    for (int ph = 0; ph <= PH_NPHASE; ++ph) {
      g_prof_ms[ph] = (double)hQ.busy[ph] / (double)clock_khz;
      g_prof_count[ph] = (long long)hQ.count[ph];
    }
    g_prof_ms[PH_NPHASE + 1] = ms;
    g_prof_count[PH_NPHASE + 1] = (long long)cus * per_cu;
  }
  BPCHK(hipMemcpy(hS.data(), dS, sizeof(BpState) * count, hipMemcpyDeviceToHost));
  int ret = WC4D_OK;
  if (hQ.error != 0 || hQ.problems_left != 0) {
    const std::string msg = "persistent batch: the launch ended with " + std::to_string(hQ.problems_left) +
                            " problems left (error flag " + std::to_string(hQ.error) + ", items done " +
                            std::to_string(hQ.items_done) + ", tickets taken " + std::to_string(hQ.head) +
                            ", issued " + std::to_string(hQ.tail) + ")";
    for (int i = 0; i < count; ++i) fail(ps[i], WC4D_EHIP, msg);
    ret = WC4D_EHIP;
  }
  for (int i = 0; i < count; ++i) {
    const BpState& s = hS[i];
    wc4d_pcg_info& inf = infos[i];
    inf.iters = s.iter;
    inf.status = s.done ? s.status : WC4D_EHIP;
    inf.relres_true = s.bnorm2 > 0 ? std::sqrt(s.ss / s.bnorm2) : 0.0;
    inf.relres_precond = s.r0norm2 > 0 ? std::sqrt(s.rr / s.r0norm2) : 0.0;
    inf.J = -0.5 * s.xbs;
    status[i] = inf.status;
    if (status[i] != WC4D_OK && status[i] != WC4D_ENOCONV && status[i] != WC4D_EBREAKDOWN && ret == WC4D_OK)
      ret = status[i];
  }
  free_all();
  return ret;
#undef BPCHK
}

extern "C" int wc4d_batch_persistent_profile(double* ms, long long* count, int n) {
  if (ms == nullptr || count == nullptr || n < 1) return WC4D_EINVAL;
  std::lock_guard<std::mutex> lk(g_prof_mu);
  for (int i = 0; i < n && i < PH_NPHASE + 2; ++i) {
    ms[i] = g_prof_ms[i];
    count[i] = g_prof_count[i];
  }
  return PH_NPHASE + 2;
}
