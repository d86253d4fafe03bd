// Learned sketch network: per time level, a periodic 1-D convolution net along the grid
// axis maps a Gaussian start block and four features of the trajectory and the
// observation pattern to the start block G of the randomised eigendecompositions
// (Section 4, the Gaussian start matrix of Algorithms 3-5).  Float16 weights and
// activations, float32 MFMA accumulation.
//
// Layouts (P = (N+1) n points, p = i n + j):
//   input X0      fp16 [P][cp0]   channels 0..nz-1 Gaussian block, nz..nz+3 features,
//                                  zero up to cp0 (a multiple of 32)
//   hidden A_l    fp16 [P][64]    tanh activations
//   weights W_l   fp16 [64][5 cp] row c_out holds tap t's input channels at t*cp + c'
//   output G      fp64 column-major n_A x 64 (ld), the sketch block
// Conv: H[c][p] = b[c] + sum_{t, c'} W[c][t cp + c'] A[p + t - 2][c'], with the point
// index wrapping inside its time level.  The product runs on v_mfma_f32_16x16x32_f16
// (rows = output channels, columns = points, K = the 5 cp taps x channels): operand a
// = W[row l%16][k 8(l/16)..+8], operand b = A[point l%16][k 8(l/16)..+8], result
// register r = D[4(l/16) + r][l%16].
#include <algorithm>

#include "wc4d_internal.h"

namespace wc4d {

typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef _Float16 h4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int kCH = 64;  // hidden / output channels
constexpr int kKW = 5;   // taps
constexpr int kTP = 128; // points per tile (4 waves x 32)

static __device__ inline f4 mfma_f16(h8 a, h8 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
}

// ------------------------------------------------------------------ input features
// One workgroup per time level i.  traj: (N+1) x n float64 or null.
__global__ __launch_bounds__(256) void k_net_features(int n, int N, const double* __restrict__ traj,
                                                      const int* __restrict__ obs_off,
                                                      const int* __restrict__ obs_idx,
                                                      const double* __restrict__ Om, long long ldo,
                                                      int nz, int cp0, _Float16* __restrict__ X0) {
  const int i = blockIdx.x;
  __shared__ int s_tnext;
  if (threadIdx.x == 0) {
    int t = -1;
    for (int u = i; u <= N; ++u)
      if (obs_off[u + 1] > obs_off[u]) {
        t = u;
        break;
      }
    s_tnext = t;
  }
  __syncthreads();
  const int tn = s_tnext;
  const double fdist = (tn >= 0) ? exp(-(double)(tn - i) / 5.0) : 0.0;
  const double ftime = (double)i / (double)N;
  for (int j = threadIdx.x; j < n; j += blockDim.x) {
    const long long p = (long long)i * n + j;
    _Float16* row = X0 + p * cp0;
    for (int c8 = 0; c8 < cp0; c8 += 8) {
      h8 v;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int c = c8 + e;
        double x = 0.0;
        if (c < nz) x = Om[p + (long long)c * ldo];
        else if (c == nz) x = (traj != nullptr) ? (traj[p] - 2.3) / 3.6 : 0.0;
        else if (c == nz + 2) x = ftime;
        else if (c == nz + 3) x = fdist;
        v[e] = (_Float16)x;
      }
      *reinterpret_cast<h8*>(row + c8) = v;
    }
  }
  __syncthreads();
  for (int k = obs_off[i] + threadIdx.x; k < obs_off[i + 1]; k += blockDim.x)
    X0[((long long)i * n + obs_idx[k]) * cp0 + nz + 1] = (_Float16)1.0f;
}

hipError_t net_features(int n, int N, const double* traj, const int* obs_off, const int* obs_idx,
                        const double* Om, long long ldo, int nz, int cp0, _Float16* X0, hipStream_t s) {
  hipLaunchKernelGGL(k_net_features, dim3(N + 1), dim3(256), 0, s, n, N, traj, obs_off, obs_idx, Om, ldo,
                     nz, cp0, X0);
  return hipGetLastError();
}

// ------------------------------------------------------------------ convolution
// MODE 0: Hout = tanh(acc + b) (fp16 [P][64]); MODE 1: G = acc + b (fp64, column-major
// ld ldg); MODE 2 (backward data): Hout = acc * (1 - Aprev^2), no bias.
// Persistent: each workgroup stages W in LDS once and loops over tiles.
template <int MODE>
__global__ __launch_bounds__(256) void k_net_conv(int n, int T, int cp, const _Float16* __restrict__ X,
                                                  const _Float16* __restrict__ W,
                                                  const _Float16* __restrict__ bias,
                                                  _Float16* __restrict__ Hout, double* __restrict__ G,
                                                  long long ldg, const _Float16* __restrict__ Aprev) {
  extern __shared__ __attribute__((aligned(16))) unsigned char net_smem[];
  const int kwc = kKW * cp;   // halfs per weight row
  const int wp = kwc + 8;     // LDS pitches (halfs), multiples of 8
  const int xp = cp + 8;
  _Float16* Ws = reinterpret_cast<_Float16*>(net_smem);
  _Float16* Xs = Ws + kCH * wp;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wrow8 = kwc / 8;
  for (int e = tid; e < kCH * wrow8; e += 256) {
    const int r = e / wrow8, c8 = (e % wrow8) * 8;
    *reinterpret_cast<h8*>(Ws + r * wp + c8) = *reinterpret_cast<const h8*>(W + (size_t)r * kwc + c8);
  }
  const int tpl = (n + kTP - 1) / kTP;
  const int ntiles = T * tpl;
  const int cpr = cp / 8;
  const int kk = 8 * (lane >> 4);
  const int pw = wave * 32;
  for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int i = tile / tpl, j0 = (tile % tpl) * kTP;
    __syncthreads();  // W staged; previous tile's reads of Xs finished
    for (int e = tid; e < (kTP + 4) * cpr; e += 256) {
      const int r = e / cpr, c8 = (e % cpr) * 8;
      int j = (j0 - 2 + r) % n;
      if (j < 0) j += n;
      *reinterpret_cast<h8*>(Xs + r * xp + c8) =
          *reinterpret_cast<const h8*>(X + ((size_t)i * n + j) * cp + c8);
    }
    __syncthreads();
    f4 acc[4][2];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) acc[a][b] = f4{0.f, 0.f, 0.f, 0.f};
    for (int t = 0; t < kKW; ++t) {
      for (int c0 = 0; c0 < cp; c0 += 32) {
        h8 av[4], bv[2];
#pragma unroll
        for (int cb = 0; cb < 4; ++cb)
          av[cb] = *reinterpret_cast<const h8*>(Ws + (cb * 16 + (lane & 15)) * wp + t * cp + c0 + kk);
#pragma unroll
        for (int pb = 0; pb < 2; ++pb)
          bv[pb] = *reinterpret_cast<const h8*>(Xs + (pw + pb * 16 + (lane & 15) + t) * xp + c0 + kk);
#pragma unroll
        for (int cb = 0; cb < 4; ++cb)
#pragma unroll
          for (int pb = 0; pb < 2; ++pb) acc[cb][pb] = mfma_f16(av[cb], bv[pb], acc[cb][pb]);
      }
    }
    // acc[cb][pb][r] = H[channel cb*16 + 4(l/16) + r][point j0 + pw + pb*16 + l%16]
#pragma unroll
    for (int pb = 0; pb < 2; ++pb) {
      const int j = j0 + pw + pb * 16 + (lane & 15);
      if (j >= n) continue;
      const long long p = (long long)i * n + j;
#pragma unroll
      for (int cb = 0; cb < 4; ++cb) {
        const int c = cb * 16 + 4 * (lane >> 4);
        if (MODE == 0) {
          h4 v;
#pragma unroll
          for (int r = 0; r < 4; ++r) v[r] = (_Float16)tanhf(acc[cb][pb][r] + (float)bias[c + r]);
          *reinterpret_cast<h4*>(Hout + p * kCH + c) = v;
        } else if (MODE == 1) {
#pragma unroll
          for (int r = 0; r < 4; ++r) G[p + (long long)(c + r) * ldg] = (double)(acc[cb][pb][r] + (float)bias[c + r]);
        } else {
          const h4 a = *reinterpret_cast<const h4*>(Aprev + p * kCH + c);
          h4 v;
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const float af = (float)a[r];
            v[r] = (_Float16)(acc[cb][pb][r] * (1.0f - af * af));
          }
          *reinterpret_cast<h4*>(Hout + p * kCH + c) = v;
        }
      }
    }
  }
}

size_t net_conv_lds_bytes(int cp) {
  return sizeof(_Float16) * ((size_t)kCH * (kKW * cp + 8) + (size_t)(kTP + 4) * (cp + 8));
}

static int net_grid(long long ntiles) {
  return (int)std::min<long long>(ntiles, 512);
}

template <int MODE>
static hipError_t conv_launch(int n, int T, int cp, const _Float16* X, const _Float16* W, const _Float16* b,
                              _Float16* H, double* G, long long ldg, const _Float16* Aprev, hipStream_t s) {
  const size_t lds = net_conv_lds_bytes(cp);
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_net_conv<MODE>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  const long long ntiles = (long long)T * ((n + kTP - 1) / kTP);
  hipLaunchKernelGGL(k_net_conv<MODE>, dim3(net_grid(ntiles)), dim3(256), lds, s, n, T, cp, X, W, b, H, G,
                     ldg, Aprev);
  return hipGetLastError();
}

hipError_t net_conv_hidden(int n, int T, int cp, const _Float16* X, const _Float16* W, const _Float16* b,
                           _Float16* H, hipStream_t s) {
  return conv_launch<0>(n, T, cp, X, W, b, H, nullptr, 0, nullptr, s);
}
hipError_t net_conv_out(int n, int T, int cp, const _Float16* X, const _Float16* W, const _Float16* b,
                        double* G, long long ldg, hipStream_t s) {
  return conv_launch<1>(n, T, cp, X, W, b, nullptr, G, ldg, nullptr, s);
}
hipError_t net_conv_bwd_data(int n, int T, const _Float16* dH, const _Float16* Wt, const _Float16* Aprev,
                             _Float16* dHprev, hipStream_t s) {
  return conv_launch<2>(n, T, kCH, dH, Wt, nullptr, dHprev, nullptr, 0, Aprev, s);
}

// ------------------------------------------------------------------ weight gradient
// part[blk][c * 5cp + t cp + c'] = sum over the workgroup's points p of dH[p][c] X[p+t-2][c'],
// part[blk][64 * 5cp + c] = sum_p dH[p][c].  MFMA rows = c, columns = (t, c'), K = points.
template <int CP>
__global__ __launch_bounds__(256) void k_net_wgrad(int n, int T, const _Float16* __restrict__ X,
                                                   const _Float16* __restrict__ dH, float* __restrict__ part) {
  constexpr int NKB = kKW * CP / 16;      // 16-column blocks of the (t, c') axis
  constexpr int NKW = (NKB + 3) / 4;      // per wave
  constexpr int DP = kTP + 8;             // dHs pitch (halfs)
  constexpr int XP = kTP + 8;             // Xs pitch (rows r = 0..kTP+3 <-> j0 - 2 + r)
  __shared__ __attribute__((aligned(16))) _Float16 dHs[kCH * DP];
  __shared__ __attribute__((aligned(16))) _Float16 Xs[CP * XP];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int tpl = (n + kTP - 1) / kTP;
  const int ntiles = T * tpl;
  f4 acc[NKW][4];
#pragma unroll
  for (int a = 0; a < NKW; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = f4{0.f, 0.f, 0.f, 0.f};
  float bsum = 0.f;
  for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int i = tile / tpl, j0 = (tile % tpl) * kTP;
    __syncthreads();
    for (int e = tid; e < kTP * (kCH / 8); e += 256) {
      const int r = e / (kCH / 8), c8 = (e % (kCH / 8)) * 8;
      const int j = j0 + r;
      h8 v = h8{0, 0, 0, 0, 0, 0, 0, 0};
      if (j < n) v = *reinterpret_cast<const h8*>(dH + ((size_t)i * n + j) * kCH + c8);
#pragma unroll
      for (int q = 0; q < 8; ++q) dHs[(c8 + q) * DP + r] = v[q];
    }
    for (int e = tid; e < (kTP + 4) * (CP / 8); e += 256) {
      const int r = e / (CP / 8), c8 = (e % (CP / 8)) * 8;
      int j = (j0 - 2 + r) % n;
      if (j < 0) j += n;
      const h8 v = *reinterpret_cast<const h8*>(X + ((size_t)i * n + j) * CP + c8);
#pragma unroll
      for (int q = 0; q < 8; ++q) Xs[(c8 + q) * XP + r] = v[q];
    }
    __syncthreads();
    if (tid < kCH) {
      float sacc = 0.f;
      for (int r = 0; r < kTP; ++r) sacc += (float)dHs[tid * DP + r];
      bsum += sacc;
    }
#pragma unroll
    for (int ks = 0; ks < kTP / 32; ++ks) {
      const int pb = ks * 32 + 8 * (lane >> 4);
      h8 av[4];
#pragma unroll
      for (int cb = 0; cb < 4; ++cb)
        av[cb] = *reinterpret_cast<const h8*>(dHs + (cb * 16 + (lane & 15)) * DP + pb);
#pragma unroll
      for (int w = 0; w < NKW; ++w) {
        const int kb = wave + 4 * w;
        if (kb >= NKB) break;
        const int k = kb * 16 + (lane & 15);
        const int t = k / CP, c = k % CP;
        const _Float16* xr = Xs + c * XP + pb + t;
        h8 bv;
#pragma unroll
        for (int e = 0; e < 8; ++e) bv[e] = xr[e];
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) acc[w][cb] = mfma_f16(av[cb], bv, acc[w][cb]);
      }
    }
  }
  // acc[w][cb][r] = D[c = cb*16 + 4(l/16) + r][k = (wave + 4w)*16 + l%16]
  float* out = part + (size_t)blockIdx.x * (kCH * kKW * CP + kCH);
#pragma unroll
  for (int w = 0; w < NKW; ++w) {
    const int kb = wave + 4 * w;
    if (kb >= NKB) break;
    const int k = kb * 16 + (lane & 15);
#pragma unroll
    for (int cb = 0; cb < 4; ++cb)
#pragma unroll
      for (int r = 0; r < 4; ++r) out[(size_t)(cb * 16 + 4 * (lane >> 4) + r) * (kKW * CP) + k] = acc[w][cb][r];
  }
  if (tid < kCH) out[kCH * kKW * CP + tid] = bsum;
}

int net_wgrad_blocks(int n, int T) {
  const long long ntiles = (long long)T * ((n + kTP - 1) / kTP);
  return (int)std::min<long long>(ntiles, 256);
}

hipError_t net_wgrad(int n, int T, int cp, const _Float16* X, const _Float16* dH, float* part, hipStream_t s) {
  const int nb = net_wgrad_blocks(n, T);
  if (cp == 32) hipLaunchKernelGGL(k_net_wgrad<32>, dim3(nb), dim3(256), 0, s, n, T, X, dH, part);
  else if (cp == 64) hipLaunchKernelGGL(k_net_wgrad<64>, dim3(nb), dim3(256), 0, s, n, T, X, dH, part);
  else if (cp == 96) hipLaunchKernelGGL(k_net_wgrad<96>, dim3(nb), dim3(256), 0, s, n, T, X, dH, part);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

// grad[e] = inv_scale[0] * sum_b part[b][e], fixed order.
__global__ void k_net_reduce(int nb, int len, const float* __restrict__ part, const float* __restrict__ scal,
                             float* __restrict__ grad) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= len) return;
  float acc = 0.f;
  for (int b = 0; b < nb; ++b) acc += part[(size_t)b * len + e];
  grad[e] = acc * scal[1];
}

hipError_t net_reduce(int nb, int len, const float* part, const float* scal, float* grad, hipStream_t s) {
  hipLaunchKernelGGL(k_net_reduce, dim3((len + 255) / 256), dim3(256), 0, s, nb, len, part, scal, grad);
  return hipGetLastError();
}

// ------------------------------------------------------------------ loss scaling
// Largest |dG| over the block (two stages), then scal = {2^e, 2^-e} with 2^e |dG|max in
// (512, 1024]; both stay 1 when the block is zero.
constexpr int kAB = 512;
__global__ void k_absmax_partial(long long rows, int cols, const double* __restrict__ X, long long ldx,
                                 double* __restrict__ part) {
  double mx = 0.0;
  const long long tot = rows * cols;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < tot;
       e += (long long)gridDim.x * blockDim.x) {
    const long long c = e / rows, r = e % rows;
    mx = fmax(mx, fabs(X[r + c * ldx]));
  }
  __shared__ double sh[256];
  sh[threadIdx.x] = mx;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ void k_absmax_final(const double* __restrict__ part, float* __restrict__ scal) {
  __shared__ double sh[256];
  double mx = 0.0;
  for (int b = threadIdx.x; b < kAB; b += 256) mx = fmax(mx, part[b]);
  sh[threadIdx.x] = mx;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double m = sh[0];
    int e = 0;
    if (m > 0.0 && isfinite(m)) {
      int ex;
      (void)frexp(m, &ex);            // m in [2^(ex-1), 2^ex)
      e = 10 - ex;
      e = e > 100 ? 100 : (e < -100 ? -100 : e);
    }
    scal[0] = ldexpf(1.0f, e);
    scal[1] = ldexpf(1.0f, -e);
  }
}

// dH[p][c] = fp16(scal[0] * dG[p + c ldg]) for the 64 output channels.
__global__ void k_net_dg_to_h(long long P, const double* __restrict__ dG, long long ldg,
                              const float* __restrict__ scal, _Float16* __restrict__ dH) {
  const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  const double sc = (double)scal[0];
  for (int c8 = 0; c8 < kCH; c8 += 8) {
    h8 v;
#pragma unroll
    for (int e = 0; e < 8; ++e) v[e] = (_Float16)(sc * dG[p + (long long)(c8 + e) * ldg]);
    *reinterpret_cast<h8*>(dH + p * kCH + c8) = v;
  }
}

size_t net_scale_ws_doubles() { return kAB; }

hipError_t net_loss_scale(long long P, const double* dG, long long ldg, double* ws, float* scal,
                          _Float16* dH, hipStream_t s) {
  hipLaunchKernelGGL(k_absmax_partial, dim3(kAB), dim3(256), 0, s, P, kCH, dG, ldg, ws);
  hipLaunchKernelGGL(k_absmax_final, dim3(1), dim3(256), 0, s, ws, scal);
  hipLaunchKernelGGL(k_net_dg_to_h, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, s, P, dG, ldg, scal, dH);
  return hipGetLastError();
}

// ------------------------------------------------------------------ parameters
// Adam (Kingma and Ba) on the float32 master copy; writes the float16 weights.
// c1 = 1 / (1 - beta1^step), c2 = 1 / (1 - beta2^step).
__global__ void k_net_adam(long long len, float* __restrict__ th, float* __restrict__ m, float* __restrict__ v,
                           const float* __restrict__ g, float lr, float b1, float b2, float eps, float c1,
                           float c2, _Float16* __restrict__ w16) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= len) return;
  const float ge = g[e];
  const float me = b1 * m[e] + (1.f - b1) * ge;
  const float ve = b2 * v[e] + (1.f - b2) * ge * ge;
  m[e] = me;
  v[e] = ve;
  const float t = th[e] - lr * (me * c1) / (sqrtf(ve * c2) + eps);
  th[e] = t;
  w16[e] = (_Float16)t;
}

hipError_t net_adam(long long len, float* th, float* m, float* v, const float* g, float lr, float b1, float b2,
                    float eps, float c1, float c2, _Float16* w16, hipStream_t s) {
  hipLaunchKernelGGL(k_net_adam, dim3((unsigned)((len + 255) / 256)), dim3(256), 0, s, len, th, m, v, g, lr, b1,
                     b2, eps, c1, c2, w16);
  return hipGetLastError();
}

__global__ void k_net_to_f16(long long len, const float* __restrict__ th, _Float16* __restrict__ w16) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < len) w16[e] = (_Float16)th[e];
}

hipError_t net_to_f16(long long len, const float* th, _Float16* w16, hipStream_t s) {
  hipLaunchKernelGGL(k_net_to_f16, dim3((unsigned)((len + 255) / 256)), dim3(256), 0, s, len, th, w16);
  return hipGetLastError();
}

// Wt[c'][t' 64 + c] = W[c][(4 - t') 64 + c'] for a 64-in / 64-out layer: the weights of
// the backward-data convolution (taps mirrored, channels transposed).
__global__ void k_net_pack_t(const _Float16* __restrict__ W, _Float16* __restrict__ Wt) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= kCH * kKW * kCH) return;
  const int cpr = e / (kKW * kCH), rem = e % (kKW * kCH);
  const int tp = rem / kCH, c = rem % kCH;
  Wt[e] = W[(size_t)c * (kKW * kCH) + (kKW - 1 - tp) * kCH + cpr];
}

hipError_t net_pack_t(const _Float16* W, _Float16* Wt, hipStream_t s) {
  hipLaunchKernelGGL(k_net_pack_t, dim3((kCH * kKW * kCH + 255) / 256), dim3(256), 0, s, W, Wt);
  return hipGetLastError();
}

// ------------------------------------------------------------------ capture loss helpers
// w[i] = 1 - 1/theta[i], sums[0] = sum w (single workgroup).
__global__ void k_loss_weights(int k, const double* __restrict__ theta, double* __restrict__ w,
                               double* __restrict__ sums) {
  __shared__ double sh[256];
  double acc = 0.0;
  for (int i = threadIdx.x; i < k; i += 256) {
    const double wi = 1.0 - 1.0 / theta[i];
    w[i] = wi;
    acc += wi;
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) sums[0] = sh[0];
}

// f = -sum_ij Sinv(i,j) T(j,i) / sums[0]; then M1 *= 2/sums[0], M2 *= -2/sums[0].
__global__ void k_loss_finish(int m, int k, const double* __restrict__ Sinv, const double* __restrict__ Tm,
                              const double* __restrict__ sums, double* __restrict__ f, double* __restrict__ M1,
                              double* __restrict__ M2) {
  __shared__ double sh[256];
  double acc = 0.0;
  for (int e = threadIdx.x; e < m * m; e += 256) {
    const int i = e % m, j = e / m;
    acc += Sinv[i + (size_t)j * m] * Tm[j + (size_t)i * m];
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  const double sw = sums[0];
  if (threadIdx.x == 0) f[0] = -sh[0] / sw;
  const double c = 2.0 / sw;
  for (int e = threadIdx.x; e < m * m; e += 256) M1[e] *= c;
  for (int e = threadIdx.x; e < k * m; e += 256) M2[e] *= -c;
}

hipError_t loss_weights(int k, const double* theta, double* w, double* sums, hipStream_t s) {
  hipLaunchKernelGGL(k_loss_weights, dim3(1), dim3(256), 0, s, k, theta, w, sums);
  return hipGetLastError();
}
hipError_t loss_finish(int m, int k, const double* Sinv, const double* Tm, const double* sums, double* f,
                       double* M1, double* M2, hipStream_t s) {
  hipLaunchKernelGGL(k_loss_finish, dim3(1), dim3(256), 0, s, m, k, Sinv, Tm, sums, f, M1, M2);
  return hipGetLastError();
}

}  // namespace wc4d
