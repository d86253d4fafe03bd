// Gaussian start block of the randomised eigendecompositions (Section 4, Algorithms 3-5:
// G has independent N(0, 1) entries), drawn on the device by a counter-based generator
// so that no host draw or host-to-device copy sits in front of an LMP build.
//
// Generator: Philox-4x32-10 (Salmon, Moraes, Dror and Shaw, SC 2011) -- ten rounds of two
// 32 x 32 -> 64-bit multiplications by 0xD2511F53 and 0xCD9E8D57, the halves crossed with
// the other two counter words and the key, the key advanced by 0x9E3779B9 / 0xBB67AE85
// between rounds -- followed by the Box-Muller transform (Box and Muller 1958).
//
// Mapping of the block: entry (r, c) of the block of seed s uses key (s mod 2^32, s >> 32)
// and counter (r >> 1, c, 0, 0).  The words (w0, w1, w2, w3) give two uniforms
// u1 = ((w0 >> 6) 2^26 + (w1 >> 6) + 1/2) 2^-52 and u2 likewise from (w2, w3), each exact
// in float64 and inside [2^-53, 1 - 2^-53]; even rows take sqrt(-2 ln u1) cos(2 pi u2),
// odd rows sqrt(-2 ln u1) sin(2 pi u2).  An entry depends on (s, r, c) only, so any column
// range of a block can be drawn on its own and every entry is written by one thread.
#include "wc4d_internal.h"

namespace wc4d {
namespace {

struct Words4 {
  uint32_t w0, w1, w2, w3;
};

__device__ inline Words4 philox4x32_10(Words4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint32_t hi0 = __umulhi(0xD2511F53u, c.w0), lo0 = 0xD2511F53u * c.w0;
    const uint32_t hi1 = __umulhi(0xCD9E8D57u, c.w2), lo1 = 0xCD9E8D57u * c.w2;
    c = Words4{hi1 ^ c.w1 ^ k0, lo1, hi0 ^ c.w3 ^ k1, lo0};
  }
  return c;
}

// uniform in (0, 1) from the top 26 bits of two words; every operation is exact in float64
__device__ inline double uniform52(uint32_t hi, uint32_t lo) {
  return ((double)(hi >> 6) * 67108864.0 + (double)(lo >> 6) + 0.5) * (1.0 / 4503599627370496.0);
}

// in: count x 6 words (c0 c1 c2 c3 k0 k1), out: count x 4 words
__global__ void __launch_bounds__(256) k_philox_words(const uint32_t* __restrict__ in, uint32_t* __restrict__ out,
                                                      long long count) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= count) return;
  const uint32_t* q = in + 6 * t;
  const Words4 w = philox4x32_10(Words4{q[0], q[1], q[2], q[3]}, q[4], q[5]);
  uint32_t* o = out + 4 * t;
  o[0] = w.w0;
  o[1] = w.w1;
  o[2] = w.w2;
  o[3] = w.w3;
}

// One thread per (row pair, column): grid.x over row pairs, grid.y over columns (strided).
__global__ void __launch_bounds__(256) k_gauss_block(uint32_t k0, uint32_t k1, long long nrows, int ncols,
                                                     long long col0, double* __restrict__ G, long long ldg) {
  const long long pair = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long npairs = (nrows + 1) >> 1;
  if (pair >= npairs) return;
  for (int c = blockIdx.y; c < ncols; c += gridDim.y) {
    const long long col = col0 + c;
    const Words4 w = philox4x32_10(Words4{(uint32_t)pair, (uint32_t)col, 0u, 0u}, k0, k1);
    const double u1 = uniform52(w.w0, w.w1), u2 = uniform52(w.w2, w.w3);
    const double rad = sqrt(-2.0 * log(u1));
    const double phi = 6.283185307179586 * u2;  // 2 pi rounded to float64
    double* g = G + (long long)c * ldg + 2 * pair;
    g[0] = rad * cos(phi);
    if (2 * pair + 1 < nrows) g[1] = rad * sin(phi);
  }
}

}  // namespace

hipError_t philox_words(const uint32_t* in, uint32_t* out, long long count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  const long long blocks = (count + 255) / 256;
  k_philox_words<<<dim3((unsigned)blocks), dim3(256), 0, s>>>(in, out, count);
  return hipGetLastError();
}

hipError_t gauss_block(unsigned long long seed, long long nrows, int ncols, long long col0, double* G,
                       long long ldg, hipStream_t s) {
  if (nrows <= 0 || ncols <= 0) return hipSuccess;
  const long long npairs = (nrows + 1) / 2;
  const long long bx = (npairs + 255) / 256;
  const int by = ncols < 65535 ? ncols : 65535;
  k_gauss_block<<<dim3((unsigned)bx, (unsigned)by), dim3(256), 0, s>>>(
      (uint32_t)(seed & 0xFFFFFFFFull), (uint32_t)(seed >> 32), nrows, ncols, col0, G, ldg);
  return hipGetLastError();
}

}  // namespace wc4d
