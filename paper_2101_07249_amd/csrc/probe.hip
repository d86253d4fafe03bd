// Hardware reference for the float64 roofline: a register-only stream of
// v_mfma_f64_16x16x4_f64 (eight independent accumulators per wave, no memory traffic
// until the final store), i.e. the float64 matrix rate the part sustains for a given
// number of waves per SIMD and run length.
#include "abi_common.h"

namespace wc4d {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
constexpr int kPA = 8;  // independent accumulators per wave

__global__ __launch_bounds__(256) void k_mfma_f64_stream(int iters, double* __restrict__ out) {
  d4 acc[kPA];
#pragma unroll
  for (int a = 0; a < kPA; ++a) acc[a] = d4{0.0, 0.0, 0.0, 0.0};
  const double x = 1e-3 * threadIdx.x, y = 1e-3 * blockIdx.x;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int a = 0; a < kPA; ++a) acc[a] = __builtin_amdgcn_mfma_f64_16x16x4f64(x, y, acc[a], 0, 0, 0);
  }
  double s = 0.0;
#pragma unroll
  for (int a = 0; a < kPA; ++a) s += acc[a][0] + acc[a][1] + acc[a][2] + acc[a][3];
  out[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

}  // namespace
}  // namespace wc4d

extern "C" int wc4d_probe_mfma_f64(int device, int waves_per_simd, int iters, int reps, double* tflops) {
  using namespace wc4d;
  if (waves_per_simd < 1 || waves_per_simd > 8 || iters < 1 || reps < 1 || tflops == nullptr) return WC4D_EINVAL;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return WC4D_EINVAL;
  int prev = 0;
  if (hipGetDevice(&prev) != hipSuccess || hipSetDevice(device) != hipSuccess) return WC4D_EHIP;
  int cus = 0;
  hipError_t e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
  const int grid = cus * waves_per_simd;  // 256-thread workgroups: one wave on each SIMD of a CU
  double* out = nullptr;
  hipEvent_t a = nullptr, b = nullptr;
  if (e == hipSuccess) e = hipMalloc((void**)&out, sizeof(double) * (size_t)grid * 256);
  if (e == hipSuccess) e = hipEventCreate(&a);
  if (e == hipSuccess) e = hipEventCreate(&b);
  float ms = 0.f;
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_mfma_f64_stream, dim3(grid), dim3(256), 0, 0, iters, out);  // warm-up
    e = hipDeviceSynchronize();
  }
  if (e == hipSuccess) e = hipEventRecord(a, 0);
  for (int r = 0; r < reps && e == hipSuccess; ++r) {
    hipLaunchKernelGGL(k_mfma_f64_stream, dim3(grid), dim3(256), 0, 0, iters, out);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipEventRecord(b, 0);
  if (e == hipSuccess) e = hipEventSynchronize(b);
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
  if (a) (void)hipEventDestroy(a);
  if (b) (void)hipEventDestroy(b);
  if (out) (void)hipFree(out);
  (void)hipSetDevice(prev);
  if (e != hipSuccess || !(ms > 0.f)) return WC4D_EHIP;
  const double flops = (double)reps * grid * 4.0 * iters * kPA * 2.0 * 16 * 16 * 4;
  *tflops = flops / (ms * 1e-3) / 1e12;
  return WC4D_OK;
}
