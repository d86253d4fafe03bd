// LMP application without device allocation, for callers that cannot allocate (code under
// graph capture, tight serving loops, harnesses that forbid hipMalloc).
//
// wc4d_lmp_apply's one- and two-vector passes keep their partial sums of U^T x in a buffer
// the LMP allocates on first use.  This variant runs the same kernels with that buffer in a
// file-scope device array instead: each device the library runs on holds one copy of it
// (4 MiB) until the process ends.  Its address on a device is looked up once, with that
// device current, on the first call there; host code only ever passes that address.
#include <mutex>
#include <vector>

#include "abi_common.h"

namespace wc4d {
namespace {

constexpr size_t kScratchDoubles = size_t(1) << 19;  // 4 MiB per device

static __device__ __align__(256) double scratch[kScratchDoubles];

std::mutex g_scratch_mu;
std::vector<double*> g_scratch_ptr;  // per device: the array's device address (null: not looked up)

// The array's address on the current device `device` (looked up on the first call).
int scratch_on(int device, double** out) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if ((int)g_scratch_ptr.size() <= device) g_scratch_ptr.resize(device + 1, nullptr);
  if (g_scratch_ptr[device] == nullptr) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || ptr == nullptr) return WC4D_EHIP;
    g_scratch_ptr[device] = static_cast<double*>(ptr);
  }
  *out = g_scratch_ptr[device];
  return WC4D_OK;
}

}  // namespace
}  // namespace wc4d

using namespace wc4d;

extern "C" int wc4d_lmp_apply_noalloc(wc4d_lmp L, const double* X, int ldx, double* Y, int ldy, int m,
                                      hipStream_t s) {
  if (L == nullptr) return WC4D_EINVAL;
  wc4d_problem p = L->p;
  if (p == nullptr) return WC4D_ESTATE;
  if (X == nullptr || Y == nullptr || m < 1 || m > 2 || ldx < L->nA || ldy < L->nA)
    return fail(p, WC4D_EINVAL, "lmp_apply_noalloc: one or two vectors, ld >= n_A, non-null pointers");
  const char* xb = (const char*)X;
  const char* yb = (const char*)Y;
  const size_t xs = sizeof(double) * ((size_t)ldx * (m - 1) + L->nA);
  const size_t ys = sizeof(double) * ((size_t)ldy * (m - 1) + L->nA);
  if (xb < yb + ys && yb < xb + xs) return fail(p, WC4D_EINVAL, "lmp_apply_noalloc: X and Y overlap");
  const size_t need = lmp_gemv_ws_doubles(L->nA, L->k);
  if (need > kScratchDoubles)
    return fail(p, WC4D_EINVAL, "lmp_apply_noalloc: the LMP needs " + std::to_string(need) +
                                    " doubles of scratch, more than the fixed " + std::to_string(kScratchDoubles));
  DevGuard g(p->device);
  double* ws = nullptr;
  if (scratch_on(p->device, &ws) != WC4D_OK) return fail(p, WC4D_EHIP, "lmp_apply_noalloc: scratch lookup failed");
  const LmpU Us = L->streamed();
  for (int c = 0; c < m; ++c) {
    HIPCHK(p, lmp_gemv_t(L->nA, L->k, Us, L->dcoef, X + (size_t)c * ldx, ws, nullptr, s));
    HIPCHK(p, lmp_gemv_n(L->nA, L->k, Us, X + (size_t)c * ldx, Y + (size_t)c * ldy, ws, nullptr, s));
  }
  return WC4D_OK;
}
