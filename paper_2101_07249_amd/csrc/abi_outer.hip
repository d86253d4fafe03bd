// C-ABI entry points of the outer loop's preconditioner from the previous inner loop
// (declared and documented in include/wc4d.h): Ritz pairs from the Lanczos information
// CG gathers (Section 3.4) and a spectral LMP from given Ritz pairs (Section 3.2, eq.
// spectral_LMP_factor), so that pairs found on one inner loop's Hessian precondition the
// next.  Host orchestration; the arithmetic runs in the dense and GEMM kernels.
#include <hip/hip_runtime.h>

#include <cmath>
#include <new>
#include <string>
#include <vector>

#include "abi_common.h"

using namespace wc4d;

extern "C" {

int wc4d_lanczos_pairs(wc4d_problem p, int j, const double* alphas, const double* betas, const double* F,
                       long long ldf, int k, double* U, long long ldu, double* theta, hipStream_t s) {
  if (!is_state_ok(p)) return p ? fail(p, WC4D_ESTATE, "not finalized") : WC4D_EINVAL;
  if (j < 1 || j > 512 || k < 1 || k > j || alphas == nullptr || betas == nullptr || F == nullptr ||
      U == nullptr || theta == nullptr || ldf < p->nA || ldu < p->nA)
    return fail(p, WC4D_EINVAL, "lanczos_pairs: 1 <= k <= j <= 512, ldf and ldu >= n_A, non-null arrays");
  for (int i = 0; i < j; ++i)
    if (!(alphas[i] > 0.0) || !(betas[i] >= 0.0) || !std::isfinite(alphas[i]) || !std::isfinite(betas[i]))
      return fail(p, WC4D_EINVAL, "lanczos_pairs: CG coefficients must be finite, alpha > 0, beta >= 0");
  DevGuard g(p->device);
  // T_j (Section 3.4): gamma_1 = 1/alpha_1, gamma_i = 1/alpha_i + beta_{i-1}/alpha_{i-1},
  // tau_i = sqrt(beta_i)/alpha_i; column-major j x j
  std::vector<double> T((size_t)j * j, 0.0);
  for (int i = 0; i < j; ++i) {
    T[(size_t)i * j + i] = 1.0 / alphas[i] + (i > 0 ? betas[i - 1] / alphas[i - 1] : 0.0);
    if (i + 1 < j) {
      const double t = std::sqrt(betas[i]) / alphas[i];
      T[(size_t)(i + 1) * j + i] = t;
      T[(size_t)i * j + i + 1] = t;
    }
  }
  double* buf = nullptr;
  int* ctrl = nullptr;
  int rc = dev_alloc(p, &buf, (size_t)2 * j * j + j);
  if (rc == WC4D_OK) rc = dev_alloc(p, &ctrl, 2);
  if (rc != WC4D_OK) {
    dev_free(&buf);
    return rc;
  }
  double* dT = buf;
  double* dV = buf + (size_t)j * j;
  double* dlam = buf + (size_t)2 * j * j;
  auto done = [&](int code) {
    (void)hipStreamSynchronize(s);
    dev_free(&buf);
    dev_free(&ctrl);
    return code;
  };
  hipError_t e = hipMemcpyAsync(dT, T.data(), sizeof(double) * T.size(), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = jacobi_evd(j, dT, j, dlam, dV, j, ctrl, s, true);
  // Ritz vectors u_i = F_j w_i for the k largest Ritz values
  if (e == hipSuccess)
    e = gemm_f64((int)p->nA, k, j, 1.0, F, ldf, dV, plain_cols(j), U, plain_cols(ldu), nullptr, plain_cols(ldu),
                 nullptr, s);
  int conv = 0;
  if (e == hipSuccess) e = hipMemcpyAsync(theta, dlam, sizeof(double) * k, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipMemcpyAsync(&conv, ctrl, sizeof(int), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return done(fail(p, WC4D_EHIP, hipGetErrorString(e)));
  if (conv == 0) return done(fail(p, WC4D_ENOCONV, "lanczos_pairs: Jacobi EVD of T_j did not converge"));
  return done(WC4D_OK);
}

int wc4d_lmp_from_pairs(wc4d_problem p, int k, const double* U, long long ldu, const double* theta,
                        wc4d_lmp* out, hipStream_t s) {
  if (out == nullptr) return WC4D_EINVAL;
  *out = nullptr;
  if (!is_state_ok(p)) return p ? fail(p, WC4D_ESTATE, "not finalized") : WC4D_EINVAL;
  if (k < 1 || k > 512 || U == nullptr || theta == nullptr || ldu < p->nA)
    return fail(p, WC4D_EINVAL, "lmp_from_pairs: 1 <= k <= 512, ldu >= n_A, non-null U and theta");
  for (int i = 0; i < k; ++i)
    if (!(theta[i] > 0.0) || !std::isfinite(theta[i]))
      return fail(p, WC4D_EINVAL, "lmp_from_pairs: Ritz values must be positive and finite");
  DevGuard g(p->device);
  wc4d_lmp L = new (std::nothrow) wc4d_lmp_s();
  if (L == nullptr) return WC4D_ENOMEM;
  L->p = p;
  p->lmps.push_back(L);
  L->nA = p->nA;
  L->ldu = (p->nA + 3) / 4 * 4;
  L->k = k;
  L->applies = 0;
  auto cleanup = [&](int code) {
    wc4d_lmp_destroy(L);
    return code;
  };
  int rc;
  if ((rc = dev_alloc(p, &L->U, (size_t)L->ldu * k))) return cleanup(rc);
  if ((rc = dev_alloc(p, &L->theta, k))) return cleanup(rc);
  if ((rc = dev_alloc(p, &L->dcoef, k))) return cleanup(rc);
  if ((rc = dev_alloc(p, &L->GU, (size_t)k * k))) return cleanup(rc);
  if ((rc = dev_alloc(p, &L->fu, (size_t)3 * k))) return cleanup(rc);
  if ((rc = ensure_gram(p, gram_ws_doubles(k, k, p->nA)))) return cleanup(rc);
  hipError_t e = hipMemcpy2DAsync(L->U, sizeof(double) * L->ldu, U, sizeof(double) * ldu, sizeof(double) * p->nA, k,
                                  hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(L->theta, theta, sizeof(double) * k, hipMemcpyHostToDevice, s);
  // theta as given; dcoef = theta^{-1/2} - 1 (the LMP's diagonal)
  if (e == hipSuccess) e = ritz_finish(k, L->theta, 0, L->theta, L->dcoef, s);
  // U^T U for the fused PCG recursion (the identity for orthonormal pairs)
  if (e == hipSuccess)
    e = gram_f64(k, k, p->nA, L->U, plain_cols(L->ldu), L->U, plain_cols(L->ldu), L->GU, k, p->wsGram, nullptr, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return cleanup(fail(p, WC4D_EHIP, hipGetErrorString(e)));
  *out = L;
  return WC4D_OK;
}

}  // extern "C"
