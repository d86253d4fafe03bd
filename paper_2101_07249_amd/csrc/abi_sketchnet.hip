// C-ABI entry points of the learned sketch (declared and documented in include/wc4d.h):
// network handle, inference, backward, Adam, the capture loss and the LMP build that
// falls back to the Gaussian block.  Host orchestration only; the arithmetic runs in
// sketchnet.hip and the operator / dense kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "abi_common.h"

using namespace wc4d;

struct wc4d_sketchnet_s {
  int device = 0, layers = 4, nz = 64;
  std::vector<int> cin, cp;      // per layer: input channels, padded to a multiple of 32
  std::vector<size_t> woff;      // per layer offset of W_l in the padded arrays; b_l follows
  size_t npad = 0;               // padded parameter count
  long long nparams = 0;         // parameter count in the ABI order
  float* th = nullptr;           // float32 master parameters (padded layout)
  float* am = nullptr;           // Adam moments
  float* av = nullptr;
  float* grad = nullptr;
  _Float16* w16 = nullptr;       // float16 parameters (padded layout)
  _Float16* wt16 = nullptr;      // layers - 1 backward-data weight blocks (64 x 320)
  int step = 0;
  long long Pcap = 0;
  _Float16* X0 = nullptr;        // P x cp[0]
  std::vector<_Float16*> act;    // layers - 1 hidden activations, P x 64
  _Float16* dha = nullptr;
  _Float16* dhb = nullptr;
  float* part = nullptr;
  size_t partFloats = 0;
  double* red = nullptr;
  float* scal = nullptr;         // {loss scale, 1 / loss scale}
  int lastN = 0, lastT = 0;
  bool haveActs = false;
  double* Gb = nullptr;          // training: G and dG (n_A x 64)
  double* dGb = nullptr;
  long long blkRows = 0;
  double* fdev = nullptr;        // capture loss value
  std::string err;
};

namespace {

constexpr int kNetCH = 64, kNetKW = 5;

int nfail(wc4d_sketchnet net, int code, const std::string& msg) {
  if (net != nullptr) net->err = msg;
  return code;
}

#define NETCHK(net, call)                                                                        \
  do {                                                                                          \
    hipError_t e_ = (call);                                                                     \
    if (e_ != hipSuccess)                                                                       \
      return nfail((net), WC4D_EHIP, std::string(#call) + ": " + hipGetErrorString(e_));         \
  } while (0)

template <class T>
int nalloc(wc4d_sketchnet net, T** ptr, size_t count) {
  if (*ptr != nullptr) {
    (void)hipFree(*ptr);
    *ptr = nullptr;
  }
  if (count == 0) count = 1;
  hipError_t e = hipMalloc((void**)ptr, count * sizeof(T));
  if (e != hipSuccess) {
    *ptr = nullptr;
    return nfail(net, WC4D_ENOMEM, std::string("hipMalloc of ") + std::to_string(count * sizeof(T)) +
                                       " bytes failed: " + hipGetErrorString(e));
  }
  return WC4D_OK;
}

size_t layer_len(const wc4d_sketchnet net, int l) { return (size_t)kNetCH * kNetKW * net->cp[l] + kNetCH; }

// activations and backward buffers for P points
int net_ensure(wc4d_sketchnet net, long long P, int n, int T) {
  int rc;
  if (net->Pcap < P) {
    if ((rc = nalloc(net, &net->X0, (size_t)P * net->cp[0]))) return rc;
    for (auto& a : net->act)
      if ((rc = nalloc(net, &a, (size_t)P * kNetCH))) return rc;
    if ((rc = nalloc(net, &net->dha, (size_t)P * kNetCH))) return rc;
    if ((rc = nalloc(net, &net->dhb, (size_t)P * kNetCH))) return rc;
    net->Pcap = P;
  }
  size_t maxlen = 0;
  for (int l = 0; l < net->layers; ++l) maxlen = std::max(maxlen, layer_len(net, l));
  const size_t need = (size_t)net_wgrad_blocks(n, T) * maxlen;
  if (net->partFloats < need) {
    if ((rc = nalloc(net, &net->part, need))) return rc;
    net->partFloats = need;
  }
  return WC4D_OK;
}

// ABI order (c_out, c_in, t) + bias  <->  padded layout [c_out][t cp + c'] + bias
void to_padded(const wc4d_sketchnet net, const float* src, std::vector<float>& dst) {
  dst.assign(net->npad, 0.f);
  size_t o = 0;
  for (int l = 0; l < net->layers; ++l) {
    const int ci = net->cin[l], cp = net->cp[l];
    float* W = dst.data() + net->woff[l];
    for (int c = 0; c < kNetCH; ++c)
      for (int cc = 0; cc < ci; ++cc)
        for (int t = 0; t < kNetKW; ++t) W[(size_t)c * kNetKW * cp + t * cp + cc] = src[o++];
    float* b = W + (size_t)kNetCH * kNetKW * cp;
    for (int c = 0; c < kNetCH; ++c) b[c] = src[o++];
  }
}

void from_padded(const wc4d_sketchnet net, const std::vector<float>& src, float* dst) {
  size_t o = 0;
  for (int l = 0; l < net->layers; ++l) {
    const int ci = net->cin[l], cp = net->cp[l];
    const float* W = src.data() + net->woff[l];
    for (int c = 0; c < kNetCH; ++c)
      for (int cc = 0; cc < ci; ++cc)
        for (int t = 0; t < kNetKW; ++t) dst[o++] = W[(size_t)c * kNetKW * cp + t * cp + cc];
    const float* b = W + (size_t)kNetCH * kNetKW * cp;
    for (int c = 0; c < kNetCH; ++c) dst[o++] = b[c];
  }
}

// float16 copies of the parameters and the backward-data weights
int refresh_f16(wc4d_sketchnet net, hipStream_t s) {
  NETCHK(net, net_to_f16((long long)net->npad, net->th, net->w16, s));
  for (int l = 1; l < net->layers; ++l)
    NETCHK(net, net_pack_t(net->w16 + net->woff[l], net->wt16 + (size_t)(l - 1) * kNetCH * kNetKW * kNetCH, s));
  return WC4D_OK;
}

int infer_core(wc4d_sketchnet net, wc4d_problem p, const double* Omega, long long ldo, double* G, long long ldg,
               hipStream_t s) {
  const int n = p->n, N = p->N, T = N + 1;
  const long long P = p->nA;
  int rc = net_ensure(net, P, n, T);
  if (rc) return rc;
  double fl = 0.0;
  for (int l = 0; l < net->layers; ++l) fl += 2.0 * (double)P * kNetCH * kNetKW * net->cin[l];
  ProfScope ps(p, s, PROF_NET, 8.0 * (double)P * (net->nz + kNetCH), fl);
  NETCHK(net, net_features(n, N, p->dTraj, p->dObsOff, p->dObsIdx, Omega, ldo, net->nz, net->cp[0], net->X0, s));
  const _Float16* in = net->X0;
  for (int l = 0; l < net->layers; ++l) {
    const _Float16* W = net->w16 + net->woff[l];
    const _Float16* b = W + (size_t)kNetCH * kNetKW * net->cp[l];
    if (l + 1 < net->layers) {
      NETCHK(net, net_conv_hidden(n, T, net->cp[l], in, W, b, net->act[l], s));
      in = net->act[l];
    } else {
      NETCHK(net, net_conv_out(n, T, net->cp[l], in, W, b, G, ldg, s));
    }
  }
  net->lastN = n;
  net->lastT = T;
  net->haveActs = true;
  return WC4D_OK;
}

int backward_core(wc4d_sketchnet net, const double* dG, long long lddg, hipStream_t s) {
  const int n = net->lastN, T = net->lastT;
  const long long P = (long long)n * T;
  const int nb = net_wgrad_blocks(n, T);
  NETCHK(net, net_loss_scale(P, dG, lddg, net->red, net->scal, net->dha, s));
  _Float16* dH = net->dha;
  _Float16* other = net->dhb;
  for (int l = net->layers - 1; l >= 0; --l) {
    const _Float16* X = (l == 0) ? net->X0 : net->act[l - 1];
    NETCHK(net, net_wgrad(n, T, net->cp[l], X, dH, net->part, s));
    NETCHK(net, net_reduce(nb, (int)layer_len(net, l), net->part, net->scal, net->grad + net->woff[l], s));
    if (l > 0) {
      NETCHK(net, net_conv_bwd_data(n, T, dH, net->wt16 + (size_t)(l - 1) * kNetCH * kNetKW * kNetCH,
                                    net->act[l - 1], other, s));
      std::swap(dH, other);
    }
  }
  return WC4D_OK;
}

int adam_core(wc4d_sketchnet net, double lr, hipStream_t s) {
  net->step += 1;
  const double b1 = 0.9, b2 = 0.999;
  const double c1 = 1.0 / (1.0 - std::pow(b1, net->step));
  const double c2 = 1.0 / (1.0 - std::pow(b2, net->step));
  NETCHK(net, net_adam((long long)net->npad, net->th, net->am, net->av, net->grad, (float)lr, (float)b1, (float)b2,
                       1e-8f, (float)c1, (float)c2, net->w16, s));
  for (int l = 1; l < net->layers; ++l)
    NETCHK(net, net_pack_t(net->w16 + net->woff[l], net->wt16 + (size_t)(l - 1) * kNetCH * kNetKW * kNetCH, s));
  return WC4D_OK;
}

// Capture loss (see wc4d_sketch_loss).  Uses the problem's build scratch bufA (Y) and
// bufB (dY), its block workspace and lossWs; dStatus[8] flags a singular S.
int loss_core(wc4d_problem p, const double* G, long long ldg, int m, const double* U, long long ldu,
              const double* theta, int k, double* f, double* dG, long long lddg, hipStream_t s) {
  int rc = ensure_build(p, m);
  if (rc) return rc;
  const size_t mm = (size_t)m * m, km = (size_t)k * m;
  const size_t need = 6 * mm + 3 * km + (size_t)k + 2;
  if (p->lossWsDoubles < need) {
    if ((rc = dev_alloc(p, &p->lossWs, need))) return rc;
    p->lossWsDoubles = need;
  }
  if ((rc = ensure_gram(p, std::max(gram_ws_doubles(m, m, p->nA), gram_ws_doubles(k, m, p->nA))))) return rc;
  double* S = p->lossWs;
  double* Ri = S + mm;
  double* Sinv = Ri + mm;
  double* Tm = Sinv + mm;
  double* tmp = Tm + mm;
  double* M1 = tmp + mm;
  double* V = M1 + mm;
  double* Vw = V + km;
  double* M2 = Vw + km;
  double* w = M2 + km;
  double* sums = w + k;
  const long long nA = p->nA;
  const ColMap cm = plain_cols(nA);
  double* Y = p->bufA;
  double* dY = p->bufB;
  int* st = p->dStatus + 8;
  HIPCHK(p, hipMemsetAsync(st, 0, sizeof(int), s));
  if ((rc = apply_A_core(p, G, ldg, Y, nA, m, nullptr, s))) return rc;
  HIPCHK(p, gram_f64(m, m, nA, Y, cm, Y, cm, S, m, p->wsGram, nullptr, s));
  HIPCHK(p, gram_f64(k, m, nA, U, plain_cols(ldu), Y, cm, V, k, p->wsGram, nullptr, s));
  HIPCHK(p, loss_weights(k, theta, w, sums, s));
  HIPCHK(p, vec_copy(Vw, V, (long long)km, s));
  HIPCHK(p, vec_scale_rows(Vw, k, m, k, w, nullptr, s));
  HIPCHK(p, small_gemm(m, m, k, 1.0, V, k, 1, Vw, k, 0, Tm, m, s));           // T = Y^T P_w Y
  HIPCHK(p, chol_upper(m, S, m, st, s));                                       // S = R^T R
  HIPCHK(p, tri_inv_upper(m, S, m, Ri, m, s));
  HIPCHK(p, small_gemm(m, m, m, 1.0, Ri, m, 0, Ri, m, 1, Sinv, m, s));        // S^{-1} = R^{-1} R^{-T}
  HIPCHK(p, small_gemm(m, m, m, 1.0, Sinv, m, 0, Tm, m, 0, tmp, m, s));
  HIPCHK(p, small_gemm(m, m, m, 1.0, tmp, m, 0, Sinv, m, 0, M1, m, s));       // S^{-1} T S^{-1}
  HIPCHK(p, small_gemm(k, m, m, 1.0, Vw, k, 0, Sinv, m, 0, M2, k, s));        // diag(w) U^T Y S^{-1}
  HIPCHK(p, loss_finish(m, k, Sinv, Tm, sums, f, M1, M2, s));
  HIPCHK(p, gemm_f64((int)nA, m, m, 1.0, Y, nA, M1, plain_cols(m), dY, cm, nullptr, cm, nullptr, s));
  HIPCHK(p, gemm_f64((int)nA, m, k, 1.0, U, ldu, M2, plain_cols(k), dY, cm, dY, cm, nullptr, s));
  return apply_A_core(p, dY, nA, dG, lddg, m, nullptr, s);
}

int loss_status(wc4d_problem p, hipStream_t s) {
  int st = 0;
  HIPCHK(p, hipMemcpyAsync(&st, p->dStatus + 8, sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(p, hipStreamSynchronize(s));
  if (st != 0) return fail(p, WC4D_ENOTSPD, "capture loss: Y^T Y is singular (rank-deficient start block)");
  return WC4D_OK;
}

}  // namespace

extern "C" {

int wc4d_sketchnet_create(wc4d_sketchnet* out, int layers, int channels, int width, int noise_channels,
                          int device) {
  if (out == nullptr) return WC4D_EINVAL;
  *out = nullptr;
  if (layers < 2 || layers > 8 || channels != kNetCH || width != kNetKW || noise_channels < 0 ||
      noise_channels > 92)
    return WC4D_EINVAL;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return WC4D_EINVAL;
  wc4d_sketchnet net = new (std::nothrow) wc4d_sketchnet_s();
  if (net == nullptr) return WC4D_ENOMEM;
  net->device = device;
  net->layers = layers;
  net->nz = noise_channels;
  size_t off = 0;
  long long cnt = 0;
  for (int l = 0; l < layers; ++l) {
    const int ci = (l == 0) ? noise_channels + 4 : kNetCH;
    const int cpl = (ci + 31) / 32 * 32;
    net->cin.push_back(ci);
    net->cp.push_back(cpl);
    net->woff.push_back(off);
    off += (size_t)kNetCH * kNetKW * cpl + kNetCH;
    cnt += (long long)kNetCH * ci * kNetKW + kNetCH;
  }
  net->npad = off;
  net->nparams = cnt;
  net->act.assign(layers - 1, nullptr);
  DevGuard g(device);
  int rc = 0;
  if ((rc = nalloc(net, &net->th, off)) || (rc = nalloc(net, &net->am, off)) || (rc = nalloc(net, &net->av, off)) ||
      (rc = nalloc(net, &net->grad, off)) || (rc = nalloc(net, &net->w16, off)) ||
      (rc = nalloc(net, &net->wt16, (size_t)(layers - 1) * kNetCH * kNetKW * kNetCH)) ||
      (rc = nalloc(net, &net->red, net_scale_ws_doubles())) || (rc = nalloc(net, &net->scal, 2)) ||
      (rc = nalloc(net, &net->fdev, 1))) {
    wc4d_sketchnet_destroy(net);
    return rc;
  }
  std::vector<float> zero(off, 0.f);
  hipError_t e = hipMemcpy(net->th, zero.data(), sizeof(float) * off, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(net->am, zero.data(), sizeof(float) * off, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(net->av, zero.data(), sizeof(float) * off, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(net->grad, zero.data(), sizeof(float) * off, hipMemcpyHostToDevice);
  if (e == hipSuccess && refresh_f16(net, nullptr) != WC4D_OK) e = hipErrorUnknown;
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    wc4d_sketchnet_destroy(net);
    return WC4D_EHIP;
  }
  *out = net;
  return WC4D_OK;
}

int wc4d_sketchnet_destroy(wc4d_sketchnet net) {
  if (net == nullptr) return WC4D_OK;
  DevGuard g(net->device);
  for (void* q : {(void*)net->th, (void*)net->am, (void*)net->av, (void*)net->grad, (void*)net->w16,
                  (void*)net->wt16, (void*)net->X0, (void*)net->dha, (void*)net->dhb, (void*)net->part,
                  (void*)net->red, (void*)net->scal, (void*)net->Gb, (void*)net->dGb, (void*)net->fdev})
    if (q != nullptr) (void)hipFree(q);
  for (auto* a : net->act)
    if (a != nullptr) (void)hipFree(a);
  delete net;
  return WC4D_OK;
}

const char* wc4d_sketchnet_last_error(wc4d_sketchnet net) {
  if (net == nullptr) return "null network handle";
  return net->err.c_str();
}

int wc4d_sketchnet_nparams(wc4d_sketchnet net, long long* count) {
  if (net == nullptr || count == nullptr) return WC4D_EINVAL;
  *count = net->nparams;
  return WC4D_OK;
}

int wc4d_sketchnet_set_params(wc4d_sketchnet net, const float* theta) {
  if (net == nullptr || theta == nullptr) return WC4D_EINVAL;
  DevGuard g(net->device);
  std::vector<float> pad;
  to_padded(net, theta, pad);
  std::vector<float> zero(net->npad, 0.f);
  NETCHK(net, hipMemcpy(net->th, pad.data(), sizeof(float) * net->npad, hipMemcpyHostToDevice));
  NETCHK(net, hipMemcpy(net->am, zero.data(), sizeof(float) * net->npad, hipMemcpyHostToDevice));
  NETCHK(net, hipMemcpy(net->av, zero.data(), sizeof(float) * net->npad, hipMemcpyHostToDevice));
  net->step = 0;
  int rc = refresh_f16(net, nullptr);
  if (rc) return rc;
  NETCHK(net, hipDeviceSynchronize());
  return WC4D_OK;
}

int wc4d_sketchnet_get_params(wc4d_sketchnet net, float* theta) {
  if (net == nullptr || theta == nullptr) return WC4D_EINVAL;
  DevGuard g(net->device);
  NETCHK(net, hipDeviceSynchronize());
  std::vector<float> pad(net->npad);
  NETCHK(net, hipMemcpy(pad.data(), net->th, sizeof(float) * net->npad, hipMemcpyDeviceToHost));
  from_padded(net, pad, theta);
  return WC4D_OK;
}

int wc4d_sketchnet_get_grad(wc4d_sketchnet net, float* grad) {
  if (net == nullptr || grad == nullptr) return WC4D_EINVAL;
  DevGuard g(net->device);
  NETCHK(net, hipDeviceSynchronize());
  std::vector<float> pad(net->npad);
  NETCHK(net, hipMemcpy(pad.data(), net->grad, sizeof(float) * net->npad, hipMemcpyDeviceToHost));
  from_padded(net, pad, grad);
  return WC4D_OK;
}

int wc4d_sketchnet_set_grad(wc4d_sketchnet net, const float* grad) {
  if (net == nullptr || grad == nullptr) return WC4D_EINVAL;
  DevGuard g(net->device);
  std::vector<float> pad;
  to_padded(net, grad, pad);
  NETCHK(net, hipMemcpy(net->grad, pad.data(), sizeof(float) * net->npad, hipMemcpyHostToDevice));
  return WC4D_OK;
}

int wc4d_sketchnet_infer(wc4d_sketchnet net, wc4d_problem p, const double* Omega, int ldo, double* G, int ldg,
                         hipStream_t s) {
  if (net == nullptr) return WC4D_EINVAL;
  if (!is_state_ok(p)) return nfail(net, WC4D_ESTATE, "problem not finalized");
  if (p->strong) return nfail(net, WC4D_EINVAL, "the sketch network serves weak-constraint problems");
  if (p->device != net->device) return nfail(net, WC4D_EINVAL, "network and problem on different devices");
  if ((net->nz > 0 && (Omega == nullptr || ldo < p->nA)) || G == nullptr || ldg < p->nA)
    return nfail(net, WC4D_EINVAL, "invalid Omega / G (null or leading dimension < n_A)");
  DevGuard g(net->device);
  return infer_core(net, p, Omega, ldo, G, ldg, s);
}

int wc4d_sketchnet_backward(wc4d_sketchnet net, const double* dG, int lddg, hipStream_t s) {
  if (net == nullptr) return WC4D_EINVAL;
  if (!net->haveActs) return nfail(net, WC4D_ESTATE, "backward without a preceding inference");
  if (dG == nullptr || lddg < (long long)net->lastN * net->lastT)
    return nfail(net, WC4D_EINVAL, "invalid dG (null or leading dimension < n_A)");
  DevGuard g(net->device);
  return backward_core(net, dG, lddg, s);
}

int wc4d_sketchnet_adam(wc4d_sketchnet net, double lr, hipStream_t s) {
  if (net == nullptr || !(lr >= 0.0) || !std::isfinite(lr)) return WC4D_EINVAL;
  DevGuard g(net->device);
  return adam_core(net, lr, s);
}

int wc4d_sketch_loss(wc4d_problem p, const double* G, int ldg, int m, const double* U, int ldu,
                     const double* theta, int k, double* f, double* dG, int lddg, hipStream_t s) {
  if (!is_state_ok(p)) return p ? fail(p, WC4D_ESTATE, "not finalized") : WC4D_EINVAL;
  if (p->strong) return fail(p, WC4D_EINVAL, "the sketch network serves weak-constraint problems");
  if (G == nullptr || U == nullptr || theta == nullptr || f == nullptr || dG == nullptr || m < 1 || m > 512 ||
      k < 1 || k > 512 || ldg < p->nA || ldu < p->nA || lddg < p->nA || m > p->nA)
    return fail(p, WC4D_EINVAL, "invalid capture-loss arguments");
  DevGuard g(p->device);
  int rc = loss_core(p, G, ldg, m, U, ldu, theta, k, f, dG, lddg, s);
  if (rc) return rc;
  return loss_status(p, s);
}

int wc4d_sketchnet_train_step(wc4d_sketchnet net, wc4d_problem p, const double* Omega, int ldo, wc4d_lmp ref,
                              int k, double lr, double* loss, hipStream_t s) {
  if (net == nullptr) return WC4D_EINVAL;
  if (!is_state_ok(p)) return nfail(net, WC4D_ESTATE, "problem not finalized");
  if (p->strong) return nfail(net, WC4D_EINVAL, "the sketch network serves weak-constraint problems");
  if (ref == nullptr || ref->p != p || k < 1 || k > ref->k)
    return nfail(net, WC4D_EINVAL, "reference LMP must belong to p and hold at least k pairs");
  if (net->nz > 0 && (Omega == nullptr || ldo < p->nA)) return nfail(net, WC4D_EINVAL, "invalid Omega");
  if (!(lr >= 0.0) || !std::isfinite(lr)) return nfail(net, WC4D_EINVAL, "invalid learning rate");
  DevGuard g(net->device);
  int rc;
  if (net->blkRows < p->nA) {
    if ((rc = nalloc(net, &net->Gb, (size_t)p->nA * kNetCH))) return rc;
    if ((rc = nalloc(net, &net->dGb, (size_t)p->nA * kNetCH))) return rc;
    net->blkRows = p->nA;
  }
  if ((rc = infer_core(net, p, Omega, ldo, net->Gb, p->nA, s))) return rc;
  if ((rc = loss_core(p, net->Gb, p->nA, kNetCH, ref->U, ref->ldu, ref->theta, k, net->fdev, net->dGb, p->nA, s)))
    return nfail(net, rc, std::string("capture loss: ") + p->err);
  if ((rc = backward_core(net, net->dGb, p->nA, s))) return rc;
  if ((rc = adam_core(net, lr, s))) return rc;
  if ((rc = loss_status(p, s))) return nfail(net, rc, p->err);
  if (loss != nullptr) NETCHK(net, hipMemcpy(loss, net->fdev, sizeof(double), hipMemcpyDeviceToHost));
  return WC4D_OK;
}

int wc4d_lmp_build_sketch(wc4d_problem p, wc4d_sketchnet net, int method, int k_r, int l, const double* Omega,
                          wc4d_lmp* out, int* used_net, hipStream_t s) {
  if (used_net != nullptr) *used_net = 0;
  if (out == nullptr) return WC4D_EINVAL;
  *out = nullptr;
  if (!is_state_ok(p)) return p ? fail(p, WC4D_ESTATE, "not finalized") : WC4D_EINVAL;
  if (p->strong) return fail(p, WC4D_EINVAL, "the sketch network serves weak-constraint problems");
  if (Omega == nullptr) return fail(p, WC4D_EINVAL, "null Gaussian block");
  if (net == nullptr) return wc4d_lmp_build(p, method, k_r, l, Omega, 0, out, s);
  if (k_r + l != kNetCH || net->nz != kNetCH)
    return fail(p, WC4D_EINVAL, "the learned sketch needs k_r + l = 64 and a network with 64 noise channels");
  DevGuard g(p->device);
  int rc;
  if (net->blkRows < p->nA) {
    if ((rc = nalloc(net, &net->Gb, (size_t)p->nA * kNetCH))) return fail(p, rc, net->err);
    if ((rc = nalloc(net, &net->dGb, (size_t)p->nA * kNetCH))) return fail(p, rc, net->err);
    net->blkRows = p->nA;
  }
  if ((rc = infer_core(net, p, Omega, p->nA, net->Gb, p->nA, s))) return fail(p, rc, net->err);
  rc = wc4d_lmp_build(p, method, k_r, l, net->Gb, 0, out, s);
  if (rc == WC4D_ENOTSPD) return wc4d_lmp_build(p, method, k_r, l, Omega, 0, out, s);
  if (rc == WC4D_OK && used_net != nullptr) *used_net = 1;
  return rc;
}

int wc4d_sketchnet_save(wc4d_sketchnet net, const char* path) {
  if (net == nullptr || path == nullptr) return WC4D_EINVAL;
  std::vector<float> th(net->nparams);
  int rc = wc4d_sketchnet_get_params(net, th.data());
  if (rc) return rc;
  FILE* fp = std::fopen(path, "wb");
  if (fp == nullptr) return nfail(net, WC4D_EINVAL, std::string("cannot open ") + path);
  const int32_t hdr[4] = {net->layers, kNetCH, kNetKW, net->nz};
  const int64_t cnt = net->nparams;
  bool ok = std::fwrite("WC4DSKN1", 1, 8, fp) == 8 && std::fwrite(hdr, sizeof(int32_t), 4, fp) == 4 &&
            std::fwrite(&cnt, sizeof(int64_t), 1, fp) == 1 &&
            std::fwrite(th.data(), sizeof(float), th.size(), fp) == th.size();
  ok = (std::fclose(fp) == 0) && ok;
  return ok ? WC4D_OK : nfail(net, WC4D_EINVAL, std::string("write failed: ") + path);
}

int wc4d_sketchnet_load(wc4d_sketchnet* out, const char* path, int device) {
  if (out == nullptr || path == nullptr) return WC4D_EINVAL;
  *out = nullptr;
  FILE* fp = std::fopen(path, "rb");
  if (fp == nullptr) return WC4D_EINVAL;
  char magic[8];
  int32_t hdr[4];
  int64_t cnt = 0;
  bool ok = std::fread(magic, 1, 8, fp) == 8 && std::memcmp(magic, "WC4DSKN1", 8) == 0 &&
            std::fread(hdr, sizeof(int32_t), 4, fp) == 4 && std::fread(&cnt, sizeof(int64_t), 1, fp) == 1;
  wc4d_sketchnet net = nullptr;
  if (ok && wc4d_sketchnet_create(&net, hdr[0], hdr[1], hdr[2], hdr[3], device) != WC4D_OK) ok = false;
  std::vector<float> th;
  if (ok && cnt != net->nparams) ok = false;
  if (ok) {
    th.resize(cnt);
    ok = std::fread(th.data(), sizeof(float), th.size(), fp) == th.size();
  }
  std::fclose(fp);
  if (ok) {
    for (float v : th)
      if (!std::isfinite(v)) ok = false;
  }
  if (!ok || wc4d_sketchnet_set_params(net, th.data()) != WC4D_OK) {
    wc4d_sketchnet_destroy(net);
    return WC4D_EINVAL;
  }
  *out = net;
  return WC4D_OK;
}

}  // extern "C"
