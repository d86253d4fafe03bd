// C-ABI entry points of libwc4d (declared and documented in include/wc4d.h).
// Host orchestration only: every step of the operator, the randomised
// eigendecompositions, the LMP and PCG runs in this library's HIP kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "abi_common.h"

using namespace wc4d;

namespace {

constexpr int kVersion = 100;  // 0.1.0

int prof_collect(wc4d_problem p) {
  if (p->recs.empty()) return WC4D_OK;
  hipError_t e = hipEventSynchronize(p->recs.back().b);
  if (e != hipSuccess) return fail(p, WC4D_EHIP, hipGetErrorString(e));
  for (const ProfRec& r : p->recs) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) continue;
    p->profMs[r.cls] += ms;
    p->profBytes[r.cls] += r.bytes;
    p->profFlops[r.cls] += r.flops;
    p->profCalls[r.cls] += 1;
  }
  p->recs.clear();
  p->evnext = 0;
  return WC4D_OK;
}

// L96 tendency (Section 5.2, eq. lorenz96) on the host, for the trajectory helper
// and the RK4 stage inputs uploaded at finalize.
void l96_f(const double* x, double* f, int n, double F) {
  for (int j = 0; j < n; ++j) {
    const double xm2 = x[(j - 2 + n) % n], xm1 = x[(j - 1 + n) % n], xp1 = x[(j + 1) % n];
    f[j] = (xp1 - xm2) * xm1 - x[j] + F;
  }
}

void l96_stage_inputs(const double* x, int n, double F, double dt, double* y /* 4 n */) {
  std::vector<double> k(n), tmp(n);
  std::memcpy(y, x, sizeof(double) * n);
  l96_f(x, k.data(), n, F);
  for (int j = 0; j < n; ++j) y[n + j] = x[j] + 0.5 * dt * k[j];
  l96_f(y + n, k.data(), n, F);
  for (int j = 0; j < n; ++j) y[2 * n + j] = x[j] + 0.5 * dt * k[j];
  l96_f(y + 2 * n, k.data(), n, F);
  for (int j = 0; j < n; ++j) y[3 * n + j] = x[j] + dt * k[j];
}

}  // namespace

wc4d::SweepModel wc4d_problem_s::sweep() const {
  SweepModel md{};
  md.kind = model;
  md.n = n;
  md.N = N;
  md.ca = c + r;
  md.cb = 1.0 - c - 2.0 * r;
  md.cc = r;
  md.dt = dt;
  md.stages = dStages;
  md.obs_off = dObsOff;
  md.obs_idx = dObsIdx;
  md.obs_rinv = dObsRinv;
  md.tw_pe = twPe;
  md.tw_W = twW;
  md.tw_e = dTwE;
  md.tw_dummy = dTwDummy;
  return md;
}

extern "C" {

int wc4d_version(void) { return kVersion; }

const char* wc4d_status_string(int st) {
  switch (st) {
    case WC4D_OK: return "WC4D_OK";
    case WC4D_EINVAL: return "WC4D_EINVAL";
    case WC4D_ENOMEM: return "WC4D_ENOMEM";
    case WC4D_EHIP: return "WC4D_EHIP";
    case WC4D_ENOTSPD: return "WC4D_ENOTSPD";
    case WC4D_EBREAKDOWN: return "WC4D_EBREAKDOWN";
    case WC4D_ENOCONV: return "WC4D_ENOCONV";
    case WC4D_ESTATE: return "WC4D_ESTATE";
    default: return "unknown status";
  }
}

int wc4d_create(wc4d_problem* out, int n, int N, int device) {
  if (out == nullptr) return WC4D_EINVAL;
  *out = nullptr;
  if (n < 1 || N < 1) return WC4D_EINVAL;
  if ((long long)n * (N + 1) > (1LL << 31) - 1) return WC4D_EINVAL;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return WC4D_EINVAL;
  wc4d_problem p = new (std::nothrow) wc4d_problem_s();
  if (p == nullptr) return WC4D_ENOMEM;
  p->n = n;
  p->N = N;
  p->device = device;
  p->nA = (long long)n * (N + 1);
  p->nL = p->nA;
  p->obs_idx.assign(N + 1, {});
  p->obs_r.assign(N + 1, {});
  *out = p;
  return WC4D_OK;
}

int wc4d_destroy(wc4d_problem p) {
  if (p == nullptr) return WC4D_OK;
  DevGuard g(p->device);
  // LMPs still alive lose their device memory; their handles stay valid for
  // wc4d_lmp_destroy and every other call on them returns WC4D_ESTATE
  for (wc4d_lmp L : p->lmps) {
    lmp_release(L);
    L->p = nullptr;
  }
  p->lmps.clear();
  dev_free(&p->dB);
  dev_free(&p->dQ);
  dev_free(&p->ozSs);
  dev_free(&p->ozEs);
  dev_free(&p->ozXs);
  dev_free(&p->ozFs);
  dev_free(&p->ozP);
  dev_free(&p->dBhi);
  dev_free(&p->dBh16);
  dev_free(&p->dBl16);
  dev_free(&p->dQh16);
  dev_free(&p->dQl16);
  dev_free(&p->dBexp);
  dev_free(&p->dQexp);
  dev_free(&p->dColExp);
  dev_free(&p->dBlo);
  dev_free(&p->dQhi);
  dev_free(&p->dQlo);
  dev_free(&p->dQf);
  dev_free(&p->dQf16);
  dev_free(&p->dXf);
  p->xfCap = 0;
  dev_free(&p->dStages);
  dev_free(&p->dTraj);
  dev_free(&p->lossWs);
  dev_free(&p->dObsOff);
  dev_free(&p->dObsIdx);
  dev_free(&p->dObsRinv);
  dev_free(&p->dTwE);
  dev_free(&p->dTwDummy);
  dev_free(&p->wsBlock);
  dev_free(&p->wsStash);
  dev_free(&p->wsGram);
  dev_free(&p->wsSplit);

  dev_free(&p->bufA);
  dev_free(&p->bufB);
  dev_free(&p->small);
  dev_free(&p->dStatus);
  dev_free(&p->pcgVec);
  dev_free(&p->pcgHist);
  dev_free(&p->pcgRed);
  dev_free(&p->pcgState);
  if (p->pcgStateHost != nullptr) (void)hipHostFree(p->pcgStateHost);
  for (int q = 0; q < 2; ++q) {
    if (p->pcgPoll[q] != nullptr) (void)hipHostFree(p->pcgPoll[q]);
    if (p->pcgPollEv[q] != nullptr) (void)hipEventDestroy(p->pcgPollEv[q]);
    if (p->evdPoll.host[q] != nullptr) (void)hipHostFree(p->evdPoll.host[q]);
    if (p->evdPoll.ev[q] != nullptr) (void)hipEventDestroy(p->evdPoll.ev[q]);
  }
  for (auto& e : p->ev)
    if (e != nullptr) (void)hipEventDestroy(e);
  for (auto& e : p->evpool) (void)hipEventDestroy(e);
  delete p;
  return WC4D_OK;
}

const char* wc4d_last_error(wc4d_problem p) {
  if (p == nullptr) return "null problem handle";
  return p->err.c_str();
}

int wc4d_set_model_advdiff(wc4d_problem p, double c, double r) {
  if (p == nullptr) return WC4D_EINVAL;
  if (p->finalized) return fail(p, WC4D_ESTATE, "setup after finalize");
  if (!(c >= 0.0) || !(r >= 0.0) || !(c + 2.0 * r <= 1.0))
    return fail(p, WC4D_EINVAL, "advection-diffusion needs c >= 0, r >= 0, c + 2r <= 1");
  p->model = 0;
  p->c = c;
  p->r = r;
  return WC4D_OK;
}

int wc4d_set_model_l96(wc4d_problem p, const double* traj, double F, double dt) {
  if (p == nullptr) return WC4D_EINVAL;
  if (p->finalized) return fail(p, WC4D_ESTATE, "setup after finalize");
  if (traj == nullptr || p->n < 4 || !(dt > 0.0) || !std::isfinite(F))
    return fail(p, WC4D_EINVAL, "Lorenz-96 needs a trajectory, n >= 4 and dt > 0");
  p->model = 1;
  p->F = F;
  p->dt = dt;
  p->traj.assign(traj, traj + (size_t)(p->N + 1) * p->n);
  return WC4D_OK;
}

int wc4d_l96_trajectory(int n, int N, double F, double dt, const double* x0, double* traj) {
  return wc4d_l96_trajectory_forced(n, N, F, dt, x0, nullptr, traj);
}

int wc4d_l96_trajectory_forced(int n, int N, double F, double dt, const double* x0, const double* eta,
                               double* traj) {
  if (n < 4 || N < 0 || x0 == nullptr || traj == nullptr || !(dt > 0.0)) return WC4D_EINVAL;
  std::vector<double> k1(n), k2(n), k3(n), k4(n), y(n);
  std::memcpy(traj, x0, sizeof(double) * n);
  for (int i = 0; i < N; ++i) {
    const double* x = traj + (size_t)i * n;
    double* xn = traj + (size_t)(i + 1) * n;
    l96_f(x, k1.data(), n, F);
    for (int j = 0; j < n; ++j) y[j] = x[j] + 0.5 * dt * k1[j];
    l96_f(y.data(), k2.data(), n, F);
    for (int j = 0; j < n; ++j) y[j] = x[j] + 0.5 * dt * k2[j];
    l96_f(y.data(), k3.data(), n, F);
    for (int j = 0; j < n; ++j) y[j] = x[j] + dt * k3[j];
    l96_f(y.data(), k4.data(), n, F);
    for (int j = 0; j < n; ++j) xn[j] = x[j] + (dt / 6.0) * (k1[j] + 2.0 * k2[j] + 2.0 * k3[j] + k4[j]);
    if (eta != nullptr)
      for (int j = 0; j < n; ++j) xn[j] += eta[(size_t)i * n + j];
  }
  return WC4D_OK;
}

int wc4d_corr_sqrt(int n, int kind, double L, double sigma, double* out) {
  if (n < 1 || out == nullptr || !(L > 0.0) || !(sigma >= 0.0)) return WC4D_EINVAL;
  if (kind != WC4D_CORR_SOAR && kind != WC4D_CORR_GAUSS) return WC4D_EINVAL;
  const double pi = 3.14159265358979323846;
  // first column of the circulant correlation matrix
  std::vector<double> c(n), ct(n), lam(n), s(n);
  for (int d = 0; d < n; ++d) {
    const double dist = (n / pi) * std::sin(pi * d / n);
    c[d] = (kind == WC4D_CORR_SOAR) ? (1.0 + dist / L) * std::exp(-dist / L)
                                    : std::exp(-(dist * dist) / (2.0 * L * L));
    ct[d] = std::cos(2.0 * pi * d / n);
  }
  // real spectrum lambda_k = sum_d c_d cos(2 pi k d / n)
  double lmax = 0.0;
  for (int k = 0; k < n; ++k) {
    double acc = 0.0;
    for (int d = 0; d < n; ++d) acc += c[d] * ct[(int)(((long long)k * d) % n)];
    lam[k] = acc;
    lmax = std::max(lmax, acc);
  }
  for (int k = 0; k < n; ++k) {
    if (lam[k] < -1e-10 * lmax) return WC4D_ENOTSPD;
    lam[k] = std::sqrt(std::max(lam[k], 0.0));
  }
  // first column of the root: s_d = (1/n) sum_k sqrt(lambda_k) cos(2 pi k d / n)
  for (int d = 0; d < n; ++d) {
    double acc = 0.0;
    for (int k = 0; k < n; ++k) acc += lam[k] * ct[(int)(((long long)k * d) % n)];
    s[d] = sigma * acc / n;
  }
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i) out[i + (size_t)j * n] = s[(i - j + n) % n];
  return WC4D_OK;
}

int wc4d_set_Bsqrt(wc4d_problem p, const double* B) {
  if (p == nullptr) return WC4D_EINVAL;
  if (p->finalized) return fail(p, WC4D_ESTATE, "setup after finalize");
  if (B == nullptr) return fail(p, WC4D_EINVAL, "null B^{1/2}");
  p->Bsqrt.assign(B, B + (size_t)p->n * p->n);
  p->haveB = true;
  return WC4D_OK;
}

int wc4d_set_Qsqrt(wc4d_problem p, const double* Q) {
  if (p == nullptr) return WC4D_EINVAL;
  if (p->finalized) return fail(p, WC4D_ESTATE, "setup after finalize");
  if (Q == nullptr) return fail(p, WC4D_EINVAL, "null Q^{1/2}");
  p->Qsqrt.assign(Q, Q + (size_t)p->n * p->n);
  p->haveQ = true;
  return WC4D_OK;
}

int wc4d_set_obs(wc4d_problem p, int i, int q_i, const int* idx, const double* rdiag) {
  if (p == nullptr) return WC4D_EINVAL;
  if (p->finalized) return fail(p, WC4D_ESTATE, "setup after finalize");
  if (i < 0 || i > p->N || q_i < 0 || q_i > p->n || (q_i > 0 && (idx == nullptr || rdiag == nullptr)))
    return fail(p, WC4D_EINVAL, "invalid observation time, count or pointers");
  std::vector<char> seen(p->n, 0);
  for (int k = 0; k < q_i; ++k) {
    if (idx[k] < 0 || idx[k] >= p->n) return fail(p, WC4D_EINVAL, "observation index out of range");
    if (seen[idx[k]]) return fail(p, WC4D_EINVAL, "repeated observation index in one time level");
    seen[idx[k]] = 1;
    if (!(rdiag[k] > 0.0) || !std::isfinite(rdiag[k]))
      return fail(p, WC4D_EINVAL, "observation error variance must be positive");
  }
  p->obs_idx[i].assign(idx, idx + q_i);
  p->obs_r[i].assign(rdiag, rdiag + q_i);
  return WC4D_OK;
}

int wc4d_set_strong_constraint(wc4d_problem p, int on) {
  if (p == nullptr) return WC4D_EINVAL;
  if (p->finalized) return fail(p, WC4D_ESTATE, "set_strong_constraint: already finalized");
  p->strong = on != 0;
  p->nA = p->strong ? (long long)p->n : p->nL;
  return WC4D_OK;
}

int wc4d_finalize(wc4d_problem p, int prec_mode, hipStream_t s) {
  if (p == nullptr) return WC4D_EINVAL;
  if (p->finalized) return fail(p, WC4D_ESTATE, "already finalized");
  if (p->model < 0) return fail(p, WC4D_ESTATE, "no model set");
  if (p->strong && p->haveB && !p->haveQ) {
    // no model error: Q^{1/2} is never applied
    p->Qsqrt.assign((size_t)p->n * p->n, 0.0);
    p->haveQ = true;
  }
  if (!p->haveB || !p->haveQ) return fail(p, WC4D_ESTATE, "B^{1/2} and Q^{1/2} must be set");
  if (p->strong && (prec_mode & (WC4D_PREC_SKETCH_BF16X3 | WC4D_PREC_SKETCH_FP16X3)))
    return fail(p, WC4D_EINVAL, "strong-constraint problems take float64 products only");
  if (prec_mode & ~(WC4D_PREC_SKETCH_BF16X3 | WC4D_PREC_LMP_FP32 | WC4D_PREC_SKETCH_FP16X3 | WC4D_PREC_LMP_FP16 |
                    WC4D_PREC_DSQRT_OZ7))
    return fail(p, WC4D_EINVAL, "unknown precision flags");
  if (p->strong && (prec_mode & WC4D_PREC_DSQRT_OZ7))
    return fail(p, WC4D_EINVAL, "strong-constraint problems take float64 products only");
  if ((prec_mode & WC4D_PREC_LMP_FP32) && (prec_mode & WC4D_PREC_LMP_FP16))
    return fail(p, WC4D_EINVAL, "WC4D_PREC_LMP_FP32 and WC4D_PREC_LMP_FP16 exclude each other");
  if ((prec_mode & WC4D_PREC_SKETCH_BF16X3) && (prec_mode & WC4D_PREC_SKETCH_FP16X3))
    return fail(p, WC4D_EINVAL, "WC4D_PREC_SKETCH_BF16X3 and WC4D_PREC_SKETCH_FP16X3 exclude each other");
  DevGuard g(p->device);
  const int n = p->n, N = p->N;
  std::vector<int> off(N + 2, 0), idx;
  std::vector<double> rinv;
  for (int i = 0; i <= N; ++i) {
    off[i + 1] = off[i] + (int)p->obs_idx[i].size();
    for (size_t k = 0; k < p->obs_idx[i].size(); ++k) {
      idx.push_back(p->obs_idx[i][k]);
      rinv.push_back(1.0 / p->obs_r[i][k]);
    }
  }
  p->q = off[N + 1];
  int rc;
  if ((rc = dev_alloc(p, &p->dB, (size_t)n * n))) return rc;
  if ((rc = dev_alloc(p, &p->dQ, (size_t)n * n))) return rc;
  if ((rc = dev_alloc(p, &p->dObsOff, off.size()))) return rc;
  if ((rc = dev_alloc(p, &p->dObsIdx, std::max<size_t>(idx.size(), 1)))) return rc;
  if ((rc = dev_alloc(p, &p->dObsRinv, std::max<size_t>(rinv.size(), 1)))) return rc;
  HIPCHK(p, hipMemcpyAsync(p->dB, p->Bsqrt.data(), sizeof(double) * n * n, hipMemcpyHostToDevice, s));
  HIPCHK(p, hipMemcpyAsync(p->dQ, p->Qsqrt.data(), sizeof(double) * n * n, hipMemcpyHostToDevice, s));
  HIPCHK(p, hipMemcpyAsync(p->dObsOff, off.data(), sizeof(int) * off.size(), hipMemcpyHostToDevice, s));
  if (!idx.empty()) {
    HIPCHK(p, hipMemcpyAsync(p->dObsIdx, idx.data(), sizeof(int) * idx.size(), hipMemcpyHostToDevice, s));
    HIPCHK(p, hipMemcpyAsync(p->dObsRinv, rinv.data(), sizeof(double) * rinv.size(), hipMemcpyHostToDevice, s));
  }
  // per-wavefront observation slots of the single-wave advection-diffusion sweeps
  int twPe = 0, twW = 0;
  std::vector<wc4d::TwEntry> went;
  if (p->model == 0 && tw_setup(n, N, off, idx, rinv, &twPe, &twW, went)) {
    if ((rc = dev_alloc(p, &p->dTwE, went.size()))) return rc;
    if ((rc = dev_alloc(p, &p->dTwDummy, 2))) return rc;  // 16 bytes: a double2 store target
    HIPCHK(p, hipMemcpyAsync(p->dTwE, went.data(), sizeof(TwEntry) * went.size(), hipMemcpyHostToDevice, s));
    p->twPe = twPe;
    p->twW = twW;
  }
  std::vector<double> stages;
  if (p->model == 1) {
    stages.resize((size_t)N * 4 * n);
    for (int i = 0; i < N; ++i)
      l96_stage_inputs(p->traj.data() + (size_t)i * n, n, p->F, p->dt, stages.data() + (size_t)i * 4 * n);
    if ((rc = dev_alloc(p, &p->dStages, stages.size()))) return rc;
    HIPCHK(p, hipMemcpyAsync(p->dStages, stages.data(), sizeof(double) * stages.size(), hipMemcpyHostToDevice, s));
    if ((rc = dev_alloc(p, &p->dTraj, p->traj.size()))) return rc;
    HIPCHK(p, hipMemcpyAsync(p->dTraj, p->traj.data(), sizeof(double) * p->traj.size(), hipMemcpyHostToDevice, s));
  }
  // LDS the sweeps need must fit the device
  int maxLds = 0;
  HIPCHK(p, hipDeviceGetAttribute(&maxLds, hipDeviceAttributeMaxSharedMemoryPerBlock, p->device));
  const size_t need = sweep_lds_required(p->sweep());
  if (need > (size_t)maxLds)
    return fail(p, WC4D_EINVAL, "state too large for the sweep's LDS (" + std::to_string(need) +
                                    " > " + std::to_string(maxLds) + " bytes)");
  if (prec_mode & WC4D_PREC_SKETCH_BF16X3) {
    const size_t nn = (size_t)n * n;
    if ((rc = dev_alloc(p, &p->dBhi, nn)) || (rc = dev_alloc(p, &p->dBlo, nn)) ||
        (rc = dev_alloc(p, &p->dQhi, nn)) || (rc = dev_alloc(p, &p->dQlo, nn)))
      return rc;
    HIPCHK(p, split_bf16_rows(n, n, p->dB, n, p->dBhi, p->dBlo, s));
    HIPCHK(p, split_bf16_rows(n, n, p->dQ, n, p->dQhi, p->dQlo, s));
    if ((rc = dev_alloc(p, &p->dQf, bf16_frag_elems(n, n)))) return rc;
    HIPCHK(p, split_frag_set_lds_limit());
    HIPCHK(p, split_bf16_frag_rows(n, n, p->dQ, n, p->dQf, s));
  }
  if (prec_mode & WC4D_PREC_SKETCH_FP16X3) {
    const size_t nn = (size_t)n * n;
    if ((rc = dev_alloc(p, &p->dBh16, nn)) || (rc = dev_alloc(p, &p->dBl16, nn)) ||
        (rc = dev_alloc(p, &p->dQh16, nn)) || (rc = dev_alloc(p, &p->dQl16, nn)) ||
        (rc = dev_alloc(p, &p->dBexp, (size_t)n)) || (rc = dev_alloc(p, &p->dQexp, (size_t)n)))
      return rc;
    HIPCHK(p, split_f16_rows(n, n, p->dB, n, p->dBh16, p->dBl16, p->dBexp, s));
    HIPCHK(p, split_f16_rows(n, n, p->dQ, n, p->dQh16, p->dQl16, p->dQexp, s));
    if ((rc = dev_alloc(p, &p->dQf16, bf16_frag_elems(n, n)))) return rc;
    HIPCHK(p, split_frag_set_lds_limit());
    HIPCHK(p, split_f16_frag_rows(n, n, p->dQ, n, p->dQexp, p->dQf16, s));
  }
  if ((rc = dev_alloc(p, &p->dStatus, 16))) return rc;
  // split-K partials: up to 512 workgroups' worth of n x 112 tiles
  p->wsSplitDoubles = std::min<size_t>((size_t)8 * n * (112 + 2), (size_t)1 << 24);
  if ((rc = dev_alloc(p, &p->wsSplit, p->wsSplitDoubles))) return rc;

  HIPCHK(p, hipMemsetAsync(p->dStatus, 0, 16 * sizeof(int), s));
  HIPCHK(p, hipStreamSynchronize(s));
  // B^{1/2} = c Q^{1/2} (the same correlation with another variance): then D^{1/2} is one
  // product with Q^{1/2} over all N + 1 time levels and a scaling of level 0
  {
    // c from the entry of largest |Q^{1/2}| (one rounding), then every entry checked
    size_t emax = 0;
    double bmax = 0.0, qmax = 0.0;
    for (size_t e = 0; e < (size_t)n * n; ++e) {
      bmax = std::max(bmax, std::fabs(p->Bsqrt[e]));
      if (std::fabs(p->Qsqrt[e]) > qmax) {
        qmax = std::fabs(p->Qsqrt[e]);
        emax = e;
      }
    }
    p->scaledB = false;
    if (qmax > 0.0 && bmax > 0.0) {
      const double c = p->Bsqrt[emax] / p->Qsqrt[emax];
      double dev = 0.0;
      for (size_t e = 0; e < (size_t)n * n && dev <= 1e-13 * bmax; ++e)
        dev = std::max(dev, std::fabs(p->Bsqrt[e] - c * p->Qsqrt[e]));
      if (dev <= 1e-13 * bmax && c > 0.0) {
        p->scaledB = true;
        p->bScale = c;
      }
    }
  }
  if (prec_mode & WC4D_PREC_DSQRT_OZ7) {
    // int8 slices of Q^{1/2} for the one-vector products (all levels in one product)
    if (!p->scaledB)
      return fail(p, WC4D_EINVAL, "WC4D_PREC_DSQRT_OZ7 needs B^{1/2} = c Q^{1/2} (one product over all levels)");
    const int L = N + 1;
    if ((rc = dev_alloc(p, &p->ozSs, oz_slices_bytes(n))) || (rc = dev_alloc(p, &p->ozEs, (size_t)oz_padded(n))) ||
        (rc = dev_alloc(p, &p->ozXs, oz_xs_bytes(n, L))) || (rc = dev_alloc(p, &p->ozFs, (size_t)oz_lpad(L))) ||
        (rc = dev_alloc(p, &p->ozP, oz_partials_doubles(n, L))))
      return rc;
    HIPCHK(p, oz_set_lds_limit());
    HIPCHK(p, oz_split_matrix(p->dQ, n, n, p->ozSs, p->ozEs, s));
    HIPCHK(p, hipStreamSynchronize(s));
  }
  // the host copies of the square roots are no longer needed once uploaded
  std::vector<double>().swap(p->Bsqrt);
  std::vector<double>().swap(p->Qsqrt);
  p->prec = prec_mode;
  p->finalized = true;
  return WC4D_OK;
}

int wc4d_dims(wc4d_problem p, int* nA, int* q) {
  if (!is_state_ok(p)) return p ? fail(p, WC4D_ESTATE, "not finalized") : WC4D_EINVAL;
  if (nA) *nA = (int)p->nA;
  if (q) *q = p->q;
  return WC4D_OK;
}

int wc4d_prof_enable(wc4d_problem p, int enable) {
  if (p == nullptr || enable < 0) return WC4D_EINVAL;
  DevGuard g(p->device);
  int rc = prof_collect(p);
  if (rc) return rc;
  for (int c = 0; c < PROF_NCLASS; ++c) {
    p->profMs[c] = p->profBytes[c] = p->profFlops[c] = 0.0;
    p->profCalls[c] = 0;
  }
  p->kprof = enable & ((1 << PROF_NCLASS) - 1);
  for (auto& q : p->kprofSeq) q = 0;
  return WC4D_OK;
}

int wc4d_prof_stride(wc4d_problem p, int every) {
  if (p == nullptr || every < 1) return WC4D_EINVAL;
  p->kprofEvery = every;
  return WC4D_OK;
}

int wc4d_prof_read(wc4d_problem p, int cls, double* ms, long long* calls, double* bytes,
                   double* flops) {
  if (p == nullptr || cls < 0 || cls >= PROF_NCLASS) return WC4D_EINVAL;
  DevGuard g(p->device);
  int rc = prof_collect(p);
  if (rc) return rc;
  if (ms) *ms = p->profMs[cls];
  if (calls) *calls = p->profCalls[cls];
  if (bytes) *bytes = p->profBytes[cls];
  if (flops) *flops = p->profFlops[cls];
  return WC4D_OK;
}

int wc4d_set_profiling(wc4d_problem p, int enable) {
  if (p == nullptr) return WC4D_EINVAL;
  DevGuard g(p->device);
  if (enable && p->ev[0] == nullptr)
    for (auto& e : p->ev) HIPCHK(p, hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
  p->prof = enable != 0;
  return WC4D_OK;
}

int wc4d_last_apply_timing(wc4d_problem p, float* ms4) {
  if (p == nullptr || ms4 == nullptr) return WC4D_EINVAL;
  if (!p->prof) return fail(p, WC4D_ESTATE, "profiling is off");
  DevGuard g(p->device);
  HIPCHK(p, hipEventSynchronize(p->ev[4]));
  for (int k = 0; k < 4; ++k) HIPCHK(p, hipEventElapsedTime(&ms4[k], p->ev[k], p->ev[k + 1]));
  return WC4D_OK;
}

}  // extern "C"

// ------------------------------------------------------------ operator core

namespace {

// Y(time levels) = D^{1/2} X [+ E]: B^{1/2} on time 0, Q^{1/2} on times 1..N.
int dsqrt_apply(wc4d_problem p, const double* X, long long ldx, double* Y, long long ldy, int m,
                const double* E, long long lde, const int* skip, hipStream_t s, int mixed = SPLIT_NONE) {
  const int n = p->n, N = p->N;
  if (mixed == SPLIT_FP16 || mixed == SPLIT_BF16) {
    const bool f16 = mixed == SPLIT_FP16;
    if (f16) {  // column exponents of the right operand, all levels
      const size_t need = (size_t)m * (N + 1);
      if (p->colExpCap < need) {
        int rc = dev_alloc(p, &p->dColExp, need);
        if (rc) return rc;
        p->colExpCap = need;
      }
    }
    // products with Q^{1/2} (columns c0 .. of the exponent workspace): the fragment-major
    // kernel when the shape has enough tiles, else the LDS-tiled one
    auto q_product = [&](int ncol, ColMap xm, ColMap ym, ColMap em, int c0) -> int {
      if (!split_use_frag(n, ncol)) {
        if (f16)
          HIPCHK(p, gemm_fp16x3(n, ncol, n, 1.0, p->dQh16, p->dQl16, p->dQexp, X, xm, p->dColExp + c0, Y, ym, E,
                                em, s));
        else
          HIPCHK(p, gemm_bf16x3(n, ncol, n, 1.0, p->dQhi, p->dQlo, X, xm, Y, ym, E, em, s));
        return WC4D_OK;
      }
      const size_t need = bf16_frag_elems(ncol, n);
      if (p->xfCap < need) {
        int rc = dev_alloc(p, &p->dXf, need);
        if (rc) return rc;
        p->xfCap = need;
      }
      if (f16)
        HIPCHK(p, gemm_fp16x3_frag(n, ncol, n, 1.0, p->dQf16, p->dQexp, X, xm, p->dColExp + c0,
                                   reinterpret_cast<_Float16*>(p->dXf), Y, ym, E, em, s));
      else
        HIPCHK(p, gemm_bf16x3_frag(n, ncol, n, 1.0, p->dQf, X, xm, p->dXf, Y, ym, E, em, s));
      return WC4D_OK;
    };
    if (p->scaledB)  // all levels in one product with Q^{1/2}, level 0 scaled by c in the epilogue
      return q_product(m * (N + 1), ColMap{ldx, N + 1, 0, n}, ColMap{ldy, N + 1, 0, n, p->bScale},
                       ColMap{lde, N + 1, 0, n}, 0);
    if (f16)
      HIPCHK(p, gemm_fp16x3(n, m, n, 1.0, p->dBh16, p->dBl16, p->dBexp, X, ColMap{ldx, 1, 0, n}, p->dColExp, Y,
                            ColMap{ldy, 1, 0, n}, E, ColMap{lde, 1, 0, n}, s));
    else
      HIPCHK(p, gemm_bf16x3(n, m, n, 1.0, p->dBhi, p->dBlo, X, ColMap{ldx, 1, 0, n}, Y, ColMap{ldy, 1, 0, n}, E,
                            ColMap{lde, 1, 0, n}, s));
    return q_product(m * N, ColMap{ldx, N, 1, n}, ColMap{ldy, N, 1, n}, ColMap{lde, N, 1, n}, m);
  }
  if (m == 1 && p->ozSs != nullptr) {
    // one vector: all levels in one int8-sliced product with Q^{1/2}, level 0 scaled by c
    HIPCHK(p, oz_gemm(n, N + 1, p->ozSs, p->ozEs, X, n, p->bScale, E, Y, p->ozXs, p->ozFs, p->ozP, skip, s));
    return WC4D_OK;
  }
  const DsqrtTune* t = find_tune(p, m);
  if (p->scaledB) {
    // all levels with Q^{1/2} in one product, then level 0 rescaled by c (B^{1/2} = c Q^{1/2})
    // output columns of level 0 are scaled by c in the product's epilogue (before + E)
    const ColMap xa{ldx, N + 1, 0, n}, ya{ldy, N + 1, 0, n, p->bScale}, ea{lde, N + 1, 0, n};
    if (t != nullptr && t->twoSeg) {
      HIPCHK(p, dsqrt2_f64_v(t->segVariant, t->segSplits, n, n, X, Y, E, p->dQ, xa, ya, ea, m * (N + 1), nullptr,
                             xa, ya, ea, 0, skip, p->wsSplit, p->wsSplitDoubles, s));
    } else {
      HIPCHK(p, gemm_f64_tile(t ? t->tileAll : GEMM_AUTO, 0, n, m * (N + 1), n, 1.0, p->dQ, n, X, xa, Y, ya, E, ea,
                              skip, s, p->wsSplit, p->wsSplitDoubles));
    }
    return WC4D_OK;
  }
  const int var = t ? t->segVariant : 0, spl = t ? t->segSplits : 0;
  const bool two_ok = (long long)m * N <= 112 && m <= 112 &&
                      dsqrt2_feasible(var, spl, n, m * N, m, n, p->wsSplitDoubles);
  const bool two = two_ok && (t != nullptr ? t->twoSeg : n >= 512);
  if (two) {
    HIPCHK(p, dsqrt2_f64_v(var, spl, n, n, X, Y, E, p->dQ, ColMap{ldx, N, 1, n}, ColMap{ldy, N, 1, n},
                           ColMap{lde, N, 1, n}, m * N, p->dB, ColMap{ldx, 1, 0, n}, ColMap{ldy, 1, 0, n},
                           ColMap{lde, 1, 0, n}, m, skip, p->wsSplit, p->wsSplitDoubles, s));
    return WC4D_OK;
  }
  HIPCHK(p, gemm_f64_tile(t ? t->tileB : GEMM_AUTO, 0, n, m, n, 1.0, p->dB, n, X, ColMap{ldx, 1, 0, n}, Y,
                          ColMap{ldy, 1, 0, n}, E, ColMap{lde, 1, 0, n}, skip, s, p->wsSplit, p->wsSplitDoubles));
  HIPCHK(p, gemm_f64_tile(t ? t->tileQ : GEMM_AUTO, 0, n, m * N, n, 1.0, p->dQ, n, X, ColMap{ldx, N, 1, n}, Y,
                          ColMap{ldy, N, 1, n}, E, ColMap{lde, N, 1, n}, skip, s, p->wsSplit, p->wsSplitDoubles));
  return WC4D_OK;
}

int check_block_args(wc4d_problem p, const void* X, int ldx, const void* Y, int ldy, int m) {
  if (!is_state_ok(p)) return p ? fail(p, WC4D_ESTATE, "not finalized") : WC4D_EINVAL;
  if (X == nullptr || Y == nullptr || m < 1 || ldx < p->nA || ldy < p->nA)
    return fail(p, WC4D_EINVAL, "invalid block arguments (null pointer, m < 1 or ld < n_A)");
  const char* xb = (const char*)X;
  const char* yb = (const char*)Y;
  const size_t xs = sizeof(double) * ((size_t)ldx * (m - 1) + p->nA);
  const size_t ys = sizeof(double) * ((size_t)ldy * (m - 1) + p->nA);
  if (xb < yb + ys && yb < xb + xs) return fail(p, WC4D_EINVAL, "X and Y overlap");
  return WC4D_OK;
}

}  // namespace

namespace {

// Strong-constraint operator (control x_0 only): level 0 of the block = B^{1/2} X, the other
// levels zero (no forcing); the forward sweep with its observation stash, the adjoint sweep,
// then Y = X + B^{1/2} w_0.
int apply_A_sc(wc4d_problem p, const double* X, long long ldx, double* Y, long long ldy, int m, const int* skip,
               hipStream_t s) {
  const int n = p->n;
  const long long nL = p->nL;
  if (p->q == 0) {
    HIPCHK(p, block_copy(Y, ldy, X, ldx, n, m, s));
    return WC4D_OK;
  }
  const SweepModel md = p->sweep();
  double* P = p->wsBlock;
  const double n2 = (double)n * n, blk = 8.0 * (double)nL * m, stash = 8.0 * (double)p->q * m;
  const double gflops = 2.0 * n2 * m;
  HIPCHK(p, vec_fill(P, 0.0, nL * m, s));
  {
    ProfScope ps(p, s, PROF_DSQRT, 8.0 * n2 + 16.0 * n * m, gflops);
    HIPCHK(p, gemm_f64_tile(GEMM_AUTO, 0, n, m, n, 1.0, p->dB, n, X, ColMap{ldx, 1, 0, n}, P, ColMap{nL, 1, 0, n},
                            nullptr, ColMap{nL, 1, 0, n}, skip, s, p->wsSplit, p->wsSplitDoubles));
  }
  {
    ProfScope ps(p, s, PROF_SWEEP_FWD, blk + stash, 0.0);
    HIPCHK(p, sweep_fwd(md, P, nL, m, p->wsStash, p->q, nullptr, 0, skip, s));
  }
  {
    ProfScope ps(p, s, PROF_SWEEP_BWD, blk + stash, 0.0);
    HIPCHK(p, sweep_bwd(md, p->wsStash, p->q, nullptr, 0, m, P, nL, skip, s));
  }
  {
    ProfScope ps(p, s, PROF_DSQRT, 8.0 * n2 + 24.0 * n * m, gflops);
    HIPCHK(p, gemm_f64_tile(GEMM_AUTO, 0, n, m, n, 1.0, p->dB, n, P, ColMap{nL, 1, 0, n}, Y, ColMap{ldy, 1, 0, n},
                            X, ColMap{ldx, 1, 0, n}, skip, s, p->wsSplit, p->wsSplitDoubles));
  }
  return WC4D_OK;
}

}  // namespace

// Y = A X using the problem's block workspace (must hold m columns).
int wc4d::apply_A_core(wc4d_problem p, const double* X, long long ldx, double* Y, long long ldy,
                       int m, const int* skip, hipStream_t s, int mixed) {
  if (p->strong) return apply_A_sc(p, X, ldx, Y, ldy, m, skip, s);
  const long long nA = p->nA;
  if (p->q == 0) {
    HIPCHK(p, block_copy(Y, ldy, X, ldx, nA, m, s));
    return WC4D_OK;
  }
  const SweepModel md = p->sweep();
  double* P = p->wsBlock;
  const double n2 = (double)p->n * p->n, blk = 8.0 * (double)nA * m, stash = 8.0 * (double)p->q * m;
  const double gflops = 2.0 * n2 * (p->N + 1) * m;
  const double traj = (p->model == 1) ? 8.0 * 4.0 * p->n * p->N : 0.0;  // stage inputs, read once
  if (p->prof) HIPCHK(p, hipEventRecord(p->ev[0], s));
  int rc;
  const int dcls = mixed ? PROF_DSQRT_BF16 : PROF_DSQRT;
  const double dfl = mixed ? 3.0 * gflops : gflops;
  {
    ProfScope ps(p, s, dcls, (mixed ? 8.0 : 16.0) * n2 + 2.0 * blk, dfl);
    rc = dsqrt_apply(p, X, ldx, P, nA, m, nullptr, 0, skip, s, mixed);
  }
  if (rc) return rc;
  if (p->prof) HIPCHK(p, hipEventRecord(p->ev[1], s));
  {
    ProfScope ps(p, s, PROF_SWEEP_FWD, blk + stash + traj, 0.0);
    HIPCHK(p, sweep_fwd(md, P, nA, m, p->wsStash, p->q, nullptr, 0, skip, s));
  }
  if (p->prof) HIPCHK(p, hipEventRecord(p->ev[2], s));
  {
    ProfScope ps(p, s, PROF_SWEEP_BWD, blk + stash + traj, 0.0);
    HIPCHK(p, sweep_bwd(md, p->wsStash, p->q, nullptr, 0, m, P, nA, skip, s));
  }
  if (p->prof) HIPCHK(p, hipEventRecord(p->ev[3], s));
  {
    ProfScope ps(p, s, dcls, (mixed ? 8.0 : 16.0) * n2 + 3.0 * blk, dfl);
    rc = dsqrt_apply(p, P, nA, Y, ldy, m, X, ldx, skip, s, mixed);
  }
  if (rc) return rc;
  if (p->prof) HIPCHK(p, hipEventRecord(p->ev[4], s));
  return WC4D_OK;
}

extern "C" {

int wc4d_apply_A(wc4d_problem p, const double* X, int ldx, double* Y, int ldy, int m, hipStream_t s) {
  int rc = check_block_args(p, X, ldx, Y, ldy, m);
  if (rc) return rc;
  DevGuard g(p->device);
  if ((rc = ensure_block(p, m))) return rc;
  return apply_A_core(p, X, ldx, Y, ldy, m, nullptr, s);
}

int wc4d_apply_A_prec(wc4d_problem p, const double* X, int ldx, double* Y, int ldy, int m, int prec,
                      hipStream_t s) {
  int rc = check_block_args(p, X, ldx, Y, ldy, m);
  if (rc) return rc;
  if (prec != WC4D_PREC_FP64 && prec != WC4D_PREC_SKETCH_BF16X3 && prec != WC4D_PREC_SKETCH_FP16X3)
    return fail(p, WC4D_EINVAL, "prec must be WC4D_PREC_FP64, WC4D_PREC_SKETCH_BF16X3 or WC4D_PREC_SKETCH_FP16X3");
  if (p->strong && prec != WC4D_PREC_FP64)
    return fail(p, WC4D_EINVAL, "strong-constraint problems take float64 products only");
  if (prec == WC4D_PREC_SKETCH_BF16X3 && p->dBhi == nullptr)
    return fail(p, WC4D_ESTATE, "finalize without WC4D_PREC_SKETCH_BF16X3");
  if (prec == WC4D_PREC_SKETCH_FP16X3 && p->dBh16 == nullptr)
    return fail(p, WC4D_ESTATE, "finalize without WC4D_PREC_SKETCH_FP16X3");
  DevGuard g(p->device);
  if ((rc = ensure_block(p, m))) return rc;
  const int mode = prec == WC4D_PREC_SKETCH_BF16X3 ? SPLIT_BF16 : prec == WC4D_PREC_SKETCH_FP16X3 ? SPLIT_FP16 : SPLIT_NONE;
  return apply_A_core(p, X, ldx, Y, ldy, m, nullptr, s, mode);
}

int wc4d_apply_Linv(wc4d_problem p, const double* X, int ldx, double* Y, int ldy, int m, hipStream_t s) {
  int rc = check_block_args(p, X, ldx, Y, ldy, m);
  if (rc) return rc;
  if (p->strong) return fail(p, WC4D_EINVAL, "apply_Linv: not defined for a strong-constraint problem");
  DevGuard g(p->device);
  HIPCHK(p, sweep_fwd(p->sweep(), X, ldx, m, nullptr, 0, Y, ldy, nullptr, s));
  return WC4D_OK;
}

int wc4d_apply_LinvT(wc4d_problem p, const double* X, int ldx, double* Y, int ldy, int m, hipStream_t s) {
  int rc = check_block_args(p, X, ldx, Y, ldy, m);
  if (rc) return rc;
  if (p->strong) return fail(p, WC4D_EINVAL, "apply_LinvT: not defined for a strong-constraint problem");
  DevGuard g(p->device);
  HIPCHK(p, sweep_bwd(p->sweep(), nullptr, 0, X, ldx, m, Y, ldy, nullptr, s));
  return WC4D_OK;
}

int wc4d_apply_Dsqrt(wc4d_problem p, const double* X, int ldx, double* Y, int ldy, int m, hipStream_t s) {
  int rc = check_block_args(p, X, ldx, Y, ldy, m);
  if (rc) return rc;
  if (p->strong) return fail(p, WC4D_EINVAL, "apply_Dsqrt: not defined for a strong-constraint problem");
  DevGuard g(p->device);
  return dsqrt_apply(p, X, ldx, Y, ldy, m, nullptr, 0, nullptr, s);
}

int wc4d_rhs(wc4d_problem p, const double* d, const double* bt, double* rhs, hipStream_t s) {
  if (!is_state_ok(p)) return p ? fail(p, WC4D_ESTATE, "not finalized") : WC4D_EINVAL;
  if (rhs == nullptr || (p->q > 0 && d == nullptr)) return fail(p, WC4D_EINVAL, "null pointer");
  DevGuard g(p->device);
  int rc = ensure_block(p, 1);
  if (rc) return rc;
  const long long nA = p->nA;
  if (p->q == 0) {
    if (bt != nullptr) HIPCHK(p, vec_copy(rhs, bt, nA, s));
    else HIPCHK(p, vec_fill(rhs, 0.0, nA, s));
    return WC4D_OK;
  }
  HIPCHK(p, stash_from_innov(d, p->dObsRinv, p->wsStash, p->q, s));
  HIPCHK(p, sweep_bwd(p->sweep(), p->wsStash, p->q, nullptr, 0, 1, p->wsBlock, p->nL, nullptr, s));
  if (p->strong) {
    // B^{1/2} w_0 (+ bt)
    const int n = p->n;
    HIPCHK(p, gemm_f64_tile(GEMM_AUTO, 0, n, 1, n, 1.0, p->dB, n, p->wsBlock, ColMap{p->nL, 1, 0, n}, rhs,
                            ColMap{nA, 1, 0, n}, bt, ColMap{nA, 1, 0, n}, nullptr, s, p->wsSplit, p->wsSplitDoubles));
    return WC4D_OK;
  }
  return dsqrt_apply(p, p->wsBlock, nA, rhs, nA, 1, bt, nA, nullptr, s);
}

}  // extern "C"

// ------------------------------------------------------------ LMP build

// Frees an LMP's device memory (its problem's device must be current).
void wc4d::lmp_release(wc4d_lmp L) {
  dev_free(&L->AU);
  dev_free(&L->ninv);
  dev_free(&L->rzw);
  dev_free(&L->U);
  dev_free(&L->theta);
  dev_free(&L->dcoef);
  dev_free(&L->T);
  dev_free(&L->ws);
  dev_free(&L->wsv);
  dev_free(&L->wsr);
  dev_free(&L->GU);
  dev_free(&L->fu);
  dev_free(&L->Up);
  dev_free(&L->cexp);
}

int wc4d::ensure_build(wc4d_problem p, int m) {
  int rc;
  if (p->bufCols < m) {
    if ((rc = dev_alloc(p, &p->bufA, (size_t)(p->nA + 4) * m))) return rc;
    if ((rc = dev_alloc(p, &p->bufB, (size_t)(p->nA + 4) * m))) return rc;
    p->bufCols = m;
  }
  if (p->smallM < m) {
    if ((rc = dev_alloc(p, &p->small, (size_t)6 * m * m + 2 * (size_t)m))) return rc;
    p->smallM = m;
  }
  if ((rc = ensure_block(p, m))) return rc;
  if ((rc = ensure_gram(p, gram_ws_doubles(m, m, p->nA)))) return rc;
  return WC4D_OK;
}


namespace {

struct Small {
  double *G, *R1, *Ri, *R2, *K, *V, *lam, *dg;
  explicit Small(double* base, int m) {
    const size_t mm = (size_t)m * m;
    G = base;
    R1 = base + mm;
    Ri = base + 2 * mm;
    R2 = base + 3 * mm;
    K = base + 4 * mm;
    V = base + 5 * mm;
    lam = base + 6 * mm;
    dg = lam + m;
  }
};

// CholeskyQR2 of the n_A x m block Y (in place): Y = Q R with Q^T Q = I.
// tmp: n_A x m scratch.  When Rout != null, R (the product of the passes' triangular
// factors) is written there (m x m).  With p->cholShift the first pass Cholesky-factors
// Y^T Y + s I, s = 11 (n_A m + m (m + 1)) u trace(Y^T Y), and two plain passes follow
// (shifted CholeskyQR3): the form for blocks too ill-conditioned for CholeskyQR2; it
// flags the block rank deficient when R's diagonal spans more than 1 / (1e3 u).
int cholqr2(wc4d_problem p, double* Y, double* tmp, int m, Small& sm, double* Rout, hipStream_t s) {
  const long long nA = p->nA;
  const bool shifted = p->cholShift;
  const int passes = shifted ? 3 : 2;
  ProfScope ps(p, s, PROF_BUILD, 8.0 * 3.0 * passes * (double)nA * m, 4.0 * passes * (double)nA * m * m);
  const ColMap cm = plain_cols(nA);
  int* st = p->dStatus;
  double* src = Y;
  double* dst = tmp;
  for (int k = 0; k < passes; ++k) {
    HIPCHK(p, gram_f64(m, m, nA, src, cm, src, cm, sm.G, m, p->wsGram, nullptr, s));
    if (shifted && k == 0) {
      const double c = 11.0 * ((double)nA * m + (double)m * (m + 1)) * 1.1102230246251565e-16;
      HIPCHK(p, shift_diag_trace(m, sm.G, m, c, s));
    }
    HIPCHK(p, chol_upper(m, sm.G, m, st, s));
    if (shifted) HIPCHK(p, diag_accumulate(m, sm.G, m, sm.dg, k == 0, s));
    HIPCHK(p, tri_inv_upper(m, sm.G, m, sm.Ri, m, s));
    HIPCHK(p, gemm_f64((int)nA, m, m, 1.0, src, nA, sm.Ri, upper_cols(m), dst, cm, nullptr, cm, nullptr, s));
    if (Rout != nullptr) {
      if (k == 0) {
        HIPCHK(p, vec_copy(sm.R1, sm.G, (long long)m * m, s));
      } else {
        HIPCHK(p, small_gemm(m, m, m, 1.0, sm.G, m, 0, sm.R1, m, 0, sm.K, m, s));
        HIPCHK(p, vec_copy(sm.R1, sm.K, (long long)m * m, s));
      }
    }
    std::swap(src, dst);
  }
  if (src != Y) HIPCHK(p, vec_copy(Y, src, nA * m, s));
  if (Rout != nullptr) HIPCHK(p, vec_copy(Rout, sm.R1, (long long)m * m, s));
  // the shift makes any Gram matrix factorable: a block whose R (diagonal = product of
  // the passes' diagonals) has min/max below 1e3 u is numerically rank deficient
  if (shifted) HIPCHK(p, rank_check(m, sm.dg, 1e3 * 2.220446049250313e-16, st, s));
  return WC4D_OK;
}

// The start block G of Algorithms 3-5: the caller's (G != null), or the n_A x m Gaussian
// block of `seed` drawn on the device into dst (*Guse then points at dst).
int start_block(wc4d_problem p, const double* G, unsigned long long seed, int m, double* dst,
                const double** Guse, hipStream_t s) {
  *Guse = G;
  if (G != nullptr) return WC4D_OK;
  HIPCHK(p, gauss_block(seed, p->nA, m, 0, dst, p->nA, s));
  *Guse = dst;
  return WC4D_OK;
}

int lmp_build_once(wc4d_problem p, int method, int k_r, int l, const double* G, unsigned long long seed,
                   wc4d_lmp* out, hipStream_t s) {
  if (out == nullptr) return WC4D_EINVAL;
  *out = nullptr;
  if (!is_state_ok(p)) return p ? fail(p, WC4D_ESTATE, "not finalized") : WC4D_EINVAL;
  const int m = k_r + l;
  if (method < WC4D_REVD || method > WC4D_NYSTROM_1P || k_r < 1 || l < 0 || m > p->nA || m > 512)
    return fail(p, WC4D_EINVAL, "invalid LMP arguments (method, k_r >= 1, l >= 0, m <= min(n_A, 512))");
  DevGuard g(p->device);
  int rc = ensure_build(p, m);
  if (rc) return rc;
  wc4d_lmp L = new (std::nothrow) wc4d_lmp_s();
  if (L == nullptr) return WC4D_ENOMEM;
  L->p = p;
  p->lmps.push_back(L);
  L->nA = p->nA;
  L->ldu = (p->nA + 3) / 4 * 4;
  L->k = k_r;
  auto cleanup = [&](int code) {
    wc4d_lmp_destroy(L);
    return code;
  };
  if ((rc = dev_alloc(p, &L->U, (size_t)L->ldu * k_r))) return cleanup(rc);
  if ((rc = dev_alloc(p, &L->theta, k_r))) return cleanup(rc);
  if ((rc = dev_alloc(p, &L->dcoef, k_r))) return cleanup(rc);

  const long long nA = p->nA;
  const ColMap cm = plain_cols(nA);
  Small sm(p->small, m);
  double* A_ = p->bufA;
  double* B_ = p->bufB;
  hipError_t he = hipMemsetAsync(p->dStatus, 0, sizeof(int), s);
  if (he != hipSuccess) return cleanup(fail(p, WC4D_EHIP, hipGetErrorString(he)));
  double* Zfinal = nullptr;
  int mode = 0;
  bool evd_sym = true;
  const int mx = (p->prec & WC4D_PREC_SKETCH_BF16X3) ? SPLIT_BF16
                 : (p->prec & WC4D_PREC_SKETCH_FP16X3) ? SPLIT_FP16 : SPLIT_NONE;
  if (method == WC4D_REVD) {
    // Algorithm 3: Y = A G; Z = orth(Y); K = Z^T A Z; EVD; U = Z W
    if ((rc = start_block(p, G, seed, m, B_, &G, s))) return cleanup(rc);
    if ((rc = apply_A_core(p, G, nA, A_, nA, m, nullptr, s, mx))) return cleanup(rc);
    if ((rc = cholqr2(p, A_, B_, m, sm, nullptr, s))) return cleanup(rc);
    if ((rc = apply_A_core(p, A_, nA, B_, nA, m, nullptr, s, mx))) return cleanup(rc);
    L->applies = 2;
    he = gram_f64(m, m, nA, A_, cm, B_, cm, sm.K, m, p->wsGram, nullptr, s);
    if (he != hipSuccess) return cleanup(fail(p, WC4D_EHIP, hipGetErrorString(he)));
    Zfinal = A_;
  } else if (method == WC4D_NYSTROM) {
    // Algorithm 4: Y = A G; Z = orth(Y); E1 = A Z; E2 = Z^T E1 = C^T C; F = E1 C^{-1};
    // SVD F = U Sigma V^T via F = Q_F R_F and the EVD of R_F R_F^T; Theta = Sigma^2
    if ((rc = start_block(p, G, seed, m, B_, &G, s))) return cleanup(rc);
    if ((rc = apply_A_core(p, G, nA, A_, nA, m, nullptr, s, mx))) return cleanup(rc);
    if ((rc = cholqr2(p, A_, B_, m, sm, nullptr, s))) return cleanup(rc);
    if ((rc = apply_A_core(p, A_, nA, B_, nA, m, nullptr, s, mx))) return cleanup(rc);
    L->applies = 2;
    he = gram_f64(m, m, nA, A_, cm, B_, cm, sm.G, m, p->wsGram, nullptr, s);
    if (he == hipSuccess) he = chol_upper(m, sm.G, m, p->dStatus, s);
    if (he == hipSuccess) he = tri_inv_upper(m, sm.G, m, sm.Ri, m, s);
    if (he == hipSuccess)
      he = gemm_f64((int)nA, m, m, 1.0, B_, nA, sm.Ri, upper_cols(m), A_, cm, nullptr, cm, nullptr, s);
    if (he != hipSuccess) return cleanup(fail(p, WC4D_EHIP, hipGetErrorString(he)));
    if ((rc = cholqr2(p, A_, B_, m, sm, sm.R2, s))) return cleanup(rc);
    // the EVD of R_F R_F^T as the one-sided Jacobi SVD of R_F^T (no squared condition
    // number): singular values sigma, left singular vectors of R_F; Theta = sigma^2
    he = transpose_small(m, sm.R2, m, sm.K, m, s);
    evd_sym = false;
    mode = 2;
    if (he != hipSuccess) return cleanup(fail(p, WC4D_EHIP, hipGetErrorString(he)));
    Zfinal = A_;
  } else if (method == WC4D_NYSTROM_1P) {
    // single-pass Nystrom: G_4 = orth(G); Y = A G_4; E = G_4^T Y = C^T C; F = Y C^{-1};
    // SVD F = U Sigma V^T via F = Q_F R_F and the one-sided Jacobi SVD of R_F^T; Theta = Sigma^2
    he = G != nullptr ? vec_copy(A_, G, nA * m, s) : gauss_block(seed, nA, m, 0, A_, nA, s);
    if (he != hipSuccess) return cleanup(fail(p, WC4D_EHIP, hipGetErrorString(he)));
    if ((rc = cholqr2(p, A_, B_, m, sm, nullptr, s))) return cleanup(rc);
    if ((rc = apply_A_core(p, A_, nA, B_, nA, m, nullptr, s, mx))) return cleanup(rc);
    L->applies = 1;
    he = gram_f64(m, m, nA, A_, cm, B_, cm, sm.G, m, p->wsGram, nullptr, s);
    if (he == hipSuccess) he = chol_upper(m, sm.G, m, p->dStatus, s);
    if (he == hipSuccess) he = tri_inv_upper(m, sm.G, m, sm.Ri, m, s);
    if (he == hipSuccess)
      he = gemm_f64((int)nA, m, m, 1.0, B_, nA, sm.Ri, upper_cols(m), A_, cm, nullptr, cm, nullptr, s);
    if (he != hipSuccess) return cleanup(fail(p, WC4D_EHIP, hipGetErrorString(he)));
    if ((rc = cholqr2(p, A_, B_, m, sm, sm.R2, s))) return cleanup(rc);
    he = transpose_small(m, sm.R2, m, sm.K, m, s);
    evd_sym = false;
    mode = 2;
    if (he != hipSuccess) return cleanup(fail(p, WC4D_EHIP, hipGetErrorString(he)));
    Zfinal = A_;
  } else {
    // Algorithm 5: G_3 = orth(G); Y_3 = A G_3 = Z_3 R_3; K_3 = R_3 R_3^T = W Theta^2 W^T
    he = G != nullptr ? vec_copy(A_, G, nA * m, s) : gauss_block(seed, nA, m, 0, A_, nA, s);
    if (he != hipSuccess) return cleanup(fail(p, WC4D_EHIP, hipGetErrorString(he)));
    if ((rc = cholqr2(p, A_, B_, m, sm, nullptr, s))) return cleanup(rc);
    if ((rc = apply_A_core(p, A_, nA, B_, nA, m, nullptr, s, mx))) return cleanup(rc);
    L->applies = 1;
    if ((rc = cholqr2(p, B_, A_, m, sm, sm.R2, s))) return cleanup(rc);
    // W Theta^2 W^T = R_3 R_3^T as the one-sided Jacobi SVD of R_3^T: Theta = sigma
    he = transpose_small(m, sm.R2, m, sm.K, m, s);
    evd_sym = false;
    mode = 0;
    if (he != hipSuccess) return cleanup(fail(p, WC4D_EHIP, hipGetErrorString(he)));
    Zfinal = B_;
  }
  ProfScope ps_tail(p, s, PROF_BUILD, 8.0 * (double)nA * (m + k_r), 2.0 * (double)nA * m * k_r);
  // pinned flags for the EVD's convergence poll (made at the first build)
  for (int q = 0; q < 2 && he == hipSuccess; ++q) {
    if (p->evdPoll.host[q] == nullptr)
      he = hipHostMalloc((void**)&p->evdPoll.host[q], sizeof(int), hipHostMallocDefault);
    if (he == hipSuccess && p->evdPoll.ev[q] == nullptr)
      he = hipEventCreateWithFlags(&p->evdPoll.ev[q], hipEventDisableTiming);
  }
  if (he == hipSuccess) he = jacobi_evd(m, sm.K, m, sm.lam, sm.V, m, p->dStatus + 4, s, evd_sym, &p->evdPoll);
  if (he == hipSuccess) he = ritz_finish(k_r, sm.lam, mode, L->theta, L->dcoef, s);
  if (he == hipSuccess)
    he = gemm_f64((int)nA, k_r, m, 1.0, Zfinal, nA, sm.V, plain_cols(m), L->U, plain_cols(L->ldu), nullptr,
                  cm, nullptr, s);
  if (he != hipSuccess) return cleanup(fail(p, WC4D_EHIP, hipGetErrorString(he)));
  // status words 0 (Cholesky / rank) and 4 (Jacobi converged flag)
  int stw[5] = {0, 0, 0, 0, 0};
  he = hipMemcpyAsync(stw, p->dStatus, sizeof stw, hipMemcpyDeviceToHost, s);
  if (he == hipSuccess) he = hipStreamSynchronize(s);
  if (he != hipSuccess) return cleanup(fail(p, WC4D_EHIP, hipGetErrorString(he)));
  const int st = stw[0];
  if (st == 0 && stw[4] == 0)
    return cleanup(fail(p, WC4D_ENOCONV, "one-sided Jacobi of the small problem did not converge in 20 sweeps"));
  if (st != 0)
    return cleanup(fail(p, WC4D_ENOTSPD,
                        std::string(st == 2 ? "start block numerically rank deficient (R diagonal spans > 1/(1e3 u))"
                                            : "Cholesky met a non-positive pivot (rank-deficient sketch?)") +
                            (p->cholShift ? " after shifted CholeskyQR3" : "")));
  // U^T U of the U the PCG streams, for the fused recursion (identity up to rounding
  // for an orthonormal U; computed from the values of the panel copy when there is one)
  if ((rc = dev_alloc(p, &L->GU, (size_t)k_r * k_r))) return cleanup(rc);
  if ((rc = dev_alloc(p, &L->fu, (size_t)3 * k_r))) return cleanup(rc);
  if ((rc = ensure_gram(p, gram_ws_doubles(k_r, k_r, nA)))) return cleanup(rc);
  // panel-major float32 or float16 copy for the PCG passes; the build's scratch block B_
  // (n_A x m doubles) receives the rounded values column-major for the Gram (rows n_A .. ldu
  // of it are never read)
  auto make_copy = [&](LmpFmt fmt) -> int {
    dev_free(&L->Up);
    dev_free(&L->cexp);
    L->ufmt = fmt;
    const double* Ug = L->U;
    if (fmt != LMP_F64) {
      if (L->ldu * k_r > (nA + 4) * m) return fail(p, WC4D_EHIP, "panel copy of U: scratch too small");
      int r;
      if (fmt == LMP_P16) {
        _Float16* P16 = nullptr;
        if ((r = dev_alloc(p, &P16, lmp_panel_elems(nA, k_r)))) return r;
        L->Up = P16;
        if ((r = dev_alloc(p, &L->cexp, (size_t)k_r))) return r;
        he = lmp_to_panels16(P16, L->cexp, L->U, L->ldu, nA, k_r, B_, s);
      } else {
        float* P32 = nullptr;
        if ((r = dev_alloc(p, &P32, lmp_panel_elems(nA, k_r)))) return r;
        L->Up = P32;
        he = lmp_to_panels(P32, L->U, L->ldu, nA, k_r, B_, s);
      }
      if (he != hipSuccess) return fail(p, WC4D_EHIP, "panel copy of U failed");
      Ug = B_;
    }
    he = gram_f64(k_r, k_r, nA, Ug, plain_cols(L->ldu), Ug, plain_cols(L->ldu), L->GU, k_r, p->wsGram,
                  nullptr, s);
    if (he == hipSuccess) he = hipStreamSynchronize(s);
    if (he != hipSuccess) return fail(p, WC4D_EHIP, hipGetErrorString(he));
    return WC4D_OK;
  };
  const LmpFmt want = (p->prec & WC4D_PREC_LMP_FP16) ? LMP_P16 : (p->prec & WC4D_PREC_LMP_FP32) ? LMP_P32 : LMP_F64;
  if ((rc = make_copy(want))) return cleanup(rc);
  if (want == LMP_P16) {
    // C = I + Ũ diag(d) Ũ^T with d_i = theta_i^{-1/2} - 1 > -1 has smallest eigenvalue at
    // least 1 + d_min (1 + ||Ũ^T Ũ - I||_2) (1 + d_min for an orthonormal U).  Keep the
    // float16 copy while its Gram defect (Frobenius bound) is at most half of 1 + d_min,
    // so C stays positive definite with at least half its exact smallest eigenvalue;
    // otherwise stream the float32 copy.
    double chk[2] = {0.0, 0.0};
    he = lmp_copy_check(k_r, L->GU, L->dcoef, L->fu, s);
    if (he == hipSuccess) he = hipMemcpyAsync(chk, L->fu, sizeof chk, hipMemcpyDeviceToHost, s);
    if (he == hipSuccess) he = hipStreamSynchronize(s);
    if (he != hipSuccess) return cleanup(fail(p, WC4D_EHIP, hipGetErrorString(he)));
    const double dmin = chk[1] < 0.0 ? chk[1] : 0.0;
    if (!(chk[0] <= 0.5 * (1.0 + dmin)) && (rc = make_copy(LMP_P32))) return cleanup(rc);
  }
  *out = L;
  return WC4D_OK;
}

}  // namespace

extern "C" {

int wc4d_lmp_build(wc4d_problem p, int method, int k_r, int l, const double* G, unsigned long long seed,
                   wc4d_lmp* out, hipStream_t s) {
  int rc = lmp_build_once(p, method, k_r, l, G, seed, out, s);
  if (rc != WC4D_ENOTSPD) return rc;
  // a Cholesky factorisation broke down: once more with shifted CholeskyQR3
  p->cholShift = true;
  rc = lmp_build_once(p, method, k_r, l, G, seed, out, s);
  p->cholShift = false;
  return rc;
}

int wc4d_gaussian_block(int device, unsigned long long seed, long long n_rows, int n_cols, long long col0,
                        double* G, long long ldg, hipStream_t s) {
  if (n_rows < 0 || n_cols < 0 || col0 < 0 || col0 + n_cols > 0xFFFFFFFFll || (n_rows + 1) / 2 > 0xFFFFFFFFll)
    return WC4D_EINVAL;
  if (n_rows == 0 || n_cols == 0) return WC4D_OK;
  if (G == nullptr || ldg < n_rows || !device_ok(device)) return WC4D_EINVAL;
  DevGuard g(device);
  return gauss_block(seed, n_rows, n_cols, col0, G, ldg, s) == hipSuccess ? WC4D_OK : WC4D_EHIP;
}

int wc4d_philox4x32_10(int device, const unsigned int* ctr_key, unsigned int* out, long long count,
                       hipStream_t s) {
  if (count < 0) return WC4D_EINVAL;
  if (count == 0) return WC4D_OK;
  if (ctr_key == nullptr || out == nullptr || !device_ok(device)) return WC4D_EINVAL;
  DevGuard g(device);
  return philox_words(ctr_key, out, count, s) == hipSuccess ? WC4D_OK : WC4D_EHIP;
}

int wc4d_lmp_theta(wc4d_lmp L, double* theta_host) {
  if (L == nullptr || theta_host == nullptr) return WC4D_EINVAL;
  if (L->p == nullptr) return WC4D_ESTATE;
  DevGuard g(L->p->device);
  HIPCHK(L->p, hipMemcpy(theta_host, L->theta, sizeof(double) * L->k, hipMemcpyDeviceToHost));
  return WC4D_OK;
}

int wc4d_lmp_vectors(wc4d_lmp L, double* U, int ldu, hipStream_t s) {
  if (L == nullptr || U == nullptr || ldu < L->nA) return WC4D_EINVAL;
  if (L->p == nullptr) return WC4D_ESTATE;
  DevGuard g(L->p->device);
  HIPCHK(L->p, block_copy(U, ldu, L->U, L->ldu, L->nA, L->k, s));
  return WC4D_OK;
}

int wc4d_lmp_copy_format(wc4d_lmp L, int* prec_flag) {
  if (L == nullptr || prec_flag == nullptr) return WC4D_EINVAL;
  if (L->p == nullptr) return WC4D_ESTATE;
  *prec_flag = L->Up == nullptr ? 0 : (L->ufmt == LMP_P16 ? WC4D_PREC_LMP_FP16 : WC4D_PREC_LMP_FP32);
  return WC4D_OK;
}

int wc4d_lmp_applies(wc4d_lmp L, int* count) {
  if (L == nullptr || count == nullptr) return WC4D_EINVAL;
  *count = L->applies;
  return WC4D_OK;
}

}  // extern "C"

namespace {

// Y = C X = X + U diag(theta^{-1/2} - 1) U^T X
int lmp_apply_core(wc4d_lmp L, const double* X, long long ldx, double* Y, long long ldy, int m,
                   const int* skip, hipStream_t s) {
  wc4d_problem p = L->p;
  int rc;
  if (m <= 2) {
    const size_t need = lmp_gemv_ws_doubles(L->nA, L->k);
    if (L->wsvDoubles < need) {
      if ((rc = dev_alloc(p, &L->wsv, need))) return rc;
      L->wsvDoubles = need;
    }
    const LmpU Us = L->streamed();
    const double ub = lmp_elem_bytes(Us.fmt) * (double)L->nA * L->k, fl = 2.0 * (double)L->nA * L->k;
    for (int c = 0; c < m; ++c) {
      {
        ProfScope ps(p, s, PROF_LMP_T, ub + 8.0 * L->nA, fl);
        HIPCHK(p, lmp_gemv_t(L->nA, L->k, Us, L->dcoef, X + (size_t)c * ldx, L->wsv, skip, s));
      }
      ProfScope ps(p, s, PROF_LMP_N, ub + 16.0 * L->nA, fl);
      HIPCHK(p, lmp_gemv_n(L->nA, L->k, Us, X + (size_t)c * ldx, Y + (size_t)c * ldy, L->wsv, skip, s));
    }
    return WC4D_OK;
  }
  if (L->tcap < m) {
    if ((rc = dev_alloc(p, &L->T, (size_t)L->k * m))) return rc;
    L->tcap = m;
  }
  const size_t wsn = gram_ws_doubles(L->k, m, L->nA);
  if (L->wsDoubles < wsn) {
    if ((rc = dev_alloc(p, &L->ws, wsn))) return rc;
    L->wsDoubles = wsn;
  }
  HIPCHK(p, gram_f64(L->k, m, L->nA, L->U, plain_cols(L->ldu), X, plain_cols(ldx), L->T, L->k, L->ws,
                     skip, s));
  HIPCHK(p, vec_scale_rows(L->T, L->k, m, L->k, L->dcoef, skip, s));
  HIPCHK(p, gemm_f64((int)L->nA, m, L->k, 1.0, L->U, L->ldu, L->T, plain_cols(L->k), Y,
                     plain_cols(ldy), X, plain_cols(ldx), skip, s));
  return WC4D_OK;
}

// Y = P X for the Ritz-LMP of eq. Ritz_LMP, P = (I - U Theta^{-1} U^T A)(I - A U Theta^{-1} U^T)
// + U Theta^{-1} U^T, with A U kept from wc4d_lmp_ritz_prepare (A symmetric: U^T A y = (AU)^T y).
// Per vector: t1 = -Theta^{-1} U^T x; y1 = x + (AU) t1; t2 = -Theta^{-1} (AU)^T y1;
// y = y1 + U (t2 - t1).  Four passes over n_A x k.
int ritz_apply_core(wc4d_lmp L, const double* X, long long ldx, double* Y, long long ldy, int m, const int* skip,
                    hipStream_t s) {
  wc4d_problem p = L->p;
  LmpU Uu, AUu;
  Uu.p = L->U;
  Uu.fmt = LMP_F64;
  Uu.ldu = L->ldu;
  AUu.p = L->AU;
  AUu.fmt = LMP_F64;
  AUu.ldu = L->ldu;
  const long long nA = L->nA;
  const int k = L->k;
  double* y1 = L->rzw;
  double* t1 = L->rzw + nA;
  double* t = L->wsv + lmp_gemv_t_offset(nA, k);
  const double pb = 8.0 * (double)nA * k, fl = 2.0 * (double)nA * k;
  for (int c = 0; c < m; ++c) {
    const double* x = X + (size_t)c * ldx;
    double* y = Y + (size_t)c * ldy;
    ProfScope ps(p, s, PROF_LMP_T, 4.0 * pb + 5.0 * 8.0 * nA, 4.0 * fl);
    HIPCHK(p, lmp_gemv_t(nA, k, Uu, L->ninv, x, L->wsv, skip, s));
    HIPCHK(p, vec_copy_skip(t1, t, k, skip, s));
    HIPCHK(p, lmp_gemv_n(nA, k, AUu, x, y1, L->wsv, skip, s));
    HIPCHK(p, lmp_gemv_t(nA, k, AUu, L->ninv, y1, L->wsv, skip, s));
    HIPCHK(p, vec_sub_small(t, t1, k, skip, s));
    HIPCHK(p, lmp_gemv_n(nA, k, Uu, y1, y, L->wsv, skip, s));
  }
  return WC4D_OK;
}

}  // namespace

extern "C" {

int wc4d_lmp_ritz_prepare(wc4d_lmp L, hipStream_t s) {
  if (L == nullptr) return WC4D_EINVAL;
  wc4d_problem p = L->p;
  if (p == nullptr) return WC4D_ESTATE;
  if (!is_state_ok(p)) return fail(p, WC4D_ESTATE, "not finalized");
  DevGuard g(p->device);
  int rc;
  if (L->AU == nullptr) {
    if ((rc = dev_alloc(p, &L->AU, (size_t)L->ldu * L->k))) return rc;
    if ((rc = dev_alloc(p, &L->ninv, L->k))) return rc;
    if ((rc = dev_alloc(p, &L->rzw, (size_t)L->nA + L->k))) return rc;
  }
  const size_t need = lmp_gemv_ws_doubles(L->nA, L->k);
  if (L->wsvDoubles < need) {
    if ((rc = dev_alloc(p, &L->wsv, need))) return rc;
    L->wsvDoubles = need;
  }
  if ((rc = ensure_block(p, L->k))) return rc;
  // one block product with A (the k Ritz vectors), in float64 whatever the problem's mode
  if ((rc = apply_A_core(p, L->U, L->ldu, L->AU, L->ldu, L->k, nullptr, s))) return rc;
  HIPCHK(p, vec_neg_inv(L->theta, L->ninv, L->k, s));
  HIPCHK(p, hipStreamSynchronize(s));
  return WC4D_OK;
}

int wc4d_lmp_ritz_apply(wc4d_lmp L, const double* X, int ldx, double* Y, int ldy, int m, hipStream_t s) {
  if (L == nullptr) return WC4D_EINVAL;
  if (L->p == nullptr) return WC4D_ESTATE;
  if (L->AU == nullptr) return fail(L->p, WC4D_ESTATE, "lmp_ritz_apply: call wc4d_lmp_ritz_prepare first");
  int rc = check_block_args(L->p, X, ldx, Y, ldy, m);
  if (rc) return rc;
  DevGuard g(L->p->device);
  return ritz_apply_core(L, X, ldx, Y, ldy, m, nullptr, s);
}

int wc4d_lmp_apply(wc4d_lmp L, const double* X, int ldx, double* Y, int ldy, int m, hipStream_t s) {
  if (L == nullptr) return WC4D_EINVAL;
  if (L->p == nullptr) return WC4D_ESTATE;
  int rc = check_block_args(L->p, X, ldx, Y, ldy, m);
  if (rc) return rc;
  DevGuard g(L->p->device);
  return lmp_apply_core(L, X, ldx, Y, ldy, m, nullptr, s);
}

int wc4d_lmp_destroy(wc4d_lmp L) {
  if (L == nullptr) return WC4D_OK;
  if (L->p != nullptr) {
    auto& v = L->p->lmps;
    v.erase(std::remove(v.begin(), v.end(), L), v.end());
    DevGuard g(L->p->device);
    lmp_release(L);
  }
  delete L;
  return WC4D_OK;
}

// ------------------------------------------------------------------ PCG

namespace {

// Algorithm 1 on the device.  With F != null (no LMP only) the normalised residuals
// f_j = (-1)^j r_j / ||r_j|| go into the columns of F and the CG coefficients into
// alphas / betas (host): the Lanczos information of Section 3.4.  With reorth each new
// residual is orthogonalised twice against f_0..f_{j-1} before r_j^T r_j and beta_j.
int pcg_run(wc4d_problem p, wc4d_lmp L, const double* b, double* x, const wc4d_pcg_opts* opts,
            wc4d_pcg_info* info, double* hist_true, double* hist_precond, double* hist_J, double* alphas,
            double* betas, double* F, long long ldf, bool reorth, hipStream_t s, bool ritz = false) {
  if (!is_state_ok(p)) return p ? fail(p, WC4D_ESTATE, "not finalized") : WC4D_EINVAL;
  if (b == nullptr || x == nullptr || opts == nullptr || info == nullptr || opts->maxit < 1 ||
      !(opts->tol >= 0.0) || (opts->criterion != WC4D_RES_TRUE && opts->criterion != WC4D_RES_PRECOND))
    return fail(p, WC4D_EINVAL, "invalid PCG arguments");
  if (L != nullptr && L->p != p) return fail(p, WC4D_EINVAL, "LMP built for another problem (or orphaned)");
  if (opts->variant != WC4D_PCG_FUSED && opts->variant != WC4D_PCG_PLAIN)
    return fail(p, WC4D_EINVAL, "unknown PCG variant");
  const bool fused = (L != nullptr && opts->variant == WC4D_PCG_FUSED && !ritz);
  if (ritz && (L == nullptr || L->AU == nullptr))
    return fail(p, WC4D_ESTATE, "pcg_ritz: the LMP needs wc4d_lmp_ritz_prepare first");
  if (reorth && (F == nullptr || L != nullptr || opts->maxit > 512))
    return fail(p, WC4D_EINVAL, "reorthogonalised CG: no LMP, Lanczos vectors kept, maxit <= 512");
  DevGuard g(p->device);
  const long long nA = p->nA;
  int rc;
  if ((rc = ensure_block(p, 1))) return rc;
  // reorthogonalisation scratch: the partial sums of F^T r for up to maxit columns and t
  double* rws = nullptr;
  struct FreeOnExit {
    double** q;
    ~FreeOnExit() { dev_free(q); }
  } rws_guard{&rws};
  size_t rws_t = 0;
  if (reorth) {
    for (int j = 1; j <= opts->maxit; ++j) rws_t = std::max(rws_t, lmp_gemv_ws_doubles(nA, j));
    if ((rc = dev_alloc(p, &rws, rws_t + (size_t)opts->maxit))) return rc;
  }
  if (p->pcgVec == nullptr) {
    if ((rc = dev_alloc(p, &p->pcgVec, (size_t)6 * nA))) return rc;
    if ((rc = dev_alloc(p, &p->pcgRed, pcg_red_doubles()))) return rc;
    if ((rc = dev_alloc(p, &p->pcgState, 1))) return rc;
    HIPCHK(p, hipHostMalloc((void**)&p->pcgStateHost, sizeof(PcgState), hipHostMallocDefault));
    for (int q = 0; q < 2; ++q) {
      HIPCHK(p, hipHostMalloc((void**)&p->pcgPoll[q], sizeof(PcgState), hipHostMallocDefault));
      HIPCHK(p, hipEventCreateWithFlags(&p->pcgPollEv[q], hipEventDisableTiming));
    }
  }
  if (p->pcgHistCap < opts->maxit) {
    if ((rc = dev_alloc(p, &p->pcgHist, (size_t)5 * opts->maxit))) return rc;
    p->pcgHistCap = opts->maxit;
  }
  double* r = p->pcgVec;
  double* pv = r + nA;
  double* Ap = pv + nA;
  double* sres = Ap + nA;
  double* w = sres + nA;
  double* z = w + nA;
  PcgState* st = p->pcgState;
  const int* done = &st->done;
  int* xzero = p->dStatus + 1;
  // s_0 = b - A x_0 (the product is skipped for x_0 = 0), r_0 = C^T s_0, p_0 = C r_0
  HIPCHK(p, pcg_x0_zero_flag(x, nA, p->pcgRed, xzero, s));
  if ((rc = apply_A_core(p, x, nA, Ap, nA, 1, xzero, s))) return rc;
  HIPCHK(p, pcg_s0(b, Ap, xzero, sres, nA, s));
  if (ritz) {
    // standard preconditioned CG: z_0 = P s_0, p_0 = z_0 (r is the true residual s)
    if ((rc = ritz_apply_core(L, sres, nA, z, nA, 1, nullptr, s))) return rc;
    HIPCHK(p, vec_copy(pv, z, nA, s));
    HIPCHK(p, pcg_kernels_init_std(st, b, sres, z, nA, opts->tol, opts->maxit, opts->criterion, p->pcgRed, s));
  } else if (L != nullptr) {
    if ((rc = lmp_apply_core(L, sres, nA, r, nA, 1, nullptr, s))) return rc;
    if ((rc = lmp_apply_core(L, r, nA, pv, nA, 1, nullptr, s))) return rc;
  } else {
    HIPCHK(p, vec_copy(r, sres, nA, s));
    HIPCHK(p, vec_copy(pv, r, nA, s));
  }
  if (!ritz) HIPCHK(p, pcg_kernels_init(st, b, sres, r, nA, opts->tol, opts->maxit, opts->criterion, p->pcgRed, s));
  if (F != nullptr) HIPCHK(p, pcg_lanczos_col(st, 0, r, F, ldf, nA, s));
  double* u = nullptr;
  double* d12 = nullptr;
  double* tvec = nullptr;
  const LmpU Us = (L == nullptr) ? LmpU() : L->streamed();
  const bool panels = Us.fmt != LMP_F64;
  // float16 panels: the refresh of u = U^T r shares the p-update launch and the next
  // iteration's final-sum launch (same arithmetic as the separate refresh launches)
  const bool share_refresh = fused && Us.fmt == LMP_P16;
  if (share_refresh && L->wsr == nullptr) {
    if ((rc = dev_alloc(p, &L->wsr, lmp_pan16_refresh_doubles(nA, L->k)))) return rc;
  }
  if (fused) {
    u = L->fu;
    d12 = L->fu + L->k;
    tvec = L->wsv + lmp_gemv_t_offset(nA, L->k);
    HIPCHK(p, lmp_gemv_t(nA, L->k, Us, nullptr, r, L->wsv, nullptr, s, u));
  }
  // The host enqueues chunks of `poll` iterations and reads the device state after each
  // chunk; the next chunk is already enqueued while it waits (two pinned copies of the
  // state, one event each), so the stream does not idle during the poll.  Kernels return
  // at once after the solve is done, so the chunk in flight at that point costs launches only.
  const int poll = 8;
  int it = 0, issued = 0, pending = 0;
  for (;;) {
   while (pending < 2 && it < opts->maxit) {
    const int chunk = std::min(poll, opts->maxit - it);
    for (int c = 0; c < chunk; ++c) {
      if (fused && panels) {
        // after the operator: U^T Ap (+ p.Ap) and its partials' sum, coefficients (+ alpha),
        // the dual pass (+ x, s), beta (+ the refresh decision), p, the refresh of u = U^T r
        const double ub = lmp_elem_bytes(Us.fmt) * (double)nA * L->k, fl = 2.0 * (double)nA * L->k;
        if ((rc = apply_A_core(p, pv, nA, Ap, nA, 1, done, s))) return rc;
        {
          ProfScope ps(p, s, PROF_LMP_T, ub + 16.0 * nA, fl + 2.0 * nA);
          if (share_refresh)
            HIPCHK(p, lmp_pan16_t_partials_refresh(nA, L->k, Us, Ap, pv, L->wsv, pcg_dot_slots(p->pcgRed), done,
                                                   L->wsr, u, &st->no_refresh, s));
          else
            HIPCHK(p, lmp_pan_t_partials(nA, L->k, Us, Ap, pv, L->wsv, pcg_dot_slots(p->pcgRed), done, s));
        }
        HIPCHK(p, pcg_lmp_coeffs_pan(st, L->k, lmp_pan_t_splits(nA, L->k, Us.fmt), tvec, p->pcgRed, L->dcoef,
                                     L->GU, u, d12, s));
        {
          ProfScope ps(p, s, PROF_LMP_N, ub + 8.0 * 9.0 * nA, 2.0 * fl);
          HIPCHK(p, pcg_lmp_dual_pan(st, nA, L->k, Us, d12, Ap, r, z, x, sres, b, pv, p->pcgRed, p->pcgHist, s));
        }
        if (share_refresh) {
          HIPCHK(p, pcg_update_p_refresh16(st, pv, z, nA, L->k, Us, r, L->wsr, s));
        } else {
          HIPCHK(p, pcg_update_p(st, pv, z, nA, s));
          HIPCHK(p, lmp_gemv_t(nA, L->k, Us, nullptr, r, L->wsv, &st->no_refresh, s, u));
        }
        continue;
      }
      if (fused) {
        const double ub = 8.0 * (double)nA * L->k, fl = 2.0 * (double)nA * L->k;
        if ((rc = apply_A_core(p, pv, nA, Ap, nA, 1, done, s))) return rc;
        HIPCHK(p, pcg_dot_alpha(st, pv, Ap, nA, p->pcgRed, s));
        HIPCHK(p, pcg_update_xs(st, x, sres, b, pv, Ap, nA, p->pcgRed, s));
        {
          ProfScope ps(p, s, PROF_LMP_T, ub + 8.0 * nA, fl);
          HIPCHK(p, lmp_gemv_t(nA, L->k, Us, nullptr, Ap, L->wsv, done, s));
        }
        HIPCHK(p, pcg_lmp_coeffs(st, L->k, tvec, L->dcoef, L->GU, u, d12, s));
        {
          ProfScope ps(p, s, PROF_LMP_N, ub + 8.0 * 4.0 * nA, 2.0 * fl);
          HIPCHK(p, pcg_lmp_dual(st, nA, L->k, L->U, L->ldu, d12, Ap, r, z, p->pcgRed, p->pcgHist, s));
        }
        HIPCHK(p, pcg_update_p(st, pv, z, nA, s));
        // u = U^T r recomputed exactly when beta's kernel decided so (no_refresh = 0)
        HIPCHK(p, lmp_gemv_t(nA, L->k, Us, nullptr, r, L->wsv, &st->no_refresh, s, u));
        continue;
      }
      if ((rc = apply_A_core(p, pv, nA, Ap, nA, 1, done, s))) return rc;
      HIPCHK(p, pcg_dot_alpha(st, pv, Ap, nA, p->pcgRed, s));
      HIPCHK(p, pcg_update_xs(st, x, sres, b, pv, Ap, nA, p->pcgRed, s));
      if (ritz) {
        // z = P s; beta from s^T z; p = z + beta p
        if ((rc = ritz_apply_core(L, sres, nA, z, nA, 1, done, s))) return rc;
        HIPCHK(p, pcg_dot_rz(st, sres, z, nA, p->pcgRed, s));
        HIPCHK(p, pcg_beta_final(st, p->pcgRed, p->pcgHist, s));
        HIPCHK(p, pcg_update_p(st, pv, z, nA, s));
        continue;
      }
      const double* wv = Ap;
      if (L != nullptr) {
        if ((rc = lmp_apply_core(L, Ap, nA, w, nA, 1, done, s))) return rc;
        wv = w;
      }
      if (reorth) {
        // r_j -= F_j (F_j^T r_j), twice (classical Gram-Schmidt), over f_0..f_{j-1}
        const int j = it + c + 1;
        LmpU Fu;
        Fu.p = F;
        Fu.fmt = LMP_F64;
        Fu.ldu = ldf;
        double* tj = rws + rws_t;
        HIPCHK(p, pcg_update_r_only(st, r, wv, nA, p->pcgRed, s));
        HIPCHK(p, lmp_gemv_t(nA, j, Fu, nullptr, r, rws, done, s, tj));
        HIPCHK(p, pcg_reorth_sub(st, j, F, ldf, tj, r, z, nA, nullptr, s));
        HIPCHK(p, lmp_gemv_t(nA, j, Fu, nullptr, z, rws, done, s, tj));
        HIPCHK(p, pcg_reorth_sub(st, j, F, ldf, tj, z, r, nA, p->pcgRed, s));
        HIPCHK(p, pcg_beta_final(st, p->pcgRed, p->pcgHist, s));
      } else {
        HIPCHK(p, pcg_update_r(st, r, wv, nA, p->pcgRed, p->pcgHist, s));
      }
      if (F != nullptr) HIPCHK(p, pcg_lanczos_col(st, it + c + 1, r, F, ldf, nA, s));
      const double* zv = r;
      if (L != nullptr) {
        if ((rc = lmp_apply_core(L, r, nA, z, nA, 1, done, s))) return rc;
        zv = z;
      }
      HIPCHK(p, pcg_update_p(st, pv, zv, nA, s));
    }
    it += chunk;
    const int slot = issued & 1;
    HIPCHK(p, hipMemcpyAsync(p->pcgPoll[slot], st, sizeof(PcgState), hipMemcpyDeviceToHost, s));
    HIPCHK(p, hipEventRecord(p->pcgPollEv[slot], s));
    ++issued;
    ++pending;
   }
   if (pending == 0) break;  // maxit iterations enqueued and read back
   const int oldest = (issued - pending) & 1;
   HIPCHK(p, hipEventSynchronize(p->pcgPollEv[oldest]));
   --pending;
   if (p->pcgPoll[oldest]->done != 0) break;
  }
  HIPCHK(p, hipMemcpyAsync(p->pcgStateHost, st, sizeof(PcgState), hipMemcpyDeviceToHost, s));
  HIPCHK(p, hipStreamSynchronize(s));
  const PcgState hs = *p->pcgStateHost;
  info->iters = hs.iter;
  info->status = hs.done ? hs.status : WC4D_ENOCONV;
  info->relres_true = hs.bnorm2 > 0 ? std::sqrt(hs.ss / hs.bnorm2) : 0.0;
  info->relres_precond = hs.r0norm2 > 0 ? std::sqrt(hs.rr / hs.r0norm2) : 0.0;
  info->J = -0.5 * hs.xbs;
  if (hs.iter == 0) {
    info->relres_true = 0.0;
    info->relres_precond = 0.0;
  }
  const int ni = hs.iter;
  if (ni > 0) {
    if (hist_true) HIPCHK(p, hipMemcpy(hist_true, p->pcgHist, sizeof(double) * ni, hipMemcpyDeviceToHost));
    if (hist_precond)
      HIPCHK(p, hipMemcpy(hist_precond, p->pcgHist + opts->maxit, sizeof(double) * ni, hipMemcpyDeviceToHost));
    if (hist_J)
      HIPCHK(p, hipMemcpy(hist_J, p->pcgHist + 2 * opts->maxit, sizeof(double) * ni, hipMemcpyDeviceToHost));
    if (alphas)
      HIPCHK(p, hipMemcpy(alphas, p->pcgHist + 3 * opts->maxit, sizeof(double) * ni, hipMemcpyDeviceToHost));
    if (betas)
      HIPCHK(p, hipMemcpy(betas, p->pcgHist + 4 * opts->maxit, sizeof(double) * ni, hipMemcpyDeviceToHost));
  }
  return info->status;
}

}  // namespace

int wc4d_pcg(wc4d_problem p, wc4d_lmp L, const double* b, double* x, const wc4d_pcg_opts* opts,
             wc4d_pcg_info* info, double* hist_true, double* hist_precond, double* hist_J,
             hipStream_t s) {
  return pcg_run(p, L, b, x, opts, info, hist_true, hist_precond, hist_J, nullptr, nullptr, nullptr, 0, false,
                 s);
}

int wc4d_pcg_ritz(wc4d_problem p, wc4d_lmp L, const double* b, double* x, const wc4d_pcg_opts* opts,
                  wc4d_pcg_info* info, double* hist_true, double* hist_J, hipStream_t s) {
  if (L == nullptr) return p ? fail(p, WC4D_EINVAL, "pcg_ritz: an LMP is required") : WC4D_EINVAL;
  return pcg_run(p, L, b, x, opts, info, hist_true, nullptr, hist_J, nullptr, nullptr, nullptr, 0, false, s, true);
}

int wc4d_pcg_lanczos(wc4d_problem p, const double* b, double* x, const wc4d_pcg_opts* opts, wc4d_pcg_info* info,
                     double* alphas, double* betas, double* F, long long ldf, int flags, hipStream_t s) {
  if (!is_state_ok(p)) return p ? fail(p, WC4D_ESTATE, "not finalized") : WC4D_EINVAL;
  if (alphas == nullptr || betas == nullptr || F == nullptr || ldf < p->nA)
    return fail(p, WC4D_EINVAL, "pcg_lanczos: alphas, betas, F (ldf >= n_A) required");
  if ((flags & ~WC4D_LANCZOS_REORTH) != 0) return fail(p, WC4D_EINVAL, "pcg_lanczos: unknown flags");
  return pcg_run(p, nullptr, b, x, opts, info, nullptr, nullptr, nullptr, alphas, betas, F, ldf,
                 (flags & WC4D_LANCZOS_REORTH) != 0, s);
}

}  // extern "C"
