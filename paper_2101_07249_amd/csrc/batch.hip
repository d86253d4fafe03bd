// Batched inner loops and the tile autotuner (declared in include/wc4d.h).
//
// Autotuner: for a problem and block width m it times every feasible tile shape of the
// two D^{1/2} products (B^{1/2} on m columns, Q^{1/2} on m N columns; Section 2.2's
// D^{1/2} = blockdiag(B^{1/2}, Q^{1/2}, ...)) and the two-segment split-K form, keeps
// the fastest on the problem, and caches it per (device, n, N, m) for the process.
//
// Batch: independent problems are solved concurrently by host workers, each with its
// own non-blocking HIP stream, taking problems largest first from a shared counter;
// every problem runs the same LMP build (Section 4) and split PCG (Algorithm 1) as a
// single call would, so results are identical to one-by-one solves.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdio>
#include <map>
#include <mutex>
#include <numeric>
#include <thread>
#include <tuple>
#include <vector>

#include "abi_common.h"

using namespace wc4d;

namespace {

std::mutex g_tune_mu;
std::map<std::tuple<int, int, int, int, int>, DsqrtTune> g_tune_cache;  // (device, n, N, m, scaledB)

struct EvPair {
  hipEvent_t a = nullptr, b = nullptr;
  EvPair() {
    (void)hipEventCreateWithFlags(&a, hipEventDisableSystemFence);
    (void)hipEventCreateWithFlags(&b, hipEventDisableSystemFence);
  }
  ~EvPair() {
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
  }
};

// Mean ms of `reps` runs of launch() after one warm-up run; < 0 on a launch error.
template <class F>
float time_launch(hipStream_t s, EvPair& ev, F&& launch) {
  // one warm launch, timed alone to size the batches; then the best of three batches of
  // about 2 ms each (tile shapes of the one-vector products differ by ~1%)
  auto batch = [&](int reps) -> float {
    if (hipEventRecord(ev.a, s) != hipSuccess) return -1.f;
    for (int r = 0; r < reps; ++r)
      if (launch() != hipSuccess) return -1.f;
    if (hipEventRecord(ev.b, s) != hipSuccess || hipEventSynchronize(ev.b) != hipSuccess) return -1.f;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, ev.a, ev.b) != hipSuccess) return -1.f;
    return ms / reps;
  };
  const float one = batch(1);
  if (one < 0.f) return -1.f;
  const int reps = one > 0.f ? std::max(1, std::min(20, (int)(2.0f / one))) : 20;
  float best = -1.f;
  for (int t = 0; t < 3; ++t) {
    const float ms = batch(reps);
    if (ms < 0.f) return -1.f;
    if (best < 0.f || ms < best) best = ms;
  }
  return best;
}

void set_tune(wc4d_problem p, int m, const DsqrtTune& t) {
  for (auto& e : p->tune)
    if (e.first == m) {
      e.second = t;
      return;
    }
  p->tune.emplace_back(m, t);
}

}  // namespace

extern "C" {

int wc4d_autotune(wc4d_problem p, int m, hipStream_t s) {
  if (!is_state_ok(p)) return p ? fail(p, WC4D_ESTATE, "not finalized") : WC4D_EINVAL;
  if (p->strong) return fail(p, WC4D_EINVAL, "autotune: the tile table covers weak-constraint D^{1/2} products");
  if (m < 1 || m > 512) return fail(p, WC4D_EINVAL, "block width must be in [1, 512]");
  DevGuard g(p->device);
  const int n = p->n, N = p->N;
  const auto key = std::make_tuple(p->device, n, N, m, p->scaledB ? 1 : 0);
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune_cache.find(key);
    if (it != g_tune_cache.end()) {
      set_tune(p, m, it->second);
      return WC4D_OK;
    }
  }
  int rc = ensure_build(p, m);
  if (rc) return rc;
  const long long nA = p->nA;
  double* X = p->bufA;
  double* Y = p->bufB;
  HIPCHK(p, vec_fill(X, 0.5, nA * m, s));
  EvPair ev;
  if (p->scaledB) {
    // one product with Q^{1/2} over all levels
    const ColMap xa{nA, N + 1, 0, n};
    DsqrtTune best{};
    float bestAll = -1.f;
    for (int t = GEMM_AUTO + 1; t < GEMM_NTILES; ++t) {
      if (!gemm_tile_feasible(t, n, m * (N + 1), n, p->wsSplit, p->wsSplitDoubles)) continue;
      const float ms = time_launch(s, ev, [&] {
        return gemm_f64_tile(t, 0, n, m * (N + 1), n, 1.0, p->dQ, n, X, xa, Y, xa, X, xa, nullptr, s, p->wsSplit,
                             p->wsSplitDoubles);
      });
      if (ms >= 0.f && (bestAll < 0.f || ms < bestAll)) {
        bestAll = ms;
        best.tileAll = t;
      }
    }
    (void)hipGetLastError();
    if (bestAll < 0.f) return fail(p, WC4D_EHIP, "autotune: no tile shape could be timed");
    best.ms = bestAll;
    if ((long long)m * (N + 1) <= 112) {
      // the split-K segment kernel with one segment
      for (int v = 0; v < DSQRT2_NVARIANTS; ++v)
        for (int sp : {0, 4, 8, 16, 32}) {
          if (!dsqrt2_feasible(v, sp, n, m * (N + 1), 0, n, p->wsSplitDoubles)) continue;
          const float ms = time_launch(s, ev, [&] {
            return dsqrt2_f64_v(v, sp, n, n, X, Y, X, p->dQ, xa, xa, xa, m * (N + 1), nullptr, xa, xa, xa, 0, nullptr,
                                p->wsSplit, p->wsSplitDoubles, s);
          });
          (void)hipGetLastError();
          if (ms >= 0.f && ms < best.ms) {
            best.twoSeg = true;
            best.segVariant = v;
            best.segSplits = sp;
            best.ms = ms;
          }
        }
    }
    set_tune(p, m, best);
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache[key] = best;
    return WC4D_OK;
  }
  const ColMap x0{nA, 1, 0, n}, xq{nA, N, 1, n};
  float bestB = -1.f, bestQ = -1.f;
  int tileB = GEMM_AUTO, tileQ = GEMM_AUTO;
  for (int t = GEMM_AUTO + 1; t < GEMM_NTILES; ++t) {
    if (gemm_tile_feasible(t, n, m, n, p->wsSplit, p->wsSplitDoubles)) {
      const float ms = time_launch(s, ev, [&] {
        return gemm_f64_tile(t, 0, n, m, n, 1.0, p->dB, n, X, x0, Y, x0, X, x0, nullptr, s, p->wsSplit,
                             p->wsSplitDoubles);
      });
      if (ms >= 0.f && (bestB < 0.f || ms < bestB)) {
        bestB = ms;
        tileB = t;
      }
    }
    if (gemm_tile_feasible(t, n, m * N, n, p->wsSplit, p->wsSplitDoubles)) {
      const float ms = time_launch(s, ev, [&] {
        return gemm_f64_tile(t, 0, n, m * N, n, 1.0, p->dQ, n, X, xq, Y, xq, X, xq, nullptr, s, p->wsSplit,
                             p->wsSplitDoubles);
      });
      if (ms >= 0.f && (bestQ < 0.f || ms < bestQ)) {
        bestQ = ms;
        tileQ = t;
      }
    }
  }
  (void)hipGetLastError();
  if (bestB < 0.f || bestQ < 0.f) return fail(p, WC4D_EHIP, "autotune: no tile shape could be timed");
  DsqrtTune best{tileB, tileQ, false, 0, 0, 0, bestB + bestQ};
  if ((long long)m * N <= 112 && m <= 112) {
    for (int v = 0; v < DSQRT2_NVARIANTS; ++v)
      for (int sp : {0, 4, 8, 16, 32}) {
        if (!dsqrt2_feasible(v, sp, n, m * N, m, n, p->wsSplitDoubles)) continue;
        const float ms = time_launch(s, ev, [&] {
          return dsqrt2_f64_v(v, sp, n, n, X, Y, X, p->dQ, xq, xq, xq, m * N, p->dB, x0, x0, x0, m, nullptr,
                              p->wsSplit, p->wsSplitDoubles, s);
        });
        (void)hipGetLastError();
        if (ms >= 0.f && ms < best.ms) best = DsqrtTune{tileB, tileQ, true, v, sp, 0, ms};
      }
  }
  set_tune(p, m, best);
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune_cache[key] = best;
  return WC4D_OK;
}

int wc4d_autotune_info(wc4d_problem p, int m, int* tile_b, int* tile_q, int* two_segment, float* ms) {
  if (p == nullptr) return WC4D_EINVAL;
  const DsqrtTune* t = find_tune(p, m);
  if (t == nullptr) return fail(p, WC4D_ESTATE, "no autotuned shape for this block width");
  if (tile_b) *tile_b = t->tileAll ? t->tileAll : t->tileB;
  if (tile_q) *tile_q = t->tileAll ? 0 : t->tileQ;
  if (two_segment) *two_segment = t->twoSeg ? 1 + t->segVariant + 8 * t->segSplits : 0;
  if (ms) *ms = t->ms;
  return WC4D_OK;
}

int wc4d_autotune_save(const char* path) {
  if (path == nullptr) return WC4D_EINVAL;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  FILE* fp = std::fopen(path, "w");
  if (fp == nullptr) return WC4D_EINVAL;
  bool ok = std::fprintf(fp, "# wc4d autotune cache: device n N m scaled_b tile_b tile_q two_segment variant splits "
                             "tile_all ms\n") > 0;
  for (const auto& e : g_tune_cache) {
    const DsqrtTune& t = e.second;
    ok = ok && std::fprintf(fp, "%d %d %d %d %d %d %d %d %d %d %d %.6f\n", std::get<0>(e.first), std::get<1>(e.first),
                            std::get<2>(e.first), std::get<3>(e.first), std::get<4>(e.first), t.tileB, t.tileQ,
                            t.twoSeg ? 1 : 0, t.segVariant, t.segSplits, t.tileAll, (double)t.ms) > 0;
  }
  ok = (std::fclose(fp) == 0) && ok;
  return ok ? WC4D_OK : WC4D_EINVAL;
}

int wc4d_autotune_load(const char* path) {
  if (path == nullptr) return WC4D_EINVAL;
  FILE* fp = std::fopen(path, "r");
  if (fp == nullptr) return WC4D_EINVAL;
  std::map<std::tuple<int, int, int, int, int>, DsqrtTune> got;
  char line[256];
  bool ok = true;
  while (std::fgets(line, sizeof(line), fp) != nullptr) {
    if (line[0] == '#' || line[0] == '\n') continue;
    int d, n, N, m, sc, tb, tq, two, var, spl, ta;
    double ms;
    if (std::sscanf(line, "%d %d %d %d %d %d %d %d %d %d %d %lf", &d, &n, &N, &m, &sc, &tb, &tq, &two, &var, &spl, &ta,
                    &ms) != 12 ||
        (sc != 0 && sc != 1) || tb < GEMM_AUTO || tb >= GEMM_NTILES || tq < GEMM_AUTO || tq >= GEMM_NTILES ||
        ta < GEMM_AUTO || ta >= GEMM_NTILES || (sc == 0 && ta != GEMM_AUTO) || var < 0 || var >= DSQRT2_NVARIANTS ||
        spl < 0) {
      ok = false;
      break;
    }
    got[std::make_tuple(d, n, N, m, sc)] = DsqrtTune{tb, tq, two != 0, var, spl, ta, (float)ms};
  }
  std::fclose(fp);
  if (!ok) return WC4D_EINVAL;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  for (const auto& e : got) g_tune_cache[e.first] = e.second;
  return WC4D_OK;
}

int wc4d_batch_solve(wc4d_problem* ps, int count, int method, int k_r, int l, const double* const* G,
                     const double* const* b, double* const* x, const wc4d_pcg_opts* opts, wc4d_pcg_info* infos,
                     int* status, int workers, int autotune) {
  if (ps == nullptr || count < 1 || G == nullptr || b == nullptr || x == nullptr || opts == nullptr ||
      infos == nullptr || status == nullptr || workers < 1 || workers > 16)
    return WC4D_EINVAL;
  int device = -1;
  for (int i = 0; i < count; ++i) {
    if (!is_state_ok(ps[i]) || G[i] == nullptr || b[i] == nullptr || x[i] == nullptr) return WC4D_EINVAL;
    if (device < 0) device = ps[i]->device;
    if (ps[i]->device != device) return fail(ps[i], WC4D_EINVAL, "batch problems must share one device");
    for (int j = 0; j < i; ++j)
      if (ps[j] == ps[i]) return fail(ps[i], WC4D_EINVAL, "a problem appears twice in the batch");
  }
  DevGuard g(device);
  const int m = k_r + l;
  std::vector<int> order(count);
  std::iota(order.begin(), order.end(), 0);
  auto cost = [&](int i) {
    const double n = ps[i]->n, T = ps[i]->N + 1.0;
    return n * n * T + 64.0 * n * T;
  };
  std::stable_sort(order.begin(), order.end(), [&](int a, int c) { return cost(a) > cost(c); });
  for (int i = 0; i < count; ++i) status[i] = WC4D_OK;
  // set-up pass (one stream): tiles and the build scratch, so the workers allocate little
  hipStream_t s0 = nullptr;
  HIPCHK(ps[0], hipStreamCreateWithFlags(&s0, hipStreamNonBlocking));
  for (int i = 0; i < count; ++i) {
    int rc = autotune ? wc4d_autotune(ps[i], m, s0) : ensure_build(ps[i], m);
    if (rc == WC4D_OK && autotune) rc = wc4d_autotune(ps[i], 1, s0);
    if (rc != WC4D_OK) {
      (void)hipStreamDestroy(s0);
      return rc;
    }
  }
  (void)hipStreamSynchronize(s0);
  (void)hipStreamDestroy(s0);
  std::atomic<int> next{0};
  auto work = [&]() {
    (void)hipSetDevice(device);
    hipStream_t st = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
      for (int i = next.fetch_add(count); i < count; ++i) status[order[i]] = WC4D_EHIP;
      return;
    }
    for (int i = next.fetch_add(1); i < count; i = next.fetch_add(1)) {
      const int q = order[i];
      wc4d_lmp L = nullptr;
      int rc = wc4d_lmp_build(ps[q], method, k_r, l, G[q], 0, &L, st);
      if (rc == WC4D_OK) {
        rc = wc4d_pcg(ps[q], L, b[q], x[q], opts, &infos[q], nullptr, nullptr, nullptr, st);
        wc4d_lmp_destroy(L);
      }
      status[q] = rc;
    }
    (void)hipStreamSynchronize(st);
    (void)hipStreamDestroy(st);
  };
  const int nw = std::min(workers, count);
  std::vector<std::thread> pool;
  pool.reserve(nw);
  for (int w = 0; w < nw; ++w) pool.emplace_back(work);
  for (auto& t : pool) t.join();
  for (int i = 0; i < count; ++i)
    if (status[i] != WC4D_OK && status[i] != WC4D_ENOCONV && status[i] != WC4D_EBREAKDOWN) return status[i];
  return WC4D_OK;
}

}  // extern "C"
