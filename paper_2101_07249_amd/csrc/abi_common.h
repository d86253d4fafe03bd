// Host-side helpers shared by the C-ABI translation units (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <string>

#include "wc4d_internal.h"

namespace wc4d {

inline int fail(wc4d_problem p, int code, const std::string& msg) {
  if (p != nullptr) p->err = msg;
  return code;
}

inline bool device_ok(int d) {
  int n = 0;
  return d >= 0 && hipGetDeviceCount(&n) == hipSuccess && d < n;
}

struct DevGuard {
  int prev = -1;
  bool changed = false;
  explicit DevGuard(int d) {
    if (hipGetDevice(&prev) == hipSuccess && prev != d) {
      changed = (hipSetDevice(d) == hipSuccess);
    }
  }
  ~DevGuard() {
    if (changed) (void)hipSetDevice(prev);
  }
};

#define HIPCHK(p, call)                                                                         \
  do {                                                                                          \
    hipError_t e_ = (call);                                                                     \
    if (e_ != hipSuccess)                                                                       \
      return fail((p), WC4D_EHIP, std::string(#call) + ": " + hipGetErrorString(e_));            \
  } while (0)

template <class T>
inline int dev_alloc(wc4d_problem p, T** ptr, size_t count) {
  if (*ptr != nullptr) {
    (void)hipFree(*ptr);
    *ptr = nullptr;
  }
  if (count == 0) count = 1;
  hipError_t e = hipMalloc((void**)ptr, count * sizeof(T));
  if (e != hipSuccess) {
    *ptr = nullptr;
    return fail(p, WC4D_ENOMEM, std::string("hipMalloc of ") + std::to_string(count * sizeof(T)) +
                                    " bytes failed: " + hipGetErrorString(e));
  }
  return WC4D_OK;
}

template <class T>
inline void dev_free(T** ptr) {
  if (*ptr != nullptr) (void)hipFree(*ptr);
  *ptr = nullptr;
}

inline int ensure_block(wc4d_problem p, long long m) {
  if (p->wsBlockCols >= m && p->wsStashCols >= m) return WC4D_OK;
  int rc = dev_alloc(p, &p->wsBlock, (size_t)p->nL * m);
  if (rc) return rc;
  p->wsBlockCols = m;
  rc = dev_alloc(p, &p->wsStash, (size_t)std::max(p->q, 1) * m);
  if (rc) return rc;
  p->wsStashCols = m;
  return WC4D_OK;
}

inline int ensure_gram(wc4d_problem p, size_t doubles) {
  if (p->wsGramDoubles >= doubles) return WC4D_OK;
  int rc = dev_alloc(p, &p->wsGram, doubles);
  if (rc) return rc;
  p->wsGramDoubles = doubles;
  return WC4D_OK;
}

inline bool is_state_ok(wc4d_problem p) { return p != nullptr && p->finalized; }

// ---- per-class kernel timing: an event pair around each timed launch group
inline hipEvent_t prof_event(wc4d_problem p) {
  if (p->evnext == p->evpool.size()) {
    hipEvent_t e = nullptr;
    // timing only: no system-scope fence on record (it stalls the stream for several us)
    if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
    p->evpool.push_back(e);
  }
  return p->evpool[p->evnext++];
}

struct ProfScope {
  wc4d_problem p;
  hipStream_t s;
  int cls;
  double bytes, flops;
  hipEvent_t a = nullptr;
  ProfScope(wc4d_problem p_, hipStream_t s_, int cls_, double bytes_, double flops_)
      : p(p_), s(s_), cls(cls_), bytes(bytes_), flops(flops_) {
    // one launch group in kprofEvery of each timed class is bracketed (the others run
    // without event records: each record leaves the stream idle for a few us)
    if (((p->kprof >> cls) & 1) && (p->kprofSeq[cls]++ % p->kprofEvery) == 0) {
      a = prof_event(p);
      if (a != nullptr) (void)hipEventRecord(a, s);
    }
  }
  ~ProfScope() {
    if (a == nullptr) return;
    hipEvent_t b = prof_event(p);
    if (b == nullptr) return;
    (void)hipEventRecord(b, s);
    p->recs.push_back(ProfRec{cls, a, b, bytes, flops});
  }
};

// Autotuned D^{1/2} tiles of block width m on p, or null (then the built-in heuristic).
inline const DsqrtTune* find_tune(wc4d_problem p, int m) {
  for (const auto& e : p->tune)
    if (e.first == m) return &e.second;
  return nullptr;
}

// Frees an LMP's device memory (its problem's device must be current).
void lmp_release(wc4d_lmp L);

// Build scratch: bufA / bufB (n_A + 4) x m, small matrices, block and Gram workspaces.
int ensure_build(wc4d_problem p, int m);

// Y = A X (Section 2.2, the first-level preconditioned Hessian) using the problem's
// block workspace, which must hold m columns (ensure_block).  mixed: split-bf16 D^{1/2}.
int apply_A_core(wc4d_problem p, const double* X, long long ldx, double* Y, long long ldy, int m,
                 const int* skip, hipStream_t s, int mixed = SPLIT_NONE);

}  // namespace wc4d
