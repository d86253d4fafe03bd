// Internal declarations of libwc4d: device data layout, kernel launchers and the
// problem / LMP handle structs.  Everything here is gfx950 (CDNA4) HIP.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <string>
#include <vector>

#include "wc4d.h"

namespace wc4d {

// Column map of a matrix whose columns are contiguous runs of doubles:
// column t starts at  (t / per) * ld + (base + t % per) * stride.
// A block of m vectors of length n_A = n (N+1) (ld >= n_A) viewed as the
// n x ((N+1) m) matrix of its time levels is {ld, N+1, 0, n}; its time-0
// columns are {ld, 1, 0, n}; its time-1..N columns are {ld, N, 1, n};
// a plain column-major matrix is {ld, 1, 0, 0}.
struct ColMap {
  long long ld;
  int per;
  int base;
  int stride;
  // product epilogues multiply the columns with t % per == 0 by scale0 (level 0 of a
  // time-level view; 1 = no scaling)
  double scale0 = 1.0;
  // a product's right operand is upper triangular (rows k > t of column t are zero): the
  // float64 product may stop each column tile's K loop at the tile's last column
  int upper = 0;
  __host__ __device__ inline long long off(int t) const {
    return (long long)(t / per) * ld + (long long)(base + t % per) * stride;
  }
  __host__ __device__ inline double colscale(int t) const { return (t % per == 0) ? scale0 : 1.0; }
};

inline ColMap plain_cols(long long ld) { return ColMap{ld, 1, 0, 0}; }
// columns of an upper triangular matrix (see ColMap::upper)
inline ColMap upper_cols(long long ld) {
  ColMap c{ld, 1, 0, 0};
  c.upper = 1;
  return c;
}

// ---------------------------------------------------------------- launchers
// All launchers enqueue on `s` and return hipError_t of the launch.

// C(:, t) = alpha * A * B(:, t) [+ E(:, t)] for t < ncol; A column-major M x K (lda),
// B columns K long via bmap, C / E columns M long via cmap / emap.  float64 MFMA.
// skip: optional device flag; when *skip != 0 the kernel returns immediately.
// ws (ws_doubles long, may be null): split-K partials for few-column products.
hipError_t gemm_f64(int M, int ncol, int K, double alpha, const double* A, long long lda,
                    const double* B, ColMap bmap, double* C, ColMap cmap, const double* E,
                    ColMap emap, const int* skip, hipStream_t s, double* ws = nullptr,
                    size_t ws_doubles = 0);

// Explicit tile shapes of gemm_f64 (the autotuner's candidates): split-K with 64 x 16 or
// 64 x 112 tiles (needs ws), plain 128 x 16, 128 x 128, 64 x 64, 32 x 32 tiles, or split-K
// 64 x 112 with each wave's A rows loaded straight into registers and a double-buffered B.
enum GemmTile { GEMM_AUTO = 0, GEMM_SPLIT_64x16, GEMM_SPLIT_64x112, GEMM_128x16, GEMM_128x128, GEMM_64x64,
                GEMM_32x32, GEMM_SPLIT_64x112_PA, GEMM_NTILES };
bool gemm_tile_feasible(int tile, int M, int ncol, int K, const double* ws, size_t ws_doubles);
hipError_t gemm_f64_tile(int tile, int splits, int M, int ncol, int K, double alpha, const double* A,
                         long long lda, const double* B, ColMap bmap, double* C, ColMap cmap, const double* E,
                         ColMap emap, const int* skip, hipStream_t s, double* ws, size_t ws_doubles);

// Two-segment few-column product (n1 in [1, 112], n2 in [0, 112]; n2 = 0: one segment): C(:, c1(t)) = A1 B(:, b1(t)) [+ E]
// for t < n1 and C(:, c2(t)) = A2 B(:, b2(t)) [+ E] for t < n2, A1 / A2 M x K with lda = M,
// one split-K launch plus one reduction.  ws: dsqrt2_ws_doubles(M, n1, n2, K).
size_t dsqrt2_ws_doubles(int M, int n1, int n2, int K);
hipError_t dsqrt2_f64(int M, int K, const double* B, double* C, const double* E, const double* A1,
                      ColMap b1, ColMap c1, ColMap e1, int n1, const double* A2, ColMap b2, ColMap c2,
                      ColMap e2, int n2, const int* skip, double* ws, size_t ws_doubles, hipStream_t s);

// Tile variants of the two-segment product (autotuner candidates): 0 = 64 rows, K step 32;
// 1 = 128 rows, K step 16; 2 = 128 rows, K step 32.  splits = 0 picks the count.
constexpr int DSQRT2_NVARIANTS = 3;
bool dsqrt2_feasible(int variant, int splits, int M, int n1, int n2, int K, size_t ws_doubles);
hipError_t dsqrt2_f64_v(int variant, int splits, int M, int K, const double* B, double* C, const double* E,
                        const double* A1, ColMap b1, ColMap c1, ColMap e1, int n1, const double* A2, ColMap b2,
                        ColMap c2, ColMap e2, int n2, const int* skip, double* ws, size_t ws_doubles,
                        hipStream_t s);

// G(i, j) = sum_k X(k, i) Y(k, j), i < m1, j < m2, k < K; X / Y columns via maps.
// Deterministic split-K: partial tiles then a fixed-order sum.  G column-major, ldg.
// ws must hold gram_ws_doubles(m1, m2, K) doubles.
size_t gram_ws_doubles(int m1, int m2, long long K);
hipError_t gram_f64(int m1, int m2, long long K, const double* X, ColMap xmap, const double* Y,
                    ColMap ymap, double* G, int ldg, double* ws, const int* skip, hipStream_t s);

// Split-bfloat16 GEMM (see gemm_bf16x3.hip): C(:, t) = alpha S B(:, t) [+ E(:, t)] with S
// given as row-major bf16 hi/lo parts (row i = S(i, 0..K-1)).
hipError_t split_bf16_rows(int M, int K, const double* S, long long lds, __bf16* Shi, __bf16* Slo,
                           hipStream_t s);
// Few-column products Y = S X on the int8 matrix cores by a 6-slice error-free splitting
// (gemm_oz.hip).  oz_split_matrix: slices of S (n x n, column-major, ld lds) into Ss
// (oz_slices_bytes(n)) and its row exponents es (oz_padded(n) ints), once.  oz_gemm:
// Y(:, j) = E(:, j) + sc_j (S X)(:, j) for the L columns X + j ldc (sc_0 = scale0, else 1),
// with Xs (oz_xs_bytes(n, L)), fs (oz_lpad(L) ints) and P (oz_partials_doubles(n, L))
// as scratch; every launch returns at once when *skip != 0.  oz_set_lds_limit: once per
// process, before the first oz_gemm (its LDS exceeds the 64 KB default).
int oz_padded(int n);
int oz_lpad(int L);
size_t oz_slices_bytes(int n);
size_t oz_xs_bytes(int n, int L);
size_t oz_partials_doubles(int n, int L);
hipError_t oz_split_matrix(const double* S, long long lds, int n, signed char* Ss, int* es, hipStream_t s);
hipError_t oz_gemm(int n, int L, const signed char* Ss, const int* es, const double* X, long long ldc,
                   double scale0, const double* E, double* Y, signed char* Xs, int* fs, double* P,
                   const int* skip, hipStream_t s);
hipError_t oz_set_lds_limit();

hipError_t gemm_bf16x3(int M, int ncol, int K, double alpha, const __bf16* Shi, const __bf16* Slo,
                       const double* B, ColMap bmap, double* C, ColMap cmap, const double* E,
                       ColMap emap, hipStream_t s);
// Fragment-major forms for products with many 256 x 256 tiles (see gemm_bf16x3.hip):
// split_bf16_frag_rows / split_f16_frag_rows split S (M x K, column-major, ld lds; the
// float16 form with the row exponents of split_f16_rows) once into F (bf16_frag_elems(M, K)
// elements); gemm_bf16x3_frag / gemm_fp16x3_frag split the columns of X into Xf
// (bf16_frag_elems(ncol, K) elements of workspace; the float16 form first fills colexp, ncol
// ints) and form C = alpha S X [+ E], with cmap.colscale applied.  split_use_frag: whether a
// product of that shape takes these forms (environment WC4D_SPLIT_GEMM_KERNEL=frag|tiled
// overrides the size rule).  split_frag_set_lds_limit: once per process before the first
// fragment-major product (its LDS exceeds the 64 KB default).
size_t bf16_frag_elems(int R, int K);
bool split_use_frag(int M, int ncol);
hipError_t split_bf16_frag_rows(int M, int K, const double* S, long long lds, __bf16* F, hipStream_t s);
hipError_t split_f16_frag_rows(int M, int K, const double* S, long long lds, const int* rowexp, _Float16* F,
                               hipStream_t s);
hipError_t gemm_bf16x3_frag(int M, int ncol, int K, double alpha, const __bf16* Sf, const double* B, ColMap bmap,
                            __bf16* Xf, double* C, ColMap cmap, const double* E, ColMap emap, hipStream_t s);
hipError_t gemm_fp16x3_frag(int M, int ncol, int K, double alpha, const _Float16* Sf, const int* rowexp,
                            const double* B, ColMap bmap, int* colexp, _Float16* Xf, double* C, ColMap cmap,
                            const double* E, ColMap emap, hipStream_t s);
hipError_t split_frag_set_lds_limit();
// Float16 form: S split per row with power-of-two row exponents (rowexp, M ints), X per
// column (colexp: ncol ints of workspace, filled by the call).  See gemm_bf16x3.hip.
hipError_t split_f16_rows(int M, int K, const double* S, long long lds, _Float16* Shi, _Float16* Slo, int* rowexp,
                          hipStream_t s);
hipError_t gemm_fp16x3(int M, int ncol, int K, double alpha, const _Float16* Shi, const _Float16* Slo,
                       const int* rowexp, const double* B, ColMap bmap, int* colexp, double* C, ColMap cmap,
                       const double* E, ColMap emap, hipStream_t s);
// D^{1/2} product precision of an operator apply: float64, split bfloat16 x3, split float16 x3
enum SplitMode { SPLIT_NONE = 0, SPLIT_BF16 = 1, SPLIT_FP16 = 2 };

// Tangent-linear sweeps.  P/X/W are blocks of m columns (leading dimension ld*).
// observation k at local point l of a sweep wavefront's extended range (l < 0: empty)
struct alignas(16) TwEntry {
  int k, l;
  double v;  // 1 / R_kk
};

struct SweepModel {
  int kind;                 // 0 advdiff, 1 l96
  int n, N;
  double ca, cb, cc;        // advdiff stencil: x'_j = ca x_{j-1} + cb x_j + cc x_{j+1}
  double dt;                // l96 RK4 step
  const double* stages;     // l96: device (N x 4 x n) RK4 stage inputs y1..y4 of every step
  const int* obs_off;       // device (N+2): time i's observations are [obs_off[i], obs_off[i+1])
  const int* obs_idx;       // device q grid indices
  const double* obs_rinv;   // device q values 1 / R_ii
  // advection-diffusion single-wave trapezoids (tw_pe = 0: not used): PE points per lane,
  // W owned points per wavefront, fixed-slot observation entries (see sweep.hip)
  int tw_pe, tw_W;
  const TwEntry* tw_e;
  double* tw_dummy;   // two device doubles (16-byte aligned): target of the stores of unowned slots
};

// Trapezoid shape for the advection-diffusion sweeps of one or a few columns (the
// smallest PE in {4, 8} with E = 64 PE, W = E - 2N > 0, n >= E and 8W >= E for PE = 4,
// 4W >= E for PE = 8) and the
// per (wavefront, level) observation slots; false when no shape fits or a wavefront's
// level holds more observations than its slots.
bool tw_setup(int n, int N, const std::vector<int>& off, const std::vector<int>& idx,
              const std::vector<double>& rinv, int* pe, int* W, std::vector<TwEntry>& ent);

// Forward sweep x_0 = p_0, x_{i+1} = M_i x_i + p_{i+1}.  Writes stash(k, c) =
// rinv[k] * x_{i(k)}[idx[k]] (ldst >= q) when stash != null, and every x_i into
// Xout when Xout != null.
hipError_t sweep_fwd(const SweepModel& md, const double* P, long long ldp, int m, double* stash,
                     long long ldst, double* Xout, long long ldx, const int* skip, hipStream_t s);
// Adjoint sweep w_N = z_N, w_i = z_i + M_i^T w_{i+1}.  z from the stash (z_i =
// H_i^T stash_i) when stash != null, else from the dense block Z.  Writes W.
hipError_t sweep_bwd(const SweepModel& md, const double* stash, long long ldst, const double* Z,
                     long long ldz, int m, double* W, long long ldw, const int* skip,
                     hipStream_t s);

// Dynamic LDS bytes the sweeps need for this model.
size_t sweep_lds_required(const SweepModel& md);

// Small dense float64 kernels (one workgroup unless stated); matrices column-major.
// Upper Cholesky in place: G = R^T R, strict lower set to 0; *status = 1 on a
// non-positive or non-finite pivot (status untouched otherwise).
hipError_t chol_upper(int m, double* G, int ldg, int* status, hipStream_t s);
// d[i] = |R(i, i)| (first) or d[i] *= |R(i, i)|, i < m.
hipError_t diag_accumulate(int m, const double* R, int ldr, double* d, bool first, hipStream_t s);
// *status = 2 when min d < tol * max d (or d has a non-finite entry).
hipError_t rank_check(int m, const double* d, double tol, int* status, hipStream_t s);
// G(i, i) += c * trace(G) for i < m (single workgroup).
hipError_t shift_diag_trace(int m, double* G, int ldg, double c, hipStream_t s);
// Rinv = R^{-1} for upper triangular R (one wavefront per column).
hipError_t tri_inv_upper(int m, const double* R, int ldr, double* Rinv, int ldi, hipStream_t s);
// C = alpha op(A) op(B), op = transpose when t* != 0; M x N result, inner K.
hipError_t small_gemm(int M, int N, int K, double alpha, const double* A, int lda, int tA,
                      const double* B, int ldb, int tB, double* C, int ldc, hipStream_t s);
// EVD of the symmetric positive definite part of K (m x m, m <= 512) by one-sided
// block Jacobi.  Outputs eigenvalues lam (decreasing) and eigenvectors V (m x m,
// ldv), each vector's largest-magnitude entry positive.  K is overwritten; ctrl:
// 2 device ints of scratch.  With sym = false K is taken as it is (any square F): the
// same iteration then gives the singular values of F in lam and its right singular
// vectors in V, i.e. the eigenpairs (lam^2, V) of F^T F without forming it.  With poll
// (two pinned ints and two events, owned by the caller) the host keeps two sweeps in
// flight and enqueues no more once a finished sweep has found the iteration converged
// (it waits on the events); without it all 20 sweeps are enqueued, the ones after
// convergence returning at once.  The results are the same either way.
struct EvdPoll {
  int* host[2];
  hipEvent_t ev[2];
};
hipError_t jacobi_evd(int m, double* K, int ldk, double* lam, double* V, int ldv, int* ctrl,
                      hipStream_t s, bool sym = true, const EvdPoll* poll = nullptr);
// B = A^T for m x m matrices (column-major).
hipError_t transpose_small(int m, const double* A, int lda, double* B, int ldb, hipStream_t s);
// theta[i] = f(lam[i]) for i < k: f = identity (mode 0), sqrt (mode 1) or square (mode 2);
// dcoef[i] = theta[i]^{-1/2} - 1 (the LMP's diagonal).
hipError_t ritz_finish(int k, const double* lam, int mode, double* theta, double* dcoef,
                       hipStream_t s);

// y = x + U diag(dcoef) U^T x for one vector; ws: lmp_gemv_ws_doubles(nA, k).
// Single vector: lmp_gemv_t leaves t = dcoef .* (U^T x) (or U^T x when dcoef is
// null) at ws + lmp_gemv_t_offset(nA, k), lmp_gemv_n then writes y = x + U t.
// ws: lmp_gemv_ws_doubles(nA, k).
size_t lmp_gemv_ws_doubles(long long nA, int k);
size_t lmp_gemv_t_offset(long long nA, int k);
// The U a pass streams: float64 column-major (leading dimension ldu), or a panel-major
// copy in float32 or float16: panel p holds rows [kPanel p, kPanel p + kPanel) of all k
// columns, column-major with leading dimension kPanel, at offset kPanel k p; rows at or
// past n_A are zero.  The float16 copy stores column c as U * 2^-cexp[c], cexp[c] chosen
// so that the column's largest magnitude lands in [2^14, 2^15).
constexpr int kPanel = 256;
__host__ __device__ inline long long lmp_panels(long long nA) { return (nA + kPanel - 1) / kPanel; }
enum LmpFmt { LMP_F64 = 0, LMP_P32 = 1, LMP_P16 = 2 };
struct LmpU {
  const void* p = nullptr;
  LmpFmt fmt = LMP_F64;
  long long ldu = 0;          // LMP_F64 only
  const int* cexp = nullptr;  // LMP_P16 only (k)
};
inline double lmp_elem_bytes(LmpFmt f) { return f == LMP_P16 ? 2.0 : (f == LMP_P32 ? 4.0 : 8.0); }
// Sum over the wavefront, the same value in every lane: DPP within rows of 16 (xor 1, xor 2,
// half-row and row mirrors), then two lane shuffles across the rows.
template <int CTRL>
__device__ inline double dpp_d(double v) {
  const int lo = __double2loint(v), hi = __double2hiint(v);
  return __hiloint2double(__builtin_amdgcn_update_dpp(hi, hi, CTRL, 0xf, 0xf, false),
                          __builtin_amdgcn_update_dpp(lo, lo, CTRL, 0xf, 0xf, false));
}
__device__ inline double wave_sum_d(double v) {
  v += dpp_d<0xB1>(v);   // quad_perm [1, 0, 3, 2]
  v += dpp_d<0x4E>(v);   // quad_perm [2, 3, 0, 1]
  v += dpp_d<0x141>(v);  // row_half_mirror
  v += dpp_d<0x140>(v);  // row_mirror
  v += __shfl_xor(v, 16, 64);
  v += __shfl_xor(v, 32, 64);
  return v;
}
// 4 consecutive panel rows of one column (a 16-byte float32 or 8-byte float16 load)
__device__ inline float4 pan_ld4(const float* p) { return *reinterpret_cast<const float4*>(p); }
__device__ inline float4 pan_ld4(const _Float16* p) {
  typedef _Float16 h4 __attribute__((ext_vector_type(4)));
  const h4 v = *reinterpret_cast<const h4*>(p);
  return make_float4((float)v[0], (float)v[1], (float)v[2], (float)v[3]);
}
// elements of a panel copy (either precision)
size_t lmp_panel_elems(long long nA, int k);
// blocks of a pass over all panels (at most 1024, an equal panel count each but the last)
int lmp_panel_grid(long long nA);
// P = panel copy of (float)U; Uround (optional, column-major, ldu) = (double)(float)U.
hipError_t lmp_to_panels(float* P, const double* U, long long ldu, long long nA, int k,
                         double* Uround, hipStream_t s);
// P = float16 panel copy of U with column exponents cexp (k ints, written here); Uround as
// above with the values the float16 copy represents.
hipError_t lmp_to_panels16(_Float16* P, int* cexp, const double* U, long long ldu, long long nA, int k,
                           double* Uround, hipStream_t s);
// out[0] = ||GU - I||_F and out[1] = min(0, min_i dcoef_i) (2 device doubles).
hipError_t lmp_copy_check(int k, const double* GU, const double* dcoef, double* out, hipStream_t s);
hipError_t lmp_gemv_t(long long nA, int k, const LmpU& U, const double* dcoef, const double* x, double* ws,
                      const int* skip, hipStream_t s, double* tout = nullptr);
hipError_t lmp_gemv_n(long long nA, int k, const LmpU& U, const double* x, double* y, const double* ws,
                      const int* skip, hipStream_t s);

// Vector kernels for PCG and the LMP (n_A long).
struct PcgState {
  double rr, rr_new, pAp, alpha, beta, bnorm2, r0norm2, ss, xbs;
  double tol;
  int iter, done, status, criterion, maxit, pad;
  double rr_ref;      // r.r at the last exact refresh of u = U^T r (fused variant)
  int last_refresh;   // iteration of that refresh
  int no_refresh;     // 1: skip this iteration's refresh
};
hipError_t pcg_kernels_init(PcgState* st, const double* b, const double* s0, const double* r0,
                            long long nA, double tol, int maxit, int criterion, double* red,
                            hipStream_t s);
// red: reduction workspace of pcg_red_doubles() doubles.
size_t pcg_red_doubles();
hipError_t pcg_dot_alpha(PcgState* st, const double* p, const double* Ap, long long nA,
                         double* red, hipStream_t s);
hipError_t pcg_update_xs(PcgState* st, double* x, double* sres, const double* b, const double* p,
                         const double* Ap, long long nA, double* red, hipStream_t s);
hipError_t pcg_update_r(PcgState* st, double* r, const double* w, long long nA, double* red,
                        double* hist, hipStream_t s);
hipError_t pcg_update_p(PcgState* st, double* p, const double* z, long long nA, hipStream_t s);
// r -= alpha w and the partials of r^T r, without the beta kernel (reorthogonalised CG
// recomputes them); y = x - F t over j <= 512 columns of F (+ the partials of y^T y when
// red != null); both skipped once st->done.
hipError_t pcg_update_r_only(PcgState* st, double* r, const double* w, long long nA, double* red, hipStream_t s);
hipError_t pcg_reorth_sub(const PcgState* st, int j, const double* F, long long ldf, const double* t,
                          const double* x, double* y, long long nA, double* red, hipStream_t s);
// Preconditioned CG with a preconditioner function: state from b, s0 and z0 = P s0 (r^T z
// in st->rr), the r^T z partials of an iteration, and beta / convergence from the partials.
hipError_t pcg_kernels_init_std(PcgState* st, const double* b, const double* s0, const double* z0, long long nA,
                                double tol, int maxit, int criterion, double* red, hipStream_t s);
hipError_t pcg_dot_rz(PcgState* st, const double* a, const double* b, long long nA, double* red, hipStream_t s);
hipError_t pcg_beta_final(PcgState* st, double* red, double* hist, hipStream_t s);
// out = -1/theta (k); a -= b (k; skipped when *skip != 0); y = x (n; skipped likewise)
hipError_t vec_neg_inv(const double* theta, double* out, int k, hipStream_t s);
hipError_t vec_sub_small(double* a, const double* b, int k, const int* skip, hipStream_t s);
hipError_t vec_copy_skip(double* y, const double* x, long long n, const int* skip, hipStream_t s);
// f_j = (-1)^j r_j / ||r_j|| into column j of F (ldf) when st->iter == j.
hipError_t pcg_lanczos_col(const PcgState* st, int j, const double* r, double* F, long long ldf, long long nA,
                           hipStream_t s);
hipError_t vec_copy(double* y, const double* x, long long n, hipStream_t s);
// Fused LMP inside PCG (see vec.hip): coefficients d1 = dcoef.*t, u <- u - alpha (t + GU d1),
// d2 = dcoef.*u into d12 (2k); then the dual pass updating r, writing z, and beta.  U as for
// lmp_gemv_t (float32: the panel copy).
hipError_t pcg_lmp_coeffs(const PcgState* st, int k, const double* t, const double* dcoef,
                          const double* GU, double* u, double* d12, hipStream_t s);
hipError_t pcg_lmp_dual(PcgState* st, long long nA, int k, const double* U, long long ldu,
                        const double* d12, const double* Ap, double* r, double* z, double* red,
                        double* hist, hipStream_t s);
// Panel copy (either precision): one U^T Ap pass that also sums p.Ap (lmp_pan_t_partials
// with pdot = p, dotpart = pcg_dot_slots(red); t = U^T Ap left at ws + lmp_gemv_t_offset),
// then pcg_lmp_coeffs_pan (p.Ap -> alpha, u, d12; sp = lmp_pan_t_splits), then the dual
// pass that also updates x and s (the true residual) and ends with beta.
int lmp_pan_t_splits(long long nA, int k, LmpFmt fmt);
hipError_t lmp_pan_t_partials(long long nA, int k, const LmpU& U, const double* x, const double* pdot,
                              double* ws, double* dotpart, const int* skip, hipStream_t s);
double* pcg_dot_slots(double* red);
// The fused PCG's launches over a float16 panel copy with the refresh of u = U^T r spread
// over two launches (same arithmetic and order as lmp_gemv_t's): the partials of U^T r
// (into rpart, lmp_pan16_refresh_doubles(nA, k)) ride in the p-update launch
// (pcg_update_p_refresh16), and their sum into u in the launch that sums the next
// iteration's U^T Ap partials (lmp_pan16_t_partials_refresh; u untouched when *no_refresh).
hipError_t lmp_pan16_t_partials_refresh(long long nA, int k, const LmpU& U, const double* x, const double* pdot,
                                        double* ws, double* dotpart, const int* skip, const double* rpart,
                                        double* u, const int* no_refresh, hipStream_t s);
size_t lmp_pan16_refresh_doubles(long long nA, int k);
hipError_t pcg_update_p_refresh16(const PcgState* st, double* p, const double* z, long long nA, int k,
                                  const LmpU& U, const double* r, double* rpart, hipStream_t s);
hipError_t pcg_lmp_coeffs_pan(PcgState* st, int k, int sp, const double* t, const double* red,
                              const double* dcoef, const double* GU, double* u, double* d12,
                              hipStream_t s);
hipError_t pcg_lmp_dual_pan(PcgState* st, long long nA, int k, const LmpU& U, const double* d12,
                            const double* Ap, double* r, double* z, double* x, double* sres,
                            const double* b, const double* p, double* red, double* hist, hipStream_t s);
hipError_t vec_scale_rows(double* T, int k, int m, int ldt, const double* dcoef, const int* skip,
                          hipStream_t s);
hipError_t stash_from_innov(const double* d, const double* rinv, double* stash, int q,
                            hipStream_t s);
hipError_t vec_fill(double* y, double v, long long n, hipStream_t s);
hipError_t vec_to_f32(float* y, const double* x, long long n, hipStream_t s);
hipError_t vec_to_f64(double* y, const float* x, long long n, hipStream_t s);
hipError_t pcg_x0_zero_flag(const double* x, long long n, double* red, int* flag, hipStream_t s);
hipError_t pcg_s0(const double* b, const double* Ax, const int* xzero, double* s0, long long n,
                  hipStream_t s);
hipError_t block_copy(double* Y, long long ldy, const double* X, long long ldx, long long rows,
                      int cols, hipStream_t s);

// Counter-based Gaussian start block (philox.hip).  philox_words: raw Philox-4x32-10 of
// count (counter, key) tuples (in: count x 6 words c0..c3 k0 k1; out: count x 4 words).
// gauss_block: G(r, c) for r < nrows, c < ncols = the N(0, 1) entry (r, col0 + c) of the
// block of `seed` (column-major, ldg).
hipError_t philox_words(const uint32_t* in, uint32_t* out, long long count, hipStream_t s);
hipError_t gauss_block(unsigned long long seed, long long nrows, int ncols, long long col0, double* G,
                       long long ldg, hipStream_t s);

// Learned sketch network (sketchnet.hip).  fp16 = _Float16; layouts there.
hipError_t net_features(int n, int N, const double* traj, const int* obs_off, const int* obs_idx,
                        const double* Om, long long ldo, int nz, int cp0, _Float16* X0, hipStream_t s);
size_t net_conv_lds_bytes(int cp);
hipError_t net_conv_hidden(int n, int T, int cp, const _Float16* X, const _Float16* W, const _Float16* b,
                           _Float16* H, hipStream_t s);
hipError_t net_conv_out(int n, int T, int cp, const _Float16* X, const _Float16* W, const _Float16* b,
                        double* G, long long ldg, hipStream_t s);
hipError_t net_conv_bwd_data(int n, int T, const _Float16* dH, const _Float16* Wt, const _Float16* Aprev,
                             _Float16* dHprev, hipStream_t s);
int net_wgrad_blocks(int n, int T);
hipError_t net_wgrad(int n, int T, int cp, const _Float16* X, const _Float16* dH, float* part, hipStream_t s);
hipError_t net_reduce(int nb, int len, const float* part, const float* scal, float* grad, hipStream_t s);
size_t net_scale_ws_doubles();
hipError_t net_loss_scale(long long P, const double* dG, long long ldg, double* ws, float* scal,
                          _Float16* dH, hipStream_t s);
hipError_t net_adam(long long len, float* th, float* m, float* v, const float* g, float lr, float b1, float b2,
                    float eps, float c1, float c2, _Float16* w16, hipStream_t s);
hipError_t net_to_f16(long long len, const float* th, _Float16* w16, hipStream_t s);
hipError_t net_pack_t(const _Float16* W, _Float16* Wt, hipStream_t s);
hipError_t loss_weights(int k, const double* theta, double* w, double* sums, hipStream_t s);
hipError_t loss_finish(int m, int k, const double* Sinv, const double* Tm, const double* sums, double* f,
                       double* M1, double* M2, hipStream_t s);

}  // namespace wc4d

// ------------------------------------------------------------------- handles

// Kernel classes timed by the in-library profiler (HIP events on the launch stream).
enum ProfClass {
  PROF_DSQRT = 0,   // D^{1/2} products inside the operator
  PROF_SWEEP_FWD,   // tangent-linear sweep + observation gather
  PROF_SWEEP_BWD,   // adjoint sweep + observation scatter
  PROF_LMP_T,       // U^T x pass of a single-vector LMP application
  PROF_LMP_N,       // x + U t pass of a single-vector LMP application
  PROF_BUILD,       // orthonormalisation, Gram, small dense and Ritz-vector kernels of a build
  PROF_DSQRT_BF16,  // split-bf16 D^{1/2} products (flops counted as the 3 bf16 products)
  PROF_NET,         // learned-sketch network inference (features + convolutions)
  PROF_NCLASS
};

struct ProfRec {
  int cls;
  hipEvent_t a, b;
  double bytes, flops;
};

// Tile choice of the D^{1/2} products for one block width m (set by the autotuner).
struct DsqrtTune {
  int tileB = 0;      // GemmTile of the B^{1/2} product (m columns)
  int tileQ = 0;      // GemmTile of the Q^{1/2} product (m N columns)
  bool twoSeg = false;  // the split-K segment kernel (two segments, or one with scaledB)
  int segVariant = 0;   // its tile variant and K splits (0: heuristic)
  int segSplits = 0;
  int tileAll = 0;      // GemmTile of the single product over all levels (B^{1/2} = c Q^{1/2})
  float ms = 0.f;     // measured time of the chosen form
};

struct wc4d_problem_s {
  int n = 0, N = 0, device = 0;
  long long nA = 0;          // control vector size: n (N+1), or n for a strong-constraint problem
  long long nL = 0;          // n (N+1): the time-level blocks of the sweeps
  bool strong = false;       // strong-constraint operator (control x_0 only)
  int q = 0;
  int model = -1;  // 0 advdiff, 1 l96
  double c = 0, r = 0, F = 8, dt = 0.025;
  std::vector<double> traj;  // (N+1) x n
  std::vector<double> Bsqrt, Qsqrt;
  std::vector<std::vector<int>> obs_idx;
  std::vector<std::vector<double>> obs_r;
  bool haveB = false, haveQ = false, finalized = false;
  int prec = 0;
  // device data
  double* dB = nullptr;
  double* dQ = nullptr;
  __bf16* dBhi = nullptr;  // split-bf16 B^{1/2}, Q^{1/2} (row-major), when prec has BF16X3
  __bf16* dBlo = nullptr;
  __bf16* dQhi = nullptr;
  __bf16* dQlo = nullptr;
  __bf16* dQf = nullptr;      // fragment-major split-bf16 Q^{1/2} (large products)
  _Float16* dQf16 = nullptr;  // the same in split float16 (scaled rows)
  __bf16* dXf = nullptr;      // fragment-major split of a product's right operand (workspace,
                              // 16-bit values of either form)
  size_t xfCap = 0;
  _Float16* dBh16 = nullptr;  // split-float16 B^{1/2}, Q^{1/2} (row-major, scaled rows), when prec has FP16X3
  _Float16* dBl16 = nullptr;
  _Float16* dQh16 = nullptr;
  _Float16* dQl16 = nullptr;
  int* dBexp = nullptr;       // their row exponents
  int* dQexp = nullptr;
  int* dColExp = nullptr;     // column exponents of a float16 product's right operand
  signed char* ozSs = nullptr;  // int8 slices of Q^{1/2} (WC4D_PREC_DSQRT_OZ7), see gemm_oz.hip
  int* ozEs = nullptr;          // their row exponents
  signed char* ozXs = nullptr;  // slices of one vector's levels (per product)
  int* ozFs = nullptr;
  double* ozP = nullptr;        // split-K partials
  size_t colExpCap = 0;
  double* dStages = nullptr;
  double* dTraj = nullptr;  // l96: (N+1) x n trajectory (sketch-network features)
  int* dObsOff = nullptr;
  int* dObsIdx = nullptr;
  double* dObsRinv = nullptr;
  int twPe = 0, twW = 0;     // single-wave sweep shape (advection-diffusion), 0: none
  wc4d::TwEntry* dTwE = nullptr;
  double* dTwDummy = nullptr;
  // workspaces (grown on demand)
  double* wsBlock = nullptr;  // n_A x cap
  long long wsBlockCols = 0;
  double* wsStash = nullptr;  // q x cap
  long long wsStashCols = 0;
  double* wsGram = nullptr;
  size_t wsGramDoubles = 0;
  double* wsSplit = nullptr;  // split-K partials of the few-column D^{1/2} products
  size_t wsSplitDoubles = 0;

  // LMP build scratch: two n_A x cap blocks and m x m matrices
  double* bufA = nullptr;
  double* bufB = nullptr;
  long long bufCols = 0;
  double* small = nullptr;  // 6 m x m + 2 m doubles
  int smallM = 0;
  int* dStatus = nullptr;   // device status words (0 build Cholesky, 1 PCG x0 == 0,
                            // 4-5 Jacobi control, 8 capture-loss Cholesky)
  double* lossWs = nullptr; // capture-loss small matrices
  size_t lossWsDoubles = 0;
  // PCG vectors and state
  double* pcgVec = nullptr;  // 6 n_A
  double* pcgHist = nullptr;
  int pcgHistCap = 0;
  double* pcgRed = nullptr;
  wc4d::PcgState* pcgState = nullptr;
  wc4d::PcgState* pcgStateHost = nullptr;  // pinned
  wc4d::PcgState* pcgPoll[2] = {nullptr, nullptr};  // pinned copies read while the next chunk runs
  hipEvent_t pcgPollEv[2] = {nullptr, nullptr};
  wc4d::EvdPoll evdPoll = {{nullptr, nullptr}, {nullptr, nullptr}};  // the build's Jacobi EVD
  // per-class kernel timing
  int kprof = 0;           // classes timed by ProfScope (bit c: class c)
  int kprofEvery = 1;      // ... one launch group in kprofEvery per class
  long long kprofSeq[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  std::vector<ProfRec> recs;
  std::vector<hipEvent_t> evpool;
  size_t evnext = 0;
  double profMs[PROF_NCLASS] = {0};
  double profBytes[PROF_NCLASS] = {0};
  double profFlops[PROF_NCLASS] = {0};
  long long profCalls[PROF_NCLASS] = {0};
  // profiling of the last apply
  bool prof = false;
  hipEvent_t ev[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  std::vector<wc4d_lmp> lmps;  // live LMPs built on this problem
  bool cholShift = false;       // LMP build: shifted CholeskyQR3 (set for a retry)
  bool scaledB = false;         // B^{1/2} = bScale Q^{1/2} (detected at finalize)
  double bScale = 1.0;
  std::vector<std::pair<int, DsqrtTune>> tune;  // autotuned D^{1/2} tiles per block width
  std::string err;
  wc4d::SweepModel sweep() const;
};

struct wc4d_lmp_s {
  wc4d_problem p = nullptr;  // null once the problem has been destroyed
  long long nA = 0;
  long long ldu = 0;        // leading dimension of U: n_A rounded up to 4
  int k = 0;
  int applies = 0;
  double* U = nullptr;      // n_A x k
  double* theta = nullptr;  // k
  double* dcoef = nullptr;  // k: theta^{-1/2} - 1
  double* T = nullptr;      // k x tcap scratch for U^T X
  int tcap = 0;
  double* ws = nullptr;     // gram workspace
  size_t wsDoubles = 0;
  double* wsv = nullptr;    // single-vector workspace
  size_t wsvDoubles = 0;
  double* wsr = nullptr;    // partials of the fused PCG's u = U^T r refresh (float16 copy)
  void* Up = nullptr;       // panel copy of U (WC4D_PREC_LMP_FP32 / _FP16), see kPanel
  wc4d::LmpFmt ufmt = wc4d::LMP_F64;  // format of the U the PCG streams
  int* cexp = nullptr;      // float16 copy: column exponents (k)
  double* AU = nullptr;     // n_A x k (ldu): A U for the Ritz-LMP (wc4d_lmp_ritz_prepare)
  double* ninv = nullptr;   // k: -1/theta
  double* rzw = nullptr;    // n_A + k scratch of a Ritz-LMP application
  double* GU = nullptr;     // k x k: U^T U of the U the PCG streams
  double* fu = nullptr;     // 3 k: u = U^T r, d1, d2 (fused PCG)
  // the U the passes stream: the panel copy when there is one, else U itself
  wc4d::LmpU streamed() const {
    wc4d::LmpU u;
    u.p = (Up != nullptr) ? (const void*)Up : (const void*)U;
    u.fmt = (Up != nullptr) ? ufmt : wc4d::LMP_F64;
    u.ldu = ldu;
    u.cexp = cexp;
    return u;
  }
};
