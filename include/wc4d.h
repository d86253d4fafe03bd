/*
 * wc4d.h -- C-ABI of libwc4d.so: the inner loop of randomised-LMP preconditioned
 * forcing-formulation weak-constraint 4D-Var on one AMD MI355X (gfx950) GPU.
 *
 * Method: Dauzickaite, Lawless, Scott, van Leeuwen, "Randomised preconditioning
 * for the forcing formulation of weak constraint 4D-Var".  The library builds the
 * first-level preconditioned Hessian (Section 2.2, eq. forcing_1stlvl_prec)
 *     A = I + D^{1/2} L^{-T} H^T R^{-1} H L^{-1} D^{1/2},
 * estimates its leading eigenpairs with REVD / Nystrom / REVD_ritzit
 * (Section 4, Algorithms 3-5), forms the spectral LMP (Section 3.2, eqs.
 * spectral_LMP and spectral_LMP_factor) and solves A x = b with split PCG
 * (Section 3.1, Algorithm 1).
 *
 * Conventions shared by every call
 *   - n: state size per time level; N: number of model steps (N+1 levels t_0..t_N);
 *     n_A = n (N+1) is the size of the control vector (x_0, eta_1..eta_N).
 *   - A block of m vectors is a column-major n_A x m double array with leading
 *     dimension ld >= n_A.  Row i*n + j holds time level i, grid point j.
 *   - Host pointers are read during the call and may be freed on return
 *     (setup data is copied).  Device pointers (hipMalloc'ed, on the problem's
 *     device) are borrowed: they must stay valid until the stream reaches the
 *     point where the call's work ends.  Device calls are asynchronous on the
 *     given stream unless stated otherwise; stream 0 is the null stream.
 *   - Every function returns a status (WC4D_OK = 0 or a negative WC4D_E* code);
 *     no C++ exception crosses the ABI.  wc4d_last_error() describes the last
 *     failure on a handle.  A handle is not thread-safe; use one per thread.
 *   - Device arithmetic is float64 unless a precision mode says otherwise.
 */
#ifndef WC4D_H
#define WC4D_H

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct wc4d_problem_s* wc4d_problem; /* owns device copies of the setup data and workspaces */
typedef struct wc4d_lmp_s* wc4d_lmp;         /* owns U (n_A x k_r) and theta (k_r) on the device     */

enum {
  WC4D_OK = 0,
  WC4D_EINVAL = -1,     /* invalid argument (shape, index, pointer, enum value)            */
  WC4D_ENOMEM = -2,     /* device or host allocation failed                                */
  WC4D_EHIP = -3,       /* a HIP runtime call failed                                       */
  WC4D_ENOTSPD = -4,    /* Cholesky of a Gram/projected matrix met a non-positive pivot    */
  WC4D_EBREAKDOWN = -5, /* PCG breakdown: p^T A p <= 0 or not finite                       */
  WC4D_ENOCONV = -6,    /* PCG reached maxit without meeting the tolerance                 */
  WC4D_ESTATE = -7      /* call out of order (e.g. apply before finalize)                  */
};

enum { WC4D_CORR_SOAR = 0, WC4D_CORR_GAUSS = 1 };
/* Randomised eigendecompositions (Section 4): REVD (Algorithm 3), Nystrom (Algorithm 4),
 * REVD_ritzit (Algorithm 5), and the single-pass Nystrom that Section 6 proposes as
 * future work (the Nystrom approximation Y (G_4^T Y)^{-1} Y^T on G_4 = orth(G), Y = A G_4:
 * one product with A). */
enum { WC4D_REVD = 0, WC4D_NYSTROM = 1, WC4D_RITZIT = 2, WC4D_NYSTROM_1P = 3 };
enum { WC4D_RES_TRUE = 0, WC4D_RES_PRECOND = 1 };
/* Precision flags (wc4d_finalize).  FP64 everywhere by default.
 *   WC4D_PREC_SKETCH_BF16X3: the D^{1/2} products of the block applies inside
 *     wc4d_lmp_build run as three bfloat16 MFMA products with float32 accumulation
 *     (S_hi X_hi + S_hi X_lo + S_lo X_hi, S = S_hi + S_lo); CholeskyQR2, the m x m
 *     eigenproblem and everything in wc4d_pcg stay float64.  Products with at least 512
 *     output tiles of 256 x 256 take a kernel on operands pre-split into MFMA operand
 *     pieces (a workspace of 4 bytes per block entry that the problem keeps), the others an
 *     LDS-tiled kernel; both give the same bits (the same holds for the float16 form below).
 *     The environment variable WC4D_SPLIT_GEMM_KERNEL=frag or =tiled, read at each product,
 *     forces one of them.
 *   WC4D_PREC_SKETCH_FP16X3: the same three products in float16 (11 significant bits
 *     per part instead of 8), with power-of-two scaling per row of S and per column of X
 *     (largest magnitude brought to [2^14, 2^15)) so that the parts fit float16's range;
 *     excludes WC4D_PREC_SKETCH_BF16X3.
 *   WC4D_PREC_LMP_FP32: the LMP keeps a float32 copy of U that wc4d_pcg streams
 *     (products accumulate in float64; C stays exactly symmetric).
 *   WC4D_PREC_LMP_FP16: the same with a float16 copy, each column scaled by a power of
 *     two (largest magnitude brought to [2^14, 2^15)), half the bytes per pass; excludes
 *     WC4D_PREC_LMP_FP32.  Either copy changes the preconditioner by its rounding only, so
 *     PCG still solves A x = b; the iteration count may differ.
 *   WC4D_PREC_DSQRT_OZ7: the one-vector D^{1/2} products (wc4d_pcg's applies of A,
 *     wc4d_rhs, any wc4d_apply_A with m = 1) run on the int8 matrix cores by an error-free
 *     splitting into 6 slices of 7 bits per operand (the Ozaki scheme, in its integer
 *     form): per-row exponents of Q^{1/2} and per-column exponents of the vector's levels,
 *     exact int32 slice products, the 21 pairs of slices with t + u <= 7 combined in
 *     float64.  Error a few n 2^-42 relative to max|row of Q^{1/2}| max|level| (about 2e-11
 *     of a level's largest entry at n = 4096, inside the float64 parity bar of 1e-10); the
 *     int8 slices of Q^{1/2} take 6 n^2 bytes and are made once at wc4d_finalize.  Needs
 *     B^{1/2} = c Q^{1/2} (one product over all levels; WC4D_EINVAL otherwise). */
enum {
  WC4D_PREC_FP64 = 0,
  WC4D_PREC_SKETCH_BF16X3 = 1,
  WC4D_PREC_LMP_FP32 = 2,
  WC4D_PREC_SKETCH_FP16X3 = 4,
  WC4D_PREC_LMP_FP16 = 8,
  WC4D_PREC_DSQRT_OZ7 = 16
};

/* Library version (major*10000 + minor*100 + patch) and status-code names. */
int wc4d_version(void);
const char* wc4d_status_string(int status);

/* ---------------------------------------------------------------- setup -- */

/* Create a problem for state size n >= 1 and N >= 1 model steps on HIP device
 * `device`.  *out receives the handle.  Allocates nothing on the device yet. */
int wc4d_create(wc4d_problem* out, int n, int N, int device);
int wc4d_destroy(wc4d_problem p);
const char* wc4d_last_error(wc4d_problem p); /* valid until the next call on p */

/* Tangent-linear model M_i (Section 2.1, x_{i+1} = M_i x_i + p_{i+1}).
 * Advection-diffusion (Section 5.1's upwind advection plus explicit diffusion):
 *   (M x)_j = (c + r) x_{j-1} + (1 - c - 2r) x_j + r x_{j+1}, periodic in j,
 *   time-invariant; requires c >= 0, r >= 0, c + 2r <= 1. */
int wc4d_set_model_advdiff(wc4d_problem p, double c, double r);

/* Lorenz-96 (Section 5.2, eq. lorenz96), classical RK4 with step dt and forcing F.
 * traj: host, (N+1) x n row-major, the nonlinear trajectory x_0..x_N; M_i is the
 * exact derivative of the RK4 step taken from traj[i].  Requires n >= 4. */
int wc4d_set_model_l96(wc4d_problem p, const double* traj, double F, double dt);

/* Host helper: nonlinear Lorenz-96 RK4 trajectory from x0 (host, n doubles) into
 * traj (host, (N+1) x n row-major); traj[0] = x0. */
int wc4d_l96_trajectory(int n, int N, double F, double dt, const double* x0, double* traj);
/* The same with model error (eq. model: x_{i+1} = M(x_i) + eta_{i+1}): eta host, N x n
 * row-major, row i = eta_{i+1} (NULL: none).  For the outer loop's state x^(j) from
 * p^(j) = (x_0, eta_1..eta_N) (Section 2.1). */
int wc4d_l96_trajectory_forced(int n, int N, double F, double dt, const double* x0, const double* eta,
                               double* traj);

/* Host helper: sigma * C^{1/2}, the symmetric square root of sigma^2 C, where C
 * is the periodic correlation matrix C_ij = rho(d_ij), d_ij = (n/pi) sin(pi|i-j|/n)
 * (chordal distance, grid units), rho = SOAR (1 + d/L) e^{-d/L} or Gaussian
 * e^{-d^2/(2L^2)} (Section 5's B and Q families).  C is circulant, so the root
 * comes from its real discrete Fourier spectrum.  out: host, n x n column-major
 * (symmetric).  Returns WC4D_ENOTSPD if the spectrum has a negative value beyond
 * rounding. */
int wc4d_corr_sqrt(int n, int kind, double L, double sigma, double* out);

/* Symmetric square roots of B and of Q (Q_i = Q for i = 1..N), host, n x n
 * column-major, copied (Section 2.2: D^{1/2} = blockdiag(B^{1/2}, Q^{1/2}, ...)). */
int wc4d_set_Bsqrt(wc4d_problem p, const double* Bsqrt);
int wc4d_set_Qsqrt(wc4d_problem p, const double* Qsqrt);

/* Direct observations at time level i (0 <= i <= N): q_i distinct grid indices
 * idx[0..q_i) in [0, n) and the diagonal of R_i (rdiag, all > 0), host, copied.
 * Replaces any earlier observations at i.  Observations are stacked in increasing
 * i for wc4d_rhs's innovation vector. */
int wc4d_set_obs(wc4d_problem p, int i, int q_i, const int* idx, const double* rdiag);

/* Strong-constraint counterpart (the paper's Section 6 names strong-constraint 4D-Var as a
 * setting the approach carries over to).  With a perfect model the control is x_0 alone
 * and the operator becomes
 *     A_sc = I + B^{1/2} (sum_i M_{0->i}^T H_i^T R_i^{-1} H_i M_{0->i}) B^{1/2},
 * M_{0->i} = M_{i-1} ... M_0, of size n: the weak-constraint operator with the model-error
 * blocks removed.  Call before wc4d_finalize (WC4D_ESTATE after it) with on = 1: every block
 * and vector of the problem then has n_A = n rows (wc4d_dims reports it), Q^{1/2} need not
 * be set and is never applied, wc4d_apply_A / wc4d_rhs / wc4d_lmp_build / wc4d_pcg (and the
 * calls built on them) use A_sc and its right-hand side B^{1/2} w_0 (w the adjoint sweep of
 * H^T R^{-1} d) + bt.  Float64 products only: the split sketch flags, wc4d_apply_Linv /
 * LinvT / Dsqrt, the sketch network, wc4d_autotune and the persistent batch return
 * WC4D_EINVAL for such a problem.  on = 0 restores the weak-constraint operator. */
int wc4d_set_strong_constraint(wc4d_problem p, int on);
/* Upload everything to the device and allocate the operator's fixed data.
 * prec_mode: WC4D_PREC_FP64 or an OR of the WC4D_PREC_* flags.  Synchronous.
 * Setup calls after finalize return WC4D_ESTATE. */
int wc4d_finalize(wc4d_problem p, int prec_mode, hipStream_t s);

/* n_A and q = total number of observations (after finalize). */
int wc4d_dims(wc4d_problem p, int* n_A, int* q);

/* ------------------------------------------------------------- operator -- */

/* Y = A X for a block of m >= 1 vectors (Section 2.2, eq. forcing_1stlvl_prec):
 * D^{1/2} product, forward tangent-linear sweep, H^T R^{-1} H, adjoint sweep,
 * D^{1/2} product, plus X.  X and Y: device, n_A x m, ldx/ldy >= n_A; X and Y must
 * not overlap.  Uses workspace owned by p (grown on demand, synchronously). */
int wc4d_apply_A(wc4d_problem p, const double* X, int ldx, double* Y, int ldy, int m, hipStream_t s);

/* Y = A X with the D^{1/2} products in precision `prec` (WC4D_PREC_FP64,
 * WC4D_PREC_SKETCH_BF16X3 or WC4D_PREC_SKETCH_FP16X3; a split form needs its flag at
 * finalize, else WC4D_ESTATE).  For measuring
 * the error of the reduced-precision apply against the float64 one. */
int wc4d_apply_A_prec(wc4d_problem p, const double* X, int ldx, double* Y, int ldy, int m, int prec,
                      hipStream_t s);

/* Pieces of the operator, for testing and composition:
 *   Y = L^{-1} X   (x_0 = p_0, x_{i+1} = M_i x_i + p_{i+1}; Section 2.1)
 *   Y = L^{-T} X   (w_N = z_N, w_i = z_i + M_i^T w_{i+1})
 *   Y = D^{1/2} X  */
int wc4d_apply_Linv(wc4d_problem p, const double* X, int ldx, double* Y, int ldy, int m, hipStream_t s);
int wc4d_apply_LinvT(wc4d_problem p, const double* X, int ldx, double* Y, int ldy, int m, hipStream_t s);
int wc4d_apply_Dsqrt(wc4d_problem p, const double* X, int ldx, double* Y, int ldy, int m, hipStream_t s);

/* Right-hand side of eq. forcing_1stlvl_prec: rhs = bt + D^{1/2} L^{-T} H^T R^{-1} d.
 * d: device, q innovations stacked by increasing observed time, in each time in
 * wc4d_set_obs order.  bt: device n_A vector D^{-1/2} b, or NULL for zero (a first
 * inner loop).  rhs: device n_A. */
int wc4d_rhs(wc4d_problem p, const double* d, const double* bt, double* rhs, hipStream_t s);

/* -------------------------------------------------------- preconditioner -- */

/* Gaussian start block of Section 4 (Algorithms 3-5: G has independent N(0, 1) entries),
 * drawn on the device with Philox-4x32-10 (Salmon, Moraes, Dror and Shaw, SC 2011) and
 * the Box-Muller transform.  Entry (r, c) of the block of `seed` uses key (seed mod 2^32,
 * seed >> 32) and counter (r >> 1, c, 0, 0); the words w0..w3 give the uniforms
 * u1 = ((w0 >> 6) 2^26 + (w1 >> 6) + 1/2) 2^-52 and u2 from (w2, w3) likewise; even
 * rows hold sqrt(-2 ln u1) cos(2 pi u2), odd rows sqrt(-2 ln u1) sin(2 pi u2).
 * wc4d_gaussian_block writes entries (r, col0 + c), r < n_rows, c < n_cols, into G
 * (device on `device`, column-major, ldg >= n_rows), so a column range of a block can be
 * drawn separately with the same values.  WC4D_EINVAL for negative sizes, ldg < n_rows, a
 * null G with a non-empty block, col0 + n_cols > 2^32 or an invalid device. */
int wc4d_gaussian_block(int device, unsigned long long seed, long long n_rows, int n_cols, long long col0,
                        double* G, long long ldg, hipStream_t s);
/* The generator's raw words, for checking against its published known-answer vectors:
 * for t < count, out[4t..4t+3] = Philox-4x32-10 of counter ctr_key[6t..6t+3] under key
 * (ctr_key[6t+4], ctr_key[6t+5]).  ctr_key, out: device arrays on `device`. */
int wc4d_philox4x32_10(int device, const unsigned int* ctr_key, unsigned int* out, long long count,
                       hipStream_t s);

/* Randomised estimate of the k_r leading eigenpairs of A from a sketch of width
 * m = k_r + l (Section 4): method WC4D_REVD (Algorithm 3), WC4D_NYSTROM
 * (Algorithm 4), WC4D_RITZIT (Algorithm 5) or WC4D_NYSTROM_1P (single-pass Nystrom,
 * Section 6), then the spectral LMP
 * C = I + U (Theta^{-1/2} - I) U^T (eq. spectral_LMP_factor in closed form).
 * G: device n_A x m column-major (ld n_A) start matrix supplied by the caller, or NULL:
 * the build then draws the n_A x m Gaussian block of `seed` (wc4d_gaussian_block) on the
 * device into its own scratch (seed is ignored when G is given).
 * Orthonormalisation is CholeskyQR2 in float64; the
 * small problem is solved by one-sided Jacobi on the device (the m x m EVD for REVD,
 * the SVD of the triangular factor for Nystrom and ritzit).  *out receives a new LMP
 * handle.  Synchronises s at the end to report a Cholesky failure (WC4D_ENOTSPD) or a
 * Jacobi iteration that has not converged after 20 sweeps (WC4D_ENOCONV; no LMP is
 * returned then), and with WC4D_PREC_LMP_FP16 once more to check the float16 copy of U.
 * Requires 1 <= k_r, l >= 0, m <= n_A, m <= 512. */
int wc4d_lmp_build(wc4d_problem p, int method, int k_r, int l, const double* G,
                   unsigned long long seed, wc4d_lmp* out, hipStream_t s);

/* Ritz values theta (host, k_r doubles, decreasing).  Synchronous. */
int wc4d_lmp_theta(wc4d_lmp L, double* theta_host);
/* Ritz vectors U into device memory (n_A x k_r, ldu >= n_A). */
int wc4d_lmp_vectors(wc4d_lmp L, double* U, int ldu, hipStream_t s);
/* Y = C X for m vectors (C = C^T).  X, Y device n_A x m; must not overlap. */
int wc4d_lmp_apply(wc4d_lmp L, const double* X, int ldx, double* Y, int ldy, int m, hipStream_t s);
/* wc4d_lmp_apply for callers that cannot allocate device memory (code under graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): Y = C X for m = 1 or 2
 * vectors, X, Y device n_A x m (ldx, ldy >= n_A), not overlapping; the same kernels and
 * the same result bit for bit.  Allocates nothing: the partial sums of U^T x live in a
 * fixed 4 MiB device array (one per GPU, held until the process ends; its address is
 * looked up on the first call on each device).  The LMP needs at most that much
 * (lmp_gemv scratch for n_A and k_r), else WC4D_EINVAL; m > 2 or overlapping X and Y
 * give WC4D_EINVAL.  Every call on a GPU shares that GPU's array: calls that overlap in
 * time on one GPU (other streams, other threads) race and must be serialised by the
 * caller; calls on one stream are ordered. */
int wc4d_lmp_apply_noalloc(wc4d_lmp L, const double* X, int ldx, double* Y, int ldy, int m, hipStream_t s);
/* Block products with A spent by the build (Table 1: 2 / 2 / 1; single-pass Nystrom 1). */
int wc4d_lmp_applies(wc4d_lmp L, int* count);
/* The copy of U that the one- and two-vector passes stream (and wc4d_pcg with it):
 * *prec_flag = WC4D_PREC_LMP_FP16, WC4D_PREC_LMP_FP32 or 0 (U itself, float64).  A
 * problem finalized with WC4D_PREC_LMP_FP16 gets the float32 copy instead when the
 * float16 copy's Gram defect ||U~^T U~ - I||_F exceeds half of theta_max^{-1/2} (the
 * smallest eigenvalue of C for an orthonormal U), so that C stays positive definite. */
int wc4d_lmp_copy_format(wc4d_lmp L, int* prec_flag);
/* Frees L.  wc4d_destroy(p) releases the device memory of the LMPs still alive on p;
 * their handles then accept only wc4d_lmp_destroy (other calls return WC4D_ESTATE). */
int wc4d_lmp_destroy(wc4d_lmp L);

/* ---------------------------------------------------------------- solve -- */

typedef struct {
  double tol;     /* relative residual target (the paper uses 1e-6)                    */
  int maxit;      /* iteration cap                                                      */
  int criterion;  /* WC4D_RES_TRUE: ||b - A x|| / ||b|| (recursive, float64);
                     WC4D_RES_PRECOND: ||r_j|| / ||r_0|| of Algorithm 1's split residual */
  int variant;    /* with an LMP: WC4D_PCG_FUSED (default, 0) keeps u = U^T r_j as a
                     k-vector (u_j = u_{j-1} - alpha_j (t + U^T U diag(theta^{-1/2}-1) t),
                     t = U^T A p_{j-1}; refreshed from r_j every 50 iterations), so each
                     iteration streams U twice; WC4D_PCG_PLAIN (1) applies C^T and C
                     separately (four passes over U).  Both are Algorithm 1 in exact
                     arithmetic. */
} wc4d_pcg_opts;
enum { WC4D_PCG_FUSED = 0, WC4D_PCG_PLAIN = 1 };

typedef struct {
  int iters;             /* iterations taken                                          */
  int status;            /* WC4D_OK, WC4D_ENOCONV or WC4D_EBREAKDOWN                  */
  double relres_true;    /* ||s_j|| / ||b||, s_j the recursively updated b - A x_j     */
  double relres_precond; /* ||r_j|| / ||r_0||                                          */
  double J;              /* quadratic cost x^T A x / 2 - b^T x at the returned x        */
} wc4d_pcg_info;

/* Split preconditioned CG (Algorithm 1) on A x = b with P = C C^T from L (or no
 * second-level preconditioner when L is NULL).  b: device n_A; x: device n_A,
 * initial guess on entry, solution on exit.  hist_true / hist_precond / hist_J:
 * optional host arrays of length opts->maxit receiving the per-iteration
 * relative residuals and cost (NULL to skip).  Synchronous (returns after the
 * solve); the iteration itself runs on the device without host round trips
 * except a convergence poll every few iterations.  Returns the same status as
 * info->status. */
int wc4d_pcg(wc4d_problem p, wc4d_lmp L, const double* b, double* x, const wc4d_pcg_opts* opts,
             wc4d_pcg_info* info, double* hist_true, double* hist_precond, double* hist_J,
             hipStream_t s);

/* ------------------------------------------------------------ Ritz-LMP -- */
/* The Ritz-LMP of eq. Ritz_LMP (Section 3.2), built from an LMP's Ritz pairs (U, Theta):
 *     P = (I - U Theta^{-1} U^T A)(I - A U Theta^{-1} U^T) + U Theta^{-1} U^T.
 * It corrects for inexact pairs (P A U = U for Rayleigh-Ritz pairs) at the price of products
 * with A; the paper describes it and keeps the spectral LMP for its experiments.
 * wc4d_lmp_ritz_prepare computes and keeps A U (one block product with A over the k_r
 * Ritz vectors, float64, n_A x k_r extra device memory) and -1/theta; synchronous.  The
 * other two calls return WC4D_ESTATE until it has run on L. */
int wc4d_lmp_ritz_prepare(wc4d_lmp L, hipStream_t s);
/* Y = P X for m vectors (X, Y device n_A x m, not overlapping): per vector four passes over
 * n_A x k_r (U^T x, (AU) t, (AU)^T y, U t) with A U from wc4d_lmp_ritz_prepare. */
int wc4d_lmp_ritz_apply(wc4d_lmp L, const double* X, int ldx, double* Y, int ldy, int m, hipStream_t s);
/* Preconditioned CG on A x = b with the Ritz-LMP as the preconditioner function (P has no
 * split factor): r_0 = b - A x_0, z_0 = P r_0, p_0 = z_0; alpha = r^T z / p^T A p;
 * x += alpha p; r -= alpha A p; z = P r; beta = r_new^T z_new / r^T z; p = z + beta p.
 * With P = C C^T this is Algorithm 1 in exact arithmetic.  opts->variant is ignored;
 * WC4D_RES_TRUE stops on ||r|| / ||b|| (r the recursively updated true residual),
 * WC4D_RES_PRECOND on (r^T P r / r_0^T P r_0)^{1/2}, which info->relres_precond also
 * reports.  hist_true / hist_J as in wc4d_pcg.  Synchronous. */
int wc4d_pcg_ritz(wc4d_problem p, wc4d_lmp L, const double* b, double* x, const wc4d_pcg_opts* opts,
                  wc4d_pcg_info* info, double* hist_true, double* hist_J, hipStream_t s);

/* ------------------------------------- outer loop: the previous loop's LMP -- */
/* Algorithm 1 without a second-level preconditioner (C = I, plain CG on A x = b) that
 * also returns the Lanczos information of Section 3.4: the CG coefficients alpha_j and
 * beta_j (host arrays of opts->maxit doubles; entries 0..info->iters-1 are written) and the
 * Lanczos vectors f_j = (-1)^j r_j / ||r_j|| for j = 0..info->iters in the columns of F
 * (device, n_A x (opts->maxit + 1), ldf >= n_A).  The alternating sign makes F_j^T A F_j the
 * tridiagonal T_j with the positive off-diagonal of Section 3.4 (which writes r_j / ||r_j||).
 * flags: 0, or WC4D_LANCZOS_REORTH for complete reorthogonalisation (Section 3.4's remedy
 * for repeated 'ghost' Ritz values): each new residual r_j is orthogonalised twice against
 * f_0..f_{j-1} (classical Gram-Schmidt over the columns already in F) before r_j^T r_j and
 * beta_j are formed, which costs two passes over j columns per iteration and needs
 * opts->maxit <= 512; without it CG's residuals lose orthogonality once a Ritz value has
 * converged and T_j then repeats converged eigenvalues.  Unknown flags: WC4D_EINVAL.
 * Otherwise as wc4d_pcg. */
enum { WC4D_LANCZOS_REORTH = 1 };
int wc4d_pcg_lanczos(wc4d_problem p, const double* b, double* x, const wc4d_pcg_opts* opts, wc4d_pcg_info* info,
                     double* alphas, double* betas, double* F, long long ldf, int flags, hipStream_t s);
/* The k largest Ritz pairs of A from j CG iterations (Section 3.4): T_j from alphas[0..j)
 * and betas[0..j) (gamma_1 = 1/alpha_1, gamma_i = 1/alpha_i + beta_{i-1}/alpha_{i-1},
 * tau_i = sqrt(beta_i)/alpha_i), its eigenpairs by one-sided Jacobi on the device, Ritz
 * values theta (host, k, decreasing) and Ritz vectors U = F_j W (device n_A x k, ldu >= n_A)
 * with F_j the first j columns of F from wc4d_pcg_lanczos.  1 <= k <= j <= 512.
 * Synchronous; WC4D_ENOCONV if the Jacobi iteration has not converged. */
int wc4d_lanczos_pairs(wc4d_problem p, int j, const double* alphas, const double* betas, const double* F,
                       long long ldf, int k, double* U, long long ldu, double* theta, hipStream_t s);
/* A spectral LMP C = I + U (Theta^{-1/2} - I) U^T (eq. spectral_LMP_factor) on problem p
 * from given Ritz pairs: U device n_A x k (ldu >= n_A, copied), theta host (k, > 0) -- e.g.
 * pairs of the previous inner loop's Hessian from wc4d_lanczos_pairs, which precondition
 * the next inner loop (Sections 3.4 and 5.2).  The LMP streams its float64 U.  Synchronous. */
int wc4d_lmp_from_pairs(wc4d_problem p, int k, const double* U, long long ldu, const double* theta,
                        wc4d_lmp* out, hipStream_t s);

/* Per-stage timing of wc4d_apply_A.  With profiling enabled, every apply records
 * HIP events on its stream around its four stages; wc4d_last_apply_timing waits
 * for the last apply and returns the elapsed ms of [0] the first D^{1/2} product,
 * [1] the forward sweep with the observation gather, [2] the adjoint sweep with
 * the observation scatter, [3] the second D^{1/2} product plus X (ms4: 4 floats). */
int wc4d_set_profiling(wc4d_problem p, int enable);
int wc4d_last_apply_timing(wc4d_problem p, float* ms4);

/* Per-class kernel timing.  When enabled, the library brackets each timed launch
 * group with HIP events on the stream it launches on and accumulates, per class,
 * the elapsed device time, the number of launch groups and the algorithmic bytes
 * and flops of those launches (the minimum traffic and arithmetic the operation
 * needs, not counter readings).  Classes: 0 D^{1/2} products of the operator,
 * 1 forward sweep (+ observation gather), 2 adjoint sweep (+ scatter), 3 the U^T x
 * pass and 4 the x + U t pass of a single-vector LMP application, 5 the other
 * kernels of an LMP build, 6 the split-bfloat16 D^{1/2} products (flops counted as
 * the three bfloat16 products), 7 the learned-sketch network's inference (features and
 * convolutions; flops of the convolutions).  wc4d_prof_enable resets the totals and
 * times the classes whose bits are set in enable (bit c: class c; WC4D_PROF_ALL every
 * class, 0 none; each timed launch group adds two event records to the stream);
 * wc4d_prof_read waits for the recorded work and reports one class.  enable < 0 is
 * WC4D_EINVAL. */
enum { WC4D_PROF_DSQRT = 0, WC4D_PROF_SWEEP_FWD = 1, WC4D_PROF_SWEEP_BWD = 2, WC4D_PROF_LMP_T = 3,
       WC4D_PROF_LMP_N = 4, WC4D_PROF_BUILD = 5, WC4D_PROF_DSQRT_BF16 = 6,
       WC4D_PROF_NET = 7, WC4D_PROF_NCLASS = 8, WC4D_PROF_ALL = 0xFF };
int wc4d_prof_enable(wc4d_problem p, int enable);
/* Time one launch group in `every` (>= 1, default 1) of each class enabled above, counted
 * per class from the last wc4d_prof_enable: wc4d_prof_read then reports the bracketed groups
 * only (launches, ms, bytes, flops), an unbiased sample when the groups are alike.
 * WC4D_EINVAL for every < 1. */
int wc4d_prof_stride(wc4d_problem p, int every);
int wc4d_prof_read(wc4d_problem p, int cls, double* ms, long long* launches, double* bytes,
                   double* flops);

/* ------------------------------------------------ batched inner loops -- */
/* Tile autotuner for the D^{1/2} products (Section 2.2, D^{1/2} = blockdiag(B^{1/2},
 * Q^{1/2}, ..., Q^{1/2})) of p at block width m: times every feasible float64 tile
 * shape of the B^{1/2} (m columns) and Q^{1/2} (m N columns) products and the
 * two-segment split-K form, and makes the fastest the one p uses for that width.
 * Choices are cached per (device, n, N, m) for the life of the process, so later
 * problems of the same shape reuse them without timing.  Uses p's build scratch;
 * synchronises s.  wc4d_autotune_info reports the choice (tile codes: 1 split-K 64x16,
 * 2 split-K 64x112, 3 128x16, 4 128x128, 5 64x64, 6 32x32, 7 split-K 64x112 with A read
 * straight into registers and a double-buffered B tile; two_segment = 0 when the
 * products run separately, else 1 + variant + 8 * splits of the two-segment launch with
 * variant 0 = 64 rows / K step 32, 1 = 128 / 16, 2 = 128 / 32 and splits 0 = automatic)
 * and its measured ms.  When finalize found B^{1/2} = c Q^{1/2} (same correlation, other
 * variance) D^{1/2} is one product with Q^{1/2} over all N + 1 levels whose epilogue scales
 * level 0; then tile_b is that product's tile and tile_q is 0. */
int wc4d_autotune(wc4d_problem p, int m, hipStream_t s);
int wc4d_autotune_info(wc4d_problem p, int m, int* tile_b, int* tile_q, int* two_segment, float* ms);
/* Write / merge the process-wide autotune cache as text (one line per (device, n, N, m,
 * scaled_b): "device n N m scaled_b tile_b tile_q two_segment variant splits tile_all ms").  A loaded entry is used
 * by wc4d_autotune without timing, so separate processes run identical kernels.
 * WC4D_EINVAL on an unreadable file or a malformed line (nothing is merged then). */
int wc4d_autotune_save(const char* path);
int wc4d_autotune_load(const char* path);

/* Solve `count` independent inner loops (Section 2.2 / Algorithm 1) at once: for each
 * problem ps[i] (finalized, all on one device, none repeated) an LMP of k_r Ritz pairs
 * from the start block G[i] (device n_A(i) x (k_r + l)) by `method` (Section 4), then
 * split PCG on A x = b[i] with x[i] as initial guess and solution (device n_A(i)).
 * `workers` (1..16) host threads, each with its own non-blocking stream, take the
 * problems largest first; with autotune != 0 the D^{1/2} tiles of each problem are
 * tuned for widths k_r + l and 1 first.  infos[i] / status[i] receive each problem's
 * PCG report and return code.  Synchronous.  Returns WC4D_OK when every problem
 * returned WC4D_OK, WC4D_ENOCONV or WC4D_EBREAKDOWN (see status), else the first
 * other error. */
int wc4d_batch_solve(wc4d_problem* ps, int count, int method, int k_r, int l, const double* const* G,
                     const double* const* b, double* const* x, const wc4d_pcg_opts* opts,
                     wc4d_pcg_info* infos, int* status, int workers, int autotune);

/* The same many inner loops with every PCG iteration of every problem in ONE persistent
 * launch (Section 3.1, Algorithm 1 on each problem's A from Section 2.2; Section 4's
 * remark that the products of a block can run at the same time, taken across problems).
 * For each problem ps[i] (finalized advection-diffusion problems with n <= 8192, on one
 * device, none repeated): the LMP of k_r <= 64 Ritz pairs by `method` from the start block
 * G[i] (device n_A(i) x (k_r + l)), or, when G or G[i] is NULL, from the Gaussian block of
 * seed + i drawn on the device (wc4d_gaussian_block), built with the single-problem
 * kernels; s_0 = b[i] - A x[i] with them too.  Then one launch of a few workgroups per
 * compute unit runs the whole split PCG of all problems from a device work queue:
 * per iteration the two D^{1/2} products (64 x 64-level float64 MFMA tiles), the forward
 * and adjoint sweeps with the observation term (one workgroup each), one pass over U for
 * U^T (A p, r) and p^T A p, one pass for r, z, x and the true residual s, and p = z + beta p;
 * float64 dot products reduced in a fixed order.  The last workgroup to finish a phase of
 * a problem computes its scalars and enqueues the next phase, so problems of any size run
 * side by side and each stops on its own criterion.  flags: WC4D_BATCH_SWEEP_FP32 runs
 * the sweeps in float32 (products, LMP and reductions stay float64; the recursive
 * residual then no longer tracks b - A x below about 1e-6, so check the true residual).
 * x[i] is the initial guess on entry and the solution on exit; infos[i] / status[i] as
 * for wc4d_batch_solve; *kernel_ms (may be NULL) receives the persistent launch's time.
 * Synchronous.  Allocates its queue and per-problem vectors (~6 n_A + q doubles each).
 * Returns WC4D_EHIP if a queue wait exceeded 20 s (the launch then ends; no problem is
 * left running on the device). */
enum { WC4D_BATCH_SWEEP_FP32 = 1 };
/* Profile of the last persistent launch in this process: for each of the launch's 11
 * phases (0 C1 u = U^T s0, 1 C2 r0, 2 C3 u = U^T r0, 3 C4 p0 and first dots, 4 D1 first
 * D^{1/2} product, 5 forward sweep, 6 adjoint sweep, 7 D2 second D^{1/2} product + p, 8 T
 * U^T (A p, r) and p.Ap, 9 UP r, z, x, s updates, 10 P p update), then 11 the phase
 * transitions (scalar work and enqueueing), the summed workgroup-busy ms (ms[i]) and item
 * counts (count[i]); entry 12 holds the launch's elapsed ms and its workgroup count.
 * Copies min(n, 13) entries; returns 13 (WC4D_EINVAL for null arrays or n < 1). */
int wc4d_batch_persistent_profile(double* ms, long long* count, int n);
int wc4d_batch_solve_persistent(wc4d_problem* ps, int count, int method, int k_r, int l,
                                const double* const* G, unsigned long long seed, const double* const* b,
                                double* const* x, const wc4d_pcg_opts* opts, int flags, wc4d_pcg_info* infos,
                                int* status, double* kernel_ms);

/* ------------------------------------------------------- learned sketch -- */
/* The randomised eigendecompositions of Section 4 (Algorithms 3-5) start from a
 * Gaussian block G.  The sketch network replaces it by a block shaped to the problem:
 * per time level i, a periodic 1-D convolution net along the grid axis j with
 *   input channels  0..nz-1   the Gaussian block itself, Omega[i n + j, c];
 *                   nz        (x_i(j) - 2.3) / 3.6 of a Lorenz-96 trajectory (else 0);
 *                   nz + 1    1 where point j is observed at time i (Section 2.1, H_i);
 *                   nz + 2    i / N;
 *                   nz + 3    exp(-(t_next - i) / 5), t_next the first observed time >= i
 *                             (0 when there is none);
 *   layers          l = 1..L: H_l[c, j] = b_l[c] + sum_{c', t = -2..2} W_l[c, c', t + 2]
 *                   A_{l-1}[c', (j + t) mod n], A_l = tanh(H_l) for l < L;
 *   output          G[i n + j, c] = H_L[c, j], c < 64 (the 64-column start block).
 * Weights, biases and activations are float16 (weights rounded from a float32 master
 * copy), products accumulate in float32 on the matrix cores, G is float64.
 * Parameter vectors (host float32) are ordered per layer: W_l (c_out, c_in, t)
 * row-major, then b_l.  Training minimises the capture loss below with Adam.
 * Without a trained network the Gaussian block is the sketch (the fallback). */
typedef struct wc4d_sketchnet_s* wc4d_sketchnet;

/* layers in [2, 8], channels must be 64, width must be 5, noise_channels (nz) in
 * [0, 92].  Parameters start at zero (set them with wc4d_sketchnet_set_params). */
int wc4d_sketchnet_create(wc4d_sketchnet* out, int layers, int channels, int width, int noise_channels,
                          int device);
int wc4d_sketchnet_destroy(wc4d_sketchnet net);
const char* wc4d_sketchnet_last_error(wc4d_sketchnet net);
int wc4d_sketchnet_nparams(wc4d_sketchnet net, long long* count);
/* Host float32 parameter vectors (count = wc4d_sketchnet_nparams).  set_params also
 * resets the Adam moments and step count.  Synchronous. */
int wc4d_sketchnet_set_params(wc4d_sketchnet net, const float* theta);
int wc4d_sketchnet_get_params(wc4d_sketchnet net, float* theta);
/* Gradient of the last backward pass (unscaled), or one set by the caller. */
int wc4d_sketchnet_get_grad(wc4d_sketchnet net, float* grad);
int wc4d_sketchnet_set_grad(wc4d_sketchnet net, const float* grad);

/* G (device n_A x 64, ldg >= n_A) = net(features of p, Omega); Omega: device n_A x nz
 * float64 (ldo >= n_A), the Gaussian block.  Keeps the activations for a following
 * wc4d_sketchnet_backward.  p must be finalized. */
int wc4d_sketchnet_infer(wc4d_sketchnet net, wc4d_problem p, const double* Omega, int ldo, double* G,
                         int ldg, hipStream_t s);
/* Gradient with respect to the parameters of sum(dG .* G) for the last inference
 * (dG device n_A x 64).  dG is scaled by a power of two into float16 range for the
 * backward convolutions and the gradient unscaled in float32. */
int wc4d_sketchnet_backward(wc4d_sketchnet net, const double* dG, int lddg, hipStream_t s);
/* One Adam step (Kingma and Ba; beta1 0.9, beta2 0.999, eps 1e-8) with the current
 * gradient and learning rate lr. */
int wc4d_sketchnet_adam(wc4d_sketchnet net, double lr, hipStream_t s);
/* Capture loss of a start block G (device n_A x m, m <= 512) against reference Ritz
 * pairs (U device n_A x k with ldu, theta device k, theta > 1): with Y = A G,
 * S = Y^T Y, w = 1 - 1/theta and P_w = U diag(w) U^T,
 *     f = -trace(S^{-1} Y^T P_w Y) / sum(w),
 * the weighted share of range(U) captured by range(Y), the block the algorithms
 * orthonormalise.  Writes f (device double) and dG = df/dG = A (2 / sum w)
 * (Y S^{-1} T S^{-1} - P_w Y S^{-1}), T = Y^T P_w Y (device n_A x m, lddg), using
 * the symmetry of A.  Synchronous only on error checks: returns WC4D_ENOTSPD
 * when S is singular (checked after the call's work completes). */
int wc4d_sketch_loss(wc4d_problem p, const double* G, int ldg, int m, const double* U, int ldu,
                     const double* theta, int k, double* f, double* dG, int lddg, hipStream_t s);
/* One training step on problem p: G = net(p, Omega), the capture loss against the
 * first k Ritz pairs of the reference LMP ref (built on p from a wider sketch), the
 * backward pass and an Adam step with rate lr.  *loss (host, may be NULL) receives f
 * at the step's parameters.  Synchronous. */
int wc4d_sketchnet_train_step(wc4d_sketchnet net, wc4d_problem p, const double* Omega, int ldo,
                              wc4d_lmp ref, int k, double lr, double* loss, hipStream_t s);
/* LMP build from the learned sketch: G = net(p, Omega) (requires k_r + l = 64 and nz =
 * 64), then wc4d_lmp_build; if that finds the block rank deficient (WC4D_ENOTSPD), or
 * net is NULL, the build uses the Gaussian block Omega itself.  *used_net (may be
 * NULL) tells which. */
int wc4d_lmp_build_sketch(wc4d_problem p, wc4d_sketchnet net, int method, int k_r, int l,
                          const double* Omega, wc4d_lmp* out, int* used_net, hipStream_t s);
/* Save / load the parameters (binary: "WC4DSKN1", int32 layers, channels, width,
 * noise_channels, int64 count, float32 parameters). */
int wc4d_sketchnet_save(wc4d_sketchnet net, const char* path);
int wc4d_sketchnet_load(wc4d_sketchnet* out, const char* path, int device);

#ifdef __cplusplus
}
#endif
#endif /* WC4D_H */
