"""FP64 CPU oracle for the inner loop of randomised-LMP preconditioned
forcing-formulation weak-constraint 4D-Var (Dauzickaite, Lawless, Scott and
van Leeuwen, "Randomised preconditioning for the forcing formulation of weak
constraint 4D-Var").

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the bench's
CPU-baseline leg may import this module.  It shares no code with the HIP
library or its Python binding and imports nothing from them; the product path
never calls it.

Plain, slow, obviously correct numpy in float64.  Library primitives used as
single steps: numpy.linalg.qr (Householder), eigh, svd, cholesky and
scipy.linalg.solve_triangular.  There is no blocking, fusion or reordering
beyond what the paper's equations and algorithms state.

Conventions (readings of the paper where it is silent):
  * blocks of vectors are arrays of shape (n_A, m), n_A = n (N+1), row index
    i*n + j (time level i, grid point j);
  * x_{i+1} = M_i x_i + p_{i+1}, M_i the tangent-linear model of the step from
    t_i (Section 2.1, the L^{-1} block structure);
  * the operator is the first-level preconditioned Hessian
    A = I + D^{1/2} L^{-T} H^T R^{-1} H L^{-1} D^{1/2} (Section 2.2);
  * eigenpairs are sorted by decreasing value; eigenvector signs are not
    fixed because every downstream use (U U^T, the LMP, Theta) is sign-free.
"""
from __future__ import annotations

import functools
from dataclasses import dataclass, field
from typing import Callable, Dict, List, Optional, Tuple

import numpy as np
import scipy.linalg as sla

# ---------------------------------------------------------------------------
# Models (Section 5.1: upwind advection, here with explicit diffusion;
# Section 5.2: Lorenz-96 integrated with classical RK4)
# ---------------------------------------------------------------------------


def advdiff_step(x: np.ndarray, c: float, r: float) -> np.ndarray:
    """One step of periodic upwind advection (Courant number c > 0) plus
    explicit diffusion (number r), acting along axis 0:
        x'_j = (c + r) x_{j-1} + (1 - c - 2r) x_j + r x_{j+1}.
    Linear, so it is its own tangent-linear model."""
    return (c + r) * np.roll(x, 1, axis=0) + (1.0 - c - 2.0 * r) * x + r * np.roll(x, -1, axis=0)


def advdiff_step_T(w: np.ndarray, c: float, r: float) -> np.ndarray:
    """Transpose of advdiff_step: (M^T w)_j = (c + r) w_{j+1} + (1 - c - 2r) w_j + r w_{j-1}."""
    return (c + r) * np.roll(w, -1, axis=0) + (1.0 - c - 2.0 * r) * w + r * np.roll(w, 1, axis=0)


def l96_rhs(x: np.ndarray, F: float) -> np.ndarray:
    """Lorenz-96 tendency (Section 5.2, eq. lorenz96), cyclic in j (axis 0):
    dX^j/dt = -X^{j-2} X^{j-1} + X^{j-1} X^{j+1} - X^j + F."""
    xm2 = np.roll(x, 2, axis=0)
    xm1 = np.roll(x, 1, axis=0)
    xp1 = np.roll(x, -1, axis=0)
    return -xm2 * xm1 + xm1 * xp1 - x + F


def l96_rk4_step(x: np.ndarray, F: float, dt: float) -> np.ndarray:
    """Classical fourth-order Runge-Kutta step of the Lorenz-96 system."""
    k1 = l96_rhs(x, F)
    k2 = l96_rhs(x + 0.5 * dt * k1, F)
    k3 = l96_rhs(x + 0.5 * dt * k2, F)
    k4 = l96_rhs(x + dt * k3, F)
    return x + (dt / 6.0) * (k1 + 2.0 * k2 + 2.0 * k3 + k4)


def l96_trajectory(x0: np.ndarray, F: float, dt: float, N: int) -> np.ndarray:
    """Nonlinear trajectory x_0..x_N (eq. model with zero model error), shape (N+1, n)."""
    traj = np.empty((N + 1, x0.shape[0]))
    traj[0] = x0
    for i in range(N):
        traj[i + 1] = l96_rk4_step(traj[i], F, dt)
    return traj


def _l96_jac(y: np.ndarray, d: np.ndarray) -> np.ndarray:
    """Jacobian of the L96 tendency at y applied to d (d may carry extra columns)."""
    if d.ndim == 2:
        y = y[:, None]
    ym2 = np.roll(y, 2, axis=0)
    ym1 = np.roll(y, 1, axis=0)
    yp1 = np.roll(y, -1, axis=0)
    dm2 = np.roll(d, 2, axis=0)
    dm1 = np.roll(d, 1, axis=0)
    dp1 = np.roll(d, -1, axis=0)
    return (dp1 - dm2) * ym1 + (yp1 - ym2) * dm1 - d


def _l96_jac_T(y: np.ndarray, a: np.ndarray) -> np.ndarray:
    """Transpose of _l96_jac: (J^T a)_j = y_{j-2} a_{j-1} - y_{j+1} a_{j+2}
    + (y_{j+2} - y_{j-1}) a_{j+1} - a_j."""
    if a.ndim == 2:
        y = y[:, None]
    ym2 = np.roll(y, 2, axis=0)
    ym1 = np.roll(y, 1, axis=0)
    yp1 = np.roll(y, -1, axis=0)
    yp2 = np.roll(y, -2, axis=0)
    am1 = np.roll(a, 1, axis=0)
    ap1 = np.roll(a, -1, axis=0)
    ap2 = np.roll(a, -2, axis=0)
    return ym2 * am1 - yp1 * ap2 + (yp2 - ym1) * ap1 - a


def _l96_stages(x: np.ndarray, F: float, dt: float):
    """Inputs of the four RK4 stage evaluations at trajectory point x."""
    k1 = l96_rhs(x, F)
    y2 = x + 0.5 * dt * k1
    k2 = l96_rhs(y2, F)
    y3 = x + 0.5 * dt * k2
    k3 = l96_rhs(y3, F)
    y4 = x + dt * k3
    return x, y2, y3, y4


def l96_tlm_step(x: np.ndarray, dx: np.ndarray, F: float, dt: float) -> np.ndarray:
    """Tangent-linear model M_i: the exact derivative of l96_rk4_step at x applied to dx."""
    y1, y2, y3, y4 = _l96_stages(x, F, dt)
    d1 = _l96_jac(y1, dx)
    d2 = _l96_jac(y2, dx + 0.5 * dt * d1)
    d3 = _l96_jac(y3, dx + 0.5 * dt * d2)
    d4 = _l96_jac(y4, dx + dt * d3)
    return dx + (dt / 6.0) * (d1 + 2.0 * d2 + 2.0 * d3 + d4)


def l96_adj_step(x: np.ndarray, a: np.ndarray, F: float, dt: float) -> np.ndarray:
    """Adjoint M_i^T of l96_tlm_step (reverse-mode sweep through the RK4 stages)."""
    y1, y2, y3, y4 = _l96_stages(x, F, dt)
    ax = a.copy()
    a1 = (dt / 6.0) * a
    a2 = (dt / 3.0) * a
    a3 = (dt / 3.0) * a
    a4 = (dt / 6.0) * a
    u4 = _l96_jac_T(y4, a4)
    ax = ax + u4
    a3 = a3 + dt * u4
    u3 = _l96_jac_T(y3, a3)
    ax = ax + u3
    a2 = a2 + 0.5 * dt * u3
    u2 = _l96_jac_T(y2, a2)
    ax = ax + u2
    a1 = a1 + 0.5 * dt * u2
    ax = ax + _l96_jac_T(y1, a1)
    return ax


# ---------------------------------------------------------------------------
# Covariances (Section 5: R_i = sigma_o^2 I, B = sigma_b^2 C_b, Q = sigma_q^2 C_q)
# ---------------------------------------------------------------------------


def chordal_distance(n: int) -> np.ndarray:
    """Distance (in grid units) between points i, j of a periodic grid of n
    points placed on a circle of circumference n: (n/pi) sin(pi |i-j| / n)."""
    k = np.abs(np.arange(n)[:, None] - np.arange(n)[None, :])
    return (n / np.pi) * np.sin(np.pi * k / n)


def correlation_matrix(n: int, kind: str, L: float) -> np.ndarray:
    """SOAR rho(d) = (1 + d/L) exp(-d/L) or Gaussian rho(d) = exp(-d^2 / (2 L^2))."""
    d = chordal_distance(n)
    if kind == "soar":
        return (1.0 + d / L) * np.exp(-d / L)
    if kind == "gauss":
        return np.exp(-(d * d) / (2.0 * L * L))
    raise ValueError(kind)


def sym_sqrt(C: np.ndarray) -> np.ndarray:
    """Symmetric square root (Section 2.2: D = D^{1/2} D^{1/2}) by dense EVD."""
    lam, V = np.linalg.eigh(C)
    if lam.min() < -1e-10 * lam.max():
        raise ValueError("matrix is not positive semidefinite")
    lam = np.clip(lam, 0.0, None)
    return (V * np.sqrt(lam)) @ V.T


@functools.lru_cache(maxsize=2)
def _corr_sqrt(n: int, kind: str, L: float) -> np.ndarray:
    """C^{1/2} of one correlation family (kept for reuse: B and Q often share it)."""
    S = sym_sqrt(correlation_matrix(n, kind, L))
    S.setflags(write=False)
    return S


def cov_sqrt(n: int, kind: str, L: float, sigma: float) -> np.ndarray:
    """sigma * C^{1/2}: the symmetric square root of sigma^2 C."""
    return sigma * _corr_sqrt(int(n), str(kind), float(L))


# ---------------------------------------------------------------------------
# The inner-loop problem (Section 2.1, eq. incr_wc4d-var_forcing)
# ---------------------------------------------------------------------------


@dataclass
class Problem:
    n: int
    N: int
    model: str                       # 'advdiff' | 'l96'
    Bsqrt: np.ndarray                # n x n
    Qsqrt: np.ndarray                # n x n (same Q_i for every i)
    obs: List[Tuple[int, np.ndarray, np.ndarray]] = field(default_factory=list)  # (i, idx, rdiag)
    c: float = 0.0
    r: float = 0.0
    F: float = 8.0
    dt: float = 0.025
    traj: Optional[np.ndarray] = None  # (N+1, n) for l96
    n_apply: int = 0                  # number of block applications of A so far

    @property
    def n_A(self) -> int:
        return self.n * (self.N + 1)

    @property
    def q(self) -> int:
        return int(sum(len(idx) for _, idx, _ in self.obs))

    # --- tangent-linear model M_i and its transpose ---
    def M(self, i: int, x: np.ndarray) -> np.ndarray:
        if self.model == "advdiff":
            return advdiff_step(x, self.c, self.r)
        return l96_tlm_step(self.traj[i], x, self.F, self.dt)

    def MT(self, i: int, w: np.ndarray) -> np.ndarray:
        if self.model == "advdiff":
            return advdiff_step_T(w, self.c, self.r)
        return l96_adj_step(self.traj[i], w, self.F, self.dt)


def make_problem(w, pattern, sigma_o2: Optional[float] = None, x0: Optional[np.ndarray] = None) -> Problem:
    """Build the oracle's problem from workload parameters (sizes and parameters only)."""
    s2 = w.sigma_o2 if sigma_o2 is None else sigma_o2
    obs = [(int(i), np.asarray(idx, dtype=np.int64), np.full(len(idx), s2)) for i, idx in pattern]
    prob = Problem(n=w.n, N=w.N, model=w.model,
                   Bsqrt=cov_sqrt(w.n, w.corr, w.Lb, w.sigma_b),
                   Qsqrt=cov_sqrt(w.n, w.corr, w.Lq, w.sigma_q),
                   obs=obs, c=w.c, r=w.r, F=w.F, dt=w.dt)
    if w.model == "l96":
        if x0 is None:
            raise ValueError("l96 needs an initial state")
        prob.traj = l96_trajectory(np.asarray(x0, dtype=np.float64), w.F, w.dt, w.N)
    return prob


def _levels(prob: Problem, X: np.ndarray) -> np.ndarray:
    return X.reshape(prob.N + 1, prob.n, -1)


def apply_Linv(prob: Problem, P: np.ndarray) -> np.ndarray:
    """L^{-1} p (Section 2.1): x_0 = p_0, x_{i+1} = M_i x_i + p_{i+1}."""
    Pl = _levels(prob, np.asarray(P, dtype=np.float64))
    Xl = np.empty_like(Pl)
    Xl[0] = Pl[0]
    for i in range(prob.N):
        Xl[i + 1] = prob.M(i, Xl[i]) + Pl[i + 1]
    return Xl.reshape(P.shape)


def apply_LinvT(prob: Problem, Z: np.ndarray) -> np.ndarray:
    """L^{-T} z: w_N = z_N, w_i = z_i + M_i^T w_{i+1}."""
    Zl = _levels(prob, np.asarray(Z, dtype=np.float64))
    Wl = np.empty_like(Zl)
    Wl[prob.N] = Zl[prob.N]
    for i in range(prob.N - 1, -1, -1):
        Wl[i] = Zl[i] + prob.MT(i, Wl[i + 1])
    return Wl.reshape(Z.shape)


def apply_HtRinvH(prob: Problem, X: np.ndarray) -> np.ndarray:
    """H^T R^{-1} H x for direct observations (Section 2.1 notation, Section 5)."""
    Xl = _levels(prob, X)
    Zl = np.zeros_like(Xl)
    for i, idx, rdiag in prob.obs:
        vals = Xl[i][idx] / rdiag[:, None]
        np.add.at(Zl[i], idx, vals)
    return Zl.reshape(X.shape)


def apply_HtRinv(prob: Problem, d: np.ndarray, m_cols: int = 1) -> np.ndarray:
    """H^T R^{-1} d for d stacked over observed times in pattern order."""
    Z = np.zeros((prob.N + 1, prob.n))
    off = 0
    for i, idx, rdiag in prob.obs:
        np.add.at(Z[i], idx, d[off:off + len(idx)] / rdiag)
        off += len(idx)
    return Z.reshape(-1)


def apply_Dsqrt(prob: Problem, X: np.ndarray) -> np.ndarray:
    """D^{1/2} X with D^{1/2} = blockdiag(B^{1/2}, Q^{1/2}, ..., Q^{1/2})."""
    Xl = _levels(prob, np.asarray(X, dtype=np.float64))
    Yl = np.empty_like(Xl)
    Yl[0] = prob.Bsqrt @ Xl[0]
    for i in range(1, prob.N + 1):
        Yl[i] = prob.Qsqrt @ Xl[i]
    return Yl.reshape(X.shape)


def apply_A(prob: Problem, X: np.ndarray) -> np.ndarray:
    """A X = X + D^{1/2} L^{-T} H^T R^{-1} H L^{-1} D^{1/2} X (Section 2.2, eq. forcing_1stlvl_prec)."""
    X = np.asarray(X, dtype=np.float64)
    squeeze = X.ndim == 1
    if squeeze:
        X = X[:, None]
    prob.n_apply += 1
    P = apply_Dsqrt(prob, X)
    Xs = apply_Linv(prob, P)
    Z = apply_HtRinvH(prob, Xs)
    W = apply_LinvT(prob, Z)
    Y = X + apply_Dsqrt(prob, W)
    return Y[:, 0] if squeeze else Y


def rhs(prob: Problem, d: np.ndarray, bt: Optional[np.ndarray] = None) -> np.ndarray:
    """Right-hand side of eq. forcing_1stlvl_prec: D^{-1/2} b + D^{1/2} L^{-T} H^T R^{-1} d,
    with bt = D^{-1/2} b supplied by the caller (zero in a first inner loop)."""
    z = apply_HtRinv(prob, d)
    out = apply_Dsqrt(prob, apply_LinvT(prob, z[:, None]))[:, 0]
    if bt is not None:
        out = out + bt
    return out


# --- strong-constraint counterpart (Section 6: the approach carries over) ---
# With a perfect model there is no forcing: the control is x_0 alone, the trajectory is
# x_i = M_{i-1} ... M_0 x_0, and the B^{1/2}-preconditioned Hessian is
#     A_sc = I + B^{1/2} (sum_i M_{0->i}^T H_i^T R_i^{-1} H_i M_{0->i}) B^{1/2},
# of size n.  It is the weak-constraint operator with the model-error blocks removed.


def apply_A_sc(prob: Problem, X: np.ndarray) -> np.ndarray:
    """A_sc X: x_0 = B^{1/2} X, x_{i+1} = M_i x_i; z_i = H_i^T R_i^{-1} H_i x_i; w_N = z_N,
    w_i = z_i + M_i^T w_{i+1}; A_sc X = X + B^{1/2} w_0."""
    X = np.asarray(X, dtype=np.float64)
    squeeze = X.ndim == 1
    if squeeze:
        X = X[:, None]
    prob.n_apply += 1
    xs = [prob.Bsqrt @ X]
    for i in range(prob.N):
        xs.append(prob.M(i, xs[-1]))
    Z = apply_HtRinvH(prob, np.concatenate(xs, axis=0))
    Zl = _levels(prob, Z)
    w = Zl[prob.N]
    for i in range(prob.N - 1, -1, -1):
        w = Zl[i] + prob.MT(i, w)
    Y = X + prob.Bsqrt @ w
    return Y[:, 0] if squeeze else Y


def rhs_sc(prob: Problem, d: np.ndarray, bt: Optional[np.ndarray] = None) -> np.ndarray:
    """Right-hand side of the strong-constraint system: B^{1/2} w_0 with w the adjoint sweep of
    H^T R^{-1} d (plus bt = B^{-1/2} (x^b - x_0) in later outer loops)."""
    Zl = _levels(prob, apply_HtRinv(prob, d)[:, None])
    w = Zl[prob.N]
    for i in range(prob.N - 1, -1, -1):
        w = Zl[i] + prob.MT(i, w)
    out = (prob.Bsqrt @ w)[:, 0]
    if bt is not None:
        out = out + bt
    return out


def dense_A_sc(prob: Problem) -> np.ndarray:
    """A_sc assembled from explicit products M_{0->i} = M_{i-1} ... M_0 (tiny problems)."""
    n = prob.n
    H = np.zeros((n, n))
    Mp = np.eye(n)
    obs_by_t = {}
    for i, idx, rdiag in prob.obs:
        obs_by_t.setdefault(i, []).append((idx, rdiag))
    for i in range(prob.N + 1):
        if i > 0:
            Mp = dense_M(prob, i - 1) @ Mp
        for idx, rdiag in obs_by_t.get(i, []):
            Hi = np.zeros((len(idx), n))
            Hi[np.arange(len(idx)), idx] = 1.0
            H += Mp.T @ Hi.T @ np.diag(1.0 / rdiag) @ Hi @ Mp
    return np.eye(n) + prob.Bsqrt @ H @ prob.Bsqrt


# --- dense assembly from the block definitions (tiny problems only) ---


def dense_M(prob: Problem, i: int) -> np.ndarray:
    """Dense M_i, column by column from the tangent-linear model."""
    return prob.M(i, np.eye(prob.n))


def dense_Linv(prob: Problem) -> np.ndarray:
    """Dense L^{-1} from its block structure: identity blocks on the diagonal and
    block (l+1, i) = M_{i,l} = M_l ... M_i below it (Section 2.1)."""
    n, N = prob.n, prob.N
    Ms = [dense_M(prob, i) for i in range(N)]
    L = np.zeros(((N + 1) * n, (N + 1) * n))
    for i in range(N + 1):
        L[i * n:(i + 1) * n, i * n:(i + 1) * n] = np.eye(n)
    for i in range(N):
        prod = np.eye(n)
        for l_ in range(i, N):
            prod = Ms[l_] @ prod
            L[(l_ + 1) * n:(l_ + 2) * n, i * n:(i + 1) * n] = prod
    return L


def dense_H_Rinv(prob: Problem) -> Tuple[np.ndarray, np.ndarray]:
    """Dense H (q x n_A) selecting the observed entries and R^{-1} (q x q)."""
    rows, rinv = [], []
    for i, idx, rdiag in prob.obs:
        for j, rv in zip(idx, rdiag):
            e = np.zeros(prob.n_A)
            e[i * prob.n + j] = 1.0
            rows.append(e)
            rinv.append(1.0 / rv)
    return np.array(rows).reshape(-1, prob.n_A), np.diag(rinv)


def dense_D(prob: Problem, power: str) -> np.ndarray:
    """Dense blockdiag of B, Q (power 'sqrt' or 'full')."""
    blocks = [prob.Bsqrt] + [prob.Qsqrt] * prob.N
    if power == "full":
        blocks = [b @ b for b in blocks]
    return sla.block_diag(*blocks)


def dense_hessian_unprec(prob: Problem, Dinv: np.ndarray) -> np.ndarray:
    """The Hessian of eq. forcing_form_matrix: D^{-1} + L^{-T} H^T R^{-1} H L^{-1}."""
    Li = dense_Linv(prob)
    H, Ri = dense_H_Rinv(prob)
    return Dinv + Li.T @ H.T @ Ri @ H @ Li


def dense_A(prob: Problem) -> np.ndarray:
    """Dense A assembled by applying the operator to the identity."""
    saved = prob.n_apply
    A = apply_A(prob, np.eye(prob.n_A))
    prob.n_apply = saved
    return A


# ---------------------------------------------------------------------------
# Randomised eigenvalue decompositions (Section 4)
# ---------------------------------------------------------------------------


def _eig_desc(K: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    """Symmetric EVD of (the symmetric part of) K, eigenvalues decreasing."""
    Ks = 0.5 * (K + K.T)
    lam, W = np.linalg.eigh(Ks)
    order = np.argsort(-lam, kind="stable")
    return lam[order], W[:, order]


def _orth(Y: np.ndarray) -> np.ndarray:
    Q, _ = np.linalg.qr(Y, mode="reduced")
    return Q


def revd(applyA: Callable, G: np.ndarray, k: int) -> Tuple[np.ndarray, np.ndarray]:
    """Algorithm 3 (REVD): Y = A G; Z_1 = orth(Y); K_1 = Z_1^T A Z_1;
    EVD sorted decreasing; keep k; U_1 = Z_1 W_1.  Two block products with A."""
    Y = applyA(G)
    Z1 = _orth(Y)
    K1 = Z1.T @ applyA(Z1)
    theta, W1 = _eig_desc(K1)
    return Z1 @ W1[:, :k], theta[:k]


def nystrom(applyA: Callable, G: np.ndarray, k: int) -> Tuple[np.ndarray, np.ndarray]:
    """Algorithm 4 (Nystrom): Y = A G; Z_1 = orth(Y); E1 = A Z_1; E2 = Z_1^T E1;
    E2 = C^T C (Cholesky); solve F C = E1; SVD F = U_2 Sigma V^T; keep k;
    Theta_2 = Sigma^2.  Two block products with A."""
    Y = applyA(G)
    Z1 = _orth(Y)
    E1 = applyA(Z1)
    E2 = Z1.T @ E1
    E2 = 0.5 * (E2 + E2.T)
    C = np.linalg.cholesky(E2).T            # upper triangular, E2 = C^T C
    F = sla.solve_triangular(C, E1.T, trans="T", lower=False).T   # F C = E1
    U2, sig, _ = np.linalg.svd(F, full_matrices=False)
    return U2[:, :k], sig[:k] ** 2


def ritzit(applyA: Callable, G: np.ndarray, k: int) -> Tuple[np.ndarray, np.ndarray]:
    """Algorithm 5 (REVD_ritzit): G_3 = orth(G); Y_3 = A G_3 = Z_3 R_3 (QR);
    K_3 = R_3 R_3^T = W_3 Theta_3^2 W_3^T sorted decreasing; keep k;
    U_3 = Z_3 W_3.  One block product with A."""
    G3 = _orth(G)
    Y3 = applyA(G3)
    Z3, R3 = np.linalg.qr(Y3, mode="reduced")
    K3 = R3 @ R3.T
    theta2, W3 = _eig_desc(K3)
    return Z3 @ W3[:, :k], np.sqrt(np.clip(theta2[:k], 0.0, None))


def nystrom_single_pass(applyA: Callable, G: np.ndarray, k: int) -> Tuple[np.ndarray, np.ndarray]:
    """Single-pass Nystrom, the variant Section 6 names as future work (the single-pass
    Nystrom of Halko, Martinsson and Tropp 2011, Section 5.5): the Nystrom approximation
    A ~ Y (G_4^T Y)^{-1} Y^T built on the start block's own range, so A is applied once.
    G_4 = orth(G); Y = A G_4; E = G_4^T Y = C^T C (Cholesky); solve F C = Y;
    SVD F = U Sigma V^T; keep k; Theta = Sigma^2."""
    G4 = _orth(G)
    Y = applyA(G4)
    E = G4.T @ Y
    E = 0.5 * (E + E.T)
    C = np.linalg.cholesky(E).T             # upper triangular, E = C^T C
    F = sla.solve_triangular(C, Y.T, trans="T", lower=False).T    # F C = Y
    U, sig, _ = np.linalg.svd(F, full_matrices=False)
    return U[:, :k], sig[:k] ** 2


METHODS = {"revd": revd, "nystrom": nystrom, "ritzit": ritzit, "nystrom1p": nystrom_single_pass}


# ---------------------------------------------------------------------------
# Spectral LMP (Section 3.2, eqs. spectral_LMP and spectral_LMP_factor)
# ---------------------------------------------------------------------------


def lmp_apply(U: np.ndarray, theta: np.ndarray, X: np.ndarray) -> np.ndarray:
    """C X with C = I + U (Theta^{-1/2} - I) U^T (symmetric, so C^T = C)."""
    X = np.asarray(X, dtype=np.float64)
    dcoef = theta ** -0.5 - 1.0
    if X.ndim == 1:
        return X + U @ (dcoef * (U.T @ X))
    return X + U @ (dcoef[:, None] * (U.T @ X))


def lmp_dense_C(U: np.ndarray, theta: np.ndarray) -> np.ndarray:
    return np.eye(U.shape[0]) + U @ np.diag(theta ** -0.5 - 1.0) @ U.T


def lmp_dense_P(U: np.ndarray, theta: np.ndarray) -> np.ndarray:
    """P = I - sum_i (1 - theta_i^{-1}) u_i u_i^T (eq. spectral_LMP)."""
    P = np.eye(U.shape[0])
    for i in range(U.shape[1]):
        P -= (1.0 - 1.0 / theta[i]) * np.outer(U[:, i], U[:, i])
    return P


def lmp_dense_C_product(U: np.ndarray, theta: np.ndarray) -> np.ndarray:
    """C = prod_i (I - (1 - theta_i^{-1/2}) u_i u_i^T) (eq. spectral_LMP_factor)."""
    C = np.eye(U.shape[0])
    for i in range(U.shape[1]):
        C = C @ (np.eye(U.shape[0]) - (1.0 - theta[i] ** -0.5) * np.outer(U[:, i], U[:, i]))
    return C


# ---------------------------------------------------------------------------
# Split preconditioned CG (Algorithm 1)
# ---------------------------------------------------------------------------

def ritz_lmp_dense(U: np.ndarray, theta: np.ndarray, A: np.ndarray) -> np.ndarray:
    """The Ritz-LMP of eq. Ritz_LMP written out densely:
    P = (I - U Theta^{-1} U^T A)(I - A U Theta^{-1} U^T) + U Theta^{-1} U^T."""
    n = A.shape[0]
    T = U @ np.diag(1.0 / theta) @ U.T
    return (np.eye(n) - T @ A) @ (np.eye(n) - A @ T) + T


def ritz_lmp_apply(U: np.ndarray, theta: np.ndarray, AU: np.ndarray, r: np.ndarray) -> np.ndarray:
    """P r for the Ritz-LMP of eq. Ritz_LMP, with A U given (A symmetric):
    c = Theta^{-1} U^T r; w = r - (A U) c; e = Theta^{-1} (A U)^T w; P r = w - U e + U c."""
    c = (U.T @ r) / theta
    w = r - AU @ c
    e = (AU.T @ w) / theta
    return w - U @ e + U @ c


RES_TRUE = 0
RES_PRECOND = 1


@dataclass
class PCGResult:
    x: np.ndarray
    iters: int
    converged: bool
    relres_true: float
    relres_precond: float
    J: float
    hist_true: List[float]
    hist_precond: List[float]
    hist_J: List[float]
    alphas: List[float]
    betas: List[float]
    residuals: Optional[List[np.ndarray]] = None   # r_0, r_1, ... when asked for


def pcg(applyA: Callable, b: np.ndarray, x0: Optional[np.ndarray] = None,
        lmp: Optional[Tuple[np.ndarray, np.ndarray]] = None, tol: float = 1e-6,
        maxit: int = 100, criterion: int = RES_TRUE, keep_residuals: bool = False,
        reorth: bool = False) -> PCGResult:
    """Algorithm 1, split preconditioned CG on C^T A C xhat = C^T b with P = C C^T:
        r_0 = C^T (b - A x_0), p_0 = C r_0;
        alpha_j = r^T r / p^T A p;  x_j = x_{j-1} + alpha_j p_{j-1};
        r_j = r_{j-1} - alpha_j C^T A p_{j-1};  beta_j = r_j^T r_j / r_{j-1}^T r_{j-1};
        p_j = C r_j + beta_j p_{j-1}.
    Alongside it keeps s_j = b - A x_j by the recursion s_j = s_{j-1} - alpha_j A p_{j-1}
    (the true residual) and the quadratic cost J(x) = x^T A x / 2 - b^T x = -x^T (b + s) / 2.
    Stops when ||s_j|| / ||b|| <= tol (criterion RES_TRUE) or ||r_j|| / ||r_0|| <= tol
    (RES_PRECOND), or after maxit iterations.

    reorth (no LMP only): complete reorthogonalisation, Section 3.4's remedy for the repeated
    ('ghost') Ritz values that loss of orthogonality brings: each new r_j is orthogonalised
    against all earlier normalised residuals r_i / ||r_i|| (classical Gram-Schmidt, applied
    twice) before r_j^T r_j and beta_j are formed.  In exact arithmetic the residuals are
    already orthogonal and the iterates are those of CG."""
    b = np.asarray(b, dtype=np.float64)
    if reorth and lmp is not None:
        raise ValueError("pcg: reorthogonalisation is defined here for CG without an LMP")
    if lmp is None:
        C = lambda v: v  # noqa: E731
    else:
        U, theta = lmp
        C = lambda v: lmp_apply(U, theta, v)  # noqa: E731  (C^T = C)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    s = b - applyA(x) if x0 is not None and np.any(x0) else b.copy()
    r = C(s)
    p = C(r)
    bnorm = np.linalg.norm(b)
    r0norm = np.linalg.norm(r)
    rr = r @ r
    ht, hp, hJ, al, be = [], [], [], [], []
    res = [r.copy()] if keep_residuals else None
    Q = [r / np.sqrt(rr)] if reorth and rr > 0.0 else []
    it = 0
    converged = False
    if bnorm == 0.0:
        return PCGResult(x, 0, True, 0.0, 0.0, 0.0, [], [], [], [], [], res)
    for it in range(1, maxit + 1):
        Ap = applyA(p)
        alpha = rr / (p @ Ap)
        x = x + alpha * p
        s = s - alpha * Ap
        r = r - alpha * C(Ap)
        if reorth:
            Qm = np.stack(Q, axis=1)
            for _ in range(2):
                r = r - Qm @ (Qm.T @ r)
            Q.append(r / np.linalg.norm(r))
        if keep_residuals:
            res.append(r.copy())
        rr_new = r @ r
        beta = rr_new / rr
        rr = rr_new
        p = C(r) + beta * p
        rt = np.linalg.norm(s) / bnorm
        rp = np.sqrt(rr) / r0norm
        ht.append(rt)
        hp.append(rp)
        hJ.append(-0.5 * (x @ (b + s)))
        al.append(alpha)
        be.append(beta)
        if (rt if criterion == RES_TRUE else rp) <= tol:
            converged = True
            break
    return PCGResult(x, it, converged, ht[-1], hp[-1], hJ[-1], ht, hp, hJ, al, be, res)


def pcg_standard(applyA: Callable, b: np.ndarray, precond: Callable, tol: float = 1e-6,
                 maxit: int = 100) -> PCGResult:
    """Preconditioned CG with a symmetric positive definite preconditioner P given as a
    function (for an LMP that has no split factor C, such as the Ritz-LMP):
        r_0 = b, z_0 = P r_0, p_0 = z_0;  alpha = r^T z / p^T A p;  x += alpha p;
        r -= alpha A p;  z = P r;  beta = r_new^T z_new / r^T z;  p = z + beta p.
    With P = C C^T this is Algorithm 1 in exact arithmetic (x_j are the same iterates).
    Stops when ||r_j|| / ||b|| <= tol (r is the true residual's recursion) or after maxit."""
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b)
    r = b.copy()
    z = precond(r)
    p = z.copy()
    rz = r @ z
    bnorm = np.linalg.norm(b)
    ht, hJ, al, be = [], [], [], []
    it = 0
    converged = False
    if bnorm == 0.0:
        return PCGResult(x, 0, True, 0.0, 0.0, 0.0, [], [], [], [], [])
    for it in range(1, maxit + 1):
        Ap = applyA(p)
        alpha = rz / (p @ Ap)
        x = x + alpha * p
        r = r - alpha * Ap
        z = precond(r)
        rz_new = r @ z
        beta = rz_new / rz
        rz = rz_new
        p = z + beta * p
        rt = np.linalg.norm(r) / bnorm
        ht.append(rt)
        hJ.append(-0.5 * (x @ (b + r)))
        al.append(alpha)
        be.append(beta)
        if rt <= tol:
            converged = True
            break
    return PCGResult(x, it, converged, ht[-1], float("nan"), hJ[-1], ht, [], hJ, al, be)


# ---------------------------------------------------------------------------
# Spectral information from CG (Section 3.4): the Lanczos tridiagonal T_j
# ---------------------------------------------------------------------------


def cg_tridiagonal(alphas: List[float], betas: List[float], j: int) -> np.ndarray:
    """T_j of Section 3.4 from the first j CG coefficients: gamma_1 = 1/alpha_1,
    gamma_i = 1/alpha_i + beta_{i-1}/alpha_{i-1}; tau_i = sqrt(beta_i)/alpha_i."""
    T = np.zeros((j, j))
    for i in range(j):
        T[i, i] = 1.0 / alphas[i] + (betas[i - 1] / alphas[i - 1] if i > 0 else 0.0)
        if i + 1 < j:
            T[i, i + 1] = T[i + 1, i] = np.sqrt(betas[i]) / alphas[i]
    return T


def cg_lanczos_pairs(res: PCGResult, k: int, j: Optional[int] = None) -> Tuple[np.ndarray, np.ndarray]:
    """The k largest Ritz pairs of A from j iterations of CG (Section 3.4): Ritz values are
    the eigenvalues of T_j, Ritz vectors u_i = F_j w_i with w_i the eigenvectors of T_j and
    F_j = (f_0, ..., f_{j-1}).  The Lanczos vectors are f_i = (-1)^i r_i / ||r_i|| (the signs
    make F_j^T A F_j = T_j with T_j's positive off-diagonal; Section 3.4 writes r_i / ||r_i||)."""
    j = res.iters if j is None else j
    T = cg_tridiagonal(res.alphas, res.betas, j)
    F = np.stack([(-1.0) ** i * res.residuals[i] / np.linalg.norm(res.residuals[i]) for i in range(j)], axis=1)
    theta, W = _eig_desc(T)
    return F @ W[:, :k], theta[:k]


# ---------------------------------------------------------------------------
# Gauss-Newton outer loop (Section 2.1, eqs. error_update and incr_wc4d-var_forcing)
# ---------------------------------------------------------------------------


def innovations_from_state(prob: Problem, y: List[np.ndarray], X: np.ndarray) -> np.ndarray:
    """d = (y_i - H_i x_i) stacked over the observed times (direct observations); y[a] are
    the observations of the a-th observed time of prob.obs, X the (N+1, n) state."""
    if not prob.obs:
        return np.zeros(0)
    return np.concatenate([y[a] - X[i][idx] for a, (i, idx, _) in enumerate(prob.obs)])


def model_step(prob: Problem, x: np.ndarray) -> np.ndarray:
    """One step of the nonlinear model M (eq. model): the advection-diffusion stencil (a
    linear model) or one RK4 step of Lorenz-96."""
    if prob.model == "advdiff":
        return advdiff_step(x, prob.c, prob.r)
    return l96_rk4_step(x, prob.F, prob.dt)


def forced_trajectory(prob: Problem, x0: np.ndarray, eta: np.ndarray) -> np.ndarray:
    """x_{i+1} = M(x_i) + eta_{i+1} (eq. model); eta: (N, n), row i is eta_{i+1}."""
    out = np.empty((prob.N + 1, prob.n))
    out[0] = x0
    for i in range(prob.N):
        out[i + 1] = model_step(prob, out[i]) + eta[i]
    return out


def nonlinear_cost(prob: Problem, xb: np.ndarray, y: List[np.ndarray], x0: np.ndarray, eta: np.ndarray) -> float:
    """J(x_0, eta_1..eta_N) of eq. 4D-var_error for direct observations."""
    X = forced_trajectory(prob, x0, eta)
    Binv = np.linalg.inv(prob.Bsqrt @ prob.Bsqrt)
    Qinv = np.linalg.inv(prob.Qsqrt @ prob.Qsqrt)
    J = 0.5 * (x0 - xb) @ Binv @ (x0 - xb)
    for a, (i, idx, rd) in enumerate(prob.obs):
        dv = y[a] - X[i][idx]
        J += 0.5 * dv @ (dv / rd)
    for i in range(prob.N):
        J += 0.5 * eta[i] @ Qinv @ eta[i]
    return float(J)


def twin_experiment(prob: Problem, draws) -> Tuple[np.ndarray, List[np.ndarray], np.ndarray]:
    """Identical twin (Section 5): the truth x^t from draws['x0'] with model errors
    Q^{1/2} xi_model, the background x^b = x^t_0 + B^{1/2} xi_b and observations
    y_i = H_i x^t_i + sigma_o zeta.  Returns (x^b, y, truth trajectory)."""
    eta_t = draws["xi_model"] @ prob.Qsqrt.T
    Xt = forced_trajectory(prob, draws["x0"], eta_t)
    xb = Xt[0] + prob.Bsqrt @ draws["xi_b"]
    y, off = [], 0
    for i, idx, rd in prob.obs:
        y.append(Xt[i][idx] + np.sqrt(rd) * draws["zeta"][off:off + len(idx)])
        off += len(idx)
    return xb, y, Xt


def gauss_newton(prob: Problem, xb: np.ndarray, y: List[np.ndarray], n_outer: int, inner: Callable):
    """The incremental outer loop (Section 2.1): p^(0) = (x^b, 0, ..., 0); for j = 0, 1, ...
    the state x^(j) from p^(j) by eq. model, the problem linearised about it, b^(j), d^(j),
    the inner loop on eq. forcing_1stlvl_prec (rhs = D^{-1/2} b + D^{1/2} L^{-T} H^T R^{-1} d)
    by inner(prob_j, rhs, j) -> delta p~, and p^(j+1) = p^(j) + D^{1/2} delta p~ (eq.
    error_update).  Returns per-loop records (rhs, delta p~, nonlinear cost before the loop)."""
    n, N = prob.n, prob.N
    p = np.zeros((N + 1) * n)
    p[:n] = xb
    pb = p.copy()
    recs = []
    for j in range(n_outer):
        x0, eta = p[:n], p[n:].reshape(N, n)
        X = forced_trajectory(prob, x0, eta)
        pj = Problem(n=n, N=N, model=prob.model, Bsqrt=prob.Bsqrt, Qsqrt=prob.Qsqrt, obs=prob.obs, c=prob.c,
                     r=prob.r, F=prob.F, dt=prob.dt, traj=X)
        d = innovations_from_state(pj, y, X)
        b = pb - p                                   # (x^b - x_0^(j), -eta_1^(j), ..., -eta_N^(j))
        rhs_j = rhs(pj, d, bt=dinv_sqrt(pj, b))
        recs.append({"J": nonlinear_cost(pj, xb, y, x0, eta), "rhs": rhs_j, "prob": pj, "b": b})
        dpt = inner(pj, rhs_j, j)
        recs[-1]["dpt"] = dpt
        p = p + apply_Dsqrt(pj, dpt[:, None])[:, 0]
    x0, eta = p[:n], p[n:].reshape(N, n)
    recs.append({"J": nonlinear_cost(prob, xb, y, x0, eta), "p": p})
    return recs


def dinv_sqrt(prob: Problem, v: np.ndarray) -> np.ndarray:
    """D^{-1/2} v by solving with the symmetric square roots level by level."""
    Lv = _levels(prob, v[:, None])[:, :, 0]
    out = np.empty_like(Lv)
    out[0] = np.linalg.solve(prob.Bsqrt, Lv[0])
    for i in range(1, prob.N + 1):
        out[i] = np.linalg.solve(prob.Qsqrt, Lv[i])
    return out.reshape(-1)


# ---------------------------------------------------------------------------
# Inner loop (Section 4, last paragraphs): randomised method -> LMP -> PCG
# ---------------------------------------------------------------------------


def inner_loop(prob: Problem, b: np.ndarray, G: np.ndarray, method: str, k: int,
               tol: float = 1e-6, maxit: int = 5000, criterion: int = RES_TRUE):
    """Estimate Ritz pairs with one randomised method, build the spectral LMP,
    solve the exact system with split PCG."""
    U, theta = METHODS[method](lambda X: apply_A(prob, X), G, k)
    res = pcg(lambda v: apply_A(prob, v), b, lmp=(U, theta), tol=tol, maxit=maxit, criterion=criterion)
    return U, theta, res
