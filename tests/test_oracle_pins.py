"""Pins of the FP64 oracle to facts other than itself: sizes printed in the
paper, closed forms, textbook special cases, invariants the paper states, and
brute force on tiny inputs.  CPU only."""
import json
import os

import numpy as np
import pytest
import scipy.integrate
import scipy.linalg as sla

from oracle import wc4d_oracle as O
from synthetic import (C1, C2, Workload, innovations, l96_initial_state, obs_count, obs_pattern, twin_draws,
                       random_block, sketch_block)

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def tiny_advdiff(n=8, N=4, c=0.5, r=0.1, vs=2, ts=2, m=4, corr="soar", L=2.0):
    return Workload(name="tiny", model="advdiff", n=n, N=N, c=c, r=r, corr=corr, Lb=L, Lq=L,
                    sigma_b=1.0, sigma_q=0.3, obs_var_stride=vs, obs_time_stride=ts,
                    sigma_o2=0.01, m=m, l=2, seed=17)


def tiny_l96(n=10, N=4, vs=2, ts=2, m=4):
    return Workload(name="tinyl96", model="l96", n=n, N=N, F=8.0, dt=0.025, corr="gauss",
                    Lb=2.0, Lq=2.0, sigma_b=0.2, sigma_q=0.1, obs_var_stride=vs,
                    obs_time_stride=ts, sigma_o2=0.04, m=m, l=2, seed=29)


def build(w):
    x0 = l96_initial_state(w.n, w.seed) if w.model == "l96" else None
    return O.make_problem(w, obs_pattern(w), x0=x0)


# ----------------------------------------------------------------- sizes


def test_paper_sizes_and_observation_counts():
    cases = json.load(open(os.path.join(GOLDEN, "paper_sizes.json")))["cases"]
    for c in cases:
        w = Workload(name="p", model="advdiff", n=c["n"], N=c["N"], obs_var_stride=c["var_stride"],
                     obs_time_stride=c["time_stride"])
        assert w.n_A == c.get("n_A", w.n_A)
        pat = obs_pattern(w)
        assert obs_count(pat) == c["q"], c["cite"]
        assert pat[-1][0] == w.N  # the final step is observed
        prob = O.Problem(n=w.n, N=w.N, model="advdiff", Bsqrt=np.eye(w.n), Qsqrt=np.eye(w.n),
                         obs=[(i, idx, np.ones(len(idx))) for i, idx in pat])
        assert prob.n_A == c.get("n_A", prob.n_A) and prob.q == c["q"]


# ----------------------------------------------------------------- models


def test_advdiff_pure_upwind_courant_one_is_exact_shift():
    # c = 1, r = 0: the upwind scheme moves the field exactly one cell per step.
    w = tiny_advdiff(n=12, N=7, c=1.0, r=0.0)
    prob = build(w)
    e = np.random.default_rng(0).standard_normal(12)
    P = np.zeros((prob.n_A, 1))
    P[:12, 0] = e
    X = O.apply_Linv(prob, P).reshape(8, 12)
    for i in range(8):
        np.testing.assert_array_equal(X[i], np.roll(e, i))


@pytest.mark.parametrize("c,r", [(0.5, 0.1), (0.8, 0.0), (0.0, 0.25), (0.3, 0.05)])
def test_advdiff_fourier_multiplier(c, r):
    # M e^{i theta j} = g(theta) e^{i theta j}, g = (c+r) e^{-i theta} + (1-c-2r) + r e^{i theta}.
    n = 16
    j = np.arange(n)
    for k in range(n):
        th = 2 * np.pi * k / n
        g = (c + r) * np.exp(-1j * th) + (1 - c - 2 * r) + r * np.exp(1j * th)
        mode = np.exp(1j * th * j)
        got = O.advdiff_step(mode.real, c, r) + 1j * O.advdiff_step(mode.imag, c, r)
        np.testing.assert_allclose(got, g * mode, atol=1e-14)


def test_advdiff_transpose():
    rng = np.random.default_rng(1)
    x, y = rng.standard_normal((2, 20, 3))
    lhs = np.sum(O.advdiff_step(x, 0.5, 0.1) * y)
    rhs = np.sum(x * O.advdiff_step_T(y, 0.5, 0.1))
    assert abs(lhs - rhs) < 1e-13 * abs(lhs)


def test_l96_equilibrium_and_constant_forcing():
    F = 8.0
    np.testing.assert_allclose(O.l96_rhs(np.full(12, F), F), 0.0, atol=1e-14)
    np.testing.assert_allclose(O.l96_rhs(np.zeros(12), F), F)
    # a one-point state: the product terms vanish, only the damping -X^j remains
    x = np.zeros(12)
    x[3] = 2.0
    f = O.l96_rhs(x, 0.0)
    expect = np.zeros(12)
    expect[3] = -2.0
    np.testing.assert_allclose(f, expect)
    # a two-point state exercises every product term: X^2 = a, X^3 = b
    a, b = 1.5, -0.7
    x = np.zeros(12)
    x[2], x[3] = a, b
    f = O.l96_rhs(x, 0.0)
    # by hand: dX^2/dt = -a, dX^3/dt = -b, dX^4/dt = -X^2 X^3 = -ab, every other tendency is 0
    expect = np.zeros(12)
    expect[2], expect[3], expect[4] = -a, -b, -a * b
    np.testing.assert_allclose(f, expect, atol=1e-15)


def test_l96_rk4_fourth_order_against_reference_integrator():
    x0 = l96_initial_state(20, 123)
    T = 0.2
    ref = scipy.integrate.solve_ivp(lambda t, y: O.l96_rhs(y, 8.0), (0, T), x0, method="DOP853",
                                    rtol=1e-13, atol=1e-13).y[:, -1]
    errs = []
    for steps in (8, 16):
        dt = T / steps
        x = x0.copy()
        for _ in range(steps):
            x = O.l96_rk4_step(x, 8.0, dt)
        errs.append(np.linalg.norm(x - ref))
    order = np.log2(errs[0] / errs[1])
    assert 3.7 < order < 4.4, order


def test_l96_tlm_matches_finite_differences():
    x = l96_initial_state(24, 5)
    dx = np.random.default_rng(2).standard_normal(24)
    h = 1e-6
    fd = (O.l96_rk4_step(x + h * dx, 8.0, 0.025) - O.l96_rk4_step(x - h * dx, 8.0, 0.025)) / (2 * h)
    tl = O.l96_tlm_step(x, dx, 8.0, 0.025)
    assert np.linalg.norm(fd - tl) <= 1e-8 * np.linalg.norm(tl)


def test_l96_adjoint_dot_product():
    x = l96_initial_state(24, 6)
    rng = np.random.default_rng(3)
    u, v = rng.standard_normal((2, 24))
    lhs = O.l96_tlm_step(x, u, 8.0, 0.025) @ v
    rhs = u @ O.l96_adj_step(x, v, 8.0, 0.025)
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)


@pytest.mark.parametrize("maker", [tiny_advdiff, tiny_l96, lambda: C1, lambda: C2])
def test_Linv_adjoint_dot_product(maker):
    prob = build(maker())
    rng = np.random.default_rng(4)
    u = rng.standard_normal((prob.n_A, 3))
    v = rng.standard_normal((prob.n_A, 3))
    lhs = np.sum(O.apply_Linv(prob, u) * v)
    rhs = np.sum(u * O.apply_LinvT(prob, v))
    assert abs(lhs - rhs) <= 1e-12 * np.abs(O.apply_Linv(prob, u)).max() * np.abs(v).sum()


@pytest.mark.parametrize("maker", [tiny_advdiff, tiny_l96])
def test_Linv_equals_block_formula(maker):
    prob = build(maker())
    Lsweep = O.apply_Linv(prob, np.eye(prob.n_A))
    np.testing.assert_allclose(Lsweep, O.dense_Linv(prob), atol=1e-12)


# ----------------------------------------------------------------- covariances


def test_chordal_distance_is_euclidean_on_circle():
    n = 40
    ang = 2 * np.pi * np.arange(n) / n
    R = n / (2 * np.pi)
    pts = R * np.stack([np.cos(ang), np.sin(ang)], 1)
    eu = np.linalg.norm(pts[:, None, :] - pts[None, :, :], axis=2)
    np.testing.assert_allclose(O.chordal_distance(n), eu, atol=1e-12)


def test_correlation_values():
    # rho(0) = 1 and the closed forms evaluated at geometric (circle) distances
    n = 64
    ang = 2 * np.pi * np.arange(n) / n
    pts = (n / (2 * np.pi)) * np.stack([np.cos(ang), np.sin(ang)], 1)
    d = np.linalg.norm(pts[:, None, :] - pts[None, :, :], axis=2)
    L = 4.0
    np.testing.assert_allclose(O.correlation_matrix(n, "soar", L), (1 + d / L) * np.exp(-d / L), atol=1e-13)
    L = 2.0
    np.testing.assert_allclose(O.correlation_matrix(n, "gauss", L), np.exp(-d * d / (2 * L * L)), atol=1e-13)
    np.testing.assert_allclose(np.diag(O.correlation_matrix(n, "soar", 3.0)), 1.0)


@pytest.mark.parametrize("n,kind,L", [(40, "soar", 4.0), (40, "soar", 10.0), (80, "gauss", 2.0), (64, "soar", 4.0)])
def test_correlation_spd_circulant_and_sqrt(n, kind, L):
    C = O.correlation_matrix(n, kind, L)
    lam = np.linalg.eigvalsh(C)
    assert lam.min() > 0
    # circulant: eigenvalues are the DFT of the first row
    fft_eigs = np.sort(np.fft.fft(C[0]).real)
    np.testing.assert_allclose(np.sort(lam), fft_eigs, atol=1e-10 * lam.max())
    S = O.sym_sqrt(C)
    np.testing.assert_allclose(S, S.T, atol=1e-14)
    np.testing.assert_allclose(S @ S, C, atol=1e-12)
    assert np.linalg.eigvalsh(S).min() > 0


def test_wrap_distance_soar_would_be_indefinite():
    # why the chordal distance: SOAR on the wrap-around distance min(k, n-k) is indefinite
    n, L = 40, 10.0
    k = np.abs(np.arange(n)[:, None] - np.arange(n)[None, :])
    dw = np.minimum(k, n - k)
    Cw = (1 + dw / L) * np.exp(-dw / L)
    assert np.linalg.eigvalsh(Cw).min() < 0
    assert np.linalg.eigvalsh(O.correlation_matrix(n, "soar", L)).min() > 0


# ----------------------------------------------------------------- the operator


@pytest.mark.parametrize("maker", [tiny_advdiff, tiny_l96, lambda: C1])
def test_A_symmetric_with_unit_cluster_and_q_large_eigenvalues(maker):
    prob = build(maker())
    A = O.dense_A(prob)
    assert np.abs(A - A.T).max() <= 1e-12 * np.abs(A).max()
    lam = np.linalg.eigvalsh(0.5 * (A + A.T))
    assert abs(lam.min() - 1.0) < 1e-10 * lam.max()
    assert int(np.sum(lam > 1 + 1e-8 * lam.max())) == prob.q
    assert int(np.sum(np.abs(lam - 1) <= 1e-8 * lam.max())) == prob.n_A - prob.q


@pytest.mark.parametrize("maker", [tiny_advdiff, tiny_l96])
def test_A_equals_transformed_unpreconditioned_hessian(maker):
    # A^pr = D^{1/2} (D^{-1} + L^{-T} H^T R^{-1} H L^{-1}) D^{1/2}, D^{-1} from the covariances
    w = maker()
    prob = build(w)
    B = (w.sigma_b ** 2) * O.correlation_matrix(w.n, w.corr, w.Lb)
    Q = (w.sigma_q ** 2) * O.correlation_matrix(w.n, w.corr, w.Lq)
    Dinv = sla.block_diag(np.linalg.inv(B), *([np.linalg.inv(Q)] * w.N))
    Hess = O.dense_hessian_unprec(prob, Dinv)
    Ds = O.dense_D(prob, "sqrt")
    Apr = Ds @ Hess @ Ds
    A = O.dense_A(prob)
    np.testing.assert_allclose(A, Apr, atol=1e-8 * np.abs(A).max())


def test_rhs_matches_dense_formula():
    w = tiny_advdiff()
    prob = build(w)
    d = innovations(prob.q, 3, 0.1)
    Li = O.dense_Linv(prob)
    H, Ri = O.dense_H_Rinv(prob)
    want = O.dense_D(prob, "sqrt") @ Li.T @ H.T @ Ri @ d
    np.testing.assert_allclose(O.rhs(prob, d), want, atol=1e-12 * np.abs(want).max())



@pytest.mark.parametrize("maker", [tiny_advdiff, tiny_l96])
def test_solution_minimises_the_forcing_cost_function(maker):
    """A x = rhs is the stationarity condition of the forcing-formulation cost (Section 2.1,
    its quadratic inner-loop form; Section 2.2's variable change p = D^{1/2} x):
    J(p) = p^T D^{-1} p / 2 + (H L^{-1} p - d)^T R^{-1} (H L^{-1} p - d) / 2.  The minimiser
    is found here as a stacked least-squares problem, independently of A and rhs, and the
    PCG cost diagnostic plus d^T R^{-1} d / 2 equals J at every iterate."""
    prob = build(maker())
    d = innovations(prob.q, 21, 0.1)
    Ds = O.dense_D(prob, "sqrt")
    Dmh = np.linalg.inv(Ds)
    Li = O.dense_Linv(prob)
    H, Ri = O.dense_H_Rinv(prob)
    Rmh = np.diag(np.sqrt(np.diag(Ri)))
    M = np.vstack([Dmh, Rmh @ H @ Li])
    t = np.concatenate([np.zeros(prob.n_A), Rmh @ d])
    p_star = np.linalg.lstsq(M, t, rcond=None)[0]
    x = np.linalg.solve(O.dense_A(prob), O.rhs(prob, d))
    np.testing.assert_allclose(Ds @ x, p_star, atol=1e-9 * np.abs(p_star).max())

    def cost(p):
        e = H @ Li @ p - d
        return 0.5 * p @ np.linalg.solve(Ds @ Ds, p) + 0.5 * e @ Ri @ e

    res = O.pcg(lambda v: O.apply_A(prob, v), O.rhs(prob, d), tol=1e-12, maxit=3)
    xs = [np.zeros(prob.n_A)]
    r = O.rhs(prob, d)
    pvec = r.copy()
    A = O.dense_A(prob)
    for _ in range(res.iters):          # the textbook CG iterates, to evaluate J on each
        a = (r @ r) / (pvec @ A @ pvec)
        xs.append(xs[-1] + a * pvec)
        rn = r - a * (A @ pvec)
        pvec = rn + (rn @ rn) / (r @ r) * pvec
        r = rn
    c0 = 0.5 * d @ Ri @ d
    for j in range(res.iters):
        np.testing.assert_allclose(res.hist_J[j] + c0, cost(Ds @ xs[j + 1]), rtol=1e-9)


def test_dsqrt_squares_to_covariance():
    w = tiny_advdiff()
    prob = build(w)
    Ds = O.dense_D(prob, "sqrt")
    B = (w.sigma_b ** 2) * O.correlation_matrix(w.n, w.corr, w.Lb)
    Q = (w.sigma_q ** 2) * O.correlation_matrix(w.n, w.corr, w.Lq)
    np.testing.assert_allclose(Ds @ Ds, sla.block_diag(B, *([Q] * w.N)), atol=1e-13)


# ----------------------------------------------------------------- randomised EVDs


def small_problem():
    w = tiny_advdiff(n=6, N=3, vs=2, ts=1)   # n_A = 24, q = 9
    return build(w)


@pytest.mark.parametrize("method", ["revd", "nystrom", "ritzit"])
def test_full_sketch_recovers_exact_spectrum(method):
    prob = small_problem()
    A = O.dense_A(prob)
    lam = np.sort(np.linalg.eigvalsh(A))[::-1]
    G = sketch_block(prob.n_A, prob.n_A, 11)
    U, th = O.METHODS[method](lambda X: O.apply_A(prob, X), G, prob.n_A)
    np.testing.assert_allclose(th, lam, rtol=1e-10, atol=1e-10 * lam[0])
    np.testing.assert_allclose(U.T @ U, np.eye(prob.n_A), atol=1e-10)
    np.testing.assert_allclose(U @ np.diag(th) @ U.T, A, atol=1e-9 * lam[0])


@pytest.mark.parametrize("method", ["revd", "nystrom", "ritzit"])
def test_invariant_subspace_gives_exact_pairs(method):
    # Rayleigh-Ritz is exact on an invariant subspace (Section 3.3)
    prob = small_problem()
    A = O.dense_A(prob)
    lam, V = np.linalg.eigh(A)
    lam, V = lam[::-1], V[:, ::-1]
    m = 6
    G = V[:, :m] @ np.linalg.qr(np.random.default_rng(5).standard_normal((m, m)))[0]
    U, th = O.METHODS[method](lambda X: O.apply_A(prob, X), G, 4)
    np.testing.assert_allclose(th, lam[:4], rtol=1e-11)
    np.testing.assert_allclose(A @ U, U * th, atol=1e-10 * lam[0])


@pytest.mark.parametrize("method", ["revd", "nystrom", "ritzit"])
def test_ritz_values_bounds_and_orthonormality(method):
    prob = build(C1)
    A = O.dense_A(prob)
    lam = np.sort(np.linalg.eigvalsh(A))[::-1]
    G = sketch_block(prob.n_A, C1.m, C1.seed)
    U, th = O.METHODS[method](lambda X: O.apply_A(prob, X), G, C1.k_r)
    assert np.all(np.diff(th) <= 1e-12 * th[0])           # decreasing
    assert th.min() >= 1 - 1e-10                           # A >= I
    assert np.all(th <= lam[:C1.k_r] * (1 + 1e-10))       # interlacing / A_nys <= A / sigma(AG) <= lambda
    np.testing.assert_allclose(U.T @ U, np.eye(C1.k_r), atol=1e-10)


def _table1():
    with open(os.path.join(GOLDEN, "table1.json")) as f:
        return json.load(f)["methods"]



@pytest.mark.parametrize("method", ["revd", "nystrom", "ritzit"])
def test_untruncated_outputs_equal_closed_forms(method):
    """Keeping all m pairs, each method's U diag(.) U^T is a matrix with a closed form in the
    sketch (Section 4): REVD the Rayleigh-Ritz projection P_Z A P_Z with Z = orth(A G);
    Nystrom the approximation (A Z)(Z^T A Z)^{-1}(A Z)^T; ritzit Y Y^T = U Theta^2 U^T with
    Y = A orth(G).  The closed forms use a plain solve, not the algorithms' Cholesky,
    triangular solve, SVD or EVD."""
    prob = build(C1)
    A = O.dense_A(prob)
    G = sketch_block(prob.n_A, C1.m, C1.seed)
    U, th = O.METHODS[method](lambda X: O.apply_A(prob, X), G, C1.m)
    if method == "revd":
        Z = np.linalg.qr(A @ G)[0]
        want, got = Z @ (Z.T @ A @ Z) @ Z.T, U @ np.diag(th) @ U.T
    elif method == "nystrom":
        Z = np.linalg.qr(A @ G)[0]
        E1 = A @ Z
        want, got = E1 @ np.linalg.solve(Z.T @ E1, E1.T), U @ np.diag(th) @ U.T
    else:
        Y = A @ np.linalg.qr(G)[0]
        want, got = Y @ Y.T, U @ np.diag(th ** 2) @ U.T
    np.testing.assert_allclose(got, want, atol=1e-9 * np.abs(want).max())


def test_block_product_counts_match_table_1():
    prob = build(C1)
    G = sketch_block(prob.n_A, C1.m, C1.seed)
    for method, row in _table1().items():
        prob.n_apply = 0
        O.METHODS[method](lambda X: O.apply_A(prob, X), G, C1.k_r)
        assert prob.n_apply == row["products_with_A"]


@pytest.mark.parametrize("method", ["revd", "nystrom", "ritzit"])
def test_dense_operations_match_table_1(method, monkeypatch):
    """Every dense factorisation the oracle performs, by kind and operand shape, is the one
    Table 1 lists for the method: orthogonalisation and QR of n_A x (k+l) blocks, Cholesky,
    EVD of (k+l) x (k+l) matrices, the triangular solve and SVD of Nystrom's F."""
    prob = build(C1)
    m = C1.m
    G = sketch_block(prob.n_A, m, C1.seed)
    calls = []

    def shape_of(a):
        return {(prob.n_A, m): "nA", (m, prob.n_A): "nA", (m, m): "small"}[tuple(np.shape(a))]

    def spy(kind, fn, arg=0):
        def wrapped(*a, **kw):
            calls.append((kind, shape_of(a[arg]), a[arg]))
            return fn(*a, **kw)
        return wrapped

    monkeypatch.setattr(np.linalg, "qr", spy("qr", np.linalg.qr))
    monkeypatch.setattr(np.linalg, "cholesky", spy("cholesky", np.linalg.cholesky))
    monkeypatch.setattr(np.linalg, "eigh", spy("evd", np.linalg.eigh))
    monkeypatch.setattr(np.linalg, "svd", spy("svd", np.linalg.svd))
    monkeypatch.setattr(sla, "solve_triangular", spy("triangular_solve", sla.solve_triangular, 1))
    O.METHODS[method](lambda X: O.apply_A(prob, X), G, C1.k_r)
    row = _table1()[method]
    # the first QR-type call orthogonalises G itself (ritzit) or Y = A G (REVD, Nystrom)
    first = calls[0]
    assert first[0] == "qr" and first[1] == "nA"
    assert np.array_equal(first[2], G) == (row["orthogonalise"] == "G")
    rest = calls[1:]
    for kind in ("qr", "cholesky", "triangular_solve", "evd", "svd"):
        assert sorted(s_ for k_, s_, _ in rest if k_ == kind) == sorted(row[kind]), (method, kind)


@pytest.mark.parametrize("method", ["revd", "nystrom", "ritzit"])
def test_outputs_depend_only_on_range_of_sketch(method):
    # any orthonormalisation gives the same Ritz pairs: G -> G O changes nothing
    prob = build(C1)
    G = sketch_block(prob.n_A, C1.m, C1.seed)
    Orot = np.linalg.qr(np.random.default_rng(6).standard_normal((C1.m, C1.m)))[0]
    U1, t1 = O.METHODS[method](lambda X: O.apply_A(prob, X), G, C1.k_r)
    U2, t2 = O.METHODS[method](lambda X: O.apply_A(prob, X), G @ Orot, C1.k_r)
    np.testing.assert_allclose(t1, t2, rtol=1e-9)
    np.testing.assert_allclose(U1 @ U1.T, U2 @ U2.T, atol=1e-8)


# ----------------------------------------------------------------- LMP


def test_lmp_factor_identities():
    prob = build(C1)
    G = sketch_block(prob.n_A, C1.m, C1.seed)
    U, th = O.nystrom(lambda X: O.apply_A(prob, X), G, C1.k_r)
    C = O.lmp_dense_C(U, th)
    P = O.lmp_dense_P(U, th)
    np.testing.assert_allclose(C, C.T, atol=1e-14)
    np.testing.assert_allclose(C @ C.T, P, atol=1e-12)
    np.testing.assert_allclose(O.lmp_dense_C_product(U, th), C, atol=1e-12)
    x = random_block(prob.n_A, 3, 1)
    np.testing.assert_allclose(O.lmp_apply(U, th, x), C @ x, atol=1e-12)


def test_exact_pair_lmp_spectrum_theorem():
    # k exact pairs: at least k unit eigenvalues are added to the n_A - q cluster and the
    # rest stay within [lambda_min, lambda_max] (Section 3.2).  k at a spectral gap.
    prob = build(C1)
    A = O.dense_A(prob)
    lam, V = np.linalg.eigh(A)
    lam, V = lam[::-1], V[:, ::-1]
    gaps = np.where(np.diff(lam[:prob.q]) < -1e-6 * lam[0])[0]
    k = int(gaps[gaps >= 4][0] + 1)
    C = O.lmp_dense_C(V[:, :k], lam[:k])
    mu = np.linalg.eigvalsh(C.T @ A @ C)
    ones = int(np.sum(np.abs(mu - 1) < 1e-8 * lam[0]))
    assert ones == prob.n_A - prob.q + k
    assert mu.min() > 1 - 1e-8 and mu.max() <= lam[k] * (1 + 1e-9)


def test_full_rank_exact_lmp_converges_in_one_iteration():
    prob = build(tiny_advdiff())
    A = O.dense_A(prob)
    lam, V = np.linalg.eigh(A)
    lam, V = lam[::-1], V[:, ::-1]
    q = prob.q
    b = O.rhs(prob, innovations(q, 4, 0.1))
    res = O.pcg(lambda v: A @ v, b, lmp=(V[:, :q], lam[:q]), tol=1e-10, maxit=10)
    assert res.iters == 1 and res.converged


# ----------------------------------------------------------------- PCG


def test_cg_finite_termination_on_three_distinct_eigenvalues():
    rng = np.random.default_rng(7)
    Qm = np.linalg.qr(rng.standard_normal((30, 30)))[0]
    lam = np.repeat([1.0, 7.0, 50.0], 10)
    A = Qm @ np.diag(lam) @ Qm.T
    b = rng.standard_normal(30)
    res = O.pcg(lambda v: A @ v, b, tol=1e-10, maxit=10)
    assert res.iters == 3 and res.converged
    np.testing.assert_allclose(res.x, np.linalg.solve(A, b), rtol=1e-9)


def test_cg_worst_case_bound_and_monotone_cost():
    prob = build(C1)
    A = O.dense_A(prob)
    b = O.rhs(prob, innovations(prob.q, 8, 0.1))
    xs = np.linalg.solve(A, b)
    lam = np.linalg.eigvalsh(A)
    kappa = lam.max() / lam.min()
    rho = (np.sqrt(kappa) - 1) / (np.sqrt(kappa) + 1)
    xs_list = []

    def applyA(v):
        return A @ v

    res = O.pcg(applyA, b, tol=1e-9, maxit=200)
    # recompute iterates through the same recursion to get the A-norm errors
    x = np.zeros_like(b)
    r = b.copy()
    p = r.copy()
    rr = r @ r
    e0 = np.sqrt(xs @ A @ xs)
    for j in range(1, res.iters + 1):
        Ap = A @ p
        a = rr / (p @ Ap)
        x = x + a * p
        r = r - a * Ap
        rn = r @ r
        p = r + (rn / rr) * p
        rr = rn
        e = xs - x
        assert np.sqrt(e @ A @ e) / e0 <= 2 * rho ** j + 1e-12
        xs_list.append(x)
    # oracle iterates agree with this textbook CG and its cost decreases monotonically
    assert np.all(np.diff(res.hist_J) <= 1e-9 * abs(res.hist_J[0]))
    np.testing.assert_allclose(res.x, xs_list[-1], rtol=1e-8)


@pytest.mark.parametrize("method", ["revd", "nystrom", "ritzit"])
def test_pcg_converged_solution_matches_direct_solve(method):
    prob = build(C1)
    A = O.dense_A(prob)
    b = O.rhs(prob, innovations(prob.q, 9, 0.1))
    G = sketch_block(prob.n_A, C1.m, C1.seed)
    U, th = O.METHODS[method](lambda X: O.apply_A(prob, X), G, C1.k_r)
    res = O.pcg(lambda v: O.apply_A(prob, v), b, lmp=(U, th), tol=1e-12, maxit=500)
    assert res.converged
    xs = np.linalg.solve(A, b)
    assert np.linalg.norm(res.x - xs) <= 1e-8 * np.linalg.norm(xs)
    # the recursive true residual agrees with an explicit one
    s = b - A @ res.x
    assert abs(np.linalg.norm(s) / np.linalg.norm(b) - res.relres_true) < 1e-9


def test_pcg_precond_criterion_is_split_residual():
    prob = build(C1)
    b = O.rhs(prob, innovations(prob.q, 10, 0.1))
    G = sketch_block(prob.n_A, C1.m, C1.seed)
    U, th = O.nystrom(lambda X: O.apply_A(prob, X), G, C1.k_r)
    res = O.pcg(lambda v: O.apply_A(prob, v), b, lmp=(U, th), tol=1e-6, maxit=500,
                criterion=O.RES_PRECOND)
    Cb = O.lmp_apply(U, th, b)
    xhat_res = Cb - O.lmp_apply(U, th, O.apply_A(prob, res.x))   # C^T (b - A x)
    assert abs(np.linalg.norm(xhat_res) / np.linalg.norm(Cb) - res.relres_precond) < 1e-9
    assert res.relres_precond <= 1e-6


# ----------------------------------------------------------------- the paper's qualitative results


def section51_workload():
    # Section 5.1's advection experiment: n = 40, N = 50, Courant number 0.8 with the pure
    # upwind scheme, sigma_o = 0.05, sigma_q = 0.05, sigma_b = 0.1, length scales of 10 grid
    # spacings, every 4th variable at every 5th step (100 observations), l = 5, k = 25.  SOAR
    # stands in for Q's Laplacian correlation, which the paper does not specify.
    return Workload(name="sec51", model="advdiff", n=40, N=50, c=0.8, r=0.0, corr="soar", Lb=10.0,
                    Lq=10.0, sigma_b=0.1, sigma_q=0.05, obs_var_stride=4, obs_time_stride=5,
                    sigma_o2=0.05 ** 2, m=30, l=5, seed=5100)


@pytest.mark.parametrize("seed", [5100, 5101])
def test_paper_section51_configuration_statements(seed):
    """Statements of Section 5.1 about its own configuration that a seeded Gaussian start
    block reproduces: Nystrom's leading Ritz values are the most accurate, REVD's slightly
    worse and ritzit's far too small; every preconditioned spectrum drops below one at its
    lower end (REVD furthest, ritzit least) and its largest eigenvalue is far below A's;
    the Nystrom and ritzit LMPs give a smaller condition number than the REVD one; and with
    either of them the quadratic cost falls faster than without preconditioning."""
    w = section51_workload()
    prob = build(w)
    assert (prob.n_A, prob.q) == (2040, 100)
    A = O.dense_A(prob)
    lam = np.sort(np.linalg.eigvalsh(A))[::-1]
    G = sketch_block(prob.n_A, w.m, seed)
    k = w.m - w.l
    top5, mu_min, mu_max, J = {}, {}, {}, {}
    b = O.rhs(prob, innovations(prob.q, seed, 0.05))
    J[None] = O.pcg(lambda v: A @ v, b, tol=1e-14, maxit=5).hist_J
    for method in ("revd", "nystrom", "ritzit"):
        U, th = O.METHODS[method](lambda X: O.apply_A(prob, X), G, k)
        assert np.all(th <= lam[:k] * (1 + 1e-10))
        top5[method] = np.max(np.abs(th[:5] - lam[:5]) / lam[:5])
        C = O.lmp_dense_C(U, th)
        mu = np.linalg.eigvalsh(C @ A @ C)
        mu_min[method], mu_max[method] = mu.min(), mu.max()
        J[method] = O.pcg(lambda v: A @ v, b, lmp=(U, th), tol=1e-14, maxit=5).hist_J
    assert top5["nystrom"] < 1e-3 and top5["nystrom"] < top5["revd"] < 0.1 and top5["ritzit"] > 0.5
    assert mu_min["revd"] < mu_min["nystrom"] < mu_min["ritzit"] < 1.0 and mu_min["revd"] < 0.5
    assert max(mu_max.values()) < 0.05 * lam[0]
    cond = {m_: mu_max[m_] / mu_min[m_] for m_ in mu_max}
    assert cond["nystrom"] < cond["revd"] and cond["ritzit"] < cond["revd"]
    for method in ("nystrom", "ritzit"):
        assert np.all(np.array(J[method][:5]) < np.array(J[None][:5]))


def test_paper_section52_lorenz96_statements():
    """Section 5.2's Lorenz-96 configuration (n = 80, N = 150, F = 8, RK4 with dt = 0.025,
    sigma_o = 0.15, sigma_b = 0.2, sigma_q = 0.1, length scales 2 grid spacings, every 10th
    variable at every 10th step: 120 observations; k = 5, l = 5; SOAR stands in for Q's
    unspecified Laplacian correlation).  The section reports that ritzit gives the worst
    estimate of the largest eigenvalue, and that the smallest eigenvalue of C^T A C is one
    for the Nystrom and ritzit LMPs but below one for REVD's.  A - I has rank q, so every
    eigenvalue of C^T A C other than one lies in span(U, range(A - I)); the test takes them
    from that subspace, exactly, without forming the 12080 x 12080 matrix."""
    w = Workload(name="sec52", model="l96", n=80, N=150, F=8.0, dt=0.025, corr="soar", Lb=2.0, Lq=2.0,
                 sigma_b=0.2, sigma_q=0.1, obs_var_stride=10, obs_time_stride=10, sigma_o2=0.15 ** 2,
                 m=10, l=5, seed=5200)
    prob = build(w)
    assert (prob.n_A, prob.q) == (12080, 120)
    HtR = np.stack([O.apply_HtRinv(prob, e) for e in np.eye(prob.q)], axis=1)
    QW, _ = np.linalg.qr(O.apply_Dsqrt(prob, O.apply_LinvT(prob, HtR)))   # range(A - I)
    lam = np.linalg.eigvalsh(QW.T @ O.apply_A(prob, QW))
    lam_max = lam.max()
    G = sketch_block(prob.n_A, w.m, w.seed)
    err, mu_min = {}, {}
    for method in ("revd", "nystrom", "ritzit"):
        U, th = O.METHODS[method](lambda X: O.apply_A(prob, X), G, w.m - w.l)
        err[method] = abs(th[0] - lam_max) / lam_max
        S, _ = np.linalg.qr(np.hstack([U, QW]))
        M = S.T @ O.lmp_apply(U, th, O.apply_A(prob, O.lmp_apply(U, th, S)))
        mu_min[method] = min(1.0, np.linalg.eigvalsh(0.5 * (M + M.T)).min())
    assert err["ritzit"] > 0.5 and max(err["revd"], err["nystrom"]) < 1e-3
    # "equal to one" as an iterative eigensolver reports it: to three digits
    assert mu_min["nystrom"] >= 1.0 - 1e-3 and mu_min["ritzit"] >= 1.0 - 1e-3
    assert mu_min["revd"] < 0.99


def test_paper_qualitative_lmp_spectra_on_advection():
    # Section 5.1: the REVD-LMP pushes the smallest eigenvalue of C^T A C below one, the
    # Nystrom and ritzit LMPs keep it close to one; ritzit underestimates the largest
    # eigenvalues most.
    prob = build(C1)
    A = O.dense_A(prob)
    lam_max = np.linalg.eigvalsh(A).max()
    G = sketch_block(prob.n_A, C1.m, C1.seed)
    mins, th0 = {}, {}
    for method in ("revd", "nystrom", "ritzit"):
        U, th = O.METHODS[method](lambda X: O.apply_A(prob, X), G, C1.k_r)
        C = O.lmp_dense_C(U, th)
        mins[method] = np.linalg.eigvalsh(C.T @ A @ C).min()
        th0[method] = th[0]
    assert mins["revd"] < 0.9
    assert mins["nystrom"] > mins["revd"] and mins["ritzit"] > mins["revd"]
    assert th0["ritzit"] < th0["revd"] <= lam_max * (1 + 1e-12) and th0["ritzit"] < th0["nystrom"]


# ----------------------------------------------------------------- single-pass Nystrom


def test_single_pass_nystrom_full_sketch_and_invariant_subspace():
    """With a full sketch (m = n_A) the Nystrom approximation is A itself, so every
    eigenvalue comes back; on an invariant subspace the pairs are exact."""
    prob = small_problem()
    A = O.dense_A(prob)
    lam, V = np.linalg.eigh(A)
    lam, V = lam[::-1], V[:, ::-1]
    G = sketch_block(prob.n_A, prob.n_A, 12)
    U, th = O.nystrom_single_pass(lambda X: O.apply_A(prob, X), G, prob.n_A)
    np.testing.assert_allclose(th, lam, rtol=1e-10, atol=1e-10 * lam[0])
    np.testing.assert_allclose(U @ np.diag(th) @ U.T, A, atol=1e-9 * lam[0])
    m = 6
    Gi = V[:, :m] @ np.linalg.qr(np.random.default_rng(5).standard_normal((m, m)))[0]
    U, th = O.nystrom_single_pass(lambda X: O.apply_A(prob, X), Gi, 4)
    np.testing.assert_allclose(th, lam[:4], rtol=1e-11)
    np.testing.assert_allclose(A @ U, U * th, atol=1e-10 * lam[0])


def test_single_pass_nystrom_closed_form_bounds_and_one_product():
    """All m pairs kept: U Theta U^T equals Y (G^T Y)^{-1} Y^T with Y = A G (a plain solve; the
    approximation depends on range(G) only).  It is A^{1/2} P A^{1/2} with P an orthogonal
    projector, so 1 <= theta_i <= lambda_i (A >= I); A is applied once."""
    prob = build(C1)
    A = O.dense_A(prob)
    lam = np.sort(np.linalg.eigvalsh(A))[::-1]
    G = sketch_block(prob.n_A, C1.m, C1.seed)
    prob.n_apply = 0
    U, th = O.nystrom_single_pass(lambda X: O.apply_A(prob, X), G, C1.m)
    assert prob.n_apply == 1
    Y = A @ G
    want = Y @ np.linalg.solve(G.T @ Y, Y.T)
    np.testing.assert_allclose(U @ np.diag(th) @ U.T, want, atol=1e-9 * np.abs(want).max())
    assert np.all(np.diff(th) <= 1e-12 * th[0]) and th.min() >= 1 - 1e-10
    assert np.all(th <= lam[:C1.m] * (1 + 1e-10))
    np.testing.assert_allclose(U.T @ U, np.eye(C1.m), atol=1e-10)


# ----------------------------------------------------------------- Ritz-LMP


def test_ritz_lmp_identities():
    """eq. Ritz_LMP with Rayleigh-Ritz pairs (REVD: U^T A U = Theta) is the general LMP of
    eq. LMP_general with S = U: symmetric, P A U = U, and with exact eigenpairs it equals the
    spectral LMP (eq. spectral_LMP); with all n_A exact pairs it is A^{-1}.  The applied form
    (with A U precomputed) equals the dense formula."""
    prob = small_problem()
    A = O.dense_A(prob)
    G = sketch_block(prob.n_A, 8, 21)
    U, th = O.revd(lambda X: O.apply_A(prob, X), G, 6)
    np.testing.assert_allclose(U.T @ A @ U, np.diag(th), atol=1e-10 * th[0])
    P = O.ritz_lmp_dense(U, th, A)
    np.testing.assert_allclose(P, P.T, atol=1e-12)
    np.testing.assert_allclose(P @ A @ U, U, atol=1e-10)
    S = U @ np.linalg.inv(U.T @ A @ U) @ U.T
    general = (np.eye(prob.n_A) - S @ A) @ (np.eye(prob.n_A) - A @ S) + S
    np.testing.assert_allclose(P, general, atol=1e-10)
    assert np.linalg.eigvalsh(0.5 * (P + P.T)).min() > 0
    v = random_block(prob.n_A, 1, 3)[:, 0]
    np.testing.assert_allclose(O.ritz_lmp_apply(U, th, A @ U, v), P @ v, atol=1e-12)
    lam, V = np.linalg.eigh(A)
    lam, V = lam[::-1], V[:, ::-1]
    np.testing.assert_allclose(O.ritz_lmp_dense(V[:, :5], lam[:5], A), O.lmp_dense_P(V[:, :5], lam[:5]),
                               atol=1e-10)
    np.testing.assert_allclose(O.ritz_lmp_dense(V, lam, A), np.linalg.inv(A), atol=1e-10)


def test_standard_pcg_equals_split_pcg_and_cg():
    """Preconditioned CG with P = C C^T produces Algorithm 1's iterates (exact arithmetic);
    with P = I it is plain CG; with the Ritz-LMP it solves A x = b."""
    prob = build(C1)
    b = O.rhs(prob, innovations(prob.q, C1.seed, np.sqrt(C1.sigma_o2)))
    G = sketch_block(prob.n_A, C1.m, C1.seed)
    U, th = O.revd(lambda X: O.apply_A(prob, X), G, C1.k_r)
    Aop = lambda v: O.apply_A(prob, v)  # noqa: E731
    split = O.pcg(Aop, b, lmp=(U, th), tol=1e-10, maxit=500)
    std = O.pcg_standard(Aop, b, lambda r: O.lmp_apply(U, th, O.lmp_apply(U, th, r)), tol=1e-10, maxit=500)
    k = min(8, split.iters)
    np.testing.assert_allclose(std.hist_J[:k], split.hist_J[:k], rtol=1e-9)
    assert abs(std.iters - split.iters) <= 2
    plain = O.pcg(Aop, b, tol=1e-8, maxit=500)
    ident = O.pcg_standard(Aop, b, lambda r: r, tol=1e-8, maxit=500)
    np.testing.assert_allclose(ident.hist_true[:6], plain.hist_true[:6], rtol=1e-9)
    AU = O.apply_A(prob, U)
    rl = O.pcg_standard(Aop, b, lambda r: O.ritz_lmp_apply(U, th, AU, r), tol=1e-10, maxit=500)
    A = O.dense_A(prob)
    assert rl.converged
    np.testing.assert_allclose(rl.x, np.linalg.solve(A, b), rtol=0, atol=1e-7 * np.abs(np.linalg.solve(A, b)).max())


# ----------------------------------------------------------------- Lanczos-CG and the outer loop


def test_cg_tridiagonal_is_the_lanczos_projection():
    """Section 3.4: T_j built from the CG coefficients is F_j^T A F_j for the normalised
    residuals taken with alternating signs, and its eigenvalues are the Ritz values of A on
    the Krylov space K_j(A, b) (an orthonormal Krylov basis computed independently by QR)."""
    prob = small_problem()
    A = O.dense_A(prob)
    b = random_block(prob.n_A, 1, 31)[:, 0]
    j = 6
    res = O.pcg(lambda v: O.apply_A(prob, v), b, tol=0.0, maxit=j, keep_residuals=True)
    T = O.cg_tridiagonal(res.alphas, res.betas, j)
    F = np.stack([(-1.0) ** i * res.residuals[i] / np.linalg.norm(res.residuals[i]) for i in range(j)], axis=1)
    # the three-term (tridiagonal) relation holds to rounding; entries off the band grow
    # as CG's residuals lose orthogonality, so the full projection is compared for j = 4
    D = F.T @ A @ F - T
    assert np.abs(np.triu(np.tril(D, 1), -1)).max() <= 1e-12 * np.abs(T).max()
    np.testing.assert_allclose(D[:4, :4], 0.0, atol=1e-12 * np.abs(T).max())
    K = np.stack([np.linalg.matrix_power(A, i) @ b for i in range(j)], axis=1)
    Qk = np.linalg.qr(K)[0]
    np.testing.assert_allclose(np.sort(np.linalg.eigvalsh(T)), np.sort(np.linalg.eigvalsh(Qk.T @ A @ Qk)),
                               rtol=1e-8)
    U, th = O.cg_lanczos_pairs(res, 3, j)
    np.testing.assert_allclose(np.einsum("ij,ij->j", U, A @ U), th, rtol=1e-9)   # Rayleigh quotients


def test_cg_lanczos_pairs_converge_to_the_largest_eigenpairs():
    w = tiny_l96(n=20, N=6, vs=2, ts=2)
    prob = build(w)
    A = O.dense_A(prob)
    lam, V = np.linalg.eigh(A)
    b = random_block(prob.n_A, 1, 32)[:, 0]
    res = O.pcg(lambda v: O.apply_A(prob, v), b, tol=0.0, maxit=40, keep_residuals=True)
    U, th = O.cg_lanczos_pairs(res, 2, 40)
    assert abs(th[0] - lam[-1]) <= 1e-8 * lam[-1]
    assert abs(abs(U[:, 0] @ V[:, -1]) - 1.0) <= 1e-6


# ----------------------------------------------------------------- strong constraint


def _no_model_error(prob):
    import copy
    q = copy.copy(prob)
    q.Qsqrt = np.zeros_like(prob.Qsqrt)
    return q


@pytest.mark.parametrize("model", ["advdiff", "l96"])
def test_strong_constraint_is_weak_constraint_without_model_error(model):
    """Section 6's strong-constraint counterpart: with Q^{1/2} = 0 the weak-constraint operator
    maps (x_0, 0, ..., 0) to (A_sc x_0, 0, ..., 0) and its right-hand side is (b_sc, 0, ..., 0)."""
    w = tiny_advdiff(n=8, N=4, vs=2, ts=1) if model == "advdiff" else tiny_l96(n=10, N=4)
    prob = build(w)
    pz = _no_model_error(prob)
    n, N = prob.n, prob.N
    X = random_block(n, 3, 41)
    Xp = np.zeros((prob.n_A, 3))
    Xp[:n] = X
    Yw = O.apply_A(pz, Xp)
    Ys = O.apply_A_sc(prob, X)
    np.testing.assert_allclose(Yw[:n], Ys, rtol=0, atol=1e-12 * np.abs(Ys).max())
    np.testing.assert_allclose(Yw[n:], 0.0, atol=1e-12 * np.abs(Ys).max())
    d = innovations(prob.q, 42, 0.2)
    bw = O.rhs(pz, d)
    bs = O.rhs_sc(prob, d)
    np.testing.assert_allclose(bw[:n], bs, rtol=0, atol=1e-12 * np.abs(bs).max())
    np.testing.assert_allclose(bw[n:], 0.0, atol=1e-12 * np.abs(bs).max())


def test_strong_constraint_dense_assembly_and_spectrum():
    """A_sc from the sweeps equals I + B^{1/2} (sum_i M_{0->i}^T H_i^T R_i^{-1} H_i M_{0->i}) B^{1/2}
    built from explicit matrix products; it is symmetric with eigenvalues >= 1, at most
    min(n, q) of them above one, and a full sketch recovers its spectrum."""
    prob = build(tiny_advdiff(n=12, N=5, vs=3, ts=2))
    n = prob.n
    A = O.apply_A_sc(prob, np.eye(n))
    Ad = O.dense_A_sc(prob)
    np.testing.assert_allclose(A, Ad, rtol=0, atol=1e-12 * np.abs(Ad).max())
    np.testing.assert_allclose(A, A.T, rtol=0, atol=1e-12 * np.abs(A).max())
    lam = np.sort(np.linalg.eigvalsh(A))[::-1]
    assert lam[-1] >= 1.0 - 1e-12
    assert int(np.sum(lam > 1.0 + 1e-9)) <= min(n, prob.q)
    U, th = O.nystrom(lambda Z: O.apply_A_sc(prob, Z), sketch_block(n, n, 5), n)
    np.testing.assert_allclose(th, lam, rtol=1e-10, atol=1e-10 * lam[0])


def _ghost_matrix():
    """A symmetric matrix with five large, well separated eigenvalues over a bulk in [1, 50]
    (the shape of the Hessian's spectrum: a few large eigenvalues above a cluster)."""
    rng = np.random.default_rng(7)
    n = 300
    lam = np.concatenate([[1e4, 5e3, 2.5e3, 1.2e3, 600.0], np.geomspace(1.0, 50.0, n - 5)])
    Q = np.linalg.qr(rng.standard_normal((n, n)))[0]
    A = (Q * lam) @ Q.T
    return 0.5 * (A + A.T), lam, Q, rng.standard_normal(n)


def test_cg_reorthogonalisation_removes_ghost_ritz_values():
    """Section 3.4: without reorthogonalisation, 60 CG iterations repeat the converged largest
    eigenvalue as 'ghost' Ritz values (the normalised residuals lose orthogonality); with
    complete reorthogonalisation the residuals stay orthonormal, the five largest Ritz values
    and vectors are A's five largest eigenpairs, and the first iterates are CG's."""
    A, lam, Q, b = _ghost_matrix()
    plain = O.pcg(lambda v: A @ v, b, tol=0.0, maxit=60, keep_residuals=True)
    _, thp = O.cg_lanczos_pairs(plain, 2, 60)
    assert abs(thp[1] - lam[0]) <= 1e-6 * lam[0]          # a ghost of the largest
    res = O.pcg(lambda v: A @ v, b, tol=0.0, maxit=60, keep_residuals=True, reorth=True)
    F = np.stack([r / np.linalg.norm(r) for r in res.residuals[:60]], axis=1)
    np.testing.assert_allclose(F.T @ F, np.eye(60), atol=1e-13)
    U, th = O.cg_lanczos_pairs(res, 5, 60)
    np.testing.assert_allclose(th, lam[:5], rtol=1e-10)
    for i in range(5):
        assert abs(abs(U[:, i] @ Q[:, i]) - 1.0) <= 1e-10
    # the same iterates as CG while the residuals are still orthogonal
    x5 = O.pcg(lambda v: A @ v, b, tol=0.0, maxit=5).x
    x5r = O.pcg(lambda v: A @ v, b, tol=0.0, maxit=5, reorth=True).x
    np.testing.assert_allclose(x5r, x5, rtol=0.0, atol=1e-13 * np.abs(x5).max())
    with pytest.raises(ValueError):
        O.pcg(lambda v: A @ v, b, lmp=(Q[:, :2], lam[:2]), reorth=True)


def _twin(w, n_outer, inner):
    prob = build(w)
    draws = twin_draws(w, prob.q)
    if draws["x0"] is None:
        draws["x0"] = np.sin(2 * np.pi * np.arange(w.n) / w.n)
    xb, y, _ = O.twin_experiment(prob, draws)
    return prob, O.gauss_newton(prob, xb, y, n_outer, inner)


def _exact_inner(prob, b, j):
    return np.linalg.solve(O.dense_A(prob), b)


def test_gauss_newton_linear_model_converges_in_one_outer_loop():
    """With a linear model and direct observations the incremental cost is the exact cost,
    so one exact inner solve reaches the minimum: the second loop's right-hand side vanishes
    and the nonlinear cost stays at its minimum."""
    w = tiny_advdiff(n=8, N=4)
    prob, recs = _twin(w, 2, _exact_inner)
    assert np.linalg.norm(recs[1]["rhs"]) <= 1e-10 * np.linalg.norm(recs[0]["rhs"])
    assert recs[1]["J"] < recs[0]["J"]
    assert abs(recs[2]["J"] - recs[1]["J"]) <= 1e-10 * recs[1]["J"]


def test_gauss_newton_lorenz96_decreases_the_cost_and_tracks_b():
    """Lorenz-96: each exact Gauss-Newton step lowers the nonlinear cost, the steps shrink,
    and D^{-1/2} b^(1) = -delta p~^(0) (b^(1) = p^(0) - p^(1) with p^(0) = (x^b, 0, ..., 0))."""
    w = tiny_l96(n=12, N=5, vs=2, ts=1)
    prob, recs = _twin(w, 3, _exact_inner)
    Js = [r["J"] for r in recs]
    assert Js[1] < Js[0] and Js[2] < Js[1] and Js[3] <= Js[2] * (1 + 1e-12)
    assert np.linalg.norm(recs[2]["dpt"]) < np.linalg.norm(recs[1]["dpt"]) < np.linalg.norm(recs[0]["dpt"])
    np.testing.assert_allclose(O.dinv_sqrt(recs[1]["prob"], recs[1]["b"]), -recs[0]["dpt"],
                               atol=1e-9 * np.abs(recs[0]["dpt"]).max())
