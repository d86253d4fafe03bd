"""The outer loop and the previous loop's preconditioner (Sections 2.1, 3.4 and 5.2) on the
GPU against the oracle.

Bars: the CG coefficients and Lanczos vectors of the first iterations per entry / column to
1e-9 (later ones drift as CG loses orthogonality, differently in each evaluation order);
the converged Ritz values of T_j to 1e-8 of themselves; an LMP from given pairs applies
I + U (Theta^{-1/2} - I) U^T to 1e-12 per column; outer-loop right-hand sides per column to
1e-10 for the first loop and, after first loops solved to 1e-12, 1e-7 for the second (the
nonlinear trajectory carries the solves' differences); iteration counts of the second loop
within max(2, 3%) (reading on long CG-like runs)."""
import numpy as np
import pytest

from oracle import philox as PX
from oracle import wc4d_oracle as O
from parity import assert_cols_close, assert_entries_rel
from synthetic import C2, SEC52, Workload, innovations, l96_initial_state, obs_pattern, twin_draws

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    return torch


def dev():
    return _torch().device("cuda", 0)


def say(*a):
    print("[case]", *a, flush=True)


def _pair(w):
    from paper_2101_07249_amd import Problem
    pat = obs_pattern(w)
    x0 = l96_initial_state(w.n, w.seed)
    return Problem.from_workload(w, pat, x0=x0), O.make_problem(w, pat, x0=x0)


def _separated(th, i, gap=1e-3):
    """theta_i is apart from its neighbours by more than gap (relative): its Ritz vector is
    determined up to sign."""
    return all(abs(th[i] - th[q]) > gap * th[i] for q in (i - 1, i + 1) if 0 <= q < len(th))


@pytest.mark.parametrize("reorth", [False, True], ids=["plain", "reorth"])
def test_pcg_lanczos_information_and_ritz_pairs(reorth):
    say("pcg lanczos C2, reorth", reorth)
    w = C2
    gp, op = _pair(w)
    d = innovations(op.q, w.seed, np.sqrt(w.sigma_o2))
    b = O.rhs(op, d)
    x = _torch().zeros(op.n_A, dtype=_torch().float64, device=dev())
    info, al, be, F = gp.pcg_lanczos(gp.rhs(_torch().from_numpy(d).to(dev())), x, tol=1e-6, maxit=300,
                                     reorth=reorth)
    ro = O.pcg(lambda v: O.apply_A(op, v), b, tol=1e-6, maxit=300, keep_residuals=True, reorth=reorth)
    say("  iters gpu", info["iters"], "oracle", ro.iters)
    assert info["status"] == 0 and ro.converged
    assert abs(info["iters"] - ro.iters) <= max(2, int(0.03 * ro.iters))
    assert_entries_rel(al[:5], ro.alphas[:5], 1e-9, "alpha")
    assert_entries_rel(be[:5], ro.betas[:5], 1e-9, "beta")
    Fh = F[:6].cpu().numpy().T
    Fo = np.stack([(-1.0) ** i * ro.residuals[i] / np.linalg.norm(ro.residuals[i]) for i in range(6)], axis=1)
    assert_cols_close(Fh, Fo, 1e-9, "Lanczos vectors")
    j = min(info["iters"], ro.iters)
    U, th = gp.lanczos_pairs(al, be, F, j, 3)
    Uo, tho = O.cg_lanczos_pairs(ro, 3, j)
    say("  Ritz values gpu", th, "oracle", tho)
    assert_entries_rel(th, tho, 1e-8, "Ritz values of T_j")
    Uh = U.cpu().numpy().T
    if reorth:
        # no repeated values: the Lanczos vectors stay orthonormal and every separated Ritz
        # vector matches the oracle's up to sign
        Fj = F[:j].cpu().numpy().T
        G = Fj.T @ Fj
        assert np.abs(G - np.eye(j)).max() <= 1e-10, np.abs(G - np.eye(j)).max()
        assert th[0] > th[1] * (1 + 1e-6)
        for i in range(3):
            if _separated(tho, i):
                assert abs(abs(Uh[:, i] @ Uo[:, i]) - 1.0) <= 1e-8, i
    else:
        # ghosts: a converged value repeats and its Ritz vectors are not unique; the leading
        # vector's Rayleigh quotient must still be its Ritz value
        UA = O.apply_A(op, Uh[:, :1])[:, 0]
        assert abs(Uh[:, 0] @ UA / (Uh[:, 0] @ Uh[:, 0]) - th[0]) <= 1e-6 * th[0]
    # a spectral LMP from these pairs applies I + U (Theta^{-1/2} - I) U^T
    L = gp.lmp_from_pairs(U, th)
    V = np.random.default_rng(3).standard_normal((op.n_A, 2))
    CV = L.apply(_torch().from_numpy(np.ascontiguousarray(V.T)).to(dev())).cpu().numpy().T
    assert_cols_close(CV, O.lmp_apply(Uh, th, V), 1e-12, "C V from given pairs")
    x2 = _torch().zeros(op.n_A, dtype=_torch().float64, device=dev())
    i2 = gp.pcg(gp.rhs(_torch().from_numpy(d).to(dev())), x2, L, tol=1e-6, maxit=300)
    assert i2["status"] == 0


def _small_l96():
    return Workload(name="gn_l96", model="l96", n=40, N=10, F=8.0, dt=0.025, corr="soar", Lb=2.0, Lq=2.0,
                    sigma_b=0.2, sigma_q=0.1, obs_var_stride=2, obs_time_stride=2, sigma_o2=0.15 ** 2, m=10, l=5,
                    seed=5300)


def test_outer_loop_against_oracle():
    """Two Gauss-Newton loops with first loops solved to 1e-12: the right-hand sides of both
    loops against the oracle's outer loop on the same identical-twin draws."""
    from paper_2101_07249_amd.outer_loop import OuterLoopL96
    say("outer loop small L96")
    w = _small_l96()
    pat = obs_pattern(w)
    op = O.make_problem(w, pat, x0=l96_initial_state(w.n, w.seed))
    draws = twin_draws(w, op.q)
    exp = OuterLoopL96(w, pat, draws)

    def inner(prob, rhs, j):
        x = _torch().zeros(prob.n_A, dtype=_torch().float64, device=dev())
        info = prob.pcg(rhs, x, None, tol=1e-12, maxit=2000)
        assert info["status"] == 0
        return x

    recs = exp.run(2, inner)
    xb, y, _ = O.twin_experiment(op, draws)
    np.testing.assert_allclose(exp.xb, xb, rtol=0, atol=1e-12 * np.abs(xb).max())
    orecs = O.gauss_newton(op, xb, y, 2, lambda prob, b, j: O.pcg(lambda v: O.apply_A(prob, v), b, tol=1e-12,
                                                                  maxit=2000).x)
    assert_cols_close(recs[0]["rhs"], orecs[0]["rhs"], 1e-10, "rhs of the first loop")
    assert_cols_close(recs[1]["rhs"], orecs[1]["rhs"], 1e-7, "rhs of the second loop")
    assert orecs[2]["J"] < orecs[1]["J"] < orecs[0]["J"]


def test_second_loop_study_section52():
    """Section 5.2's configuration: the first loop's reorthogonalised CG (solved to 1e-10 here
    so that both sides linearise the second loop about the same state to ~1e-10) and its
    previous-loop LMP (k = 5), against the oracle's same study: the first loop's largest Ritz
    value, and per preconditioner of the second loop the outcome (converged or not within
    1000 iterations), the quadratic cost (the quantity Section 5.2's figures plot): monotone
    over the first ten iterations and the first three to 1e-6 of the oracle's (with condition
    numbers ~1e8 the two evaluation orders part after a few iterations: measured 10% apart at
    the eighth without an LMP), and the iteration count (within max(2, 15%) when converged:
    the true residual of these solves jumps by up to 100x between iterations, so where it
    first crosses 1e-6 depends on rounding; measured 11%)."""
    from paper_2101_07249_amd.outer_loop import OuterLoopL96, second_loop_study
    say("second loop study, Section 5.2 configuration")
    w = SEC52
    pat = obs_pattern(w)
    op = O.make_problem(w, pat, x0=l96_initial_state(w.n, w.seed))
    draws = twin_draws(w, op.q)
    exp = OuterLoopL96(w, pat, draws)
    res = second_loop_study(exp, ks=(5,), methods=("nystrom", "ritzit"), seed=11, first_tol=1e-10, first_maxit=300)
    say("  ", {k: (v["iters"], v["status"]) for k, v in res["second"].items()})
    # the oracle's study on the same draws
    xb, y, _ = O.twin_experiment(op, draws)
    st = {}

    def inner(prob, b, j):
        if j == 0:
            r = O.pcg(lambda v: O.apply_A(prob, v), b, tol=1e-10, maxit=300, keep_residuals=True, reorth=True)
            st["first"] = r
            return r.x
        st["prob1"], st["b1"] = prob, b
        return np.zeros_like(b)

    O.gauss_newton(op, xb, y, 2, inner)
    assert abs(st["first"].iters - res["first_loop_iters"]) <= max(2, int(0.03 * st["first"].iters))
    U, th = O.cg_lanczos_pairs(st["first"], 5)
    say("   first loop's largest Ritz value gpu", res["second"]["previous_loop_k5"]["theta_max"], "oracle", th[0])
    assert abs(res["second"]["previous_loop_k5"]["theta_max"] - th[0]) <= 1e-8 * th[0]
    p1, b1 = st["prob1"], st["b1"]
    r_none = O.pcg(lambda v: O.apply_A(p1, v), b1, tol=1e-6, maxit=1000)
    r_prev = O.pcg(lambda v: O.apply_A(p1, v), b1, lmp=(U, th), tol=1e-6, maxit=1000)
    G = PX.gaussian_block(11, p1.n_A, 10)
    Un, tn = O.nystrom(lambda X: O.apply_A(p1, X), G, 5)
    r_ny = O.pcg(lambda v: O.apply_A(p1, v), b1, lmp=(Un, tn), tol=1e-6, maxit=1000)
    Ur, tr = O.ritzit(lambda X: O.apply_A(p1, X), G, 5)
    r_rz = O.pcg(lambda v: O.apply_A(p1, v), b1, lmp=(Ur, tr), tol=1e-6, maxit=1000)
    for name, ro in (("none", r_none), ("previous_loop_k5", r_prev), ("nystrom_k5", r_ny), ("ritzit_k5", r_rz)):
        got = res["second"][name]
        say("  ", name, "gpu", got["iters"], got["status"], "oracle", ro.iters, ro.converged)
        say("     J gpu", np.array(got["J"][:6]), "oracle", np.array(ro.hist_J[:6]))
        # CG lowers J monotonically; on this ill-conditioned system (kappa ~ 1e8) the two
        # evaluation orders part after a few iterations, so only the first three are compared
        Jg = np.array(got["J"][:10])
        assert np.all(np.diff(Jg) <= 1e-9 * np.abs(Jg[1:])), (name, Jg)
        assert_entries_rel(Jg[:3], np.array(ro.hist_J[:3]), 1e-6, name + " J")
        assert (got["status"] == 0) == ro.converged
        if ro.converged:
            # the true residual oscillates by up to two orders of magnitude between
            # iterations on this configuration, so its 1e-6 crossing moves with rounding
            assert abs(got["iters"] - ro.iters) <= max(2, int(0.15 * ro.iters)), name
        else:
            assert got["iters"] == ro.iters
