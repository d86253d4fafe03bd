"""GPU parity: the HIP path (through the C-ABI) against the FP64 CPU oracle on the
same seeded inputs.  FP64 path bar: every column within 1e-10 of its largest entry
(max-abs per column) and every Ritz value within 1e-10 of itself, unless a test
states and justifies another bound."""
import numpy as np
import pytest

from oracle import wc4d_oracle as O
from parity import assert_cols_close, assert_entries_rel
from synthetic import (C1, C2, Workload, innovations, l96_initial_state, obs_pattern, random_block,
                       sketch_block)

pytestmark = pytest.mark.gpu

TOL = 1e-10


def _torch():
    import torch
    return torch


def dev():
    return _torch().device("cuda", 0)


def to_dev(A):
    """(n_A, m) numpy -> (m, n_A) contiguous CUDA tensor (column-major block)."""
    t = _torch()
    A = np.asarray(A, dtype=np.float64)
    if A.ndim == 1:
        return t.from_numpy(A.copy()).to(dev())
    return t.from_numpy(np.ascontiguousarray(A.T)).to(dev())


def to_host(T):
    a = T.cpu().numpy()
    return a if a.ndim == 1 else a.T


def relerr(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def say(*a):
    print("[case]", *a, flush=True)


def tiny(model="advdiff", n=8, N=4, vs=2, ts=2, m=4, **kw):
    if model == "advdiff":
        return Workload(name="tiny", model="advdiff", n=n, N=N, c=0.5, r=0.1, corr="soar", Lb=2.0,
                        Lq=2.0, sigma_b=1.0, sigma_q=0.3, obs_var_stride=vs, obs_time_stride=ts,
                        sigma_o2=0.01, m=m, l=2, seed=17, **kw)
    return Workload(name="tinyl96", model="l96", n=n, N=N, F=8.0, dt=0.025, corr="gauss", Lb=2.0,
                    Lq=2.0, sigma_b=0.2, sigma_q=0.1, obs_var_stride=vs, obs_time_stride=ts,
                    sigma_o2=0.04, m=m, l=2, seed=29, **kw)


def pair(w, pattern=None):
    from paper_2101_07249_amd import Problem
    pat = obs_pattern(w) if pattern is None else pattern
    x0 = l96_initial_state(w.n, w.seed) if w.model == "l96" else None
    gp = Problem.from_workload(w, pat, x0=x0)
    op = O.make_problem(w, pat, x0=x0)
    return gp, op


CASES = {
    "C1": C1,
    "C2": C2,
    "tiny_adv": tiny(),
    "tiny_l96": tiny("l96", n=10),
    "ragged_adv": tiny(n=37, N=7, vs=3, ts=1),           # n not a multiple of any tile
    "ragged_l96": tiny("l96", n=67, N=5, vs=5, ts=1),    # several waves, ragged tail
    "wide_adv": tiny(n=300, N=3, vs=7, ts=3),             # PE 4, W 250 (m > 8: 2 points/thread)
    "n1_adv": tiny(n=1, N=6, vs=1, ts=2),
    # single-wave trapezoid sweeps (m <= 8): each wavefront owns W points and runs the
    # extended range of 64 PE points, W = 64 PE - 2N; the last wavefront owns fewer
    "tb_adv": tiny(n=600, N=30, vs=5, ts=3),      # PE 4, W 196: 4 wavefronts, last owns 12
    "tb_adv2": tiny(n=1100, N=100, vs=7, ts=2),   # PE 8, W 312: 4 wavefronts, last owns 164
    "tb_adv4": tiny(n=1100, N=150, vs=9, ts=5),   # PE 8, W 212: 6 wavefronts, last owns 40
    "tb_adv3": tiny(n=1100, N=200, vs=9, ts=5),   # N = 200 leaves W < 128: the general kernel
    # B and Q with different length scales: D^{1/2} as two products (no B = c Q shortcut)
    "bq_adv": tiny(n=600, N=30, vs=5, ts=3).with_(Lq=3.0),
    # (Gaussian L = 1.5: smallest correlation eigenvalue 1.5e-5; a longer scale on n = 256
    # drops eigenvalues below rounding, where any two square roots differ near sqrt(eps))
    "bq_l96": tiny("l96", n=256, N=9, vs=3, ts=2).with_(Lb=1.5),
    # single-vector Lorenz-96 sweeps (m = 1, n = 64 PPT): one wavefront, shuffled halos
    "l96_v4": tiny("l96", n=256, N=9, vs=3, ts=2),
    "l96_v16": tiny("l96", n=1024, N=20, vs=5, ts=4),
}


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("m", [1, 3, 17])
def test_operator_pieces(name, m):
    w = CASES[name]
    say("operator pieces", name, "m", m)
    gp, op = pair(w)
    X = random_block(op.n_A, m, 100 + m)
    Xd = to_dev(X)
    for what, gfn, ofn in (("Dsqrt", gp.apply_Dsqrt, O.apply_Dsqrt),
                           ("Linv", gp.apply_Linv, O.apply_Linv),
                           ("LinvT", gp.apply_LinvT, O.apply_LinvT),
                           ("A", gp.apply_A, O.apply_A)):
        Y = to_host(gfn(Xd))
        Yo = ofn(op, X)
        assert_cols_close(Y, Yo, TOL, what)


@pytest.mark.parametrize("m", [1, 130, 260])
def test_apply_A_block_widths_C2(m):
    # widths across the GEMM tile configurations (16 / 32 / 64 / 128 columns) and ragged tails
    say("apply_A widths C2", m)
    gp, op = pair(C2)
    X = sketch_block(op.n_A, m, 7)
    Y = to_host(gp.apply_A(to_dev(X)))
    assert_cols_close(Y, O.apply_A(op, X), TOL, "A")


def test_rhs_and_no_observation_operator():
    say("rhs C1")
    gp, op = pair(C1)
    d = innovations(op.q, 5, 0.1)
    b = to_host(gp.rhs(to_dev(d)))
    assert_cols_close(b, O.rhs(op, d), TOL, "rhs")
    bt = random_block(op.n_A, 1, 3)[:, 0]
    b2 = to_host(gp.rhs(to_dev(d), bt=to_dev(bt)))
    assert_cols_close(b2, O.rhs(op, d, bt=bt), TOL, "rhs + bt")
    # without observations A is the identity
    say("q = 0")
    w = tiny()
    gp0, op0 = pair(w, pattern=[])
    X = random_block(op0.n_A, 3, 4)
    np.testing.assert_array_equal(to_host(gp0.apply_A(to_dev(X))), X)


def test_symmetry_and_adjoint_on_device():
    say("symmetry C2")
    gp, op = pair(C2)
    U = random_block(op.n_A, 2, 8)
    AU = to_host(gp.apply_A(to_dev(U)))
    assert abs(U[:, 0] @ AU[:, 1] - U[:, 1] @ AU[:, 0]) <= 1e-12 * abs(U[:, 0] @ AU[:, 1])
    LU = to_host(gp.apply_Linv(to_dev(U)))
    LTU = to_host(gp.apply_LinvT(to_dev(U)))
    assert abs(LU[:, 0] @ U[:, 1] - U[:, 0] @ LTU[:, 1]) <= 1e-12 * abs(LU[:, 0] @ U[:, 1])


def _lmp_check(w, method, G=None):
    gp, op = pair(w)
    G = sketch_block(op.n_A, w.m, w.seed) if G is None else G
    L = gp.lmp_build(method, w.k_r, w.l, to_dev(G))
    th = L.theta()
    U = to_host(L.vectors())
    op.n_apply = 0
    Uo, tho = O.METHODS[method](lambda Z: O.apply_A(op, Z), G, w.k_r)
    assert L.applies == op.n_apply
    e_th = assert_entries_rel(th, tho, TOL, f"{method} theta")
    assert np.all(np.diff(th) <= 0)
    np.testing.assert_allclose(U.T @ U, np.eye(w.k_r), atol=1e-10)
    # the preconditioner's action (independent of the basis chosen inside clusters)
    V = random_block(op.n_A, 4, 9)
    CV = to_host(L.apply(to_dev(V)))
    CVo = O.lmp_apply(Uo, tho, V)
    return gp, op, L, e_th, (CV, CVo)


@pytest.mark.parametrize("method", ["revd", "nystrom", "ritzit", "nystrom1p"])
@pytest.mark.parametrize("wname", ["C1", "C2"])
def test_lmp_build_matches_oracle(method, wname):
    say("lmp build", wname, method)
    w = CASES[wname]
    _, _, _, e_th, (CV, CVo) = _lmp_check(w, method)
    # C V depends on the Ritz vectors, whose rounding error is eps * ||A|| / gap for
    # nearly repeated Ritz values; the bound below is that of the oracle itself
    # under a different (Householder vs CholeskyQR2) orthonormalisation.
    assert_cols_close(CV, CVo, 1e-8, f"{method} C V")


@pytest.mark.parametrize("variant", [0, 1])
@pytest.mark.parametrize("method", ["revd", "nystrom", "ritzit", "nystrom1p"])
def test_pcg_matches_oracle_C1(method, variant):
    say("pcg C1", method, "variant", variant)
    w = C1
    gp, op = pair(w)
    G = sketch_block(op.n_A, w.m, w.seed)
    L = gp.lmp_build(method, w.k_r, w.l, to_dev(G))
    d = innovations(op.q, w.seed, np.sqrt(w.sigma_o2))
    b = O.rhs(op, d)
    bd = gp.rhs(to_dev(d))
    x = _torch().zeros(op.n_A, dtype=_torch().float64, device=dev())
    info = gp.pcg(bd, x, L, tol=1e-6, maxit=500, variant=variant)
    Uo, tho = O.METHODS[method](lambda Z: O.apply_A(op, Z), G, w.k_r)
    ro = O.pcg(lambda v: O.apply_A(op, v), b, lmp=(Uo, tho), tol=1e-6, maxit=500)
    assert info["status"] == 0 and ro.converged
    assert abs(info["iters"] - ro.iters) <= 2, (info["iters"], ro.iters)
    # first iterations agree closely (evaluation orders differ after that)
    k = min(5, info["iters"], ro.iters)
    np.testing.assert_allclose(info["hist_true"][:k], ro.hist_true[:k], rtol=1e-8)
    np.testing.assert_allclose(info["hist_J"][:k], ro.hist_J[:k], rtol=1e-8)
    # solved to tol: the two solutions differ by at most the two solves' errors
    A = O.dense_A(op)
    xs = np.linalg.solve(A, b)
    xg = to_host(x)
    kappa = np.linalg.cond(A)
    assert np.linalg.norm(xg - xs) <= kappa * 1e-6 * np.linalg.norm(xs)
    s = b - A @ xg
    assert np.linalg.norm(s) / np.linalg.norm(b) <= 1.01e-6


@pytest.mark.parametrize("variant", [0, 1])
@pytest.mark.parametrize("method", ["revd", "nystrom", "ritzit", None])
def test_pcg_tight_solution_C2(method, variant):
    say("pcg tight C2", method, "variant", variant)
    w = C2
    gp, op = pair(w)
    G = sketch_block(op.n_A, w.m, w.seed)
    L = gp.lmp_build(method, w.k_r, w.l, to_dev(G)) if method else None
    d = innovations(op.q, w.seed, np.sqrt(w.sigma_o2))
    b = O.rhs(op, d)
    x = _torch().zeros(op.n_A, dtype=_torch().float64, device=dev())
    info = gp.pcg(gp.rhs(to_dev(d)), x, L, tol=1e-11, maxit=3000, variant=variant)
    assert info["status"] == 0, info
    if method:
        Uo, tho = O.METHODS[method](lambda Z: O.apply_A(op, Z), G, w.k_r)
        ro = O.pcg(lambda v: O.apply_A(op, v), b, lmp=(Uo, tho), tol=1e-11, maxit=3000)
    else:
        ro = O.pcg(lambda v: O.apply_A(op, v), b, tol=1e-11, maxit=3000)
    assert ro.converged
    # both solutions satisfy ||b - A x|| <= 1e-11 ||b||; they agree to kappa-scaled 1e-11
    xg = to_host(x)
    # measured on the CPU: two FP64 solves to 1e-11 differ by ~1e-11 of the largest entry
    assert_cols_close(xg, ro.x, 1e-8, "x")
    assert np.linalg.norm(b - O.apply_A(op, xg)) / np.linalg.norm(b) <= 2e-11
    # iteration counts at 1e-6: within 2 with an LMP; without a second-level preconditioner
    # (177 iterations here) within max(2, 3%): plain CG is the Lanczos process (Section 3.4)
    # and loses orthogonality at a rate set by rounding, so rounding-level differences of
    # the operator move the 1e-6 crossing of its flat residual curve by a few iterations
    x6 = _torch().zeros(op.n_A, dtype=_torch().float64, device=dev())
    i6 = gp.pcg(gp.rhs(to_dev(d)), x6, L, tol=1e-6, maxit=3000, variant=variant)
    r6 = O.pcg(lambda v: O.apply_A(op, v), b, lmp=(Uo, tho) if method else None, tol=1e-6, maxit=3000)
    slack = 2 if method else max(2, int(0.03 * r6.iters))
    assert abs(i6["iters"] - r6.iters) <= slack, (i6["iters"], r6.iters)


def test_pcg_precond_criterion_and_nonzero_start():
    say("pcg precond criterion / x0")
    from paper_2101_07249_amd import wc4d
    w = C1
    gp, op = pair(w)
    G = sketch_block(op.n_A, w.m, w.seed)
    L = gp.lmp_build("nystrom", w.k_r, w.l, to_dev(G))
    d = innovations(op.q, w.seed, np.sqrt(w.sigma_o2))
    b = O.rhs(op, d)
    x0 = random_block(op.n_A, 1, 12)[:, 0]
    x = to_dev(x0)
    info = gp.pcg(gp.rhs(to_dev(d)), x, L, tol=1e-6, maxit=500, criterion=wc4d.RES_PRECOND)
    Uo, tho = O.nystrom(lambda Z: O.apply_A(op, Z), G, w.k_r)
    ro = O.pcg(lambda v: O.apply_A(op, v), b, x0=x0, lmp=(Uo, tho), tol=1e-6, maxit=500,
               criterion=O.RES_PRECOND)
    assert info["status"] == 0 and abs(info["iters"] - ro.iters) <= 2
    assert info["relres_precond"] <= 1e-6


def test_error_paths():
    from paper_2101_07249_amd import Problem, Wc4dError, wc4d
    t = _torch()
    say("error paths")
    # repeated observation index
    p = Problem(8, 3)
    with pytest.raises(Wc4dError) as ei:
        p.set_obs(1, np.array([1, 1]), np.array([0.1, 0.1]))
    assert ei.value.code == wc4d.EINVAL
    # apply before finalize
    with pytest.raises(Wc4dError) as ei:
        p.apply_A(t.zeros((1, 32), dtype=t.float64, device=dev()))
    assert ei.value.code == wc4d.ESTATE
    # rank-deficient sketch: duplicated columns -> Cholesky failure
    gp, op = pair(C1)
    G = sketch_block(op.n_A, C1.m, 3)
    G[:, 1] = G[:, 0]
    with pytest.raises(Wc4dError) as ei:
        gp.lmp_build("revd", C1.k_r, C1.l, to_dev(G))
    assert ei.value.code == wc4d.ENOTSPD
    # NaN right-hand side -> breakdown; tiny maxit -> no convergence
    b = t.full((op.n_A,), float("nan"), dtype=t.float64, device=dev())
    x = t.zeros(op.n_A, dtype=t.float64, device=dev())
    assert gp.pcg(b, x, None, tol=1e-6, maxit=10)["status"] == wc4d.EBREAKDOWN
    d = innovations(op.q, 1, 0.1)
    x = t.zeros(op.n_A, dtype=t.float64, device=dev())
    assert gp.pcg(gp.rhs(to_dev(d)), x, None, tol=1e-12, maxit=3)["status"] == wc4d.ENOCONV
    # zero right-hand side: x = 0 in zero iterations
    x = t.zeros(op.n_A, dtype=t.float64, device=dev())
    info = gp.pcg(t.zeros(op.n_A, dtype=t.float64, device=dev()), x, None, tol=1e-6, maxit=10)
    assert info["status"] == 0 and info["iters"] == 0


def test_lmp_outliving_its_problem_is_rejected():
    from paper_2101_07249_amd import Wc4dError
    say("lmp after problem destroy")
    w = tiny()
    gp, op = pair(w)
    L = gp.lmp_build("revd", 2, 2, to_dev(sketch_block(op.n_A, 4, 5)))
    gp.close()
    with pytest.raises(Wc4dError) as e:
        L.theta()
    assert e.value.code == -7
    L.close()


@pytest.mark.parametrize("method", ["revd", "nystrom", "ritzit"])
def test_ill_conditioned_sketch_takes_shifted_choleskyqr(method):
    """Column 1 of G is column 0 plus 1e-9 times an independent Gaussian vector (full
    rank, condition about 1e9): the Gram matrix of A G is far too
    ill-conditioned for CholeskyQR2 (its Cholesky breaks down), so the build retries with
    shifted CholeskyQR3.  The leading Ritz pairs still match the oracle (Householder QR)."""
    say("shifted CholeskyQR", method)
    gp, op = pair(C2)
    G = sketch_block(op.n_A, C2.m, 41)
    G[:, 1] = G[:, 0] + 1e-9 * random_block(op.n_A, 1, 42)[:, 0]
    L = gp.lmp_build(method, C2.k_r, C2.l, to_dev(G))
    th = L.theta()
    U = to_host(L.vectors())
    L.close()
    _, th_o = O.METHODS[method](lambda X: O.apply_A(op, X), G, C2.k_r)
    assert np.all(th >= 1.0 - 1e-8)
    np.testing.assert_allclose(th[:5], th_o[:5], rtol=1e-4)
    assert np.abs(U.T @ U - np.eye(C2.k_r)).max() <= 1e-9


@pytest.mark.parametrize("variant", [0, 1])
def test_pcg_maxit_at_chunk_boundaries(variant):
    """The host enqueues iterations in chunks of 8 and reads the state of one chunk while the
    next runs: a solve that cannot converge stops after exactly maxit iterations for maxit on
    either side of the chunk boundaries, and its first iterations follow the oracle's."""
    from paper_2101_07249_amd import wc4d
    t = _torch()
    say("pcg maxit chunks, variant", variant)
    w = C1
    gp, op = pair(w)
    G = sketch_block(op.n_A, w.m, w.seed)
    L = gp.lmp_build("nystrom", w.k_r, w.l, to_dev(G))
    d = innovations(op.q, w.seed, np.sqrt(w.sigma_o2))
    b = O.rhs(op, d)
    Uo, tho = O.METHODS["nystrom"](lambda Z: O.apply_A(op, Z), G, w.k_r)
    ro = O.pcg(lambda v: O.apply_A(op, v), b, lmp=(Uo, tho), tol=1e-14, maxit=17)
    for maxit in (1, 7, 8, 9, 16, 17):
        x = t.zeros(op.n_A, dtype=t.float64, device=dev())
        info = gp.pcg(gp.rhs(to_dev(d)), x, L, tol=1e-14, maxit=maxit, variant=variant)
        assert info["status"] == wc4d.ENOCONV and info["iters"] == maxit, (maxit, info["status"], info["iters"])
        k = min(maxit, 5)
        np.testing.assert_allclose(info["hist_true"][:k], ro.hist_true[:k], rtol=1e-8)


def test_prof_stride_samples_launch_groups():
    """With stride s only every s-th launch group of a timed class is bracketed by events."""
    say("prof stride")
    t = _torch()
    gp, op = pair(C2)
    X = to_dev(random_block(op.n_A, 3, 5))
    Y = t.empty_like(X)
    for every, want in ((1, 16), (4, 4), (5, 4)):
        gp.prof_enable(True, classes=["dsqrt_gemm"])
        gp.prof_stride(every)
        for _ in range(8):   # two D^{1/2} launch groups per apply
            gp.apply_A(X, Y)
        prof = gp.prof_read()
        gp.prof_enable(False)
        gp.prof_stride(1)
        assert prof["dsqrt_gemm"]["launches"] == want, (every, prof["dsqrt_gemm"])
        assert prof["sweep_fwd"]["launches"] == 0
        assert prof["dsqrt_gemm"]["ms"] > 0
