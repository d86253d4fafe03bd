"""Full-size checks in the launch configurations the benchmark and the batched solve use,
on outputs the oracle can compute one by one.

  * n = 4096, N = 100, m = 256 (the benchmark's workload): sampled columns of a block
    Hessian apply, the Nystrom build the benchmark times (float64 and split-bfloat16
    block products) against the oracle's Nystrom on the same start block, Rayleigh
    quotients of REVD pairs, and the true residual of the float64 and mixed PCG solves;
  * shapes of the 64-problem batch the single-problem tests do not reach: the block sweep
    of n in (4096, 8192] (16 points per thread) at m >= 9, and the single-vector general
    sweep at n > 4096 with N = 200;
  * the learned-sketch workload at full size (Lorenz-96 n = 1024, N = 100, m = 64):
    sampled columns of A and the Nystrom Ritz values.

Bars: float64 blocks per column (largest error within 1e-10 of the column's largest
entry), Ritz values per entry (1e-10 of themselves); the split-bfloat16 build's Ritz
values within 1e-4 theta_1 each (Weyl's bound for the apply's ~1e-5 relative error)."""
import numpy as np
import pytest

from oracle import wc4d_oracle as O
from parity import assert_cols_close, assert_entries_rel
from synthetic import C3, C5, Workload, innovations, l96_initial_state, obs_pattern, random_block, sketch_block

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)


def _dev(A):
    import torch
    A = np.asarray(A, dtype=np.float64)
    return torch.from_numpy(np.ascontiguousarray(A.T if A.ndim == 2 else A)).to("cuda")


@pytest.fixture(scope="module")
def c3():
    from paper_2101_07249_amd import Problem
    say("full-size setup")
    pat = obs_pattern(C3)
    gp = Problem.from_workload(C3, pat)
    op = O.make_problem(C3, pat)
    G = sketch_block(gp.n_A, C3.m, C3.seed)
    Gd = _dev(G)
    return gp, op, G, Gd


@pytest.fixture(scope="module")
def c3_oracle_nystrom(c3):
    """The oracle's Nystrom build on the benchmark's workload and start block (two block
    applies of 256 columns, Householder QR, SVD of F): about a minute of host time."""
    gp, op, G, Gd = c3
    say("full-size oracle Nystrom (host)")
    return O.nystrom(lambda Z: O.apply_A(op, Z), G, C3.k_r)


def test_block_apply_sampled_columns(c3):
    gp, op, G, Gd = c3
    say("full-size block apply")
    Y = gp.apply_A(Gd)
    cols = [0, 137, 255]
    Yg = Y[cols].cpu().numpy().T
    Yo = O.apply_A(op, G[:, cols])
    assert_cols_close(Yg, Yo, 1e-10, "A G")
    # the single-vector (time-blocked) path gives the same column
    y1 = gp.apply_A(Gd[137].contiguous())
    assert_cols_close(y1.cpu().numpy(), Yo[:, 1], 1e-10, "A g (one vector)")


def test_nystrom_build_matches_oracle_fp64(c3, c3_oracle_nystrom):
    """The benchmark's build (Algorithm 4, m = 256) in float64: every Ritz value, and the
    LMP's action on probe vectors, against the oracle's Nystrom from the same block."""
    gp, op, G, Gd = c3
    Uo, tho = c3_oracle_nystrom
    say("full-size nystrom fp64")
    L = gp.lmp_build("nystrom", C3.k_r, C3.l, Gd)
    th = L.theta()
    assert_entries_rel(th, tho, 1e-10, "nystrom theta (C3)")
    V = random_block(gp.n_A, 2, 41)
    CV = L.apply(_dev(V)).cpu().numpy().T
    assert_cols_close(CV, O.lmp_apply(Uo, tho, V), 1e-8, "C V (C3)")
    # single-vector passes (the PCG's): the same action
    cv = L.apply(_dev(V[:, 0])).cpu().numpy()
    assert_cols_close(cv, O.lmp_apply(Uo, tho, V[:, :1])[:, 0], 1e-8, "C v (C3, one vector)")


def test_nystrom_build_matches_oracle_split_bf16(c3, c3_oracle_nystrom):
    """The mixed variant's build (split-bfloat16 block products): Ritz values within 1e-4
    theta_1 of the oracle's float64 ones, each."""
    from paper_2101_07249_amd import Problem, wc4d
    gp, op, G, Gd = c3
    Uo, tho = c3_oracle_nystrom
    say("full-size nystrom split-bf16")
    gm = Problem.from_workload(C3, obs_pattern(C3), prec=wc4d.PREC_SKETCH_BF16X3 | wc4d.PREC_LMP_FP16)
    th = gm.lmp_build("nystrom", C3.k_r, C3.l, Gd).theta()
    e = float(np.abs(th - tho).max() / tho[0])
    print("[result] C3 split-bf16 theta err / theta_1", e, "per entry", float((np.abs(th - tho) / tho).max()),
          flush=True)
    assert e <= 1e-4
    assert e > 1e-12   # really computed from the reduced-precision products


def test_revd_rayleigh_quotients_and_pcg_residual(c3):
    import torch
    gp, op, G, Gd = c3
    say("full-size revd + pcg")
    L = gp.lmp_build("revd", C3.k_r, C3.l, Gd)
    th = L.theta()
    U = L.vectors()
    sel = [0, 1, 50, 250]
    Us = U[sel].cpu().numpy().T
    AU = O.apply_A(op, Us)
    rq = np.einsum("ij,ij->j", Us, AU)
    # Algorithm 3 is a Rayleigh-Ritz projection: theta_i = u_i^T A u_i
    assert_entries_rel(rq, th[sel], 1e-9, "Rayleigh quotients")
    assert np.all(np.diff(th) <= 0) and th[-1] >= 1.0 - 1e-10
    d = torch.from_numpy(innovations(gp.q, C3.seed, np.sqrt(C3.sigma_o2))).to("cuda")
    b = gp.rhs(d)
    x = torch.zeros(gp.n_A, dtype=torch.float64, device="cuda")
    info = gp.pcg(b, x, gp.lmp_build("nystrom", C3.k_r, C3.l, Gd), tol=1e-6, maxit=3000)
    assert info["status"] == 0
    bo = O.rhs(op, innovations(op.q, C3.seed, np.sqrt(C3.sigma_o2)))
    assert_cols_close(b.cpu().numpy(), bo, 1e-10, "rhs (C3)")
    xo = x.cpu().numpy()
    res = np.linalg.norm(bo - O.apply_A(op, xo)) / np.linalg.norm(bo)
    assert res <= 1.05e-6, res
    assert abs(res - info["relres_true"]) <= 1e-8


def test_mixed_precision_pcg_true_residual(c3):
    """The benchmark's headline configuration (split-bf16 sketch products, float16 copy of
    U for the PCG): the solution's true residual from the oracle's float64 operator, and
    the iteration count against the float64 build's (within 5% + 2)."""
    import torch
    from paper_2101_07249_amd import Problem, wc4d
    gp, op, G, Gd = c3
    say("full-size mixed pcg")
    gm = Problem.from_workload(C3, obs_pattern(C3), prec=wc4d.PREC_SKETCH_BF16X3 | wc4d.PREC_LMP_FP16)
    d = torch.from_numpy(innovations(gp.q, C3.seed, np.sqrt(C3.sigma_o2))).to("cuda")
    xm = torch.zeros(gp.n_A, dtype=torch.float64, device="cuda")
    im = gm.pcg(gm.rhs(d), xm, gm.lmp_build("nystrom", C3.k_r, C3.l, Gd), tol=1e-6, maxit=3000)
    xd = torch.zeros(gp.n_A, dtype=torch.float64, device="cuda")
    idd = gp.pcg(gp.rhs(d), xd, gp.lmp_build("nystrom", C3.k_r, C3.l, Gd), tol=1e-6, maxit=3000)
    assert im["status"] == 0 and idd["status"] == 0
    bo = O.rhs(op, innovations(op.q, C3.seed, np.sqrt(C3.sigma_o2)))
    res = np.linalg.norm(bo - O.apply_A(op, xm.cpu().numpy())) / np.linalg.norm(bo)
    print("[result] iters mixed", im["iters"], "fp64", idd["iters"], "true res", res, flush=True)
    assert res <= 1.05e-6, res
    assert im["iters"] <= 1.05 * idd["iters"] + 2


def _adv(n, N, seed, m=16):
    """An advection-diffusion problem shaped like the batched workload's (Bernoulli(1/8)
    observations over (i >= 1, j), SOAR L = 4)."""
    return Workload(name=f"adv_n{n}_N{N}", model="advdiff", n=n, N=N, c=0.5, r=0.1, corr="soar", Lb=4.0,
                    Lq=4.0, sigma_b=1.0, sigma_q=0.1, obs_kind="bernoulli", obs_prob=0.125, sigma_o2=0.01,
                    m=m, l=5, seed=seed)


@pytest.mark.parametrize("n,N,m", [(8192, 6, 9), (6011, 9, 17), (4097, 5, 64)])
def test_large_n_block_sweeps(n, N, m):
    """n in (4096, 8192]: the block sweeps hold 16 points per thread (the widest
    batched problems); every column of L^{-1} X, L^{-T} X and A X against the oracle,
    including a prime n (ragged thread tail)."""
    from paper_2101_07249_amd import Problem
    w = _adv(n, N, 4500 + n)
    say("large-n block sweeps", n, N, m)
    pat = obs_pattern(w)
    gp = Problem.from_workload(w, pat)
    op = O.make_problem(w, pat)
    X = random_block(op.n_A, m, 51)
    Xd = _dev(X)
    for what, gfn, ofn in (("Linv", gp.apply_Linv, O.apply_Linv), ("LinvT", gp.apply_LinvT, O.apply_LinvT),
                           ("A", gp.apply_A, O.apply_A)):
        assert_cols_close(gfn(Xd).cpu().numpy().T, ofn(op, X), 1e-10, f"{what} n={n} m={m}")


@pytest.mark.parametrize("n,N", [(5003, 200), (4500, 137)])
def test_single_vector_long_windows(n, N):
    """One vector at n > 4096 with long windows (N = 200 leaves the single-wave trapezoids
    no owned width, so the general sweep kernels run): L^{-1}, L^{-T} and A against the
    oracle, and a short PCG without an LMP against the oracle's first iterations."""
    import torch
    from paper_2101_07249_amd import Problem
    w = _adv(n, N, 4600 + n)
    say("single vector long window", n, N)
    pat = obs_pattern(w)
    gp = Problem.from_workload(w, pat)
    op = O.make_problem(w, pat)
    x = random_block(op.n_A, 1, 52)[:, 0]
    for what, gfn, ofn in (("Linv", gp.apply_Linv, O.apply_Linv), ("LinvT", gp.apply_LinvT, O.apply_LinvT),
                           ("A", gp.apply_A, O.apply_A)):
        assert_cols_close(gfn(_dev(x)).cpu().numpy(), ofn(op, x[:, None])[:, 0], 1e-10, f"{what} n={n} N={N}")
    d = innovations(op.q, w.seed, 0.1)
    b = O.rhs(op, d)
    xg = torch.zeros(op.n_A, dtype=torch.float64, device="cuda")
    info = gp.pcg(gp.rhs(_dev(d)), xg, None, tol=1e-30, maxit=4)
    ro = O.pcg(lambda v: O.apply_A(op, v), b, tol=1e-30, maxit=4)
    np.testing.assert_allclose(info["hist_true"][:4], ro.hist_true[:4], rtol=1e-8)


@pytest.fixture(scope="module")
def c5():
    from paper_2101_07249_amd import Problem
    say("learned-sketch workload setup (full size)")
    w = C5
    pat = obs_pattern(w, instance=3)
    x0 = l96_initial_state(w.n, w.seed, instance=3)
    gp = Problem.from_workload(w, pat, x0=x0)
    op = O.make_problem(w, pat, x0=x0)
    return w, gp, op


def test_c5_full_size_apply_and_nystrom(c5):
    """Lorenz-96 n = 1024, N = 100 (n_A = 103,424), Bernoulli(1/2) observations at every
    5th step, m = 64: sampled columns of the block apply (the m = 64 launch) and of the
    single-vector apply, and every Nystrom Ritz value against the oracle."""
    w, gp, op = c5
    say("C5 full size")
    G = sketch_block(op.n_A, w.m, w.seed, instance=3)
    Gd = _dev(G)
    Y = gp.apply_A(Gd)
    cols = [0, 31, 63]
    assert_cols_close(Y[cols].cpu().numpy().T, O.apply_A(op, G[:, cols]), 1e-10, "A G (C5)")
    y1 = gp.apply_A(Gd[31].contiguous()).cpu().numpy()
    assert_cols_close(y1, O.apply_A(op, G[:, [31]])[:, 0], 1e-10, "A g (C5, one vector)")
    th = gp.lmp_build("nystrom", w.k_r, w.l, Gd).theta()
    _, tho = O.nystrom(lambda Z: O.apply_A(op, Z), G, w.k_r)
    assert_entries_rel(th, tho, 1e-10, "nystrom theta (C5)")
