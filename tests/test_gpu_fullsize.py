"""Full-size checks at n = 4096, N = 100, m = 256 (the benchmark's workload), in the
launch configurations the benchmark uses, on outputs the oracle can compute one by
one: sampled columns of a block Hessian apply, Rayleigh quotients of REVD Ritz
pairs, and the true residual of a PCG solution."""
import numpy as np
import pytest

from oracle import wc4d_oracle as O
from synthetic import C3, innovations, obs_pattern, sketch_block

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def c3():
    import torch
    from paper_2101_07249_amd import Problem
    print("[case] full-size setup", flush=True)
    pat = obs_pattern(C3)
    gp = Problem.from_workload(C3, pat)
    op = O.make_problem(C3, pat)
    G = sketch_block(gp.n_A, C3.m, C3.seed)
    Gd = torch.from_numpy(np.ascontiguousarray(G.T)).to("cuda")
    return gp, op, G, Gd


def test_block_apply_sampled_columns(c3):
    gp, op, G, Gd = c3
    print("[case] full-size block apply", flush=True)
    Y = gp.apply_A(Gd)
    cols = [0, 137, 255]
    Yg = Y[cols].cpu().numpy().T
    Yo = O.apply_A(op, G[:, cols])
    assert np.linalg.norm(Yg - Yo) <= 1e-10 * np.linalg.norm(Yo)
    # the single-vector (time-blocked) path gives the same column
    y1 = gp.apply_A(Gd[137].contiguous())
    assert np.linalg.norm(y1.cpu().numpy() - Yo[:, 1]) <= 1e-10 * np.linalg.norm(Yo[:, 1])


def test_revd_rayleigh_quotients_and_pcg_residual(c3):
    import torch
    gp, op, G, Gd = c3
    print("[case] full-size revd + pcg", flush=True)
    L = gp.lmp_build("revd", C3.k_r, C3.l, Gd)
    th = L.theta()
    U = L.vectors()
    sel = [0, 1, 50, 250]
    Us = U[sel].cpu().numpy().T
    AU = O.apply_A(op, Us)
    rq = np.einsum("ij,ij->j", Us, AU)
    # Algorithm 3 is a Rayleigh-Ritz projection: theta_i = u_i^T A u_i
    np.testing.assert_allclose(rq, th[sel], rtol=1e-9)
    assert np.all(np.diff(th) <= 0) and th[-1] >= 1.0 - 1e-10
    d = torch.from_numpy(innovations(gp.q, C3.seed, np.sqrt(C3.sigma_o2))).to("cuda")
    b = gp.rhs(d)
    x = torch.zeros(gp.n_A, dtype=torch.float64, device="cuda")
    info = gp.pcg(b, x, gp.lmp_build("nystrom", C3.k_r, C3.l, Gd), tol=1e-6, maxit=3000)
    assert info["status"] == 0
    bo = O.rhs(op, innovations(op.q, C3.seed, np.sqrt(C3.sigma_o2)))
    assert np.linalg.norm(b.cpu().numpy() - bo) <= 1e-10 * np.linalg.norm(bo)
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
    print("[case] full-size mixed pcg", flush=True)
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
