"""The strong-constraint operator (control x_0 only) on the GPU against the oracle's
strong-constraint functions: A_sc X and the right-hand side per column to 1e-10 of the
column's largest entry (float64 throughout: the weak-constraint apply's bar; 150 Lorenz-96
tangent-linear steps amplify rounding to ~1e-12), Ritz values of the randomised builds to 1e-10 of themselves, PCG iterations within
2 of the oracle's with an LMP (short runs) and the true residual reached; size-dependent
errors on the host."""
import numpy as np
import pytest

from oracle import wc4d_oracle as O
from parity import assert_cols_close, assert_entries_rel
from synthetic import C1, C3, SEC52, innovations, l96_initial_state, obs_pattern, random_block, sketch_block

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)


def _pair(w):
    from paper_2101_07249_amd import Problem
    pat = obs_pattern(w)
    x0 = l96_initial_state(w.n, w.seed) if w.model == "l96" else None
    return Problem.from_workload(w, pat, x0=x0, strong=True), O.make_problem(w, pat, x0=x0)


def _t(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a).T)).to("cuda")


@pytest.mark.parametrize("w", [C1, SEC52], ids=["advdiff", "l96"])
def test_strong_apply_and_rhs(w):
    say("strong apply", w.name)
    gp, op = _pair(w)
    assert gp.n_A == w.n
    X = random_block(w.n, 5, 3)
    Y = gp.apply_A(_t(X)).cpu().numpy().T
    assert_cols_close(Y, O.apply_A_sc(op, X), 1e-10, "A_sc X")
    d = innovations(op.q, w.seed, np.sqrt(w.sigma_o2))
    import torch
    b = gp.rhs(torch.from_numpy(d).to("cuda")).cpu().numpy()
    assert_cols_close(b[:, None], O.rhs_sc(op, d)[:, None], 1e-10, "b_sc")
    bt = random_block(w.n, 1, 9)[:, 0]
    b2 = gp.rhs(torch.from_numpy(d).to("cuda"), bt=torch.from_numpy(bt).to("cuda")).cpu().numpy()
    assert_cols_close(b2[:, None], O.rhs_sc(op, d, bt)[:, None], 1e-10, "b_sc + bt")


@pytest.mark.parametrize("method", ["revd", "nystrom", "ritzit"])
def test_strong_lmp_and_pcg(method):
    import torch
    w = C1
    say("strong lmp", method)
    gp, op = _pair(w)
    m = 24
    G = sketch_block(w.n, m, w.seed)
    L = gp.lmp_build(method, m - 4, 4, _t(G))
    _, tho = O.METHODS[method](lambda Z: O.apply_A_sc(op, Z), G, m - 4)
    assert_entries_rel(L.theta(), tho, 1e-10, "Ritz values")
    d = innovations(op.q, w.seed, np.sqrt(w.sigma_o2))
    b = O.rhs_sc(op, d)
    x = torch.zeros(w.n, dtype=torch.float64, device="cuda")
    info = gp.pcg(torch.from_numpy(b).to("cuda"), x, L, tol=1e-8, maxit=500)
    U = L.vectors().cpu().numpy().T
    ro = O.pcg(lambda v: O.apply_A_sc(op, v), b, lmp=(U, L.theta()), tol=1e-8, maxit=500)
    say("  iters gpu", info["iters"], "oracle", ro.iters)
    assert info["status"] == 0 and ro.converged
    assert abs(info["iters"] - ro.iters) <= 2
    xh = x.cpu().numpy()
    assert np.linalg.norm(b - O.apply_A_sc(op, xh)) <= 1.05e-8 * np.linalg.norm(b)


def test_strong_full_size_sampled_columns():
    """n = 4096, N = 100: two columns of A_sc and the right-hand side against the oracle."""
    say("strong full size")
    w = C3
    gp, op = _pair(w)
    X = random_block(w.n, 2, 5)
    Y = gp.apply_A(_t(X)).cpu().numpy().T
    assert_cols_close(Y, O.apply_A_sc(op, X), 1e-10, "A_sc X at n = 4096")


def test_strong_errors():
    import torch
    from paper_2101_07249_amd import Problem
    from paper_2101_07249_amd.wc4d import EINVAL, PREC_SKETCH_BF16X3, Wc4dError
    say("strong errors")
    w = C1
    with pytest.raises(Wc4dError) as e:
        Problem.from_workload(w, obs_pattern(w), strong=True, prec=PREC_SKETCH_BF16X3)
    assert e.value.code == EINVAL
    gp, _ = _pair(w)
    X = torch.zeros((1, w.n), dtype=torch.float64, device="cuda")
    with pytest.raises(Wc4dError) as e:
        gp.apply_Linv(X)
    assert e.value.code == EINVAL
