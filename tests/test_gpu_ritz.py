"""The Ritz-LMP of eq. Ritz_LMP on the GPU against the oracle: the application with the
GPU's own Ritz pairs written into the oracle's formula (per column 1e-11 of the column's
largest entry), with the oracle's own pairs from the same start block (1e-8: the pairs
agree to their rounding), P A U = U for REVD's Rayleigh-Ritz pairs, and preconditioned CG with it against the oracle's
standard PCG (iterations within max(2, 3%), the first costs per entry to 1e-9)."""
import ctypes

import numpy as np
import pytest

from oracle import wc4d_oracle as O
from parity import assert_cols_close, assert_entries_rel
from synthetic import C1, C2, innovations, l96_initial_state, obs_pattern, random_block, sketch_block

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)


def _setup(w):
    import torch
    from paper_2101_07249_amd import Problem
    pat = obs_pattern(w)
    x0 = l96_initial_state(w.n, w.seed) if w.model == "l96" else None
    gp = Problem.from_workload(w, pat, x0=x0)
    op = O.make_problem(w, pat, x0=x0)
    G = sketch_block(w.n_A, w.m, w.seed)
    L = gp.lmp_build("nystrom", w.k_r, w.l, torch.from_numpy(np.ascontiguousarray(G.T)).to("cuda"))
    return gp, op, G, L


@pytest.mark.parametrize("w", [C1, C2], ids=["C1", "C2"])
def test_ritz_apply_against_oracle(w):
    import torch
    say("ritz apply", w.name)
    gp, op, G, L = _setup(w)
    X = random_block(op.n_A, 2, 17)
    Xt = torch.from_numpy(np.ascontiguousarray(X.T)).to("cuda")
    from paper_2101_07249_amd.wc4d import ESTATE, Wc4dError
    with pytest.raises(Wc4dError) as e:
        L.ritz_apply(Xt)
    assert e.value.code == ESTATE
    L.ritz_prepare()
    Y = L.ritz_apply(Xt).cpu().numpy().T
    U = L.vectors().cpu().numpy().T
    th = L.theta()
    AU = O.apply_A(op, U)
    Yo = np.stack([O.ritz_lmp_apply(U, th, AU, X[:, c]) for c in range(2)], axis=1)
    assert_cols_close(Y, Yo, 1e-11, "P X with the GPU's pairs")
    Uo, tho = O.nystrom(lambda Z: O.apply_A(op, Z), G, w.k_r)
    AUo = O.apply_A(op, Uo)
    Yo2 = np.stack([O.ritz_lmp_apply(Uo, tho, AUo, X[:, c]) for c in range(2)], axis=1)
    assert_cols_close(Y, Yo2, 1e-8, "P X with the oracle's pairs")
    # P A U = U for Rayleigh-Ritz pairs (U^T A U = Theta: REVD's; Nystrom's pairs are not
    # Rayleigh-Ritz pairs of A), eq. Ritz_LMP's defining property
    Lr = gp.lmp_build("revd", w.k_r, w.l, torch.from_numpy(np.ascontiguousarray(G.T)).to("cuda"))
    Lr.ritz_prepare()
    Ur = Lr.vectors().cpu().numpy().T
    AUr = O.apply_A(op, Ur[:, :4])
    PAU = Lr.ritz_apply(torch.from_numpy(np.ascontiguousarray(AUr.T)).to("cuda")).cpu().numpy().T
    assert_cols_close(PAU, Ur[:, :4], 1e-8, "P A U = U")


@pytest.mark.parametrize("w", [C1, C2], ids=["C1", "C2"])
def test_pcg_ritz_against_oracle(w):
    import torch
    say("pcg ritz", w.name)
    gp, op, G, L = _setup(w)
    d = innovations(op.q, w.seed, np.sqrt(w.sigma_o2))
    b = O.rhs(op, d)
    bt = gp.rhs(torch.from_numpy(d).to("cuda"))
    x = torch.zeros(op.n_A, dtype=torch.float64, device="cuda")
    from paper_2101_07249_amd.wc4d import ESTATE, Wc4dError
    with pytest.raises(Wc4dError) as e:
        gp.pcg_ritz(bt, x, L)
    assert e.value.code == ESTATE
    L.ritz_prepare()
    info = gp.pcg_ritz(bt, x, L, tol=1e-6, maxit=1000)
    U = L.vectors().cpu().numpy().T
    th = L.theta()
    AU = O.apply_A(op, U)
    ro = O.pcg_standard(lambda v: O.apply_A(op, v), b, lambda r: O.ritz_lmp_apply(U, th, AU, r), tol=1e-6,
                        maxit=1000)
    say("  iters gpu", info["iters"], "oracle", ro.iters)
    assert info["status"] == 0 and ro.converged
    assert abs(info["iters"] - ro.iters) <= max(2, int(0.03 * ro.iters))
    assert_entries_rel(info["hist_J"][:5], np.array(ro.hist_J[:5]), 1e-9, "cost")
    xh = x.cpu().numpy()
    res = np.linalg.norm(b - O.apply_A(op, xh)) / np.linalg.norm(b)
    assert res <= 1.05e-6, res
    # against the spectral LMP's split PCG on the same pairs: both converge; the Ritz-LMP
    # takes no more iterations (up to rounding) since it corrects the pairs' inexactness
    x2 = torch.zeros(op.n_A, dtype=torch.float64, device="cuda")
    i2 = gp.pcg(bt, x2, L, tol=1e-6, maxit=1000)
    say("  spectral LMP iters", i2["iters"])
    assert i2["status"] == 0
