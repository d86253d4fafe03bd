"""One-vector D^{1/2} products on the int8 matrix cores (WC4D_PREC_DSQRT_OZ7: 6-slice
error-free splitting) against the oracle: A x and the right-hand side per column to 1e-10 of
the column's largest entry, the float64 bar (the splitting's truncation leaves a few n 2^-42
relative to max|row of Q^{1/2}| max|level|: ~2e-11 measured in a CPU model of the same
arithmetic at n = 4096), bit-identical repeats, and the full inner loop at n = 4096 reaching the true
residual 1e-6 of the float64 operator with an iteration count within 3% of the float64
solve."""
import numpy as np
import pytest

from oracle import wc4d_oracle as O
from parity import assert_cols_close
from synthetic import C1, C2, C3, SEC52, innovations, l96_initial_state, obs_pattern, random_block

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)


def _pair(w, prec):
    from paper_2101_07249_amd import Problem
    pat = obs_pattern(w)
    x0 = l96_initial_state(w.n, w.seed) if w.model == "l96" else None
    return Problem.from_workload(w, pat, x0=x0, prec=prec), O.make_problem(w, pat, x0=x0)


@pytest.mark.parametrize("w", [C1, C2, SEC52, C3], ids=["C1", "C2", "SEC52", "C3"])
def test_oz_apply_and_rhs(w):
    import torch
    from paper_2101_07249_amd.wc4d import PREC_DSQRT_OZ7
    say("oz apply", w.name)
    gp, op = _pair(w, PREC_DSQRT_OZ7)
    for seed in (3, 4):
        x = random_block(op.n_A, 1, seed)
        y = gp.apply_A(torch.from_numpy(np.ascontiguousarray(x.T)).to("cuda")).cpu().numpy().T
        yo = O.apply_A(op, x)
        # per time level (one column of the level view) and per vector
        assert_cols_close(y.reshape(w.N + 1, w.n).T, yo.reshape(w.N + 1, w.n).T, 1e-10, "A x by level")
        assert_cols_close(y, yo, 1e-10, "A x")
    y2 = gp.apply_A(torch.from_numpy(np.ascontiguousarray(x.T)).to("cuda")).cpu().numpy().T
    assert np.array_equal(y, y2)
    d = innovations(op.q, w.seed, np.sqrt(w.sigma_o2))
    b = gp.rhs(torch.from_numpy(d).to("cuda")).cpu().numpy()
    assert_cols_close(b[:, None], O.rhs(op, d)[:, None], 1e-10, "rhs")


def test_oz_full_inner_loop_c3():
    import torch
    from paper_2101_07249_amd import Problem
    from paper_2101_07249_amd.wc4d import PREC_DSQRT_OZ7, PREC_LMP_FP16, PREC_SKETCH_BF16X3
    say("oz inner loop C3")
    w = C3
    pat = obs_pattern(w)
    op = O.make_problem(w, pat)
    d = innovations(op.q, w.seed, np.sqrt(w.sigma_o2))
    out = {}
    for name, prec in (("mixed", PREC_SKETCH_BF16X3 | PREC_LMP_FP16),
                       ("mixed_oz", PREC_SKETCH_BF16X3 | PREC_LMP_FP16 | PREC_DSQRT_OZ7)):
        gp = Problem.from_workload(w, pat, prec=prec)
        b = gp.rhs(torch.from_numpy(d).to("cuda"))
        L = gp.lmp_build("nystrom", w.m - w.l, w.l, seed=w.seed)
        x = torch.zeros(gp.n_A, dtype=torch.float64, device="cuda")
        info = gp.pcg(b, x, L, tol=1e-6, maxit=3000)
        xh = x.cpu().numpy()
        bo = O.rhs(op, d)
        res = np.linalg.norm(bo - O.apply_A(op, xh)) / np.linalg.norm(bo)
        say("  ", name, "iters", info["iters"], "true residual (oracle)", res)
        assert info["status"] == 0 and res <= 1.05e-6
        out[name] = info["iters"]
        L.close()
        gp.close()
    assert abs(out["mixed_oz"] - out["mixed"]) <= max(2, int(0.03 * out["mixed"]))


def test_oz_rejected_for_strong_constraint():
    from paper_2101_07249_amd import Problem
    from paper_2101_07249_amd.wc4d import EINVAL, PREC_DSQRT_OZ7, Wc4dError
    with pytest.raises(Wc4dError) as e:
        Problem.from_workload(C1, obs_pattern(C1), strong=True, prec=PREC_DSQRT_OZ7)
    assert e.value.code == EINVAL
