"""Gauss-Newton outer loop of incremental weak-constraint 4D-Var on Lorenz-96 (Section 2.1,
eqs. error_update and incr_wc4d-var_forcing) around the library's inner loop, and the
preconditioners Section 5.2 compares in the second inner loop.

Loop j linearises about the state x^(j) that p^(j) = (x_0, eta_1..eta_N) produces through
eq. model, forms d^(j) = y - H x^(j) and D^{-1/2} b^(j), and solves eq. forcing_1stlvl_prec;
then p^(j+1) = p^(j) + D^{1/2} delta p~^(j).  With p^(0) = (x^b, 0, ..., 0), b^(j) =
p^(0) - p^(j), so D^{-1/2} b^(j) = -(delta p~^(0) + ... + delta p~^(j-1)).  All operator,
preconditioner and solver work runs in the library (libwc4d); this module keeps the outer
bookkeeping (the identical-twin data of Section 5, the state vector p, the innovations) on
the host.

Preconditioners of the second inner loop (Section 5.2.1):
  * none;
  * the deterministic LMP from the previous inner loop: the k largest Ritz pairs of A^(0)
    from the Lanczos information its CG gathered (Section 3.4), applied to A^(1);
  * the randomised LMPs (REVD, Nystrom, ritzit; Section 4) built on A^(1) itself.
"""
from __future__ import annotations

from typing import Callable, Dict, List, Optional

import numpy as np

from . import wc4d as W4
from .wc4d import Problem


class OuterLoopL96:
    """An identical-twin Lorenz-96 experiment (Section 5) and its Gauss-Newton outer loop."""

    def __init__(self, w, pattern, draws: Dict[str, np.ndarray], device: int = 0):
        self.w, self.pattern, self.device = w, pattern, device
        self.B = W4.corr_sqrt(w.n, w.corr, w.Lb, w.sigma_b)
        self.Q = W4.corr_sqrt(w.n, w.corr, w.Lq, w.sigma_q)
        # truth with model error Q^{1/2} xi, background x^b = x^t_0 + B^{1/2} xi_b,
        # observations y_i = H_i x^t_i + sigma_o zeta (Section 5)
        eta_t = draws["xi_model"] @ self.Q.T
        self.Xt = W4.l96_trajectory(draws["x0"], w.F, w.dt, w.N, eta=eta_t)
        self.xb = self.Xt[0] + self.B @ draws["xi_b"]
        so = np.sqrt(w.sigma_o2)
        self.y, off = [], 0
        for i, idx in pattern:
            self.y.append(self.Xt[i][idx] + so * draws["zeta"][off:off + len(idx)])
            off += len(idx)
        self.n_A = w.n * (w.N + 1)

    def problem(self, p: np.ndarray, prec: int = W4.PREC_FP64) -> Problem:
        """The inner-loop problem linearised about the state of p (eq. model)."""
        w = self.w
        x0, eta = p[:w.n], p[w.n:].reshape(w.N, w.n)
        prob = Problem(w.n, w.N, self.device)
        prob.traj = W4.l96_trajectory(x0, w.F, w.dt, w.N, eta=eta)
        prob.set_model_l96(prob.traj, w.F, w.dt)
        prob.set_Bsqrt(self.B)
        prob.set_Qsqrt(self.Q)
        for i, idx in self.pattern:
            prob.set_obs(i, idx, np.full(len(idx), w.sigma_o2))
        prob.finalize(prec)
        return prob

    def innovations(self, prob: Problem) -> np.ndarray:
        """d = y - H x^(j), stacked over the observed times (direct observations)."""
        return np.concatenate([self.y[a] - prob.traj[i][idx] for a, (i, idx) in enumerate(self.pattern)])

    def run(self, n_outer: int, inner: Callable[[Problem, object, int], object]) -> List[dict]:
        """n_outer Gauss-Newton iterations; inner(prob, rhs, j) returns delta p~ (a device
        tensor of n_A).  Returns per-loop records with the problem, rhs and delta p~ (host)."""
        import torch
        w = self.w
        p = np.zeros(self.n_A)
        p[:w.n] = self.xb
        bt = np.zeros(self.n_A)          # D^{-1/2} b^(j)
        recs = []
        for j in range(n_outer):
            prob = self.problem(p)
            dev = prob.torch_device
            d = torch.from_numpy(self.innovations(prob)).to(dev)
            rhs = prob.rhs(d, bt=torch.from_numpy(bt.copy()).to(dev))
            dpt = inner(prob, rhs, j)
            dp = prob.apply_Dsqrt(dpt).cpu().numpy()
            dpt_h = dpt.cpu().numpy()
            recs.append({"prob": prob, "rhs": rhs.cpu().numpy(), "dpt": dpt_h})
            p = p + dp
            bt = bt - dpt_h
        recs.append({"p": p})
        return recs


def second_loop_study(exp: OuterLoopL96, ks=(5, 10, 15), l: int = 5, first_maxit: int = 100, tol: float = 1e-6,
                      maxit: int = 1000, methods=("revd", "nystrom", "ritzit"), seed: int = 11,
                      n_j: int = 10, reorth: bool = True, realisations: int = 1,
                      first_tol: Optional[float] = None) -> Dict[str, object]:
    """Section 5.2.1's comparison: the first inner loop runs CG without a second-level
    preconditioner (first_maxit iterations or first_tol, default tol) and gathers its Lanczos
    information; the
    second inner loop is solved without an LMP, with the deterministic LMP of the first
    loop's k largest Ritz pairs, and with each randomised LMP (k pairs, oversampling l)
    built on the second loop's Hessian.  The first loop's CG reorthogonalises its residuals
    (reorth), so that its Ritz pairs are accurate eigenpairs of the first Hessian without
    repeated ('ghost') values (Section 3.4); the paper takes them from an accurate
    eigensolver instead.  Returns iterations and the quadratic cost J at the first n_j
    iterations of the second loop per preconditioner and k; the randomised LMPs are built
    from `realisations` start blocks (seeds seed, seed + 1, ...), reported for the first and
    as means over all."""
    import torch
    store = {}

    def inner(prob, rhs, j):
        x = torch.zeros(prob.n_A, dtype=torch.float64, device=prob.torch_device)
        if j == 0:
            info, al, be, F = prob.pcg_lanczos(rhs, x, tol=tol if first_tol is None else first_tol,
                                               maxit=first_maxit, reorth=reorth)
            store.update(prob0=prob, first=info, alphas=al, betas=be, F=F)
            return x
        store["prob1"], store["rhs1"] = prob, rhs
        return x

    exp.run(2, inner)
    p1, b1 = store["prob1"], store["rhs1"]
    jits = store["first"]["iters"]
    out = {"first_loop_iters": jits, "second": {}}

    def solve(L):
        x = torch.zeros(p1.n_A, dtype=torch.float64, device=p1.torch_device)
        info = p1.pcg(b1, x, L, tol=tol, maxit=maxit)
        return {"iters": info["iters"], "status": info["status"], "relres_true": info["relres_true"],
                "J": [float(v) for v in info["hist_J"][:n_j]]}

    out["second"]["none"] = solve(None)
    for k in ks:
        if k <= jits:
            # Ritz pairs of the first loop's Hessian, preconditioning the second loop's
            U, th = store["prob0"].lanczos_pairs(store["alphas"], store["betas"], store["F"], jits, k)
            Ld = p1.lmp_from_pairs(U, th)
            out["second"][f"previous_loop_k{k}"] = dict(solve(Ld), theta_max=float(th[0]))
            Ld.close()
        for m in methods:
            runs = []
            for r in range(int(realisations)):
                L = p1.lmp_build(m, k, l, seed=seed + r)
                runs.append(dict(solve(L), theta_max=float(L.theta()[0])))
                L.close()
            rec = dict(runs[0])
            rec.update(iters_mean=float(np.mean([q["iters"] for q in runs])),
                       iters_std=float(np.std([q["iters"] for q in runs])),
                       J_mean=np.mean([np.pad(q["J"], (0, n_j - len(q["J"])), mode="edge") for q in runs],
                                      axis=0).tolist(),
                       realisations=int(realisations))
            out["second"][f"{m}_k{k}"] = rec
    return out
