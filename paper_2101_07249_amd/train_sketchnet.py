"""Train the learned sketch on the GPU and compare it with the Gaussian sketch.

Training data: seeded Lorenz-96 inner-loop problems (initial state, observation
pattern and Gaussian block drawn per instance).  For each instance the method itself
produces the reference: a Nystrom LMP from a wider Gaussian sketch (ref_m columns),
whose leading k Ritz pairs define the capture loss; the network then takes
`steps` Adam steps on that instance (a fresh Gaussian block each step).  Every
operation runs in libwc4d's kernels.

Usage:
  python -m paper_2101_07249_amd.train_sketchnet --instances 2000 --out weights.bin
  python -m paper_2101_07249_amd.train_sketchnet --eval weights.bin --eval-instances 8
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

_ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if _ROOT not in sys.path:
    sys.path.insert(0, _ROOT)

from paper_2101_07249_amd import wc4d as W4  # noqa: E402
from paper_2101_07249_amd.wc4d import Problem, SketchNet  # noqa: E402
from synthetic import C5, l96_initial_state, obs_pattern, sketch_block, sketchnet_init  # noqa: E402

DEFAULT_WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights",
                               "sketchnet_l96_n1024_N100_m64.bin")
EVAL_OFFSET = 1_000_000     # held-out instances start here (training uses 0 .. instances-1)


class Instances:
    """Seeded inner-loop problems of one workload sharing B^{1/2}, Q^{1/2}."""

    def __init__(self, w=C5, device: int = 0):
        self.w = w
        self.device = device
        self.B = W4.corr_sqrt(w.n, w.corr, w.Lb, w.sigma_b)
        self.Q = W4.corr_sqrt(w.n, w.corr, w.Lq, w.sigma_q)

    def problem(self, instance: int) -> Problem:
        w = self.w
        p = Problem(w.n, w.N, self.device)
        x0 = l96_initial_state(w.n, w.seed, instance)
        p.traj = W4.l96_trajectory(x0, w.F, w.dt, w.N)
        p.set_model_l96(p.traj, w.F, w.dt)
        p.set_Bsqrt(self.B)
        p.set_Qsqrt(self.Q)
        for i, idx in obs_pattern(w, instance):
            p.set_obs(i, idx, np.full(len(idx), w.sigma_o2))
        p.finalize()
        return p

    def omega(self, p: Problem, instance: int, m: int, draw: int = 0):
        import torch
        G = sketch_block(p.n_A, m, self.w.seed + 104729 * draw, instance)
        return torch.from_numpy(np.ascontiguousarray(G.T)).to(p.torch_device)


def train(net: SketchNet, inst: Instances, instances: int, steps: int = 2, ref_m: int = 256, k: int = 59,
          lr: float = 1e-3, lr_final: float = 1e-4, log_every: int = 50, start: int = 0):
    """One pass over `instances` problems; cosine decay of the rate from lr to lr_final."""
    hist = []
    t0 = time.perf_counter()
    total = instances * steps
    done = 0
    for a in range(start, start + instances):
        p = inst.problem(a)
        try:
            ref = p.lmp_build("nystrom", ref_m - 5, 5, inst.omega(p, a, ref_m, draw=1))
        except W4.Wc4dError as e:   # no reference for this instance: skip it
            print(json.dumps({"instance": a, "skipped": str(e)}), flush=True)
            p.close()
            continue
        for s in range(steps):
            frac = done / max(total - 1, 1)
            rate = lr_final + 0.5 * (lr - lr_final) * (1.0 + np.cos(np.pi * frac))
            try:
                f = net.train_step(p, inst.omega(p, a, 64, draw=2 + s), ref, k, rate)
            except W4.Wc4dError as e:
                print(json.dumps({"instance": a, "step": s, "skipped": str(e)}), flush=True)
                continue
            finally:
                done += 1
            hist.append(f)
        ref.close()
        p.close()
        if log_every and (a - start + 1) % log_every == 0:
            print(json.dumps({"instance": a + 1, "loss_mean_last": float(np.mean(hist[-log_every * steps:])),
                              "elapsed_s": round(time.perf_counter() - t0, 1)}), flush=True)
    return hist


def ritz_residuals(p: Problem, L) -> np.ndarray:
    """||A u_i - theta_i u_i|| / theta_i for the LMP's Ritz pairs (diagnostic)."""
    import torch
    U = L.vectors()
    th = torch.from_numpy(L.theta()).to(U.device)
    AU = p.apply_A(U)
    return ((AU - th[:, None] * U).norm(dim=1) / th).cpu().numpy()


def evaluate(net, inst: Instances, instances, method: str = "nystrom", tol: float = 1e-6, maxit: int = 5000):
    """Gaussian vs learned sketch on held-out problems: PCG iterations, Ritz residuals and
    time to the 1e-6 true residual (LMP build + PCG)."""
    import torch
    w = inst.w
    rows = []
    for a in instances:
        p = inst.problem(a)
        d = torch.from_numpy(np.random.default_rng([w.seed, a, 9]).standard_normal(p.q) * np.sqrt(w.sigma_o2)).to(
            p.torch_device)
        b = p.rhs(d)
        Om = inst.omega(p, a, 64, draw=0)
        row = {"instance": a}
        for name, use in (("gaussian", None), ("learned", net)):
            x = torch.zeros(p.n_A, dtype=torch.float64, device=p.torch_device)
            for rep in range(2):   # the second repetition is timed
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                L, used = p.lmp_build_sketch(use, method, w.k_r, w.l, Om)
                x.zero_()
                info = p.pcg(b, x, L, tol=tol, maxit=maxit, history=False)
                torch.cuda.synchronize()
                ms = 1e3 * (time.perf_counter() - t0)
                if rep == 0:
                    L.close()
            rr = ritz_residuals(p, L)
            row[name] = {"iters": info["iters"], "relres_true": info["relres_true"], "ms": ms,
                         "used_net": used, "theta_max": float(L.theta()[0]),
                         "ritz_res_median": float(np.median(rr)), "ritz_res_max": float(rr.max())}
            L.close()
        rows.append(row)
        p.close()
    return rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--instances", type=int, default=2000)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--ref-m", type=int, default=256)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--lr-final", type=float, default=1e-4)
    ap.add_argument("--seed", type=int, default=7000)
    ap.add_argument("--init", default=None, help="start from these weights")
    ap.add_argument("--out", default=DEFAULT_WEIGHTS)
    ap.add_argument("--eval", default=None, help="evaluate these weights instead of training")
    ap.add_argument("--eval-instances", type=int, default=4)
    args = ap.parse_args()
    inst = Instances()
    if args.eval:
        net = SketchNet.load(args.eval)
        rows = evaluate(net, inst, range(EVAL_OFFSET, EVAL_OFFSET + args.eval_instances))
        for r in rows:
            print(json.dumps(r), flush=True)
        return
    if args.init:
        net = SketchNet.load(args.init)
    else:
        net = SketchNet()
        net.set_params(sketchnet_init(seed=args.seed))
    hist = train(net, inst, args.instances, steps=args.steps, ref_m=args.ref_m, lr=args.lr, lr_final=args.lr_final)
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    net.save(args.out)
    print(json.dumps({"saved": args.out, "steps": len(hist), "loss_first": float(np.mean(hist[:20])),
                      "loss_last": float(np.mean(hist[-20:]))}), flush=True)


if __name__ == "__main__":
    main()
