"""Benchmark: time to a 1e-6 residual of one randomised-LMP preconditioned inner loop.

One step = the whole hot path on one synthetic problem already resident in HBM:
right-hand side (D^{1/2} L^{-T} H^T R^{-1} d), LMP build from a Gaussian sketch
(two block Hessian applies, CholeskyQR2, the small eigenproblem, Ritz vectors) and
split PCG on the exact Hessian until ||b - A x|| <= 1e-6 ||b||.

Default workload: periodic advection-diffusion n = 4096, N = 100 (n_A = 413,696),
SOAR B / Q, every 4th point observed at every 2nd step (q = 51,200), a sketch of
m = 256 columns (k_r = 251 Ritz pairs, oversampling 5), Nystrom.

Variants (each timed over the same number of steps):
  plain         float64 throughout;
  mixed         the sketch's D^{1/2} products as three bfloat16 MFMA products with float32
                accumulation, a float16 copy of U (power-of-two column scaling) for the
                PCG's LMP passes, and the PCG's one-vector D^{1/2} products on the int8
                matrix cores by a 6-slice error-free splitting (about 2e-11 of float64);
                CholeskyQR2, the small eigenproblem, the sweeps and all PCG vectors stay
                float64, and the stop is the true residual;
  mixed_f64pcg  the same with float64 one-vector D^{1/2} products;
  mixed_u32     mixed_f64pcg with a float32 copy of U;
  mixed_fp16    split-float16 instead of split-bfloat16 sketch products, float16 U.
`value` is the mixed variant's ms per step; the others are reported beside it.

Prints one JSON line (see the fields below).  Only --gpus 1 is supported.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0      # MI355X HBM3E
FP64_PEAK_TFLOPS = 78.6    # MI355X dense FP64 (matrix and vector)
BF16_PEAK_TFLOPS = 2500.0  # MI355X dense BF16 MFMA
INT8_PEAK_TOPS = 5000.0    # MI355X dense INT8 MFMA
OZ_PAIRS = 21              # int8 slice products per one-vector D^{1/2} product (6 slices, t + u <= 7)

# HBM bytes per launch group of the single-vector float64 D^{1/2} product at n = 4096,
# N = 100, measured with rocprofv3 FETCH_SIZE / WRITE_SIZE (each scaled by a 1 GiB copy's
# reading; profiles/dsqrt_vec_n4096_N100_counters.md), per tuned tile code of the one
# product with Q^{1/2} over all levels.  Valid only for the kernels that were measured:
# those tile codes, built from this gemm_f64.hip (product and split-K reduction).
MEASURED_TRAFFIC = {"n": 4096, "N": 100,
                    "tune": {"single_product": True, "two_segment": False},
                    "sources": {"paper_2101_07249_amd/csrc/gemm_f64.hip":
                                "7d77e6e0c0c0a03f8aa5b42f710c13d72289138b95b47149a76721ecbe82e54d"},
                    "bytes_per_launch": {2: 216.7e6, 7: 216.6e6}}

# HBM bytes per launch group of the int8-sliced one-vector D^{1/2} product at n = 4096, N = 100
# (k_oz_split_cols + k_oz_gemm<16> + k_oz_reduce), measured the same way
# (profiles/dsqrt_oz_n4096_N100_kernel_stats.md); valid only for this gemm_oz.hip.
OZ_MEASURED_TRAFFIC = {"n": 4096, "N": 100,
                       "sources": {"paper_2101_07249_amd/csrc/gemm_oz.hip":
                                   "ad5282a403afa4148e09e066f2d7b9e83a81c841a2e5a15945bd652b596de7b0"},
                       "bytes_per_launch": 163.2e6}

# Measured tile choices for MI355X (loaded unless --tune-cache or --retune is given).
TUNING_TABLE = os.path.join(ROOT, "paper_2101_07249_amd", "tuning", "mi355x.txt")


def dominant_class(prof):
    """The kernel class (other than the build's remaining kernels) with the most time."""
    classes = {k: v for k, v in prof.items() if v["launches"] > 0 and k != "build_other"}
    return max(classes, key=lambda k: classes[k]["ms"])


def measured_traffic(w, tune):
    """The counted bytes when this run uses the measured kernels, else None."""
    import hashlib
    t = MEASURED_TRAFFIC
    if tune is None or (w.n, w.N) != (t["n"], t["N"]):
        return None
    if any(tune.get(k) != v for k, v in t["tune"].items()):
        return None
    for path, digest in t["sources"].items():
        with open(os.path.join(ROOT, path), "rb") as f:
            if hashlib.sha256(f.read()).hexdigest() != digest:
                return None
    return t["bytes_per_launch"].get(tune.get("tile_b"))


def oz_measured_traffic(w):
    """The counted bytes of the int8-sliced product group when this run uses the measured
    gemm_oz.hip, else None."""
    import hashlib
    t = OZ_MEASURED_TRAFFIC
    if (w.n, w.N) != (t["n"], t["N"]):
        return None
    for path, digest in t["sources"].items():
        with open(os.path.join(ROOT, path), "rb") as f:
            if hashlib.sha256(f.read()).hexdigest() != digest:
                return None
    return t["bytes_per_launch"]


def dsqrt_kernel_name(tune):
    """The kernels of one single-vector D^{1/2} launch group for this run's tuned form."""
    if tune is None:
        return "float64 D^{1/2} products (PCG, one vector)"
    rows_k = {0: (64, 32), 1: (128, 16), 2: (128, 32)}
    if tune.get("two_segment"):
        r, kk = rows_k.get(tune.get("segment_variant"), (0, 0))
        core = f"k_dsqrt2<{r}, {kk}> ({tune.get('segment_splits') or 'auto'} splits) + k_dsqrt2_reduce"
    else:
        names = {2: "k_gemm_f64<64, 112, 32, 4, 1, true> + k_gemm_splitk_reduce",
                 7: "k_gemm_f64_pa<112, 32> + k_gemm_splitk_reduce"}
        core = (names.get(tune.get("tile_b"), f"k_gemm_f64 tile code {tune.get('tile_b')}")
                + ("" if tune.get("single_product") else f" / tile code {tune.get('tile_q')}"))
    if tune.get("single_product"):
        return f"Q^(1/2) over all N+1 levels, level 0 scaled in the epilogue: {core}"
    return f"B^(1/2), Q^(1/2): {core}"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="C3", choices=["C1", "C2", "C3"])
    ap.add_argument("--method", default="nystrom", choices=["revd", "nystrom", "ritzit", "nystrom1p"])
    ap.add_argument("--variants", default="plain,mixed,mixed_f64pcg,mixed_u32,mixed_fp16",
                    help="comma list of plain (FP64), mixed (split-bf16 block products, float16 U, "
                         "int8-sliced PCG products), mixed_f64pcg (float64 PCG products), mixed_u32 "
                         "(float32 U), mixed_fp16 (split-float16 products, float16 U)")
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--maxit", type=int, default=5000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-sketch comparison")
    ap.add_argument("--learned-problems", type=int, default=8, help="held-out problems of the learned comparison")
    ap.add_argument("--no-oversampling", action="store_true", help="skip the realisation / oversampling statistics")
    ap.add_argument("--realisations", type=int, default=50)
    ap.add_argument("--no-second-loop", action="store_true",
                    help="skip the Gauss-Newton second-loop comparison (Section 5.2)")
    ap.add_argument("--second-loop-realisations", type=int, default=5)
    ap.add_argument("--no-strong", action="store_true", help="skip the strong-constraint inner loop")
    ap.add_argument("--no-ritz", action="store_true", help="skip the Ritz-LMP cost study")
    ap.add_argument("--no-batched", action="store_true", help="skip the 64-problem batched solve")
    ap.add_argument("--batched-count", type=int, default=64)
    ap.add_argument("--batched-f32", action="store_true",
                    help="also run the persistent batch with float32 sweeps (another ~60 s)")
    ap.add_argument("--batched-compare", action="store_true",
                    help="also time the host-worker batched solve on the same problems")
    ap.add_argument("--retune", action="store_true",
                    help="autotune every product shape instead of loading the MI355X tuning table")
    ap.add_argument("--tune-cache", default=None,
                    help="autotune cache file: loaded when present, written after tuning")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain 1 GiB device copy 5 times (reference for HBM counters)")
    ap.add_argument("--prof-every", type=int, default=8,
                    help="time one launch group in this many of the dominant class in the timed steps")
    return ap.parse_args()


def copy_probe():
    """A plain device-to-device copy of 2^27 doubles (1 GiB read + 1 GiB written), five
    times: the reference that scales FETCH_SIZE / WRITE_SIZE counter readings to bytes."""
    import torch
    x = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    for _ in range(5):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_read": x.numel() * 8, "copy_probe_bytes_written": y.numel() * 8,
                      "launches": 5}), flush=True)


def learned_section(args):
    """Gaussian vs learned start block on held-out Lorenz-96 problems (n = 1024, N = 100,
    m = 64, Nystrom): per problem, ms from the LMP build (net inference included) to the
    1e-6 true residual, PCG iterations, and the Ritz residuals ||A u - theta u|| / theta of
    the leading pairs; then the means over the problems."""
    import numpy as np
    import torch

    from paper_2101_07249_amd.train_sketchnet import DEFAULT_WEIGHTS, EVAL_OFFSET, Instances, ritz_residuals
    from paper_2101_07249_amd.wc4d import SketchNet

    if not os.path.exists(DEFAULT_WEIGHTS):
        return {"error": f"no trained weights at {os.path.relpath(DEFAULT_WEIGHTS, ROOT)}"}
    net = SketchNet.load(DEFAULT_WEIGHTS)
    inst = Instances()
    w = inst.w
    rows = []
    for a in range(EVAL_OFFSET, EVAL_OFFSET + args.learned_problems):
        p = inst.problem(a)
        d = torch.from_numpy(np.random.default_rng([w.seed, a, 9]).standard_normal(p.q) * np.sqrt(w.sigma_o2)).to(
            p.torch_device)
        b = p.rhs(d)
        Om = inst.omega(p, a, 64, draw=0)
        row = {"instance": a}
        x = torch.zeros(p.n_A, dtype=torch.float64, device=p.torch_device)
        for name, use in (("gaussian", None), ("learned", net)):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            L, used = p.lmp_build_sketch(use, "nystrom", w.k_r, w.l, Om)
            x.zero_()
            info = p.pcg(b, x, L, tol=args.tol, maxit=args.maxit, history=False)
            torch.cuda.synchronize()
            ms = 1e3 * (time.perf_counter() - t0)
            rr = ritz_residuals(p, L)
            row[name] = {"ms": ms, "pcg_iters": info["iters"], "relres_true": info["relres_true"],
                         "used_net": bool(used), "ritz_res_leading10_median": float(np.median(rr[:10])),
                         "ritz_res_median": float(np.median(rr))}
            L.close()
        rows.append(row)
        print(f"learned: problem {a}: iterations {row['gaussian']['pcg_iters']} (gaussian) / "
              f"{row['learned']['pcg_iters']} (learned)", file=sys.stderr, flush=True)
        p.close()
    it_ratio = [r["learned"]["pcg_iters"] / r["gaussian"]["pcg_iters"] for r in rows]
    ms_ratio = [r["learned"]["ms"] / r["gaussian"]["ms"] for r in rows]
    return {"workload": w.name, "method": "nystrom", "problems": len(rows),
            "instances": [r["instance"] for r in rows], "per_problem": rows,
            "mean_iters_ratio_learned_over_gaussian": float(np.mean(it_ratio)),
            "mean_time_ratio_learned_over_gaussian": float(np.mean(ms_ratio)),
            "speedup_vs_gaussian": float(np.sum([r["gaussian"]["ms"] for r in rows]) /
                                         np.sum([r["learned"]["ms"] for r in rows])),
            "ritz_res_leading10_median": {k: float(np.median([r[k]["ritz_res_leading10_median"] for r in rows]))
                                          for k in ("gaussian", "learned")}}


def batched_section(args):
    """64 uneven advection-diffusion inner loops (n in [512, 8192], N in [10, 200], m = 64,
    Nystrom): every problem's LMP built from its seeded device Gaussian block, then all PCG
    iterations of all problems in one persistent launch (wc4d_batch_solve_persistent),
    with float64 sweeps (and with float32 sweeps under --batched-f32); then the host-worker form (wc4d_batch_solve,
    4 workers) with the PCG's one-vector D^{1/2} products on the int8 matrix cores; wall time
    of the whole call (builds included), the persistent launch's own time, iterations and
    true residuals with the float64 operator.  With --batched-compare also the host-worker
    form in float64."""
    import numpy as np
    import torch

    from paper_2101_07249_amd import Problem, batch_solve, batch_solve_persistent, gaussian_block
    from synthetic import batched_workloads, innovations, obs_pattern

    ws = batched_workloads(count=args.batched_count)
    probs, b = [], []
    for w in ws:
        p = Problem.from_workload(w, obs_pattern(w))
        probs.append(p)
        b.append(p.rhs(torch.from_numpy(innovations(p.q, w.seed, np.sqrt(w.sigma_o2))).to(p.torch_device)))
    k_r, l = ws[0].k_r, ws[0].l
    out = {"problems": len(ws), "sum_n_A": int(sum(p.n_A for p in probs)), "m": k_r + l, "method": "nystrom",
           "n_range": [min(w.n for w in ws), max(w.n for w in ws)], "N_range": [min(w.N for w in ws), max(w.N for w in ws)]}
    runs = [("persistent_f64", False)] + ([("persistent_f32_sweeps", True)] if args.batched_f32 else [])
    for name, f32 in runs:
        x = [torch.zeros(p.n_A, dtype=torch.float64, device=p.torch_device) for p in probs]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        infos, status, kms = batch_solve_persistent(probs, "nystrom", k_r, l, b, x, seed=4000, tol=args.tol,
                                                    maxit=args.maxit, sweep_fp32=f32)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        # achieved true residual of every problem with the float64 operator
        res = []
        for i, p in enumerate(probs):
            r = b[i] - p.apply_A(x[i])
            res.append(float(r.norm() / b[i].norm()))
        from paper_2101_07249_amd.wc4d import batch_persistent_profile
        prof = batch_persistent_profile()
        out[name] = {"s": t, "persistent_launch_s": kms * 1e-3, "iters_total": int(sum(i["iters"] for i in infos)),
                     "phase_busy_s": {k: round(v["busy_ms"] * 1e-3, 3) for k, v in prof.items() if k != "launch"},
                     "workgroups": prof["launch"]["workgroups"],
                     "iters_max": int(max(i["iters"] for i in infos)),
                     "converged_recursive": all(s == 0 for s in status),
                     "true_residual_max": max(res), "true_residual_median": float(np.median(res))}
        print(f"batched: {name} {t:.1f} s (persistent launch {kms * 1e-3:.1f} s)", file=sys.stderr, flush=True)
    # host workers (a stream each, the single-problem kernels) with the PCG's one-vector D^{1/2}
    # products on the int8 matrix cores; true residuals with the float64 operator
    from paper_2101_07249_amd import wc4d as W4
    probs_i8 = [Problem.from_workload(w, obs_pattern(w), prec=W4.PREC_DSQRT_OZ7) for w in ws]
    G = [gaussian_block(4000 + i, p.n_A, k_r + l) for i, p in enumerate(probs_i8)]
    x = [torch.zeros(p.n_A, dtype=torch.float64, device=p.torch_device) for p in probs_i8]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos, status = batch_solve(probs_i8, "nystrom", k_r, l, G, b, x, tol=args.tol, maxit=args.maxit, workers=4,
                                autotune=False)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    res = [float((b[i] - p.apply_A(x[i])).norm() / b[i].norm()) for i, p in enumerate(probs)]
    out["host_workers_i8"] = {"s": t, "iters_total": int(sum(i["iters"] for i in infos)),
                              "converged_recursive": all(s_ == 0 for s_ in status),
                              "true_residual_max": max(res), "true_residual_median": float(np.median(res)),
                              "workers": 4}
    print(f"batched: host workers, int8 D^(1/2) {t:.1f} s", file=sys.stderr, flush=True)
    for p in probs_i8:
        p.close()
    del G, x
    if args.batched_compare:
        G = [gaussian_block(4000 + i, p.n_A, k_r + l) for i, p in enumerate(probs)]
        x = [torch.zeros(p.n_A, dtype=torch.float64, device=p.torch_device) for p in probs]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        infos, status = batch_solve(probs, "nystrom", k_r, l, G, b, x, tol=args.tol, maxit=args.maxit, workers=4,
                                    autotune=False)
        torch.cuda.synchronize()
        out["host_workers"] = {"s": time.perf_counter() - t0, "iters_total": int(sum(i["iters"] for i in infos)),
                               "converged": all(s == 0 for s in status)}
    return out


def oversampling_section(args):
    """Realisation and oversampling statistics (Section 5.2.3) on Section 5.2's Lorenz-96
    configuration (n = 80, N = 150, 120 observations, k = 15): for each randomised method and
    oversampling l in {5, 10, 15}, args.realisations start blocks drawn on the device from
    seeds; the mean and standard deviation over the realisations of the quadratic cost J at
    each of the first ten PCG iterations, and of the iterations to a 1e-6 true residual."""
    import numpy as np
    import torch

    from paper_2101_07249_amd import Problem
    from synthetic import SEC52, innovations, l96_initial_state, obs_pattern

    w = SEC52
    pat = obs_pattern(w)
    p = Problem.from_workload(w, pat, x0=l96_initial_state(w.n, w.seed))
    b = p.rhs(torch.from_numpy(innovations(p.q, w.seed, np.sqrt(w.sigma_o2))).to(p.torch_device))
    x = torch.zeros(p.n_A, dtype=torch.float64, device=p.torch_device)
    k, nj = 15, 10
    out = {"workload": w.name, "n_A": p.n_A, "q": p.q, "k": k, "realisations": args.realisations, "rows": []}
    info0 = p.pcg(b, x, None, tol=args.tol, maxit=args.maxit)
    out["no_lmp"] = {"iters": info0["iters"], "J": [float(v) for v in info0["hist_J"][:nj]]}
    t0 = time.perf_counter()
    for method in ("revd", "nystrom", "ritzit", "nystrom1p"):
        for l in (5, 10, 15):
            Js, its = [], []
            for r in range(args.realisations):
                L = p.lmp_build(method, k, l, seed=1000 * l + r)
                x.zero_()
                info = p.pcg(b, x, L, tol=args.tol, maxit=args.maxit)
                L.close()
                Js.append(np.pad(info["hist_J"][:nj], (0, max(0, nj - info["iters"])), mode="edge"))
                its.append(info["iters"])
            Js = np.array(Js)
            out["rows"].append({"method": method, "l": l, "J_mean": Js.mean(axis=0).tolist(),
                                "J_std": Js.std(axis=0).tolist(), "iters_mean": float(np.mean(its)),
                                "iters_std": float(np.std(its)), "iters_min": int(min(its)), "iters_max": int(max(its))})
        print(f"oversampling: {method} done", file=sys.stderr, flush=True)
    out["s"] = time.perf_counter() - t0
    p.close()
    return out


def second_loop_section(args):
    """Section 5.2's headline comparison on its Lorenz-96 configuration, per observation
    network (120, 480 and 3000 observations: every 10th, 5th and 2nd variable at every 10th,
    5th and 2nd step): an identical-twin experiment, a first inner loop of CG (100 iterations
    or 1e-6) with reorthogonalised Lanczos information, then the second loop's PCG without an
    LMP, with the previous loop's k Ritz pairs (the deterministic LMP) and with the randomised
    LMPs built on the second loop's Hessian (l = 5; means over the realisations)."""
    import numpy as np

    from paper_2101_07249_amd.outer_loop import OuterLoopL96, second_loop_study
    from synthetic import SEC52, obs_count, obs_pattern, twin_draws

    out = {"workload": SEC52.name, "realisations": args.second_loop_realisations, "networks": []}
    t0 = time.perf_counter()
    for stride, ks in ((10, (5, 10, 15)), (5, (5, 15)), (2, (5, 15))):
        w = SEC52.with_(obs_var_stride=stride, obs_time_stride=stride)
        pat = obs_pattern(w)
        draws = twin_draws(w, obs_count(pat))
        exp = OuterLoopL96(w, pat, draws)
        res = second_loop_study(exp, ks=ks, l=5, tol=args.tol, maxit=args.maxit,
                                realisations=args.second_loop_realisations, seed=7000)
        rows = {}
        for name, r in res["second"].items():
            rows[name] = {"iters": r.get("iters_mean", r["iters"]), "iters_std": r.get("iters_std", 0.0),
                          "J": [float(v) for v in r.get("J_mean", r["J"])], "theta_max": r.get("theta_max")}
        out["networks"].append({"obs": obs_count(pat), "stride": stride, "first_loop_iters": res["first_loop_iters"],
                                "second_loop": rows})
        print(f"second loop: {obs_count(pat)} observations done", file=sys.stderr, flush=True)
    out["s"] = time.perf_counter() - t0
    return out


def strong_section(args):
    """The strong-constraint counterpart at the benchmark's sizes (n = 4096, N = 100: the
    control is x_0 alone, the operator I + B^{1/2} (sum_i M_{0->i}^T H_i^T R_i^{-1} H_i
    M_{0->i}) B^{1/2}): rhs, Nystrom LMP from a device-drawn block, PCG to the tolerance,
    against PCG without an LMP."""
    import numpy as np
    import torch

    from paper_2101_07249_amd import Problem
    from synthetic import C3, innovations, obs_pattern

    w = C3
    p = Problem.from_workload(w, obs_pattern(w), strong=True)
    d = torch.from_numpy(innovations(p.q, w.seed, np.sqrt(w.sigma_o2))).to(p.torch_device)
    out = {"workload": "strong_" + w.name, "n_A": p.n_A, "q": p.q}
    x = torch.zeros(p.n_A, dtype=torch.float64, device=p.torch_device)
    for label, k_r in (("none", 0), ("nystrom", w.m - w.l)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b = p.rhs(d)
        L = p.lmp_build("nystrom", k_r, w.l, seed=w.seed) if k_r else None
        x.zero_()
        info = p.pcg(b, x, L, tol=args.tol, maxit=args.maxit)
        torch.cuda.synchronize()
        out[label] = {"ms": 1e3 * (time.perf_counter() - t0), "pcg_iters": info["iters"],
                      "relres_true": info["relres_true"], "converged": info["status"] == 0}
        if L is not None:
            out[label]["theta_max"] = float(L.theta()[0])
            L.close()
    p.close()
    return out


def ritz_section(args):
    """The Ritz-LMP of eq. Ritz_LMP against the spectral LMP on the benchmark's workload
    (float64): one Nystrom LMP (k_r = 251); PCG with the spectral LMP (split, fused: two
    passes over U per iteration) and with the Ritz-LMP (one extra block product for A U, then
    four passes over U and A U per iteration); iterations and time of each solve."""
    import numpy as np
    import torch

    from paper_2101_07249_amd import Problem
    from synthetic import C3, innovations, obs_pattern

    w = C3
    p = Problem.from_workload(w, obs_pattern(w))
    b = p.rhs(torch.from_numpy(innovations(p.q, w.seed, np.sqrt(w.sigma_o2))).to(p.torch_device))
    L = p.lmp_build("nystrom", w.m - w.l, w.l, seed=w.seed)
    x = torch.zeros(p.n_A, dtype=torch.float64, device=p.torch_device)
    out = {"workload": w.name, "k_r": w.m - w.l}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    info = p.pcg(b, x, L, tol=args.tol, maxit=args.maxit)
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0)
    out["spectral"] = {"ms": ms, "pcg_iters": info["iters"], "ms_per_iter": ms / max(info["iters"], 1),
                       "relres_true": info["relres_true"]}
    t0 = time.perf_counter()
    L.ritz_prepare()
    torch.cuda.synchronize()
    prep = 1e3 * (time.perf_counter() - t0)
    x.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    info = p.pcg_ritz(b, x, L, tol=args.tol, maxit=args.maxit)
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0)
    out["ritz"] = {"prepare_ms": prep, "ms": ms, "pcg_iters": info["iters"], "ms_per_iter": ms / max(info["iters"], 1),
                   "relres_true": info["relres_true"]}
    L.close()
    p.close()
    return out


def cpu_baseline(w, pat, gpu_iters, args):
    """The oracle's whole inner loop on the same workload, measured (not extrapolated):
    the right-hand side, the randomised build from the same seeded Gaussian block (the
    oracle draws it with its own Philox-4x32-10 + Box-Muller) and PCG with the LMP until
    the true relative residual reaches the tolerance."""
    import numpy as np

    from oracle import philox as PX
    from oracle import wc4d_oracle as O
    from synthetic import innovations

    try:
        from threadpoolctl import threadpool_info
        cores = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
    except Exception:  # pragma: no cover
        cores = os.cpu_count() or 1
    op = O.make_problem(w, pat)
    d = innovations(op.q, w.seed, np.sqrt(w.sigma_o2))
    print(f"cpu_baseline: oracle inner loop on {w.name} ({cores} threads): build", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    b = O.rhs(op, d)
    G = PX.gaussian_block(w.seed, op.n_A, w.m)
    t1 = time.perf_counter()
    U, theta = O.METHODS[args.method](lambda X: O.apply_A(op, X), G, w.k_r)
    t2 = time.perf_counter()
    print(f"cpu_baseline: build {t2 - t1:.1f} s; PCG", file=sys.stderr, flush=True)
    res = O.pcg(lambda v: O.apply_A(op, v), b, lmp=(U, theta), tol=args.tol, maxit=args.maxit)
    t3 = time.perf_counter()
    print(f"cpu_baseline: PCG {t3 - t2:.1f} s, {res.iters} iterations", file=sys.stderr, flush=True)
    return {"value": 1e3 * (t3 - t0), "unit": "ms per step", "cores": int(cores), "kind": "oracle",
            "scope": "measured in full: one whole inner loop, not extrapolated",
            "sample": (f"one inner loop of {w.name} (the benchmark's workload and seed): rhs + Gaussian block "
                       f"{1e3 * (t1 - t0):.0f} ms, {args.method} build with m = {w.m} "
                       f"{1e3 * (t2 - t1):.0f} ms, PCG to a true relative residual of {args.tol:g} "
                       f"{1e3 * (t3 - t2):.0f} ms ({res.iters} iterations, {1e3 * (t3 - t2) / max(res.iters, 1):.0f} "
                       f"ms/iteration)"),
            "oracle_pcg_iters": int(res.iters), "oracle_relres_true": float(res.relres_true),
            "oracle_converged": bool(res.converged), "gpu_pcg_iters_fp64": gpu_iters}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark measures one GPU only; --gpus must be 1"}))
        sys.exit(2)
    if args.copy_probe:
        copy_probe()
        return
    import numpy as np
    import torch

    from paper_2101_07249_amd import Problem
    from synthetic import WORKLOADS, innovations, obs_pattern

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(1)
    from paper_2101_07249_amd import wc4d as W4

    t_start = time.perf_counter()
    dev = torch.device("cuda", 0)
    w = WORKLOADS[args.workload]
    pat = obs_pattern(w)
    G = W4.gaussian_block(w.seed, w.n_A, w.m)   # the start block the seeded builds draw
    dnp = innovations(sum(len(i) for _, i in pat), w.seed, np.sqrt(w.sigma_o2))
    d = torch.from_numpy(dnp).to(dev)
    x = torch.zeros(w.n_A, dtype=torch.float64, device=dev)
    precs = {"plain": W4.PREC_FP64,
             "mixed": W4.PREC_SKETCH_BF16X3 | W4.PREC_LMP_FP16 | W4.PREC_DSQRT_OZ7,
             "mixed_f64pcg": W4.PREC_SKETCH_BF16X3 | W4.PREC_LMP_FP16,
             "mixed_u32": W4.PREC_SKETCH_BF16X3 | W4.PREC_LMP_FP32,
             "mixed_fp16": W4.PREC_SKETCH_FP16X3 | W4.PREC_LMP_FP16}
    names = [v for v in args.variants.split(",") if v]
    results = {}
    tunes = {}
    tile_source = "autotuned at set-up"
    if args.tune_cache and os.path.exists(args.tune_cache):
        W4.autotune_load(args.tune_cache)
        tile_source = "tune cache " + os.path.basename(args.tune_cache) + " (autotuned where absent)"
    elif not args.tune_cache and not args.retune and os.path.exists(TUNING_TABLE):
        W4.autotune_load(TUNING_TABLE)
        tile_source = "MI355X tuning table paper_2101_07249_amd/tuning/mi355x.txt (autotuned where absent)"
    for vname in names:
        prob = Problem.from_workload(w, pat, prec=precs[vname])
        # one-time setup, outside the timed region: tile shapes of the D^{1/2} products for
        # the single-vector PCG applies and the m-column block applies
        tunes[vname] = {"m1": prob.autotune(1), f"m{w.m}": prob.autotune(w.m)}
        if args.tune_cache:
            W4.autotune_save(args.tune_cache)

        def step():
            b = prob.rhs(d)
            # the Gaussian start block is drawn on the device inside the build (seeded)
            L = prob.lmp_build(args.method, w.k_r, w.l, seed=w.seed)
            x.zero_()
            info = prob.pcg(b, x, L, tol=args.tol, maxit=args.maxit, history=False)
            info["lmp_copy"] = L.copy_format()
            L.close()
            return info

        # every kernel class is timed (HIP events around each launch group) in the last
        # warm-up step; the timed steps record events around the dominant class only, so
        # the per-class markers do not sit in the measured stream
        prof_all = None
        for wi in range(args.warmup):
            if wi == args.warmup - 1:
                prob.prof_enable(True)
            step()
        if args.warmup > 0:
            prof_all = prob.prof_read()
            dom_cls = dominant_class(prof_all)
        torch.cuda.synchronize()
        prob.prof_enable(True, classes=None if prof_all is None else [dom_cls])
        prob.prof_stride(args.prof_every)
        infos = []
        t0 = time.perf_counter()
        for _ in range(args.steps):
            infos.append(step())
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        prof = prob.prof_read()
        prob.prof_enable(False)
        prob.prof_stride(1)
        results[vname] = {"ms_per_step": 1e3 * (t1 - t0) / args.steps,
                          "pcg_iters": int(np.median([i["iters"] for i in infos])),
                          "relres_true": max(i["relres_true"] for i in infos),
                          "converged": all(i["status"] == 0 and i["relres_true"] <= args.tol for i in infos),
                          "lmp_copy": {0: "f64", W4.PREC_LMP_FP32: "f32", W4.PREC_LMP_FP16: "f16"}[infos[-1]["lmp_copy"]],
                          "prof": prof, "prof_classes": prof_all if prof_all is not None else prof,
                          "classes_steps": 1 if prof_all is not None else args.steps, "prob": prob}
    head = "mixed" if "mixed" in results else names[0]
    prob = results[head]["prob"]
    prof = results[head]["prof"]
    ms_per_step = results[head]["ms_per_step"]
    ok = results[head]["converged"]

    # Hessian apply on the sketch-width block in float64 (per-stage HIP events)
    prob = results["plain"]["prob"] if "plain" in results else prob
    Y = torch.empty_like(G)
    prob.set_profiling(True)
    stages = np.zeros(4)
    reps = 3
    for _ in range(reps):
        prob.apply_A(G, Y)
        stages += prob.last_apply_timing()
    prob.set_profiling(False)
    stages /= reps
    nA, q, m = prob.n_A, prob.q, w.m
    sweep_bytes = 8.0 * (nA + q) * m
    gemm_flops = 2.0 * w.n * w.n * (w.N + 1) * m
    hess = {"m": m, "ms": float(stages.sum()),
            "sweep_fwd_GBps": sweep_bytes / (stages[1] * 1e-3) / 1e9,
            "sweep_adj_GBps": sweep_bytes / (stages[2] * 1e-3) / 1e9,
            "sweep_hbm_frac": (2 * sweep_bytes / ((stages[1] + stages[2]) * 1e-3) / 1e9) / HBM_PEAK_GBS,
            "dsqrt_gemm_TFLOPs": 2 * gemm_flops / ((stages[0] + stages[3]) * 1e-3) / 1e12,
            "stage_ms": [float(v) for v in stages]}
    # composite roofline of the whole apply: each stage at its own bound (the two D^{1/2}
    # products at the float64 MFMA peak, the two sweeps at the HBM peak), summed
    comp = [gemm_flops / (FP64_PEAK_TFLOPS * 1e12) * 1e3, sweep_bytes / (HBM_PEAK_GBS * 1e9) * 1e3,
            sweep_bytes / (HBM_PEAK_GBS * 1e9) * 1e3, gemm_flops / (FP64_PEAK_TFLOPS * 1e12) * 1e3]
    hess.update({"composite_roofline_ms": float(sum(comp)), "composite_roofline_stage_ms": comp,
                 "composite_roofline_frac": float(sum(comp)) / float(stages.sum())})

    # roofline of the kernel class that takes the most time (timed live over the timed region)
    dom = dominant_class(results[head]["prof_classes"])
    dv = prof[dom]
    oz_head = bool(precs[head] & W4.PREC_DSQRT_OZ7)
    if dom == "dsqrt_gemm" and oz_head:
        # int8 slice products: OZ_PAIRS x 2 n^2 (N + 1) operations per launch group
        achieved = OZ_PAIRS * dv["flops"] / (dv["ms"] * 1e-3) / 1e12
        roof = {"bound": "mfma", "achieved": achieved, "peak": INT8_PEAK_TOPS, "unit": "TOP/s (int8)",
                "frac": achieved / INT8_PEAK_TOPS, "traffic": oz_measured_traffic(w)}
    elif dom in ("dsqrt_gemm", "dsqrt_bf16x3"):
        peak = FP64_PEAK_TFLOPS if dom == "dsqrt_gemm" else BF16_PEAK_TFLOPS
        achieved = dv["flops"] / (dv["ms"] * 1e-3) / 1e12
        traffic = measured_traffic(w, (tunes.get(head) or {}).get("m1")) if dom == "dsqrt_gemm" else None
        roof = {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                "frac": achieved / peak, "traffic": traffic}
    else:
        achieved = dv["bytes"] / (dv["ms"] * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": None}
    names_k = {"dsqrt_gemm": ("k_oz_split_cols + k_oz_gemm<16> + k_oz_reduce (6-slice int8 splitting of Q^(1/2) "
                              "and the vector's levels, level 0 scaled in the reduction)") if oz_head
               else dsqrt_kernel_name((tunes.get(head) or {}).get("m1")),
               "dsqrt_bf16x3": "k_gemm_bf16x3", "lmp_un": "k_pcg_lmp_dual_pan", "lmp_ut": "k_lmp_pan_t_partial",
               "sweep_fwd": "k_sweep_fwd_w", "sweep_bwd": "k_sweep_bwd_w"}
    roof.update({"kernel": names_k.get(dom, dom), "class": dom, "launches": dv["launches"],
                 "traffic_unit": "HBM bytes per launch group (rocprofv3 FETCH_SIZE x2.0 + WRITE_SIZE x1.0)",
                 "avg_launch_us": 1e3 * dv["ms"] / dv["launches"],
                 "sampled": f"HIP events around 1 in {args.prof_every} launch groups of the timed steps",
                 "algorithmic_per_launch": ((OZ_PAIRS if oz_head and dom == "dsqrt_gemm" else 1) *
                                            (dv["flops"] if dom.startswith("dsqrt") else dv["bytes"]) / dv["launches"])})
    if oz_head and dom == "dsqrt_gemm":
        roof["traffic_unit"] = ("HBM bytes per launch group of the three kernels (rocprofv3 FETCH_SIZE x2.0 + "
                                "WRITE_SIZE x1.0); algorithmic: 6 n^2 bytes of slices of Q^(1/2) (100.7 MB) + "
                                "the vector in and out")

    iters = results[head]["pcg_iters"]
    variants = {k: {kk: vv for kk, vv in v.items() if kk not in ("prof", "prob")} for k, v in results.items()}
    for k, v in results.items():
        variants[k]["kernel_classes_ms"] = {c: round(e["ms"] / v["classes_steps"], 3)
                                            for c, e in v["prof_classes"].items()}
        variants[k]["kernel_classes_from"] = ("last warm-up step (every class timed)" if v["classes_steps"] == 1
                                              and args.warmup > 0 else "timed steps (every class timed)")
    out = {
        "metric": "PCG time-to-1e-6 residual (learned/mixed vs plain FP64); Hessian-apply HBM GB/s",
        "value": ms_per_step, "unit": "ms", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_per_step, "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64+bf16x3+f16+i8x6" if head == "mixed" else "f64", "data": "synthetic",
        "config": {"workload": w.name, "variant": head, "method": args.method,
                   "pcg": "fused LMP (two passes over U per iteration)",
                   "n": w.n, "N": w.N, "n_A": nA, "q": q, "m": m, "k_r": w.k_r, "l": w.l, "tol": args.tol,
                   "criterion": "true residual ||b - A x|| / ||b||",
                   "autotuned_tiles": tunes.get(head), "tile_source": tile_source},
        "pcg_iters": iters, "relres_true": results[head]["relres_true"], "converged": ok,
        "variants": variants,
        "hessian_apply": hess,
        "roofline": roof,
    }
    sections_s = {"variants": time.perf_counter() - t_start}

    def section(name, fn):
        t = time.perf_counter()
        out[name] = fn()
        sections_s[name] = round(time.perf_counter() - t, 1)

    if not args.no_learned:
        section("learned", lambda: learned_section(args))
    if not args.no_second_loop:
        section("second_loop", lambda: second_loop_section(args))
    if not args.no_strong:
        section("strong_constraint", lambda: strong_section(args))
    if not args.no_ritz:
        section("ritz_lmp", lambda: ritz_section(args))
    if not args.no_batched:
        section("batched", lambda: batched_section(args))
    if not args.no_oversampling:
        section("oversampling", lambda: oversampling_section(args))
    if not args.no_cpu_baseline:
        section("cpu_baseline", lambda: cpu_baseline(w, pat, results["plain"]["pcg_iters"] if "plain" in results
                                                     else None, args))
    sections_s["variants"] = round(sections_s["variants"], 1)
    out["sections_s"] = sections_s
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
