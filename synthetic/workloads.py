"""Workload parameters and seeded random draws for the inner-loop problems.

The workloads are identical-twin style systems shaped like the paper's idealised
experiments (Section 5: linear advection and Lorenz-96 with direct observations,
diagonal R, correlated B and Q).  The paper publishes no dataset; every array
here is synthetic and seeded (seed = 1000 * config + instance).

Nothing in this module evaluates the method: no model step, no covariance
square root, no Hessian product.  It only fixes sizes/parameters and draws
random numbers (sketch matrices, innovations, initial states, observation
masks), which both the GPU path and the oracle then consume as inputs.
"""
from __future__ import annotations

from dataclasses import dataclass, replace
from typing import List, Tuple

import numpy as np

__all__ = [
    "Workload", "C1", "C2", "C3", "C5", "SEC52", "WORKLOADS", "batched_workloads",
    "obs_pattern", "obs_count", "sketch_block", "innovations", "l96_initial_state",
    "rng_for",
]

# purpose tags for independent random substreams of one seed
_PURPOSE = {"sketch": 1, "innov": 2, "x0": 3, "obsmask": 4, "sizes": 5, "vec": 6, "net": 7, "twin": 8}


def rng_for(seed: int, purpose: str) -> np.random.Generator:
    """Independent numpy PCG64 stream for (seed, purpose)."""
    return np.random.default_rng([int(seed), _PURPOSE[purpose]])


@dataclass(frozen=True)
class Workload:
    """One inner-loop problem (sizes and parameters only).

    model     'advdiff' (periodic upwind advection + explicit diffusion) or 'l96'
    n, N      state size per time level, number of model steps (N+1 levels)
    c, r      advection Courant number and diffusion number (advdiff)
    F, dt     forcing and RK4 step (l96)
    corr      correlation family for B and Q: 'soar' or 'gauss' (chordal distance)
    Lb, Lq    correlation length scales in grid points
    sigma_b, sigma_q   standard deviations of B and Q
    obs_kind  'regular' (every obs_var_stride-th point at every obs_time_stride-th
              step, times s, 2s, ..., N) or 'bernoulli' (seeded mask)
    sigma_o2  observation error variance (R_i = sigma_o2 * I)
    m, l      sketch width (block of Gaussian vectors) and oversampling; the LMP
              keeps k_r = m - l Ritz pairs
    """
    name: str
    model: str
    n: int
    N: int
    c: float = 0.0
    r: float = 0.0
    F: float = 8.0
    dt: float = 0.025
    corr: str = "soar"
    Lb: float = 4.0
    Lq: float = 4.0
    sigma_b: float = 1.0
    sigma_q: float = 0.1
    obs_kind: str = "regular"
    obs_var_stride: int = 4
    obs_time_stride: int = 2
    obs_prob: float = 0.125
    obs_all_times: bool = False
    sigma_o2: float = 0.01
    m: int = 10
    l: int = 5
    seed: int = 1000

    @property
    def n_A(self) -> int:
        return self.n * (self.N + 1)

    @property
    def k_r(self) -> int:
        return self.m - self.l

    def with_(self, **kw) -> "Workload":
        return replace(self, **kw)


# Plain FP64 advection-diffusion: n=40, N=20 (dim 840), SOAR L=4, sigma_b=1,
# sigma_q=0.1, every 4th point every 2nd step, R=0.01 I, sketch of 10.
C1 = Workload(name="advdiff_n40_N20_m10", model="advdiff", n=40, N=20, c=0.5, r=0.1,
              corr="soar", Lb=4.0, Lq=4.0, sigma_b=1.0, sigma_q=0.1,
              obs_var_stride=4, obs_time_stride=2, sigma_o2=0.01, m=10, l=5, seed=1000)

# Plain FP64 Lorenz-96: n=80, F=8, dt=0.025, N=50 (dim 4080), Gaussian L=2,
# sigma_b=0.2 / sigma_q=0.1 (the paper's L96 values), every 2nd variable every
# 5th step, R=0.04 I, sketch of 50.
C2 = Workload(name="l96_n80_N50_m50", model="l96", n=80, N=50, F=8.0, dt=0.025,
              corr="gauss", Lb=2.0, Lq=2.0, sigma_b=0.2, sigma_q=0.1,
              obs_var_stride=2, obs_time_stride=5, sigma_o2=0.04, m=50, l=5, seed=2000)

# Mixed-precision / roofline workload: advection-diffusion n=4096, N=100
# (dim 413,696), SOAR L=4, inherits C1's covariances and observation pattern,
# sketch of 256.
C3 = Workload(name="advdiff_n4096_N100_m256", model="advdiff", n=4096, N=100, c=0.5, r=0.1,
              corr="soar", Lb=4.0, Lq=4.0, sigma_b=1.0, sigma_q=0.1,
              obs_var_stride=4, obs_time_stride=2, sigma_o2=0.01, m=256, l=5, seed=3000)

# Learned-sketch workload: Lorenz-96 n=1024, N=100, sketch of 64; Bernoulli(1/2)
# observed points at every 5th step (final step included); C2 covariances.
C5 = Workload(name="l96_n1024_N100_m64", model="l96", n=1024, N=100, F=8.0, dt=0.025,
              corr="gauss", Lb=2.0, Lq=2.0, sigma_b=0.2, sigma_q=0.1,
              obs_kind="bernoulli_times", obs_time_stride=5, obs_prob=0.5,
              sigma_o2=0.04, m=64, l=5, seed=5000)

# Section 5.2's own Lorenz-96 configuration (n = 80, N = 150, 120 observations: every 10th
# variable at every 10th step; sigma_o = 0.15, sigma_b = 0.2, sigma_q = 0.1, length scales
# 2 grid spacings; k = 15 of the oversampling study), SOAR for both covariances.
SEC52 = Workload(name="l96_n80_N150_sec52", model="l96", n=80, N=150, F=8.0, dt=0.025, corr="soar", Lb=2.0,
                 Lq=2.0, sigma_b=0.2, sigma_q=0.1, obs_var_stride=10, obs_time_stride=10, sigma_o2=0.15 ** 2,
                 m=20, l=5, seed=5200)

WORKLOADS = {"C1": C1, "C2": C2, "C3": C3, "C5": C5, "SEC52": SEC52}


def batched_workloads(count: int = 64, seed: int = 4000, m: int = 64,
                      n_range=(512, 8192), N_range=(10, 200)) -> List[Workload]:
    """Uneven advection-diffusion problems: n ~ U{n_range}, N ~ U{N_range},
    Bernoulli(1/8) observation mask over (i >= 1, j), sigma_o = 0.1, SOAR L=4."""
    rng = rng_for(seed, "sizes")
    ns = rng.integers(n_range[0], n_range[1] + 1, size=count)
    Ns = rng.integers(N_range[0], N_range[1] + 1, size=count)
    out = []
    for b in range(count):
        out.append(Workload(name=f"batch{b}", model="advdiff", n=int(ns[b]), N=int(Ns[b]),
                            c=0.5, r=0.1, corr="soar", Lb=4.0, Lq=4.0, sigma_b=1.0,
                            sigma_q=0.1, obs_kind="bernoulli", obs_prob=0.125,
                            sigma_o2=0.01, m=m, l=5, seed=seed + b))
    return out


def obs_pattern(w: Workload, instance: int = 0) -> List[Tuple[int, np.ndarray]]:
    """Observed (time index i, int32 point indices) pairs.

    'regular': times s, 2s, ..., N (s = obs_time_stride; t_0 unobserved, the final
    step observed) and points j = 0, v, 2v, ... (v = obs_var_stride); with
    obs_all_times the times are 0, s, 2s, ... instead.
    'bernoulli': every (i >= 1, j) observed independently with prob obs_prob.
    'bernoulli_times': times s, 2s, ..., N, points drawn with prob obs_prob.
    """
    out = []
    if w.obs_kind == "regular":
        s = w.obs_time_stride
        times = range(0 if w.obs_all_times else s, w.N + 1, s)
        idx = np.arange(0, w.n, w.obs_var_stride, dtype=np.int32)
        for i in times:
            out.append((int(i), idx.copy()))
    elif w.obs_kind == "bernoulli":
        rng = rng_for(w.seed + 7919 * instance, "obsmask")
        mask = rng.random((w.N + 1, w.n)) < w.obs_prob
        mask[0, :] = False
        for i in range(1, w.N + 1):
            idx = np.nonzero(mask[i])[0].astype(np.int32)
            if idx.size:
                out.append((i, idx))
    elif w.obs_kind == "bernoulli_times":
        rng = rng_for(w.seed + 7919 * instance, "obsmask")
        for i in range(w.obs_time_stride, w.N + 1, w.obs_time_stride):
            idx = np.nonzero(rng.random(w.n) < w.obs_prob)[0].astype(np.int32)
            if idx.size:
                out.append((i, idx))
    else:
        raise ValueError(w.obs_kind)
    return out


def obs_count(pattern) -> int:
    return int(sum(len(idx) for _, idx in pattern))


def sketch_block(n_A: int, m: int, seed: int, instance: int = 0) -> np.ndarray:
    """Gaussian start matrix G (n_A x m), iid N(0,1), column-major (Fortran order)."""
    rng = rng_for(seed + 7919 * instance, "sketch")
    return np.asfortranarray(rng.standard_normal((m, n_A)).T)


def innovations(q: int, seed: int, sigma: float, instance: int = 0) -> np.ndarray:
    """Innovation vector d (q,), iid N(0, sigma^2), stacked in observed-time order."""
    rng = rng_for(seed + 7919 * instance, "innov")
    return sigma * rng.standard_normal(q)


def l96_initial_state(n: int, seed: int, instance: int = 0,
                      mean: float = 2.3, std: float = 3.6) -> np.ndarray:
    """Initial state for a Lorenz-96 window: iid N(mean, std^2) per point (a
    climatology-sized random state; no model integration happens here)."""
    rng = rng_for(seed + 7919 * instance, "x0")
    return mean + std * rng.standard_normal(n)


def random_block(rows: int, cols: int, seed: int, instance: int = 0) -> np.ndarray:
    """Generic iid N(0,1) test block, column-major."""
    rng = rng_for(seed + 7919 * instance, "vec")
    return np.asfortranarray(rng.standard_normal((cols, rows)).T)


__all__.append("random_block")


def twin_draws(w: Workload, q: int, instance: int = 0):
    """Standard normal draws of an identical-twin experiment (Section 5): the truth's initial
    state x0 (climatology-sized, as l96_initial_state), its model errors xi_model (N, n),
    the background error xi_b (n,) and the observation errors zeta (q,).  Scaling by
    Q^{1/2}, B^{1/2} and sigma_o is left to the caller."""
    rng = rng_for(w.seed + 7919 * instance, "twin")
    return {"x0": l96_initial_state(w.n, w.seed, instance) if w.model == "l96" else None,
            "xi_model": rng.standard_normal((w.N, w.n)), "xi_b": rng.standard_normal(w.n),
            "zeta": rng.standard_normal(q)}


__all__.append("twin_draws")


def sketchnet_init(layers: int = 4, noise_channels: int = 64, seed: int = 7000, channels: int = 64,
                   width: int = 5) -> np.ndarray:
    """Initial parameters of the sketch network, float32, in the library's order (per
    layer W (c_out, c_in, t) row-major, then the bias): W ~ N(0, 1/(c_in width)), b = 0."""
    rng = rng_for(seed, "net")
    parts = []
    cin = noise_channels + 4
    for _ in range(layers):
        parts.append(rng.standard_normal(channels * cin * width) / np.sqrt(cin * width))
        parts.append(np.zeros(channels))
        cin = channels
    return np.concatenate(parts).astype(np.float32)


__all__.append("sketchnet_init")
