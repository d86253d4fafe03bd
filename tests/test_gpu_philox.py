"""GPU parity of the device Gaussian start block (Section 4, Algorithms 3-5: G has
independent N(0, 1) entries) against the oracle's own Philox-4x32-10 + Box-Muller.

Bars: the generator's words are integers, so they must match bit for bit (the published
known-answer vectors and random counters/keys).  The normals go through log, sqrt, cos and
sin, which the device math library and numpy each round within a couple of ulps, so each
entry must agree to 1e-15 of its magnitude (plus 1e-17 absolute for entries near a zero
of the cosine or sine).  An LMP built from a seed must equal the LMP built from the block
the same seed draws (same kernels, same values: bit-identical Ritz values), and match the
oracle's build from the oracle's block to the FP64 bar per Ritz value."""
import json
import os

import numpy as np
import pytest

from oracle import philox as PX
from oracle import wc4d_oracle as O
from synthetic import C1, C3, innovations, obs_pattern

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "philox4x32_10_kat.json")


def _torch():
    import torch
    return torch


def dev():
    return _torch().device("cuda", 0)


def say(*a):
    print("[case]", *a, flush=True)


def words_on_device(ctr_key_u32: np.ndarray) -> np.ndarray:
    from paper_2101_07249_amd import wc4d
    t = _torch()
    ck = t.from_numpy(ctr_key_u32.astype(np.uint32).view(np.int32).copy()).to(dev())
    return wc4d.philox4x32_10(ck).cpu().numpy().view(np.uint32)


def test_philox_known_answer_vectors():
    say("philox KAT")
    kat = json.load(open(GOLDEN))["vectors"]
    rows = np.array([[int(v, 16) for v in e["counter"] + e["key"]] for e in kat], dtype=np.uint64)
    out = words_on_device(rows)
    want = np.array([[int(v, 16) for v in e["output"]] for e in kat], dtype=np.uint32)
    assert np.array_equal(out, want)


def test_philox_words_match_oracle_bit_for_bit():
    say("philox random counters and keys")
    rng = np.random.default_rng(20110101)
    rows = rng.integers(0, 2 ** 32, size=(5000, 6), dtype=np.uint64)
    out = words_on_device(rows)
    want = np.stack([PX.philox4x32_10(rows[i:i + 1, :4], (int(rows[i, 4]), int(rows[i, 5])))[0]
                     for i in range(rows.shape[0])])
    assert np.array_equal(out, want)


def _check_normals(G, Go):
    d = np.abs(G - Go)
    bound = 1e-15 * np.abs(Go) + 1e-17
    bad = np.argwhere(d > bound)
    assert bad.size == 0, (bad[:5], d[tuple(bad[0])] if bad.size else None)


@pytest.mark.parametrize("seed,n_rows,n_cols,col0", [(0, 1, 1, 0), (7, 1001, 7, 3), (2 ** 40 + 5, 840, 10, 0),
                                                     (123456789, 4097, 3, 4294967000)])
def test_gaussian_block_matches_oracle(seed, n_rows, n_cols, col0):
    """Odd row counts (the last pair keeps only its cosine normal), seeds above 2^32 (the
    key's high word), column offsets up to the top of the 32-bit counter word."""
    from paper_2101_07249_amd import wc4d
    say("gaussian block", seed, n_rows, n_cols, col0)
    G = wc4d.gaussian_block(seed, n_rows, n_cols, col0).cpu().numpy().T
    Go = PX.gaussian_columns(seed, n_rows, range(col0, col0 + n_cols))
    _check_normals(G, Go)


def test_gaussian_block_at_benchmark_size_sampled_columns_and_moments():
    """The n_A x m block of the benchmark workload (413,696 x 256): sampled columns against
    the oracle (rows past 2^17 pairs exercise the full counter word), column ranges drawn
    separately give the same entries, and the moments of all 106M entries are those of
    N(0, 1) within 6 standard errors."""
    from paper_2101_07249_amd import wc4d
    t = _torch()
    say("gaussian block C3 size")
    nA, m, seed = C3.n_A, C3.m, 31337
    G = wc4d.gaussian_block(seed, nA, m)
    for c in (0, 1, 128, 255):
        _check_normals(G[c].cpu().numpy()[:, None], PX.gaussian_columns(seed, nA, [c]))
    part = wc4d.gaussian_block(seed, nA, 5, col0=100)
    assert t.equal(part, G[100:105])
    cnt = G.numel()
    mean = G.mean().item()
    var = G.var().item()
    m4 = (G ** 4).mean().item()
    assert abs(mean) <= 6.0 / np.sqrt(cnt)
    assert abs(var - 1.0) <= 6.0 * np.sqrt(2.0 / cnt)
    assert abs(m4 - 3.0) <= 6.0 * np.sqrt(96.0 / cnt)
    # each row parity draws its own normal: cosine and sine halves are uncorrelated
    ev, od = G[:, 0:nA - 1:2], G[:, 1:nA:2]
    corr = (ev * od).mean().item()
    assert abs(corr) <= 6.0 / np.sqrt(ev.numel())


@pytest.mark.parametrize("method", ["revd", "nystrom", "ritzit"])
def test_seeded_lmp_build_equals_explicit_block_and_oracle(method):
    from paper_2101_07249_amd import Problem, wc4d
    say("seeded lmp build", method)
    w = C1
    pat = obs_pattern(w)
    gp = Problem.from_workload(w, pat)
    op = O.make_problem(w, pat)
    seed = 4242
    Ls = gp.lmp_build(method, w.k_r, w.l, seed=seed)
    Lg = gp.lmp_build(method, w.k_r, w.l, wc4d.gaussian_block(seed, w.n_A, w.m))
    ths, thg = Ls.theta(), Lg.theta()
    assert np.array_equal(ths, thg)
    Go = PX.gaussian_block(seed, w.n_A, w.m)
    _, tho = O.METHODS[method](lambda Z: O.apply_A(op, Z), Go, w.k_r)
    assert np.all(np.abs(ths - tho) <= 1e-10 * np.abs(tho)), (ths, tho)
    # and the seeded LMP preconditions PCG to the true 1e-6
    d = _torch().from_numpy(innovations(op.q, w.seed, np.sqrt(w.sigma_o2))).to(dev())
    b = gp.rhs(d)
    x = _torch().zeros(w.n_A, dtype=_torch().float64, device=dev())
    info = gp.pcg(b, x, Ls, tol=1e-6, maxit=200)
    assert info["status"] == 0 and info["relres_true"] <= 1e-6


def test_gaussian_block_rejects_bad_arguments():
    from paper_2101_07249_amd import wc4d
    say("gaussian block bad arguments")
    t = _torch()
    out = t.empty((2, 10), dtype=t.float64, device=dev())
    L = wc4d.lib()
    assert L.wc4d_gaussian_block(0, 1, 10, 2, 0, out.data_ptr(), 9, None) == wc4d.EINVAL      # ldg < rows
    assert L.wc4d_gaussian_block(0, 1, -1, 2, 0, out.data_ptr(), 10, None) == wc4d.EINVAL     # negative rows
    assert L.wc4d_gaussian_block(0, 1, 10, 2, 2 ** 32 - 1, out.data_ptr(), 10, None) == wc4d.EINVAL
    assert L.wc4d_gaussian_block(99, 1, 10, 2, 0, out.data_ptr(), 10, None) == wc4d.EINVAL    # no such device
    assert L.wc4d_gaussian_block(0, 1, 10, 2, 0, None, 10, None) == wc4d.EINVAL
    assert L.wc4d_gaussian_block(0, 1, 0, 0, 0, None, 1, None) == wc4d.OK                      # empty block
    with pytest.raises(ValueError):
        wc4d.gaussian_block(1, 10, 2, out=t.empty((3, 10), dtype=t.float64, device=dev()))
