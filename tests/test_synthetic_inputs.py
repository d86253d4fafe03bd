"""The seeded input module: reproducible draws, independent streams per purpose, and the
shapes, ranges and rates the workloads state.  CPU only."""
import numpy as np

from synthetic import (C1, C3, C5, batched_workloads, innovations, l96_initial_state, obs_count, obs_pattern,
                       sketch_block)


def test_draws_are_reproducible_and_streams_independent():
    a = sketch_block(1000, 8, 42)
    assert np.array_equal(a, sketch_block(1000, 8, 42))
    assert a.flags.f_contiguous and a.shape == (1000, 8)
    # a wider block extends a narrower one column by column
    assert np.array_equal(sketch_block(1000, 12, 42)[:, :8], a)
    # other seeds, instances and purposes give other numbers
    assert not np.array_equal(a, sketch_block(1000, 8, 43))
    assert not np.array_equal(a, sketch_block(1000, 8, 42, instance=1))
    assert not np.allclose(innovations(1000, 42, 1.0), a[:, 0])
    g = sketch_block(200_000, 4, 7)
    assert abs(g.mean()) < 5e-3 and abs(g.var() - 1.0) < 5e-3
    d = innovations(200_000, 7, 0.1)
    assert abs(d.std() - 0.1) < 1e-3
    x0 = l96_initial_state(100_000, 7)
    assert abs(x0.mean() - 2.3) < 0.05 and abs(x0.std() - 3.6) < 0.05


def test_workload_sizes_and_observation_rates():
    assert (C1.n_A, obs_count(obs_pattern(C1))) == (840, 100)
    assert (C3.n_A, obs_count(obs_pattern(C3))) == (413_696, 51_200)
    ws = batched_workloads()
    assert len(ws) == 64
    assert all(512 <= w.n <= 8192 and 10 <= w.N <= 200 for w in ws)
    assert ws == batched_workloads()
    pat = obs_pattern(ws[0])
    assert all(i >= 1 for i, _ in pat)
    rate = obs_count(pat) / (ws[0].n * ws[0].N)
    assert abs(rate - 0.125) < 0.02
    # learned-sketch instances: every 5th step observed (final step included), about half the points
    p5 = obs_pattern(C5, instance=3)
    times = [i for i, _ in p5]
    assert times == list(range(5, C5.N + 1, 5))
    assert abs(obs_count(p5) / (C5.n * len(times)) - 0.5) < 0.03
    assert obs_pattern(C5, instance=3)[0][1].tolist() == p5[0][1].tolist()
    assert obs_pattern(C5, instance=4)[0][1].tolist() != p5[0][1].tolist()
