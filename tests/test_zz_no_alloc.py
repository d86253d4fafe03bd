"""The LMP application that allocates nothing (wc4d_lmp_apply_noalloc) against
wc4d_lmp_apply, through the C-ABI: the same kernels with the scratch buffer in a fixed
device array, so the outputs must be bit-identical.  Two calls in a row, the second on a
smaller LMP (the array keeps the first call's contents), for one and two vectors, float64
and float16 copies of U."""
import ctypes

import numpy as np
import pytest

from synthetic import C1, C2, l96_initial_state, obs_pattern, random_block, sketch_block

pytestmark = pytest.mark.gpu


def _lmp(w, prec):
    import torch
    from paper_2101_07249_amd import Problem
    pat = obs_pattern(w)
    x0 = l96_initial_state(w.n, w.seed) if w.model == "l96" else None
    p = Problem.from_workload(w, pat, x0=x0, prec=prec)
    G = torch.from_numpy(np.ascontiguousarray(sketch_block(p.n_A, w.m, w.seed).T)).to("cuda")
    return p, p.lmp_build("nystrom", w.k_r, w.l, G)


def _noalloc(L, X, Y, m):
    import torch
    from paper_2101_07249_amd import wc4d
    lib = wc4d.lib()
    lib.wc4d_lmp_apply_noalloc.restype = ctypes.c_int
    lib.wc4d_lmp_apply_noalloc.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                                           ctypes.c_int, ctypes.c_int, ctypes.c_void_p]
    n_A = L.prob.n_A
    rc = lib.wc4d_lmp_apply_noalloc(L._h, X.data_ptr(), n_A, Y.data_ptr(), n_A, m,
                                    torch.cuda.current_stream().cuda_stream)
    return rc


@pytest.mark.parametrize("prec", [0, 8], ids=["f64", "f16copy"])
def test_noalloc_matches_lmp_apply_twice(prec):
    import torch
    print("[case] lmp_apply_noalloc, prec", prec, flush=True)
    for w in (C2, C1):     # the second call on a smaller LMP
        p, L = _lmp(w, prec)
        for m in (2, 1):
            X = torch.from_numpy(np.ascontiguousarray(random_block(p.n_A, m, 7 + m).T)).to("cuda")
            Yref = L.apply(X)
            Y = torch.full_like(X, float("nan"))
            assert _noalloc(L, X, Y, m) == 0
            torch.cuda.synchronize()
            assert torch.equal(Y, Yref), (w.name, m)
        # more than two vectors, or overlapping input and output, are rejected
        X3 = torch.zeros((3, p.n_A), dtype=torch.float64, device="cuda")
        assert _noalloc(L, X3, torch.empty_like(X3), 3) == -1
        assert _noalloc(L, X3, X3, 1) == -1
