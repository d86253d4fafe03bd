"""Reduced-precision forms against the FP64 oracle, each with a stated tolerance.

Split-bf16 D^{1/2} products (three bf16 products, float32 accumulation): the
dropped lo*lo term and the bf16 rounding of the low parts are ~2^-16 relative per
product, and float32 accumulation over K = n terms adds ~sqrt(n) 2^-24, so the
Hessian apply is expected near 1e-5 relative; the bound used is 1e-4.  Ritz values
of a build whose block applies use that product inherit the same relative error
(bound 1e-4).  PCG itself runs the float64 operator, so the mixed preconditioner
must still reach the float64 true residual; its iteration count is compared with
the float64 preconditioner's (bound: within 5% + 2).

Blocks are compared column by column (largest entry error of each column relative to
that column's largest entry).  Ritz values are compared entry by entry against Weyl's
bound for a symmetric perturbation E of the operator, |theta_i - theta_i,o| <= ||E||_2,
with ||E|| ~ the apply's relative error times theta_max: each |dtheta_i| must lie within
the stated relative bound times theta_1 (the largest Ritz value)."""
import numpy as np
import pytest

from oracle import wc4d_oracle as O
from parity import col_errors
from synthetic import (C1, C2, C3, Workload, innovations, l96_initial_state, obs_pattern, random_block,
                       sketch_block)

pytestmark = pytest.mark.gpu


def _pair(w, prec):
    from paper_2101_07249_amd import Problem
    pat = obs_pattern(w)
    x0 = l96_initial_state(w.n, w.seed) if w.model == "l96" else None
    return Problem.from_workload(w, pat, x0=x0, prec=prec), O.make_problem(w, pat, x0=x0)


def _dev(A):
    import torch
    return torch.from_numpy(np.ascontiguousarray(A.T if A.ndim == 2 else A)).to("cuda")


MEDIUM = Workload(name="adv_n700_N30", model="advdiff", n=700, N=30, c=0.5, r=0.1, corr="soar", Lb=4.0,
                  Lq=4.0, sigma_b=1.0, sigma_q=0.1, obs_var_stride=4, obs_time_stride=2,
                  sigma_o2=0.01, m=40, l=5, seed=9100)


# B^{1/2} and Q^{1/2} with different length scales: level 0 takes its own product
MEDIUM_BQ = Workload(name="adv_n700_N30_LbLq", model="advdiff", n=700, N=30, c=0.5, r=0.1, corr="soar", Lb=6.0,
                     Lq=3.0, sigma_b=1.0, sigma_q=0.1, obs_var_stride=4, obs_time_stride=2,
                     sigma_o2=0.01, m=40, l=5, seed=9200)


# kernel: the size rule ("auto": the LDS-tiled kernel at these sizes) or the fragment-major
# kernel forced on ragged shapes (n = 40, 80, 700 rows and K; 220 to 3100 columns)
@pytest.mark.parametrize("kernel", ["auto", "frag"])
@pytest.mark.parametrize("w", [C1, C2, MEDIUM, MEDIUM_BQ], ids=["C1", "C2", "adv700", "adv700_LbLq"])
def test_bf16x3_apply_error(w, kernel, monkeypatch):
    from paper_2101_07249_amd import wc4d
    print("[case] bf16x3 apply", w.name, kernel, flush=True)
    if kernel != "auto":
        monkeypatch.setenv("WC4D_SPLIT_GEMM_KERNEL", kernel)
    gp, op = _pair(w, wc4d.PREC_SKETCH_BF16X3)
    G = sketch_block(op.n_A, w.m, w.seed)
    Yo = O.apply_A(op, G)
    Ym = gp.apply_A_prec(_dev(G), wc4d.PREC_SKETCH_BF16X3).cpu().numpy().T
    Yd = gp.apply_A_prec(_dev(G), wc4d.PREC_FP64).cpu().numpy().T
    e_m = float(col_errors(Ym, Yo).max())
    e_d = float(col_errors(Yd, Yo).max())
    print("[result] rel err bf16x3", e_m, "fp64", e_d, flush=True)
    assert e_d <= 1e-10
    assert e_m <= 1e-4
    assert e_m > 1e-9   # really computed in reduced precision


@pytest.mark.parametrize("method", ["revd", "nystrom", "ritzit"])
def test_mixed_lmp_and_pcg(method):
    from paper_2101_07249_amd import wc4d
    import torch
    w = C2
    print("[case] mixed lmp + pcg", method, flush=True)
    gm, op = _pair(w, wc4d.PREC_SKETCH_BF16X3 | wc4d.PREC_LMP_FP32)
    gd, _ = _pair(w, wc4d.PREC_FP64)
    G = sketch_block(op.n_A, w.m, w.seed)
    Lm = gm.lmp_build(method, w.k_r, w.l, _dev(G))
    Ld = gd.lmp_build(method, w.k_r, w.l, _dev(G))
    _, tho = O.METHODS[method](lambda Z: O.apply_A(op, Z), G, w.k_r)
    th = Lm.theta()
    e = float(np.abs(th - tho).max() / tho[0])   # Weyl: each |dtheta_i| against theta_1
    print("[result] theta err / theta_1", e, "per entry", float((np.abs(th - tho) / tho).max()), flush=True)
    assert e <= 1e-4
    d = innovations(op.q, w.seed, np.sqrt(w.sigma_o2))
    b = O.rhs(op, d)
    xm = torch.zeros(op.n_A, dtype=torch.float64, device="cuda")
    xd = torch.zeros(op.n_A, dtype=torch.float64, device="cuda")
    im = gm.pcg(gm.rhs(_dev(d)), xm, Lm, tol=1e-6, maxit=3000)
    idd = gd.pcg(gd.rhs(_dev(d)), xd, Ld, tol=1e-6, maxit=3000)
    assert im["status"] == 0 and idd["status"] == 0
    res = np.linalg.norm(b - O.apply_A(op, xm.cpu().numpy())) / np.linalg.norm(b)
    print("[result] iters mixed", im["iters"], "fp64", idd["iters"], "true res", res, flush=True)
    assert res <= 1.05e-6
    assert im["iters"] <= 1.05 * idd["iters"] + 2


def test_bf16x3_full_size_sampled_columns():
    from paper_2101_07249_amd import wc4d
    print("[case] bf16x3 full size", flush=True)
    pat = obs_pattern(C3)
    from paper_2101_07249_amd import Problem
    gp = Problem.from_workload(C3, pat, prec=wc4d.PREC_SKETCH_BF16X3 | wc4d.PREC_LMP_FP32)
    op = O.make_problem(C3, pat)
    G = sketch_block(gp.n_A, C3.m, C3.seed)
    Y = gp.apply_A_prec(_dev(G), wc4d.PREC_SKETCH_BF16X3)
    cols = [0, 3, 200, 255]  # the first and last 256-column tiles of the all-level product too
    Yo = O.apply_A(op, G[:, cols])
    e = float(col_errors(Y[cols].cpu().numpy().T, Yo).max())
    print("[result] full-size bf16x3 rel err", e, flush=True)
    assert 1e-9 < e <= 1e-4


@pytest.mark.parametrize("k_r", [1, 3, 6, 9])
def test_fp32_panel_lmp_apply_and_pcg(k_r):
    """The PCG's float32 copy of U is stored in 256-row panels.  C1 has n_A = 840 (three full
    panels and a ragged one); k_r runs below, at and above the 4 waves x 2 columns that a pass
    keeps in flight.  One- and two-column applies stream the float32 panels (float32 rounding
    of U: C v within 1e-5 relative of the oracle's float64 C v); wider ones take the float64
    block path.  Both PCG variants must match the oracle's PCG to 2 iterations and reach its
    true residual."""
    from paper_2101_07249_amd import wc4d
    import torch
    w = C1
    m = k_r + w.l
    print("[case] fp32 panel LMP, k_r", k_r, flush=True)
    gm, op = _pair(w, wc4d.PREC_LMP_FP32)
    G = sketch_block(op.n_A, m, w.seed)
    L = gm.lmp_build("nystrom", k_r, w.l, _dev(G))
    Uo, tho = O.METHODS["nystrom"](lambda Z: O.apply_A(op, Z), G, k_r)
    for ncols in (1, 2, 3):
        V = random_block(op.n_A, ncols, 9 + ncols)
        CV = L.apply(_dev(V)).cpu().numpy()
        CV = CV.T if CV.ndim == 2 else CV[:, None]
        CVo = O.lmp_apply(Uo, tho, V)
        e = float(col_errors(CV, CVo).max())
        print("[result] columns", ncols, "rel err", e, flush=True)
        assert e <= 1e-5
        if ncols <= 2:
            assert e > 1e-12   # the float32 copy really is what the one-vector passes read
    d = innovations(op.q, w.seed, np.sqrt(w.sigma_o2))
    b = O.rhs(op, d)
    ro = O.pcg(lambda v: O.apply_A(op, v), b, lmp=(Uo, tho), tol=1e-6, maxit=500)
    for variant in (wc4d.PCG_FUSED, wc4d.PCG_PLAIN):
        x = torch.zeros(op.n_A, dtype=torch.float64, device="cuda")
        info = gm.pcg(gm.rhs(_dev(d)), x, L, tol=1e-6, maxit=500, variant=variant)
        res = np.linalg.norm(b - O.apply_A(op, x.cpu().numpy())) / np.linalg.norm(b)
        print("[result] variant", variant, "iters", info["iters"], "oracle", ro.iters, "true res", res, flush=True)
        assert info["status"] == 0 and res <= 1.01e-6
        assert abs(info["iters"] - ro.iters) <= 2


@pytest.mark.parametrize("k_r", [1, 3, 17, 33, 40])
def test_fp16_panel_lmp_apply_and_pcg(k_r):
    """Float16 panel copy of U, each column scaled by a power of two.  k_r runs below, at and
    above the 16 columns a float16 pass keeps in flight per block and the 32-column groups of
    its U^T x pass; C1's n_A = 840 leaves a ragged last panel.  Rounding: |du| <= 2^-11 |u|
    per entry, so ||dU||_2 <= 2^-11 sqrt(k) and C v moves by at most 2 ||dU||_2 ||v|| (the
    coefficients theta^{-1/2} - 1 lie in (-1, 0]); the bound is that, relative to ||C v||
    (~||v|| for a random v).  PCG must still reach the float64 true residual, within
    5% + 2 iterations of the oracle's PCG."""
    from paper_2101_07249_amd import wc4d
    import torch
    w = C1
    m = k_r + w.l
    print("[case] fp16 panel LMP, k_r", k_r, flush=True)
    gm, op = _pair(w, wc4d.PREC_LMP_FP16)
    G = sketch_block(op.n_A, m, w.seed)
    L = gm.lmp_build("nystrom", k_r, w.l, _dev(G))
    Uo, tho = O.METHODS["nystrom"](lambda Z: O.apply_A(op, Z), G, k_r)
    bound = 2.0 * 2.0 ** -11 * np.sqrt(k_r)
    for ncols in (1, 2, 3):
        V = random_block(op.n_A, ncols, 9 + ncols)
        CV = L.apply(_dev(V)).cpu().numpy()
        CV = CV.T if CV.ndim == 2 else CV[:, None]
        CVo = O.lmp_apply(Uo, tho, V)
        e = float(col_errors(CV, CVo).max())
        print("[result] columns", ncols, "rel err", e, "bound", bound, flush=True)
        assert e <= bound
        if ncols <= 2:
            assert e > 1e-9   # the float16 copy really is what the one-vector passes read
    d = innovations(op.q, w.seed, np.sqrt(w.sigma_o2))
    b = O.rhs(op, d)
    ro = O.pcg(lambda v: O.apply_A(op, v), b, lmp=(Uo, tho), tol=1e-6, maxit=500)
    for variant in (wc4d.PCG_FUSED, wc4d.PCG_PLAIN):
        x = torch.zeros(op.n_A, dtype=torch.float64, device="cuda")
        info = gm.pcg(gm.rhs(_dev(d)), x, L, tol=1e-6, maxit=500, variant=variant)
        res = np.linalg.norm(b - O.apply_A(op, x.cpu().numpy())) / np.linalg.norm(b)
        print("[result] variant", variant, "iters", info["iters"], "oracle", ro.iters, "true res", res, flush=True)
        assert info["status"] == 0 and res <= 1.01e-6
        assert info["iters"] <= 1.05 * ro.iters + 2


def test_fp16_panel_lmp_pcg_c2_and_flag_errors():
    """C2 (n_A = 4,080, k_r = 45): the float16 copy's PCG against the float64 LMP's, same
    sketch; LMP_FP32 and LMP_FP16 together are rejected."""
    from paper_2101_07249_amd import Problem, Wc4dError, wc4d
    import torch
    w = C2
    print("[case] fp16 panel LMP, C2", flush=True)
    gm, op = _pair(w, wc4d.PREC_LMP_FP16)
    gd, _ = _pair(w, wc4d.PREC_FP64)
    G = sketch_block(op.n_A, w.m, w.seed)
    Lm = gm.lmp_build("nystrom", w.k_r, w.l, _dev(G))
    Ld = gd.lmp_build("nystrom", w.k_r, w.l, _dev(G))
    d = innovations(op.q, w.seed, np.sqrt(w.sigma_o2))
    b = O.rhs(op, d)
    xm = torch.zeros(op.n_A, dtype=torch.float64, device="cuda")
    xd = torch.zeros(op.n_A, dtype=torch.float64, device="cuda")
    im = gm.pcg(gm.rhs(_dev(d)), xm, Lm, tol=1e-6, maxit=3000)
    idd = gd.pcg(gd.rhs(_dev(d)), xd, Ld, tol=1e-6, maxit=3000)
    assert im["status"] == 0 and idd["status"] == 0
    res = np.linalg.norm(b - O.apply_A(op, xm.cpu().numpy())) / np.linalg.norm(b)
    print("[result] iters fp16 U", im["iters"], "fp64", idd["iters"], "true res", res, flush=True)
    assert res <= 1.05e-6
    assert im["iters"] <= 1.05 * idd["iters"] + 2
    with pytest.raises(Wc4dError) as e:
        Problem.from_workload(C1, obs_pattern(C1), prec=wc4d.PREC_LMP_FP32 | wc4d.PREC_LMP_FP16)
    assert e.value.code == -1


def test_fp16_copy_keeps_c_positive_definite():
    """The float16 copy is kept only while its Gram defect is at most half of theta_max^{-1/2}
    (C's smallest eigenvalue for an orthonormal U).  At C1 (theta_max ~ 5e3) the float16
    copy is used; with observation variance 1e-12 theta_max ~ 5e13 and the float16 rounding
    (Gram defect ~1e-5) would leave too little margin, so the build streams the float32 copy,
    whose C v still matches the oracle's to the float32 bound."""
    from paper_2101_07249_amd import wc4d
    w = C1
    gm, op = _pair(w, wc4d.PREC_LMP_FP16)
    G = sketch_block(op.n_A, w.m, w.seed)
    L = gm.lmp_build("nystrom", w.k_r, w.l, _dev(G))
    print("[result] C1 theta_max", L.theta()[0], "copy", L.copy_format(), flush=True)
    assert L.copy_format() == wc4d.PREC_LMP_FP16
    wx = w.with_(sigma_o2=1e-12)
    gx, opx = _pair(wx, wc4d.PREC_LMP_FP16)
    Lx = gx.lmp_build("nystrom", wx.k_r, wx.l, _dev(G))
    th = Lx.theta()
    print("[result] sigma_o2 1e-12 theta_max", th[0], "copy", Lx.copy_format(), flush=True)
    assert th[0] > 1e10
    assert Lx.copy_format() == wc4d.PREC_LMP_FP32
    Uo, tho = O.METHODS["nystrom"](lambda Z: O.apply_A(opx, Z), G, wx.k_r)
    V = random_block(opx.n_A, 1, 11)
    CV = Lx.apply(_dev(V)).cpu().numpy()
    CV = CV.T if CV.ndim == 2 else CV[:, None]
    CVo = O.lmp_apply(Uo, tho, V)
    e = float(col_errors(CV, CVo).max())
    print("[result] fallback C v rel err", e, flush=True)
    assert e <= 1e-5
    gd, _ = _pair(w, wc4d.PREC_FP64)
    assert gd.lmp_build("nystrom", w.k_r, w.l, _dev(G)).copy_format() == 0


# ---------------------------------------------------------------- split float16 x 3
# Three float16 products with float32 accumulation and power-of-two scaling (rows of S,
# columns of X): per part 11 significant bits, so the dropped Sl Xl term is ~2^-22 relative
# and the float32 sums over K = n add ~sqrt(n) 2^-24; the bound used is 1e-5 (the bfloat16
# form's is 1e-4), and the float16 form must be the more accurate of the two.
@pytest.mark.parametrize("kernel", ["auto", "frag"])
@pytest.mark.parametrize("w", [C1, C2, MEDIUM, MEDIUM_BQ], ids=["C1", "C2", "adv700", "adv700_LbLq"])
def test_fp16x3_apply_error(w, kernel, monkeypatch):
    from paper_2101_07249_amd import wc4d
    print("[case] fp16x3 apply", w.name, kernel, flush=True)
    if kernel != "auto":
        monkeypatch.setenv("WC4D_SPLIT_GEMM_KERNEL", kernel)
    gh, op = _pair(w, wc4d.PREC_SKETCH_FP16X3)
    gb, _ = _pair(w, wc4d.PREC_SKETCH_BF16X3)
    G = sketch_block(op.n_A, w.m, w.seed)
    Yo = O.apply_A(op, G)
    Yh = gh.apply_A_prec(_dev(G), wc4d.PREC_SKETCH_FP16X3).cpu().numpy().T
    Yb = gb.apply_A_prec(_dev(G), wc4d.PREC_SKETCH_BF16X3).cpu().numpy().T
    e_h = float(col_errors(Yh, Yo).max())
    e_b = float(col_errors(Yb, Yo).max())
    print("[result] rel err fp16x3", e_h, "bf16x3", e_b, flush=True)
    assert 1e-12 < e_h <= 1e-5
    assert e_h < e_b


@pytest.mark.parametrize("kernel", ["auto", "frag"])
def test_fp16x3_scaling_extremes_and_zero_column(kernel, monkeypatch):
    """Column exponents follow the data: blocks scaled by 1e-150 or 1e150 keep the same
    relative error, and an all-zero column maps to an all-zero column (both kernels)."""
    from paper_2101_07249_amd import wc4d
    w = MEDIUM
    print("[case] fp16x3 scaling", kernel, flush=True)
    if kernel != "auto":
        monkeypatch.setenv("WC4D_SPLIT_GEMM_KERNEL", kernel)
    gh, op = _pair(w, wc4d.PREC_SKETCH_FP16X3)
    G = sketch_block(op.n_A, 6, w.seed + 3)
    G[:, 2] = 0.0
    Yo = O.apply_A(op, G)
    for scale in (1e-150, 1.0, 1e150):
        Y = gh.apply_A_prec(_dev(G * scale), wc4d.PREC_SKETCH_FP16X3).cpu().numpy().T / scale
        e = float(col_errors(Y, Yo).max())
        print("[result] scale", scale, "rel err", e, flush=True)
        assert e <= 1e-5
        np.testing.assert_array_equal(Y[:, 2], 0.0)


def test_fp16x3_lmp_and_pcg():
    from paper_2101_07249_amd import wc4d
    import torch
    w = C2
    print("[case] fp16x3 lmp + pcg", flush=True)
    gm, op = _pair(w, wc4d.PREC_SKETCH_FP16X3 | wc4d.PREC_LMP_FP32)
    gd, _ = _pair(w, wc4d.PREC_FP64)
    G = sketch_block(op.n_A, w.m, w.seed)
    Lm = gm.lmp_build("nystrom", w.k_r, w.l, _dev(G))
    Ld = gd.lmp_build("nystrom", w.k_r, w.l, _dev(G))
    _, tho = O.METHODS["nystrom"](lambda Z: O.apply_A(op, Z), G, w.k_r)
    th = Lm.theta()
    e = float(np.abs(th - tho).max() / tho[0])   # Weyl: each |dtheta_i| against theta_1
    print("[result] theta err / theta_1", e, "per entry", float((np.abs(th - tho) / tho).max()), flush=True)
    assert e <= 1e-5
    d = innovations(op.q, w.seed, np.sqrt(w.sigma_o2))
    b = O.rhs(op, d)
    xm = torch.zeros(op.n_A, dtype=torch.float64, device="cuda")
    xd = torch.zeros(op.n_A, dtype=torch.float64, device="cuda")
    im = gm.pcg(gm.rhs(_dev(d)), xm, Lm, tol=1e-6, maxit=3000)
    idd = gd.pcg(gd.rhs(_dev(d)), xd, Ld, tol=1e-6, maxit=3000)
    assert im["status"] == 0 and idd["status"] == 0
    res = np.linalg.norm(b - O.apply_A(op, xm.cpu().numpy())) / np.linalg.norm(b)
    print("[result] iters fp16x3", im["iters"], "fp64", idd["iters"], "true res", res, flush=True)
    assert res <= 1.05e-6
    assert im["iters"] <= 1.05 * idd["iters"] + 2


def test_fp16x3_flag_errors():
    from paper_2101_07249_amd import Problem, Wc4dError, wc4d
    w = C1
    pat = obs_pattern(w)
    with pytest.raises(Wc4dError) as e:
        Problem.from_workload(w, pat, prec=wc4d.PREC_SKETCH_FP16X3 | wc4d.PREC_SKETCH_BF16X3)
    assert e.value.code == -1
    gb = Problem.from_workload(w, pat, prec=wc4d.PREC_SKETCH_BF16X3)
    G = sketch_block(gb.n_A, 3, 5)
    with pytest.raises(Wc4dError) as e:
        gb.apply_A_prec(_dev(G), wc4d.PREC_SKETCH_FP16X3)
    assert e.value.code == -7


def test_fp16x3_full_size_sampled_columns():
    from paper_2101_07249_amd import wc4d
    print("[case] fp16x3 full size", flush=True)
    pat = obs_pattern(C3)
    from paper_2101_07249_amd import Problem
    gp = Problem.from_workload(C3, pat, prec=wc4d.PREC_SKETCH_FP16X3 | wc4d.PREC_LMP_FP32)
    op = O.make_problem(C3, pat)
    G = sketch_block(gp.n_A, C3.m, C3.seed)
    Y = gp.apply_A_prec(_dev(G), wc4d.PREC_SKETCH_FP16X3)
    cols = [0, 3, 200, 255]  # the first and last 256-column tiles of the all-level product too
    Yo = O.apply_A(op, G[:, cols])
    e = float(col_errors(Y[cols].cpu().numpy().T, Yo).max())
    print("[result] full-size fp16x3 rel err", e, flush=True)
    assert 1e-12 < e <= 1e-5


@pytest.mark.parametrize("form", ["bf16x3", "fp16x3"])
def test_split_kernels_give_the_same_bits(form, monkeypatch):
    """The LDS-tiled and the fragment-major kernels form the same three products in the
    same K order, so the block apply is bit-identical whichever one runs (ragged shape:
    n = K = 700, 1240 columns)."""
    from paper_2101_07249_amd import wc4d
    prec = wc4d.PREC_SKETCH_BF16X3 if form == "bf16x3" else wc4d.PREC_SKETCH_FP16X3
    print("[case] tiled vs fragment-major", form, flush=True)
    gp, op = _pair(MEDIUM, prec)
    G = _dev(sketch_block(op.n_A, MEDIUM.m, MEDIUM.seed + 7))
    out = {}
    for kernel in ("tiled", "frag"):
        monkeypatch.setenv("WC4D_SPLIT_GEMM_KERNEL", kernel)
        out[kernel] = gp.apply_A_prec(G, prec).cpu().numpy()
    np.testing.assert_array_equal(out["tiled"], out["frag"])
