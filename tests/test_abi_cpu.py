"""CPU checks of the C-ABI library: it loads, exports every symbol the header
declares, and its host-only setup helpers agree with the oracle's independent
routes.  No device compute."""
import os
import re

import numpy as np
import pytest

from oracle import wc4d_oracle as O
from synthetic import l96_initial_state

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "wc4d.h")


def header_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(wc4d_[A-Za-z0-9_]+)\s*\(", txt)))


def test_header_declares_entry_points():
    names = header_functions()
    for must in ("wc4d_create", "wc4d_apply_A", "wc4d_lmp_build", "wc4d_pcg", "wc4d_rhs"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2101_07249_amd import wc4d
    L = wc4d.lib()
    for name in header_functions():
        assert hasattr(L, name), name
    # and the binding knows every one of them
    assert set(header_functions()) <= set(wc4d.exported_symbols())
    assert L.wc4d_version() >= 100
    assert L.wc4d_status_string(-4) == b"WC4D_ENOTSPD"


@pytest.mark.parametrize("n,kind,L,sig", [(40, "soar", 4.0, 1.0), (41, "soar", 4.0, 0.1), (80, "gauss", 2.0, 0.2),
                                          (1, "soar", 4.0, 1.0), (2, "gauss", 2.0, 1.0)])
def test_corr_sqrt_helper_matches_oracle(n, kind, L, sig):
    from paper_2101_07249_amd import corr_sqrt
    S = corr_sqrt(n, kind, L, sig)
    So = O.cov_sqrt(n, kind, L, sig)
    tol = 1e-12 if kind == "soar" else 1e-11
    assert np.abs(S - So).max() <= tol * max(1.0, np.abs(So).max())


def test_l96_trajectory_helper_matches_oracle():
    from paper_2101_07249_amd import l96_trajectory
    x0 = l96_initial_state(80, 2000)
    t = l96_trajectory(x0, 8.0, 0.025, 50)
    to = O.l96_trajectory(x0, 8.0, 0.025, 50)
    assert np.abs(t - to).max() <= 1e-12 * np.abs(to).max()


def test_corr_sqrt_rejects_bad_arguments():
    from paper_2101_07249_amd import wc4d
    out = np.empty((4, 4))
    assert wc4d.lib().wc4d_corr_sqrt(4, 7, 1.0, 1.0, out.ctypes.data_as(wc4d._c_dbl_p)) == wc4d.EINVAL
    assert wc4d.lib().wc4d_corr_sqrt(4, 0, -1.0, 1.0, out.ctypes.data_as(wc4d._c_dbl_p)) == wc4d.EINVAL


def test_autotune_cache_file_roundtrip(tmp_path):
    """The autotune cache is host-side text: loading validates every line, saving writes
    what was merged (no GPU call involved)."""
    from paper_2101_07249_amd import wc4d as W4
    good = tmp_path / "good.txt"
    good.write_text("# comment\n0 4096 100 1 0 1 2 1 1 8 0 0.116\n0 512 10 64 1 0 0 0 0 0 3 1.5\n")
    W4.autotune_load(str(good))
    out = tmp_path / "out.txt"
    W4.autotune_save(str(out))
    lines = [l.split() for l in out.read_text().splitlines() if not l.startswith("#")]
    assert ["0", "4096", "100", "1", "0", "1", "2", "1", "1", "8", "0"] in [l[:11] for l in lines]
    assert ["0", "512", "10", "64", "1", "0", "0", "0", "0", "0", "3"] in [l[:11] for l in lines]
    bad = tmp_path / "bad.txt"
    for text in ("0 4096 100 1 0 9 2 1 1 8 0 0.1\n", "0 4096 100 1 0 1 2 1 7 8 0 0.1\n", "0 4096 100\n",
                 "0 4096 100 1 0 1 2 1 1 8 3 0.1\n"):
        bad.write_text(text)
        with pytest.raises(W4.Wc4dError):
            W4.autotune_load(str(bad))
    with pytest.raises(W4.Wc4dError):
        W4.autotune_load(str(tmp_path / "missing.txt"))


def test_bench_helpers_on_cpu():
    """bench.py's host-side helpers: kernel naming from a tuned form, and the counter
    traffic only for the measured kernels (sources hashed)."""
    import bench
    from synthetic import C3
    assert bench.FP64_PEAK_TFLOPS == 78.6 and bench.BF16_PEAK_TFLOPS == 2500.0 and bench.HBM_PEAK_GBS == 8000.0
    tune = {"tile_b": 2, "tile_q": 0, "single_product": True, "two_segment": True, "segment_variant": 1,
            "segment_splits": 8}
    name = bench.dsqrt_kernel_name(tune)
    assert "k_dsqrt2<128, 16>" in name and "level 0" in name
    assert "k_gemm_f64" in bench.dsqrt_kernel_name(dict(tune, two_segment=False))
    t = bench.MEASURED_TRAFFIC
    other = dict(tune, segment_splits=(t["tune"].get("segment_splits") or 0) + 1)
    assert bench.measured_traffic(C3, other) is None
    assert bench.measured_traffic(C3.with_(n=512), tune) is None


def test_committed_tuning_table_loads():
    """The MI355X tile table shipped with the package (the benchmark's default tile
    source) parses line by line with the library's own validating loader, and saving
    writes back every tile choice it holds."""
    import bench
    from paper_2101_07249_amd import wc4d as W4
    W4.autotune_load(bench.TUNING_TABLE)
    rows = [l.split()[:11] for l in open(bench.TUNING_TABLE) if l.strip() and not l.startswith("#")]
    assert rows
    import tempfile
    with tempfile.TemporaryDirectory() as d:
        out = os.path.join(d, "saved.txt")
        W4.autotune_save(out)
        saved = [l.split()[:11] for l in open(out) if not l.startswith("#")]
    for r in rows:
        assert r in saved, r


def test_bench_refuses_more_than_one_gpu():
    """The benchmark measures one GPU; asking for more exits with a message and status 2
    before any device work."""
    import json
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in json.loads(r.stdout.strip().splitlines()[-1])["error"]


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    """Without the built HIP library the binding raises; there is no fallback path."""
    from paper_2101_07249_amd import wc4d as W4
    monkeypatch.setattr(W4, "_lib", None)
    monkeypatch.setattr(W4, "LIB_PATH", str(tmp_path / "libwc4d.so"))
    with pytest.raises(ImportError, match="no fallback"):
        W4.lib()


def test_oracle_and_library_share_no_code():
    """The oracle imports nothing from the library package, the package never imports the
    oracle, and the seeded input module imports neither."""
    import ast
    import glob

    def imported(path):
        tree = ast.parse(open(path).read())
        mods = set()
        for node in ast.walk(tree):
            if isinstance(node, ast.Import):
                mods.update(a.name.split(".")[0] for a in node.names)
            elif isinstance(node, ast.ImportFrom) and node.module and node.level == 0:
                mods.add(node.module.split(".")[0])
        return mods

    for path in glob.glob(os.path.join(ROOT, "oracle", "*.py")):
        assert not imported(path) & {"paper_2101_07249_amd", "synthetic"}, path
        assert "libwc4d" not in open(path).read(), path
    for path in glob.glob(os.path.join(ROOT, "paper_2101_07249_amd", "*.py")):
        assert "oracle" not in imported(path), path
    for path in glob.glob(os.path.join(ROOT, "synthetic", "*.py")):
        assert not imported(path) & {"oracle", "paper_2101_07249_amd"}, path
    for path in glob.glob(os.path.join(ROOT, "paper_2101_07249_amd", "csrc", "*")):
        assert "oracle" not in open(path).read(), path



def test_profile_commands_run_committed_files_with_known_flags():
    """Every command recorded in profiles/ runs a file of the repository (never a scratch
    script) and passes bench.py only options its --help lists."""
    import glob
    import re
    import shlex
    import subprocess
    import sys
    helptext = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--help"],
                              capture_output=True, text=True, timeout=300).stdout
    opts = set(re.findall(r"(--[a-z0-9-]+)", helptext))
    assert "--steps" in opts and "--copy-probe" in opts
    cmds = [l.strip() for p in glob.glob(os.path.join(ROOT, "profiles", "*.md"))
            for l in open(p) if l.startswith("    ") and ("python" in l or "rocprofv3" in l)]
    assert cmds
    for c in cmds:
        toks = shlex.split(c.replace("<out>", "OUT"))
        paths = [t for t in toks if t.startswith("/root/repo/")]
        assert paths, c
        for t in paths:
            rel = os.path.relpath(t, "/root/repo")
            assert not rel.startswith("_work") and os.path.exists(os.path.join(ROOT, rel)), c
        for t in toks[toks.index(paths[0]) + 1:]:
            if t.startswith("--"):
                assert t in opts, (t, c)


def _stub_problem(n_A=12, q=3):
    """A Problem object with sizes but no library handle: the binding's size checks run
    before any library call, so they can be exercised without a GPU."""
    from paper_2101_07249_amd.wc4d import Problem
    p = object.__new__(Problem)
    p._h = None
    p.n, p.N, p.device, p.n_A, p.q = 4, 2, 0, n_A, q
    return p


def test_binding_checks_sizes_before_any_launch():
    """The C-ABI takes bare device pointers, so a short tensor would be read or written out
    of bounds inside a kernel; the binding must raise ValueError first."""
    import torch
    from paper_2101_07249_amd import wc4d
    p = _stub_problem()
    ok_vec, short = torch.zeros(12, dtype=torch.float64), torch.zeros(11, dtype=torch.float64)
    with pytest.raises(ValueError):
        p.pcg(short, ok_vec)
    with pytest.raises(ValueError):
        p.pcg(ok_vec, short)
    with pytest.raises(ValueError):
        p.rhs(torch.zeros(2, dtype=torch.float64))                     # d needs q = 3
    with pytest.raises(ValueError):
        p.rhs(torch.zeros(3, dtype=torch.float64), bt=short)
    with pytest.raises(ValueError):
        p.rhs(torch.zeros(3, dtype=torch.float64), out=short)
    with pytest.raises(ValueError):
        p.lmp_build("revd", 3, 2, torch.zeros((4, 12), dtype=torch.float64))   # needs (5, 12)
    with pytest.raises(ValueError):
        p.lmp_build_sketch(None, "nystrom", 59, 5, torch.zeros((64, 11), dtype=torch.float64))
    with pytest.raises(ValueError):
        p.apply_A(torch.zeros((2, 11), dtype=torch.float64))
    with pytest.raises(ValueError):
        p.apply_A(torch.zeros((2, 12), dtype=torch.float64), torch.zeros((1, 12), dtype=torch.float64))
    with pytest.raises(ValueError):
        p.apply_A_prec(torch.zeros((2, 12), dtype=torch.float64), wc4d.PREC_FP64,
                       torch.zeros((2, 11), dtype=torch.float64))
    with pytest.raises(ValueError):
        p.apply_Linv(torch.zeros((1, 2, 12), dtype=torch.float64))
    with pytest.raises(ValueError):
        p.sketch_loss(torch.zeros((4, 12), dtype=torch.float64), torch.zeros((2, 12), dtype=torch.float64),
                      torch.zeros(3, dtype=torch.float64))                 # theta needs k = 2
    L = wc4d.Lmp(None, p, 3)
    with pytest.raises(ValueError):
        L.apply(torch.zeros((2, 13), dtype=torch.float64))
    with pytest.raises(ValueError):
        wc4d.batch_solve([p], "revd", 3, 2, [torch.zeros((5, 12), dtype=torch.float64)], [short], [ok_vec])
    with pytest.raises(ValueError):
        wc4d.batch_solve([p], "revd", 3, 2, [torch.zeros((5, 12), dtype=torch.float64)], [ok_vec], [])
    # right sizes on the host: the device check fires instead (nothing reaches the library)
    with pytest.raises(TypeError):
        p.pcg(ok_vec, ok_vec)
    L._h = None
