"""Thin Python binding of libwc4d (include/wc4d.h): argument marshalling only.

Every step of the operator, the randomised eigendecompositions, the LMP and PCG
runs in the HIP library.  torch is used for device memory (tensors' data
pointers) and streams.  A block of m vectors of length n_A is a float64 CUDA
tensor of shape (m, n_A), contiguous: row c is vector c, i.e. the column-major
n_A x m array with leading dimension n_A that the C-ABI expects.

There is no fallback: if the library is missing or a call fails, an exception
is raised.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libwc4d.so")

OK, EINVAL, ENOMEM, EHIP, ENOTSPD, EBREAKDOWN, ENOCONV, ESTATE = 0, -1, -2, -3, -4, -5, -6, -7
CORR_SOAR, CORR_GAUSS = 0, 1
REVD, NYSTROM, RITZIT, NYSTROM_1P = 0, 1, 2, 3
METHOD = {"revd": REVD, "nystrom": NYSTROM, "ritzit": RITZIT, "nystrom1p": NYSTROM_1P}
RES_TRUE, RES_PRECOND = 0, 1
PCG_FUSED, PCG_PLAIN = 0, 1
PREC_FP64, PREC_SKETCH_BF16X3, PREC_LMP_FP32, PREC_SKETCH_FP16X3, PREC_LMP_FP16 = 0, 1, 2, 4, 8
PREC_DSQRT_OZ7 = 16
BATCH_SWEEP_FP32 = 1
LANCZOS_REORTH = 1

_c_int_p = ctypes.POINTER(ctypes.c_int)
_c_dbl_p = ctypes.POINTER(ctypes.c_double)
_c_flt_p = ctypes.POINTER(ctypes.c_float)
_vp = ctypes.c_void_p


class PcgOpts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("maxit", ctypes.c_int), ("criterion", ctypes.c_int),
                ("variant", ctypes.c_int)]


class PcgInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("status", ctypes.c_int), ("relres_true", ctypes.c_double),
                ("relres_precond", ctypes.c_double), ("J", ctypes.c_double)]


# name -> (restype, argtypes)
_SIGS = {
    "wc4d_version": (ctypes.c_int, []),
    "wc4d_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "wc4d_create": (ctypes.c_int, [ctypes.POINTER(_vp), ctypes.c_int, ctypes.c_int, ctypes.c_int]),
    "wc4d_destroy": (ctypes.c_int, [_vp]),
    "wc4d_last_error": (ctypes.c_char_p, [_vp]),
    "wc4d_set_model_advdiff": (ctypes.c_int, [_vp, ctypes.c_double, ctypes.c_double]),
    "wc4d_set_model_l96": (ctypes.c_int, [_vp, _c_dbl_p, ctypes.c_double, ctypes.c_double]),
    "wc4d_l96_trajectory": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                           _c_dbl_p, _c_dbl_p]),
    "wc4d_corr_sqrt": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double, _c_dbl_p]),
    "wc4d_set_Bsqrt": (ctypes.c_int, [_vp, _c_dbl_p]),
    "wc4d_set_Qsqrt": (ctypes.c_int, [_vp, _c_dbl_p]),
    "wc4d_set_obs": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, _c_int_p, _c_dbl_p]),
    "wc4d_set_strong_constraint": (ctypes.c_int, [_vp, ctypes.c_int]),
    "wc4d_finalize": (ctypes.c_int, [_vp, ctypes.c_int, _vp]),
    "wc4d_dims": (ctypes.c_int, [_vp, _c_int_p, _c_int_p]),
    "wc4d_apply_A": (ctypes.c_int, [_vp, _vp, ctypes.c_int, _vp, ctypes.c_int, ctypes.c_int, _vp]),
    "wc4d_apply_A_prec": (ctypes.c_int, [_vp, _vp, ctypes.c_int, _vp, ctypes.c_int, ctypes.c_int,
                                         ctypes.c_int, _vp]),
    "wc4d_apply_Linv": (ctypes.c_int, [_vp, _vp, ctypes.c_int, _vp, ctypes.c_int, ctypes.c_int, _vp]),
    "wc4d_apply_LinvT": (ctypes.c_int, [_vp, _vp, ctypes.c_int, _vp, ctypes.c_int, ctypes.c_int, _vp]),
    "wc4d_apply_Dsqrt": (ctypes.c_int, [_vp, _vp, ctypes.c_int, _vp, ctypes.c_int, ctypes.c_int, _vp]),
    "wc4d_rhs": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp]),
    "wc4d_lmp_build": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, _vp, ctypes.c_ulonglong,
                                      ctypes.POINTER(_vp), _vp]),
    "wc4d_gaussian_block": (ctypes.c_int, [ctypes.c_int, ctypes.c_ulonglong, ctypes.c_longlong, ctypes.c_int,
                                           ctypes.c_longlong, _vp, ctypes.c_longlong, _vp]),
    "wc4d_philox4x32_10": (ctypes.c_int, [ctypes.c_int, _vp, _vp, ctypes.c_longlong, _vp]),
    "wc4d_lmp_theta": (ctypes.c_int, [_vp, _c_dbl_p]),
    "wc4d_lmp_vectors": (ctypes.c_int, [_vp, _vp, ctypes.c_int, _vp]),
    "wc4d_lmp_apply": (ctypes.c_int, [_vp, _vp, ctypes.c_int, _vp, ctypes.c_int, ctypes.c_int, _vp]),
    "wc4d_lmp_apply_noalloc": (ctypes.c_int, [_vp, _vp, ctypes.c_int, _vp, ctypes.c_int, ctypes.c_int, _vp]),
    "wc4d_lmp_applies": (ctypes.c_int, [_vp, _c_int_p]),
    "wc4d_lmp_copy_format": (ctypes.c_int, [_vp, _c_int_p]),
    "wc4d_lmp_destroy": (ctypes.c_int, [_vp]),
    "wc4d_pcg": (ctypes.c_int, [_vp, _vp, _vp, _vp, ctypes.POINTER(PcgOpts), ctypes.POINTER(PcgInfo),
                                _c_dbl_p, _c_dbl_p, _c_dbl_p, _vp]),
    "wc4d_lmp_ritz_prepare": (ctypes.c_int, [_vp, _vp]),
    "wc4d_lmp_ritz_apply": (ctypes.c_int, [_vp, _vp, ctypes.c_int, _vp, ctypes.c_int, ctypes.c_int, _vp]),
    "wc4d_pcg_ritz": (ctypes.c_int, [_vp, _vp, _vp, _vp, ctypes.POINTER(PcgOpts), ctypes.POINTER(PcgInfo), _c_dbl_p,
                                     _c_dbl_p, _vp]),
    "wc4d_pcg_lanczos": (ctypes.c_int, [_vp, _vp, _vp, ctypes.POINTER(PcgOpts), ctypes.POINTER(PcgInfo), _c_dbl_p,
                                        _c_dbl_p, _vp, ctypes.c_longlong, ctypes.c_int, _vp]),
    "wc4d_lanczos_pairs": (ctypes.c_int, [_vp, ctypes.c_int, _c_dbl_p, _c_dbl_p, _vp, ctypes.c_longlong, ctypes.c_int,
                                          _vp, ctypes.c_longlong, _c_dbl_p, _vp]),
    "wc4d_lmp_from_pairs": (ctypes.c_int, [_vp, ctypes.c_int, _vp, ctypes.c_longlong, _c_dbl_p, ctypes.POINTER(_vp),
                                           _vp]),
    "wc4d_l96_trajectory_forced": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                                  _c_dbl_p, _c_dbl_p, _c_dbl_p]),
    "wc4d_set_profiling": (ctypes.c_int, [_vp, ctypes.c_int]),
    "wc4d_prof_stride": (ctypes.c_int, [_vp, ctypes.c_int]),
    "wc4d_prof_enable": (ctypes.c_int, [_vp, ctypes.c_int]),
    "wc4d_prof_read": (ctypes.c_int, [_vp, ctypes.c_int, _c_dbl_p, ctypes.POINTER(ctypes.c_longlong),
                                      _c_dbl_p, _c_dbl_p]),
    "wc4d_last_apply_timing": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_float)]),
    "wc4d_autotune": (ctypes.c_int, [_vp, ctypes.c_int, _vp]),
    "wc4d_autotune_info": (ctypes.c_int, [_vp, ctypes.c_int, _c_int_p, _c_int_p, _c_int_p,
                                          ctypes.POINTER(ctypes.c_float)]),
    "wc4d_autotune_save": (ctypes.c_int, [ctypes.c_char_p]),
    "wc4d_autotune_load": (ctypes.c_int, [ctypes.c_char_p]),
    "wc4d_batch_solve": (ctypes.c_int, [ctypes.POINTER(_vp), ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                        ctypes.c_int, ctypes.POINTER(_vp), ctypes.POINTER(_vp),
                                        ctypes.POINTER(_vp), ctypes.POINTER(PcgOpts), ctypes.POINTER(PcgInfo),
                                        _c_int_p, ctypes.c_int, ctypes.c_int]),
    "wc4d_batch_solve_persistent": (ctypes.c_int, [ctypes.POINTER(_vp), ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                                   ctypes.c_int, ctypes.POINTER(_vp), ctypes.c_ulonglong,
                                                   ctypes.POINTER(_vp), ctypes.POINTER(_vp), ctypes.POINTER(PcgOpts),
                                                   ctypes.c_int, ctypes.POINTER(PcgInfo), _c_int_p, _c_dbl_p]),
    "wc4d_batch_persistent_profile": (ctypes.c_int, [_c_dbl_p, ctypes.POINTER(ctypes.c_longlong), ctypes.c_int]),
    "wc4d_sketchnet_create": (ctypes.c_int, [ctypes.POINTER(_vp), ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                             ctypes.c_int, ctypes.c_int]),
    "wc4d_sketchnet_destroy": (ctypes.c_int, [_vp]),
    "wc4d_sketchnet_last_error": (ctypes.c_char_p, [_vp]),
    "wc4d_sketchnet_nparams": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_longlong)]),
    "wc4d_sketchnet_set_params": (ctypes.c_int, [_vp, _c_flt_p]),
    "wc4d_sketchnet_get_params": (ctypes.c_int, [_vp, _c_flt_p]),
    "wc4d_sketchnet_get_grad": (ctypes.c_int, [_vp, _c_flt_p]),
    "wc4d_sketchnet_set_grad": (ctypes.c_int, [_vp, _c_flt_p]),
    "wc4d_sketchnet_infer": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int, _vp, ctypes.c_int, _vp]),
    "wc4d_sketchnet_backward": (ctypes.c_int, [_vp, _vp, ctypes.c_int, _vp]),
    "wc4d_sketchnet_adam": (ctypes.c_int, [_vp, ctypes.c_double, _vp]),
    "wc4d_sketch_loss": (ctypes.c_int, [_vp, _vp, ctypes.c_int, ctypes.c_int, _vp, ctypes.c_int, _vp,
                                        ctypes.c_int, _vp, _vp, ctypes.c_int, _vp]),
    "wc4d_sketchnet_train_step": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int, _vp, ctypes.c_int,
                                                 ctypes.c_double, _c_dbl_p, _vp]),
    "wc4d_lmp_build_sketch": (ctypes.c_int, [_vp, _vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, _vp,
                                             ctypes.POINTER(_vp), _c_int_p, _vp]),
    "wc4d_sketchnet_save": (ctypes.c_int, [_vp, ctypes.c_char_p]),
    "wc4d_sketchnet_load": (ctypes.c_int, [ctypes.POINTER(_vp), ctypes.c_char_p, ctypes.c_int]),
}

_lib = None


class Wc4dError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_status_name(code)}: {msg}")
        self.code = code


def _status_name(code: int) -> str:
    names = {0: "WC4D_OK", -1: "WC4D_EINVAL", -2: "WC4D_ENOMEM", -3: "WC4D_EHIP", -4: "WC4D_ENOTSPD",
             -5: "WC4D_EBREAKDOWN", -6: "WC4D_ENOCONV", -7: "WC4D_ESTATE"}
    return names.get(code, f"status {code}")


def lib() -> ctypes.CDLL:
    """Load libwc4d.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        # torch first: the library then binds to the HIP runtime torch has loaded, so
        # both share one runtime (and torch's device memory and streams are valid in it)
        import torch  # noqa: F401
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_2101_07249_amd/build.py "
                              "(there is no fallback implementation)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def exported_symbols() -> Sequence[str]:
    return list(_SIGS)


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(_c_dbl_p)


def _stream(stream) -> Optional[int]:
    if stream is not None:
        return int(stream)
    import torch
    return torch.cuda.current_stream().cuda_stream


def _check_size(t, shape, what: str):
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{what}: expected a torch tensor")
    if isinstance(shape, int):
        if t.numel() != shape:
            raise ValueError(f"{what}: expected {shape} elements, got {t.numel()}")
    elif shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{what}: expected shape {tuple(shape)}, got {tuple(t.shape)}")


def _tptr(t, shape=None, what: str = "tensor", dtype=None) -> int:
    """Data pointer of a contiguous CUDA tensor (float64 unless dtype is given).  With
    `shape`, the tensor must have exactly that shape (a tuple) or that many elements (an
    int): the C-ABI takes bare pointers, so every size is checked here, before a launch."""
    import torch
    want = torch.float64 if dtype is None else dtype
    _check_size(t, shape, what)
    if not (t.is_cuda and t.dtype == want and t.is_contiguous()):
        raise TypeError(f"{what}: expected a contiguous {want} CUDA tensor")
    return t.data_ptr()


def _ptrs(*items):
    """Data pointers of several tensors, (tensor, shape, what) each: every size is
    checked before any tensor's device or layout, so a wrongly sized argument is reported
    as such wherever it lives."""
    for t, shape, what in items:
        _check_size(t, shape, what)
    return [_tptr(t, shape, what) for t, shape, what in items]


def _block_rows(X, n_A: int, what: str):
    """(m, view) of a block of vectors: a 1-D tensor of n_A elements (m = 1) or an
    (m, n_A) tensor."""
    if X.dim() == 1:
        X2 = X.view(1, -1)
    elif X.dim() == 2:
        X2 = X
    else:
        raise ValueError(f"{what}: a block is a 1-D or 2-D tensor")
    if X2.shape[-1] != n_A or X2.shape[0] < 1:
        raise ValueError(f"{what}: block rows must have n_A = {n_A} entries, got shape {tuple(X.shape)}")
    return X2.shape[0], X2


def gaussian_block(seed: int, n_rows: int, n_cols: int, col0: int = 0, out=None, device: int = 0,
                   stream=None):
    """The Gaussian start block of `seed` drawn on the device (wc4d_gaussian_block): an
    (n_cols, n_rows) float64 tensor whose row c is column col0 + c of the block."""
    import torch
    if out is None:
        out = torch.empty((n_cols, n_rows), dtype=torch.float64, device=torch.device("cuda", device))
    ptr = _tptr(out, (n_cols, n_rows), "gaussian_block out")
    rc = lib().wc4d_gaussian_block(int(device), ctypes.c_ulonglong(int(seed) & 0xFFFFFFFFFFFFFFFF),
                                   int(n_rows), int(n_cols), int(col0), ptr, max(int(n_rows), 1), _stream(stream))
    if rc:
        raise Wc4dError(rc, "wc4d_gaussian_block")
    return out


def philox4x32_10(ctr_key, device: int = 0, stream=None):
    """Raw Philox-4x32-10 words of (count, 6) uint32 rows (c0 c1 c2 c3 k0 k1) on the device
    (wc4d_philox4x32_10); returns a (count, 4) int32 tensor holding the words' bits."""
    import torch
    t = ctr_key
    if t.dim() != 2 or t.shape[1] != 6:
        raise ValueError("ctr_key must be (count, 6)")
    out = torch.empty((t.shape[0], 4), dtype=torch.int32, device=t.device)
    rc = lib().wc4d_philox4x32_10(int(device), _tptr(t, what="ctr_key", dtype=torch.int32),
                                  _tptr(out, what="out", dtype=torch.int32), int(t.shape[0]), _stream(stream))
    if rc:
        raise Wc4dError(rc, "wc4d_philox4x32_10")
    return out


def corr_sqrt(n: int, kind: str, L: float, sigma: float) -> np.ndarray:
    """sigma * C^{1/2} (host helper of the library), as an (n, n) array."""
    out = np.empty((n, n), order="F")
    k = CORR_SOAR if kind == "soar" else CORR_GAUSS
    rc = lib().wc4d_corr_sqrt(n, k, float(L), float(sigma), _dptr(out))
    if rc:
        raise Wc4dError(rc, "wc4d_corr_sqrt")
    return out


def l96_trajectory(x0: np.ndarray, F: float, dt: float, N: int, eta: Optional[np.ndarray] = None) -> np.ndarray:
    """The Lorenz-96 RK4 trajectory from x0 ((N+1, n)), with model error eta ((N, n), row i
    added after step i) when given."""
    x0 = np.ascontiguousarray(x0, dtype=np.float64)
    n = x0.shape[0]
    out = np.empty((N + 1, n))
    if eta is None:
        rc = lib().wc4d_l96_trajectory(n, N, float(F), float(dt), _dptr(x0), _dptr(out))
    else:
        e = np.ascontiguousarray(eta, dtype=np.float64)
        if e.shape != (N, n):
            raise ValueError("eta must be (N, n)")
        rc = lib().wc4d_l96_trajectory_forced(n, N, float(F), float(dt), _dptr(x0), _dptr(e), _dptr(out))
    if rc:
        raise Wc4dError(rc, "wc4d_l96_trajectory")
    return out


class Lmp:
    def __init__(self, handle: int, prob: "Problem", k: int):
        self._h = handle
        self.prob = prob
        self.k = k

    def theta(self) -> np.ndarray:
        out = np.empty(self.k)
        rc = lib().wc4d_lmp_theta(self._h, _dptr(out))
        if rc:
            raise Wc4dError(rc, "lmp_theta")
        return out

    def vectors(self, stream=None):
        import torch
        U = torch.empty((self.k, self.prob.n_A), dtype=torch.float64, device=self.prob.torch_device)
        self.prob._chk(lib().wc4d_lmp_vectors(self._h, _tptr(U), self.prob.n_A, _stream(stream)), "lmp_vectors")
        return U

    def apply(self, X, Y=None, stream=None):
        import torch
        m, X2 = _block_rows(X, self.prob.n_A, "lmp_apply X")
        if Y is None:
            Y = torch.empty_like(X)
        xp, yp = _ptrs((X2, None, "lmp_apply X"), (Y, tuple(X.shape), "lmp_apply Y"))
        self.prob._chk(lib().wc4d_lmp_apply(self._h, xp, self.prob.n_A, yp, self.prob.n_A, m, _stream(stream)),
                       "lmp_apply")
        return Y

    def ritz_prepare(self, stream=None):
        """Compute and keep A U for the Ritz-LMP (one block product with A)."""
        self.prob._chk(lib().wc4d_lmp_ritz_prepare(self._h, _stream(stream)), "lmp_ritz_prepare")
        return self

    def ritz_apply(self, X, Y=None, stream=None):
        """Y = P X with the Ritz-LMP of eq. Ritz_LMP (after ritz_prepare)."""
        import torch
        m, X2 = _block_rows(X, self.prob.n_A, "lmp_ritz_apply X")
        if Y is None:
            Y = torch.empty_like(X)
        xp, yp = _ptrs((X2, None, "lmp_ritz_apply X"), (Y, tuple(X.shape), "lmp_ritz_apply Y"))
        self.prob._chk(lib().wc4d_lmp_ritz_apply(self._h, xp, self.prob.n_A, yp, self.prob.n_A, m,
                                                 _stream(stream)), "lmp_ritz_apply")
        return Y

    def apply_noalloc(self, X, Y, stream=None):
        """Y = C X (one or two vectors) through wc4d_lmp_apply_noalloc: no device allocation;
        Y must be given."""
        m, X2 = _block_rows(X, self.prob.n_A, "lmp_apply_noalloc X")
        xp, yp = _ptrs((X2, None, "lmp_apply_noalloc X"), (Y, tuple(X.shape), "lmp_apply_noalloc Y"))
        self.prob._chk(lib().wc4d_lmp_apply_noalloc(self._h, xp, self.prob.n_A, yp, self.prob.n_A, m,
                                                    _stream(stream)), "lmp_apply_noalloc")
        return Y

    @property
    def applies(self) -> int:
        c = ctypes.c_int(0)
        lib().wc4d_lmp_applies(self._h, ctypes.byref(c))
        return c.value

    def copy_format(self) -> int:
        """PREC_LMP_FP16, PREC_LMP_FP32 or 0: the copy of U the passes stream."""
        c = ctypes.c_int(0)
        rc = lib().wc4d_lmp_copy_format(self._h, ctypes.byref(c))
        if rc:
            raise Wc4dError(rc, "lmp_copy_format")
        return c.value

    def close(self):
        if self._h:
            lib().wc4d_lmp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Problem:
    """Handle of one inner-loop problem on one GPU."""

    def __init__(self, n: int, N: int, device: int = 0, strong: bool = False):
        h = _vp()
        rc = lib().wc4d_create(ctypes.byref(h), int(n), int(N), int(device))
        if rc:
            raise Wc4dError(rc, "wc4d_create")
        self._h = h.value
        self.n, self.N, self.device = int(n), int(N), int(device)
        self.strong = bool(strong)
        if self.strong:
            self._chk(lib().wc4d_set_strong_constraint(self._h, 1), "set_strong_constraint")
        # the control vector: (x_0, eta_1..eta_N), or x_0 alone for a strong-constraint problem
        self.n_A = self.n if self.strong else self.n * (self.N + 1)
        self.q = 0

    @property
    def torch_device(self):
        import torch
        return torch.device("cuda", self.device)

    def _chk(self, rc: int, what: str):
        if rc != OK:
            msg = lib().wc4d_last_error(self._h) if self._h else b""
            raise Wc4dError(rc, f"{what}: {msg.decode() if msg else ''}")

    # ---- setup
    def set_model_advdiff(self, c: float, r: float):
        self._chk(lib().wc4d_set_model_advdiff(self._h, float(c), float(r)), "set_model_advdiff")

    def set_model_l96(self, traj: np.ndarray, F: float, dt: float):
        t = np.ascontiguousarray(traj, dtype=np.float64)
        if t.shape != (self.N + 1, self.n):
            raise ValueError("trajectory must be (N+1, n)")
        self._chk(lib().wc4d_set_model_l96(self._h, _dptr(t), float(F), float(dt)), "set_model_l96")

    def set_Bsqrt(self, B: np.ndarray):
        b = np.asfortranarray(B, dtype=np.float64)
        self._chk(lib().wc4d_set_Bsqrt(self._h, _dptr(b)), "set_Bsqrt")

    def set_Qsqrt(self, Q: np.ndarray):
        q = np.asfortranarray(Q, dtype=np.float64)
        self._chk(lib().wc4d_set_Qsqrt(self._h, _dptr(q)), "set_Qsqrt")

    def set_obs(self, i: int, idx: np.ndarray, rdiag: np.ndarray):
        ix = np.ascontiguousarray(idx, dtype=np.int32)
        rd = np.ascontiguousarray(rdiag, dtype=np.float64)
        self._chk(lib().wc4d_set_obs(self._h, int(i), int(ix.size), ix.ctypes.data_as(_c_int_p), _dptr(rd)),
                  "set_obs")

    def finalize(self, prec_mode: int = PREC_FP64, stream=None):
        self._chk(lib().wc4d_finalize(self._h, int(prec_mode), _stream(stream)), "finalize")
        nA, q = ctypes.c_int(), ctypes.c_int()
        self._chk(lib().wc4d_dims(self._h, ctypes.byref(nA), ctypes.byref(q)), "dims")
        self.n_A, self.q = nA.value, q.value

    @classmethod
    def from_workload(cls, w, pattern, x0: Optional[np.ndarray] = None, device: int = 0,
                      sigma_o2: Optional[float] = None, prec: int = PREC_FP64,
                      strong: bool = False) -> "Problem":
        """Set up a problem from workload parameters with the library's own helpers
        (covariance square roots, Lorenz-96 trajectory); strong: the strong-constraint
        operator on x_0 alone (Q^{1/2} is then not used)."""
        p = cls(w.n, w.N, device, strong=strong)
        if w.model == "advdiff":
            p.set_model_advdiff(w.c, w.r)
        else:
            if x0 is None:
                raise ValueError("Lorenz-96 needs an initial state")
            p.traj = l96_trajectory(x0, w.F, w.dt, w.N)
            p.set_model_l96(p.traj, w.F, w.dt)
        p.set_Bsqrt(corr_sqrt(w.n, w.corr, w.Lb, w.sigma_b))
        p.set_Qsqrt(corr_sqrt(w.n, w.corr, w.Lq, w.sigma_q))
        s2 = w.sigma_o2 if sigma_o2 is None else sigma_o2
        for i, idx in pattern:
            p.set_obs(i, idx, np.full(len(idx), s2))
        p.finalize(prec)
        return p

    # ---- operator
    def _block_call(self, fn, X, Y, stream, what):
        import torch
        m, X2 = _block_rows(X, self.n_A, what + " X")
        if Y is None:
            Y = torch.empty_like(X)
        xp, yp = _ptrs((X2, None, what + " X"), (Y, tuple(X.shape), what + " Y"))
        self._chk(fn(self._h, xp, self.n_A, yp, self.n_A, m, _stream(stream)), what)
        return Y

    def apply_A(self, X, Y=None, stream=None):
        return self._block_call(lib().wc4d_apply_A, X, Y, stream, "apply_A")

    def apply_A_prec(self, X, prec: int, Y=None, stream=None):
        import torch
        m, X2 = _block_rows(X, self.n_A, "apply_A_prec X")
        if Y is None:
            Y = torch.empty_like(X)
        xp, yp = _ptrs((X2, None, "apply_A_prec X"), (Y, tuple(X.shape), "apply_A_prec Y"))
        self._chk(lib().wc4d_apply_A_prec(self._h, xp, self.n_A, yp, self.n_A, m, int(prec), _stream(stream)),
                  "apply_A_prec")
        return Y

    def apply_Linv(self, X, Y=None, stream=None):
        return self._block_call(lib().wc4d_apply_Linv, X, Y, stream, "apply_Linv")

    def apply_LinvT(self, X, Y=None, stream=None):
        return self._block_call(lib().wc4d_apply_LinvT, X, Y, stream, "apply_LinvT")

    def apply_Dsqrt(self, X, Y=None, stream=None):
        return self._block_call(lib().wc4d_apply_Dsqrt, X, Y, stream, "apply_Dsqrt")

    def rhs(self, d, bt=None, out=None, stream=None):
        import torch
        items = []
        if bt is not None:
            items.append((bt, self.n_A, "rhs bt"))
        if self.q > 0:
            items.append((d, self.q, "rhs d"))
        for t, shape, what in items:
            _check_size(t, shape, what)
        if out is None:
            out = torch.empty(self.n_A, dtype=torch.float64, device=self.torch_device)
        items.insert(0, (out, self.n_A, "rhs out"))
        ptrs = _ptrs(*items)
        bp = ptrs[1] if bt is not None else None
        dp = ptrs[-1] if self.q > 0 else None
        self._chk(lib().wc4d_rhs(self._h, dp, bp, ptrs[0], _stream(stream)), "rhs")
        return out

    # ---- preconditioner and solve
    def lmp_build(self, method, k_r: int, l: int, G=None, seed: int = 0, stream=None) -> Lmp:
        """LMP from the start block G ((k_r + l, n_A) device tensor), or, with G None, from
        the Gaussian block of `seed` drawn on the device inside the build."""
        meth = METHOD[method] if isinstance(method, str) else int(method)
        h = _vp()
        gp = _tptr(G, (int(k_r) + int(l), self.n_A), "lmp_build G") if G is not None else None
        self._chk(lib().wc4d_lmp_build(self._h, meth, int(k_r), int(l), gp,
                                       ctypes.c_ulonglong(int(seed) & 0xFFFFFFFFFFFFFFFF), ctypes.byref(h),
                                       _stream(stream)), "lmp_build")
        return Lmp(h.value, self, int(k_r))

    def lmp_build_sketch(self, net: Optional["SketchNet"], method, k_r: int, l: int, Omega, stream=None):
        """LMP from the learned sketch net(self, Omega), or from Omega itself when net is
        None or the learned block is rank deficient.  Returns (Lmp, used_net)."""
        meth = METHOD[method] if isinstance(method, str) else int(method)
        h = _vp()
        used = ctypes.c_int(0)
        op = _tptr(Omega, (int(k_r) + int(l), self.n_A), "lmp_build_sketch Omega")
        self._chk(lib().wc4d_lmp_build_sketch(self._h, net._h if net is not None else None, meth, int(k_r),
                                              int(l), op, ctypes.byref(h), ctypes.byref(used),
                                              _stream(stream)), "lmp_build_sketch")
        return Lmp(h.value, self, int(k_r)), bool(used.value)

    def sketch_loss(self, G, U, theta, dG=None, stream=None):
        """Capture loss f of the start block G (m, n_A) against Ritz pairs U (k, n_A),
        theta (k,) (device tensors); returns (f as a 1-element tensor, dG)."""
        import torch
        if G.dim() != 2 or G.shape[1] != self.n_A or U.dim() != 2 or U.shape[1] != self.n_A:
            raise ValueError(f"sketch_loss: G and U must be (columns, n_A = {self.n_A})")
        k = U.shape[0]
        _check_size(theta, k, "sketch_loss theta")
        if dG is None:
            dG = torch.empty_like(G)
        _check_size(dG, tuple(G.shape), "sketch_loss dG")
        f = torch.empty(1, dtype=torch.float64, device=self.torch_device)
        gp, up, tp, dp = _ptrs((G, None, "sketch_loss G"), (U, None, "sketch_loss U"),
                               (theta, k, "sketch_loss theta"), (dG, tuple(G.shape), "sketch_loss dG"))
        self._chk(lib().wc4d_sketch_loss(self._h, gp, self.n_A, G.shape[0], up, self.n_A, tp, k, _tptr(f), dp,
                                         self.n_A, _stream(stream)), "sketch_loss")
        return f, dG

    def autotune(self, m: int, stream=None) -> dict:
        """Tune the D^{1/2} tile shapes for block width m; returns the choice."""
        self._chk(lib().wc4d_autotune(self._h, int(m), _stream(stream)), "autotune")
        tb, tq, two = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        ms = ctypes.c_float()
        self._chk(lib().wc4d_autotune_info(self._h, int(m), ctypes.byref(tb), ctypes.byref(tq), ctypes.byref(two),
                                           ctypes.byref(ms)), "autotune_info")
        seg = two.value
        return {"tile_b": tb.value, "tile_q": tq.value, "single_product": tq.value == 0, "two_segment": seg > 0,
                "segment_variant": (seg - 1) % 8 if seg else None, "segment_splits": (seg - 1) // 8 if seg else None,
                "ms": ms.value}

    def pcg(self, b, x, lmp: Optional[Lmp] = None, tol: float = 1e-6, maxit: int = 100,
            criterion: int = RES_TRUE, history: bool = True, variant: int = PCG_FUSED, stream=None):
        opts = PcgOpts(float(tol), int(maxit), int(criterion), int(variant))
        info = PcgInfo()
        ht = np.zeros(maxit) if history else None
        hp = np.zeros(maxit) if history else None
        hj = np.zeros(maxit) if history else None
        bp, xp = _ptrs((b, self.n_A, "pcg b"), (x, self.n_A, "pcg x"))
        rc = lib().wc4d_pcg(self._h, lmp._h if lmp is not None else None, bp, xp,
                            ctypes.byref(opts), ctypes.byref(info),
                            _dptr(ht) if history else None, _dptr(hp) if history else None,
                            _dptr(hj) if history else None, _stream(stream))
        if rc not in (OK, ENOCONV, EBREAKDOWN):
            self._chk(rc, "pcg")
        out = {"iters": info.iters, "status": info.status, "relres_true": info.relres_true,
               "relres_precond": info.relres_precond, "J": info.J}
        if history:
            k = info.iters
            out.update(hist_true=ht[:k], hist_precond=hp[:k], hist_J=hj[:k])
        return out

    def pcg_ritz(self, b, x, lmp: Lmp, tol: float = 1e-6, maxit: int = 100, criterion: int = RES_TRUE,
                 stream=None):
        """Preconditioned CG with the Ritz-LMP of lmp (eq. Ritz_LMP; lmp.ritz_prepare() first)."""
        opts = PcgOpts(float(tol), int(maxit), int(criterion), PCG_PLAIN)
        info = PcgInfo()
        ht, hj = np.zeros(maxit), np.zeros(maxit)
        bp, xp = _ptrs((b, self.n_A, "pcg_ritz b"), (x, self.n_A, "pcg_ritz x"))
        rc = lib().wc4d_pcg_ritz(self._h, lmp._h, bp, xp, ctypes.byref(opts), ctypes.byref(info), _dptr(ht),
                                 _dptr(hj), _stream(stream))
        if rc not in (OK, ENOCONV, EBREAKDOWN):
            self._chk(rc, "pcg_ritz")
        k = info.iters
        return {"iters": k, "status": info.status, "relres_true": info.relres_true,
                "relres_precond": info.relres_precond, "J": info.J, "hist_true": ht[:k], "hist_J": hj[:k]}

    def pcg_lanczos(self, b, x, tol: float = 1e-6, maxit: int = 100, reorth: bool = False, stream=None):
        """Plain CG (no second-level preconditioner) that also returns the Lanczos
        information of Section 3.4: (info, alphas, betas, F) with F (maxit + 1, n_A) holding
        f_j = (-1)^j r_j / ||r_j|| in its rows 0..iters.  reorth: complete
        reorthogonalisation of each residual against the earlier ones (maxit <= 512)."""
        import torch
        bp, xp = _ptrs((b, self.n_A, "pcg_lanczos b"), (x, self.n_A, "pcg_lanczos x"))
        F = torch.zeros((int(maxit) + 1, self.n_A), dtype=torch.float64, device=self.torch_device)
        al, be = np.zeros(int(maxit)), np.zeros(int(maxit))
        opts = PcgOpts(float(tol), int(maxit), RES_TRUE, PCG_PLAIN)
        info = PcgInfo()
        rc = lib().wc4d_pcg_lanczos(self._h, bp, xp, ctypes.byref(opts), ctypes.byref(info), _dptr(al), _dptr(be),
                                    _tptr(F, what="F"), self.n_A, LANCZOS_REORTH if reorth else 0,
                                    _stream(stream))
        if rc not in (OK, ENOCONV, EBREAKDOWN):
            self._chk(rc, "pcg_lanczos")
        k = info.iters
        return ({"iters": k, "status": info.status, "relres_true": info.relres_true, "J": info.J},
                al[:k].copy(), be[:k].copy(), F)

    def lanczos_pairs(self, alphas, betas, F, j: int, k: int, stream=None):
        """The k largest Ritz pairs from j CG iterations (Section 3.4): (U (k, n_A), theta)."""
        import torch
        al = np.ascontiguousarray(alphas, dtype=np.float64)
        be = np.ascontiguousarray(betas, dtype=np.float64)
        if al.size < j or be.size < j or F.dim() != 2 or F.shape[0] < j or F.shape[1] != self.n_A:
            raise ValueError("lanczos_pairs: need j coefficients and an (>= j, n_A) F")
        U = torch.empty((int(k), self.n_A), dtype=torch.float64, device=self.torch_device)
        th = np.empty(int(k))
        self._chk(lib().wc4d_lanczos_pairs(self._h, int(j), _dptr(al), _dptr(be), _tptr(F, what="F"), self.n_A,
                                           int(k), _tptr(U, what="U"), self.n_A, _dptr(th), _stream(stream)),
                  "lanczos_pairs")
        return U, th

    def lmp_from_pairs(self, U, theta, stream=None) -> Lmp:
        """Spectral LMP on this problem from given Ritz pairs (U (k, n_A), theta (k,))."""
        th = np.ascontiguousarray(theta, dtype=np.float64)
        k = th.size
        up = _tptr(U, (k, self.n_A), "lmp_from_pairs U")
        h = _vp()
        self._chk(lib().wc4d_lmp_from_pairs(self._h, int(k), up, self.n_A, _dptr(th), ctypes.byref(h),
                                            _stream(stream)), "lmp_from_pairs")
        return Lmp(h.value, self, int(k))

    PROF_CLASSES = ("dsqrt_gemm", "sweep_fwd", "sweep_bwd", "lmp_ut", "lmp_un", "build_other",
                    "dsqrt_bf16x3", "sketch_net")

    def prof_enable(self, enable: bool = True, classes=None):
        """Reset the per-class totals and time the given classes (names or indices of
        PROF_CLASSES; all when None) while enable is true."""
        mask = 0
        if enable:
            if classes is None:
                mask = (1 << len(self.PROF_CLASSES)) - 1
            else:
                for c in classes:
                    mask |= 1 << (self.PROF_CLASSES.index(c) if isinstance(c, str) else int(c))
        self._chk(lib().wc4d_prof_enable(self._h, mask), "prof_enable")

    def prof_stride(self, every: int = 1):
        """Time one launch group in `every` of each enabled class."""
        self._chk(lib().wc4d_prof_stride(self._h, int(every)), "prof_stride")

    def prof_read(self) -> dict:
        out = {}
        for c, name in enumerate(self.PROF_CLASSES):
            ms, b, f = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
            n = ctypes.c_longlong()
            self._chk(lib().wc4d_prof_read(self._h, c, ctypes.byref(ms), ctypes.byref(n), ctypes.byref(b),
                                           ctypes.byref(f)), "prof_read")
            out[name] = {"ms": ms.value, "launches": n.value, "bytes": b.value, "flops": f.value}
        return out

    def set_profiling(self, enable: bool = True):
        self._chk(lib().wc4d_set_profiling(self._h, int(bool(enable))), "set_profiling")

    def last_apply_timing(self) -> np.ndarray:
        out = (ctypes.c_float * 4)()
        self._chk(lib().wc4d_last_apply_timing(self._h, out), "last_apply_timing")
        return np.array(list(out), dtype=np.float64)

    def close(self):
        if getattr(self, "_h", None):
            lib().wc4d_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def autotune_save(path: str):
    rc = lib().wc4d_autotune_save(os.fsencode(path))
    if rc:
        raise Wc4dError(rc, f"wc4d_autotune_save({path})")


def autotune_load(path: str):
    rc = lib().wc4d_autotune_load(os.fsencode(path))
    if rc:
        raise Wc4dError(rc, f"wc4d_autotune_load({path})")


def batch_solve(problems: Sequence[Problem], method, k_r: int, l: int, G, b, x, tol: float = 1e-6,
                maxit: int = 5000, criterion: int = RES_TRUE, variant: int = PCG_FUSED, workers: int = 4,
                autotune: bool = True):
    """Solve independent inner loops at once (wc4d_batch_solve).  G, b, x: lists of
    device tensors per problem ((m, n_A), (n_A,), (n_A,)).  Returns (infos, status)."""
    cnt = len(problems)
    meth = METHOD[method] if isinstance(method, str) else int(method)
    if not (len(G) == len(b) == len(x) == cnt):
        raise ValueError("batch_solve: G, b and x need one entry per problem")
    P = (_vp * cnt)(*[p._h for p in problems])
    m = int(k_r) + int(l)
    items = []
    for i, p in enumerate(problems):
        items += [(G[i], (m, p.n_A), f"batch_solve G[{i}]"), (b[i], p.n_A, f"batch_solve b[{i}]"),
                  (x[i], p.n_A, f"batch_solve x[{i}]")]
    ptrs = _ptrs(*items)
    Gp = (_vp * cnt)(*ptrs[0::3])
    bp = (_vp * cnt)(*ptrs[1::3])
    xp = (_vp * cnt)(*ptrs[2::3])
    infos = (PcgInfo * cnt)()
    status = (ctypes.c_int * cnt)()
    opts = PcgOpts(float(tol), int(maxit), int(criterion), int(variant))
    rc = lib().wc4d_batch_solve(P, cnt, meth, int(k_r), int(l), Gp, bp, xp, ctypes.byref(opts), infos, status,
                                int(workers), int(bool(autotune)))
    if rc != OK:
        bad = [i for i in range(cnt) if status[i] not in (OK, ENOCONV, EBREAKDOWN)]
        msg = lib().wc4d_last_error(problems[bad[0]]._h).decode() if bad else ""
        raise Wc4dError(rc, f"batch_solve: {msg}")
    out = [{"iters": i.iters, "status": i.status, "relres_true": i.relres_true, "relres_precond": i.relres_precond,
            "J": i.J} for i in infos]
    return out, list(status)


def batch_solve_persistent(problems: Sequence[Problem], method, k_r: int, l: int, b, x, G=None, seed: int = 0,
                           tol: float = 1e-6, maxit: int = 5000, criterion: int = RES_TRUE,
                           sweep_fp32: bool = False):
    """Solve independent inner loops with all PCG iterations in one persistent launch
    (wc4d_batch_solve_persistent).  b, x: lists of device tensors (n_A,) per problem; G:
    None (each problem i draws the Gaussian block of seed + i on the device) or a list of
    (k_r + l, n_A) tensors.  Returns (infos, status, kernel_ms)."""
    cnt = len(problems)
    meth = METHOD[method] if isinstance(method, str) else int(method)
    if not (len(b) == len(x) == cnt) or (G is not None and len(G) != cnt):
        raise ValueError("batch_solve_persistent: b, x (and G) need one entry per problem")
    m = int(k_r) + int(l)
    items = []
    for i, p in enumerate(problems):
        items += [(b[i], p.n_A, f"b[{i}]"), (x[i], p.n_A, f"x[{i}]")]
        if G is not None:
            items.append((G[i], (m, p.n_A), f"G[{i}]"))
    ptrs = _ptrs(*items)
    step = 2 if G is None else 3
    P = (_vp * cnt)(*[p._h for p in problems])
    bp = (_vp * cnt)(*ptrs[0::step])
    xp = (_vp * cnt)(*ptrs[1::step])
    Gp = (_vp * cnt)(*ptrs[2::step]) if G is not None else None
    infos = (PcgInfo * cnt)()
    status = (ctypes.c_int * cnt)()
    kms = ctypes.c_double(0.0)
    opts = PcgOpts(float(tol), int(maxit), int(criterion), PCG_FUSED)
    rc = lib().wc4d_batch_solve_persistent(P, cnt, meth, int(k_r), int(l), Gp,
                                           ctypes.c_ulonglong(int(seed) & 0xFFFFFFFFFFFFFFFF), bp, xp,
                                           ctypes.byref(opts), BATCH_SWEEP_FP32 if sweep_fp32 else 0, infos, status,
                                           ctypes.byref(kms))
    if rc != OK:
        msgs = []
        for p in problems:
            m_ = lib().wc4d_last_error(p._h).decode()
            if m_ and m_ not in msgs:
                msgs.append(m_)
        raise Wc4dError(rc, "batch_solve_persistent: " + "; ".join(msgs) +
                        f" (status per problem: {list(status)})")
    out = [{"iters": i.iters, "status": i.status, "relres_true": i.relres_true, "relres_precond": i.relres_precond,
            "J": i.J} for i in infos]
    return out, list(status), kms.value


BATCH_PHASES = ("C1_UtS", "C2_r0", "C3_UtR", "C4_p0", "D1_dsqrt", "FW_sweep", "BW_sweep", "D2_dsqrt",
                "T_UtAp", "UP_update", "P_update", "transitions")


def batch_persistent_profile() -> dict:
    """Per-phase workgroup-busy ms and item counts of the last persistent launch."""
    n = len(BATCH_PHASES) + 1
    ms = (ctypes.c_double * n)()
    cnt = (ctypes.c_longlong * n)()
    lib().wc4d_batch_persistent_profile(ms, cnt, n)
    out = {name: {"busy_ms": ms[i], "items": cnt[i]} for i, name in enumerate(BATCH_PHASES)}
    out["launch"] = {"ms": ms[n - 1], "workgroups": cnt[n - 1]}
    return out


class SketchNet:
    """Learned sketch network (see include/wc4d.h): parameters live on the GPU, training
    and inference run in the library's kernels."""

    def __init__(self, layers: int = 4, noise_channels: int = 64, device: int = 0, _handle=None):
        if _handle is None:
            h = _vp()
            rc = lib().wc4d_sketchnet_create(ctypes.byref(h), int(layers), 64, 5, int(noise_channels), int(device))
            if rc:
                raise Wc4dError(rc, "wc4d_sketchnet_create")
            _handle = h.value
        self._h = _handle
        self.device = int(device)
        self.noise_channels = int(noise_channels)
        c = ctypes.c_longlong()
        lib().wc4d_sketchnet_nparams(self._h, ctypes.byref(c))
        self.nparams = c.value

    @classmethod
    def load(cls, path: str, device: int = 0) -> "SketchNet":
        h = _vp()
        rc = lib().wc4d_sketchnet_load(ctypes.byref(h), os.fsencode(path), int(device))
        if rc:
            raise Wc4dError(rc, f"wc4d_sketchnet_load({path})")
        # header: "WC4DSKN1", int32 layers, channels, width, noise_channels
        hdr = np.fromfile(path, dtype=np.int32, count=6)
        return cls(layers=int(hdr[2]), noise_channels=int(hdr[5]), device=device, _handle=h.value)

    def _chk(self, rc: int, what: str):
        if rc != OK:
            msg = lib().wc4d_sketchnet_last_error(self._h) if self._h else b""
            raise Wc4dError(rc, f"{what}: {msg.decode() if msg else ''}")

    def save(self, path: str):
        self._chk(lib().wc4d_sketchnet_save(self._h, os.fsencode(path)), "save")

    def _vec(self, fn, what, src=None) -> np.ndarray:
        if src is None:
            out = np.empty(self.nparams, dtype=np.float32)
            self._chk(fn(self._h, out.ctypes.data_as(_c_flt_p)), what)
            return out
        a = np.ascontiguousarray(src, dtype=np.float32)
        if a.size != self.nparams:
            raise ValueError(f"expected {self.nparams} parameters")
        self._chk(fn(self._h, a.ctypes.data_as(_c_flt_p)), what)
        return a

    def set_params(self, theta):
        self._vec(lib().wc4d_sketchnet_set_params, "set_params", theta)

    def get_params(self) -> np.ndarray:
        return self._vec(lib().wc4d_sketchnet_get_params, "get_params")

    def get_grad(self) -> np.ndarray:
        return self._vec(lib().wc4d_sketchnet_get_grad, "get_grad")

    def set_grad(self, g):
        self._vec(lib().wc4d_sketchnet_set_grad, "set_grad", g)

    def infer(self, prob: "Problem", Omega, G=None, stream=None):
        import torch
        if G is None:
            G = torch.empty((64, prob.n_A), dtype=torch.float64, device=prob.torch_device)
        op = _tptr(Omega, (self.noise_channels, prob.n_A), "infer Omega") if Omega is not None else None
        gp = _tptr(G, (64, prob.n_A), "infer G")
        self._chk(lib().wc4d_sketchnet_infer(self._h, prob._h, op, prob.n_A, gp, prob.n_A, _stream(stream)),
                  "infer")
        return G

    def backward(self, dG, stream=None):
        if dG.dim() != 2 or dG.shape[0] != 64:
            raise ValueError("backward: dG must be (64, n_A) of the last inference")
        self._chk(lib().wc4d_sketchnet_backward(self._h, _tptr(dG, what="backward dG"), dG.shape[-1],
                                                _stream(stream)), "backward")

    def adam(self, lr: float, stream=None):
        self._chk(lib().wc4d_sketchnet_adam(self._h, float(lr), _stream(stream)), "adam")

    def train_step(self, prob: "Problem", Omega, ref: Lmp, k: int, lr: float, stream=None) -> float:
        loss = ctypes.c_double(0.0)
        op = _tptr(Omega, (self.noise_channels, prob.n_A), "train_step Omega")
        self._chk(lib().wc4d_sketchnet_train_step(self._h, prob._h, op, prob.n_A, ref._h, int(k),
                                                  float(lr), ctypes.byref(loss), _stream(stream)), "train_step")
        return loss.value

    def close(self):
        if getattr(self, "_h", None):
            lib().wc4d_sketchnet_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
