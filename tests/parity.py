"""Element-wise comparison helpers for the GPU parity tests.

Every block comparison is per column: for each column j of an n_A x m block,
    max_i |Y_ij - Yo_ij| <= tol * max_i |Yo_ij|,
so a wrong entry anywhere (a ragged tail, a trapezoid edge, the last panel) fails
on its own instead of being averaged into a block norm.  Ritz values are compared
entry by entry, each relative to itself."""
import numpy as np


def _cols(a):
    a = np.asarray(a, dtype=np.float64)
    return a[:, None] if a.ndim == 1 else a


def col_errors(Y, Yo):
    """Per-column max-abs error of Y against Yo, relative to Yo's column max-abs."""
    Y, Yo = _cols(Y), _cols(Yo)
    assert Y.shape == Yo.shape, (Y.shape, Yo.shape)
    scale = np.maximum(np.abs(Yo).max(axis=0), 1e-300)
    return np.abs(Y - Yo).max(axis=0) / scale


def assert_cols_close(Y, Yo, tol, what=""):
    e = col_errors(Y, Yo)
    j = int(np.argmax(e))
    assert e[j] <= tol, f"{what}: column {j} max-abs error {e[j]:.3e} of its largest entry > {tol:g}"
    return float(e.max())


def assert_entries_rel(th, tho, tol, what=""):
    """|th_i - tho_i| <= tol |tho_i| for every i."""
    th, tho = np.asarray(th, dtype=np.float64), np.asarray(tho, dtype=np.float64)
    assert th.shape == tho.shape, (th.shape, tho.shape)
    e = np.abs(th - tho) / np.maximum(np.abs(tho), 1e-300)
    i = int(np.argmax(e))
    assert e[i] <= tol, f"{what}: entry {i} relative error {e[i]:.3e} ({th[i]!r} vs {tho[i]!r}) > {tol:g}"
    return float(e.max())
