"""Counter-based Gaussian start block of the randomised eigendecompositions.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the bench's
CPU-baseline leg may import this module.  It shares no code with the HIP
library; the library implements the same published generator on its own.

Section 4 (Algorithms 3-5) starts every randomised method from a Gaussian
matrix G whose entries are independent N(0, 1) draws.  Both sides draw G with
the same counter-based generator, written here from its published definitions:

  * Philox-4x32-10 (Salmon, Moraes, Dror and Shaw, "Parallel random numbers: as
    easy as 1, 2, 3", SC 2011): a 128-bit counter (c0, c1, c2, c3) and a 64-bit
    key (k0, k1) go through ten rounds.  One round multiplies c0 by 0xD2511F53
    and c2 by 0xCD9E8D57 (full 64-bit products split into high and low 32-bit
    halves) and returns (hi(c2 M1) ^ c1 ^ k0, lo(c2 M1), hi(c0 M0) ^ c3 ^ k1,
    lo(c0 M0)); between rounds the key is advanced by the Weyl constants
    (0x9E3779B9, 0xBB67AE85) modulo 2^32.
  * Box-Muller (Box and Muller, Ann. Math. Statist. 1958): two independent
    uniforms u1, u2 in (0, 1) give the independent standard normals
    sqrt(-2 ln u1) cos(2 pi u2) and sqrt(-2 ln u1) sin(2 pi u2).

Mapping (this build's convention, the same on both sides): entry (r, c) of an
n_rows x n_cols block drawn with seed s uses key (s mod 2^32, s >> 32) and
counter (r >> 1, c, 0, 0).  The output words (w0, w1, w2, w3) form two 52-bit
uniforms u1 = ((w0 >> 6) 2^26 + (w1 >> 6) + 1/2) 2^-52 and u2 the same from
(w2, w3): every step is exact in float64, and both lie in [2^-53, 1 - 2^-53];
even rows take the cosine normal, odd rows the sine normal.  An entry therefore depends on (s, r, c) only.
"""
from __future__ import annotations

from typing import Optional, Sequence

import numpy as np

M0 = 0xD2511F53
M1 = 0xCD9E8D57
W0 = 0x9E3779B9
W1 = 0xBB67AE85
MASK32 = 0xFFFFFFFF
TWO_PI = 2.0 * np.pi


def _mulhilo(a: int, x: np.ndarray):
    """High and low 32-bit halves of the 64-bit product a * x (x: uint64 array < 2^32)."""
    prod = np.uint64(a) * x           # exact: both factors are below 2^32
    return prod >> np.uint64(32), prod & np.uint64(MASK32)


def philox4x32_10(ctr: np.ndarray, key: Sequence[int]) -> np.ndarray:
    """Philox-4x32-10 of counters ctr (shape (..., 4), values < 2^32) under the key
    (k0, k1).  Returns uint32 words of the same shape."""
    c = np.asarray(ctr, dtype=np.uint64) & np.uint64(MASK32)
    c0, c1, c2, c3 = (c[..., i].copy() for i in range(4))
    k0, k1 = int(key[0]) & MASK32, int(key[1]) & MASK32
    for rnd in range(10):
        if rnd > 0:
            k0 = (k0 + W0) & MASK32
            k1 = (k1 + W1) & MASK32
        hi0, lo0 = _mulhilo(M0, c0)
        hi1, lo1 = _mulhilo(M1, c2)
        c0, c1, c2, c3 = hi1 ^ c1 ^ np.uint64(k0), lo1, hi0 ^ c3 ^ np.uint64(k1), lo0
    return np.stack([c0, c1, c2, c3], axis=-1).astype(np.uint32)


def seed_key(seed: int):
    """The 64-bit seed as Philox's two key words (low, high)."""
    seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    return seed & MASK32, seed >> 32


def uniform52(hi_word: np.ndarray, lo_word: np.ndarray) -> np.ndarray:
    """((hi >> 6) 2^26 + (lo >> 6) + 1/2) / 2^52: a uniform in (0, 1) from the top 26
    bits of two words (each operation exact in float64)."""
    a = (hi_word.astype(np.uint64) >> np.uint64(6)).astype(np.float64)
    b = (lo_word.astype(np.uint64) >> np.uint64(6)).astype(np.float64)
    return (a * 67108864.0 + b + 0.5) * (1.0 / 4503599627370496.0)


def box_muller(u1: np.ndarray, u2: np.ndarray):
    """Two standard normals from two uniforms in (0, 1)."""
    rad = np.sqrt(-2.0 * np.log(u1))
    phi = TWO_PI * u2
    return rad * np.cos(phi), rad * np.sin(phi)


def gaussian_columns(seed: int, n_rows: int, cols: Sequence[int]) -> np.ndarray:
    """Columns `cols` of the n_rows x (any) Gaussian block of `seed`, as an
    (n_rows, len(cols)) float64 array."""
    key = seed_key(seed)
    rows = np.arange(n_rows, dtype=np.uint64)
    out = np.empty((n_rows, len(cols)), dtype=np.float64)
    npairs = (n_rows + 1) // 2
    for j, c in enumerate(cols):
        ctr = np.zeros((npairs, 4), dtype=np.uint64)
        ctr[:, 0] = np.arange(npairs, dtype=np.uint64)
        ctr[:, 1] = np.uint64(int(c) & MASK32)
        w = philox4x32_10(ctr, key)
        z0, z1 = box_muller(uniform52(w[:, 0], w[:, 1]), uniform52(w[:, 2], w[:, 3]))
        pair = rows >> np.uint64(1)
        out[:, j] = np.where((rows & np.uint64(1)) == 0, z0[pair], z1[pair])
    return out


def gaussian_block(seed: int, n_rows: int, n_cols: int, cols: Optional[Sequence[int]] = None) -> np.ndarray:
    """The n_rows x n_cols Gaussian start block of `seed` (all columns, or `cols`)."""
    return gaussian_columns(seed, n_rows, range(n_cols) if cols is None else cols)
