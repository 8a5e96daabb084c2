"""Counter-based Gaussian sketch matrix for the oracle (Philox4x32-10 + Box-Muller).

The paper draws its Gaussian test matrix with Matlab's randn (Alg. 1 step 1, Alg. 5/6
steps 2 and 6) and does not fix a generator. The oracle and the GPU path must draw the same
matrix, so each side implements the counter-based Philox4x32-10 generator from its
published definition (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as
1, 2, 3", SC'11): a 4x32-bit counter, a 2x32-bit key, ten rounds of two 32x32->64-bit
multiplies with multipliers 0xD2511F53 and 0xCD9E8D57, and Weyl key increments
0x9E3779B9 and 0xBB67AE85 between rounds.

Layout (a reading of the paper, which is silent on it): normal number t of the stream with
key ``seed`` comes from Philox block b = t // 4 (counter = (b mod 2^32, b div 2^32, 0, 0),
key = (seed mod 2^32, seed div 2^32)); the block's words (x0, x1) and (x2, x3) each give two
normals by the Box-Muller transform in FP64 with u1 = (x+1) 2^-32 in (0, 1] and
u2 = x 2^-32 in [0, 1): z = sqrt(-2 ln u1) * (cos 2 pi u2, sin 2 pi u2). A rows x cols
row-major matrix takes element [r, j] = normal(r * cols + j).

This is test infrastructure: only tests, the smoke check and the benchmark's CPU baseline
may use it.
"""
from __future__ import annotations

import numpy as np

PHILOX_M0 = 0xD2511F53
PHILOX_M1 = 0xCD9E8D57
PHILOX_W0 = 0x9E3779B9
PHILOX_W1 = 0xBB67AE85
_MASK32 = np.uint64(0xFFFFFFFF)


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Ten Philox4x32 rounds on uint32 arrays; returns the four output words (uint32)."""
    c0, c1, c2, c3 = (np.asarray(x, dtype=np.uint64) for x in (c0, c1, c2, c3))
    k0 = np.asarray(k0, dtype=np.uint64)
    k1 = np.asarray(k1, dtype=np.uint64)
    for rnd in range(10):
        if rnd:
            k0 = (k0 + np.uint64(PHILOX_W0)) & _MASK32
            k1 = (k1 + np.uint64(PHILOX_W1)) & _MASK32
        p0 = np.uint64(PHILOX_M0) * c0
        p1 = np.uint64(PHILOX_M1) * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & _MASK32
        hi1, lo1 = p1 >> np.uint64(32), p1 & _MASK32
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return tuple(x.astype(np.uint32) for x in (c0, c1, c2, c3))


def uint32_stream(seed: int, nblocks: int, first_block: int = 0) -> np.ndarray:
    """Words of Philox blocks first_block .. first_block+nblocks-1, shape (nblocks, 4)."""
    b = np.arange(first_block, first_block + nblocks, dtype=np.uint64)
    seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    k0, k1 = seed & 0xFFFFFFFF, seed >> 32
    out = philox4x32_10(b & _MASK32, b >> np.uint64(32), 0, 0, k0, k1)
    return np.stack(out, axis=1)


def gaussian(seed: int, rows: int, cols: int) -> np.ndarray:
    """FP64 rows x cols matrix of i.i.d. N(0,1) draws, element [r, j] = normal(r*cols + j)."""
    total = rows * cols
    nblocks = (total + 3) // 4
    w = uint32_stream(seed, nblocks).astype(np.float64)
    two32 = 2.0 ** -32
    z = np.empty((nblocks, 4))
    for a, b in ((0, 1), (2, 3)):
        u1 = (w[:, a] + 1.0) * two32
        u2 = w[:, b] * two32
        rad = np.sqrt(-2.0 * np.log(u1))
        z[:, a] = rad * np.cos(2.0 * np.pi * u2)
        z[:, b] = rad * np.sin(2.0 * np.pi * u2)
    return z.reshape(-1)[:total].reshape(rows, cols)
