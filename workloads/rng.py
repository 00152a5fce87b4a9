"""Counter-based random numbers for the synthetic workloads.

Every random value an input needs is output number ``k`` of the SplitMix64
stream seeded with ``seed`` (Steele, Lea & Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014):

    state_k = seed + (k + 1) * 0x9E3779B97F4A7C15          (mod 2**64)
    z = state_k
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9
    z = (z ^ (z >> 27)) * 0x94D049BB133111EB
    out_k = z ^ (z >> 31)

Because output ``k`` is a pure function of ``(seed, k)``, any element of any
input can be regenerated independently; the right-hand-side block uses the
counter ``k = l * n + i`` for row ``i`` of column ``l``, so column ``l`` is the
same vector whatever the block width ``m`` is.

This module holds no arithmetic of the solver; both the oracle and the GPU
path receive its outputs as plain arrays.
"""
from __future__ import annotations

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
MIX1 = np.uint64(0xBF58476D1CE4E5B9)
MIX2 = np.uint64(0x94D049BB133111EB)
_TWO_M53 = 2.0 ** -53


def splitmix64(seed: int, counters: np.ndarray) -> np.ndarray:
    """Outputs ``counters`` (uint64 array) of the SplitMix64 stream ``seed``."""
    k = np.asarray(counters, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + (k + np.uint64(1)) * GAMMA
        z = (z ^ (z >> np.uint64(30))) * MIX1
        z = (z ^ (z >> np.uint64(27))) * MIX2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform_pm1(seed: int, counters: np.ndarray) -> np.ndarray:
    """Doubles in [-1, 1): the top 53 bits of each output scaled to [0, 1),
    then mapped affinely (both steps exact in binary64)."""
    u = splitmix64(seed, counters) >> np.uint64(11)
    return u.astype(np.float64) * (2.0 * _TWO_M53) - 1.0


def rhs_block(n: int, m: int, seed: int, mean_zero: bool = False,
              col0: int = 0) -> np.ndarray:
    """Row-interleaved ``(n, m)`` float64 block of i.i.d. U[-1, 1) values.

    Entry ``(i, l)`` is output ``(col0 + l) * n + i`` of stream ``seed``.
    With ``mean_zero`` each column has its arithmetic mean (numpy's pairwise
    sum) subtracted, which makes it consistent for operators whose null space
    is the constant vector.
    """
    if n == 0 or m == 0:
        return np.zeros((n, m), dtype=np.float64)
    i = np.arange(n, dtype=np.uint64)
    cols = []
    for l in range(m):
        c = uniform_pm1(seed, np.uint64((col0 + l) * n) + i)
        if mean_zero:
            c = c - c.sum() / n
        cols.append(c)
    return np.ascontiguousarray(np.stack(cols, axis=1))


def int_block(n: int, m: int, seed: int, lo: int, hi: int) -> np.ndarray:
    """``(n, m)`` block of integers in [lo, hi] stored as float64 (exact)."""
    i = np.arange(n, dtype=np.uint64)
    span = np.uint64(hi - lo + 1)
    out = np.empty((n, m), dtype=np.float64)
    for l in range(m):
        u = splitmix64(seed, np.uint64(l * n) + i) % span
        out[:, l] = u.astype(np.int64) + lo
    return out


def permutation(n: int, seed: int) -> np.ndarray:
    """A seeded random permutation of ``range(n)``: the stable argsort of the
    first ``n`` outputs of stream ``seed`` (distinct with overwhelming
    probability; ties fall back to index order)."""
    keys = splitmix64(seed, np.arange(n, dtype=np.uint64))
    return np.argsort(keys, kind="stable").astype(np.int64)
