"""Named synthetic workloads (matrix + right-hand sides) with their sizes.

=========  ==================================================  ==========  ===========
name       matrix                                              n           nnz
=========  ==================================================  ==========  ===========
dir16      unit 7-point Dirichlet, 16^3                        4,096       27,136
chan128    stretched channel 128x64x64, tanh beta=2            524,288     3,653,632
cube192    192x96x128 channel, 4x4 array of 16^3 cubes,        2,293,760   15,990,784
           symmetric random relabelling (seed 10622)
dir32      unit 7-point Dirichlet, 32^3                        32,768      223,232
dir64      unit 7-point Dirichlet, 64^3                        262,144     1,810,432
chan256    stretched channel 256x192x256, tanh beta=2          12,582,912  87,949,312
=========  ==================================================  ==========  ===========

The channel domain is 2*pi x 2 x pi (channel half-height 1), the size the
paper uses for its plane-channel case (Section 4); the cube channel uses
12 x 6 x 8 with uniform x/z spacing 1/16 and tanh(2) stretching in y.
Right-hand sides are U[-1, 1) from the SplitMix64 stream of the stated seed;
singular (pure-Neumann/periodic) operators get mean-zero columns.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import grids, rng


@dataclass(frozen=True)
class Workload:
    name: str
    rhs_seed: int
    ms: tuple
    mean_zero: bool

    def matrix(self) -> grids.CSRMatrix:
        return MATRICES[self.name]()

    def rhs(self, n: int, m: int, col0: int = 0) -> np.ndarray:
        return rng.rhs_block(n, m, self.rhs_seed, mean_zero=self.mean_zero, col0=col0)


def _dir16():
    return grids.dirichlet7(16)


def _dir32():
    return grids.dirichlet7(32)


def _dir64():
    return grids.dirichlet7(64)


def _chan128():
    return grids.channel7(128, 64, 64, beta=2.0, name="chan128")


def _chan256():
    return grids.channel7(256, 192, 256, beta=2.0, name="chan256")


def _cube192():
    solid = grids.cube_array_solid()
    A = grids.channel7(192, 96, 128, beta=2.0, lx=12.0, ly=6.0, lz=8.0,
                       solid=solid, name="cube192")
    return grids.permute_symmetric(A, rng.permutation(A.n, 10622))


MATRICES = {
    "dir16": _dir16,
    "dir32": _dir32,
    "dir64": _dir64,
    "chan128": _chan128,
    "chan256": _chan256,
    "cube192": _cube192,
}

WORKLOADS = {
    # small correctness case: m = 4, FP64
    "dir16": Workload("dir16", 1711, (4,), False),
    # the channel case quoted in the metric: m = 1..16, FP64
    "chan128": Workload("chan128", 1712, (1, 2, 4, 8, 16), True),
    # cube channel, relabelled rows: m = 8, mixed precision vs FP64
    "cube192": Workload("cube192", 1713, (8,), True),
    # large channel: m = 1..16, FP64 vs mixed
    "chan256": Workload("chan256", 1715, tuple(range(1, 17)), True),
    # serving matrices
    "dir32": Workload("dir32", 1714, (16,), False),
    "dir64": Workload("dir64", 1714, (16,), False),
}
