"""Block multi-right-hand-side pressure-Poisson solver for MI355X (gfx950).

Implements the hot path of Krasnopolsky, arXiv 1711.10622: the SLAE with m
right-hand sides that arises when m flow realizations share one pressure
matrix (Section 2.2), solved by m concurrent Jacobi-preconditioned BiCGStab
iterations built on the generalized sparse matrix-vector product Y = A X
(Section 2.3, Figure 1).  The compute path is libmrhs.so (HIP kernels behind a
C ABI, include/mrhs.h); this package only marshals arguments.
"""
from ._lib import SHADOW_SEED, MrhsError, load  # noqa: F401
from .api import (AmgHierarchy, ChannelGrid, CsrMatrix, SolveServer, block_bicgstab, gspmv,  # noqa: F401
                  reorder_permutation, stream_probe, trace_enable, trace_read)
