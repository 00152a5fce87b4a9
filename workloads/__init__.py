"""Seeded synthetic inputs shared by the oracle and the GPU path.

Nothing here computes any step of the solver: it only builds matrices and
right-hand sides (see ``grids``, ``rng`` and ``configs``).
"""
from . import configs, grids, rng  # noqa: F401
