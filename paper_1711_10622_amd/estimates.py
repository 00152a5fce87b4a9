"""The paper's analytic performance models (Section 2.3), for reporting.

These closed forms price the block solve; the benchmark prints them beside
measured gains.  None of them runs on the solve path.

* ``traffic_paper``: bytes moved by the CRS GSpMV loop of Figure 1 as the
  paper counts them (row offsets once, column indices and values once, X once
  per nonzero and column, Y once), generalised to index width ``I`` and value
  width ``V`` (the paper takes I = 4, V = 8).
* ``gain_full``: m * Sigma_1 / Sigma_m with C = nnz/n (eq. mem_GSpMV_full).
* ``gain_compact``: its C >> 1 limit 5m/(2m+3) (eq. mem_GSpMV_compact).
* ``step_gain``: m t_1 / t_m from the solver share theta and the solver gain
  (eq. est2_1).
* ``speedup``: P_m = (1+beta)/(m+beta) * m t_1/t_m (eq. est2).
* ``speedup_est3``: P_m with the compact gain substituted (eq. est3), and
  ``m_star``, the m that maximises it.
* ``traffic_compulsory``: the minimum bytes of one GSpMV when X is read
  once (caches can make it so): I(n+1) + (I+V) nnz + 2 S m n for block
  element width S.  ``gain_compulsory`` is the matching m-gain.
"""
from __future__ import annotations

import math


def traffic_paper(n: int, nnz: int, m: int, I: int = 4, V: int = 8) -> int:
    return I * n + (I + V) * nnz + V * m * nnz + V * m * n


def gain_full(m: float, C: float) -> float:
    return m * (5.0 * C + 3.0) / (2.0 * m * (C + 1.0) + 3.0 * C + 1.0)


def gain_compact(m: float) -> float:
    return 5.0 * m / (2.0 * m + 3.0)


def step_gain(theta: float, solver_gain: float) -> float:
    return 1.0 / (theta / solver_gain + (1.0 - theta))


def speedup(beta: float, m: float, step: float) -> float:
    return (1.0 + beta) / (m + beta) * step


def speedup_est3(beta: float, theta: float, m: float) -> float:
    return (1.0 + beta) / (m + beta) * 5.0 * m / (5.0 * m - 3.0 * theta * (m - 1.0))


def m_star(beta: float, theta: float) -> float:
    return math.sqrt(3.0 * beta * theta / (5.0 - 3.0 * theta))


def traffic_compulsory(n: int, nnz: int, m: int, I: int = 4, V: int = 8, S: int = 8) -> int:
    return I * (n + 1) + (I + V) * nnz + 2 * S * m * n


def gain_compulsory(n: int, nnz: int, m: int, I: int = 4, V: int = 8, S: int = 8) -> float:
    return m * traffic_compulsory(n, nnz, 1, I, V, S) / traffic_compulsory(n, nnz, m, I, V, S)
