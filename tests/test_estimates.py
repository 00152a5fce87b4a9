"""The paper's analytic models against the values it prints (Section 2.3,
Tables 2-5, Figure 3 discussion, Section 4.3).  Fixture: golden/paper_estimates.json."""
import json
import os

import numpy as np

from paper_1711_10622_amd import estimates as est

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_estimates.json")))


def test_compact_gain_m16():
    g = GOLD["table2_3_estimate_m16"]
    assert round(est.gain_compact(g["m"]), g["digits"]) == g["value"]


def test_full_gain_reduces_to_compact():
    for m in (1, 2, 4, 8, 16):
        assert abs(est.gain_full(m, 1e9) - est.gain_compact(m)) < 1e-6
    assert est.gain_full(1, 7.0) == 1.0
    # gain_full is m * Sigma_1 / Sigma_m with the paper's traffic count
    n, nnz = 1000, 7000
    for m in (2, 4, 16):
        ratio = m * (4 * n * 3 + 12 * nnz + 8 * nnz) / (4 * n * (2 * m + 1) + 12 * nnz + 8 * m * nnz)
        assert abs(est.gain_full(m, nnz / n) - ratio) < 1e-12
        assert est.traffic_paper(n, nnz, m) == 4 * n * (2 * m + 1) + 12 * nnz + 8 * m * nnz


def test_table4_5_estimates():
    g = GOLD["table4_5_estimate"]
    for m, v in zip(g["m"], g["value"]):
        assert round(est.step_gain(g["theta"], est.gain_compact(m)), g["digits"]) == v


def test_fig3_optimal_m_and_range():
    g = GOLD["fig3_optimal_m"]
    th = g["theta"]
    for beta, mbest in g["beta_to_m"]:
        ms = [1, 2, 4, 8, 16]
        vals = [est.speedup_est3(beta, th, m) for m in ms]
        assert ms[int(np.argmax(vals))] == mbest
    r = GOLD["fig3_speedup_range"]
    lo = max(est.speedup_est3(r["beta"][0], th, m) for m in (1, 2, 4, 8, 16))
    hi = max(est.speedup_est3(r["beta"][1], th, m) for m in (1, 2, 4, 8, 16))
    assert round((lo - 1) * 100) == r["percent"][0]
    assert round((hi - 1) * 100) == r["percent"][1]
    # m* is the stationary point of est3 in m
    for beta in (5, 20, 40):
        ms = est.m_star(beta, th)
        h = 1e-5
        d = (est.speedup_est3(beta, th, ms + h) - est.speedup_est3(beta, th, ms - h)) / (2 * h)
        assert abs(d) < 1e-6


def test_channel_prediction():
    g = GOLD["channel_m2_prediction"]
    assert round(est.speedup(g["beta"], g["m"], g["step_gain"]), g["digits"]) == g["value"]


def test_asymptote():
    assert abs(est.gain_compact(1e12) - GOLD["asymptotic_gain"]["value"]) < 1e-9


def test_compulsory_traffic():
    n, nnz = 12_582_912, 87_949_312
    assert est.traffic_compulsory(n, nnz, 16) == 4 * (n + 1) + 12 * nnz + 256 * n
    assert est.gain_compulsory(n, nnz, 1) == 1.0
