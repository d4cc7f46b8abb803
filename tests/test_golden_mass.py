"""Consistency of the stored bare mass of the solve workload (written by
oracle/tune_mass.py, which calls only the oracle): kappa matches m0, the
stored smallest singular value meets the 0.01 target within the script's
5 % stopping rule on the heavy side of the critical mass, and the scan is a
V around m_c (falling below it, rising above it)."""

import json
import os

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "smooth_links_mass.json")


def test_stored_mass_is_consistent():
    with open(GOLDEN) as fh:
        g = json.load(fh)
    m0, kappa = g["m0"], g["kappa"]
    assert abs(kappa - 1.0 / (2.0 * (4.0 + m0))) < 1e-15
    assert g["t_bc_for_sigma_min"] == 1 and g["target_sigma_min"] == 0.01
    assert abs(g["sigma_min"] - 0.01) <= 0.05 * 0.01
    assert m0 > g["m_c_estimate"]
    scan = sorted((float(k), v) for k, v in g["scan"].items())
    assert any(abs(m - m0) < 6e-6 for m, _ in scan)  # scan keys carry five decimals
    above = [(m, v) for m, v in scan if m > g["m_c_estimate"]]
    below = [(m, v) for m, v in scan if m < g["m_c_estimate"]]
    assert all(v2 > v1 for (_, v1), (_, v2) in zip(above, above[1:]))
    assert all(v2 < v1 for (_, v1), (_, v2) in zip(below, below[1:]))
