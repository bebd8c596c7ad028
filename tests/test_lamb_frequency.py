"""Eqs. 43-45 (Miller-Scriven frequency) against the analytic column of the
paper's Table 1 (tests/golden/table1_lamb_frequency.txt)."""
import os

import numpy as np

from paper_1810_09299_amd import validation

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_table1_analytic_frequencies():
    rows = np.loadtxt(os.path.join(GOLD, "table1_lamb_frequency.txt"))
    for Re, _, w_ana, _ in rows:
        Rr = {43.3: 30, 56.7: 45, 68.7: 60, 79.7: 75}[round(Re, 1)]
        Re_exact = (Rr * Rr * 90.0) ** (1.0 / 3.0)          # R_e = (R_r^2 R_z)^(1/3), Sec. 3.2
        w = validation.lamb_frequency(2, Re_exact, 100.0, 1.0, 0.3, 0.1, 0.1)
        assert abs(w * 1e4 - w_ana) <= 5e-5, (Re, w * 1e4, w_ana)


def test_damped_frequency_estimator():
    t = np.arange(0, 60000, 20.0)
    w = 4.9e-4
    y = 43.0 + np.where(t < 3000, -13 * np.cos(w * t), 0) + np.where(
        t >= 3000, 6 * np.exp(-2e-4 * t) * np.cos(w * t), 0)
    assert abs(validation.damped_frequency(t, y) - w) <= 1e-3 * w
