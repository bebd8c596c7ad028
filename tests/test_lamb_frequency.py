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


def test_lamb_damping_limits():
    """The two-fluid decay rate reduces to Lamb's (n-1)(2n+1) nu / R^2 for a
    drop in vacuum and (n+2)(2n+1) nu / R^2 for a bubble in liquid, for every n."""
    for n in (2, 3, 4):
        for R in (10.0, 43.3):
            d = validation.lamb_damping(n, R, 1.0, 0.0, 0.1, 0.0)
            assert abs(d - (n - 1) * (2 * n + 1) * 0.1 / R ** 2) <= 1e-15
            b = validation.lamb_damping(n, R, 0.0, 1.0, 0.0, 0.2)
            assert abs(b - (n + 2) * (2 * n + 1) * 0.2 / R ** 2) <= 1e-15


def test_damped_frequency_estimator_returns_decay():
    t = np.arange(0, 60000, 20.0)
    y = 43.0 + 6 * np.exp(-2.7e-4 * t) * np.cos(4.6e-4 * t + 0.3)
    w, g = validation.damped_frequency(t, y, with_decay=True)
    assert abs(w - 4.6e-4) <= 1e-6 * 4.6e-4 and abs(g - 2.7e-4) <= 1e-6 * 2.7e-4
