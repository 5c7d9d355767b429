"""The rate fit of the HMF stability study on synthetic magnetization
histories (no GPU)."""
import numpy as np

from paper_1206_3229_amd.dynamics import fit_rate


def test_growth_rate_from_the_linear_phase_only():
    t = 0.05 * (np.arange(2000) + 0.5)
    m = 5e-4 * np.exp(0.116166 * t)
    m = np.where(m > 0.3, 0.3 + 0.02 * np.sin(t), m)  # saturation and nonlinear oscillation
    assert abs(fit_rate(t, m, True) - 0.116166) < 1e-9


def test_damping_rate_over_its_window():
    t = 0.05 * (np.arange(2000) + 0.5)
    m = 5e-4 * np.exp(-0.109956 * t)
    assert abs(fit_rate(t, m, False) + 0.109956) < 1e-9


def test_no_linear_phase_gives_none():
    t = 0.05 * (np.arange(100) + 0.5)
    assert fit_rate(t, np.full(100, 1e-4), True) is None
