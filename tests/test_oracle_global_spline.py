"""Pins of the oracle's global spline (eq. tridiagsys), the paper's baseline
for the local finite-difference f'' (no GPU).

The line update with f'' from the tridiagonal system is the cubic spline
through the samples evaluated at the feet, so it is checked against SciPy's
independent CubicSpline: periodic splines for periodic lines, and for zero
extension a natural spline through the line continued by many zeros.
"""
import math

import numpy as np
import pytest
from scipy.interpolate import CubicSpline

from paper_1206_3229_amd import inputs as I


@pytest.mark.parametrize("n", [16, 37, 128])
@pytest.mark.parametrize("shift", [0.3, -2.7, 5.49, 13.2, -0.999])
def test_periodic_line_is_the_periodic_cubic_spline(oracle, n, shift):
    x = np.arange(n, dtype=np.float64)
    f = np.random.default_rng(n).standard_normal(n)
    got = oracle.interpolate_line_gs(f, shift, I.BC_PERIODIC)
    cs = CubicSpline(np.append(x, n), np.append(f, f[0]), bc_type="periodic")
    assert np.max(np.abs(got - cs((x - shift) % n))) < 5e-14


@pytest.mark.parametrize("shift", [0.3, -2.7, 7.5, -40.2])
def test_zero_extended_line_is_the_spline_through_the_zero_continuation(oracle, shift):
    n, pad = 41, 300
    f = np.zeros(n)
    f[4:37] = np.random.default_rng(3).standard_normal(33)
    got = oracle.interpolate_line_gs(f, shift, I.BC_ZERO)
    xe = np.arange(-pad, n + pad, dtype=np.float64)
    fe = np.zeros(xe.size)
    fe[pad:pad + n] = f
    want = CubicSpline(xe, fe, bc_type="natural")(np.arange(n) - shift)
    assert np.max(np.abs(got - want)) < 2e-14


@pytest.mark.parametrize("q", [-5, 0, 3, 40])
def test_whole_cell_shift_is_an_exact_roll(oracle, q):
    f = np.random.default_rng(7).standard_normal(50)
    assert np.array_equal(oracle.interpolate_line_gs(f, float(q), I.BC_PERIODIC), np.roll(f, q))


def test_full_steps_conserve_mass_and_follow_the_local_spline(oracle):
    th0, p0 = I.waterbag_halfwidths(0.5, 0.69)
    p = I.Params(I.MODEL_HMF, 64, 64, -math.pi, math.pi, -2.5, 2.5, 0.1, spline=I.SPLINE_GS)
    f0 = I.gaussian(p, 0.6, 1e-2)
    f = oracle.run(p, f0, 20)
    m0, m1 = oracle.moments(p, f0), oracle.moments(p, f)
    assert abs(m1["mass"] - m0["mass"]) < 1e-13
    # a smooth state: the two splines differ by the truncation of eq. (findif)
    p_fd = I.Params(**{**p.as_dict(), "spline": I.SPLINE_FD})
    assert np.max(np.abs(f - oracle.run(p_fd, f0, 20))) < 1e-4 * np.max(np.abs(f0))


def test_fp32_storage_within_single_precision(oracle):
    f = np.random.default_rng(11).uniform(0, 1, 64)
    g64 = oracle.interpolate_line_gs(f.astype(np.float32).astype(np.float64), 2.37, I.BC_PERIODIC)
    g32 = oracle.interpolate_line_gs(f, 2.37, I.BC_PERIODIC, storage=I.STORAGE_F32)
    assert np.max(np.abs(g32 - g64)) < 2e-6


def _gs_eigenvalue(kappa, theta):
    # mode e^{i kappa l}: the system gives D = sigma f with
    # (2 cos kappa + 4) sigma = 6 (2 cos kappa - 2)
    sigma = -12.0 * math.sin(kappa / 2) ** 2 / (2.0 + math.cos(kappa))
    a, b = 1 - theta, theta
    g, d = (a ** 3 - a) / 6, (b ** 3 - b) / 6
    return a + b * np.exp(1j * kappa) + sigma * (g + d * np.exp(1j * kappa))


@pytest.mark.parametrize("q,shift", [(1, 0.3), (5, -2.6), (13, 7.45), (31, 0.5), (32, 0.5)])
def test_fourier_modes_are_eigenvectors(oracle, q, shift):
    n = 64
    kappa = 2 * math.pi * q / n
    l = np.arange(n)
    got = oracle.interpolate_line_gs(np.cos(kappa * l + 0.4), shift, I.BC_PERIODIC)
    m = math.floor(-shift)
    lam = _gs_eigenvalue(kappa, -shift - m)
    want = np.real(lam * np.exp(1j * (kappa * (l + m) + 0.4)))
    assert np.max(np.abs(got - want)) < 5e-14


def test_global_spline_never_amplifies():
    worst = max(abs(_gs_eigenvalue(k, t)) for k in np.linspace(0, math.pi, 181) for t in np.linspace(0, 1, 101))
    assert worst <= 1 + 1e-14
    # the shortest wave half way between nodes is removed, as by the local spline
    assert abs(_gs_eigenvalue(math.pi, 0.5)) < 1e-14
