"""Pins of the oracle's interpolation sweep against what the paper and the
mathematics fix (no GPU).

* eq. (findif): the coefficients are re-derived here from the Taylor
  conditions in exact rational arithmetic (independently of the printed
  numbers) and compared with the printed ones and with the oracle's impulse
  response; the stencil is exact on polynomials up to degree 9 and not on
  degree 10 (eighth order).
* eqs. (splinegen, splinecoeffs): the oracle's unscaled combination equals
  the paper's scaled formula on a non-unit grid; cubics are reproduced; whole
  cell shifts are exact rolls; Fourier modes are eigenvectors with the closed
  form eigenvalue; a 16-point line agrees with the dense operator built in
  exact rationals.
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest
from functools import lru_cache

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@lru_cache(maxsize=None)
def fornberg_second_derivative(half_width: int):
    """Centred weights c_m, m = -w..w, with sum c_m m^d = 2 delta_{d,2}, d <= 2w."""
    ms = list(range(-half_width, half_width + 1))
    n = len(ms)
    A = [[Fraction(m) ** d for m in ms] for d in range(n)]
    b = [Fraction(2 if d == 2 else 0) for d in range(n)]
    # Gauss-Jordan elimination in exact arithmetic.
    M = [row[:] + [b[r]] for r, row in enumerate(A)]
    for c in range(n):
        piv = next(r for r in range(c, n) if M[r][c] != 0)
        M[c], M[piv] = M[piv], M[c]
        inv = 1 / M[c][c]
        M[c] = [v * inv for v in M[c]]
        for r in range(n):
            if r != c and M[r][c] != 0:
                fac = M[r][c]
                M[r] = [a - fac * bb for a, bb in zip(M[r], M[c])]
    return {m: M[k][n] for k, m in enumerate(ms)}


def test_printed_coefficients_are_the_eighth_order_weights():
    g = json.load(open(os.path.join(GOLDEN, "fd_stencil.json")))
    printed = [Fraction(a, b) for a, b in zip(g["numerators"], g["denominators"])]
    derived = fornberg_second_derivative(4)
    for m in range(5):
        assert derived[m] == printed[m] == derived[-m]


def test_impulse_response_is_rounded_coefficients(oracle):
    derived = fornberg_second_derivative(4)
    n = 32
    for m in range(-6, 7):
        line = np.zeros(n)
        line[(10 + m) % n] = 1.0
        got = oracle.second_difference(line, 10, 0)
        want = float(derived.get(m, Fraction(0)))
        assert got == want, (m, got, want)


@pytest.mark.parametrize("d", range(0, 11))
def test_stencil_polynomial_order(oracle, d):
    # Unit spacing, zero boundary: samples u^d at u = -12..12, evaluate at l.
    us = np.arange(-12, 13, dtype=np.float64)
    line = us ** d
    for l in (-3, 0, 2, 5):
        got = oracle.second_difference(line, l + 12, 1)
        exact = d * (d - 1) * float(l) ** (d - 2) if d >= 2 else 0.0
        if d <= 9:
            scale = max(1.0, float(np.abs(line[l + 8:l + 17]).max()))
            assert abs(got - exact) <= 1e-14 * scale * 6.6, (d, l, got, exact)
        else:
            # Truncation error of degree 10: sum_m c_m m^10 = -1152 exactly.
            derived = fornberg_second_derivative(4)
            err = sum(c * (Fraction(l) + m) ** 10 for m, c in derived.items()) - 90 * Fraction(l) ** 8
            assert err == -1152
            assert abs(got - exact - (-1152)) <= 1e-6 * max(1.0, abs(exact))


def test_periodic_and_zero_boundaries(oracle):
    rng = np.random.default_rng(1)
    line = rng.standard_normal(20)
    derived = fornberg_second_derivative(4)
    for l in (0, 1, 3, 16, 19):
        per = sum(float(c) * line[(l + m) % 20] for m, c in derived.items())
        zer = sum(float(c) * (line[l + m] if 0 <= l + m < 20 else 0.0) for m, c in derived.items())
        assert abs(oracle.second_difference(line, l, 0) - per) < 1e-14 * 10
        assert abs(oracle.second_difference(line, l, 1) - zer) < 1e-14 * 10
    # zero extension: nodes outside the line see only the inside taps
    assert oracle.second_difference(line, -5, 1) == 0.0
    assert oracle.second_difference(line, 24, 1) == 0.0
    assert oracle.second_difference(line, -4, 1) == pytest.approx(float(derived[4]) * line[0], abs=1e-16)


def test_foot_weights_match_spline_coefficients(oracle):
    # eq. (splinecoeffs) with x_{i+1}-x_i = 1: alpha = 1-theta, beta = theta,
    # gamma = (alpha^3-alpha)/6, delta = (beta^3-beta)/6, foot at i + xi, xi = -shift.
    for shift, m_want, th in ((-0.25, 0, 0.25), (0.25, -1, 0.75), (-3.5, 3, 0.5), (2.0, -2, 0.0),
                              (-7.125, 7, 0.125)):
        m, a, b, g, d = oracle.foot(shift)
        A, B = Fraction(1) - Fraction(th), Fraction(th)
        assert m == m_want
        assert (a, b) == (float(A), float(B))
        assert g == float((A ** 3 - A) / 6) and d == float((B ** 3 - B) / 6)


def test_foot_rounding_to_one_takes_next_cell(oracle):
    # xi = -1e-20: floor is -1 and xi + 1 rounds to 1.0 -> the node itself.
    m, a, b, g, d = oracle.foot(1e-20)
    assert (m, a, b, g, d) == (0, 1.0, 0.0, 0.0, 0.0)
    line = np.random.default_rng(0).standard_normal(16)
    assert np.array_equal(oracle.interpolate_line(line, 1e-20, 0), line)


def test_nonfinite_shift_poisons_line(oracle):
    line = np.ones(16)
    assert np.isnan(oracle.interpolate_line(line, float("nan"), 0)).all()
    assert np.isnan(oracle.interpolate_line(line, 1e12, 0)).all()


def test_unscaled_combination_equals_paper_scaling(oracle):
    """Reading of eq. (findif) without 1/du^2: the paper's f'' = D/du^2 with
    gamma, delta carrying du^2 gives the same value on any spacing."""
    rng = np.random.default_rng(3)
    n, du = 40, 0.173
    line = rng.standard_normal(n)
    derived = fornberg_second_derivative(4)
    for shift in (0.3, -2.71, 5.5):
        got = oracle.interpolate_line(line, shift, 0)
        xi = -shift
        m = math.floor(xi)
        th = xi - m
        for i in range(n):
            k = i + m
            fpp = [sum(float(c) * line[(kk + mm) % n] for mm, c in derived.items()) / du ** 2 for kk in (k, k + 1)]
            x_i, x_i1, x = k * du, (k + 1) * du, (i + xi) * du
            alpha = (x_i1 - x) / (x_i1 - x_i)
            beta = 1 - alpha
            gamma = (alpha ** 3 - alpha) / 6 * (x_i1 - x_i) ** 2
            delta = (beta ** 3 - beta) / 6 * (x_i1 - x_i) ** 2
            want = alpha * line[k % n] + beta * line[(k + 1) % n] + gamma * fpp[0] + delta * fpp[1]
            assert abs(got[i] - want) < 1e-12, (shift, i)


def test_cubic_reproduced(oracle):
    n = 64
    u = np.arange(n, dtype=np.float64)
    c = (0.3, -0.02, 0.004, -1e-4)
    line = c[0] + c[1] * (u - 30) + c[2] * (u - 30) ** 2 + c[3] * (u - 30) ** 3
    for shift in (0.37, -1.61, 3.05):
        got = oracle.interpolate_line(line, shift, 1)
        for i in range(16, 48):
            x = i - shift - 30
            want = c[0] + c[1] * x + c[2] * x ** 2 + c[3] * x ** 3
            assert abs(got[i] - want) < 1e-12, (shift, i)


@pytest.mark.parametrize("q", [-70, -5, -1, 0, 1, 3, 17, 64])
def test_whole_cell_shift_is_exact_roll(oracle, q):
    line = np.random.default_rng(q + 100).standard_normal(37)
    got = oracle.interpolate_line(line, float(q), 0)
    assert np.array_equal(got, np.roll(line, q))
    gz = oracle.interpolate_line(line, float(q), 1)
    want = np.zeros_like(line)
    if abs(q) < 37:
        if q >= 0:
            want[q:] = line[:37 - q]
        else:
            want[:37 + q] = line[-q:]
    assert np.array_equal(gz, want)


def _eigenvalue(kappa, theta):
    derived = fornberg_second_derivative(4)
    sigma = float(derived[0]) + 2 * sum(float(derived[m]) * math.cos(m * kappa) for m in range(1, 5))
    a, b = 1 - theta, theta
    g, d = (a ** 3 - a) / 6, (b ** 3 - b) / 6
    return a + b * np.exp(1j * kappa) + sigma * (g + d * np.exp(1j * kappa))


@pytest.mark.parametrize("q,shift", [(1, 0.3), (5, -2.6), (13, 7.45), (31, 0.5), (32, 0.5)])
def test_fourier_modes_are_eigenvectors(oracle, q, shift):
    n = 64
    kappa = 2 * math.pi * q / n
    l = np.arange(n)
    line = np.cos(kappa * l + 0.4)
    got = oracle.interpolate_line(line, shift, 0)
    xi = -shift
    m = math.floor(xi)
    lam = _eigenvalue(kappa, xi - m)
    want = np.real(lam * np.exp(1j * (kappa * (l + m) + 0.4)))
    assert np.max(np.abs(got - want)) < 5e-14


def test_scheme_never_amplifies():
    worst = 0.0
    for kappa in np.linspace(0, math.pi, 181):
        for th in np.linspace(0, 1, 101):
            worst = max(worst, abs(_eigenvalue(kappa, th)))
    assert worst <= 1 + 1e-14
    assert abs(_eigenvalue(math.pi, 0.5)) < 1e-14


def test_dense_rational_operator(oracle):
    """Build each output as an exact rational combination from eqs. (splinegen,
    splinecoeffs, findif) for dyadic shifts and compare."""
    n = 16
    rng = np.random.default_rng(7)
    line = rng.integers(-1000, 1000, n).astype(np.float64) / 1024.0
    derived = fornberg_second_derivative(4)
    for shift in (Fraction(3, 8), Fraction(-13, 4), Fraction(21, 16), Fraction(-1, 2)):
        xi = -shift
        m = math.floor(xi)
        th = xi - m
        A, B = 1 - th, th
        G, D = (A ** 3 - A) / 6, (B ** 3 - B) / 6
        for bc in (0, 1):
            def smp(k):
                if bc == 0:
                    return Fraction(line[k % n])
                return Fraction(line[k]) if 0 <= k < n else Fraction(0)
            got = oracle.interpolate_line(line, float(shift), bc)
            for i in range(n):
                k = i + m
                Dk = sum(c * smp(k + mm) for mm, c in derived.items())
                Dk1 = sum(c * smp(k + 1 + mm) for mm, c in derived.items())
                exact = A * smp(k) + B * smp(k + 1) + G * Dk + D * Dk1
                assert abs(got[i] - float(exact)) <= 4e-16 * 8, (shift, bc, i)
