"""Pins of the oracle's higher-order time splitting and of its filter along p
(the extensions named in the paper's conclusions), no GPU.

Splitting: the substep sizes are the correctly rounded values of the
published formulas and satisfy the fourth-order conditions of a symmetric
composition.  In a harmonic well (external force F = -x) every sweep moves
the mean position and momentum of f exactly as the corresponding linear map
(the spline weights keep mass and shift the first moment by exactly the foot
offset), so the oracle's means follow the product of the shears of the
composition to rounding, whatever the interpolation error; against the exact
rotation they converge with order 2 (Strang) and 4 (the compositions).

Filter: Fourier modes are damped by 1 - sigma sin^8(kappa/2); every p-moment
of degree below 8 of a column is kept and the degree-8 moment falls by
sigma 8!/256 times the mass; it acts after the last kick of every k-th step.
"""
import math
from decimal import Decimal, getcontext

import numpy as np
import pytest

from paper_1206_3229_amd import inputs as I


def _exact_weights():
    getcontext().prec = 50
    c2 = Decimal(2) ** (Decimal(1) / 3)
    c4 = Decimal(4) ** (Decimal(1) / 3)
    w1, w0 = 1 / (2 - c2), -c2 / (2 - c2)
    p = 1 / (4 - c4)
    return {I.SPLIT_STRANG: [Decimal(1)], I.SPLIT_TRIPLE_JUMP: [w1, w0, w1],
            I.SPLIT_SUZUKI: [p, p, 1 - 4 * p, p, p]}


@pytest.mark.parametrize("scheme", [I.SPLIT_STRANG, I.SPLIT_TRIPLE_JUMP, I.SPLIT_SUZUKI])
def test_weights_are_the_rounded_formulas_and_fourth_order(oracle, scheme):
    exact = _exact_weights()[scheme]
    got = oracle.split_weights(scheme)
    assert got == [float(v) for v in exact]
    assert abs(sum(got) - 1.0) < 4e-16
    if scheme != I.SPLIT_STRANG:
        # sum w^3 = 0 cancels the dt^3 error of the Strang step
        assert abs(sum(w ** 3 for w in got)) < 1e-15 * sum(abs(w) ** 3 for w in got)
        assert got == got[::-1]  # symmetric: no even-order error terms


def _well(n_steps, scheme):
    dt = 2 * math.pi / n_steps
    p = I.Params(I.MODEL_EXTERNAL, 128, 128, -8.0, 8.0, -8.0, 8.0, dt, splitting=scheme)
    x = p.xmin + np.arange(p.nx) * p.dx
    pp = p.pmin + np.arange(p.np_) * p.dp
    f0 = np.exp(-((x[None, :] - 1.5) ** 2 + pp[:, None] ** 2) / (2 * 0.5 ** 2))
    return p, f0, -x, x, pp


def _means(f, x, pp):
    m = f.sum()
    return (f.sum(0) @ x) / m, (f.sum(1) @ pp) / m


def _shears(weights, dt, n, X, P):
    # drift x += (h/2) p, kick p -= h x, drift x += (h/2) p, for h = w dt
    for _ in range(n):
        for w in weights:
            h = w * dt
            X = X + 0.5 * h * P
            P = P - h * X
            X = X + 0.5 * h * P
    return X, P


@pytest.mark.parametrize("scheme,order", [(I.SPLIT_STRANG, 2), (I.SPLIT_TRIPLE_JUMP, 4), (I.SPLIT_SUZUKI, 4)])
def test_harmonic_well_means_follow_the_composed_map(oracle, scheme, order):
    errs = []
    for n in (16, 32, 64):
        p, f0, F, x, pp = _well(n, scheme)
        f = oracle.run(p, f0, n, F_ext=F)
        X0, P0 = _means(f0, x, pp)
        X, P = _means(f, x, pp)
        Xm, Pm = _shears([float(v) for v in _exact_weights()[scheme]], p.dt, n, X0, P0)
        assert abs(X - Xm) < 1e-13 and abs(P - Pm) < 1e-13, (n, X - Xm, P - Pm)
        # one period of the exact flow returns to the start
        errs.append(math.hypot(X - X0, P - P0))
    for a, b in zip(errs, errs[1:]):
        assert 0.85 * 2 ** order < a / b < 1.15 * 2 ** order, errs


def test_history_has_one_record_per_force_evaluation(oracle):
    th0, p0 = I.waterbag_halfwidths(0.5, 0.69)
    p = I.Params(I.MODEL_HMF, 32, 32, -math.pi, math.pi, -2.5, 2.5, 0.1, splitting=I.SPLIT_TRIPLE_JUMP)
    f0 = I.waterbag(p, th0, p0, 1e-4, 1)
    f, hist = oracle.run(p, f0, 4, history=True)
    assert hist.shape == (12, 2)
    # the first record is the magnetization after the first half drift, of size w1 dt / 2
    g = oracle.sweep_x(p, f0, 0.5 * (oracle.split_weights(p.splitting)[0] * p.dt))
    rho = g.sum(0) * p.dp
    th = p.xmin + np.arange(p.nx) * p.dx
    assert abs(hist[0, 0] - p.dx * (rho @ np.cos(th))) < 1e-14


def _filter_params(n=64, sigma=1.0, bc_p=I.BC_PERIODIC, storage=0):
    return I.Params(I.MODEL_EXTERNAL, 3, n, 0.0, 1.0, -1.0, 1.0, 0.1, bc_p=bc_p, storage=storage,
                    filter_every=1, filter_strength=sigma)


@pytest.mark.parametrize("q", [1, 5, 16, 31, 32])
@pytest.mark.parametrize("sigma", [1.0, 0.3])
def test_filter_damps_fourier_modes_by_the_closed_form(oracle, q, sigma):
    p = _filter_params(64, sigma)
    kappa = 2 * math.pi * q / 64
    col = np.cos(kappa * np.arange(64) + 0.7)
    f = np.stack([col, 2 * col, -col], axis=1)
    got = oracle.filter_p(p, f)
    assert np.max(np.abs(got - (1 - sigma * math.sin(kappa / 2) ** 8) * f)) < 1e-13


def test_filter_keeps_moments_below_degree_eight(oracle):
    n = 80
    p = _filter_params(n, 0.6, bc_p=I.BC_ZERO)
    rng = np.random.default_rng(5)
    f = np.zeros((n, 3))
    f[10:70] = rng.uniform(0, 1, (60, 3))
    got = oracle.filter_p(p, f)
    j = (np.arange(n) - 40.0) / 40.0  # a scaled coordinate keeps the powers O(1)
    for d in range(8):
        assert np.allclose(j ** d @ got, j ** d @ f, rtol=0, atol=1e-13), d
    # delta^8 of j^8 is 8! (in cell units): the eighth moment falls by sigma 8!/256 times the mass
    drop = (j ** 8 @ f) - (j ** 8 @ got)
    assert np.allclose(drop, 0.6 * 40320 / 256 * f.sum(0) / 40.0 ** 8, rtol=1e-9)


def test_filter_in_fp32_within_single_precision(oracle):
    p64 = _filter_params(64, 0.5)
    p32 = _filter_params(64, 0.5, storage=1)
    f = np.random.default_rng(2).uniform(0, 1, (64, 3)).astype(np.float32).astype(np.float64)
    assert np.max(np.abs(oracle.filter_p(p32, f) - oracle.filter_p(p64, f))) < 4e-6


def test_filter_acts_after_every_kth_step_and_dissipates(oracle):
    th0, p0 = I.waterbag_halfwidths(0.5, 0.69)
    base = I.Params(I.MODEL_HMF, 64, 64, -math.pi, math.pi, -2.5, 2.5, 0.2)
    f0 = I.waterbag(base, th0, p0, 1e-4, 3)
    filt = I.Params(**{**base.as_dict(), "filter_every": 3, "filter_strength": 1.0})
    # steps 1 and 2 are unfiltered, step 3 is
    assert np.array_equal(oracle.run(filt, f0, 2), oracle.run(base, f0, 2))
    a, b = oracle.run(filt, f0, 30), oracle.run(base, f0, 30)
    assert not np.array_equal(a, b)
    ma, mb = oracle.moments(filt, a), oracle.moments(base, b)
    assert abs(ma["mass"] - mb["mass"]) < 1e-13  # periodic p: the filter keeps the mass
    assert ma["l2"] < mb["l2"]  # and removes the finest filaments
    # a zero-strength filter changes nothing
    zero = I.Params(**{**base.as_dict(), "filter_every": 1, "filter_strength": 0.0})
    assert np.array_equal(oracle.run(zero, f0, 5), oracle.run(base, f0, 5))


def test_strang_through_the_composition_is_the_paper_step(oracle):
    # one substep of weight 1: the drift tau = 0.5 (1.0 dt) and kick dt are those of Sec. 3
    p = I.Params(I.MODEL_SHEET, 48, 40, -10.0, 10.0, -4.0, 4.0, 0.05, bc_x=I.BC_ZERO)
    f0 = I.waterbag(p, 1.0, 0.5, 1e-4, 2)
    f = f0.copy()
    for _ in range(3):
        g = oracle.sweep_x(p, f, 0.5 * p.dt)
        F = oracle.force(p, oracle.density(p, g))[0]
        f = oracle.sweep_x(p, oracle.sweep_p(p, g, F, p.dt), 0.5 * p.dt)
    assert np.array_equal(oracle.run(p, f0, 3), f)
