"""Pins of the oracle's diagnostics against direct double sums (no GPU).

The quantities are those of the accuracy study of Sec. 4.1 (energy and norm)
and the Casimir int f^2 of eq. (casimirs); the potential energies are the
pair sums of Sec. 2 (eq. hamgen with eqs. hmfpot, ringpot, sheetpot) under
unit-mass normalisation, evaluated here with exactly rounded sums and
independently computed potentials.  Also pins the FP32 storage mode on the
cases where its result is fixed exactly (whole-cell rolls) or within FP32
rounding (cubics).
"""
import math

import numpy as np
import pytest

from paper_1206_3229_amd import inputs as I


def fsum(a):
    return math.fsum(np.asarray(a).ravel().tolist())


def brute(p, f):
    x = I.nodes(p.nx, p.xmin, p.xmax)
    v = I.nodes(p.np_, p.pmin, p.pmax)
    cell = p.dx * p.dp
    rho = np.array([p.dp * fsum(f[:, i]) for i in range(p.nx)])
    out = dict(mass=cell * fsum(f), momentum=cell * fsum(v[:, None] * f),
               kinetic=cell * fsum(0.5 * v[:, None] ** 2 * f), l2=cell * fsum(f * f))
    if p.model in (I.MODEL_HMF, I.MODEL_RING):
        out["mx"] = p.dx * fsum(np.cos(x) * rho)
        out["my"] = p.dx * fsum(np.sin(x) * rho)
    d = x[:, None] - x[None, :]
    pair = rho[:, None] * rho[None, :] * p.dx * p.dx
    if p.model == I.MODEL_HMF:
        out["potential"] = 0.5 * fsum((1.0 - np.cos(d)) * pair)
    elif p.model == I.MODEL_RING:
        V = -1.0 / np.sqrt(2.0 * (1.0 + p.ring_eps - np.cos(d)))
        out["potential"] = 0.5 * fsum(V * pair)
    elif p.model == I.MODEL_SHEET:
        out["potential"] = 0.5 * fsum(2.0 * math.pi * p.sheet_G * np.abs(d) * pair)
    return out


@pytest.mark.parametrize("model", [I.MODEL_HMF, I.MODEL_RING, I.MODEL_SHEET])
def test_moments_are_the_direct_sums(oracle, model):
    if model == I.MODEL_SHEET:
        p = I.Params(model, 48, 40, -3.0, 3.0, -2.0, 2.0, 0.1, bc_x=I.BC_ZERO, sheet_G=0.7)
    else:
        p = I.Params(model, 48, 40, -math.pi, math.pi, -2.0, 2.0, 0.1, ring_eps=0.05)
    f = np.random.default_rng(model + 7).uniform(0, 1, (p.np_, p.nx))
    got = oracle.moments(p, f)
    want = brute(p, f)
    for k, w in want.items():
        assert abs(got[k] - w) <= 1e-13 * max(1.0, abs(w)), (k, got[k], w)
    assert got["energy"] == got["kinetic"] + got["potential"]


def test_hmf_potential_of_uniform_state_is_half():
    # homogeneous unit mass: M = 0, W = 1/2 (eq. hmfpot averaged)
    p = I.Params(I.MODEL_HMF, 64, 32, -math.pi, math.pi, -2.0, 2.0, 0.1)
    f = np.ones((32, 64)) / (2 * math.pi * 4.0)
    from oracle import oracle as O
    m = O.moments(p, f)
    assert abs(m["mass"] - 1.0) < 1e-14 and abs(m["potential"] - 0.5) < 1e-14
    assert abs(m["mx"]) < 1e-15 and abs(m["my"]) < 1e-15


@pytest.mark.parametrize("q", [-9, -1, 0, 3, 40])
def test_fp32_whole_cell_roll_is_exact(oracle, q):
    line = np.random.default_rng(q + 50).standard_normal(48).astype(np.float32).astype(np.float64)
    got = oracle.interpolate_line(line, float(q), 0, 1)
    assert np.array_equal(got, np.roll(line, q))


def test_fp32_cubic_within_single_precision(oracle):
    n = 64
    u = np.arange(n, dtype=np.float64) - 30
    line = (0.3 - 0.02 * u + 0.004 * u ** 2 - 1e-4 * u ** 3).astype(np.float32).astype(np.float64)
    for shift in (0.37, -1.61):
        got = oracle.interpolate_line(line, shift, 1, 1)
        assert np.all(got == got.astype(np.float32))
        for i in range(16, 48):
            x = i - shift - 30
            want = 0.3 - 0.02 * x + 0.004 * x ** 2 - 1e-4 * x ** 3
            assert abs(got[i] - want) < 2e-5, (shift, i)


# ---------------------------------------------------------------------------
# Entropy -int f log f (eq. casimirs with s(f) = -f log f) over f > 0, and the
# negative mass the spline's overshoot can create.
# ---------------------------------------------------------------------------

def test_entropy_of_a_waterbag_is_minus_log_of_its_level(oracle):
    # f = c on K cells with c K dx dp = 1: S = -K dx dp c log c = -log c
    p, f0, _ = I.hmf_waterbag_small()
    f = (f0 > 0).astype(np.float64)
    f /= p.dx * p.dp * f.sum()
    c = float(f.max())
    m = oracle.moments(p, f)
    assert abs(m["entropy"] - (-math.log(c))) <= 1e-13 * abs(math.log(c))
    assert m["neg_mass"] == 0.0


def test_entropy_and_negative_mass_are_the_direct_sums(oracle):
    p = I.Params(I.MODEL_SHEET, 70, 45, -3.0, 3.0, -2.0, 2.0, 0.1, bc_x=I.BC_ZERO)
    f = np.random.default_rng(9).normal(0.2, 0.3, (p.np_, p.nx))  # about a quarter negative
    pos = f[f > 0]
    m = oracle.moments(p, f)
    cell = p.dx * p.dp
    want_s = -cell * fsum(pos * np.log(pos))
    want_n = cell * fsum(f[f < 0])
    assert (f < 0).sum() > 500
    assert abs(m["entropy"] - want_s) <= 1e-14 * cell * fsum(np.abs(pos * np.log(pos)))
    assert abs(m["neg_mass"] - want_n) <= 1e-14 * cell * fsum(np.abs(f[f < 0]))


def test_entropy_of_a_maxwellian_is_the_continuous_value(oracle):
    # f = exp(-p^2/2T) / (L sqrt(2 pi T)) uniform in x over a box of length L:
    # S = log L + log(2 pi T)/2 + 1/2 (the grid sum converges spectrally)
    T, L = 0.5, 2 * math.pi
    p = I.Params(I.MODEL_HMF, 32, 256, -math.pi, math.pi, -8.0, 8.0, 0.1)
    v = I.nodes(p.np_, p.pmin, p.pmax)
    f = np.repeat((np.exp(-v * v / (2 * T)) / (L * math.sqrt(2 * math.pi * T)))[:, None], p.nx, axis=1)
    m = oracle.moments(p, f)
    assert abs(m["entropy"] - (math.log(L) + 0.5 * math.log(2 * math.pi * T) + 0.5)) < 1e-12
    assert abs(m["mass"] - 1.0) < 1e-13
