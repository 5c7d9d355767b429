"""The kick fused with the two half drifts after it: every tile shape gives
the same bits as the separate kick and drift kernels and as the oracle, on
ragged grids, both boundary rules on each axis, both storage types, and grids
whose drift shifts are too far apart within a tile to fuse (those fall back to
the separate kernels)."""
import math

import numpy as np
import pytest

from paper_1206_3229_amd import inputs as I

pytestmark = pytest.mark.gpu

# (kick_drift_width, kick_drift_blocks)
SHAPES = ((0, 1), (230, 1), (230, 2), (230, 3), (230, 4), (486, 1), (486, 4))


@pytest.fixture(scope="module")
def V():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1206_3229_amd import vlasov
    vlasov.load()
    return vlasov


def _log(msg):
    print(msg, flush=True)


def _hmf(nx, np_, dt=0.1, pmax=2.5, **kw):
    return I.Params(I.MODEL_HMF, nx, np_, -math.pi, math.pi, -pmax, pmax, dt, **kw)


def _sheet(nx, np_, dt=0.05, **kw):
    return I.Params(I.MODEL_SHEET, nx, np_, -10.0, 10.0, -4.0, 4.0, dt, bc_x=I.BC_ZERO, **kw)


CASES = {
    # name: (params, steps)
    "hmf600x50_ragged": (_hmf(600, 50, dt=0.01), 6),
    "hmf_zero_p_spread4": (_hmf(260, 45, bc_p=I.BC_ZERO), 6),
    "sheet300x40": (_sheet(300, 40, dt=0.04), 6),
    "sheet_zero_p": (_sheet(530, 36, dt=0.02, bc_p=I.BC_ZERO), 6),
    "ring96x64": (I.Params(I.MODEL_RING, 96, 64, -math.pi, math.pi, -3.0, 3.0, 0.05, ring_eps=0.01), 5),
    "sheet_odd_nx": (_sheet(515, 33, dt=0.02), 4),
    "hmf_f32": (_hmf(130, 70, storage=1), 6),
    "sheet_f32_zero_p": (_sheet(700, 48, dt=0.02, bc_p=I.BC_ZERO, storage=1), 5),
    "hmf1100x16": (_hmf(1100, 16, dt=0.005), 3),
    # one half drift fuses, two do not
    "hmf_mid_shift": (_hmf(96, 40, dt=0.42), 5),
    # never fusable
    "hmf_large_shift": (_hmf(96, 40, dt=9.7), 3),
}


def block_spread(p, rb=1):
    """Largest difference of the drift offsets (cells) within a tile of rb
    16-row blocks: the foot m_j = floor(-p_j (dt/2)/dx) of each row, clamped
    to +-(nx + 16) with zero extension in x.  Kick and the two half drifts
    after it fuse when 2 * spread <= 8."""
    dx, dp, tau = p.dx, p.dp, 0.5 * p.dt
    ms = []
    for j in range(p.np_):
        xi = -(((p.pmin + j * dp) * tau) / dx)
        m = math.floor(xi)
        if xi - m >= 1.0:
            m += 1
        if p.bc_x == I.BC_ZERO:
            m = max(-(p.nx + 16), min(p.nx + 16, m))
        ms.append(m)
    rows = 16 * rb
    return max(max(ms[b:b + rows]) - min(ms[b:b + rows]) for b in range(0, p.np_, rows))


def test_cases_cover_fused_and_fallback_paths():
    spreads = {k: block_spread(p) for k, (p, _) in CASES.items()}
    assert sum(2 * s <= 8 for s in spreads.values()) >= 8
    assert sum(2 * block_spread(p, 4) <= 8 for p, _ in CASES.values()) >= 6
    assert spreads["hmf_zero_p_spread4"] == 4
    assert 4 < spreads["hmf_mid_shift"] <= 8
    assert spreads["hmf_large_shift"] > 8


def _ic(p, seed=1):
    if p.model == I.MODEL_SHEET:
        return I.waterbag(p, 1.0, 0.5, 1e-4, seed)
    th0, p0 = I.waterbag_halfwidths(0.5, 0.69)
    return I.waterbag(p, th0, p0, 1e-4, seed)


def _run(V, p, f0, n, width, blocks):
    s = V.Solver(p, f0, hist_cap=n)
    s.set_tuning(128, 16, width, blocks)
    s.profile(True)
    s.step(n)
    prof = s.profile_read()
    out = (s.read_f(), s.mag_history(), prof)
    s.close()
    return out


@pytest.mark.parametrize("name", list(CASES))
def test_fused_equals_separate_and_oracle(V, oracle, name):
    p, n = CASES[name]
    f0 = _ic(p)
    _log(f"fused {name}: {p.nx}x{p.np_} bc {p.bc_x}{p.bc_p} storage {p.storage}, {n} steps")
    want, hist_want = oracle.run(p, f0, n, history=True)
    for w, b in SHAPES:
        f, hist, prof = _run(V, p, f0, n, w, b)
        assert np.array_equal(f, want, equal_nan=True), (name, w, b, float(np.nanmax(np.abs(f - want))))
        if p.model in (I.MODEL_HMF, I.MODEL_RING):
            assert np.array_equal(hist, hist_want), (name, w, b)
        fused = w != 0 and 2 * block_spread(p, b) <= 8
        if fused:
            assert prof["kick_drift2"][1] == n - 1 and prof["kick"][1] == 1, (name, w, b, prof)
        else:
            assert prof["kick_drift2"][1] == 0 and prof["kick"][1] == n, (name, w, b, prof)


def test_fused_single_step_calls(V, oracle):
    # one step per call: only the last-step form (kick + one half drift), which
    # runs as separate kernels; results are those of one four-step call
    p = _sheet(300, 40, dt=0.04)
    f0 = _ic(p)
    s = V.Solver(p, f0)
    s.set_tuning(128, 16, 486, 2)
    s.profile(True)
    for _ in range(4):
        s.step(1)
    prof = s.profile_read()
    got = s.read_f()
    s.close()
    assert prof["kick_drift2"][1] == 0 and prof["kick"][1] == 4
    assert np.array_equal(got, oracle.run(p, f0, 4))


def test_fused_tile_heights_on_a_ragged_grid(V, oracle):
    # 77 rows: tiles of 4 blocks leave a last tile of 13 rows
    p = _hmf(530, 77, dt=0.01)
    f0 = _ic(p, seed=4)
    want = oracle.run(p, f0, 5)
    assert 2 * block_spread(p, 4) <= 8
    for w, b in SHAPES:
        f, _, prof = _run(V, p, f0, 5, w, b)
        assert np.array_equal(f, want), (w, b)
        assert prof["kick_drift2"][1] == (4 if w else 0)
