"""Higher-order splitting and the p-filter on the device against the oracle:
bit for bit with the local spline (every substep's drift tables, the kicks of
size w_k dt, the filter after the last kick of every k-th step), with the
fused and the separate kernels, across calls of any length, and to rounding
with the global spline."""
import math

import numpy as np
import pytest

from paper_1206_3229_amd import inputs as I

pytestmark = pytest.mark.gpu

SCHEMES = (I.SPLIT_STRANG, I.SPLIT_TRIPLE_JUMP, I.SPLIT_SUZUKI)
NSUB = {I.SPLIT_STRANG: 1, I.SPLIT_TRIPLE_JUMP: 3, I.SPLIT_SUZUKI: 5}


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


def _with(p, **kw):
    return I.Params(**{**p.as_dict(), **kw})


CASES = {
    "hmf128": I.Params(I.MODEL_HMF, 128, 128, -math.pi, math.pi, -2.5, 2.5, 0.1),
    "hmf600x50_f32": I.Params(I.MODEL_HMF, 600, 50, -math.pi, math.pi, -2.5, 2.5, 0.01, storage=1),
    "sheet300x40": I.Params(I.MODEL_SHEET, 300, 40, -10.0, 10.0, -4.0, 4.0, 0.04, bc_x=I.BC_ZERO),
    "sheet_zero_p": I.Params(I.MODEL_SHEET, 530, 36, -10.0, 10.0, -4.0, 4.0, 0.02, bc_x=I.BC_ZERO, bc_p=I.BC_ZERO),
    "ring96x64": I.Params(I.MODEL_RING, 96, 64, -math.pi, math.pi, -3.0, 3.0, 0.05, ring_eps=0.01),
    # large shifts: no pair of substeps fuses
    "hmf_large_shift": I.Params(I.MODEL_HMF, 96, 40, -math.pi, math.pi, -2.5, 2.5, 2.3),
}


def _ic(p, seed=1):
    if p.model == I.MODEL_SHEET:
        return I.waterbag(p, 1.0, 0.5, 1e-4, seed)
    th0, p0 = I.waterbag_halfwidths(0.5, 0.69)
    return I.waterbag(p, th0, p0, 1e-4, seed)


def _run(V, p, f0, calls, shape=None, hist=0):
    s = V.Solver(p, f0, hist_cap=hist)
    if shape is not None:
        s.set_tuning(*shape)
    s.profile(True)
    for n in calls:
        s.step(n)
    out = (s.read_f(), s.mag_history(), s.profile_read())
    s.close()
    return out


@pytest.mark.parametrize("scheme", SCHEMES)
@pytest.mark.parametrize("name", list(CASES))
def test_splitting_matches_oracle_bitwise(V, oracle, name, scheme):
    p = _with(CASES[name], splitting=scheme)
    f0 = _ic(p)
    n = 5
    want, hist_want = oracle.run(p, f0, n, history=True)
    _log(f"splitting {scheme} {name}")
    for shape in ((128, 16, 230, 1), (128, 16, 486, 2), (128, 16, 0, 1)):
        got, hist, prof = _run(V, p, f0, [n], shape, hist=n * NSUB[scheme])
        assert np.array_equal(got, want), (name, scheme, shape, float(np.max(np.abs(got - want))))
        if p.model in (I.MODEL_HMF, I.MODEL_RING):
            assert np.array_equal(hist, hist_want), (name, scheme, shape)
        evals = n * NSUB[scheme]
        assert prof["force"][1] >= evals
        assert prof["kick_drift2"][1] + prof["kick"][1] == evals
        if shape[2] == 0:
            assert prof["kick_drift2"][1] == 0


@pytest.mark.parametrize("scheme", [I.SPLIT_TRIPLE_JUMP, I.SPLIT_SUZUKI])
def test_substeps_fuse_where_the_tables_allow(V, oracle, scheme):
    # small shifts: every pair of consecutive half drifts fuses with its kick
    p = _with(CASES["hmf600x50_f32"], splitting=scheme)
    f0 = _ic(p)
    got, _, prof = _run(V, p, f0, [4], (128, 16, 230, 1))
    assert prof["kick_drift2"][1] == 4 * NSUB[scheme] - 1 and prof["kick"][1] == 1
    assert np.array_equal(got, oracle.run(p, f0, 4))


def test_calls_of_any_length_give_the_same_bits(V, oracle):
    p = _with(CASES["sheet300x40"], splitting=I.SPLIT_TRIPLE_JUMP, filter_every=3, filter_strength=0.5)
    f0 = _ic(p, 2)
    want = oracle.run(p, f0, 8)
    for calls in ([8], [1, 1, 1, 1, 1, 1, 1, 1], [2, 5, 1], [3, 3, 2]):
        got, _, _ = _run(V, p, f0, calls)
        assert np.array_equal(got, want), calls


@pytest.mark.parametrize("storage", [0, 1])
@pytest.mark.parametrize("bc_p", [I.BC_PERIODIC, I.BC_ZERO])
@pytest.mark.parametrize("every", [1, 3])
def test_filter_matches_oracle_bitwise(V, oracle, storage, bc_p, every):
    p = I.Params(I.MODEL_HMF, 260, 45, -math.pi, math.pi, -2.5, 2.5, 0.1, bc_p=bc_p, storage=storage,
                 filter_every=every, filter_strength=0.7)
    f0 = _ic(p, 3)
    want = oracle.run(p, f0, 7)
    _log(f"filter storage={storage} bc_p={bc_p} every={every}")
    for shape in ((128, 16, 230, 1), (128, 16, 0, 1)):
        got, _, prof = _run(V, p, f0, [7], shape)
        assert np.array_equal(got, want), (storage, bc_p, every, shape)
        assert prof["filter"][1] == 7 // every


def test_filter_with_suzuki_on_a_sheet(V, oracle):
    p = _with(CASES["sheet_zero_p"], splitting=I.SPLIT_SUZUKI, filter_every=2, filter_strength=1.0)
    f0 = _ic(p, 4)
    got, _, _ = _run(V, p, f0, [5])
    assert np.array_equal(got, oracle.run(p, f0, 5))


def test_harmonic_well_means_follow_the_composed_map(V, oracle):
    # the device reproduces the oracle's fourth-order means (see the oracle pins)
    n = 16
    p = I.Params(I.MODEL_EXTERNAL, 128, 128, -8.0, 8.0, -8.0, 8.0, 2 * math.pi / n,
                 splitting=I.SPLIT_TRIPLE_JUMP)
    x = p.xmin + np.arange(p.nx) * p.dx
    pp = p.pmin + np.arange(p.np_) * p.dp
    f0 = np.exp(-((x[None, :] - 1.5) ** 2 + pp[:, None] ** 2) / (2 * 0.5 ** 2))
    s = V.Solver(p, f0)
    s.set_external_force(-x)
    s.step(n)
    got = s.read_f()
    s.close()
    assert np.array_equal(got, oracle.run(p, f0, n, F_ext=-x))
    m = got.sum()
    assert abs((got.sum(0) @ x) / m - 1.5) < 2e-2 and abs((got.sum(1) @ pp) / m) < 2e-2


@pytest.mark.parametrize("scheme", [I.SPLIT_TRIPLE_JUMP, I.SPLIT_SUZUKI])
def test_global_spline_with_splitting_and_filter(V, oracle, scheme):
    p = I.Params(I.MODEL_HMF, 128, 64, -math.pi, math.pi, -2.5, 2.5, 0.1, splitting=scheme,
                 spline=I.SPLINE_GS, filter_every=2, filter_strength=0.5)
    f0 = _ic(p, 5)
    got, _, _ = _run(V, p, f0, [4])
    want = oracle.run(p, f0, 4)
    assert np.max(np.abs(got - want)) <= 1e-11 * np.max(np.abs(want))


def test_individual_sweeps_use_the_first_substep(V, oracle):
    p = _with(CASES["hmf128"], splitting=I.SPLIT_TRIPLE_JUMP)
    f0 = _ic(p)
    w0 = oracle.split_weights(p.splitting)[0]
    s = V.Solver(p, f0)
    s.drift(1)
    got = s.read_f()
    s.force()
    s.kick()
    got2 = s.read_f()
    s.close()
    g = oracle.sweep_x(p, f0, 0.5 * (w0 * p.dt))
    assert np.array_equal(got, g)
    F = oracle.force(p, oracle.density(p, g))[0]
    assert np.array_equal(got2, oracle.sweep_p(p, g, F, w0 * p.dt))


def test_batches_and_server_reject_other_splittings_and_the_filter(V):
    for kw in (dict(splitting=I.SPLIT_TRIPLE_JUMP), dict(filter_every=1, filter_strength=0.5)):
        p = _with(CASES["hmf128"], **kw)
        f0 = _ic(p)
        s = V.Solver(p, f0)
        with pytest.raises(V.VlasovError) as e:
            V.batch_step([s], [2])
        assert e.value.code == V.E_INVAL
        s.close()
        srv = V.Server(64 << 20, storage=0, max_slots=2)
        with pytest.raises(V.VlasovError):
            srv.submit(p, f0, 3)
        srv.close()
