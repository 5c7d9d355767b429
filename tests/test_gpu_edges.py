"""Data at the zero-extension edges.

Random f0 over the whole grid puts nonzero samples at every edge, so every
clamped load, masked sample, first-pass zeroing near the x edges and masked
kicked column of the fused kernel meets data that a wrong mask or offset
would carry into the result.  Each case runs in every compiled launch shape
(separate kick and drift kernels in every thread and row count, and every
fused tile), for whole runs and for each sweep on its own, bitwise against
the oracle.  The last case is the box of the paper's Tables 1-2 (Sec. 4.1,
x and p in [-2, 2]) at 256^2, where mass leaves through the x edges."""
import math

import numpy as np
import pytest

from paper_1206_3229_amd import inputs as I

pytestmark = pytest.mark.gpu


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


def _sheet(nx, np_, dt, **kw):
    return I.Params(I.MODEL_SHEET, nx, np_, -3.0, 3.0, -2.0, 2.0, dt, bc_x=I.BC_ZERO, **kw)


def _ext(nx, np_, dt, **kw):
    return I.Params(I.MODEL_EXTERNAL, nx, np_, 0.0, 1.0, -1.0, 1.0, dt, bc_x=I.BC_ZERO, bc_p=I.BC_ZERO, **kw)


# name: (params, steps, external force or None)
CASES = {
    "sheet_zero_x": (_sheet(300, 64, 0.05), 6, None),
    "sheet_zero_x_and_p": (_sheet(530, 80, 0.03, bc_p=I.BC_ZERO), 5, None),
    "sheet_zero_x_and_p_odd_nx": (_sheet(515, 48, 0.03, bc_p=I.BC_ZERO), 4, None),
    "hmf_zero_p": (I.Params(I.MODEL_HMF, 260, 70, -math.pi, math.pi, -2.5, 2.5, 0.1, bc_p=I.BC_ZERO), 5, None),
    "sheet_zero_x_and_p_f32": (_sheet(530, 80, 0.03, bc_p=I.BC_ZERO, storage=1), 5, None),
    "hmf_zero_p_f32": (I.Params(I.MODEL_HMF, 260, 70, -math.pi, math.pi, -2.5, 2.5, 0.1, bc_p=I.BC_ZERO,
                                storage=1), 5, None),
    # kick shifts of up to 40 cells across the p edges, drift shifts of ~3 cells
    "external_zero_near": (_ext(200, 96, 0.0625), 4, "near"),
    # drift shifts of up to 100 cells (past the +-(n + 16) clamp of the
    # offsets) and kick shifts of up to 90 cells on a 64^2 grid
    "external_zero_far": (_ext(64, 64, 3.125), 3, "far"),
}


def _f0(p, seed=17):
    return np.random.default_rng(seed).uniform(-0.25, 1.0, (p.np_, p.nx))


def _force(p, kind):
    if kind is None:
        return None
    rng = np.random.default_rng(23)
    span = 40.0 if kind == "near" else 90.0
    q = rng.uniform(-span, span, p.nx)  # kick shift in cells, column by column
    return q * p.dp / p.dt


def _run(V, p, f0, n, Fext, shape, hist=0):
    s = V.Solver(p, f0, hist_cap=hist)
    s.set_tuning(*shape)
    if Fext is not None:
        s.set_external_force(Fext)
    s.profile(True)
    s.step(n)
    prof = s.profile_read()
    out = s.read_f(), s.mag_history(), prof
    s.close()
    return out


def test_cases_put_data_at_the_edges_and_reach_the_fused_kernel(V):
    fused = 0
    for name, (p, n, kind) in CASES.items():
        f0 = _f0(p)
        assert np.abs(f0[:, 0]).min() > 0 or np.abs(f0[:, -1]).max() > 0
        s = V.Solver(p, f0)
        s.set_tuning(128, 16, 230, 1)
        if kind is not None:
            s.set_external_force(_force(p, kind))
        s.profile(True)
        s.step(3)
        fused += s.profile_read()["kick_drift2"][1] > 0
        s.close()
    assert fused >= 6


@pytest.mark.parametrize("name", list(CASES))
def test_runs_in_every_launch_shape_match_the_oracle(V, oracle, name):
    p, n, kind = CASES[name]
    f0, Fext = _f0(p), _force(p, kind)
    want, hist_want = oracle.run(p, f0, n, F_ext=Fext, history=True)
    for shape in V.tuning_candidates():
        _log(f"edges {name}: {p.nx}x{p.np_} bc {p.bc_x}{p.bc_p} storage {p.storage}, shape {shape}")
        got, hist, _ = _run(V, p, f0, n, Fext, shape, hist=n)
        assert np.array_equal(got, want), (name, shape, float(np.max(np.abs(got - want))))
        if p.model in (I.MODEL_HMF, I.MODEL_RING):
            assert np.array_equal(hist, hist_want), (name, shape)


@pytest.mark.parametrize("name", list(CASES))
def test_each_sweep_matches_the_oracle(V, oracle, name):
    p, _, kind = CASES[name]
    f0, Fext = _f0(p), _force(p, kind)
    start = f0 if p.storage == 0 else f0.astype(np.float32).astype(np.float64)
    for shape in [(64, 8, 0, 1), (128, 16, 0, 1), (256, 32, 0, 1)]:
        _log(f"edge sweeps {name}, shape {shape}")
        s = V.Solver(p, f0)
        s.set_tuning(*shape)
        if Fext is not None:
            s.set_external_force(Fext)
        s.drift(2)
        g2 = s.read_f()
        s.drift(1)
        g3 = s.read_f()
        F, _ = s.force()
        s.kick()
        h = s.read_f()
        s.close()
        want2 = oracle.sweep_x(p, oracle.sweep_x(p, start, 0.5 * p.dt), 0.5 * p.dt)
        assert np.array_equal(g2, want2), (name, shape, "two half drifts")
        want3 = oracle.sweep_x(p, want2, 0.5 * p.dt)
        assert np.array_equal(g3, want3), (name, shape, "half drift")
        F_want, _ = oracle.force(p, oracle.density(p, want3), Fext)
        assert np.array_equal(F, F_want), (name, shape, "force")
        assert np.array_equal(h, oracle.sweep_p(p, want3, F_want, p.dt)), (name, shape, "kick")


@pytest.mark.parametrize("shape", [(128, 16, 0, 1), (128, 16, 230, 1), (128, 16, 486, 4)])
def test_tables_box_mass_leaves_through_the_x_edges(V, oracle, shape):
    # Sec. 4.1, Tables 1-2 setup at n = 256, dt = 0.1, t = 100 (1000 steps)
    from paper_1206_3229_amd import conservation as Cn
    p = Cn.sheet_table_params(256, 0.1)
    f0 = I.waterbag(p, 1.0, 0.5)
    n = 1000
    _log(f"tables box 256^2, {n} steps, shape {shape}")
    s = V.Solver(p, f0)
    s.set_tuning(*shape)
    s.step(n)
    got, mom = s.read_f(), s.moments()
    s.close()
    want = oracle.run(p, f0, n)
    assert np.array_equal(got, want)
    m_want = oracle.moments(p, want)
    for k in m_want:
        if k != "entropy":
            assert mom[k] == m_want[k], k
    # mass has left the box: far more than the roundoff of a closed run
    assert oracle.moments(p, f0)["mass"] - m_want["mass"] > 1e-7
