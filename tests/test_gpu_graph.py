"""Steps replayed from HIP graphs (vlasov_set_graph) against the eager path
and the oracle: every replay, with the program's own eager work and
synchronisations between replays, must give the same bits."""
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


def _cases():
    th0, p0 = I.waterbag_halfwidths(0.5, 0.69)
    hmf = I.Params(I.MODEL_HMF, 300, 96, -math.pi, math.pi, -2.5, 2.5, 0.1)
    sheet = I.Params(I.MODEL_SHEET, 512, 256, -10.0, 10.0, -4.0, 4.0, 0.05, bc_x=I.BC_ZERO, storage=I.STORAGE_F32)
    ring = I.Params(I.MODEL_RING, 128, 80, -math.pi, math.pi, -3.0, 3.0, 0.05, ring_eps=0.01)
    suz = I.Params(I.MODEL_HMF, 128, 64, -math.pi, math.pi, -2.5, 2.5, 0.1, splitting=I.SPLIT_SUZUKI)
    return {
        "hmf": (hmf, I.waterbag(hmf, th0, p0, 1e-4, 1)),
        "sheet_f32": (sheet, I.waterbag(sheet, 1.0, 0.5, 1e-4, 2)),
        "ring": (ring, I.waterbag(ring, 1.131, 1.766, 1e-4, 3)),
        "suzuki": (suz, I.waterbag(suz, th0, p0, 1e-4, 4)),
    }


@pytest.mark.parametrize("name", ["hmf", "sheet_f32", "ring", "suzuki"])
def test_graph_replays_equal_eager_steps_and_oracle(V, oracle, name):
    p, f0 = _cases()[name]
    print(f"graph replays: {name} {p.nx}x{p.np_}", flush=True)
    calls = [9, 4, 13, 1, 7]  # with 3 steps per graph: 2, 1, 4, 0, 2 replays per call
    g = V.Solver(p, f0, hist_cap=64)
    g.set_graph(3)
    e = V.Solver(p, f0, hist_cap=64)
    e.set_graph(0)
    want = f0
    for n in calls:
        g.step(n)
        e.step(n)
        # eager work and synchronisations between the replays
        mg, me = g.moments(), e.moments()
        fg, fe = g.read_f(), e.read_f()
        assert np.array_equal(fg, fe), (name, n)
        assert mg == me
        if p.storage == I.STORAGE_F64:
            want = oracle.run(p, want, n)
            assert np.array_equal(fg, want), (name, n)
    assert np.array_equal(g.mag_history(), e.mag_history())
    g.close()
    e.close()


def test_graph_size_change_and_bounds(V):
    p, f0 = _cases()["hmf"]
    s = V.Solver(p, f0)
    with pytest.raises(V.VlasovError):
        s.set_graph(-1)
    with pytest.raises(V.VlasovError):
        s.set_graph(5000)
    s.set_graph(2)
    s.step(7)
    s.set_graph(5)  # drops the graphs of 2 steps
    s.step(7)
    got = s.read_f()
    s.close()
    r = V.Solver(p, f0)
    r.set_graph(0)
    r.step(14)
    assert np.array_equal(got, r.read_f())
    r.close()


def test_graphs_are_not_used_with_profiling_and_results_agree(V):
    p, f0 = _cases()["hmf"]
    a = V.Solver(p, f0)
    a.set_graph(4)
    a.profile(True)
    a.step(10)
    prof = a.profile_read()
    # every launch of the profiled call was timed on its own
    assert prof["kick_drift2"][1] + prof["kick"][1] == 10
    got = a.read_f()
    a.close()
    b = V.Solver(p, f0)
    b.set_graph(4)
    b.step(10)
    assert np.array_equal(got, b.read_f())
    b.close()
