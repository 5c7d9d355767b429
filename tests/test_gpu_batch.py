"""Batched stepping and the request server: every grid's result in a batch,
and every request's result from the server, equals the CPU oracle run on the
same input (FP64 and FP32 storage, bit for bit; the entropy, whose log is the
device's, to a relative 1e-12) and the same grid stepped alone."""
import math
import time

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


def mixed_cases(storage):
    th0, p0 = I.waterbag_halfwidths(0.5, 0.69)
    out = []
    p = I.Params(I.MODEL_HMF, 128, 128, -math.pi, math.pi, -2.5, 2.5, 0.1, storage=storage)
    out.append((p, I.waterbag(p, th0, p0, 1e-4, 1), 10, None))
    p = I.Params(I.MODEL_RING, 96, 64, -math.pi, math.pi, -3.0, 3.0, 0.05, storage=storage, ring_eps=0.01)
    out.append((p, I.waterbag(p, th0, p0, 1e-4, 2), 7, None))
    p = I.Params(I.MODEL_SHEET, 200, 72, -10.0, 10.0, -4.0, 4.0, 0.05, bc_x=I.BC_ZERO, storage=storage)
    out.append((p, I.waterbag(p, 1.0, 0.5, 1e-4, 3), 12, None))
    p = I.Params(I.MODEL_EXTERNAL, 80, 48, 0.0, 1.0, -1.0, 1.0, 0.37, storage=storage)
    out.append((p, np.random.default_rng(5).uniform(0, 1, (48, 80)), 5, np.sin(np.linspace(0, 6, 80)) * 3.1))
    p = I.Params(I.MODEL_HMF, 600, 50, -math.pi, math.pi, -2.5, 2.5, 0.1, storage=storage)
    out.append((p, I.waterbag(p, th0, p0, 1e-4, 4), 0, None))
    p = I.Params(I.MODEL_HMF, 64, 512, -math.pi, math.pi, -2.5, 2.5, 0.05, storage=storage)
    out.append((p, I.gaussian(p, 0.4, 1e-3), 9, None))
    # wider grids: several drift tiles per row, both zero boundaries
    p = I.Params(I.MODEL_HMF, 1024, 40, -math.pi, math.pi, -2.5, 2.5, 0.01, storage=storage)
    out.append((p, I.waterbag(p, th0, p0, 1e-4, 6), 8, None))
    p = I.Params(I.MODEL_SHEET, 500, 37, -10.0, 10.0, -4.0, 4.0, 0.02, bc_x=I.BC_ZERO, bc_p=I.BC_ZERO,
                 storage=storage)
    out.append((p, I.waterbag(p, 1.0, 0.5, 1e-4, 7), 6, None))
    # coarse p, fine x, long steps: drift offsets spreading by 20 columns
    # inside a 16-row tile (the batched fused kernel's wide-slack tiles; the
    # EXTERNAL grid above spreads by 20 too, on a periodic x axis)
    p = I.Params(I.MODEL_SHEET, 700, 40, -10.0, 10.0, -4.0, 4.0, 0.2, bc_x=I.BC_ZERO, storage=storage)
    out.append((p, I.waterbag(p, 1.0, 0.5, 1e-4, 8), 7, None))
    # a spread beyond the wide tiles' slack (about 110 columns): never fused
    p = I.Params(I.MODEL_HMF, 1000, 32, -math.pi, math.pi, -2.5, 2.5, 0.3, storage=storage)
    out.append((p, I.waterbag(p, th0, p0, 1e-4, 9), 3, None))
    return out


def assert_moments(got, want, what=""):
    assert set(got) == set(want)
    for k in want:
        if k == "entropy":
            assert abs(got[k] - want[k]) <= 1e-12 * max(1.0, abs(want[k])), (what, k, got[k], want[k])
        else:
            assert got[k] == want[k], (what, k, got[k], want[k])


def _oracle(oracle, p, f0, n, Fext):
    f, h = oracle.run(p, f0, n, F_ext=Fext, history=True)
    return f, h, (oracle.moments(p, f) if np.isfinite(f).all() else None)


def _solo(V, p, f0, n, Fext, hist=0):
    s = V.Solver(p, f0, hist_cap=hist)
    if Fext is not None:
        s.set_external_force(Fext)
    s.step(n)
    out = (s.read_f(), s.moments() if np.isfinite(s.read_f()).all() else None, s.mag_history())
    s.close()
    return out


@pytest.mark.parametrize("storage", [0, 1])
@pytest.mark.parametrize("chunk,graph,fuse", [(4, True, False), (16, False, False), (3, True, True), (5, False, True)])
def test_batch_equals_oracle_and_each_grid_alone(V, oracle, storage, chunk, graph, fuse):
    cases = mixed_cases(storage)
    _log(f"batch storage={storage} chunk={chunk} graph={graph} fuse={fuse}")
    solvers = []
    for p, f0, n, Fext in cases:
        s = V.Solver(p, f0, hist_cap=16)
        s.set_tuning(128, 16, 230, 2)
        if Fext is not None:
            s.set_external_force(Fext)
        solvers.append(s)
    V.batch_step(solvers, [c[2] for c in cases], chunk_cycles=chunk, use_graph=graph, fuse=fuse)
    for s, (p, f0, n, Fext) in zip(solvers, cases):
        what = (p.model, p.nx, p.np_, p.storage)
        # the batched fused tiles are one 16-row block tall
        assert s.get_tuning()[2:] == ((230, 1) if fuse else (230, 2)), what
        f, h, m = s.read_f(), s.mag_history(), s.moments()
        f_ref, h_ref, m_ref = _oracle(oracle, p, f0, n, Fext)
        assert np.array_equal(f, f_ref), what
        if p.model in (I.MODEL_HMF, I.MODEL_RING):
            assert np.array_equal(h, h_ref), what
        assert_moments(m, m_ref, what)
        f_solo, m_solo, h_solo = _solo(V, p, f0, n, Fext, hist=16)
        assert np.array_equal(f, f_solo), what
        assert np.array_equal(h, h_solo)
        assert m == m_solo
        s.close()


def _drift_spread(p):
    """Largest spread of the summed drift offsets o_j = 2 m_j over the rows of
    a 16-row tile (plain splitting: both half drifts share one table), m_j the
    foot cell of the half drift of row j with the tie rule of the oracle."""
    dx = (p.xmax - p.xmin) / p.nx
    dp = (p.pmax - p.pmin) / p.np_
    pj = p.pmin + np.arange(p.np_) * dp
    xi = -(pj * (p.dt / 2)) / dx
    m = np.floor(xi)
    m = np.where(xi - m >= 1, m + 1, m)
    o = 2 * m
    return int(max(o[j:j + 16].max() - o[j:j + 16].min() for j in range(0, p.np_, 16)))


@pytest.mark.parametrize("storage", [0, 1])
def test_fused_batch_at_the_wide_tiles_slack(V, oracle, storage):
    # offsets spreading by exactly the wide tiles' 56 columns of slack (the
    # last kicked column of a tile is read) and by 58 (never fused), beside a
    # member on the narrow tiles, in one fused batch
    th0, p0 = I.waterbag_halfwidths(0.5, 0.69)
    cases = []
    for k, (nx, dt, want) in enumerate(((1000, 0.225, 56), (1000, 0.23, 58), (128, 0.1, 4))):
        p = I.Params(I.MODEL_HMF, nx, 48, -math.pi, math.pi, -2.5, 2.5, dt, storage=storage)
        assert _drift_spread(p) == want
        cases.append((p, I.waterbag(p, th0, p0, 1e-4, 20 + k), 3 + k, None))
    _log(f"fused batch at the wide slack, storage={storage}")
    solvers = [V.Solver(p, f0, hist_cap=8) for p, f0, _, _ in cases]
    V.batch_step(solvers, [c[2] for c in cases], chunk_cycles=2, use_graph=True, fuse=True)
    for s, (p, f0, n, Fext) in zip(solvers, cases):
        what = (p.nx, p.dt, p.storage)
        f, h, m = s.read_f(), s.mag_history(), s.moments()
        f_ref, h_ref, m_ref = _oracle(oracle, p, f0, n, Fext)
        assert np.array_equal(f, f_ref), what
        assert np.array_equal(h, h_ref), what
        assert_moments(m, m_ref, what)
        f_solo, m_solo, _ = _solo(V, p, f0, n, Fext)
        assert np.array_equal(f, f_solo), what
        assert m == m_solo
        s.close()


def test_batch_then_single_steps_continue(V):
    # a context stepped in a batch can go on with vlasov_step
    p, f0, _ = I.hmf_waterbag_small()
    a = V.Solver(p, f0)
    V.batch_step([a], [6], chunk_cycles=4)
    a.step(5)
    b = V.Solver(p, f0)
    b.step(11)
    assert np.array_equal(a.read_f(), b.read_f())
    a.close()
    b.close()


def test_batch_rejects_mixed_storage(V):
    p64, f0, _ = I.hmf_waterbag_small()
    p32 = I.Params(**{**p64.as_dict(), "storage": 1})
    a, b = V.Solver(p64, f0), V.Solver(p32, f0)
    with pytest.raises(V.VlasovError) as e:
        V.batch_step([a, b], [1, 1])
    assert e.value.code == V.E_INVAL
    with pytest.raises(V.VlasovError):
        V.batch_step([a, a], [1, 1])
    a.close()
    b.close()


def _serve(V, cases, storage, arena_bytes, max_slots=8, chunk=8, fuse=False):
    srv = V.Server(arena_bytes, storage=storage, max_slots=max_slots, chunk_cycles=chunk, fuse=fuse)
    tickets = []
    for p, f0, n, Fext in cases:
        tickets.append(srv.submit(p, f0, n, keep_f=True))
    results = {}
    t_end = time.time() + 120
    while len(results) < len(tickets) and time.time() < t_end:
        for t in tickets:
            if t not in results:
                r = srv.poll(t)
                if r is not None:
                    results[t] = r
        time.sleep(0.002)
    srv.close()
    assert len(results) == len(tickets), "server did not finish"
    return [results[t] for t in tickets]


@pytest.mark.parametrize("storage,fuse", [(1, False), (0, False), (1, True)])
def test_server_results_equal_oracle_and_solo_runs(V, oracle, storage, fuse):
    cases = [c for c in mixed_cases(storage) if c[3] is None]
    # arena for roughly two requests at a time: admission must queue
    need = max(V.request_footprint(c[0]) for c in cases)
    tables = V.load().vlasov_server_table_bytes(8)
    _log(f"server storage={storage} fuse={fuse}, arena {tables + 2 * need} bytes")
    res = _serve(V, cases, storage, tables + 2 * need + 4096, fuse=fuse)
    for (r, f), (p, f0, n, _) in zip(res, cases):
        what = (p.model, p.nx, p.np_, p.storage)
        assert r["status"] == 0 and r["steps_done"] == n
        f_ref, _, m_ref = _oracle(oracle, p, f0, n, None)
        assert np.array_equal(f, f_ref), what
        assert_moments(r["moments"], m_ref, what)
        f_solo, m_solo, _ = _solo(V, p, f0, n, None)
        assert np.array_equal(f, f_solo), what
        assert r["moments"] == m_solo
        assert r["t_submit"] <= r["t_admit"] <= r["t_done"]


@pytest.mark.parametrize("storage", [1, 0])
@pytest.mark.parametrize("fuse", [False, True])
def test_server_mix_of_many_requests(V, oracle, storage, fuse):
    # 24 requests of the parameter scan (three models, uneven sides up to 512),
    # six at a time: every result equals the oracle on the same input
    trace = I.serving_trace(24, seed=3, sides=(64, 128, 256, 512), steps_range=(5, 40), storage=storage)
    cases = [(q.params, q.initial_condition(), q.nsteps, None) for q in trace]
    _log(f"server mix storage={storage} fuse={fuse}")
    res = _serve(V, cases, storage, 96 << 20, max_slots=6, chunk=8, fuse=fuse)
    for (r, f), (p, f0, n, _) in zip(res, cases):
        what = (p.model, p.nx, p.np_, n)
        assert r["status"] == 0 and r["steps_done"] == n
        f_ref, _, m_ref = _oracle(oracle, p, f0, n, None)
        assert np.array_equal(f, f_ref), what
        assert_moments(r["moments"], m_ref, what)
    for i in (0, 7, 23):
        (r, f), (p, f0, n, _) = res[i], cases[i]
        f_solo, m_solo, _ = _solo(V, p, f0, n, None)
        assert np.array_equal(f, f_solo)
        assert r["moments"] == m_solo


def test_every_launch_shape_gives_identical_results(V, oracle):
    p = I.Params(I.MODEL_SHEET, 600, 90, -10.0, 10.0, -4.0, 4.0, 0.05, bc_x=I.BC_ZERO)
    f0 = I.waterbag(p, 1.0, 0.5, 1e-4, 3)
    ref = oracle.run(p, f0, 7)
    for shape in V.tuning_candidates():
        s = V.Solver(p, f0)
        s.set_tuning(*shape)
        assert s.get_tuning() == shape
        s.step(7)
        f = s.read_f()
        s.close()
        assert np.array_equal(f, ref), shape
    assert {c[2] for c in V.tuning_candidates()} == {0, 230, 486}
    s = V.Solver(p, f0)
    with pytest.raises(V.VlasovError):
        s.set_tuning(96, 16)
    with pytest.raises(V.VlasovError):
        s.set_tuning(128, 16, 384)
    with pytest.raises(V.VlasovError):
        s.set_tuning(128, 16, 230, 5)
    s.close()


def test_autotune_picks_a_compiled_shape(V, tmp_path, monkeypatch):
    from paper_1206_3229_amd import autotune
    monkeypatch.setenv("VLASOV_TUNE_CACHE", str(tmp_path / "tune.json"))
    p, f0, _ = I.hmf_waterbag_small()
    best = autotune.tune(p, f0, steps=3, reps=1)
    assert (best["drift_threads"], best["kick_rows"], best["kick_drift_width"],
            best["kick_drift_blocks"]) in V.tuning_candidates()
    assert len(best["table"]) == len(V.tuning_candidates())
    assert autotune.tune(p, f0)["us_per_step"] == best["us_per_step"]  # served from the cache


def test_server_chunk_failure_fails_the_running_requests(V, oracle, monkeypatch):
    # a failure of the third chunk, injected on the host after its planning and
    # before anything is enqueued: the three requests running then come back
    # with the error and the steps finished before it, and the server goes on
    # with a request submitted afterwards
    th0, p0 = I.waterbag_halfwidths(0.5, 0.69)
    p = I.Params(I.MODEL_HMF, 64, 64, -math.pi, math.pi, -2.5, 2.5, 0.1, storage=1)
    monkeypatch.setenv("VLASOV_TEST_FAIL_CHUNK", "2")
    srv = V.Server(64 << 20, storage=1, max_slots=8, chunk_cycles=4)
    monkeypatch.delenv("VLASOV_TEST_FAIL_CHUNK")
    f0s = [I.waterbag(p, th0, p0, 1e-4, k) for k in range(4)]

    def wait(t):
        t_end = time.time() + 60
        while time.time() < t_end:
            r = srv.poll(t)
            if r is not None:
                return r
            time.sleep(0.002)
        raise AssertionError("server did not finish")

    # submitted together: all three are running when the third chunk fails
    tickets = [srv.submit(p, f0s[k], 50, keep_f=True) for k in range(3)]
    done = []
    for t in tickets:
        r, f = wait(t)
        assert r["status"] == V.E_HIP and f is None
        assert 0 <= r["steps_done"] < 50
        done.append(r["steps_done"])
    assert max(done) > 0  # the first admitted finished two chunks before the failure
    later = srv.submit(p, f0s[3], 10, keep_f=True)
    r, f = wait(later)
    srv.close()
    assert r["status"] == 0 and r["steps_done"] == 10
    assert np.array_equal(f, _oracle(oracle, p, f0s[3], 10, None)[0])
