"""The oracle's parallel loops split the work over whole lines and sum over
lines in line order afterwards, so its results must not depend on the number
of threads: one thread and several give the same bits, for every model, both
splines, both storage types, the fourth-order splitting and the filter, and
every diagnostic."""
import math
import os

import numpy as np
import pytest

from paper_1206_3229_amd import inputs as I

TH0, P0 = I.waterbag_halfwidths(0.5, 0.69)

CASES = {
    "hmf": (I.Params(I.MODEL_HMF, 200, 136, -math.pi, math.pi, -2.5, 2.5, 0.1), 5),
    "ring": (I.Params(I.MODEL_RING, 160, 72, -math.pi, math.pi, -3.0, 3.0, 0.05, ring_eps=0.01), 4),
    "sheet_zero_x_and_p": (I.Params(I.MODEL_SHEET, 230, 96, -3.0, 3.0, -2.0, 2.0, 0.2, bc_x=I.BC_ZERO,
                                    bc_p=I.BC_ZERO), 5),
    "hmf_f32": (I.Params(I.MODEL_HMF, 150, 80, -math.pi, math.pi, -2.5, 2.5, 0.1, storage=1), 5),
    "sheet_global_spline": (I.Params(I.MODEL_SHEET, 128, 100, -3.0, 3.0, -2.0, 2.0, 0.2, bc_x=I.BC_ZERO,
                                     spline=I.SPLINE_GS), 3),
    "hmf_global_spline": (I.Params(I.MODEL_HMF, 96, 130, -math.pi, math.pi, -2.5, 2.5, 0.1,
                                   spline=I.SPLINE_GS), 3),
    "hmf_triple_jump_filter": (I.Params(I.MODEL_HMF, 100, 90, -math.pi, math.pi, -2.5, 2.5, 0.1,
                                        splitting=I.SPLIT_TRIPLE_JUMP, filter_every=2, filter_strength=0.7), 4),
}


def _ic(p):
    if p.model == I.MODEL_SHEET:
        return I.waterbag(p, 1.0, 0.5, 1e-4, 4)
    return I.waterbag(p, TH0, P0, 1e-4, 4)


@pytest.mark.parametrize("name", list(CASES))
def test_results_do_not_depend_on_the_thread_count(oracle, name):
    p, n = CASES[name]
    f0 = _ic(p)
    many = max(2, min(8, os.cpu_count() or 2))
    out = []
    try:
        for t in (1, many):
            oracle.set_threads(t)
            assert oracle.threads() == t
            f, h = oracle.run(p, f0, n, history=True)
            out.append((f, h, oracle.moments(p, f), oracle.density(p, f), oracle.force(p, oracle.density(p, f))))
    finally:
        oracle.set_threads(os.cpu_count() or 1)
    (f1, h1, m1, r1, F1), (f2, h2, m2, r2, F2) = out
    assert np.array_equal(f1, f2)
    assert np.array_equal(h1, h2)
    assert m1 == m2
    assert np.array_equal(r1, r2)
    assert np.array_equal(F1[0], F2[0]) and F1[1] == F2[1]
