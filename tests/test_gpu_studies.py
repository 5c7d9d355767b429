"""The accuracy studies on the device at their own sizes: the Table 2 energy
error of the sheet runs (n = 256 and 512 at dt = 0.1, printed with one digit)
and the HMF linear growth and damping rates on the 1024^2 grid against the
Vlasov dispersion relation."""
import json
import math
import os

import numpy as np
import pytest

from paper_1206_3229_amd import inputs as I

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "sheet_tables.json")


@pytest.fixture(scope="module")
def V():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1206_3229_amd import vlasov
    vlasov.load()
    return vlasov


def _one_digit(x: float) -> float:
    """x rounded to one significant digit (the precision the tables print)."""
    return float(f"{x:.0e}")


@pytest.mark.parametrize("n", [
    256,
    pytest.param(512, marks=pytest.mark.xfail(
        strict=True, reason="Table 2 prints 4e-4 at n = 512; this scheme gives 5.4e-4, the same splitting "
                            "error as at every other n (a stated discrepancy: the end time of the paper's "
                            "runs is not given)")),
])
def test_table_2_energy_error(V, n):
    # dt = 0.1, t = 100 (the end time the tables leave unstated); each printed
    # value is checked only to its one printed digit
    from paper_1206_3229_amd import conservation as Cn
    printed = json.load(open(GOLDEN))["fd"]["0.1"][str(n)][0]
    p = Cn.sheet_table_params(n, 0.1)
    r = Cn.track(V, p, I.waterbag(p, 1.0, 0.5), 1000, 10)
    assert r["delta_norm"] < 1e-4
    assert _one_digit(r["delta_e"]) == printed, r["delta_e"]


@pytest.mark.parametrize("T,rate", [(0.4, 0.116166), (0.6, -0.109956)])
def test_hmf_linear_rates_on_1024(V, T, rate):
    from paper_1206_3229_amd import dynamics as D
    p, f0, nsteps = I.hmf_gaussian(1024, T)
    r = D.run(V, p, f0, nsteps, 100)
    h = r["hist"]
    t = p.dt * (np.arange(len(h)) + 0.5)
    fit = D.fit_rate(t, np.hypot(h[:, 0], h[:, 1]), T < 0.5)
    assert fit is not None and abs(fit - rate) < 0.01 * abs(rate), fit
    assert r["delta_norm"] < 1e-12 and r["delta_e"] < 1e-5
