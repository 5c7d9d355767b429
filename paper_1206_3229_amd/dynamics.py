"""The HMF stability study (Sec. 4.2) and the ring runs (Sec. 4.3) at the
workloads' full sizes: the magnetization growth or damping rate fitted to the
per-step history, the largest relative energy and mass drift, and the
FP32-storage runs against the FP64 ones.

HMF: f proportional to exp(-p^2/2T)(1 + 1e-3 cos theta) at T = 0.4 (unstable,
linear growth rate 0.116166 of the Vlasov dispersion relation) and T = 0.6
(stable, the least-damped mode decays at 0.109956), dt = 0.05, 2000 steps, on
1024^2 and 2048^2 grids.  The rate is the least-squares slope of ln|M| over
the linear phase: |M| between 2e-3 and 2e-2 while it grows (T = 0.4), t in
[10, 60] while it decays (T = 0.6).  Ring: the waterbag at M0 = 0.8, e = 0.7,
eps = 0.01, dt = 0.02, 1000 steps on 2048^2.

    python -m paper_1206_3229_amd.dynamics [--sizes 1024,2048] [--every 20]
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np

from . import inputs as I


def fit_rate(t: np.ndarray, m: np.ndarray, growing: bool) -> float | None:
    """Slope of ln|M| over the linear phase, or None if it is too short."""
    if growing:
        sel = (m > 2e-3) & (m < 2e-2)
        # the first passage only (the nonlinear phase can dip back into the band)
        if sel.any():
            first = np.argmax(sel)
            end = first + np.argmin(sel[first:]) if not sel[first:].all() else len(sel)
            sel = np.zeros_like(sel)
            sel[first:end] = True
    else:
        sel = (t >= 10.0) & (t <= 60.0)
    if sel.sum() < 5:
        return None
    return float(np.polyfit(t[sel], np.log(m[sel]), 1)[0])


def run(V, p, f0, nsteps: int, every: int) -> dict:
    s = V.Solver(p, f0, hist_cap=nsteps)
    m0 = s.moments()
    e_max = n_max = 0.0
    done = 0
    t0 = time.perf_counter()
    while done < nsteps:
        k = min(every, nsteps - done)
        s.step(k)
        done += k
        m = s.moments()
        e_max = max(e_max, abs(m["energy"] - m0["energy"]) / abs(m0["energy"]))
        n_max = max(n_max, abs(m["mass"] - m0["mass"]) / abs(m0["mass"]))
    secs = time.perf_counter() - t0
    hist = s.mag_history()
    last = s.moments()
    s.close()
    return {"hist": hist, "delta_e": e_max, "delta_norm": n_max, "energy_end": last["energy"],
            "seconds": secs}


def study(V, sizes=(1024, 2048), every: int = 20) -> list[dict]:
    rows = []
    cases = []
    for n in sizes:
        for T in (0.4, 0.6):
            cases.append((f"hmf_gaussian_{n}_T{T}", lambda st, n=n, T=T: I.hmf_gaussian(n, T, storage=st), T))
    cases.append(("ring_2048", lambda st: I.ring_waterbag(2048, storage=st), None))
    for name, mk, T in cases:
        res = {}
        for storage in (I.STORAGE_F64, I.STORAGE_F32):
            p, f0, nsteps = mk(storage)
            res[storage] = run(V, p, f0, nsteps, every)
        h64, h32 = res[0]["hist"], res[1]["hist"]
        t = p.dt * (np.arange(len(h64)) + 0.5)  # the force of step k acts at its middle
        m64 = np.hypot(h64[:, 0], h64[:, 1])
        row = {"case": name, "nx": p.nx, "np": p.np_, "dt": p.dt, "steps": nsteps,
               "delta_e_f64": res[0]["delta_e"], "delta_norm_f64": res[0]["delta_norm"],
               "delta_e_f32": res[1]["delta_e"], "delta_norm_f32": res[1]["delta_norm"],
               "f32_vs_f64_M_max_abs": float(np.max(np.abs(h32 - h64))),
               "f32_vs_f64_energy_rel": abs(res[1]["energy_end"] - res[0]["energy_end"]) / abs(res[0]["energy_end"]),
               "M_end_f64": float(m64[-1]), "seconds_f64": res[0]["seconds"], "seconds_f32": res[1]["seconds"]}
        if T is not None:
            row["T"] = T
            row["rate_f64"] = fit_rate(t, m64, T < 0.5)
            row["rate_f32"] = fit_rate(t, np.hypot(h32[:, 0], h32[:, 1]), T < 0.5)
            row["rate_theory"] = 0.116166 if T < 0.5 else -0.109956
        rows.append(row)
    return rows


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--sizes", default="1024,2048")
    ap.add_argument("--every", type=int, default=20)
    args = ap.parse_args()
    import torch
    from . import vlasov as V
    if not torch.cuda.is_available():
        raise SystemExit("dynamics: no GPU visible")
    V.load()
    for row in study(V, tuple(int(v) for v in args.sizes.split(",")), args.every):
        print(json.dumps(row), flush=True)


if __name__ == "__main__":
    main()
