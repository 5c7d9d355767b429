"""Where the error of FP32 storage comes from, request by request of the
parameter-scan serving trace.

For every request of the trace (or of one model), three runs of the same
initial condition on the device: FP64 storage (the reference, equal to the
CPU oracle bit for bit), FP32 storage, and FP64 storage started from the
initial condition with every nonzero value moved by one unit in the last
place (a perturbation far below the FP32 rounding of f, about 2^-24
relative).  If the FP64 run with the perturbed start departs from the
reference as much as the FP32 run does, the difference is the sensitivity of
the trajectory (filamentation, mass crossing the zero boundaries of the sheet
model) amplifying any rounding; if it stays near roundoff while FP32 departs,
FP32 storage itself is the cause.  Per request: the relative energy
difference, the magnetization difference, the mass that left the box, and the
fitted growth of the energy difference.

    python -m paper_1206_3229_amd.precision [--model sheet] [--requests 512] [--top 20]
"""
from __future__ import annotations

import argparse
import json
import math
import sys

import numpy as np

from . import inputs as I

MODELS = {"hmf": I.MODEL_HMF, "ring": I.MODEL_RING, "sheet": I.MODEL_SHEET}


def _run(V, p, f0, nsteps):
    s = V.Solver(p, f0)
    m0 = s.moments()
    s.step(nsteps)
    m = s.moments()
    f = s.read_f()
    s.close()
    return m0, m, f


def compare(V, q) -> dict:
    ic = V.ic_waterbag_um(q.U, q.M0, 1e-4, q.seed)
    p64 = I.Params(**{**q.params.as_dict(), "storage": I.STORAGE_F64})
    p32 = I.Params(**{**q.params.as_dict(), "storage": I.STORAGE_F32})
    # the FP64 initial condition, and the same moved by one ulp where nonzero
    s = V.Solver(p64, ic)
    f0 = s.read_f()
    s.close()
    f0p = np.where(f0 != 0.0, np.nextafter(f0, np.inf), 0.0)
    m0, m64, f64 = _run(V, p64, f0, q.nsteps)
    _, m32, f32 = _run(V, p32, f0, q.nsteps)
    _, mpp, fpp = _run(V, p64, f0p, q.nsteps)
    E = abs(m64["energy"])
    scale = float(np.max(np.abs(f64))) or 1.0
    return {
        "rid": q.rid, "model": q.params.model, "nx": q.params.nx, "np": q.params.np_, "dt": q.params.dt,
        "steps": q.nsteps, "U": q.U, "M0": q.M0,
        "energy_rel_f32": abs(m32["energy"] - m64["energy"]) / E,
        "energy_rel_f64_ulp": abs(mpp["energy"] - m64["energy"]) / E,
        "magnetization_f32": math.hypot(m32["mx"] - m64["mx"], m32["my"] - m64["my"]),
        "magnetization_f64_ulp": math.hypot(mpp["mx"] - m64["mx"], mpp["my"] - m64["my"]),
        "f_rel_f32": float(np.max(np.abs(f32 - f64))) / scale,
        "f_rel_f64_ulp": float(np.max(np.abs(fpp - f64))) / scale,
        "mass_lost_f64": m0["mass"] - m64["mass"],
        "energy_change_f64": (m64["energy"] - m0["energy"]) / abs(m0["energy"]),
    }


def study(V, model: str | None, nreq: int, top: int) -> dict:
    trace = I.serving_trace(nreq, seed=0, storage=I.STORAGE_F32)
    if model:
        trace = [q for q in trace if q.params.model == MODELS[model]]
    rows = []
    for k, q in enumerate(trace):
        rows.append(compare(V, q))
        if k % 20 == 19:
            print(f"precision: {k + 1} of {len(trace)} requests", file=sys.stderr, flush=True)
    rows.sort(key=lambda r: -r["energy_rel_f32"])
    worst = rows[:top]
    ratio = [r["energy_rel_f64_ulp"] / r["energy_rel_f32"] for r in rows if r["energy_rel_f32"] > 0]
    return {
        "requests": len(rows), "model": model or "all",
        "energy_rel_f32_max": rows[0]["energy_rel_f32"] if rows else None,
        "median_ratio_ulp_over_f32": float(np.median(ratio)) if ratio else None,
        "worst": worst,
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--model", choices=sorted(MODELS), default=None)
    ap.add_argument("--requests", type=int, default=512)
    ap.add_argument("--top", type=int, default=20)
    args = ap.parse_args()
    import torch
    from . import vlasov as V
    if not torch.cuda.is_available():
        raise SystemExit("precision: no GPU visible")
    V.load()
    print(json.dumps(study(V, args.model, args.requests, args.top)), flush=True)


if __name__ == "__main__":
    main()
