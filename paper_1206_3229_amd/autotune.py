"""Launch-shape autotuner.

Times every compiled launch shape (threads per drift workgroup, rows per kick
thread, separate or fused kick and drift and the fused tile width) on the
device for one grid, keeps the
fastest and caches it in a JSON file keyed by the GPU architecture, the
storage type, the grid size and the boundaries.  All shapes compute the same
arithmetic, so the choice changes speed only, never results.

Cache: $VLASOV_TUNE_CACHE, else ~/.cache/vlasov_tuning.json.
"""
from __future__ import annotations

import json
import os

import numpy as np

from . import vlasov as V


def cache_path() -> str:
    return os.environ.get("VLASOV_TUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "vlasov_tuning.json"))


def _key(arch: str, p) -> str:
    return f"{arch}|s{p.storage}|{p.nx}x{p.np_}|bc{p.bc_x}{p.bc_p}|dt{p.dt!r}|v3"


def _load_cache() -> dict:
    try:
        with open(cache_path()) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def _store(key: str, entry: dict):
    path = cache_path()
    data = _load_cache()
    data[key] = entry
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as fh:
            json.dump(data, fh, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass


def tune(params, f0: np.ndarray, steps: int = 10, reps: int = 3, use_cache: bool = True, tie: float = 0.0) -> dict:
    """Best launch shape for this grid:
    {"drift_threads", "kick_rows", "kick_drift_width", "kick_drift_blocks", "us_per_step", "table"}.
    With tie > 0 the first candidate (in the library's order) within a
    factor 1 + tie of the fastest is taken, so that shapes whose times differ
    by noise give a repeatable choice."""
    import torch
    arch = torch.cuda.get_device_properties(torch.cuda.current_device()).gcnArchName
    key = _key(arch, params)
    if use_cache:
        hit = _load_cache().get(key)
        if hit:
            return hit
    s = V.Solver(params, f0)
    table = []
    for nt, kr, kw, kb in V.tuning_candidates():
        s.set_tuning(nt, kr, kw, kb)
        s.step(2)
        times = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            s.step(steps)
            e1.record()
            torch.cuda.synchronize()
            times.append(e0.elapsed_time(e1) * 1e3 / steps)
        table.append((float(np.median(times)), nt, kr, kw, kb))
    s.close()
    fastest = min(t[0] for t in table)
    pick = next(t for t in table if t[0] <= (1.0 + tie) * fastest)
    table.sort()
    best = {"drift_threads": pick[1], "kick_rows": pick[2], "kick_drift_width": pick[3],
            "kick_drift_blocks": pick[4], "us_per_step": pick[0],
            "table": [{"drift_threads": nt, "kick_rows": kr, "kick_drift_width": kw, "kick_drift_blocks": kb,
                       "us_per_step": t} for t, nt, kr, kw, kb in table]}
    _store(key, best)
    return best
