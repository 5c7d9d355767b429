"""Benchmark: grid-point updates per second of the time-split Vlasov step.

Default workload: self-gravitating sheets on a 4096 x 4096 (x, p) grid, FP64,
x in [-10, 10) with f = 0 outside, p in [-4, 4) periodic, waterbag initial
state (x0 = 1, p0 = 0.5, noise 1e-4, seed 0), dt = 0.01.  A "step" is one full
time step of Sec. 3 of the paper (half drift, force, kick, half drift) over
the whole grid; the timed region runs K steps through one vlasov_step call
with f resident in HBM.  Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--workload NAME] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from paper_1206_3229_amd import inputs as I  # noqa: E402

HBM_PEAK_GBPS = 8000.0

WORKLOADS = {
    "sheet_4096x4096_f64": lambda: I.sheet_waterbag(4096, storage=I.STORAGE_F64),
    "sheet_4096x4096_f32": lambda: I.sheet_waterbag(4096, storage=I.STORAGE_F32),
    "hmf_gaussian_2048x2048_T0.4_f64": lambda: I.hmf_gaussian(2048, 0.4),
    "hmf_gaussian_1024x1024_T0.4_f64": lambda: I.hmf_gaussian(1024, 0.4),
    "ring_2048x2048_f64": lambda: I.ring_waterbag(2048),
    "hmf_waterbag_128x128_f64": lambda: I.hmf_waterbag_small(),
}

KERNEL_SOURCES = [os.path.join(ROOT, "paper_1206_3229_amd", "csrc", n) for n in ("vlasov_kernels.hpp", "vlasov.hip")]


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        h.update(open(p, "rb").read())
    return h.hexdigest()[:16]


def algorithmic_bytes_per_point(kernel: str, s: int) -> float:
    """Bytes per grid point one launch must move: read f and write f once
    (s bytes each); the drifts that feed the next force also write one FP64
    partial sum per 16 rows.  The fused kick and drift moves the same bytes
    as one drift: f once in, once out."""
    if kernel in ("drift", "drift2", "kick_drift2"):
        return 2 * s + 8.0 / 16.0
    if kernel == "kick":
        return 2.0 * s
    if kernel == "moments":
        return 2 * s + 6 * 8.0 / 16.0
    return float("nan")


def shape_str(shape) -> str:
    return "/".join(str(int(v)) for v in shape)


def measured_traffic(workload: str, kernel: str, shape):
    """HBM bytes per launch from the committed rocprofv3 counter summary
    (profiles/pmc_<workload>.txt), if it was taken on the current kernel
    sources in the same launch shape; else None."""
    path = os.path.join(ROOT, "profiles", f"pmc_{workload}.txt")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m = re.search(r"^kernel_source_hash: (\S+)$", text, re.M)
    if not m or m.group(1) != kernel_source_hash():
        return None
    m = re.search(rf"^kernel {re.escape(kernel)} shape {re.escape(shape_str(shape))}: hbm_bytes_per_launch=(\S+)$",
                  text, re.M)
    return float(m.group(1)) if m else None


def traced_launch_us(workload: str, kernel: str, shape):
    """Average launch duration of `kernel` in the committed rocprofv3 kernel
    trace (profiles/kernel_trace_<workload>.md), if it was taken on the
    current kernel sources in the same launch shape; else None."""
    path = os.path.join(ROOT, "profiles", f"kernel_trace_{workload}.md")
    if not os.path.exists(path) or not shape:
        return None
    text = open(path).read()
    m = re.search(r"^kernel_source_hash: (\S+)$", text, re.M)
    sh = re.search(r"^launch_shape: (\S+)$", text, re.M)
    if not m or m.group(1) != kernel_source_hash() or not sh or sh.group(1) != shape_str(shape):
        return None
    m = re.search(rf"^\| {re.escape(kernel)} \| [^|]* \| (\d+) \| ([0-9.]+) \|", text, re.M)
    return float(m.group(2)) if m else None


def fp32_error_vs_fp64(torch, V, w64: str, w32: str, shape64, shape32) -> dict:
    """Diagnostics and f of the FP32-storage run against the FP64 run after the
    workload's full number of steps, both from the same initial condition."""
    out = {}
    res = {}
    for key, w, shape in (("f64", w64, shape64), ("f32", w32, shape32)):
        p, f0, nsteps = WORKLOADS[w]()
        s = V.Solver(p, f0)
        if shape:
            s.set_tuning(*shape)
        s.step(nsteps)
        res[key] = (s.moments(), s.read_f())
        s.close()
        out["steps"] = nsteps
    (m64, f64), (m32, f32) = res["f64"], res["f32"]
    out["energy_rel"] = abs(m32["energy"] - m64["energy"]) / abs(m64["energy"])
    out["mass_abs"] = abs(m32["mass"] - m64["mass"])
    out["momentum_abs"] = abs(m32["momentum"] - m64["momentum"])
    out["magnetization_abs"] = math.hypot(m32["mx"] - m64["mx"], m32["my"] - m64["my"])
    out["l2_rel"] = abs(m32["l2"] - m64["l2"]) / abs(m64["l2"])
    out["f_rel_max"] = float(np.max(np.abs(f32 - f64)) / np.max(np.abs(f64)))
    return out


def copy_ceiling(torch, V, nbytes=1 << 30, reps=20):
    a = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    b = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    a.fill_(1)
    for _ in range(3):
        V.device_copy(b, a, nbytes)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        V.device_copy(b, a, nbytes)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    return 2 * nbytes / (ms * 1e-3) / 1e9


def run_gpu(workload: str, steps: int, warmup: int, torch, V, tuning=None):
    """Warm up, then time exactly `steps` steps in one vlasov_step call with no
    instrumentation; then run the same number of steps again with per-kernel
    HIP events (each launch carries its own start/stop event) for the kernel
    breakdown."""
    p, f0, _ = WORKLOADS[workload]()
    s = V.Solver(p, f0)
    if tuning is not None:
        s.set_tuning(*tuning)
    s.step(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    s.profile(True)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    s.step(steps)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    prof = s.profile_read()
    s.profile(False)
    m = s.moments()
    s.close()
    return p, (t1 - t0), prof, m, (t3 - t2)


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def host_threads() -> int:
    """Threads the oracle may use here: OMP_NUM_THREADS if set, else the CPUs
    this process may run on."""
    env = os.environ.get("OMP_NUM_THREADS", "")
    if env.isdigit() and int(env) > 0:
        return int(env)
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def _oracle_rate(O, p, f, threads: int, seconds: float):
    """Updates/s of the oracle on `threads` threads: one untimed step, then
    as many whole steps as fill about `seconds` (at most 50)."""
    O.set_threads(threads)
    t0 = time.perf_counter()
    f = O.run(p, f, 1)
    one = time.perf_counter() - t0
    nsteps = max(1, min(50, int(seconds / max(one, 1e-3))))
    t0 = time.perf_counter()
    O.run(p, f, nsteps)
    el = time.perf_counter() - t0
    return p.nx * p.np_ * nsteps / el, nsteps, el


def cpu_baseline(workload: str, seconds_per_leg: float = 8.0):
    """The CPU oracle, as it stands, on a bounded sample of the same workload:
    all host threads (the value), and one thread."""
    from oracle import oracle as O
    p, f0, _ = WORKLOADS[workload]()
    n = host_threads()
    v_all, s_all, t_all = _oracle_rate(O, p, f0, n, seconds_per_leg)
    v_one, s_one, t_one = _oracle_rate(O, p, f0, 1, seconds_per_leg)
    O.set_threads(n)
    return {"value": v_all, "unit": "grid-point updates/s", "cores": n, "kind": "oracle",
            "sample": f"{s_all} time steps of {workload} on {n} threads ({t_all:.1f} s, after one untimed step); "
                      f"the plain C oracle, OpenMP over lines, results independent of the thread count",
            "cpu_model": cpu_model(),
            "single_thread": {"value": v_one, "steps": s_one, "seconds": t_one},
            "thread_speedup": v_all / v_one}


# ---------------------------------------------------------------------------
# Serving: parameter-scan requests of uneven sizes with Poisson arrivals.
# ---------------------------------------------------------------------------

def _pct(xs, q):
    xs = sorted(xs)
    if not xs:
        return None
    k = min(len(xs) - 1, max(0, int(math.ceil(q / 100.0 * len(xs))) - 1))
    return xs[k]


def run_sequential_fp64(V, torch, trace, ics, keep):
    """The requests one after another through vlasov_step in FP64 (bitwise equal
    to the CPU oracle); returns per-request service times, moments, kept f."""
    out = []
    for q, f0 in zip(trace, ics):
        p64 = I.Params(**{**q.params.as_dict(), "storage": I.STORAGE_F64})
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s = V.Solver(p64, f0)
        s.step(q.nsteps)
        m = s.moments()
        t1 = time.perf_counter()
        f = s.read_f() if q.rid in keep else None
        s.close()
        out.append((t1 - t0, m, f))
    return out


def run_server(V, trace, ics, arrivals, keep, arena_bytes, max_slots, chunk, fuse=True):
    import threading
    srv = V.Server(arena_bytes, storage=I.STORAGE_F32, max_slots=max_slots, chunk_cycles=chunk, fuse=fuse)
    tickets = [None] * len(trace)
    start = time.perf_counter()

    def submitter():
        for k, (q, f0) in enumerate(zip(trace, ics)):
            delay = arrivals[k] - (time.perf_counter() - start)
            if delay > 0:
                time.sleep(delay)
            tickets[k] = srv.submit(q.params, f0, q.nsteps, keep_f=q.rid in keep)

    th = threading.Thread(target=submitter)
    th.start()
    results = [None] * len(trace)
    pending = len(trace)
    while pending:
        for k in range(len(trace)):
            if results[k] is None and tickets[k] is not None:
                r = srv.poll(tickets[k])
                if r is not None:
                    results[k] = r
                    pending -= 1
        time.sleep(0.0005)
    th.join()
    srv.close()
    return results


def serving(V, torch, nreq, seed=0, arena_bytes=2 << 30, max_slots=256, chunk=64):
    trace = I.serving_trace(nreq, rate=math.inf, seed=seed, storage=I.STORAGE_F32)
    # each request carries its initial-condition spec (U, M0, noise, seed); the
    # server, and the sequential baseline, build f0 on the device inside the
    # measured time
    ics = [V.ic_waterbag_um(q.U, q.M0, 1e-4, q.seed) for q in trace]
    work = [q.params.nx * q.params.np_ * q.nsteps for q in trace]
    keep = set(range(0, nreq, 32))
    seq = run_sequential_fp64(V, torch, trace, ics, keep)
    t_seq = sum(x[0] for x in seq)
    burst = run_server(V, trace, ics, [0.0] * nreq, keep, arena_bytes, max_slots, chunk)
    span = max(r[0]["t_done"] for r in burst) - min(r[0]["t_submit"] for r in burst)
    rate = 0.5 * nreq / span
    rng = np.random.default_rng(seed + 1)
    arrivals = list(np.cumsum(rng.exponential(1.0 / rate, nreq)))
    pois = run_server(V, trace, ics, arrivals, keep, arena_bytes, max_slots, chunk)
    lat = [r[0]["t_done"] - r[0]["t_submit"] for r in pois]
    span_p = max(r[0]["t_done"] for r in pois) - min(r[0]["t_submit"] for r in pois)
    # sequential FP64 under the same arrivals: a single queue with the measured service times
    t_free, lat_seq = 0.0, []
    for a, (svc, _, _) in zip(arrivals, seq):
        t0 = max(a, t_free)
        t_free = t0 + svc
        lat_seq.append(t_free - a)
    # accuracy of the FP32-storage results against the FP64 results (the FP64
    # path equals the CPU oracle bit for bit), per model
    acc = {}
    dF = []
    names = {I.MODEL_HMF: "hmf", I.MODEL_RING: "ring", I.MODEL_SHEET: "sheet"}
    # the initial energy of each request (outside every timed region): the
    # final energy can vanish where the mass leaves the sheet's box, so the
    # difference is also stated relative to it
    e0 = []
    for q, ic in zip(trace, ics):
        s0 = V.Solver(I.Params(**{**q.params.as_dict(), "storage": I.STORAGE_F64}), ic)
        e0.append(s0.moments()["energy"])
        s0.close()
    for q, (r, f32), (_, m64, f64), E0 in zip(trace, burst, seq, e0):
        m32 = r["moments"]
        d = acc.setdefault(names[q.params.model], {"dE": [], "dE0": [], "dM": [], "dmass": []})
        d["dE"].append(abs(m32["energy"] - m64["energy"]) / max(abs(m64["energy"]), 1e-300))
        d["dE0"].append(abs(m32["energy"] - m64["energy"]) / max(abs(E0), 1e-300))
        d["dM"].append(math.hypot(m32["mx"] - m64["mx"], m32["my"] - m64["my"]))
        d["dmass"].append(abs(m32["mass"] - m64["mass"]))
        if f32 is not None and f64 is not None:
            dF.append(float(np.max(np.abs(f32 - f64)) / max(np.max(np.abs(f64)), 1e-300)))
    accuracy = {"f_rel_max_sampled": max(dF) if dF else None, "f_sampled_requests": len(dF)}
    for k, d in acc.items():
        accuracy[k] = {"requests": len(d["dE"]),
                       **{f"energy_rel_p{q}": _pct(d["dE"], q) for q in (50, 90, 99)},
                       "energy_rel_max": max(d["dE"]),
                       **{f"energy_rel_initial_p{q}": _pct(d["dE0"], q) for q in (50, 99)},
                       "energy_rel_initial_max": max(d["dE0"]),
                       **{f"magnetization_abs_p{q}": _pct(d["dM"], q) for q in (50, 99)},
                       "mass_abs_p50": _pct(d["dmass"], 50), "mass_abs_max": max(d["dmass"])}
    total = float(sum(work))
    return {
        "requests": nreq, "total_updates": total, "storage": "f32 f, f64 density/force/diagnostics",
        "arena_bytes": arena_bytes, "max_slots": max_slots, "chunk_cycles": chunk,
        "fused_kick_drift": True,
        "burst": {"makespan_s": span, "updates_per_s": total / span,
                  "p50_s": _pct([r[0]["t_done"] - r[0]["t_submit"] for r in burst], 50),
                  "p99_s": _pct([r[0]["t_done"] - r[0]["t_submit"] for r in burst], 99)},
        "poisson": {"rate_per_s": rate, "makespan_s": span_p, "updates_per_s": total / span_p,
                    "p50_s": _pct(lat, 50), "p99_s": _pct(lat, 99)},
        "sequential_fp64": {"busy_s": t_seq, "updates_per_s": total / t_seq,
                            "poisson_p50_s": _pct(lat_seq, 50), "poisson_p99_s": _pct(lat_seq, 99)},
        "speedup_vs_sequential_fp64": (total / span) / (total / t_seq),
        "accuracy_vs_fp64": accuracy,
    }


def model_leg(V, torch, workload: str, steps: int, warmup: int, shape) -> dict:
    """Another model at full size beside the headline: throughput, the kernel
    times (a second, profiled run) and the per-step time outside the fused
    kernel."""
    p, secs, prof, _, _ = run_gpu(workload, steps, warmup, torch, V, shape)
    us = {k: (v[0] / v[1] * 1e3 if v[1] else None) for k, v in prof.items()}
    ms = secs / steps * 1e3
    kd = us.get("kick_drift2")
    return {"workload": workload, "value": p.nx * p.np_ * steps / secs, "unit": "grid-point updates/s",
            "ms_per_step": ms, "steps": steps, "launch_shape": shape_str(shape) if shape else "library default",
            "kernels_us": us,
            "outside_fused_kernel_us_per_step": (ms * 1e3 - kd) if kd else None}


def variant_rate(V, torch, workload: str, steps: int, shape, **overrides) -> dict:
    """Throughput of the workload with other solver options (a full step each)."""
    p, f0, _ = WORKLOADS[workload]()
    p = I.Params(**{**p.as_dict(), **overrides})
    s = V.Solver(p, f0)
    if shape:
        s.set_tuning(*shape)
    s.step(2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(steps)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    s.close()
    return {"options": overrides, "value": p.nx * p.np_ * steps / t, "unit": "grid-point updates/s",
            "ms_per_step": t / steps * 1e3, "steps": steps}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default="sheet_4096x4096_f64", choices=list(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32", action="store_true", help="skip the FP32-storage leg")
    ap.add_argument("--no-copy", action="store_true", help="skip the copy-kernel ceiling")
    ap.add_argument("--no-extras", action="store_true", help="skip the FP32 leg and the copy ceiling")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the global-spline, fourth-order-splitting and filter legs")
    ap.add_argument("--serve-requests", type=int, default=512, help="requests of the serving leg (0: skip)")
    ap.add_argument("--no-autotune", action="store_true", help="use the default launch shapes")
    ap.add_argument("--shape", default=None,
                    help="fixed launch shape drift_threads/kick_rows/kick_drift_width/kick_drift_blocks "
                         "(no autotuning)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the solver runs on one GPU; --gpus {args.gpus} is not supported "
              "(a simulation is not sharded across GPUs)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1206_3229_amd import vlasov as V
    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    V.load()
    torch.cuda.set_device(0)

    def pick_shape(workload):
        if args.shape:
            return tuple(int(v) for v in args.shape.split("/")), None
        if args.no_autotune:
            return None, None
        from paper_1206_3229_amd import autotune
        pw, fw, _ = WORKLOADS[workload]()
        best = autotune.tune(pw, fw, use_cache=False, tie=0.03)
        return (best["drift_threads"], best["kick_rows"], best["kick_drift_width"], best["kick_drift_blocks"]), best

    shape, tuned = pick_shape(args.workload)
    p, secs, prof, mom, secs_events = run_gpu(args.workload, args.steps, args.warmup, torch, V, shape)
    npts = p.nx * p.np_
    value = npts * args.steps / secs
    s_bytes = 4 if p.storage == I.STORAGE_F32 else 8
    # dominant kernel: largest total time in the timed region
    dom = max((k for k in prof if prof[k][1] > 0), key=lambda k: prof[k][0])
    dom_ms, dom_n = prof[dom]
    avg_s = dom_ms / dom_n * 1e-3
    bpp = algorithmic_bytes_per_point(dom, s_bytes)
    achieved = bpp * npts / avg_s / 1e9
    traffic = measured_traffic(args.workload, dom, shape) if shape else None
    trace_us = traced_launch_us(args.workload, dom, shape)
    ms_step = secs / args.steps * 1e3
    sweeps_bpp = 6 * s_bytes + 8.0 / 16.0
    out = {
        "metric": "grid-point updates/s per Strang step",
        "value": value,
        "unit": "grid-point updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "ms_per_step_with_kernel_events": secs_events / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if s_bytes == 8 else "f32-storage/f64-reductions",
        "data": "synthetic (seeded waterbag initial condition of the paper's sheet workload)",
        "config": {"workload": args.workload, "nx": p.nx, "np": p.np_, "dt": p.dt,
                   "x": [p.xmin, p.xmax], "p": [p.pmin, p.pmax], "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBPS, "traffic": traffic,
                     "bytes_per_point": bpp, "avg_launch_us": avg_s * 1e6, "launches": dom_n,
                     "trace_avg_launch_us": trace_us,
                     "frac_trace": (bpp * npts / (trace_us * 1e-6) / 1e9 / HBM_PEAK_GBPS) if trace_us else None,
                     "three_sweep_bytes_per_update": sweeps_bpp,
                     "three_sweep_equivalent_GBps": sweeps_bpp * npts / (ms_step * 1e-3) / 1e9,
                     "note": ("bytes_per_point counts what the fused kernel moves: the kick and both half drifts "
                              "read f once and write it once (2s bytes) plus one FP64 density partial per 16 rows; "
                              "three separate sweeps would move 6s + 0.5 bytes per update, the figure "
                              "three_sweep_equivalent_GBps applies to the whole step")},
        "kernels_us": {k: (v[0] / v[1] * 1e3 if v[1] else None) for k, v in prof.items()},
        "outside_fused_kernel_us_per_step": (ms_step * 1e3 - prof["kick_drift2"][0] / prof["kick_drift2"][1] * 1e3
                                             if prof.get("kick_drift2", (0, 0))[1] else None),
        "launch_shape": {"drift_threads": shape[0], "kick_rows": shape[1], "kick_drift_width": shape[2],
                         "kick_drift_blocks": shape[3],
                         "autotune_us_per_step": {
                             f"{t['drift_threads']}/{t['kick_rows']}/{t['kick_drift_width']}/{t['kick_drift_blocks']}":
                                 round(t["us_per_step"], 2)
                             for t in tuned["table"]} if tuned else "fixed"} if shape else "default",
        "moments_end": {k: mom[k] for k in ("mass", "energy", "momentum")},
    }
    if args.no_extras:
        args.no_fp32 = args.no_copy = True
    if not args.no_fp32:
        alt = {"sheet_4096x4096_f64": "sheet_4096x4096_f32"}.get(args.workload)
        if alt:
            shape32, _ = pick_shape(alt)
            p32, secs32, prof32, _, _ = run_gpu(alt, args.steps, args.warmup, torch, V, shape32)
            kd32 = prof32.get("kick_drift2", (0.0, 0))
            roof32 = None
            if kd32[1]:
                # the fused kernel of the FP32 leg against the same peak: 4-byte f
                avg32 = kd32[0] / kd32[1] * 1e-3
                bpp32 = algorithmic_bytes_per_point("kick_drift2", 4)
                ach32 = bpp32 * p32.nx * p32.np_ / avg32 / 1e9
                tr32 = traced_launch_us(alt, "kick_drift2", shape32)
                roof32 = {"bound": "hbm", "kernel": "kick_drift2", "achieved": ach32, "peak": HBM_PEAK_GBPS,
                          "unit": "GB/s", "frac": ach32 / HBM_PEAK_GBPS,
                          "traffic": measured_traffic(alt, "kick_drift2", shape32) if shape32 else None,
                          "bytes_per_point": bpp32, "avg_launch_us": avg32 * 1e6, "trace_avg_launch_us": tr32}
            out["fp32_storage"] = {"workload": alt, "value": p32.nx * p32.np_ * args.steps / secs32,
                                   "launch_shape": shape32,
                                   "ms_per_step": secs32 / args.steps * 1e3,
                                   "kernels_us": {k: (v[0] / v[1] * 1e3 if v[1] else None)
                                                  for k, v in prof32.items()},
                                   "roofline": roof32,
                                   "error_vs_fp64": fp32_error_vs_fp64(torch, V, args.workload, alt, shape,
                                                                       shape32)}
    if not (args.no_extras or args.no_variants):
        steps_v = max(2, args.steps // 10)
        # the paper's baseline interpolation (global spline, eq. tridiagsys) on the same workload
        out["global_spline"] = variant_rate(V, torch, args.workload, steps_v, shape, spline=I.SPLINE_GS)
        # the higher-order splitting and the filter of the conclusions
        out["triple_jump"] = variant_rate(V, torch, args.workload, steps_v, shape, splitting=I.SPLIT_TRIPLE_JUMP)
        out["filter_every_step"] = variant_rate(V, torch, args.workload, steps_v, shape, filter_every=1,
                                                filter_strength=1.0)
    if not (args.no_extras or args.no_variants):
        # the other two models at their full sizes (per-step overhead beside the headline)
        out["other_models"] = [model_leg(V, torch, w, max(2, args.steps // 10), 5, None)
                               for w in ("hmf_gaussian_2048x2048_T0.4_f64", "ring_2048x2048_f64")]
    if not args.no_copy:
        out["copy_ceiling_GBps"] = copy_ceiling(torch, V)
    if args.no_extras:
        args.serve_requests = 0
    if args.serve_requests > 0:
        out["serving"] = serving(V, torch, args.serve_requests)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.workload)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
