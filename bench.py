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
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

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
    (s bytes each); the drifts also write one FP64 partial sum per 16 rows."""
    if kernel in ("drift", "drift2"):
        return 2 * s + 8.0 / 16.0
    if kernel == "kick":
        return 2.0 * s
    if kernel == "moments":
        return s + 4 * 8.0 / 16.0
    return float("nan")


def measured_traffic(workload: str, kernel: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary
    (profiles/pmc_<workload>.txt), if it was taken on the current kernel
    sources; else None."""
    path = os.path.join(ROOT, "profiles", f"pmc_{workload}.txt")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m = re.search(r"^kernel_source_hash: (\S+)$", text, re.M)
    if not m or m.group(1) != kernel_source_hash():
        return None
    m = re.search(rf"^kernel {re.escape(kernel)}: hbm_bytes_per_launch=(\S+)$", text, re.M)
    return float(m.group(1)) if m else None


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


def run_gpu(workload: str, steps: int, warmup: int, torch, V):
    """Warm up, then time exactly `steps` steps in one vlasov_step call with no
    instrumentation; then run the same number of steps again with per-kernel
    HIP events (each launch carries its own start/stop event) for the kernel
    breakdown."""
    p, f0, _ = WORKLOADS[workload]()
    s = V.Solver(p, f0)
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


def cpu_baseline(workload: str, seconds_target: float = 15.0):
    """The CPU oracle, as it stands, on a bounded sample of the same workload."""
    from oracle import oracle as O
    p, f0, _ = WORKLOADS[workload]()
    t0 = time.perf_counter()
    f = O.run(p, f0, 1)
    one = time.perf_counter() - t0
    nsteps = max(1, min(20, int(seconds_target / max(one, 1e-3))))
    t0 = time.perf_counter()
    O.run(p, f, nsteps)
    el = time.perf_counter() - t0
    return {"value": p.nx * p.np_ * nsteps / el, "unit": "grid-point updates/s", "cores": 1, "kind": "oracle",
            "sample": f"{nsteps} time steps of {workload} (single-threaded plain C oracle, after one untimed step)"}


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
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported "
              "(the multi-GPU decomposition is described in DESIGN.md but not built)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1206_3229_amd import vlasov as V
    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    V.load()
    torch.cuda.set_device(0)

    p, secs, prof, mom, secs_events = run_gpu(args.workload, args.steps, args.warmup, torch, V)
    npts = p.nx * p.np_
    value = npts * args.steps / secs
    s_bytes = 4 if p.storage == I.STORAGE_F32 else 8
    # dominant kernel: largest total time in the timed region
    dom = max((k for k in prof if prof[k][1] > 0), key=lambda k: prof[k][0])
    dom_ms, dom_n = prof[dom]
    avg_s = dom_ms / dom_n * 1e-3
    bpp = algorithmic_bytes_per_point(dom, s_bytes)
    achieved = bpp * npts / avg_s / 1e9
    traffic = measured_traffic(args.workload, dom)
    out = {
        "metric": "grid-point updates/s per Strang step",
        "value": value,
        "unit": "grid-point updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": secs / args.steps * 1e3,
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
                     "bytes_per_point": bpp, "avg_launch_us": avg_s * 1e6, "launches": dom_n},
        "kernels_us": {k: (v[0] / v[1] * 1e3 if v[1] else None) for k, v in prof.items()},
        "moments_end": {k: mom[k] for k in ("mass", "energy", "momentum")},
    }
    if args.no_extras:
        args.no_fp32 = args.no_copy = True
    if not args.no_fp32:
        alt = {"sheet_4096x4096_f64": "sheet_4096x4096_f32"}.get(args.workload)
        if alt:
            p32, secs32, prof32, _, _ = run_gpu(alt, args.steps, args.warmup, torch, V)
            out["fp32_storage"] = {"workload": alt, "value": p32.nx * p32.np_ * args.steps / secs32,
                                   "ms_per_step": secs32 / args.steps * 1e3,
                                   "kernels_us": {k: (v[0] / v[1] * 1e3 if v[1] else None)
                                                  for k, v in prof32.items()}}
    if not args.no_copy:
        out["copy_ceiling_GBps"] = copy_ceiling(torch, V)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.workload)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
