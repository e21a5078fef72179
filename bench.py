"""Benchmark of the fused polar LB detonation step on one MI355X.

A step is one time step of the whole grid through libpdbm: moments, f^eq,
BGK + chemical term + Cochran reaction, polar upwind advection of f and
lambda, and the float64 drift reductions (recorded every step here).

Default workload: the 1024 x 1024 outward detonation in float64 (2000
steps).  Prints one JSON line.  The float32 form of the same workload is
timed alongside and reported under "fp32".

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-fp32]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, vendor figure
PROFILE = os.path.join(ROOT, "profiles", "k_step_outward1024.md")
KERNEL_SOURCES = ("paper_1308_0653_amd/csrc/pdbm_kernels.hip", "paper_1308_0653_amd/csrc/pdbm_internal.h")
# Algorithmic bytes per cell-update: read and write all 33 f values and lambda.
BYTES_PER_CELL = {"f64": 33 * 8 * 2 + 8 * 2, "f32": 33 * 4 * 2 + 8 * 2}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-fp32", action="store_true", help="skip the float32 form")
    ap.add_argument("--cpu-steps", type=int, default=400, help="oracle steps of the CPU sample")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy 5 times (calibrates HBM byte counters)")
    return ap.parse_args()


def copy_probe(torch):
    """A plain copy of known size: 1 GiB read + 1 GiB written per launch."""
    n = 1 << 30
    a = torch.empty(n, dtype=torch.uint8, device="cuda")
    b = torch.empty(n, dtype=torch.uint8, device="cuda")
    a.fill_(1)
    torch.cuda.synchronize()
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_each_way": n, "launches": 5}))


def time_solver(P, w, precision, steps, warmup, torch):
    """Times `steps` steps after `warmup` untimed ones.  Returns (wall seconds,
    event seconds): the wall clock is bracketed by device synchronisation,
    the events are recorded on the stream the kernels run on."""
    stream = torch.cuda.current_stream()
    s = P.Solver(P.make_params(**w.params_kw(), precision=precision, diag_every=1), P.make_ic(**w.ic_kw()),
                 stream=stream)
    s.step(warmup)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    s.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev = e0.elapsed_time(e1) / 1e3
    _, diag = s.moments(check=False)
    s.close()
    return wall, ev, diag


def measured_traffic(kernel: str):
    """HBM bytes per launch of the step kernel from the committed rocprofv3
    counter summary (FETCH_SIZE and WRITE_SIZE, each scaled by what the same
    counter reads for a plain copy of known size), or None when the kernel
    source has changed since those counters were taken."""
    import hashlib
    import re
    try:
        txt = open(PROFILE).read()
        data = json.loads(re.search(r"```json\n(.*?)```", txt, flags=re.S).group(1))
    except (OSError, AttributeError, ValueError):
        return None
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    if h.hexdigest()[:16] != data.get("kernel_source_sha256_16"):
        return None
    return data.get(kernel, {}).get("traffic_bytes")


def roofline(cells, dtype, ev_seconds, steps, traffic=None):
    per_launch = BYTES_PER_CELL[dtype] * cells
    achieved = per_launch / (ev_seconds / steps) / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "bytes_per_launch": per_launch, "kernel": "k_step", "avg_launch_us": round(ev_seconds / steps * 1e6, 2)}


def cpu_baseline(w, steps):
    """The CPU oracle, as it stands, on a bounded sample of the same
    workload: the full grid for `steps` steps."""
    from oracle import oracle as O
    o = O.Solver(O.make_params(**w.params_kw()))
    o.init_ic(**w.ic_kw())
    t0 = time.perf_counter()
    o.step(steps)
    dt = time.perf_counter() - t0
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": round(w.cells * steps / dt, 1), "unit": "cell-updates/s", "cores": cores, "kind": "oracle",
            "sample": f"{w.nr}x{w.ntheta} grid, first {steps} of {w.nsteps} steps, float64, {dt:.1f} s"}


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {a.gpus}); this build runs one solve per GPU "
              "and has no multi-GPU path.", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1308_0653_amd import pdbm as P
    from paper_1308_0653_amd import workloads as W

    if not torch.cuda.is_available():
        print("bench.py needs an MI355X GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    if a.copy_probe:
        copy_probe(torch)
        return
    w = W.outward_fp64()
    wall, ev, diag = time_solver(P, w, P.PDBM_FP64, a.steps, a.warmup, torch)
    value = w.cells * a.steps / wall
    out = {
        "metric": "polar DBM cell-updates/s (float64, 1024x1024 outward detonation)",
        "value": round(value, 1),
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(wall / a.steps * 1e3, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "nr": w.nr, "ntheta": w.ntheta, "r": [w.r_min, w.r_max],
                   "cells": w.cells, "diag_every": 1, "parallelism": "single GPU"},
        "roofline": roofline(w.cells, "f64", ev, a.steps, measured_traffic("k_step_f64")),
        "hbm_frac_of_peak": None,
    }
    out["hbm_frac_of_peak"] = out["roofline"]["frac"]
    if diag["n_nonfinite"] or diag["n_nonphys"]:
        out["error"] = "non-physical state at the end of the run"
    if not a.no_fp32:
        w32 = W.outward_fp32()
        wall32, ev32, _ = time_solver(P, w32, P.PDBM_FP32, a.steps, a.warmup, torch)
        out["fp32"] = {"value": round(w32.cells * a.steps / wall32, 1), "unit": "cell-updates/s",
                       "ms_per_step": round(wall32 / a.steps * 1e3, 5), "speedup_vs_f64": round(wall / wall32, 3),
                       "roofline": roofline(w32.cells, "f32", ev32, a.steps, measured_traffic("k_step_f32"))}
    if not a.no_cpu:
        out["cpu_baseline"] = cpu_baseline(w, a.cpu_steps)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
