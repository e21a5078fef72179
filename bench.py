"""Benchmark of the fused polar LB detonation step on one MI355X.

A step is one time step of the whole grid through libpdbm: moments, f^eq,
BGK + chemical term + Cochran reaction, polar upwind advection of f and
lambda, and the float64 drift reductions (recorded every step here).  Both
forms advance two steps per pass over f (k_step2).

Default workload: the 1024 x 1024 outward detonation in float64 (2000
steps).  Prints one JSON line.  The float32 form of the same workload is
timed alongside and reported under "fp32"; the packed parameter sweep and
the served request stream under "packed_sweep" and "serving"; the other
kernels of the path (non-equilibrium measures, the step with a per-cell tau
field, a rotated sector) under "side_kernels"; the CPU oracle on a sample
of the float64 workload, on every host thread and on one, under
"cpu_baseline".

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-fp32] [--no-serving] [--no-side]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, vendor figure
PROFILE = os.path.join(ROOT, "profiles", "step_kernels_outward1024.md")
KERNEL_SOURCES = tuple("paper_1308_0653_amd/csrc/" + f for f in
                       ("pdbm_device.h", "pdbm_step.hip", "pdbm_step2.hip", "pdbm_internal.h", "pdbm_offsets.h"))
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
    ap.add_argument("--no-serving", action="store_true", help="skip the packed-batch and serving measurements")
    ap.add_argument("--no-side", action="store_true",
                    help="skip the other kernels (non-equilibrium measures, per-cell tau field, rotated sector)")
    ap.add_argument("--batch-solves", type=int, default=256, help="solves of the packed parameter sweep")
    ap.add_argument("--batch-steps", type=int, default=500, help="steps of each solve of the sweep")
    ap.add_argument("--serving-requests", type=int, default=1000,
                    help="requests of the Poisson serving stream (the full workload is 1000; 0 skips it)")
    ap.add_argument("--clock-warmup-ms", type=float, default=60.0,
                    help="throwaway steps of the same solve run before each timed leg, in ms of GPU time")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy 5 times (calibrates HBM byte counters)")
    ap.add_argument("--pack-probe", action="store_true",
                    help="only time packs of single columns, alone and beside annuli (float64)")
    return ap.parse_args()


def pack_probe(P, W, torch, steps=400, chunk=50):
    """Packed launches with single theta columns, float64: 64 columns of the
    printed-resolution steady detonation's grid (20000 x 1, dt = 2.5e-7),
    then 16 annuli of 512 x 512 beside 16 of those columns.  Wall clock over
    `steps` steps in graph-replayed chunks of `chunk`, on a stream of its
    own, after 100 untimed steps."""
    from dataclasses import replace
    col = replace(W.small_fp64(), name="vv_column", nr=20000, ntheta=1, r_min=1000.0, r_max=1000.1, dt=2.5e-7,
                  tau=2e-4, w1=10.0, w2=1000.0, m=1, n=1, r_split=1000.01, inner=(1.35826, 2.59709, 0.81650, 0.0, 1.0),
                  outer=(1.0, 1.0, 0.0, 0.0, 0.0), p_noise=1e-3)
    wide = replace(W.outward_fp64(), nr=512, ntheta=512)
    out = {}
    for name, ws in (("columns64", [replace(col, seed=i) for i in range(64)]),
                     ("annuli16_columns16", [replace(wide, seed=i) for i in range(16)] +
                      [replace(col, seed=100 + i) for i in range(16)])):
        ps = [P.make_params(**w.params_kw(), precision=P.PDBM_FP64, diag_every=0) for w in ws]
        st = torch.cuda.Stream()
        b = P.Batch(ps, [P.make_ic(**w.ic_kw()) for w in ws], chunk_steps=chunk, stream=st)
        b.step(100)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b.step(steps)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        cells = sum(w.nr * w.ntheta for w in ws)
        bad = sum(b.moments(i, check=False)[1]["n_nonfinite"] for i in range(len(ws)))
        out[name] = {"solves": len(ws), "cells": cells, "steps": steps, "us_per_step": round(dt / steps * 1e6, 2),
                     "cell_updates_per_s": round(cells * steps / dt, 1), "nonfinite": bad}
        b.close()
    print(json.dumps({"pack_probe": out}))


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


def copy_bandwidth(torch):
    """Read+write bandwidth of a plain 1 GiB device copy on this GPU (GB/s),
    the practical ceiling the step kernel is compared with beside the
    vendor peak."""
    n = 1 << 30
    a = torch.empty(n, dtype=torch.uint8, device="cuda")
    b = torch.empty(n, dtype=torch.uint8, device="cuda")
    a.fill_(1)
    b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) / 1e3 / 10
    del a, b
    torch.cuda.empty_cache()
    return 2 * n / sec / 1e9


def clock_warmup(P, w, precision, ms, torch):
    """Runs the step kernel on a throwaway copy of the solve for `ms`
    milliseconds.  The GPU's clock ramps up over its first ~30 ms under this
    load (launches then take ~176 us instead of the sustained ~157 us in
    float64), so a short timed region that starts on an idle GPU would time
    the ramp rather than the kernel."""
    if ms <= 0:
        return
    stream = torch.cuda.current_stream()
    t = P.Solver(P.make_params(**w.params_kw(), precision=precision, diag_every=1), P.make_ic(**w.ic_kw()),
                 stream=stream)
    t0 = time.perf_counter()
    while (time.perf_counter() - t0) * 1e3 < ms:
        t.step(32)
        torch.cuda.synchronize()
    t.close()


def time_solver(P, w, precision, steps, warmup, torch, warm_ms=0.0):
    """Times `steps` steps after `warmup` untimed ones (and, before those,
    `warm_ms` of throwaway steps of the same solve: clock_warmup).  Returns
    (wall seconds, event seconds): the wall clock is bracketed by device
    synchronisation, the events are recorded on the stream the kernels run
    on."""
    stream = torch.cuda.current_stream()
    s = P.Solver(P.make_params(**w.params_kw(), precision=precision, diag_every=1), P.make_ic(**w.ic_kw()),
                 stream=stream)
    clock_warmup(P, w, precision, warm_ms, torch)
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


GOLDEN = os.path.join(ROOT, "tests", "golden", "outward1024_golden.npz")


def _sig(x, digits=3):
    return float(f"{float(x):.{digits}g}")


def fp32_errors(P, W, torch):
    """Error of the float32 form on the outward 1024^2 run at steps 500,
    1000, 2000 (outside the timed region): normwise L_inf and L2 of rho, T,
    lambda against the float64 GPU field, and L_inf against the oracle's
    stored samples of the same run (tests/golden, written by the oracle)."""
    w = W.outward_fp64()
    stream = torch.cuda.current_stream()
    s64 = P.Solver(P.make_params(**w.params_kw(), precision=P.PDBM_FP64), P.make_ic(**w.ic_kw()), stream=stream)
    s32 = P.Solver(P.make_params(**w.params_kw(), precision=P.PDBM_FP32), P.make_ic(**w.ic_kw()), stream=stream)
    gold = np.load(GOLDEN) if os.path.exists(GOLDEN) else None
    names = {0: "rho", 3: "T", 5: "lambda"}
    out = {}
    for st in (500, 1000, 2000):
        s64.step(st - s64.step_count)
        s32.step(st - s32.step_count)
        F64, _ = s64.moments(check=False)
        F32, _ = s32.moments(check=False)
        rec = {}
        for k, name in names.items():
            d = F32[k] - F64[k]
            rec[name] = {"linf": _sig(np.abs(d).max() / np.abs(F64[k]).max()),
                         "l2": _sig(np.linalg.norm(d) / np.linalg.norm(F64[k]))}
            if gold is not None and k in list(gold["fields"]):
                row = list(gold["fields"]).index(k)
                ref = gold[f"s{st}_vals"][row]
                rec[name]["linf_vs_oracle"] = _sig(np.abs(F32[k][gold["ir"], gold["jt"]] - ref).max()
                                                   / gold[f"s{st}_maxabs"][k])
        out[str(st)] = rec
    s64.close()
    s32.close()
    return out


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


def roofline(cells, dtype, ev_seconds, steps, kernel, steps_per_launch, traffic=None, copy_gbs=None):
    """HBM roofline of the step kernel: algorithmic bytes (BYTES_PER_CELL per
    cell-update, times the cell-updates of one launch) over the launch's
    average duration.  The two-step kernel (steps_per_launch 2) moves about
    half of its algorithmic bytes; `traffic` is what the counters measured."""
    launches = steps / steps_per_launch
    per_launch = BYTES_PER_CELL[dtype] * cells * steps_per_launch
    launch_s = ev_seconds / launches
    achieved = per_launch / launch_s / 1e9
    out = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "bytes_per_launch": per_launch,
           "kernel": kernel, "steps_per_launch": steps_per_launch, "avg_launch_us": round(launch_s * 1e6, 2),
           "achieved_is": "effective: algorithmic bytes of the steps a launch takes over its duration"}
    if traffic:
        # what the HBM really moved (rocprofv3 counters), as a rate and a share of the peak
        out["traffic_gbs"] = round(traffic / launch_s / 1e9, 1)
        out["traffic_frac_of_peak"] = round(traffic / launch_s / 1e9 / HBM_PEAK_GBS, 4)
    if copy_gbs:
        # against what a plain copy reaches here, effective and measured bytes
        out["copy_gbs"] = round(copy_gbs, 1)
        out["frac_of_copy"] = round(achieved / copy_gbs, 4)
        if traffic:
            out["traffic_frac_of_copy"] = round(traffic / launch_s / 1e9 / copy_gbs, 4)
    return out


def side_kernels(P, w, torch, steps=200, calls=20, warm_ms=60.0):
    """The hot path's optional parts on the float64 workload, timed with HIP
    events on the stream they run on, after `warm_ms` of throwaway steps
    (clock_warmup):
    - k_noneq, the non-equilibrium measures Delta*_m of every cell (Sec.
      II.E): `calls` launches on the state after `steps` steps; it reads f
      (33 x 8 B per cell) and writes 12 float64 measures (96 B);
    - k_step2<double, TAUF>, the step with a per-cell relaxation time (Sec.
      IV, point (ii)): `steps` steps with a uniform tau field against the
      same steps of the plain solve, the two timed in turn twice (the
      second pair is reported); the field adds 8 B read per cell per
      launch;
    - k_step2<double, ROT>, two steps per launch of a rotated sector (Sec.
      II.D: the periodic images of a sector turn the directions): the same
      gas on half the annulus (sector 4, 1024 x 512 cells, the same dtheta),
      `steps` steps."""
    stream = torch.cuda.current_stream()

    def timed(fn):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / 1e3

    plain = P.Solver(P.make_params(**w.params_kw(), precision=P.PDBM_FP64, diag_every=1), P.make_ic(**w.ic_kw()),
                     stream=stream)
    tauf = P.Solver(P.make_params(**w.params_kw(), precision=P.PDBM_FP64, diag_every=1, flags=P.PDBM_TAU_FIELD),
                    P.make_ic(**w.ic_kw()), stream=stream)
    tauf.set_tau(None)  # every cell at the parameters' tau: the same steps as the plain solve
    plain.step(20)
    tauf.step(20)
    clock_warmup(P, w, P.PDBM_FP64, warm_ms, torch)
    for _ in range(2):
        t_plain = timed(lambda: plain.step(steps))
        t_tauf = timed(lambda: tauf.step(steps))
    out_t = torch.empty((P.PDBM_NONEQ_N, w.nr, w.ntheta), dtype=torch.float64, device="cuda")
    plain.noneq_async(out_t)
    torch.cuda.synchronize()

    def noneq_calls():
        for _ in range(calls):
            plain.noneq_async(out_t)

    t_noneq = timed(noneq_calls) / calls
    plain.close()
    tauf.close()
    kw = w.params_kw()
    kw.update(sector=4, ntheta=w.ntheta // 2)
    half = P.Solver(P.make_params(**kw, precision=P.PDBM_FP64, diag_every=1), P.make_ic(**w.ic_kw()), stream=stream)
    half.step(20)
    t_half = timed(lambda: half.step(steps))
    half.close()
    half_cells = w.nr * (w.ntheta // 2)
    nq_bytes = (33 * 8 + P.PDBM_NONEQ_N * 8) * w.cells
    launches = steps / 2
    per_launch = BYTES_PER_CELL["f64"] * w.cells * 2
    return {
        "noneq": {"kernel": "k_noneq<double>", "calls": calls, "avg_us": round(t_noneq * 1e6, 2),
                  "bytes_per_call": nq_bytes, "achieved_gbs": round(nq_bytes / t_noneq / 1e9, 1),
                  "frac_of_peak": round(nq_bytes / t_noneq / 1e9 / HBM_PEAK_GBS, 4)},
        "tau_field": {"kernel": "k_step2<double, TAUF>", "steps": steps,
                      "avg_launch_us": round(t_tauf / launches * 1e6, 2),
                      "plain_avg_launch_us": round(t_plain / launches * 1e6, 2),
                      "extra_bytes_per_launch": 8 * w.cells,
                      "effective_gbs": round(per_launch / (t_tauf / launches) / 1e9, 1),
                      "effective_frac_of_peak": round(per_launch / (t_tauf / launches) / 1e9 / HBM_PEAK_GBS, 4)},
        "sector": {"kernel": "k_step2<double, ROT>", "sector": 4, "nr": w.nr, "ntheta": w.ntheta // 2, "steps": steps,
                   "steps_per_launch": 2, "avg_launch_us": round(t_half / launches * 1e6, 2),
                   "effective_gbs": round(BYTES_PER_CELL["f64"] * half_cells / (t_half / steps) / 1e9, 1),
                   "effective_frac_of_peak": round(
                       BYTES_PER_CELL["f64"] * half_cells / (t_half / steps) / 1e9 / HBM_PEAK_GBS, 4)},
    }


def packed_sweep(P, W, torch, count, nsteps):
    """Independent float32 solves of the parameter sweep advanced together in
    packed, graph-captured launches (chunks of 50 steps)."""
    ws = W.batch_sweep(count=count, nsteps=nsteps)
    params = [P.make_params(**w.params_kw(), precision=P.PDBM_FP32) for w in ws]
    ics = [P.make_ic(**w.ic_kw()) for w in ws]
    stream = torch.cuda.Stream()
    b = P.Batch(params, ics, chunk_steps=50, stream=stream)
    b.step(50)  # warm-up (captures the graph)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.step(nsteps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    cells = sum(w.cells for w in ws)
    failed = 0
    for i in range(len(ws)):
        _, d = b.moments(i, check=False)
        failed += int(d["n_nonfinite"] > 0 or d["n_nonphys"] > 0)
    b.close()
    rate = cells * nsteps / wall
    return {"workload": f"sweep{count}_fp32", "solves": count, "steps": nsteps, "cells": cells,
            "value": round(rate, 1), "unit": "cell-updates/s", "wall_s": round(wall, 4),
            "hbm_frac": round(rate * BYTES_PER_CELL["f32"] / (HBM_PEAK_GBS * 1e9), 4),
            "latency_s": round(wall, 4), "failed": failed}


def serving_stream(P, W, torch, nreq, packed_rate):
    """Poisson arrivals served by the continuous-batching server (float32,
    chunks of 24 steps, 200 GB cap), against the plain float64 path running
    the same requests one at a time in arrival order."""
    import threading
    mean_work = W.mean_work_serving()
    rate = 0.8 * packed_rate / mean_work  # offered load 0.8 of the packed throughput
    stream = W.serving_stream(count=nreq, rate=rate)
    srv = P.Server(hbm_cap_bytes=200 * 10**9, max_slots=64, chunk_steps=24)
    ids = [None] * len(stream)
    t_start = time.perf_counter()

    def feeder():
        for k, (t_arr, w) in enumerate(stream):
            delay = t_arr - (time.perf_counter() - t_start)
            if delay > 0:
                time.sleep(delay)
            ids[k] = srv.submit(P.make_params(**w.params_kw(), precision=P.PDBM_FP32), P.make_ic(**w.ic_kw()),
                                w.nsteps)

    th = threading.Thread(target=feeder)
    th.start()
    th.join()
    srv.wait(-1)
    wall = time.perf_counter() - t_start
    lat = []
    failed = 0
    for rid in ids:
        t = srv.times(rid)
        lat.append(t[2] - t[0])
        failed += int(srv.poll(rid)[0] != P.PDBM_DONE)
    st = srv.stats()
    srv.close()
    work = sum(w.cells * w.nsteps for _, w in stream)
    served = {"requests": nreq, "offered_rate_per_s": round(rate, 3), "wall_s": round(wall, 3),
              "value": round(work / wall, 1), "unit": "cell-updates/s",
              "p50_latency_s": round(float(np.percentile(lat, 50)), 4),
              "p99_latency_s": round(float(np.percentile(lat, 99)), 4), "failed": failed,
              "steps_launched": st["steps_launched"]}
    # the plain float64 path, one solve at a time in arrival order (FIFO):
    # each solve's own time on the GPU, queued behind the ones before it
    busy_until, lat64, gpu_time = 0.0, [], 0.0
    torch.cuda.synchronize()
    for t_arr, w in stream:
        s = P.Solver(P.make_params(**w.params_kw(), precision=P.PDBM_FP64), P.make_ic(**w.ic_kw()),
                     stream=torch.cuda.current_stream())
        t0 = time.perf_counter()
        s.step(w.nsteps)
        s.moments(check=False)
        dt = time.perf_counter() - t0
        s.close()
        gpu_time += dt
        start = max(t_arr, busy_until)
        busy_until = start + dt
        lat64.append(busy_until - t_arr)
    serial = {"value": round(work / gpu_time, 1), "unit": "cell-updates/s",
              "p50_latency_s": round(float(np.percentile(lat64, 50)), 4),
              "p99_latency_s": round(float(np.percentile(lat64, 99)), 4),
              "busy_s": round(gpu_time, 3),
              "latency": "simulated FIFO: each request's measured solo float64 run, queued behind the ones "
                         "that arrived before it"}
    return served, serial


def cpu_baseline(w, steps, single_steps=4):
    """The CPU oracle, as it stands, on a bounded sample of the same
    workload: the full grid for `steps` steps on every host thread, then
    for `single_steps` more on one thread (the OpenMP runtime's thread count
    set through libgomp for that run, then restored)."""
    import ctypes
    from oracle import oracle as O
    o = O.Solver(O.make_params(**w.params_kw()))
    o.init_ic(**w.ic_kw())
    t0 = time.perf_counter()
    o.step(steps)
    dt = time.perf_counter() - t0
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    out = {"value": round(w.cells * steps / dt, 1), "unit": "cell-updates/s", "cores": cores, "kind": "oracle",
           "sample": f"{w.nr}x{w.ntheta} grid, first {steps} of {w.nsteps} steps, float64, {dt:.1f} s"}
    try:
        gomp = ctypes.CDLL("libgomp.so.1")
    except OSError:
        return out
    gomp.omp_set_num_threads(1)
    try:
        t0 = time.perf_counter()
        o.step(single_steps)
        d1 = time.perf_counter() - t0
    finally:
        gomp.omp_set_num_threads(cores)
    out["single_core"] = {"value": round(w.cells * single_steps / d1, 1), "cores": 1,
                          "sample": f"steps {steps + 1}-{steps + single_steps} of the same run, {d1:.1f} s"}
    return out


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {a.gpus}); the library runs each solve on "
              "one GPU and has no multi-GPU path.", file=sys.stderr)
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
    if a.pack_probe:
        pack_probe(P, W, torch)
        return
    copy_gbs = copy_bandwidth(torch)
    w = W.outward_fp64()
    # steps go in pairs, one k_step2 launch each (an odd count ends with one
    # k_step launch)
    wall, ev, diag = time_solver(P, w, P.PDBM_FP64, a.steps, a.warmup, torch, a.clock_warmup_ms)
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
                   "cells": w.cells, "diag_every": 1, "parallelism": "single GPU",
                   "ignition": {"r_below": w.r_split, "rho": w.inner[0], "T": w.inner[1],
                                "p": w.inner[0] * w.inner[1], "lambda": w.inner[4],
                                "reading": "burnt gas given by its pressure p = 30 is put at T = 5 (rho = p / 5): "
                                           "at the small workload's rho = 1.5 (T = 20) the model, oracle "
                                           "included, turns non-finite within ~30 steps"},
                   "clock_warmup_ms": a.clock_warmup_ms},
        "roofline": roofline(w.cells, "f64", ev, a.steps, "k_step2", 2, measured_traffic("k_step2_f64"), copy_gbs),
    }
    # effective bandwidth (algorithmic bytes) and, where the counters are
    # current, the HBM traffic they measured, each as a share of the peak
    out["effective_frac_of_peak"] = out["roofline"]["frac"]
    out["hbm_frac_of_peak"] = out["roofline"].get("traffic_frac_of_peak")
    if diag["n_nonfinite"] or diag["n_nonphys"]:
        out["error"] = "non-physical state at the end of the run"
    if not a.no_fp32:
        w32 = W.outward_fp32()
        wall32, ev32, _ = time_solver(P, w32, P.PDBM_FP32, a.steps, a.warmup, torch, a.clock_warmup_ms)
        out["fp32"] = {"value": round(w32.cells * a.steps / wall32, 1), "unit": "cell-updates/s",
                       "ms_per_step": round(wall32 / a.steps * 1e3, 5), "speedup_vs_f64": round(wall / wall32, 3),
                       "roofline": roofline(w32.cells, "f32", ev32, a.steps, "k_step2", 2,
                                            measured_traffic("k_step2_f32"), copy_gbs),
                       "error_vs_fp64": fp32_errors(P, W, torch)}
    if not a.no_serving:
        sweep = packed_sweep(P, W, torch, a.batch_solves, a.batch_steps)
        out["packed_sweep"] = sweep
        if a.serving_requests > 0:
            served, serial = serving_stream(P, W, torch, a.serving_requests, sweep["value"])
            out["serving"] = {"served_fp32": served, "serial_fp64": serial,
                              "workload": f"poisson{a.serving_requests}_logU"}
    if not a.no_side:
        out["side_kernels"] = side_kernels(P, w, torch, warm_ms=a.clock_warmup_ms)
    if not a.no_cpu:
        out["cpu_baseline"] = cpu_baseline(w, a.cpu_steps)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
