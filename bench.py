#!/usr/bin/env python3
"""Benchmark of the LB-IB adhesion hot path on one MI355X.

A step is one full time step n -> n+1 of the coupled method (particle phase + lattice
sweep) on the 4096 x 1024 FP32 channel with one aspect-ratio-3 ellipse (256 markers,
ligand density 0.7, bond strength 2, Re 1), inputs resident in HBM.  Prints one JSON line:
whole-step throughput in MLUPS over the K timed steps (host clock, bracketed by device
synchronisations; HIP events on the simulation's stream beside it, and a 1000-step window
that shows the fixed cost of a call), the lattice sweep's roofline (algorithmic bytes per
launch over its HIP-event-timed average duration, against the 8 TB/s HBM peak and the
measured copy), the same sweep on an 8192 x 4096 channel far beyond the 256 MB last-level
cache in every storage precision, the 256 x 64 FP64 channel (latency-bound), the
216-simulation parameter sweep (pool against the plain loops), 32 particles in one channel,
the serving mix, and the FP64 CPU oracle timed on this host's cores and on one thread.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
METRIC = "aggregate MLUPS & % HBM roofline; batched/served vs plain; p50/p99 solve latency"
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_sweep_4096x1024_fp32.json")
TRAFFIC_FILE_BEYOND = os.path.join(ROOT, "profiles", "traffic_sweep_8192x4096_storages.json")
# the lattice sweep's device code: the counters in the traffic files are valid for these sources only
KERNEL_SRCS = [os.path.join(ROOT, "paper_1808_01448_amd", "csrc", f)
               for f in ("lbib_sweep.hip", "lbib_collide.hpp", "lbib_device.hpp", "lbib_internal.hpp")]
LEGS = ("beyond", "c1", "batched", "multi", "serve", "cpu")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SRCS:
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(cells: int) -> dict:
    """HBM bytes per sweep launch from the committed rocprofv3 counter summary and the sweep
    kernel they were counted on (None for both when taken on a different kernel source)."""
    none = {"traffic": None, "traffic_kernel": None}
    try:
        t = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return none
    if t.get("kernel_source_sha256_16") != kernel_source_hash() or t.get("cells") != cells:
        return none
    return {"traffic": t.get("hbm_bytes_per_launch"), "traffic_kernel": t.get("kernel")}


def measured_traffic_beyond(storage: str, cells: int) -> dict:
    """HBM bytes per sweep launch of the 8192 x 4096 leg for one storage and the sweep kernel
    they were counted on, from the committed counter summary (None for both when it was taken
    on a different kernel source)."""
    none = {"traffic": None, "traffic_kernel": None}
    try:
        t = json.load(open(TRAFFIC_FILE_BEYOND))
    except (OSError, ValueError):
        return none
    if t.get("kernel_source_sha256_16") != kernel_source_hash():
        return none
    for e in t.get("entries", []):
        if e.get("storage") == storage and e.get("cells") == cells:
            return {"traffic": e.get("hbm_bytes_per_launch"), "traffic_kernel": e.get("kernel")}
    return none


def timed_window(sim, steps: int, stream, events: bool = True) -> dict:
    """`steps` whole steps bracketed by device synchronisations: host wall clock, and, with
    events, HIP events recorded on the simulation's stream (into which every lbib_step call
    joins its work) around the same calls.  The events are work on that stream: without them
    lbib_step finds the stream idle and skips its start-of-call join."""
    import torch

    if events:
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    if events:
        e0.record(stream)
    sim.step(steps)
    if events:
        e1.record(stream)
    sim.sync()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return {"seconds": dt, "gpu_seconds": e0.elapsed_time(e1) * 1e-3 if events else None}


def sweep_timing(sim, steps: int):
    """Average duration of the lattice sweep (kernel 0) and of the particle launch (kernel 1)
    from launch-attached HIP events, over `steps` steps each."""
    sim.kernel_timing(1)
    sim.step(steps)
    ms0, n0 = sim.kernel_time(0)
    sim.kernel_timing(2)
    sim.step(max(steps // 5, 20))
    ms1, n1 = sim.kernel_time(1)
    sim.kernel_timing(0)
    return ms0 / max(n0, 1), n0, ms1 / max(n1, 1)


def cpu_oracle(workload: dict, steps: int, threads: int | None = None) -> dict:
    """The FP64 oracle on a bounded sample of a workload: `steps` full steps after one
    untimed step, on `threads` threads (None: all the host's cores)."""
    import oracle

    oracle.lib()
    prev = oracle.num_threads()
    if threads is not None:
        oracle.set_threads(threads)
    try:
        o = oracle.Sim.from_workload(workload)
        o.step(1)  # first touch of the arrays outside the timed region
        t0 = time.perf_counter()
        o.step(steps)
        dt = time.perf_counter() - t0
        used = oracle.num_threads()
    finally:
        oracle.set_threads(prev)
    cells = workload["lattice"]["nx"] * workload["lattice"]["ny"]
    return {
        "value": round(cells * steps / dt / 1e6, 3),
        "unit": "MLUPS",
        "cores": used,
        "kind": "oracle",
        "sample": f"{steps} full steps (after 1 untimed) of the same {workload['lattice']['nx']}x"
                  f"{workload['lattice']['ny']} workload, FP64, {dt:.1f} s",
    }


STORAGE_TYPE = {"fp32": "float", "fp64": "double", "fp16": "half_t", "bf16": "bf16_t", "fp16_neq": "half_neq_t",
                "bf16_neq": "bf16_neq_t"}


def sweep_kernel_name(prec: str, serial: bool) -> str:
    return ("sweep_kernel" if serial else "sweep_overlap_kernel") + f"<{STORAGE_TYPE[prec]}, push>"


def beyond_cache_leg(steps: int, stream, serial: bool = False) -> dict:
    """The sweep far beyond the 256 MB last-level cache: 8192 x 4096 channel with the scaled
    ellipse, every storage precision, each with its own roofline block (HIP-event-timed sweep
    average against 8 TB/s and against a copy of one population buffer measured in the same
    run, i.e. the same bytes read and written)."""
    from paper_1808_01448_amd import lbib
    from paper_1808_01448_amd import workloads as W

    base = W.channel_beyond_cache_fp32()
    cells = base["lattice"]["nx"] * base["lattice"]["ny"]
    out = {"workload": base["name"] + " (8192 x 4096, ellipse AR3 96 x 32, 512 markers, Re 1)", "cells": cells,
           "steps_timed": steps, "storages": {}}
    for prec in ("fp32", "fp64", "fp16", "bf16", "fp16_neq", "bf16_neq"):
        w = W.with_precision(base, prec)
        sim = lbib.Sim(w, stream=stream)
        try:
            if serial:
                sim.set_overlap(0)
            bpu = sim.bytes_per_update
            sim.step(20)
            sim.sync()
            win = timed_window(sim, steps, stream)
            sweep_ms, n0, part_ms = sweep_timing(sim, steps)
            buf = (bpu // 2) * cells  # one population buffer (every population read once, written once)
            buf -= buf % 16
        finally:
            sim.close()
        copy_gbs = lbib.bandwidth_probe(buf, 10, stream=stream)
        achieved = bpu * cells / (sweep_ms * 1e-3) / 1e9
        out["storages"][prec] = {
            "bytes_per_update": bpu, "working_set_mb": round(bpu * cells / 1e6, 1),
            "mlups": round(cells * steps / win["seconds"] / 1e6, 1),
            "ms_per_step": round(win["seconds"] * 1e3 / steps, 4),
            "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(achieved / HBM_PEAK_GBS, 4), "kernel": sweep_kernel_name(prec, serial),
                         **measured_traffic_beyond(prec, cells),
                         "algorithmic_bytes_per_launch": bpu * cells,
                         "avg_launch_us": round(sweep_ms * 1e3, 2), "launches_timed": n0,
                         "copy_same_bytes_gbs": round(copy_gbs, 1),
                         "frac_of_measured_copy": round(achieved / copy_gbs, 4) if copy_gbs > 0 else None},
            "particle_launch_avg_us": round(part_ms * 1e3, 2),
            # the library's rule (both buffers at least twice the last-level cache, f - w storages)
            "tile_order": ("the same every step" if prec.endswith("_neq")
                           else "reversed on odd steps: a sweep first reads the tiles the previous one wrote last"),
        }
        log(f"bench: beyond cache {prec}: sweep {sweep_ms * 1e3:.1f} us = {achieved:.0f} GB/s "
            f"({achieved / HBM_PEAK_GBS:.3f} of 8 TB/s, {achieved / copy_gbs:.3f} of the copy {copy_gbs:.0f} GB/s)")
    return out


def c1_leg(steps: int, stream, with_cpu: bool) -> dict:
    """The 256 x 64 FP64 channel (circle, 64 markers, Re 0.1): 2.36 MB of populations stay in
    the caches, so a step is bound by the latency of the particle phase (the sweep runs beside
    it in the overlapped schedule) and the hand-over, not by HBM.  Reported as time per step;
    the oracle runs the same steps on one thread and on all cores."""
    from paper_1808_01448_amd import lbib
    from paper_1808_01448_amd import workloads as W

    w = W.channel_small_fp64()
    cells = w["lattice"]["nx"] * w["lattice"]["ny"]
    sim = lbib.Sim(w, stream=stream)
    try:
        sim.step(200)
        sim.sync()
        win = timed_window(sim, steps, stream)
        sweep_ms, _, part_ms = sweep_timing(sim, 500)
    finally:
        sim.close()
    out = {"workload": w["name"] + " (256 x 64, FP64, circle r 8, 64 markers, Re 0.1)", "steps": steps,
           "us_per_step": round(win["seconds"] * 1e6 / steps, 3),
           "us_per_step_gpu_events": round(win["gpu_seconds"] * 1e6 / steps, 3),
           "mlups": round(cells * steps / win["seconds"] / 1e6, 1),
           "sweep_avg_us": round(sweep_ms * 1e3, 2), "particle_launch_avg_us": round(part_ms * 1e3, 2),
           "bound": "latency: the particle phase's chain of dependent steps, with the sweep overlapped behind it "
                    "(2.36 MB of state stays in the caches)"}
    if with_cpu:
        out["oracle_one_thread"] = cpu_oracle(w, 2000, threads=1)
        out["oracle_all_cores"] = cpu_oracle(w, 2000)
    log(f"bench: 256x64 FP64: {out['us_per_step']} us/step")
    return out


def batched_leg(steps: int, stream) -> dict:
    """The 216-simulation parameter sweep (FP32): the pool against the plain loops."""
    from paper_1808_01448_amd import measure
    from paper_1808_01448_amd import workloads as W

    ws = W.batched_sweep(0)
    cells = sum(w["lattice"]["nx"] * w["lattice"]["ny"] for w in ws)
    log(f"bench: batched sweep, {len(ws)} simulations, {cells / 1e6:.1f} M nodes, pool {steps} steps")
    pool = measure.pool_throughput(ws, steps, 20, stream=stream, autotune=10)
    log(f"bench: pool {pool['mlups']:.0f} MLUPS; plain loop")
    seq = measure.plain_sequential(ws, steps, 5, stream=stream)
    log(f"bench: plain sequential {seq['mlups']:.0f} MLUPS; plain concurrent")
    conc = measure.plain_concurrent(ws, steps, 5)
    log(f"bench: plain concurrent {conc['mlups']:.0f} MLUPS")
    # the captured-graph form of the pool step at the autotuner's tile shape: runs of 50 steps
    # replayed as one HIP graph (the autotuner keeps it only when it is faster)
    tx, tpb, _ = pool["config"]
    graph = measure.pool_throughput(ws, steps, 20, stream=stream, config=(tx, tpb, 50))
    log(f"bench: pool with graph replay {graph['mlups']:.0f} MLUPS")
    sweep_gbs = 72.0 * cells / (pool["sweep_avg_us"] * 1e-6) / 1e9
    return {
        "workload": "parameter sweep: 216 simulations (shape x ligand density x bond strength x Re x seed), "
                    "grids nx U[512,2048] x ny U[128,256], FP32, tau 0.8",
        "simulations": len(ws), "nodes": cells, "steps": steps, "unit": "MLUPS",
        "pool": round(pool["mlups"], 1),
        "plain_sequential": round(seq["mlups"], 1),
        "plain_concurrent_streams": round(conc["mlups"], 1),
        "speedup_vs_plain_sequential": round(pool["mlups"] / seq["mlups"], 3),
        "speedup_vs_plain_concurrent": round(pool["mlups"] / conc["mlups"], 3),
        "pool_ms_per_step": round(pool["ms_per_step"], 4),
        "pool_config": dict(zip(("tile_x", "tiles_per_block", "graph_steps"), pool["config"])),
        "pool_graph_replay": {"mlups": round(graph["mlups"], 1), "ms_per_step": round(graph["ms_per_step"], 4),
                              "config": dict(zip(("tile_x", "tiles_per_block", "graph_steps"), graph["config"]))},
        "pool_sweep_avg_us": round(pool["sweep_avg_us"], 2),
        "pool_particle_avg_us": round(pool["particle_avg_us"], 2),
        "pool_sweep_roofline": {"bound": "hbm", "achieved": round(sweep_gbs, 1), "peak": HBM_PEAK_GBS,
                                "unit": "GB/s", "frac": round(sweep_gbs / HBM_PEAK_GBS, 4)},
        "accuracy": "each pooled simulation bit-identical to its plain run",
    }


def multi_leg(steps: int, err_steps: int, stream) -> dict:
    """2048 x 512 channel with 32 particles (aspect ratio 1-3, area 0.025 H^2 each), Re 0.1:
    throughput with FP32, FP16 and BF16 storage of f - w_q and FP16 and BF16 storage of
    f - f_eq (the "_neq" storages), and each storage's error against the FP64 oracle over the
    first err_steps steps."""
    import numpy as np

    import oracle
    from paper_1808_01448_amd import lbib
    from paper_1808_01448_amd import workloads as W

    w = W.multi_particle_channel(2048, 512, 32, 0)
    n = len(w["particles"])
    cells = w["lattice"]["nx"] * w["lattice"]["ny"]
    log(f"bench: 32-particle leg, FP64 oracle over {err_steps} steps")
    o = oracle.Sim.from_workload(W.with_precision(w, "fp64"))
    t0 = time.perf_counter()
    _, to = o.step_all(err_steps)
    t_orc = time.perf_counter() - t0
    _, uxo, uyo = o.fields()
    x0 = np.array([[e["particle"]["xc"], e["particle"]["yc"]] for e in w["particles"]])

    def rel(a, b):
        return float(np.linalg.norm(a - b) / np.linalg.norm(b))

    out = {"workload": "2048 x 512 channel, 32 particles (aspect ratio U[1,3], area 0.025 H^2, random angle, "
                       "boundary gaps >= 4 lu), Re 0.1, tau 0.8, ligand density and bond strength per particle",
           "schedule": "one-launch split phase (the default): workgroups claim their particles, spread, meet and "
                       "evaluate the loads; then the sweep",
           "unit": "MLUPS", "steps_timed": steps, "error_steps": err_steps,
           "oracle_seconds": round(t_orc, 2), "storages": {}}
    for prec in ("fp32", "fp16", "bf16", "fp16_neq", "bf16_neq"):
        wp = W.with_precision(w, prec)
        s = lbib.Sim(wp, stream=stream)
        for k in range(n):
            s.trace_enable(err_steps, k)
        s.step(err_steps)
        s.sync()
        tg = np.stack([s.trace(err_steps, k) for k in range(n)], axis=1)
        _, ux, uy = s.fields()
        err = {"velocity": rel(tg[..., 4:6], to[..., 4:6]),
               "displacement": rel(tg[..., 1:3] - x0, to[..., 1:3] - x0),
               "force": rel(tg[..., 7:9], to[..., 7:9]),
               "field": rel(np.stack([ux, uy]), np.stack([uxo, uyo])),
               "bond_count_steps_differing": int((tg[..., -2] != to[..., -2]).sum())}
        s.step(20)
        s.sync()
        win = timed_window(s, steps, stream)
        s.kernel_timing(7)
        s.step(50)
        k_ms = [s.kernel_time(k)[0] / max(s.kernel_time(k)[1], 1) for k in range(3)]
        s.kernel_timing(0)
        bpu = s.bytes_per_update
        s.close()
        sweep_gbs = bpu * cells / (k_ms[0] * 1e-3) / 1e9
        out["storages"][prec] = {
            "mlups": round(cells * steps / win["seconds"] / 1e6, 1),
            "ms_per_step": round(win["seconds"] * 1e3 / steps, 4),
            "bytes_per_update": bpu, "sweep_us": round(k_ms[0] * 1e3, 2),
            "particle_phase_us": round((k_ms[1] + k_ms[2]) * 1e3, 2),
            "sweep_gbs": round(sweep_gbs, 1), "sweep_frac_of_8tbs": round(sweep_gbs / HBM_PEAK_GBS, 4),
            "error_vs_fp64_oracle": {k: (round(v, 8) if isinstance(v, float) else v) for k, v in err.items()},
        }
        log(f"bench: {prec}: {out['storages'][prec]['mlups']} MLUPS, velocity error {err['velocity']:.2e}")
    # the schedules of the split particle phase on the FP32 case (results are bit-identical)
    out["schedules_fp32"] = {}
    for mode, name in ((2, "one launch (default): particles claimed by their workgroups, no co-residency needed"),
                       (1, "chained: loads launch beside the sweep, device hand-over"),
                       (3, "serial: spread, loads, sweep in order on one stream")):
        s = lbib.Sim(W.with_precision(w, "fp32"), stream=stream)
        s.set_overlap(mode)
        s.step(20)
        s.sync()
        win = timed_window(s, steps, stream)
        s.close()
        out["schedules_fp32"][f"mode_{mode}"] = {"schedule": name, "ms_per_step": round(win["seconds"] * 1e3 / steps, 4),
                                                 "mlups": round(cells * steps / win["seconds"] / 1e6, 1)}
    return out


def serving_leg(n: int, scale: float, stream) -> dict:
    """Poisson arrivals of single-particle solves at 0.7 x the server's capacity, served by
    continuous batching, against the plain one-simulation-at-a-time server on the same arrival
    trace; and both at saturation (every request of a sample arriving at once)."""
    import numpy as np

    from paper_1808_01448_amd import measure
    from paper_1808_01448_amd import workloads as W

    steps_range = (max(1, int(5_000 * scale)), max(1, int(50_000 * scale)))
    ws = W.serving_requests(n, 0, steps_range=steps_range)
    mean_lu = float(np.mean([w["lattice"]["nx"] * w["lattice"]["ny"] * w["steps"] for w in ws]))
    # saturation: the first half of the requests at a quarter of their steps, all arriving at
    # once, through the server and through the plain server; the served figure sets the rate
    sample = [dict(w, steps=max(1, w["steps"] // 4)) for w in ws[: max(1, n // 2)]]
    log(f"bench: serving at saturation, {len(sample)} requests arriving together")
    sat = measure.serve_trace(sample, np.zeros(len(sample)), stream=stream, progress=log)
    log(f"bench: served at saturation {sat['mlups']:.0f} MLUPS; plain server")
    sat_plain = measure.plain_fifo(sample, np.zeros(len(sample)), stream=stream, progress=log)
    capacity = sat["mlups"] * 1e6 / mean_lu
    rate = 0.7 * capacity
    arrivals = W.poisson_arrivals(n, rate, seed=0)
    log(f"bench: serving {n} requests at {rate:.2f}/s (capacity {capacity:.2f}/s)")
    srv = measure.serve_trace(ws, arrivals, stream=stream, progress=log)
    log(f"bench: served in {srv['makespan_s']:.2f} s; plain server on the same trace")
    plain = measure.plain_fifo(ws, arrivals, stream=stream, progress=log)
    same = all(r["final_state"] == p for r, p in zip(srv["results"], plain["finals"]))
    ls, lp = measure.percentiles(srv["latency_s"]), measure.percentiles(plain["latency_s"])
    return {
        "workload": f"{n} single-particle solves, nx log-U[256,4096] x ny log-U[64,512], steps U[{steps_range[0]},"
                    f"{steps_range[1]}], shape/ligand density/bond strength/Re from the sweep's sets, FP32",
        "lattice_updates": int(mean_lu * n),
        "saturation": {"sample": f"the first {len(sample)} requests at a quarter of their steps, all arriving at once",
                       "served_mlups": round(sat["mlups"], 1), "plain_mlups": round(sat_plain["mlups"], 1),
                       "speedup_vs_plain": round(sat["mlups"] / sat_plain["mlups"], 3),
                       "makespan_s": {"served": round(sat["makespan_s"], 3), "plain": round(sat_plain["makespan_s"], 3)}},
        "arrival_rate_per_s": round(rate, 3), "capacity_per_s": round(capacity, 3), "load": 0.7,
        "unit": "MLUPS", "served": round(srv["mlups"], 1), "plain": round(plain["mlups"], 1),
        "speedup_vs_plain": round(srv["mlups"] / plain["mlups"], 3),
        "latency_s": {"served": {k: round(v, 4) for k, v in ls.items()},
                      "plain": {k: round(v, 4) for k, v in lp.items()}},
        "wait_s_served": {k: round(v, 4) for k, v in measure.percentiles(srv["wait_s"]).items()},
        "makespan_s": {"served": round(srv["makespan_s"], 3), "plain": round(plain["makespan_s"], 3)},
        "chunk_steps": 200, "chunks": srv["chunks"], "failed": srv["failed"],
        "results_equal_plain": bool(same),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=4000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--long-steps", type=int, default=1000,
                    help="steps of the second, longer window that shows the fixed cost of a call")
    ap.add_argument("--legs", default=",".join(LEGS), help="comma-separated legs beside the headline: " + ",".join(LEGS))
    ap.add_argument("--cpu-steps", type=int, default=100, help="oracle steps of the CPU baseline on all cores")
    ap.add_argument("--cpu-steps-one-thread", type=int, default=10, help="oracle steps on one thread")
    ap.add_argument("--no-timing-events", action="store_true", help="time only the whole steps")
    ap.add_argument("--serial-schedule", action="store_true",
                    help="run the 4096 x 1024 and 8192 x 4096 legs in the serial schedule (for counter collection, "
                         "which serialises kernel dispatches: the overlapped schedule's device-side hand-over between "
                         "its two streams does not survive that, its bounded waits time out)")
    ap.add_argument("--beyond-steps", type=int, default=200, help="timed steps per storage of the 8192 x 4096 leg")
    ap.add_argument("--c1-steps", type=int, default=2000, help="timed steps of the 256 x 64 FP64 leg")
    ap.add_argument("--batched-steps", type=int, default=200, help="steps of the 216-simulation sweep")
    ap.add_argument("--serve-requests", type=int, default=256, help="requests of the serving leg")
    ap.add_argument("--serve-scale", type=float, default=1.0,
                    help="factor on the serving mix's step counts (1: 5k-50k steps per request)")
    ap.add_argument("--multi-steps", type=int, default=500,
                    help="steps of the 32-particle 2048 x 512 leg per storage precision")
    ap.add_argument("--multi-err-steps", type=int, default=200, help="steps of that leg compared with the FP64 oracle")
    args = ap.parse_args()
    legs = {x for x in args.legs.split(",") if x}
    if legs - set(LEGS):
        ap.error(f"unknown legs {sorted(legs - set(LEGS))}")

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: a single simulation of this path runs on one device and the "
              "benchmark has no multi-GPU form; run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1808_01448_amd import lbib
    from paper_1808_01448_amd import workloads as W

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    # the copy reference first, on an otherwise idle device (it allocates and frees 4 GiB)
    copy_gbs = lbib.bandwidth_probe(1 << 31, 10, stream=stream)
    log(f"bench: copy bandwidth {copy_gbs:.0f} GB/s (2 GiB read + 2 GiB written)")

    w = W.channel_large_fp32()
    nx, ny = w["lattice"]["nx"], w["lattice"]["ny"]
    cells = nx * ny
    log(f"bench: building {w['name']}")
    sim = lbib.Sim(w, stream=stream)
    if args.serial_schedule:
        sim.set_overlap(0)
    bpu = sim.bytes_per_update
    pull = sim.pull
    log(f"bench: warmup {args.warmup} steps")
    sim.step(args.warmup)
    sim.sync()

    log(f"bench: timing {args.steps} steps")
    win = timed_window(sim, args.steps, stream, events=False)
    dt = win["seconds"]
    ms_step = dt * 1e3 / args.steps
    mlups = cells * args.steps / dt / 1e6
    log(f"bench: {ms_step * 1e3:.2f} us/step ({mlups:.0f} MLUPS); {args.long_steps}-step window")
    long_win = timed_window(sim, args.long_steps, stream)
    long_ms = long_win["seconds"] * 1e3 / args.long_steps
    # what one lbib_step call costs beyond its steps (launch and synchronisation latency on
    # the host, the joins of the two streams at the call's start and end on the GPU): a short
    # window of its own against the long window's rate, the median of five
    ks = 20
    shorts = [timed_window(sim, ks, stream, events=False) for _ in range(5)]
    fixed = sorted((x["seconds"] - ks * long_ms * 1e-3) * 1e6 for x in shorts)[2]
    shorts_ev = [timed_window(sim, ks, stream) for _ in range(5)]
    fixed_gpu = sorted((x["gpu_seconds"] - ks * long_win["gpu_seconds"] / args.long_steps) * 1e6 for x in shorts_ev)[2]
    # the timed window's length again with HIP events around it (events on the stream make
    # lbib_step join its streams at the call's start, so they stay out of the timed window)
    win_ev = timed_window(sim, args.steps, stream)
    window = {
        "ms_per_step_gpu_events": round(win_ev["gpu_seconds"] * 1e3 / args.steps, 5),
        "ms_per_step_host_same_window_with_events": round(win_ev["seconds"] * 1e3 / args.steps, 5),
        "long_window": {"steps": args.long_steps, "ms_per_step": round(long_ms, 5),
                        "ms_per_step_gpu_events": round(long_win["gpu_seconds"] * 1e3 / args.long_steps, 5),
                        "mlups": round(cells * args.long_steps / long_win["seconds"] / 1e6, 1)},
        "short_window_steps": ks,
        "fixed_cost_us_per_call": round(fixed, 1),
        "fixed_cost_us_per_call_gpu_events": round(fixed_gpu, 1),
    }

    roofline = None
    if not args.no_timing_events:
        # HIP events around a launch delay the hand-over between the two streams, so the
        # whole steps above run without them; the sweep's duration comes from a third region
        # with events on the sweep launches only
        kr = 1000
        log(f"bench: {kr} steps with HIP events on the sweep")
        sweep_ms, n0, part_ms = sweep_timing(sim, kr)
        achieved = bpu * cells / (sweep_ms * 1e-3) / 1e9
        roofline = {
            "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), **measured_traffic(cells),
            "kernel": sweep_kernel_name("fp32", args.serial_schedule), "algorithmic_bytes_per_launch": bpu * cells,
            "avg_launch_us": round(sweep_ms * 1e3, 2), "launches_timed": n0,
            "timing": f"HIP events (hipExtLaunchKernelGGL) on the sweep's stream over {kr} steps after the "
                      f"timed windows",
            "frac_of_measured_copy": round(achieved / copy_gbs, 4) if copy_gbs > 0 else None,
            "working_set_note": "302 MB of populations against a 256 MB last-level cache: part of each sweep is "
                                "served from that cache; beyond_cache gives the sweep at 2.4 GB",
            "particle_launch_avg_us": round(part_ms * 1e3, 2),
            "particle_timing": ("one launch per step" if args.serial_schedule else
                                "one resident launch over a call's steps: its duration divided by the steps"),
            "schedule": ("serial: the particle phase, then a sweep of every node, on one stream"
                         if args.serial_schedule else
                         "particle phases and sweeps on two streams with no event between them, handing "
                         "over through device memory; one particle launch stays resident over a call's "
                         "steps, and the sweep's box tiles are taken by workgroups at the head of its grid "
                         "once the particle has published its spread force"),
        }
    p = sim.particle()
    sim.close()

    beyond = beyond_cache_leg(args.beyond_steps, stream, args.serial_schedule) if "beyond" in legs else None
    c1 = c1_leg(args.c1_steps, stream, "cpu" in legs) if "c1" in legs else None
    batched = batched_leg(args.batched_steps, stream) if "batched" in legs else None
    multi = multi_leg(args.multi_steps, args.multi_err_steps, stream) if "multi" in legs else None
    served = serving_leg(args.serve_requests, args.serve_scale, stream) if "serve" in legs else None

    cpu = cpu_one = None
    if "cpu" in legs:
        log(f"bench: CPU oracle baseline, {args.cpu_steps} steps on all cores, "
            f"{args.cpu_steps_one_thread} on one thread")
        cpu = cpu_oracle(w, args.cpu_steps)
        cpu_one = cpu_oracle(w, args.cpu_steps_one_thread, threads=1)

    out = {
        "metric": METRIC,
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": w["name"], "nx": nx, "ny": ny, "storage": "fp32 (f - w_q)",
            "particles": 1, "shape": "ellipse AR3 48x16", "markers": w["particle"]["n_markers"],
            "rho_l": "7/10", "bond_strength": 2, "re": w["lattice"]["re"], "tau": w["lattice"]["tau"],
            "particle_phase_dtype": "f64", "collision_dtype": "f64", "layout": "pull" if pull else "push",
        },
        "window": window,
        "roofline": roofline,
        "copy_bandwidth_gbs": round(copy_gbs, 1),
        "cpu_baseline": cpu,
        "cpu_baseline_one_thread": cpu_one,
        "beyond_cache": beyond,
        "channel_256x64_fp64": c1,
        "batched": batched,
        "served": served,
        "multi_particle": multi,
        "final_particle": {k: p[k] for k in ("step", "xc", "yc", "theta", "n_bonds")},
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
