#!/usr/bin/env python3
"""Benchmark of the LB-IB adhesion hot path on one MI355X.

A step is one full time step n -> n+1 of the coupled method (particle phase + lattice
sweep) on the 4096 x 1024 FP32 channel with one aspect-ratio-3 ellipse (256 markers,
ligand density 0.7, bond strength 2, Re 1), inputs resident in HBM.  Prints one JSON line:
whole-step throughput in MLUPS, the lattice sweep's roofline (algorithmic bytes per
launch over its HIP-event-timed average duration, against the 8 TB/s HBM peak), the
measured copy bandwidth, and the FP64 CPU oracle timed on a bounded sample of the same
workload on this host's cores.
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
# the lattice sweep's device code: the counters in TRAFFIC_FILE are valid for these sources only
KERNEL_SRCS = [os.path.join(ROOT, "paper_1808_01448_amd", "csrc", f)
               for f in ("lbib_sweep.hip", "lbib_collide.hpp", "lbib_device.hpp")]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SRCS:
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(cells: int):
    """HBM bytes per sweep launch from the committed rocprofv3 counter summary, or None when
    the counters were taken on a different kernel source."""
    try:
        t = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_sha256_16") != kernel_source_hash() or t.get("cells") != cells:
        return None
    return t.get("hbm_bytes_per_launch")


def cpu_baseline(workload: dict, steps: int):
    import oracle

    o = oracle.Sim.from_workload(workload)
    o.step(1)  # first touch of the arrays outside the timed region
    t0 = time.perf_counter()
    o.step(steps)
    dt = time.perf_counter() - t0
    cells = workload["lattice"]["nx"] * workload["lattice"]["ny"]
    return {
        "value": round(cells * steps / dt / 1e6, 3),
        "unit": "MLUPS",
        "cores": oracle.num_threads(),
        "kind": "oracle",
        "sample": f"{steps} full steps (after 1 untimed) of the same {workload['lattice']['nx']}x"
                  f"{workload['lattice']['ny']} workload, FP64, {dt:.1f} s",
    }


def batched_leg(steps: int, stream) -> dict:
    """The 216-simulation parameter sweep (FP32): the pool against the plain loops."""
    from paper_1808_01448_amd import lbib, measure
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
           "schedule": "per step: one particle launch (every particle spreads, grid barrier, loads, bonds, update), "
                       "then the sweep",
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
        t0 = time.perf_counter()
        s.step(steps)
        s.sync()
        dt = time.perf_counter() - t0
        s.kernel_timing(7)
        s.step(50)
        k_ms = [s.kernel_time(k)[0] / max(s.kernel_time(k)[1], 1) for k in range(3)]
        s.kernel_timing(0)
        bpu = s.bytes_per_update
        s.close()
        sweep_gbs = bpu * cells / (k_ms[0] * 1e-3) / 1e9
        out["storages"][prec] = {
            "mlups": round(cells * steps / dt / 1e6, 1), "ms_per_step": round(dt * 1e3 / steps, 4),
            "bytes_per_update": bpu, "sweep_us": round(k_ms[0] * 1e3, 2),
            "particle_phase_us": round((k_ms[1] + k_ms[2]) * 1e3, 2),
            "sweep_gbs": round(sweep_gbs, 1), "sweep_frac_of_8tbs": round(sweep_gbs / HBM_PEAK_GBS, 4),
            "error_vs_fp64_oracle": {k: (round(v, 8) if isinstance(v, float) else v) for k, v in err.items()},
        }
        log(f"bench: {prec}: {out['storages'][prec]['mlups']} MLUPS, velocity error {err['velocity']:.2e}")
    return out


def serving_leg(n: int, full: bool, stream) -> dict:
    """Poisson arrivals of single-particle solves at 0.7 x the server's measured capacity,
    served by continuous batching, against the plain one-simulation-at-a-time server on the
    same arrival trace."""
    import numpy as np

    from paper_1808_01448_amd import measure
    from paper_1808_01448_amd import workloads as W

    steps_range = (5_000, 50_000) if full else (1_000, 5_000)
    ws = W.serving_requests(n, 0, steps_range=steps_range)
    mean_lu = float(np.mean([w["lattice"]["nx"] * w["lattice"]["ny"] * w["steps"] for w in ws]))
    # pilot: the first half of the requests at a quarter of their steps, all arriving at once
    pilot_ws = [dict(w, steps=max(1, w["steps"] // 4)) for w in ws[: max(1, n // 2)]]
    log(f"bench: serving pilot, {len(pilot_ws)} requests arriving together")
    pilot = measure.serve_trace(pilot_ws, np.zeros(len(pilot_ws)), stream=stream)
    capacity = pilot["mlups"] * 1e6 / mean_lu
    rate = 0.7 * capacity
    arrivals = W.poisson_arrivals(n, rate, seed=0)
    log(f"bench: serving {n} requests at {rate:.2f}/s (capacity {capacity:.2f}/s)")
    srv = measure.serve_trace(ws, arrivals, stream=stream)
    log(f"bench: served in {srv['makespan_s']:.2f} s; plain server on the same trace")
    plain = measure.plain_fifo(ws, arrivals, stream=stream)
    same = all(r["final_state"] == p for r, p in zip(srv["results"], plain["finals"]))
    ls, lp = measure.percentiles(srv["latency_s"]), measure.percentiles(plain["latency_s"])
    return {
        "workload": f"{n} single-particle solves, nx log-U[256,4096] x ny log-U[64,512], steps U[{steps_range[0]},"
                    f"{steps_range[1]}], shape/ligand density/bond strength/Re from the sweep's sets, FP32"
                    + ("" if full else " (step counts 1/10 of the full mix)"),
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
    ap.add_argument("--cpu-steps", type=int, default=60, help="oracle steps of the CPU baseline (0: skip)")
    ap.add_argument("--no-timing-events", action="store_true", help="time only the whole steps")
    ap.add_argument("--batched-steps", type=int, default=200,
                    help="steps of the 216-simulation sweep, pooled and plain (0: skip)")
    ap.add_argument("--serve-requests", type=int, default=64, help="requests of the serving leg (0: skip)")
    ap.add_argument("--multi-steps", type=int, default=500,
                    help="steps of the 32-particle 2048 x 512 leg per storage precision (0: skip)")
    ap.add_argument("--multi-err-steps", type=int, default=200,
                    help="steps of that leg compared with the FP64 oracle")
    ap.add_argument("--serve-full", action="store_true",
                    help="serving leg at the full request mix: 256 requests of 5k-50k steps (several minutes)")
    args = ap.parse_args()

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
    w = W.channel_large_fp32()
    nx, ny = w["lattice"]["nx"], w["lattice"]["ny"]
    cells = nx * ny

    stream = torch.cuda.Stream()
    log(f"bench: building {w['name']}")
    sim = lbib.Sim(w, stream=stream)
    bpu = sim.bytes_per_update
    pull = sim.pull
    log(f"bench: warmup {args.warmup} steps")
    sim.step(args.warmup)
    sim.sync()

    copy_gbs = lbib.bandwidth_probe(1 << 31, 10, stream=stream)
    log(f"bench: copy bandwidth {copy_gbs:.0f} GB/s")

    torch.cuda.synchronize()
    log(f"bench: timing {args.steps} steps")
    t0 = time.perf_counter()
    sim.step(args.steps)
    sim.sync()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_step = dt * 1e3 / args.steps
    mlups = cells * args.steps / dt / 1e6

    roofline = None
    if not args.no_timing_events:
        # HIP events around a launch delay the hand-over between the two streams by ~9 us per
        # step, so the whole steps above run without them; the sweep's duration comes from a
        # second region of the same run with events on the sweep launches only.
        kr = min(args.steps, 1000)
        log(f"bench: {kr} steps with HIP events on the sweep")
        sim.kernel_timing(1)
        sim.step(kr)
        ms0, n0 = sim.kernel_time(0)
        kp = min(args.steps, 200)
        sim.kernel_timing(7)
        sim.step(kp)
        ms1, n1 = sim.kernel_time(1)
        sim.kernel_timing(0)
        sweep_ms = ms0 / max(n0, 1)
        part_ms = ms1 / max(n1, 1)
        achieved = bpu * cells / (sweep_ms * 1e-3) / 1e9
        traffic = measured_traffic(cells)
        roofline = {
            "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "kernel": "sweep_overlap_kernel<float, push>", "algorithmic_bytes_per_launch": bpu * cells,
            "avg_launch_us": round(sweep_ms * 1e3, 2), "launches_timed": n0,
            "timing": f"HIP events (hipExtLaunchKernelGGL) on the sweep's stream over {kr} steps after the "
                      f"throughput region",
            "frac_of_measured_copy": round(achieved / copy_gbs, 4) if copy_gbs > 0 else None,
            "particle_launch_avg_us": round(part_ms * 1e3, 2),
            "schedule": "particle phases and sweeps on two streams with no event between them, handing "
                        "over through device memory; the sweep's box tiles are taken by workgroups at the "
                        "head of its grid once the particle has published its spread force",
        }
    p = sim.particle()
    sim.close()

    batched = None
    if args.batched_steps > 0:
        batched = batched_leg(args.batched_steps, stream)

    multi = None
    if args.multi_steps > 0:
        multi = multi_leg(args.multi_steps, args.multi_err_steps, stream)

    served = None
    if args.serve_requests > 0 or args.serve_full:
        served = serving_leg(256 if args.serve_full else args.serve_requests, args.serve_full, stream)

    cpu = None
    if args.cpu_steps > 0:
        log(f"bench: CPU oracle baseline, {args.cpu_steps} steps")
        cpu = cpu_baseline(w, args.cpu_steps)

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
            "particle_phase_dtype": "f64", "layout": "pull" if pull else "push",
        },
        "roofline": roofline,
        "copy_bandwidth_gbs": round(copy_gbs, 1),
        "cpu_baseline": cpu,
        "batched": batched,
        "served": served,
        "multi_particle": multi,
        "final_particle": {k: p[k] for k in ("step", "xc", "yc", "theta", "n_bonds")},
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
