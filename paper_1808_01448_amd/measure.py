"""Throughput of many simulations on one GPU: the pool against the plain per-simulation loop.

Used by bench.py.  Every figure is aggregate lattice updates per second over all
simulations (MLUPS), with inputs resident in HBM and the warm-up steps outside the timed
region.  The pool and the plain loops run the same kernels on the same descriptors; the
pool's results are bit-identical to the plain ones (tests/test_gpu_pool.py).
"""
from __future__ import annotations

import time

import numpy as np

from . import lbib


def _cells(w: dict) -> int:
    return int(w["lattice"]["nx"]) * int(w["lattice"]["ny"])


def pool_throughput(ws: list, steps: int, warmup: int, *, precision: int = lbib.FP32, stream=None,
                    autotune: int = 0, config=None) -> dict:
    """All simulations in one pool; `steps` pool steps timed after `warmup` untimed ones (and,
    with autotune > 0, the autotuner's trials of that many steps each).  The timed run uses
    the chosen launch configuration as it is (graph replay included); a second, shorter run
    with kernel timing on gives the per-kernel averages."""
    budget = sum(lbib.Pool.footprint(w) for w in ws) + (256 << 20)
    P = lbib.Pool(precision, budget_bytes=budget, max_members=max(len(ws), 1), stream=stream)
    try:
        for w in ws:
            P.add(w, 1 << 40)
        if config is not None:
            P.set_config(*config)
        if autotune > 0:
            P.autotune(autotune)
        P.step(warmup)
        P.poll()
        t0 = time.perf_counter()
        P.step(steps)
        P.poll()
        dt = time.perf_counter() - t0
        cells = sum(_cells(w) for w in ws)
        out = {"mlups": cells * steps / dt / 1e6, "ms_per_step": dt * 1e3 / steps, "config": P.config()}
        P.kernel_timing(True)
        k = max(steps // 4, 10)
        P.step(k)
        ms0, n0 = P.kernel_time(0)
        ms1, n1 = P.kernel_time(1)
        P.kernel_timing(False)
        out["sweep_avg_us"] = ms0 / max(n0, 1) * 1e3
        out["particle_avg_us"] = ms1 / max(n1, 1) * 1e3
        out["members"], _, out["bytes_in_use"] = P.usage()
        return out
    finally:
        P.close()


def plain_sequential(ws: list, steps: int, warmup: int, *, stream=None) -> dict:
    """The plain per-simulation loop: each simulation in turn, created, warmed up, then its
    `steps` steps timed; the figure sums the timed parts."""
    total = 0.0
    for w in ws:
        s = lbib.Sim(w, stream=stream)
        try:
            s.step(warmup)
            s.sync()
            t0 = time.perf_counter()
            s.step(steps)
            s.sync()
            total += time.perf_counter() - t0
        finally:
            s.close()
    cells = sum(_cells(w) for w in ws)
    return {"mlups": cells * steps / total / 1e6, "seconds": total}


def plain_concurrent(ws: list, steps: int, warmup: int) -> dict:
    """Every simulation on a stream of its own, all enqueued before any is waited for (the
    device runs as many streams at once as it has hardware queues)."""
    sims = []
    try:
        for w in ws:
            sims.append(lbib.Sim(w))
        for s in sims:
            s.step(warmup)
        for s in sims:
            s.sync()
        t0 = time.perf_counter()
        for s in sims:
            s.step(steps)
        for s in sims:
            s.sync()
        dt = time.perf_counter() - t0
    finally:
        for s in sims:
            s.close()
    cells = sum(_cells(w) for w in ws)
    return {"mlups": cells * steps / dt / 1e6, "seconds": dt}


def _lu(w: dict) -> int:
    return _cells(w) * int(w["steps"])


def serve_trace(ws: list, arrivals, *, chunk_steps: int = 200, max_bypass: int = 8, budget_bytes: int = 16 << 30,
                max_members: int = 4096, stream=None, autotune: bool = False, progress=None) -> dict:
    """Run the requests through the server in real time: request k is submitted when the
    server's clock passes arrivals[k] (seconds after the start) and stamped with that arrival
    time.  Returns per-request latencies (arrival -> result) and the aggregate throughput.
    progress (optional): called with a line of text after every 32nd completed request."""
    S = lbib.Server(lbib.FP32, budget_bytes=budget_bytes, max_members=max_members, chunk_steps=chunk_steps,
                    max_bypass=max_bypass, stream=stream)
    try:
        n = len(ws)
        t0 = S.clock()
        i = 0
        res = {}
        ids = {}
        while len(res) < n:
            now = S.clock() - t0
            while i < n and arrivals[i] <= now:
                ids[S.submit(ws[i], int(ws[i]["steps"]), t0 + float(arrivals[i]))] = i
                i += 1
            q, r, _, _ = S.stats()
            if q == 0 and r == 0:
                if i < n:
                    time.sleep(max(0.0, min(0.05, arrivals[i] - (S.clock() - t0))))
                continue
            S.progress()
            for rid in S.take_completed():
                res[ids[rid]] = S.result(rid)
                S.release(rid)
                if progress and len(res) % 32 == 0:
                    progress(f"served {len(res)}/{n} requests, {S.clock() - t0:.1f} s")
        t_end = S.clock()
        lat = np.array([res[k]["t_done"] - res[k]["t_arrival"] for k in range(n)])
        wait = np.array([res[k]["t_admit"] - res[k]["t_arrival"] for k in range(n)])
        makespan = t_end - t0
        lu = sum(_lu(w) for w in ws)
        _, _, _, chunks = S.stats()
        return {"latency_s": lat, "wait_s": wait, "makespan_s": makespan, "mlups": lu / makespan / 1e6,
                "results": [res[k] for k in range(n)], "chunks": chunks,
                "failed": sum(1 for k in range(n) if res[k]["state"] != lbib.REQ_DONE)}
    finally:
        S.close()


def plain_fifo(ws: list, arrivals, *, stream=None, progress=None) -> dict:
    """The plain server: one simulation at a time in arrival order, each created when the
    previous one has finished (or at its arrival), stepped to completion and read.
    progress (optional): called with a line of text after every 32nd completed request."""
    t0 = time.perf_counter()
    lat = np.zeros(len(ws))
    finals = []
    for k, w in enumerate(ws):
        now = time.perf_counter() - t0
        if arrivals[k] > now:
            time.sleep(arrivals[k] - now)
        s = lbib.Sim(w, stream=stream)
        try:
            s.step(int(w["steps"]))
            s.sync()
            finals.append(s.particle())
        finally:
            s.close()
        lat[k] = time.perf_counter() - t0 - arrivals[k]
        if progress and (k + 1) % 32 == 0:
            progress(f"plain server: {k + 1}/{len(ws)} requests, {time.perf_counter() - t0:.1f} s")
    makespan = time.perf_counter() - t0
    lu = sum(_lu(w) for w in ws)
    return {"latency_s": lat, "makespan_s": makespan, "mlups": lu / makespan / 1e6, "finals": finals}


def percentiles(x) -> dict:
    x = np.asarray(x, float)
    return {"p50": float(np.percentile(x, 50)), "p99": float(np.percentile(x, 99)), "mean": float(x.mean()),
            "max": float(x.max())}
