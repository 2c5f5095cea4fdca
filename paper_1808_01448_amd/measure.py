"""Throughput of many simulations on one GPU: the pool against the plain per-simulation loop.

Used by bench.py.  Every figure is aggregate lattice updates per second over all
simulations (MLUPS), with inputs resident in HBM and the warm-up steps outside the timed
region.  The pool and the plain loops run the same kernels on the same descriptors; the
pool's results are bit-identical to the plain ones (tests/test_gpu_pool.py).
"""
from __future__ import annotations

import time

from . import lbib


def _cells(w: dict) -> int:
    return int(w["lattice"]["nx"]) * int(w["lattice"]["ny"])


def pool_throughput(ws: list, steps: int, warmup: int, *, precision: int = lbib.FP32, stream=None,
                    autotune: int = 0, config=None) -> dict:
    """All simulations in one pool; `steps` pool steps timed after `warmup` untimed ones (and,
    with autotune > 0, the autotuner's trials of that many steps each).  The timed run uses
    the chosen launch configuration as it is (graph replay included); a second, shorter run
    with kernel timing on gives the per-kernel averages."""
    budget = 200 << 30
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
