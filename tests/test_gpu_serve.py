"""GPU tests of the continuous-batching server.

Requests arrive while others run, wait for memory and slots, join the pool between chunks
of steps and leave when done.  Each result must equal the same solve run alone, bit for
bit; admission must respect the memory budget and (with no bypass) the arrival order."""
import sys

import numpy as np
import pytest

from paper_1808_01448_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def L():
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    from paper_1808_01448_amd import lbib

    lbib.lib()
    return lbib


def requests(n=10, seed=3):
    return W.serving_requests(n, seed, steps_range=(20, 90), nx_range=(64, 160), ny_range=(32, 64))


def alone(L, w):
    s = L.Sim(w)
    s.step(int(w["steps"]))
    s.sync()
    p = s.particle()
    s.close()
    return p


def drive(L, S, ws, arrivals, budget):
    """Real-time loop; checks the budget after every round; returns results by request."""
    t0 = S.clock()
    n, i, res, ids, peak = len(ws), 0, {}, {}, 0
    while len(res) < n:
        now = S.clock() - t0
        while i < n and arrivals[i] <= now:
            ids[S.submit(ws[i], int(ws[i]["steps"]), t0 + float(arrivals[i]))] = i
            i += 1
        q, r, used, _ = S.stats()
        if q == 0 and r == 0:
            continue
        S.progress()
        q, r, used, _ = S.stats()
        peak = max(peak, used)
        assert used <= budget
        for rid in S.take_completed():
            res[ids[rid]] = S.result(rid)
            S.release(rid)
    return [res[k] for k in range(n)], peak


@pytest.mark.parametrize("bypass", [0, 2])
def test_server_results_equal_standalone(L, bypass):
    ws = requests()
    fp = [L.Pool.footprint(w) for w in ws]
    budget = sum(sorted(fp)[:3])  # about three requests at a time: the rest queue
    arrivals = W.poisson_arrivals(len(ws), 300.0, seed=3)
    S = L.Server(L.FP32, budget_bytes=budget, max_members=16, chunk_steps=7, max_bypass=bypass)
    res, peak = drive(L, S, ws, arrivals, budget)
    _, _, _, chunks = S.stats()
    S.close()
    say("bypass", bypass, "chunks", chunks, "peak bytes", peak, "budget", budget)
    for k, (w, r) in enumerate(zip(ws, res)):
        assert r["state"] == L.REQ_DONE and r["steps_done"] == w["steps"]
        assert r["t_arrival"] <= r["t_admit"] <= r["t_done"]
        assert r["final_state"] == alone(L, w), w["name"]
    if bypass == 0:  # strict arrival order of admission
        admits = [r["t_admit"] for r in res]
        assert admits == sorted(admits)


def test_server_failed_request_and_validation(L):
    ws = requests(4, seed=5)
    bad = W.channel_small_binding("fp32")
    bad["lattice"].update(nx=64, ny=32, seed=0)
    bad["particle"].update(a_major=4.0, b_minor=4.0, xc=16.0, yc=-0.5 + 1e-6 + 4.0, n_markers=48)
    bad["steps"] = 60  # touches the wall after a few tens of steps
    S = L.Server(L.FP32, budget_bytes=1 << 30, max_members=8, chunk_steps=16, max_bypass=0)
    ids = [S.submit(w, int(w["steps"])) for w in ws]
    bid = S.submit(bad, 60)
    with pytest.raises(L.LbibError) as ei:
        huge = W.serving_requests(1, 0, steps_range=(10, 10), nx_range=(4096, 4096), ny_range=(512, 512))[0]
        S2 = L.Server(L.FP32, budget_bytes=1 << 20, max_members=8, chunk_steps=16)
        try:
            S2.submit(huge, 10)
        finally:
            S2.close()
    assert ei.value.status == L.E_FULL
    with pytest.raises(L.LbibError) as ei:
        w = dict(ws[0])
        w["particle"] = dict(w["particle"], n_markers=3)
        S.submit(w, 10)
    assert ei.value.status == L.E_INVALID
    done = set()
    while len(done) < 5:
        S.progress()
        done.update(S.take_completed())
    r = S.result(bid)
    assert r["state"] == L.REQ_FAILED and 0 < r["steps_done"] < 60
    for rid, w in zip(ids, ws):
        assert S.result(rid)["final_state"] == alone(L, w)
    S.close()
