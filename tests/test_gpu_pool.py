"""GPU tests of the simulation pool (many simulations stepped by shared launches).

The pool runs the same device functions as a simulation run alone, so every member must
match its stand-alone run (serial schedule) bit for bit: populations, particle records,
bonds and trace.  The stand-alone runs are themselves held to the FP64 oracle by
test_gpu_sim.py; one member here is also compared with the oracle directly."""
import copy
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


def member(nx, ny, *, shape=0, a=4.0, b=4.0, nl=48, seed=0, tau=0.8, re=0.1, rho_l=(1, 2), strength=1,
           gap=None, xc=None, theta0=0.0, precision="fp64"):
    """A pool member: a particle close to the receptor wall (gap y_eq unless given)."""
    w = W.channel_small_binding(precision)
    lat = w["lattice"]
    lat.update(nx=nx, ny=ny, tau=tau, re=re, seed=seed)
    w["ligand"] = W._ligand(rho_l, strength)
    y_cr = W.Y_CR_HAT * ny
    g = W.Y_EQ_RATIO * y_cr if gap is None else gap
    hs = a if shape == 0 else float(np.hypot(a * np.cos(theta0), b * np.sin(theta0)))
    w["particle"] = dict(shape=shape, a_major=a, b_minor=b if shape == 1 else a, xc=nx / 4 if xc is None else xc,
                         yc=-0.5 + g + hs, theta0=theta0, rho_p=1.0, n_markers=nl)
    w["name"] = f"member_{nx}x{ny}_s{shape}_a{a}_nl{nl}_seed{seed}"
    return w


def mix(precision):
    """Members of different size, shape, marker count, ligands, flow and seed; one with a box
    too large for LDS (global scratch path) and one above 256 markers (more markers per
    thread for the whole launch)."""
    return [
        (member(64, 32, seed=0, precision=precision), 50),
        (member(96, 40, shape=1, a=6.0, b=2.0, nl=64, seed=7, tau=0.9, re=0.5, rho_l=(7, 10), strength=2,
                theta0=0.3, precision=precision), 30),
        (member(80, 36, nl=40, seed=3, re=0.2, precision=precision), 70),
        (member(128, 72, a=28.0, nl=256, seed=11, precision=precision), 20),
        (member(160, 64, shape=1, a=20.0, b=8.0, nl=300, seed=5, precision=precision), 40),
    ]


_ALONE = {}


def alone(L, w, steps):
    key = (w["name"], w["lattice"]["precision"], steps)
    if key not in _ALONE:
        _ALONE[key] = _alone(L, w, steps)
    return _ALONE[key]


def _alone(L, w, steps):
    s = L.Sim(w)
    s.set_overlap(0)
    s.trace_enable(steps)
    s.step(steps)
    s.sync()
    out = dict(particle=s.particle(), bonds=s.bonds()[0], f=s.f, trace=s.trace(steps))
    s.close()
    return out


def pooled(P, slot, steps):
    return dict(particle=P.particle(slot), bonds=P.bonds(slot)[0], f=P.field(slot, 3), trace=P.trace(slot, steps))


def assert_same(a, b, what):
    assert a["particle"] == b["particle"], what
    np.testing.assert_array_equal(a["bonds"], b["bonds"], err_msg=what)
    np.testing.assert_array_equal(a["f"], b["f"], err_msg=what)
    np.testing.assert_array_equal(a["trace"], b["trace"], err_msg=what)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_pool_members_match_standalone(L, prec):
    cases = mix(prec)
    P = L.Pool(W.PRECISION[prec])
    slots = []
    for w, n in cases:
        s = P.add(w, n)
        P.trace_enable(s, n)
        slots.append(s)
    say("pool", prec, "members", len(slots), "usage", P.usage())
    P.step(max(n for _, n in cases) + 5)  # members idle once they reach their own count
    done = P.poll()
    assert sorted(done) == sorted(slots)
    for (w, n), s in zip(cases, slots):
        assert P.status(s) == (n, L.POOL_FINISHED)
        ref = alone(L, w, n)
        got = pooled(P, s, n)
        say("member", w["name"], "steps", n, "bonds", int(got["bonds"].sum()), "x", got["particle"]["xc"])
        assert got["particle"]["step"] == n - 1
        assert_same(got, ref, w["name"])
    P.close()


@pytest.mark.parametrize("k", [0, 1])
def test_pool_member_against_oracle(L, orc, k):
    w, n = mix("fp64")[k]
    P = L.Pool(L.FP64)
    s = P.add(w, n)
    P.trace_enable(s, n)
    P.step(n)
    P.poll()
    tg = P.trace(s, n)
    o = orc.Sim.from_workload(w)
    _, to = o.step(n, trace=True)
    x0 = np.array([w["particle"]["xc"], w["particle"]["yc"]])

    def rel(a, b):
        return float(np.linalg.norm(a - b) / np.linalg.norm(b))

    eX = rel(tg[:, 1:3] - x0, to[:, 1:3] - x0)
    eU = rel(tg[:, 4:6], to[:, 4:6])
    eT = rel(tg[:, 3], to[:, 3])
    say("pool vs oracle: displacement", eX, "velocity", eU, "angle", eT)
    assert max(eX, eU, eT) < 1e-10
    np.testing.assert_array_equal(tg[:, -2], to[:, -2])  # bond counts
    np.testing.assert_array_equal(P.bonds(s)[0], o.bonds()[0])
    P.close()


def test_pool_join_and_leave_mid_run(L):
    cases = mix("fp32")
    P = L.Pool(L.FP32)
    s0 = P.add(cases[0][0], 60)
    s1 = P.add(cases[1][0], 60)
    P.step(10)
    s2 = P.add(cases[2][0], 25)  # joins at pool step 10
    P.trace_enable(s2, 25)
    P.step(7)
    P.remove(s1)  # leaves after 17 steps
    P.step(50)
    done = P.poll()
    assert sorted(done) == sorted([s0, s2])
    assert P.status(s0) == (60, L.POOL_FINISHED)
    assert P.status(s2) == (25, L.POOL_FINISHED)
    assert_same(pooled(P, s0, 0), dict(alone(L, cases[0][0], 60), trace=np.zeros((0, 20))), "s0")
    assert_same(pooled(P, s2, 25), alone(L, cases[2][0], 25), "s2")
    with pytest.raises(L.LbibError):
        P.status(s1)
    members, running, used = P.usage()
    assert members == 2 and running == 0 and used == P.footprint(cases[0][0]) + P.footprint(cases[2][0])
    P.close()


def test_pool_failed_member_is_frozen_and_others_continue(L):
    good, n = mix("fp64")[0]
    bad = member(64, 32, gap=1e-6, seed=0)  # touches the wall within a few tens of steps
    ref = L.Sim(bad)
    ref.set_overlap(0)
    fail_step = None
    for k in range(60):
        ref.step(1)
        try:
            ref.sync()
        except L.LbibError as e:
            assert e.status == L.E_NUMERIC and "wall" in str(e)
            fail_step = k + 1
            break
    assert fail_step is not None, "the stand-alone run did not touch the wall"
    ref.close()
    ref = L.Sim(bad)  # the records before the failing step (a failed handle refuses reads)
    ref.set_overlap(0)
    ref.trace_enable(60)
    ref.step(fail_step - 1)
    tref = ref.trace(60)
    ref.close()
    say("stand-alone contact after", fail_step, "steps")
    P = L.Pool(L.FP64)
    sg = P.add(good, n)
    sb = P.add(bad, 60)
    P.trace_enable(sb, 60)
    P.step(60)
    done = P.poll()
    assert sorted(done) == sorted([sg, sb])
    steps, state = P.status(sb)
    assert state == L.POOL_FAILED and steps == fail_step
    assert "wall" in P.last_error()
    tb = P.trace(sb, 60)
    assert tb.shape[0] == fail_step
    np.testing.assert_array_equal(tb[: fail_step - 1], tref)
    assert P.status(sg) == (n, L.POOL_FINISHED)
    assert_same(pooled(P, sg, 0), dict(alone(L, good, n), trace=np.zeros((0, 20))), "good member")
    P.close()


def test_pool_admission_by_budget(L):
    cases = mix("fp32")
    fp = [L.Pool.footprint(w) for w, _ in cases[:3]]
    P = L.Pool(L.FP32, budget_bytes=fp[0] + fp[1], max_members=8)
    a = P.add(cases[0][0], 5)
    b = P.add(cases[1][0], 5)
    with pytest.raises(L.LbibError) as ei:
        P.add(cases[2][0], 5)
    assert ei.value.status == L.E_FULL
    assert P.usage() == (2, 2, fp[0] + fp[1])
    P.step(5)
    assert sorted(P.poll()) == sorted([a, b])
    assert fp[2] <= fp[1]
    P.remove(b)
    c = P.add(cases[2][0], 5)
    P.step(5)
    assert P.poll() == [c]
    with pytest.raises(L.LbibError) as ei:
        P.add(W.with_precision(cases[0][0], "fp64"), 5)
    assert ei.value.status == L.E_INVALID
    P.close()


def test_pool_zero_steps_and_empty(L):
    P = L.Pool(L.FP32)
    P.step(3)  # empty pool: nothing to do
    assert P.poll() == []
    w, _ = mix("fp32")[0]
    s = P.add(w, 0)
    assert P.poll() == [s]
    assert P.status(s) == (0, L.POOL_FINISHED)
    assert P.particle(s)["step"] == -1
    P.step(4)
    assert P.status(s) == (0, L.POOL_FINISHED)
    P.close()


def test_pool_kernel_timing(L):
    P = L.Pool(L.FP32)
    for w, _ in mix("fp32"):
        P.add(w, 100)
    P.kernel_timing(True)
    P.step(10)
    ms0, n0 = P.kernel_time(0)
    ms1, n1 = P.kernel_time(1)
    say("pool timing: sweep", ms0, n0, "particle", ms1, n1)
    assert n0 == 10 and n1 == 10 and ms0 > 0 and ms1 > 0
    P.close()


@pytest.mark.parametrize("cfg", [(64, 1, 0), (128, 2, 0), (256, 8, 0), (64, 4, 8), (128, 4, 16)])
def test_pool_launch_shapes_and_graph_replay_are_bit_identical(L, cfg):
    """Every sweep launch shape, and steps replayed from a captured HIP graph (several
    replays with host reads and ordinary launches in between), give the stand-alone result."""
    cases = mix("fp32")
    P = L.Pool(L.FP32)
    P.set_config(*cfg)
    assert P.config() == cfg
    slots = [P.add(w, n) for w, n in cases]
    done = []
    for _ in range(3):
        P.step(16)
        done += P.poll()
        P.particle(slots[0])
    P.step(3)
    P.step(60)
    done += P.poll()
    assert sorted(done) == sorted(slots)
    for (w, n), s in zip(cases, slots):
        assert_same(pooled(P, s, 0), dict(alone(L, w, n), trace=np.zeros((0, 20))), f"{w['name']} {cfg}")
    P.close()


def test_pool_autotune(L):
    cases = mix("fp32")
    P = L.Pool(L.FP32)
    slots = [P.add(w, 1000) for w, _ in cases]
    us = P.autotune(5)
    cfg = P.config()
    say("autotune picked", cfg, f"{us:.1f} us/step")
    assert us > 0 and cfg[0] in (64, 128, 256) and cfg[1] in (1, 2, 4, 8) and cfg[2] in (0, 5)
    assert all(P.status(s)[0] < 1000 for s in slots)
    P.step(1000)
    assert sorted(P.poll()) == sorted(slots)
    w, _ = cases[2]
    assert_same(pooled(P, slots[2], 0), dict(alone(L, w, 1000), trace=np.zeros((0, 20))), "after autotune")
    P.close()


def test_pool_fp32_member_of_sweep_size_against_oracle(L, orc):
    """A member of the parameter sweep's largest grid (2048 x 256, aspect-ratio-3 ellipse of
    area 0.025 H^2 at a gap of 3e-3 H, ligand density 0.7, bond strength 2, Re 1), FP32,
    pooled beside two smaller members for 200 steps with the launch shape the autotuner
    would pick among: its particle series within 1e-5 of the FP64 oracle, bond counts and
    final flags bit-exact."""
    from _parity import col, trace_errors

    w = W.sweep_member(2048, 256, "ar3", (7, 10), 2, 1.0, 0, precision="fp32")
    others = [W.sweep_member(600, 130, "circle", (1, 2), 1, 0.1, 1, precision="fp32"),
              W.sweep_member(1111, 201, "ar2", (9, 10), 2, 0.01, 2, precision="fp32")]
    n = 200
    P = L.Pool(L.FP32)
    P.set_config(128, 2, 0)
    s = P.add(w, n)
    for o_ in others:
        P.add(o_, n)
    P.trace_enable(s, n)
    P.step(n)
    P.poll()
    tg = P.trace(s, n)
    o = orc.Sim.from_workload(w)
    _, to = o.step(n, trace=True)
    errs = trace_errors(tg, to, w["particle"])
    say("sweep-size member vs oracle:", " ".join(f"{k}={v:.2e}" for k, v in errs.items()),
        "bonds max", int(to[:, col("n_bonds")].max()))
    for k, v in errs.items():
        assert v <= 1e-5, (k, v)
    np.testing.assert_array_equal(tg[:, col("n_bonds")], to[:, col("n_bonds")])
    np.testing.assert_array_equal(P.bonds(s)[0], o.bonds()[0])
    assert to[:, col("n_bonds")].max() > 0
    P.close()
