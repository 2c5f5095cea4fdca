"""GPU tests of the 16-bit population storages (FP16 with a power-of-two scale, BF16).

Populations are stored as f - w_q in IEEE binary16 (times 2^S) or bfloat16 and collided in
FP32; the particle phase stays FP64.  The error against the FP64 oracle is set by the
storage's unit roundoff u (2^-11 for FP16, 2^-8 for BF16): every stored deviation carries a
relative rounding of up to u/2 each step, and the flow's velocity (a sum of deviations)
inherits a few u.  Measured on the 256 x 64 cases: velocity 1.0-1.6e-3 (FP16) and 2.5e-2
(BF16), displacement 1.6-2.2e-4 and 1.7-3.8e-3, hydrodynamic force 7.8e-3 and 0.14 (a
derivative of the field), field 1.2e-3 and 1.1e-2.  The bars below are about 3x those.

The non-equilibrium storages (fp16_neq, bf16_neq) store f - f_eq of the emitting node's
stored moments in the same formats and collide in FP32, like the other 16-bit storages; the
stored values are ~10^-2 of f - w_q, so the storage rounding shrinks by that factor and the
FP32 arithmetic of the collision becomes visible: it rounds each post-collision deviation
(~1e-4 here) by up to 2^-24 of its size, so a node's momentum misses exact conservation by
~1e-11 per step and the flow drifts over the viscous time (the same drift an FP32 collision
gives FP32 storage).  Measured velocity 2.6e-5 / 4.1e-4, displacement 7.3e-6 / 8.0e-5,
force 2.9e-4 / 4.9e-3, field 6.4e-5 / 1.25e-4 (with an FP64 collision the field error was
2.6e-6 / 5.1e-5, at 1.3x the sweep time); bars again about 3x."""
import sys

import numpy as np
import pytest

from paper_1808_01448_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {  # velocity series, displacement series, force series, final velocity field
    "fp16": dict(U=5e-3, X=1e-3, F=3e-2, field=4e-3),
    "bf16": dict(U=8e-2, X=1.5e-2, F=0.4, field=4e-2),
    "fp16_neq": dict(U=8e-5, X=2.5e-5, F=1e-3, field=2e-4),
    "bf16_neq": dict(U=1.2e-3, X=2.5e-4, F=1.5e-2, field=4e-4),
}
ALL16 = ["fp16", "bf16", "fp16_neq", "bf16_neq"]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def L():
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    from paper_1808_01448_amd import lbib

    lbib.lib()
    return lbib


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("prec", ALL16)
def test_16bit_storage_against_oracle(L, orc, prec):
    w0 = W.channel_small_binding("fp64")
    steps = 1500
    o = orc.Sim.from_workload(w0)
    _, to = o.step(steps, trace=True)
    _, uxo, uyo = o.fields()
    w = W.with_precision(w0, prec)
    s = L.Sim(w)
    assert s.bytes_per_update == (60 if prec.endswith("neq") else 36)
    s.trace_enable(steps)
    s.step(steps)
    s.sync()
    tg = s.trace(steps)
    _, ux, uy = s.fields()
    x0 = np.array([w0["particle"]["xc"], w0["particle"]["yc"]])
    e = dict(U=rel(tg[:, 4:6], to[:, 4:6]), X=rel(tg[:, 1:3] - x0, to[:, 1:3] - x0), F=rel(tg[:, 7:9], to[:, 7:9]),
             field=rel(np.stack([ux, uy]), np.stack([uxo, uyo])))
    say(prec, " ".join(f"{k}={v:.2e}" for k, v in e.items()))
    for k, v in e.items():
        assert v <= TOL[prec][k], (prec, k, v)
    # bond counts: the decisions use FP64 distances, which move by ~1e-4 (FP16) to 1e-3 (BF16)
    # of the gap; a draw near its threshold may flip, so allow a handful of differing steps
    diff = np.abs(tg[:, -2] - to[:, -2])
    say("  bond-count steps differing:", int((diff > 0).sum()), "of", steps)
    assert (diff > 0).mean() <= 0.01 and diff.max() <= 2
    s.close()


@pytest.mark.parametrize("nx", [256, 200])
@pytest.mark.parametrize("prec", ALL16)
def test_16bit_layouts_and_schedules_agree(L, prec, nx):
    """Push, pull and the overlapped schedule give the same fields and records bit for bit;
    nx = 200 pads every row and leaves a partial tile at the end of it."""
    w = W.channel_small_binding(prec)
    w["lattice"]["nx"] = nx
    out = []
    for layout, overlap in ((0, 0), (1, 0), (1, 1)):
        s = L.Sim(w, layout=layout)
        s.set_overlap(overlap)
        s.trace_enable(300)
        s.step(300)
        s.sync()
        out.append((s.trace(300), s.f))
        s.close()
    for t, f in out[1:]:
        np.testing.assert_array_equal(t, out[0][0])
        np.testing.assert_array_equal(f, out[0][1])


def fp16_scale(w):
    """The FP16 storage scale of a lattice, by the rule lbib.h states."""
    lat = w["lattice"]
    nu = (lat["tau"] - 0.5) / 3.0
    u = max(4.0 * lat["re"] * nu / lat["ny"], 1e-6)
    d = (4.0 / 9.0) * (3.0 * u + 4.5 * u * u)
    return 2.0 ** min(40, max(0, int(np.floor(np.log2(8192.0 / d)))))


@pytest.mark.parametrize("nx", [256, 200])
@pytest.mark.parametrize("prec", ["fp16", "bf16"])
def test_16bit_population_roundtrip(L, prec, nx):
    """Written populations read back as the storage's rounding (to nearest even) of f - w,
    FP16 after its power-of-two scale, for deviations from 1e-9 to 1e-3; nx = 200 leaves
    padding after every population segment of a row."""
    w = W.channel_small_binding(prec)
    w["lattice"]["nx"] = nx
    s = L.Sim(w)
    f = s.f
    wq = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)[:, None, None]
    dev = W.random_perturbation(11, f.shape, 1.0) * np.logspace(-9, -3, f.shape[2])[None, None, :]
    s.write_populations(wq + dev)
    v = (wq + dev) - wq
    if prec == "fp16":
        sc = fp16_scale(w)
        h = (v.astype(np.float32) * np.float32(sc)).astype(np.float16)
        back = h.astype(np.float64) * (1.0 / sc)
    else:
        u = v.astype(np.float32).view(np.uint32).astype(np.uint64)
        back = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16 << 16).astype(np.uint32).view(np.float32).astype(np.float64)
    np.testing.assert_array_equal(s.f, wq + back)
    s.close()


@pytest.mark.parametrize("prec", ALL16)
def test_16bit_pool_member_equals_standalone(L, prec):
    w = W.channel_small_binding(prec)
    s = L.Sim(w)
    s.step(120)
    s.sync()
    ref = (s.particle(), s.f)
    s.close()
    P = L.Pool(W.PRECISION[prec], budget_bytes=1 << 30)
    k = P.add(w, 120)
    P.step(130)
    assert P.poll() == [k]
    assert P.particle(k) == ref[0]
    np.testing.assert_array_equal(P.field(k, 3), ref[1])
    P.close()


@pytest.mark.parametrize("nx", [256, 200])
@pytest.mark.parametrize("prec", ["fp16_neq", "bf16_neq"])
def test_neq_population_roundtrip(L, prec, nx):
    """Written populations read back to the storage's rounding of f - f_eq, the equilibrium of
    each emitting node's moments (rho - 1, u) computed from the written values: for random
    deviations from 1e-9 to 1e-3 of the weights the error stays below u/2 of the largest
    stored value (measured 9.3e-7 / 7.2e-6 absolute against deviations up to 1e-3).  With
    nx = 200 every population segment and moment row of a row carries padding, so the host's
    encoding and the kernels' must agree on the padded strides."""
    w = W.channel_small_binding(prec)
    w["lattice"]["nx"] = nx
    s = L.Sim(w)
    f = s.f
    wq = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)[:, None, None]
    dev = W.random_perturbation(11, f.shape, 1.0) * np.logspace(-9, -3, f.shape[2])[None, None, :]
    s.write_populations(wq + dev)
    back = s.f
    err = np.abs(back - (wq + dev)).max() / np.abs(dev).max()
    say(prec, f"round trip error {err:.2e} of the largest deviation")
    assert err <= {"fp16_neq": 2e-3, "bf16_neq": 1.6e-2}[prec]
    # the same values evolve identically through either layout
    outs = []
    for layout in (0, 1):
        t = L.Sim(w, layout=layout)
        t.write_populations(wq + dev)
        t.step(20)
        outs.append(t.f)
        t.close()
    np.testing.assert_array_equal(outs[0], outs[1])
    s.close()


@pytest.mark.parametrize("prec", ["fp16", "fp16_neq", "bf16_neq"])
def test_16bit_checkpoint_resume(L, prec):
    """A checkpoint carries the stored values (and the moment planes of the f - f_eq
    storages): resuming from it reproduces the uninterrupted run bit for bit."""
    w = W.channel_small_binding(prec)
    a = L.Sim(w)
    a.step(60)
    blob = a.save()
    a.step(90)
    b = L.Sim(w)
    b.load(blob)
    b.step(90)
    assert a.particle() == b.particle()
    np.testing.assert_array_equal(a.f, b.f)
    a.close()
    b.close()
