"""GPU tests of the two population-buffer layouts (push and pull streaming).

Streaming is a permutation of values, so the pull layout (buffers hold post-collision
values, each node gathers its inflow) must reproduce the push layout (buffers hold the
streamed values, each node scatters its outflow) bit for bit: fields, particle records,
bonds, through the overlapped schedule, checkpoints and population overwrites.  The push
layout is held to the FP64 oracle by test_gpu_sim.py; the pull layout is also compared with
the oracle directly here."""
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


def run(L, w, steps, layout, overlap=0):
    s = L.Sim(w, layout=layout)
    assert s.pull == (layout == 1)
    s.set_overlap(overlap)
    s.trace_enable(steps)
    s.step(steps)
    s.sync()
    out = dict(trace=s.trace(steps), f=s.f, bonds=s.bonds()[0], particle=s.particle())
    return s, out


def same(a, b, what):
    np.testing.assert_array_equal(a["trace"], b["trace"], err_msg=what)
    np.testing.assert_array_equal(a["f"], b["f"], err_msg=what)
    np.testing.assert_array_equal(a["bonds"], b["bonds"], err_msg=what)
    assert a["particle"] == b["particle"], what


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("overlap", [0, 1])
def test_pull_equals_push(L, prec, overlap):
    w = W.channel_small_binding(prec)
    sa, a = run(L, w, 300, 0, overlap)
    sb, b = run(L, w, 300, 1, overlap)
    say("layouts", prec, "overlap", overlap, "bonds", int(a["bonds"].sum()))
    same(a, b, f"{prec} overlap {overlap}")
    sa.close()
    sb.close()


def test_pull_ragged_lattice_and_seam(L):
    """Padded rows, partial tiles and a particle across the periodic seam."""
    w = W.channel_small_binding("fp64")
    w["lattice"].update(nx=100, ny=37)
    w["particle"].update(shape=1, a_major=7.0, b_minor=3.5, xc=1.2, yc=-0.5 + 0.15 + 7.0, theta0=0.4)
    sa, a = run(L, w, 200, 0)
    sb, b = run(L, w, 200, 1)
    same(a, b, "ragged")
    sa.close()
    sb.close()


def test_pull_against_oracle(L, orc):
    w = W.channel_small_binding("fp64")
    steps = 400
    s, g = run(L, w, steps, 1)
    o = orc.Sim.from_workload(w)
    _, to = o.step(steps, trace=True)
    x0 = np.array([w["particle"]["xc"], w["particle"]["yc"]])
    eX = np.linalg.norm(g["trace"][:, 1:3] - to[:, 1:3]) / np.linalg.norm(to[:, 1:3] - x0)
    eU = np.linalg.norm(g["trace"][:, 4:6] - to[:, 4:6]) / np.linalg.norm(to[:, 4:6])
    ef = np.linalg.norm(g["f"] - o.f) / np.linalg.norm(o.f - orc.lattice()[2][:, None, None])
    say(f"pull vs oracle: displacement {eX:.2e} velocity {eU:.2e} populations {ef:.2e}")
    assert max(eX, eU) < 1e-10
    # populations are compared by their deviation from the weights (~1e-5 here): the oracle
    # stores plain f ~ 0.4, whose FP64 rounding is ~5e-12 of that deviation per step, a random
    # walk of ~1e-10 after 400 steps; the GPU stores f - w and does not add it
    assert ef < 2e-9
    np.testing.assert_array_equal(g["trace"][:, -2], to[:, -2])
    s.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_pull_populations_roundtrip_and_overwrite(L, orc, prec):
    """write_populations / read-outs are layout-independent: the same plain populations
    written into both layouts read back identically and evolve identically."""
    w = W.with_precision(W.channel_small_binding(prec), prec)
    f0 = None
    out = []
    for layout in (0, 1):
        s = L.Sim(w, layout=layout)
        s.step(20)
        if f0 is None:
            f0 = s.f + W.random_perturbation(5, (9, w["lattice"]["ny"], w["lattice"]["nx"]), 1e-6)
        s.write_populations(f0)
        back = s.f
        s.step(30)
        out.append((back, s.f, s.particle()))
        s.close()
    np.testing.assert_array_equal(out[0][0], out[1][0])
    np.testing.assert_array_equal(out[0][1], out[1][1])
    assert out[0][2] == out[1][2]
    if prec == "fp64":
        np.testing.assert_allclose(out[0][0], f0, rtol=0, atol=1e-15)


def test_pull_checkpoint_resume(L):
    w = W.channel_small_binding("fp32")
    a = L.Sim(w, layout=1)
    a.step(120)
    blob = a.save()
    a.step(80)
    b = L.Sim(w, layout=1)
    b.load(blob)
    b.step(80)
    np.testing.assert_array_equal(a.f, b.f)
    assert a.particle() == b.particle()
    c = L.Sim(w, layout=0)
    with pytest.raises(L.LbibError) as ei:
        c.load(blob)  # a checkpoint loads only into the layout it was made in
    assert ei.value.status == L.E_INVALID
    for s in (a, b, c):
        s.close()


def test_full_size_layouts_agree(L):
    """The 4096 x 1024 FP32 workload in both layouts, overlapped schedule: 30 steps, particle
    trace bit-identical and sampled populations equal."""
    w = W.channel_large_fp32()
    sa, a = run_light(L, w, 30, 0)
    sb, b = run_light(L, w, 30, 1)
    np.testing.assert_array_equal(a["trace"], b["trace"])
    np.testing.assert_array_equal(a["u"], b["u"])
    sa.close()
    sb.close()


def run_light(L, w, steps, layout):
    s = L.Sim(w, layout=layout)
    s.set_overlap(1)
    s.trace_enable(steps)
    s.step(steps)
    s.sync()
    _, ux, uy = s.fields()
    return s, dict(trace=s.trace(steps), u=np.stack([ux[::7, ::5], uy[::7, ::5]]))


@pytest.mark.parametrize("layout", [0, 1])
@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp16", "bf16", "fp16_neq", "bf16_neq"])
def test_sweep_commutes_with_periodic_shift(L, prec, layout):
    """The lattice update is the same at every node, so stepping a state shifted by k columns
    (x is periodic) gives the shifted result bit for bit.  A random, x-dependent state on a
    100-column lattice with k = 37 moves every value across the sweep's wave and tile edges and
    the periodic seam: it holds the scalar-base addressing, the column wrap and, for the
    f - f_eq storages, the neighbour moments taken by wave shifts with their edge values from
    scalar loads, to the same arithmetic at every position."""
    w = W.without_particle(W.channel_small_binding(prec))
    w["lattice"].update(nx=100, ny=40)
    k, steps = 37, 30
    base = L.Sim(w, layout=layout)
    f0 = base.f + 1e-4 * W.random_perturbation(11, (9, 40, 100), 1.0)
    base.close()
    out = []
    for shift in (0, k):
        s = L.Sim(w, layout=layout)
        s.write_populations(np.roll(f0, shift, axis=2))
        s.step(steps)
        s.sync()
        out.append(s.f)
        s.close()
    say("shift", prec, "layout", layout, "largest change over the run", float(np.abs(out[0] - f0).max()))
    np.testing.assert_array_equal(out[1], np.roll(out[0], k, axis=2))


@pytest.mark.parametrize("layout", [0, 1])
@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp16", "bf16", "fp16_neq", "bf16_neq"])
def test_particle_across_the_seam_is_a_shifted_copy(L, prec, layout):
    """A particle moved by 80 columns (560 -> 640 on a 640-column lattice, where it straddles
    the periodic seam) gives the shifted run bit for bit: every x coordinate stays in the binade
    [512, 1024) in both runs, so no rounding changes (the FP64 oracle does the same, tested on
    the CPU).  It holds the particle phase's wrapped supports, node loads (for the f - f_eq
    storages the moments of the columns across the seam), spreads and probes, and the sweep's
    box at the seam, to the arithmetic of the interior, in the default schedule."""
    k, steps = 80, 40
    out = []
    for xc in (560.0, 560.0 + k):
        w = W.channel_small_binding(prec)
        w["lattice"]["nx"] = 640
        w["particle"]["xc"] = xc
        s = L.Sim(w, layout=layout)
        s.trace_enable(steps)
        s.step(steps)
        s.sync()
        out.append(dict(trace=s.trace(steps), f=s.f, bonds=s.bonds()[0]))
        s.close()
    a, b = out
    ix = L.STATE_FIELDS.index("xc")
    rest = [c for c in range(len(L.STATE_FIELDS)) if c != ix]
    say("seam shift", prec, "layout", layout, "bonds", int(a["bonds"].sum()), "final xc", a["trace"][-1, ix])
    np.testing.assert_array_equal(b["trace"][:, ix], a["trace"][:, ix] + k)
    np.testing.assert_array_equal(b["trace"][:, rest], a["trace"][:, rest])
    np.testing.assert_array_equal(b["f"], np.roll(a["f"], k, axis=2))
    np.testing.assert_array_equal(b["bonds"], a["bonds"])
