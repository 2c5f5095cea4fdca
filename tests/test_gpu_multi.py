"""GPU tests of simulations with several particles (the split particle phase).

Every particle spreads into its own fixed-point tile; the step's tile mask lists which
particles reach each 64 x 4 tile; probes read the spread force of every particle that
reaches them and the sweep adds every reaching particle's force, in particle order.  The
oracle runs the same step in plain FP64 (tests/test_oracle_multi.py pins it)."""
import copy
import sys

import numpy as np
import pytest

from paper_1808_01448_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {  # velocity, displacement, force, angular velocity series (relative)
    "fp64": dict(U=1e-10, X=1e-10, F=1e-10, omega=1e-10),
    "fp32": dict(U=1e-5, X=1e-5, F=1e-5, omega=1e-5),
    "fp16": dict(U=5e-3, X=1e-3, F=3e-2, omega=3e-2),  # the FP16 storage bars (test_gpu_precision)
    "fp16_neq": dict(U=8e-5, X=1e-5, F=1e-3, omega=1e-3),
}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def L():
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    from paper_1808_01448_amd import lbib

    lbib.lib()
    return lbib


def pair(prec="fp64", dx=64.0, dy=0.0, nx=128, ny=48, ligands=True):
    """Two ellipses 12 x 6 near the receptor wall, the second dx further and dy higher."""
    w = W.channel_small_binding(prec)
    w["lattice"].update(nx=nx, ny=ny)
    lig = w.pop("ligand")
    if not ligands:
        lig = dict(lig, rho_l_num=0, rho_l_den=1)
    y_eq = W.Y_EQ_RATIO * W.Y_CR_HAT * ny
    base = dict(shape=1, a_major=6.0, b_minor=3.0, xc=30.0, yc=-0.5 + y_eq + 6.0, theta0=0.0, rho_p=1.0,
                n_markers=48)
    w.pop("particle")
    w["particles"] = [dict(particle=base, ligand=lig),
                      dict(particle=dict(base, xc=30.0 + dx, yc=base["yc"] + dy, theta0=0.3), ligand=dict(lig))]
    return w


def gpu_run(L, w, steps, layout=2, overlap=2):
    s = L.Sim(w, layout=layout)
    s.set_overlap(overlap)
    n = len(w.get("particles", [0]))
    for k in range(n):
        s.trace_enable(steps, k)
    s.step(steps)
    s.sync()
    tr = [s.trace(steps, k) for k in range(n)]
    return s, tr


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def compare(tg, to, w, k, tol, label):
    x0 = np.array([w["particles"][k]["particle"]["xc"], w["particles"][k]["particle"]["yc"]])
    e = dict(U=rel(tg[:, 4:6], to[:, 4:6]), X=rel(tg[:, 1:3] - x0, to[:, 1:3] - x0),
             F=rel(tg[:, 7:9], to[:, 7:9]), omega=rel(tg[:, 6], to[:, 6]))
    say(label, f"particle {k}", " ".join(f"{a}={b:.2e}" for a, b in e.items()))
    for a, b in e.items():
        assert b <= tol[a], (label, k, a, b)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_split_phase_equals_fused_for_one_particle(L, prec):
    """Mode 3 (two particle launches, mask-driven sweep) on a single particle reproduces the
    fused single-particle step bit for bit."""
    w = W.channel_small_binding(prec)
    out = []
    for mode in (0, 3):
        s, tr = gpu_run(L, w, 300, overlap=mode)
        out.append((tr[0], s.f, s.bonds()[0]))
        s.close()
    np.testing.assert_array_equal(out[0][0], out[1][0])
    np.testing.assert_array_equal(out[0][1], out[1][1])
    np.testing.assert_array_equal(out[0][2], out[1][2])


@pytest.mark.parametrize("case", ["apart", "neighbours"])
def test_two_particles_against_oracle(L, orc, case):
    """Two ellipses with bonds: far apart, and close enough that each one's probe supports
    reach the other's spread force (the probes must see the total force)."""
    # neighbours: boundary gap ~3 lu, so each one's probe supports (2.7 lu out) reach the
    # other's spread supports (1.5 lu out)
    w = pair(dx=64.0) if case == "apart" else pair(dx=9.5, dy=1.0)
    steps = 600
    s, tg = gpu_run(L, w, steps)
    o = orc.Sim.from_workload(w)
    _, to = o.step_all(steps)
    for k in range(2):
        np.testing.assert_array_equal(tg[k][:, -2], to[:, k, -2])  # bond counts
        compare(tg[k], to[:, k, :], w, k, TOL["fp64"], case)
        np.testing.assert_array_equal(s.bonds(k)[0], o.bonds_k(k)[0])
    ef = np.linalg.norm(s.f - o.f) / np.linalg.norm(o.f - orc.lattice()[2][:, None, None])
    say(case, f"populations {ef:.2e}")
    assert ef < 2e-9  # relative to the deviation from the weights (see the layout tests)
    s.close()


@pytest.mark.parametrize("prec", ["fp32", "fp16", "fp16_neq"])
def test_eight_particles_against_oracle(L, orc, prec):
    w = W.multi_particle_channel(256, 96, 8, seed=1, precision=prec, area_frac=0.02, steps=300)
    steps = 300
    s, tg = gpu_run(L, w, steps)
    o = orc.Sim.from_workload(W.with_precision(w, "fp64"))
    _, to = o.step_all(steps)
    for k in range(8):
        compare(tg[k], to[:, k, :], w, k, TOL[prec], prec)
    s.close()


def test_multi_layouts_and_checkpoint(L):
    """Pull and push layouts agree bit for bit with several particles; a checkpoint restores
    every particle."""
    w = W.multi_particle_channel(256, 96, 6, seed=2, precision="fp32", area_frac=0.02)
    outs = []
    for layout in (0, 1):
        s, tr = gpu_run(L, w, 200, layout=layout)
        outs.append((tr, s.f))
        s.close()
    for k in range(6):
        np.testing.assert_array_equal(outs[0][0][k], outs[1][0][k])
    np.testing.assert_array_equal(outs[0][1], outs[1][1])
    a = L.Sim(w)
    a.step(80)
    blob = a.save()
    a.step(70)
    b = L.Sim(w)
    b.load(blob)
    b.step(70)
    for k in range(6):
        assert a.particle(k) == b.particle(k)
        np.testing.assert_array_equal(a.bonds(k)[0], b.bonds(k)[0])
    np.testing.assert_array_equal(a.f, b.f)
    a.close()
    b.close()


def test_multi_overlapped_schedule_identical(L):
    """Mode 1 (the chained schedule: the loads launch beside the sweep on a second stream,
    handing over through device counters) gives the results of the serial schedule bit for
    bit."""
    w = W.multi_particle_channel(256, 96, 6, seed=4, precision="fp32", area_frac=0.02)
    outs = []
    for mode in (0, 1):
        s, tr = gpu_run(L, w, 150, overlap=mode)
        s.step(7)  # a second call: the schedule joins its streams at the end of each call
        s.sync()
        outs.append(([s.particle(k) for k in range(6)], tr, s.f))
        s.close()
    assert outs[0][0] == outs[1][0]
    for k in range(6):
        np.testing.assert_array_equal(outs[0][1][k], outs[1][1][k])
    np.testing.assert_array_equal(outs[0][2], outs[1][2])


def test_sixty_four_particles_against_oracle(L, orc):
    """The most particles a lattice takes: 64 small ellipses on 2048 x 512 (every bit of the
    64-bit tile-mask words in use), FP32, 120 steps."""
    w = W.multi_particle_channel(2048, 512, 64, seed=5, precision="fp32", area_frac=0.004, steps=120)
    assert len(w["particles"]) == 64
    steps = 120
    s, tg = gpu_run(L, w, steps)
    o = orc.Sim.from_workload(W.with_precision(w, "fp64"))
    _, to = o.step_all(steps)
    for k in (0, 31, 62, 63):
        compare(tg[k], to[:, k, :], w, k, TOL["fp32"], "64 particles")
    s.close()


@pytest.mark.parametrize("prec", ["fp64", "fp16"])
def test_schedules_of_several_particles_agree(L, prec):
    """Several particles: the chained schedule (mode 1), the two launches in order on one
    stream (mode 3), the one launch whose workgroups claim the particles and meet before the
    loads (mode 4) and the same launch on a single workgroup (mode 5: it claims the first
    particle, finds the others unclaimed, spreads them itself and runs every particle's loads,
    the path a launch takes when its workgroups are not resident together) give the same
    particles, bonds and populations bit for bit, including neighbours whose probe supports
    reach each other's spread."""
    w = W.multi_particle_channel(256, 96, 8, seed=6, precision=prec, area_frac=0.03)
    outs = []
    for mode in (1, 3, 4, 5, 2):
        s, tr = gpu_run(L, w, 200, overlap=mode)
        outs.append(([s.particle(k) for k in range(8)], tr, s.f, [s.bonds(k)[0] for k in range(8)]))
        s.close()
    for o in outs[1:]:
        assert outs[0][0] == o[0]
        for k in range(8):
            np.testing.assert_array_equal(outs[0][1][k], o[1][k])
            np.testing.assert_array_equal(outs[0][3][k], o[3][k])
        np.testing.assert_array_equal(outs[0][2], o[2])


@pytest.mark.parametrize("mode", [1, 4])
def test_chained_simulations_interleaved_beside_other_work(L, mode):
    """Two simulations with several particles, each on its own stream in the chained schedule
    (mode 1) or the one-launch phase (mode 4), enqueued alternately in calls of different
    lengths while a third stream keeps the device busy with matrix products: each equals its
    serial run (mode 3) bit for bit.  Neither schedule needs its workgroups resident together,
    so other work only delays it."""
    wa = W.multi_particle_channel(512, 128, 6, seed=8, precision="fp32", area_frac=0.02)
    wb = W.multi_particle_channel(384, 96, 5, seed=9, precision="fp16", area_frac=0.02)
    calls = [(17, 5), (3, 40), (60, 1), (20, 25)]
    n_a, n_b = sum(c[0] for c in calls), sum(c[1] for c in calls)
    refs = []
    for w, n in ((wa, n_a), (wb, n_b)):
        s, tr = gpu_run(L, w, n, overlap=3)
        refs.append((tr, s.f, [s.bonds(k)[0] for k in range(len(w["particles"]))]))
        s.close()
    sa_, sb_, sx = torch.cuda.Stream(), torch.cuda.Stream(), torch.cuda.Stream()
    a, b = L.Sim(wa, stream=sa_), L.Sim(wb, stream=sb_)
    for sim, w, n in ((a, wa, n_a), (b, wb, n_b)):
        sim.set_overlap(mode)
        for k in range(len(w["particles"])):
            sim.trace_enable(n, k)
    x = torch.randn(6144, 6144, device="cuda")
    torch.cuda.synchronize()
    with torch.cuda.stream(sx):
        y = x
        for _ in range(4):
            y = torch.mm(y, x) * 1e-4
    for ka, kb in calls:
        a.step(ka)
        b.step(kb)
    a.sync()
    b.sync()
    torch.cuda.synchronize()
    for sim, w, n, ref in ((a, wa, n_a, refs[0]), (b, wb, n_b, refs[1])):
        np_ = len(w["particles"])
        for k in range(np_):
            np.testing.assert_array_equal(sim.trace(n, k), ref[0][k])
            np.testing.assert_array_equal(sim.bonds(k)[0], ref[2][k])
        np.testing.assert_array_equal(sim.f, ref[1])
    a.close()
    b.close()
    del y
