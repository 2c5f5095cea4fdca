"""GPU tests of the shear drive (drive 1): a resting receptor wall, a top wall moving along x
at u_max = Re nu / H (moving-wall bounce-back) and no body force, as in the computational
domain of the paper's adhesion study.  The oracle's shear drive is pinned by
tests/test_oracle_couette.py; here the GPU path is held to it."""
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


def shear_small(prec="fp64", re=0.5):
    """The 256 x 64 binding case under the shear drive."""
    w = W.channel_small_binding(prec)
    w["lattice"].update(drive=1, re=re)
    return w


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("layout", [0, 1])
def test_linear_shear_is_steady_on_gpu(L, layout):
    """Without a particle the developed linear profile stays put (FP64, both layouts)."""
    w = W.without_particle(shear_small("fp64"))
    s = L.Sim(w, layout=layout)
    s.step(500)
    s.sync()
    rho, ux, uy = s.fields()
    H = w["lattice"]["ny"]
    umax = w["lattice"]["re"] * (w["lattice"]["tau"] - 0.5) / 3.0 / H
    lin = umax * (np.arange(H) + 0.5) / H
    say("layout", layout, "linear-profile error", np.abs(ux - lin[:, None]).max() / umax)
    assert np.abs(ux - lin[:, None]).max() <= 5e-12 * umax
    assert np.abs(uy).max() <= 5e-12 * umax
    assert np.abs(rho - 1.0).max() <= 1e-13
    s.close()


@pytest.mark.parametrize("layout", [0, 1])
def test_shear_with_particle_against_oracle(L, orc, layout):
    w = shear_small("fp64")
    steps = 400
    s = L.Sim(w, layout=layout)
    s.trace_enable(steps)
    s.step(steps)
    s.sync()
    tg = s.trace(steps)
    o = orc.Sim.from_workload(w)
    _, to = o.step(steps, trace=True)
    x0 = np.array([w["particle"]["xc"], w["particle"]["yc"]])
    eX = rel(tg[:, 1:3] - x0, to[:, 1:3] - x0)
    eU = rel(tg[:, 4:6], to[:, 4:6])
    eF = rel(tg[:, 7:9], to[:, 7:9])
    ef = np.linalg.norm(s.f - o.f) / np.linalg.norm(o.f - orc.lattice()[2][:, None, None])
    say(f"layout {layout}: displacement {eX:.2e} velocity {eU:.2e} force {eF:.2e} populations {ef:.2e}")
    assert max(eX, eU, eF) < 1e-10
    assert ef < 2e-9  # as for the Poiseuille drive: deviation from the weights, round-off walk
    np.testing.assert_array_equal(tg[:, -2], to[:, -2])
    np.testing.assert_array_equal(s.bonds()[0], o.bonds()[0])
    s.close()


def test_shear_layouts_and_schedules_agree(L):
    w = shear_small("fp32")
    out = []
    for layout, overlap in ((0, 0), (1, 0), (1, 1), (0, 3)):
        s = L.Sim(w, layout=layout)
        s.set_overlap(overlap)
        s.trace_enable(250)
        s.step(250)
        s.sync()
        out.append((s.trace(250), s.f))
        s.close()
    for t, f in out[1:]:
        np.testing.assert_array_equal(t, out[0][0])
        np.testing.assert_array_equal(f, out[0][1])


@pytest.mark.parametrize("prec", ["fp32", "fp16", "fp16_neq"])
def test_shear_storage_precisions_against_oracle(L, orc, prec):
    w0 = shear_small("fp64")
    steps = 800
    o = orc.Sim.from_workload(w0)
    _, to = o.step(steps, trace=True)
    s = L.Sim(W.with_precision(w0, prec))
    s.trace_enable(steps)
    s.step(steps)
    s.sync()
    tg = s.trace(steps)
    x0 = np.array([w0["particle"]["xc"], w0["particle"]["yc"]])
    eU, eX = rel(tg[:, 4:6], to[:, 4:6]), rel(tg[:, 1:3] - x0, to[:, 1:3] - x0)
    say(prec, f"velocity {eU:.2e} displacement {eX:.2e}")
    tol = {"fp32": 1e-5, "fp16": 5e-3, "fp16_neq": 8e-5}[prec]  # the storage bars of the Poiseuille drive
    assert eU <= tol and eX <= tol
    s.close()


def test_shear_populations_roundtrip(L):
    """Plain populations written into either layout read back to round-off (the top row's
    wall term is taken off on writing and added on reading) and evolve identically."""
    w = shear_small("fp64")
    out = []
    f0 = None
    for layout in (0, 1):
        s = L.Sim(w, layout=layout)
        s.step(10)
        if f0 is None:
            f0 = s.f + W.random_perturbation(9, (9, w["lattice"]["ny"], w["lattice"]["nx"]), 1e-6)
        s.write_populations(f0)
        back = s.f
        s.step(25)
        out.append((back, s.f, s.particle()))
        s.close()
    np.testing.assert_allclose(out[0][0], f0, rtol=0, atol=1e-16)
    np.testing.assert_array_equal(out[0][0], out[1][0])
    np.testing.assert_array_equal(out[0][1], out[1][1])
    assert out[0][2] == out[1][2]


def test_shear_pool_member_equals_standalone(L):
    w = shear_small("fp32")
    s = L.Sim(w)
    s.step(150)
    s.sync()
    ref = (s.particle(), s.f)
    s.close()
    P = L.Pool(L.FP32, budget_bytes=1 << 30)
    k = P.add(w, 150)
    P.add(W.channel_small_binding("fp32"), 150)  # a Poiseuille member beside it
    P.step(160)
    assert k in P.poll()
    assert P.particle(k) == ref[0]
    np.testing.assert_array_equal(P.field(k, 3), ref[1])
    P.close()


def test_shear_two_particles_against_oracle(L, orc):
    w = shear_small("fp64")
    lig = w.pop("ligand")
    base = w.pop("particle")
    w["particles"] = [dict(particle=base, ligand=lig),
                      dict(particle=dict(base, xc=base["xc"] + 60.0, yc=base["yc"] + 20.0), ligand=dict(lig))]
    steps = 300
    s = L.Sim(w)
    for k in range(2):
        s.trace_enable(steps, k)
    s.step(steps)
    s.sync()
    o = orc.Sim.from_workload(w)
    _, to = o.step_all(steps)
    for k in range(2):
        tg = s.trace(steps, k)
        eU = rel(tg[:, 4:6], to[:, k, 4:6])
        say("particle", k, f"velocity {eU:.2e}")
        assert eU < 1e-10
        np.testing.assert_array_equal(tg[:, -2], to[:, k, -2])
    s.close()


def test_adhesion_study_trends(L):
    """The paper's domain (H = 200, [0, 10 H], tau = 1, Re 0.1, y0 = 3e-3 H), 30k steps in one
    pool: the mean bond count grows with the ligand density (the trend of Tables 2-4), a flat
    AR3 ellipse binds more ligands than the circle of the same area, and the bound circle rolls
    clockwise with the shear (Omega < 0 here, counter-clockwise positive)."""
    from paper_1808_01448_amd import experiments as E

    res = E.adhesion_study(("circle", "ar3"), re=0.1, steps=30_000, precision="fp32", theta0=np.pi / 2,
                           chunk=10_000)
    for r in res:
        say(r["case"], f"bonds {r['bonds']:.2f} y_min/H {r['y_min_over_H']:.2e} Omega H/u {r['omega_H_over_umax']:.3f}")
        assert r["finished"]
    circ = [r for r in res if r["shape"] == "circle"]
    ell = [r for r in res if r["shape"] == "ellipse"]
    for group in (circ, ell):
        b = [r["bonds"] for r in sorted(group, key=lambda r: r["rho_l"])]
        assert all(x < y for x, y in zip(b, b[1:])), b
    for c, e in zip(sorted(circ, key=lambda r: r["rho_l"]), sorted(ell, key=lambda r: r["rho_l"])):
        assert e["bonds"] > c["bonds"]
    assert all(-0.5 < r["omega_H_over_umax"] < -0.05 for r in circ)
