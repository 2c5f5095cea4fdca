"""Pins of the oracle's multi-particle step: particles meet only through the fluid, their
spread forces add up, and the step is invariant under translation and relabelling.

Every case uses particles without ligands (ligand density 0), so the bond draws -- keyed by
the particle's index -- play no part and relabelling must not change anything."""
import copy

import numpy as np
import pytest

from paper_1808_01448_amd import workloads as W


def two_particles(nx=128, ny=48, x0=32.0, dx=64.0, dy=0.0, shape=1, theta1=0.0):
    w = W.channel_small_binding("fp64")
    w["lattice"].update(nx=nx, ny=ny)
    lig = dict(w["ligand"], rho_l_num=0, rho_l_den=1)
    base = dict(shape=shape, a_major=6.0, b_minor=3.0 if shape == 1 else 6.0, xc=x0, yc=14.0, theta0=0.0,
                rho_p=1.0, n_markers=48)
    p1 = dict(base, xc=x0 + dx, yc=14.0 + dy, theta0=theta1)
    w.pop("particle")
    w.pop("ligand")
    w["particles"] = [dict(particle=base, ligand=lig), dict(particle=p1, ligand=lig)]
    return w


def only(w, k):
    v = copy.deepcopy(w)
    v["particles"] = [v["particles"][k]]
    return v


def test_spread_of_separate_particles_adds_exactly(orc):
    """Disjoint supports: the first step's spread field of two particles is the sum of the
    fields each makes alone (the node fields they interpolate are the same initial state)."""
    w = two_particles()
    both = orc.Sim.from_workload(w)
    both.step_all(1)
    f0 = orc.Sim.from_workload(only(w, 0))
    f0.step_all(1)
    f1 = orc.Sim.from_workload(only(w, 1))
    f1.step_all(1)
    np.testing.assert_array_equal(both.fib, f0.fib + f1.fib)
    assert np.abs(f0.fib).max() > 0 and np.abs(f1.fib).max() > 0


def test_fluid_momentum_balance_with_two_particles(orc):
    """Fully periodic box (no walls) with two particles whose supports interact: each step the
    fluid gains N g plus the total spread force of both, to round-off."""
    w = two_particles(nx=64, ny=40, x0=20.0, dx=14.0, dy=2.0)
    w["lattice"]["re"] = 0.0
    g = 2e-6
    o = orc.Sim.from_workload(w, walls=False, init_rest=True, extra_g=(g, 0.0))
    ex, ey, _, _ = orc.lattice()
    N = 64 * 40
    for _ in range(30):
        f0 = o.f
        p0 = np.array([(f0 * ex[:, None, None]).sum(), (f0 * ey[:, None, None]).sum()])
        o.step_all(1)
        f1 = o.f
        p1 = np.array([(f1 * ex[:, None, None]).sum(), (f1 * ey[:, None, None]).sum()])
        fib = o.fib.reshape(2, -1).sum(axis=1)
        # round-off of summing 9 N populations of size ~0.1: ~1e-13 absolute
        np.testing.assert_allclose(p1 - p0, np.array([N * g, 0.0]) + fib, rtol=1e-9, atol=1e-12)


def test_translation_symmetry(orc):
    """Two identical particles half a period apart in a periodic channel move identically:
    the flow is invariant under a shift by nx/2."""
    w = two_particles(nx=128, x0=30.0, dx=64.0)
    o = orc.Sim.from_workload(w)
    _, tr = o.step_all(200)
    a, b = tr[:, 0, :], tr[:, 1, :]
    np.testing.assert_allclose(b[:, 1] - a[:, 1], 64.0, rtol=0, atol=1e-10)
    # positions agree to their round-off (a few ulp of ~14 per step); the rest relative to
    # the norm of each vector (the wall-normal components are ~1e-4 of the axial ones)
    np.testing.assert_allclose(b[:, 2], a[:, 2], rtol=0, atol=1e-12)
    for cols in ((3,), (4, 5), (6,), (7, 8), (9,)):
        c = list(cols)
        err = np.linalg.norm(b[:, c] - a[:, c]) / np.linalg.norm(a[:, c])
        assert err <= 1e-9, (cols, err)


def seam_shift_workload(xc: float) -> dict:
    """The 256 x 64 binding case on a 640-column lattice with the circle at xc."""
    w = W.channel_small_binding("fp64")
    w["lattice"]["nx"] = 640
    w["particle"]["xc"] = xc
    return w


def test_shift_across_the_seam_is_exact(orc):
    """Moving the particle by a whole number of columns moves the solution with it, bit for bit,
    as long as every x coordinate stays in one binade in both runs (here [512, 1024): markers,
    probes, and the second-order update's intermediates), so that no rounding changes.  The
    circle at xc = 640 straddles the periodic seam of the 640-column lattice; at 560 it does
    not: the seam's wrapped supports, spreads and probes must act exactly like interior ones.
    Bonds form (their draws are keyed by step, element and particle, not position)."""
    k, steps = 80, 40
    runs = []
    for xc in (560.0, 560.0 + k):
        o = orc.Sim.from_workload(seam_shift_workload(xc))
        flags, tr = o.step_all(steps)
        assert flags == 0
        runs.append((tr[:, 0, :], o.f, o.bonds_k(0)[0]))
        o.close()
    (ta, fa, ba), (tb, fb, bb) = runs
    np.testing.assert_array_equal(tb[:, 1], ta[:, 1] + k)
    rest = [c for c in range(ta.shape[1]) if c != 1]
    np.testing.assert_array_equal(tb[:, rest], ta[:, rest])
    np.testing.assert_array_equal(fb, np.roll(fa, k, axis=2))
    np.testing.assert_array_equal(bb, ba)
    assert ba.sum() > 0


def test_relabelling_permutes_trajectories(orc):
    """Listing the same two particles in the other order gives the same motions, swapped."""
    w = two_particles(nx=160, x0=30.0, dx=80.0, shape=1, theta1=0.4)
    v = copy.deepcopy(w)
    v["particles"] = v["particles"][::-1]
    _, ta = orc.Sim.from_workload(w).step_all(150)
    _, tb = orc.Sim.from_workload(v).step_all(150)
    np.testing.assert_array_equal(ta[:, 0, 1:], tb[:, 1, 1:])
    np.testing.assert_array_equal(ta[:, 1, 1:], tb[:, 0, 1:])


def test_neighbours_interact_through_the_fluid(orc):
    """A particle's motion changes when another moves nearby (they share the fluid), and the
    change shrinks as the neighbour moves away."""
    alone = orc.Sim.from_workload(only(two_particles(nx=256), 0))
    _, t0 = alone.step_all(200)
    diffs = []
    for dx in (16.0, 40.0):
        o = orc.Sim.from_workload(two_particles(nx=256, dx=dx))
        _, t = o.step_all(200)
        diffs.append(np.abs(t[:, 0, 4] - t0[:, 0, 4]).max() / np.abs(t0[:, 0, 4]).max())
    assert diffs[0] > 1e-3 and diffs[1] < diffs[0]
