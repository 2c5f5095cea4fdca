"""Pins of the oracle's shear drive (drive 1): a resting bottom wall and a top wall moving
along x at u_max = Re nu / H with half-way bounce-back, no body force (the computational
domain of the "Modeling the adhesion dynamics" section, with its linear shear flow).

The pins are the exact linear steady state, the start-up transient against its Fourier
series (second-order convergence in H), and the reflection at a moving wall link by link."""
import math

import numpy as np
import pytest

from paper_1808_01448_amd import workloads as W


def couette(orc, H, tau, steps, init_rest, re=1.0, nx=4):
    w = W.without_particle(W.channel_small_fp64())
    w["lattice"].update(nx=nx, ny=H, tau=tau, re=re, drive=1)
    s = orc.Sim.from_workload(w, init_rest=init_rest)
    s.step(steps)
    rho, ux, uy = s.fields()
    return rho, ux, uy, s.derived


@pytest.mark.parametrize("tau", [0.6, 0.8, 1.0, 1.5])
def test_linear_shear_is_the_steady_state(orc, tau):
    """Started from the linear profile u = u_max (y + 1/2) / H, the flow stays on it to
    round-off: half-way bounce-back at a moving wall is exact for linear shear at any tau.
    No body force acts."""
    H = 16
    rho, ux, uy, d = couette(orc, H, tau, 1000, False)
    assert d["gx"] == 0.0 and d["gy"] == 0.0
    lin = d["umax"] * (np.arange(H) + 0.5) / H
    assert np.abs(ux - lin[:, None]).max() <= 5e-12 * d["umax"]
    assert np.abs(uy).max() <= 5e-12 * d["umax"]
    assert np.abs(rho - 1.0).max() <= 1e-13


def _startup_series(H, U, nu, t, y):
    """u(eta, t) = U eta / H + sum_n 2 U / (n pi) (-1)^n sin(n pi eta / H) exp(-nu (n pi / H)^2 t),
    eta = y + 1/2: the fluid at rest at t = 0 between a resting wall (eta = 0) and a wall
    moving at U (eta = H)."""
    eta = y + 0.5
    u = U * eta / H
    for n in range(1, 4000):
        u = u + 2 * U / (n * math.pi) * (-1) ** n * np.sin(n * math.pi * eta / H) * math.exp(
            -nu * (n * math.pi / H) ** 2 * t)
    return u


def test_startup_follows_the_series_with_second_order_error(orc):
    """From rest, the profile at t = 0.05 H^2 / nu matches the series solution of the
    diffusion equation to 1.5e-4 u_max at H = 64, and the error falls as 1/H^2."""
    tau = 0.8
    nu = (tau - 0.5) / 3
    errs = {}
    for H in (16, 32, 64):
        t = int(0.05 * H * H / nu)
        _, ux, uy, d = couette(orc, H, tau, t, True)
        us = _startup_series(H, d["umax"], nu, t, np.arange(H))
        errs[H] = np.abs(ux[:, 0] - us).max() / d["umax"]
        assert np.abs(uy).max() <= 1e-12 * d["umax"]
    assert errs[64] < 1.5e-4, errs
    r1, r2 = errs[16] / errs[32], errs[32] / errs[64]
    assert 3.8 < r1 < 4.2 and 3.8 < r2 < 4.2, errs


def test_moving_wall_reflection_link_by_link(orc):
    """A sweep with the top wall moving at uw differs from the resting-wall sweep only in the
    two diagonal populations the top row receives from the wall: f_7 (direction (-1, -1))
    by -2 w_5 e_5x uw / cs^2 = -uw / 6 and f_8 (direction (1, -1)) by +uw / 6."""
    rng = np.random.default_rng(7)
    nx, ny = 6, 5
    f = (np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)[:, None, None]
         * (1.0 + 0.01 * rng.standard_normal((9, ny, nx))))
    uw = 0.0123
    a = orc.collide_stream(f, 0.9, 1e-5, 0.0, uw=uw)
    b = orc.collide_stream(f, 0.9, 1e-5, 0.0, uw=0.0)
    d = a - b
    expect = np.zeros_like(d)
    expect[7, ny - 1, :] = -uw / 6
    expect[8, ny - 1, :] = uw / 6
    np.testing.assert_allclose(d, expect, rtol=0, atol=1e-17)
