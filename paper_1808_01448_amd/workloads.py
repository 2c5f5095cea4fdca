"""Seeded synthetic workloads of the LB-IB adhesion hot path.

This module only *describes inputs*: lattice sizes, particle placement and the paper's
parameter values as numbers, plus seeded random arrays.  It holds none of the method's
arithmetic, so the GPU library and the CPU oracle can both be fed from it without sharing
any computation.

Parameter groups follow Table 1 of Coclite et al. (arXiv 1808.01448): the bond spring
constant, the Hamaker constant and the thermal energy are given as the paper's
dimensionless groups (sigma H / (rho nu^2), H_k / (rho nu^2 H), k_B T / (rho nu^2 H)), the
critical bond length as y_cr / H and the equilibrium length as a fraction of y_cr
("Wall-particle interaction").  Each side converts them to lattice units itself.
"""
from __future__ import annotations

import copy
import math

import numpy as np

# Table 1, dimensionless column: sigma / (rho_ref nu_ref^2 / H) for the two bond strengths.
SIGMA_HAT = {1: 27.8, 2: 55.5}
# Table 1: H_k / (rho_ref nu_ref^2 H).
HAMAKER_HAT = 1.74e-8
# "Wall-particle interaction": y_cr = 6.8e-3 H, y_cr,eq = 0.5 y_cr.
Y_CR_HAT = 6.8e-3
Y_EQ_RATIO = 0.5
# Results section: k_f / k_r0 = 8.5e3.  The paper does not give k_f itself; k_f = 1 per
# time step is the reading taken.
K_F = 1.0
K_R0 = 1.0 / 8.5e3
# k_B T is not reported either.  Reading: the thermal energy that makes the rupture rate
# of a fully stretched soft bond (sigma label 1, extension y_eq) equal to k_f:
#   (sigma - sigma*) y_eq^2 / (2 kBT) = ln(k_f / k_r0)  with sigma* = sigma / 2.
KBT_HAT = SIGMA_HAT[1] * (Y_EQ_RATIO * Y_CR_HAT) ** 2 / (4.0 * math.log(K_F / K_R0))

PRECISION = {"fp64": 0, "fp32": 1, "fp16": 2, "bf16": 3, "fp16_neq": 4, "bf16_neq": 5}


def _ligand(rho_l: tuple[int, int], strength: int) -> dict:
    return dict(
        rho_l_num=rho_l[0], rho_l_den=rho_l[1], sigma_hat=SIGMA_HAT[strength], sigma_star_ratio=0.5,
        y_cr_hat=Y_CR_HAT, y_eq_ratio=Y_EQ_RATIO, k_f=K_F, k_r0=K_R0, kbt_hat=KBT_HAT,
        hamaker_hat=HAMAKER_HAT,
    )


def channel_small_fp64() -> dict:
    """256 x 64 channel, tau 0.8, Re 0.1, FP64; circle of diameter 16 with 64 markers whose
    centroid sits 12 lattice units above the bottom wall; ligand density 1/2, bond strength
    1, seed 0, 2000 steps."""
    return dict(
        name="channel_256x64_circle_fp64",
        lattice=dict(nx=256, ny=64, tau=0.8, re=0.1, drive=0, precision=PRECISION["fp64"], seed=0),
        particle=dict(shape=0, a_major=8.0, b_minor=8.0, xc=64.0, yc=12.0, theta0=0.0, rho_p=1.0,
                      n_markers=64),
        ligand=_ligand((1, 2), 1),
        receptor=dict(wall=0, density=1.0),
        steps=2000,
    )


def channel_small_binding(precision: str = "fp64") -> dict:
    """The 256 x 64 case with the circle lowered so its gap to the receptor wall is
    y_eq = 0.5 y_cr: bonds can form from the first step."""
    w = channel_small_fp64()
    w["name"] = "channel_256x64_circle_binding_" + precision
    w["lattice"]["precision"] = PRECISION[precision]
    y_cr = Y_CR_HAT * w["lattice"]["ny"]
    w["particle"]["yc"] = -0.5 + Y_EQ_RATIO * y_cr + w["particle"]["a_major"]
    return w


def channel_large_fp32() -> dict:
    """4096 x 1024 channel, tau 0.8, Re 1, FP32 (stored as f - w_q); ellipse of aspect ratio 3
    (major axis 48, minor 16) with 256 markers, major axis normal to the wall, initial gap
    3e-3 H; ligand density 7/10, bond strength 2, seed 0, 100k steps."""
    ny = 1024
    a, b = 24.0, 8.0
    return dict(
        name="channel_4096x1024_ellipse_ar3_fp32",
        lattice=dict(nx=4096, ny=ny, tau=0.8, re=1.0, drive=0, precision=PRECISION["fp32"], seed=0),
        particle=dict(shape=1, a_major=a, b_minor=b, xc=1024.0, yc=-0.5 + 3e-3 * ny + a, theta0=0.0,
                      rho_p=1.0, n_markers=256),
        ligand=_ligand((7, 10), 2),
        receptor=dict(wall=0, density=1.0),
        steps=100_000,
    )


def channel_beyond_cache_fp32() -> dict:
    """The 4096 x 1024 problem on an 8192 x 4096 channel (2.4 GB of FP32 populations, far
    beyond the 256 MB last-level cache): the ellipse scaled with H (semi-axes 96 and 32, 512
    markers), the same Re, gap, ligands and bonds."""
    w = scaled(channel_large_fp32(), 8192, 4096, name="channel_8192x4096_ellipse_ar3_fp32")
    w["particle"]["n_markers"] = 512
    w["particle"]["xc"] = 2048.0
    return w


def scaled(w: dict, nx: int, ny: int, *, name: str | None = None) -> dict:
    """The same particle problem on a different channel: the particle keeps its size relative
    to H and its gap relative to H (used for sizes between the two configurations above)."""
    w = copy.deepcopy(w)
    s = ny / w["lattice"]["ny"]
    gap = w["particle"]["yc"] + 0.5 - w["particle"]["a_major"]
    w["lattice"]["nx"], w["lattice"]["ny"] = nx, ny
    p = w["particle"]
    p["a_major"] *= s
    p["b_minor"] *= s
    p["xc"] = nx / 4.0
    p["yc"] = -0.5 + gap * s + p["a_major"]
    if name:
        w["name"] = name
    return w


def without_particle(w: dict) -> dict:
    w = copy.deepcopy(w)
    w.pop("particle", None)
    w.pop("ligand", None)
    w.pop("particles", None)
    w["name"] = w["name"] + "_no_particle"
    return w


def with_precision(w: dict, precision: str) -> dict:
    w = copy.deepcopy(w)
    w["lattice"]["precision"] = PRECISION[precision]
    return w


# ----------------------------------------------------------------------------------------
# Parameter sweeps of the results section (many small simulations)
# ----------------------------------------------------------------------------------------

SWEEP_SHAPES = ("circle", "ar2", "ar3")
SWEEP_RHO_L = ((3, 10), (1, 2), (7, 10), (9, 10))
SWEEP_STRENGTH = (1, 2)
SWEEP_RE = (0.01, 0.1, 1.0)
SWEEP_SEEDS = (0, 1, 2)


def _semi_axes(shape: str, H: float, area_frac: float = 0.025):
    """Semi-axes (a, b) of a particle of area area_frac H^2 (the results section keeps the
    particle area fixed while the aspect ratio varies)."""
    A = area_frac * H * H
    ar = {"circle": 1.0, "ar2": 2.0, "ar3": 3.0}[shape]
    a = math.sqrt(ar * A / math.pi)
    return a, a / ar


def _n_markers(shape: str, a: float, b: float) -> int:
    """Marker count for a spacing of about 0.785 lattice units (that of the 256 x 64 case),
    rounded up to a multiple of 64."""
    h = ((a - b) / (a + b)) ** 2
    perim = math.pi * (a + b) * (1 + 3 * h / (10 + math.sqrt(4 - 3 * h)))
    return 64 * math.ceil(perim / (0.785 * 64))


def sweep_member(nx: int, ny: int, shape: str, rho_l: tuple[int, int], strength: int, re: float, seed: int,
                 *, precision: str = "fp32", steps: int = 10_000, gap_frac: float = 3e-3) -> dict:
    """One simulation of a parameter sweep: tau 0.8, the particle (area 0.025 H^2, major axis
    normal to the wall) a gap of gap_frac H above the receptor wall at x = nx / 4."""
    H = float(ny)
    a, b = _semi_axes(shape, H)
    return dict(
        name=f"sweep_{nx}x{ny}_{shape}_rl{rho_l[0]}-{rho_l[1]}_s{strength}_re{re}_seed{seed}",
        lattice=dict(nx=nx, ny=ny, tau=0.8, re=re, drive=0, precision=PRECISION[precision], seed=seed),
        particle=dict(shape=0 if shape == "circle" else 1, a_major=a, b_minor=b, xc=nx / 4.0,
                      yc=-0.5 + gap_frac * H + a, theta0=0.0, rho_p=1.0, n_markers=_n_markers(shape, a, b)),
        ligand=_ligand(rho_l, strength),
        receptor=dict(wall=0, density=1.0),
        steps=steps,
    )


def shear_setup(shape: str = "circle", rho_l: tuple[int, int] = (1, 2), re: float = 0.1, *, strength: int = 1,
                H: int = 200, precision: str = "fp64", seed: int = 0, steps: int = 100_000,
                theta0: float = 0.0) -> dict:
    """The computational domain of the paper's adhesion study ("Modeling the adhesion
    dynamics" section): [0, 10 H] x [0, H] with H = 200 nodes, tau = 1 (nu = 1/6), a resting
    receptor wall at the bottom and a top wall moving at u_max = Re nu / H (drive 1, linear
    shear); the particle (area 0.025 H^2) at rest a gap y0 = 3e-3 H above the bottom wall,
    at x = 10 H / 4.  theta0 = 0 puts the major axis normal to the wall (the paper does not
    state the initial orientation of its ellipses)."""
    a, b = _semi_axes(shape, float(H))
    half_normal = a if abs(math.cos(theta0)) > 0.5 else b  # semi-axis along y at theta0 = 0 or pi/2
    nx = 10 * H
    return dict(
        name=f"shear_{nx}x{H}_{shape}_rl{rho_l[0]}-{rho_l[1]}_s{strength}_re{re}_seed{seed}",
        lattice=dict(nx=nx, ny=H, tau=1.0, re=re, drive=1, precision=PRECISION[precision], seed=seed),
        particle=dict(shape=0 if shape == "circle" else 1, a_major=a, b_minor=b, xc=nx / 4.0,
                      yc=-0.5 + 3e-3 * H + half_normal, theta0=theta0, rho_p=1.0,
                      n_markers=_n_markers(shape, a, b)),
        ligand=_ligand(rho_l, strength),
        receptor=dict(wall=0, density=1.0),
        steps=steps,
    )


def batched_sweep(seed: int = 0, *, precision: str = "fp32", steps: int = 10_000) -> list[dict]:
    """The 216-simulation sweep: shape {circle, AR2, AR3} x ligand density {0.3, 0.5, 0.7, 0.9}
    x bond strength {1, 2} x Re {0.01, 0.1, 1} x seed {0, 1, 2}; each grid drawn (in this
    order) with nx ~ U_int[512, 2048] and ny ~ U_int[128, 256] from a generator seeded
    with `seed`."""
    g = rng(seed)
    out = []
    for shape in SWEEP_SHAPES:
        for rl in SWEEP_RHO_L:
            for st in SWEEP_STRENGTH:
                for re in SWEEP_RE:
                    for sd in SWEEP_SEEDS:
                        nx = int(g.integers(512, 2049))
                        ny = int(g.integers(128, 257))
                        out.append(sweep_member(nx, ny, shape, rl, st, re, sd, precision=precision, steps=steps))
    return out


def serving_requests(n: int, seed: int = 0, *, steps_range=(5_000, 50_000), nx_range=(256, 4096),
                     ny_range=(64, 512), precision: str = "fp32") -> list[dict]:
    """n single-particle adhesion solves for the serving loop: nx and ny log-uniform over
    their ranges (independently, rounded), shape, ligand density, bond strength and Re
    uniform over the sweep's sets, the step count uniform over steps_range; request k uses
    seed k for its bond draws.  Each workload's "steps" is its step count."""
    g = rng(seed)
    out = []
    for k in range(n):
        nx = int(round(math.exp(g.uniform(math.log(nx_range[0]), math.log(nx_range[1])))))
        ny = int(round(math.exp(g.uniform(math.log(ny_range[0]), math.log(ny_range[1])))))
        shape = SWEEP_SHAPES[int(g.integers(len(SWEEP_SHAPES)))]
        rl = SWEEP_RHO_L[int(g.integers(len(SWEEP_RHO_L)))]
        st = SWEEP_STRENGTH[int(g.integers(len(SWEEP_STRENGTH)))]
        re = SWEEP_RE[int(g.integers(len(SWEEP_RE)))]
        steps = int(g.integers(steps_range[0], steps_range[1] + 1))
        w = sweep_member(nx, ny, shape, rl, st, re, k, precision=precision, steps=steps)
        w["name"] = f"request{k}_" + w["name"]
        out.append(w)
    return out


def _ellipse_points(a: float, b: float, xc: float, yc: float, th: float, n: int = 96) -> np.ndarray:
    """n points of the boundary of the ellipse (semi-axis a along the body y axis)."""
    t = np.linspace(0.0, 2.0 * np.pi, n, endpoint=False)
    bx, by = b * np.sin(t), -a * np.cos(t)
    c, s = np.cos(th), np.sin(th)
    return np.stack([xc + c * bx - s * by, yc + s * bx + c * by], axis=1)


def multi_particle_channel(nx: int = 2048, ny: int = 512, n: int = 32, seed: int = 0, *, precision: str = "fp32",
                           re: float = 0.1, area_frac: float = 0.025, gap: float = 4.0, steps: int = 5_000,
                           max_tries: int = 200_000) -> dict:
    """n particles in one channel: aspect ratio ~ U[1, 3] (1 is a circle), area area_frac H^2
    each, angle ~ U[0, pi), placed by rejection sampling so that every boundary keeps at least
    `gap` lattice units from the walls (y = -1/2, ny - 1/2) and from every other boundary
    (periodic in x); ligand density and bond strength per particle drawn from the sweep's
    sets; tau 0.8, seed `seed`."""
    g = rng(seed)
    H = float(ny)
    parts, boundaries = [], []
    tries = 0
    while len(parts) < n:
        tries += 1
        if tries > max_tries:
            raise ValueError("placement failed: too dense for the requested gap")
        ar = float(g.uniform(1.0, 3.0))
        a = math.sqrt(ar * area_frac * H * H / math.pi)
        b = a / ar
        th = float(g.uniform(0.0, math.pi))
        hs = math.sqrt(b * b * math.sin(th) ** 2 + a * a * math.cos(th) ** 2)
        xc = float(g.uniform(0.0, nx))
        yc = float(g.uniform(-0.5 + gap + hs, ny - 0.5 - gap - hs))
        pts = _ellipse_points(a, b, xc, yc, th)
        ok = True
        for q in boundaries:
            for shift in (-nx, 0.0, nx):
                d = np.min(np.hypot(pts[:, None, 0] - q[None, :, 0] - shift, pts[:, None, 1] - q[None, :, 1]))
                if d < gap + 1.0:  # the sampled boundaries are within ~1 lu of the curves
                    ok = False
                    break
            if not ok:
                break
        if not ok:
            continue
        boundaries.append(pts)
        shape = 0 if ar < 1.0 + 1e-9 else 1
        rl = SWEEP_RHO_L[int(g.integers(len(SWEEP_RHO_L)))]
        strength = SWEEP_STRENGTH[int(g.integers(len(SWEEP_STRENGTH)))]
        parts.append(dict(
            particle=dict(shape=shape, a_major=a, b_minor=b, xc=xc, yc=yc, theta0=th, rho_p=1.0,
                          n_markers=_n_markers("circle" if shape == 0 else "ar3", a, b)),
            ligand=_ligand(rl, strength)))
    return dict(
        name=f"multi_{nx}x{ny}_{n}particles_{precision}_seed{seed}",
        lattice=dict(nx=nx, ny=ny, tau=0.8, re=re, drive=0, precision=PRECISION[precision], seed=seed),
        particles=parts,
        receptor=dict(wall=0, density=1.0),
        steps=steps,
    )


def poisson_arrivals(n: int, rate: float, seed: int = 0) -> np.ndarray:
    """Arrival times (seconds from 0) of a Poisson process of the given rate."""
    return np.cumsum(rng(seed + 1_000_003).exponential(1.0 / rate, n))


# ----------------------------------------------------------------------------------------
# Seeded random arrays (for unit-level parity tests)
# ----------------------------------------------------------------------------------------

def rng(seed: int) -> np.random.Generator:
    return np.random.default_rng(seed)


def random_points(seed: int, n: int, nx: int, ny: int, *, y_lo: float = -0.45, y_hi: float | None = None):
    """n evaluation points spread over the channel, including the periodic seam and the
    rows next to both walls."""
    g = rng(seed)
    y_hi = ny - 0.55 if y_hi is None else y_hi
    x = g.uniform(-2.0, nx + 2.0, n)
    y = g.uniform(y_lo, y_hi, n)
    # force a share of the points onto the seam and next to the walls
    k = n // 8
    x[:k] = g.uniform(-1.5, 1.5, k)
    y[k:2 * k] = g.uniform(y_lo, 1.5, k)
    y[2 * k:3 * k] = g.uniform(ny - 2.5, y_hi, k)
    return np.stack([x, y], axis=1)


def random_perturbation(seed: int, shape, scale: float) -> np.ndarray:
    return rng(seed).uniform(-scale, scale, shape)


def random_u32(seed: int, shape) -> np.ndarray:
    return rng(seed).integers(0, 2**32, size=shape, dtype=np.uint64).astype(np.uint32)
