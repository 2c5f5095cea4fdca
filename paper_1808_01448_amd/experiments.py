"""The paper's adhesion study on the GPU: particles released near the receptor wall of the
linear shear flow of its computational domain ("Modeling the adhesion dynamics of near-wall
circulating particles" and the results sections; workloads.shear_setup).  Every case runs as a
member of one pool; the per-step particle records give the quantities the paper tabulates:

  bonds       mean number of closed bonds over the second half of the run, also as a fraction
              of the ligands (the "percentage of active ligands") and of all markers;
  y_min       the smallest gap to the receptor wall over the second half, over H;
  omega       the mean angular velocity over the second half, as Omega H / u_max;
  ux          the mean translational velocity over the second half, over u_max.

The paper's Tables 2-4 are qualitative targets only: the constants it leaves out (k_f, k_B T)
are readings (workloads module), so no number is expected to match.

Usage: python -m paper_1808_01448_amd.experiments --steps 200000 --re 0.1 --shapes circle
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np

from . import lbib
from . import workloads as W

RHO_L = ((3, 10), (1, 2), (7, 10), (9, 10))


def adhesion_study(shapes=("circle",), rho_ls=RHO_L, re: float = 0.1, *, steps: int = 200_000, strength: int = 1,
                   precision: str = "fp64", seed: int = 0, H: int = 200, theta0: float = 0.0, chunk: int = 20_000,
                   k_f: float | None = None, log=None) -> list[dict]:
    """k_f: the bond formation rate per step (the paper gives only k_f / k_r0 = 8.5e3, which
    is kept; None takes the workloads reading)."""
    cases = [W.shear_setup(shape, rl, re, strength=strength, H=H, precision=precision, seed=seed, steps=steps,
                           theta0=theta0)
             for shape in shapes for rl in rho_ls]
    if k_f is not None:
        for w in cases:
            aff = w["ligand"]["k_f"] / w["ligand"]["k_r0"]
            w["ligand"]["k_f"], w["ligand"]["k_r0"] = k_f, k_f / aff
            w["name"] += f"_kf{k_f:g}"
    budget = sum(lbib.Pool.footprint(w) for w in cases) + (256 << 20)
    out = []
    with lbib.Pool(W.PRECISION[precision], budget_bytes=budget) as P:
        slots = []
        for w in cases:
            k = P.add(w, steps)
            P.trace_enable(k, steps)
            slots.append(k)
        t0 = time.perf_counter()
        done = 0
        while done < steps:
            n = min(chunk, steps - done)
            P.step(n)
            done += n
            P.poll()
            if log:
                log(f"adhesion study: {done}/{steps} steps, {time.perf_counter() - t0:.1f} s")
        wall = time.perf_counter() - t0
        for w, k in zip(cases, slots):
            st, state = P.status(k)
            tr = P.trace(k, steps)
            out.append(summarize(w, tr, state))
        for r in out:
            r["wall_seconds_all_cases"] = round(wall, 2)
    return out


def summarize(w: dict, tr: np.ndarray, state: int) -> dict:
    col = {n: c for c, n in enumerate(lbib.STATE_FIELDS)}
    lat, part, lig = w["lattice"], w["particle"], w["ligand"]
    H = float(lat["ny"])
    nu = (lat["tau"] - 0.5) / 3.0
    umax = lat["re"] * nu / H
    nl = part["n_markers"]
    n_lig = math.floor(nl * lig["rho_l_num"] / lig["rho_l_den"])
    half = tr[len(tr) // 2:]
    bonds = float(half[:, col["n_bonds"]].mean()) if len(half) else float("nan")
    return dict(
        case=w["name"], shape={0: "circle"}.get(part["shape"], "ellipse"),
        aspect=round(part["a_major"] / part["b_minor"], 3), rho_l=lig["rho_l_num"] / lig["rho_l_den"],
        re=lat["re"], k_f=lig["k_f"], steps_run=int(len(tr)), finished=state == lbib.POOL_FINISHED,
        n_markers=nl, n_ligands=n_lig, bonds=bonds, active_ligand_fraction=bonds / n_lig if n_lig else 0.0,
        bonds_per_marker=bonds / nl, max_bonds=int(tr[:, col["n_bonds"]].max()) if len(tr) else 0,
        y_min_over_H=float(half[:, col["gap"]].min() / H) if len(half) else float("nan"),
        gap_end_over_H=float(tr[-1, col["gap"]] / H) if len(tr) else float("nan"),
        omega_H_over_umax=float(half[:, col["omega"]].mean() * H / umax) if len(half) else float("nan"),
        ux_over_umax=float(half[:, col["ux"]].mean() / umax) if len(half) else float("nan"),
    )


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--steps", type=int, default=200_000)
    ap.add_argument("--re", type=float, default=0.1)
    ap.add_argument("--shapes", nargs="+", default=["circle"], choices=["circle", "ar2", "ar3"])
    ap.add_argument("--strength", type=int, default=1, choices=[1, 2])
    ap.add_argument("--precision", default="fp64", choices=list(W.PRECISION))
    ap.add_argument("--theta0", type=float, default=0.0)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--k-f", type=float, default=None, help="bond formation rate per step (affinity kept)")
    args = ap.parse_args(argv)
    res = adhesion_study(tuple(args.shapes), re=args.re, steps=args.steps, strength=args.strength,
                         precision=args.precision, seed=args.seed, theta0=args.theta0, k_f=args.k_f,
                         log=lambda m: print(m, file=sys.stderr, flush=True))
    for r in res:
        print(json.dumps(r), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
