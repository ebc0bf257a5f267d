"""Pressure-drop sweep on one sphere cell (Darcy to Forchheimer regime).

Each run is driven to the residual tolerance with lbm_run_to_residual; the
measured (|grad P|, U) pairs are fitted with eq. (Forchheimer).  Runs go in
increasing pressure drop.  With ``scale_start`` a run starts from the previous
converged state multiplied by the ratio of the pressure drops: Stokes flow is
linear in the forcing, so in the Darcy regime this is already close to the new
steady state.
"""
from __future__ import annotations

import time

import numpy as np

from . import inputs, lbm, observables


def reynolds_targets(n: int = 8, lo: float = -4.0, hi: float = 1.0) -> np.ndarray:
    """Re_p log-spaced from 10^lo to 10^hi."""
    return 10.0 ** np.linspace(lo, hi, n)


def run_sweep(shape, diameter: float, *, tau: float = 0.8, magic: float = 3 / 16,
              wall: str = "cli", storage: str = "fp32", collision: str = "trt",
              re_targets=None, K_guess: float | None = None, tol: float = 1e-8,
              max_steps: int = 400000, check_interval: int = 100, scale_start: bool = True,
              device=None, log=None):
    """Run the sweep; returns a dict with per-run records and the fit."""
    re_targets = reynolds_targets() if re_targets is None else np.asarray(re_targets, float)
    nx = shape[2]
    d = lbm.Domain(shape, tau=tau, magic=magic, delta_rho=1e-8, collision=collision,
                   wall=wall, storage=storage, spheres=inputs.centred_sphere(shape, diameter),
                   check_interval=check_interval, device=device)
    K = K_guess
    runs = []
    prev_state, prev_drho = None, None
    for i, re in enumerate(re_targets):
        if K is None:
            # first run: a Darcy estimate from a low-Re probe run
            d.set_delta_rho(1e-8)
            d.init_equilibrium()
            d.run_to_residual(1e-6, max_steps)
            K, _ = d.permeability()
        drho = observables.delta_rho_for_reynolds(re, diameter, tau, nx, K)
        d.set_delta_rho(drho)
        if scale_start and prev_state is not None:
            d.set_state(prev_state * (drho / prev_drho))
        else:
            d.init_equilibrium()
        t0 = time.perf_counter()
        status, steps, res = d.run_to_residual(tol, max_steps)
        secs = time.perf_counter() - t0
        Kapp, U = d.permeability()
        rec = dict(re_target=float(re), delta_rho=drho, status=status, steps=steps, residual=res,
                   seconds=secs, U=U, K_app=Kapp,
                   re_p=observables.reynolds_p(U, diameter, tau),
                   grad_p=observables.pressure_gradient(drho, nx))
        runs.append(rec)
        if log:
            log(rec)
        if i == 0 and K_guess is None:
            K = Kapp
        prev_state, prev_drho = d.get_state(), drho
    d.close()
    g = np.array([r["grad_p"] for r in runs])
    U = np.array([r["U"] for r in runs])
    K_D, beta, C_F = observables.forchheimer_fit(g, U, tau)
    return dict(runs=runs, K_D=K_D, beta=beta, C_F=C_F)


def report(res: dict, shape, diameter: float, tau: float) -> str:
    """Markdown table of a sweep and its Forchheimer fit."""
    nx = shape[2]
    L = nx
    r = diameter / 2.0
    lines = [
        f"| Re_p target | delta_rho | status | steps | U | K_app | Re_p | F_K | Re_K |",
        "|---|---|---|---|---|---|---|---|---|",
    ]
    for x in res["runs"]:
        fk, rek = observables.friction_factor(x["grad_p"], x["U"], res["K_D"], tau)
        lines.append(f"| {x['re_target']:.3g} | {x['delta_rho']:.4g} | {x['status']} | "
                     f"{x['steps']} | {x['U']:.5e} | {x['K_app']:.5f} | {x['re_p']:.4g} | "
                     f"{fk:.4g} | {rek:.4g} |")
    lines += ["", f"Fit of |grad P| / U = nu / K_D + beta U over the {len(res['runs'])} runs: "
              f"K_D = {res['K_D']:.5f} lattice units^2, beta = {res['beta']:.5g}, "
              f"C_F = beta sqrt(K_D) = {res['C_F']:.5g}.  Drag coefficient of the Darcy "
              f"limit, C_D = L^3 / (6 pi r K_D) = {L ** 3 / (6 * np.pi * r * res['K_D']):.4f} "
              f"(d/L = {diameter / L:.4g})."]
    return "\n".join(lines) + "\n"


def main(argv=None) -> int:
    import argparse
    import json
    import sys

    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--edge", type=int, default=128)
    ap.add_argument("--diameter", type=float, default=100.0)
    ap.add_argument("--tau", type=float, default=0.8)
    ap.add_argument("--storage", default="fp32")
    ap.add_argument("--wall", default="cli")
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--rest-starts", action="store_true",
                    help="start every run from rest instead of the scaled previous state")
    ap.add_argument("--out", required=True, help="JSON output")
    ap.add_argument("--md", help="markdown table")
    a = ap.parse_args(argv)
    shape = (a.edge,) * 3

    def log(rec):
        print(f"[sweep] Re_p target {rec['re_target']:.3g}: {rec['status']} after "
              f"{rec['steps']} steps ({rec['seconds']:.1f} s), K_app {rec['K_app']:.5f}, "
              f"Re_p {rec['re_p']:.4g}", file=sys.stderr, flush=True)

    res = run_sweep(shape, a.diameter, tau=a.tau, storage=a.storage, wall=a.wall, tol=a.tol,
                    scale_start=not a.rest_starts, log=log)
    with open(a.out, "w") as fh:
        json.dump(dict(res, shape=shape, diameter=a.diameter, tau=a.tau, storage=a.storage,
                       wall=a.wall, tol=a.tol), fh, indent=1)
    if a.md:
        with open(a.md, "w") as fh:
            fh.write(report(res, shape, a.diameter, a.tau))
    print(f"K_D {res['K_D']:.6f} beta {res['beta']:.6g} C_F {res['C_F']:.6g}", flush=True)
    return 0


if __name__ == "__main__":
    import sys

    sys.exit(main())
