"""Storage-precision study on the turbulent sphere-pack workload.

512^3 box holding 2 x 2 x 2 simple-cubic cells of 256^3, each with one sphere
of diameter 240 at its centre; TRT with Lambda = 6e-6 (Table 1, highest Re_p
range) and CLI walls, tau = 0.5005.  The pressure jump targets Re_p = 5812 via
the turbulent friction factor F = 0.026 (Sec. 4, eq. (frictionFactor):
F_K -> F, F_K = (dp/L) sqrt(K_D) / (rho U^2)) with K_D from a Stokes run of the
same solid fraction at 64^3 scaled by (256/64)^2.  The flow starts from a
seeded 1% random velocity perturbation of the target velocity.  Each storage
mode (FP32, FP16, BF16; MRT in FP32 as the second operator) runs the same
steps; the superficial U is sampled every `sample` steps and time-averaged
over the second half.

    python -m paper_1508_02960_amd.precision_study --out results.json
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

from . import inputs, lbm, observables

RE_P = 5812.0
FRICTION = 0.026
TAU = 0.5005
MAGIC = 6e-6


def stokes_permeability(cell: int, diameter: float, device=None) -> float:
    shape = (cell, cell, cell)
    d = lbm.Domain(shape, tau=0.8, magic=3 / 16, delta_rho=1e-6, collision="trt", wall="cli",
                   storage="fp32", spheres=inputs.centred_sphere(shape, diameter), device=device)
    d.run_to_residual(1e-7, 200000)
    K, _ = d.permeability()
    d.close()
    return K


def run(edge: int = 512, cells: int = 2, steps: int = 20000, sample: int = 100,
        modes=("trt-fp32", "trt-fp16", "trt-bf16", "mrt-fp32"), seed: int = 3, device=None,
        log=print):
    cell = edge // cells
    diameter = 240.0 * cell / 256.0
    # K_D of the unit cell from a Stokes run at 64^3 with the same d/L
    small = 64
    K_small = stokes_permeability(small, diameter * small / cell, device=device)
    K = K_small * (cell / small) ** 2
    nu = observables.viscosity(TAU)
    U_target = RE_P * nu / diameter
    delta_rho = 3.0 * edge * FRICTION * U_target ** 2 / np.sqrt(K)
    shape = (edge, edge, edge)
    spheres = inputs.simple_cubic_array(cells, cell, diameter)
    u0 = 0.01 * U_target * inputs.random_velocity(shape, 1.0, seed=seed)
    out = dict(edge=edge, cells=cells, diameter=diameter, tau=TAU, magic=MAGIC, K_D=K,
               K_small=K_small, U_target=U_target, delta_rho=delta_rho, steps=steps,
               sample=sample, runs={})
    log(f"[precision] K_D={K:.6g} U_target={U_target:.4g} delta_rho={delta_rho:.4g}")
    for mode in modes:
        coll, storage = mode.split("-")
        d = lbm.Domain(shape, tau=TAU, magic=MAGIC, delta_rho=delta_rho, collision=coll,
                       wall="cli", storage=storage, spheres=spheres, check_interval=sample,
                       device=device)
        d.init_equilibrium(u0=u0)
        series, status = [], "ok"
        t0 = time.perf_counter()
        for i in range(steps // sample):
            st, _, _ = d.run_to_residual(0.0, sample)
            if st == "unstable":
                status = f"unstable after {(i + 1) * sample} steps"
                break
            series.append(d.mean_velocity()[0][0])
            if (i + 1) % 20 == 0:
                log(f"[precision] {mode}: step {(i + 1) * sample}, U={series[-1]:.6g}")
        d.synchronize()
        secs = time.perf_counter() - t0
        half = len(series) // 2
        U_avg = float(np.mean(series[half:])) if series else float("nan")
        rec = dict(status=status, seconds=secs, series=series, U_avg_second_half=U_avg,
                   mflups=d.n_fluid * len(series) * sample / secs / 1e6,
                   re_p=observables.reynolds_p(U_avg, diameter, TAU),
                   K_app=observables.permeability(U_avg, delta_rho, edge, TAU))
        out["runs"][mode] = rec
        log(f"[precision] {mode}: {status}, U_avg={U_avg:.6g}, Re_p={rec['re_p']:.1f}, "
            f"{rec['mflups']:.0f} MFLUPS, {secs:.1f} s")
        d.close()
    ref = out["runs"].get("trt-fp32")
    if ref and np.isfinite(ref["U_avg_second_half"]):
        for mode, rec in out["runs"].items():
            rec["U_avg_rel_to_trt_fp32"] = rec["U_avg_second_half"] / ref["U_avg_second_half"] - 1
    return out


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--edge", type=int, default=512)
    ap.add_argument("--cells", type=int, default=2)
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--sample", type=int, default=100)
    ap.add_argument("--modes", default="trt-fp32,trt-fp16,trt-bf16,mrt-fp32")
    ap.add_argument("--out", default=None)
    a = ap.parse_args(argv)
    res = run(a.edge, a.cells, a.steps, a.sample, tuple(a.modes.split(",")),
              log=lambda s: print(s, flush=True))
    txt = json.dumps(res)
    if a.out:
        with open(a.out, "w") as f:
            f.write(txt)
    else:
        print(txt)
    return 0


if __name__ == "__main__":
    sys.exit(main())
