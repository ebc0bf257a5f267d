"""Batch of independent sphere cells run to a residual in one device loop.

256 periodic 64^3 cells, each with one sphere (diameter U[40, 60], random
offset), tau U[0.55, 1], Re_p log-uniform in [1e-3, 300]; draws whose target
velocity Re_p nu / D exceeds 0.1 (Mach ~ 0.17) are redrawn.  The pressure
jump of each cell comes from a Darcy estimate with that cell's permeability,
taken from a first low-Re batch run (Stokes flow is linear in the forcing);
the main run goes to a 1e-8 relative velocity residual with a per-cell step
cap, after the launch shape is autotuned.

    python -m paper_1508_02960_amd.batch_study --out batch.json
    python -m paper_1508_02960_amd.batch_study --speed 100   # step timing only
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

from . import inputs, lbm, observables

U_MAX = 0.1


def draw_cells(n: int, seed: int, edge: int):
    cells, rejected = [], 0
    for dr in inputs.batch_cell_draws(seed, edge):
        if len(cells) == n:
            break
        nu = observables.viscosity(dr["tau"])
        if dr["re_p"] * nu / dr["diameter"] > U_MAX:
            rejected += 1
            continue
        c = dr["centre"]
        cells.append(dict(spheres=[[c[0], c[1], c[2], dr["diameter"] / 2]], tau=dr["tau"],
                          magic=3 / 16, re_target=dr["re_p"], diameter=dr["diameter"]))
    return cells, rejected


def run(n_cells=256, edge=64, seed=4, tol=1e-8, max_steps=200000, check_interval=100,
        stokes_tol=1e-6, log=print, device=None):
    shape = (edge, edge, edge)
    cells, rejected = draw_cells(n_cells, seed, edge)
    log(f"[batch] {n_cells} cells, {rejected} draws rejected for U > {U_MAX}")
    # 1) permeability of every cell from a Stokes run (tiny forcing)
    stokes = [dict(c, delta_rho=1e-7) for c in cells]
    t0 = time.perf_counter()
    b = lbm.Batch(shape, stokes, wall="cli", storage="fp32", check_interval=check_interval,
                  device=device)
    log(f"[batch] geometry + bind {time.perf_counter() - t0:.1f} s, "
        f"{b.info.n_fluid} fluid cells")
    by, zp, ms = b.autotune(steps=10)
    sw = b.solid_writes
    log(f"[batch] autotuned shape: wavefronts/block {by}, z planes/block {zp}, solid writes {sw}, "
        f"{ms:.3f} ms/step")
    t1 = time.perf_counter()
    b.run_to_residual(stokes_tol, max_steps)
    r0 = b.results()
    t_stokes = time.perf_counter() - t1
    b.close()
    K = r0["K_D"]
    log(f"[batch] Stokes pass {t_stokes:.1f} s, K_D median {np.median(K):.4g}")
    # 2) the target pressure jumps (Darcy estimate) and the main run
    for c, k in zip(cells, K):
        c["delta_rho"] = observables.delta_rho_for_reynolds(c["re_target"], c["diameter"],
                                                            c["tau"], edge, k)
    b = lbm.Batch(shape, cells, wall="cli", storage="fp32", check_interval=check_interval,
                  device=device)
    b.set_shape(by, zp)
    b.set_solid_writes(sw)
    t2 = time.perf_counter()
    st, steps, _ = b.run_to_residual(tol, max_steps)
    secs = time.perf_counter() - t2
    r = b.results()
    fluid = (b.mask() == 0).reshape(n_cells, -1).sum(axis=1)
    b.close()
    updates = float(np.sum(fluid * r["steps"]))
    re = [observables.reynolds_p(u[0], c["diameter"], c["tau"]) for u, c in zip(r["U"], cells)]
    out = dict(n_cells=n_cells, edge=edge, seed=seed, rejected=rejected, tol=tol,
               max_steps=max_steps, shape=dict(waves_per_block=by, z_planes_per_block=zp,
                                               solid_writes=sw, ms_per_step_all_cells=ms),
               stokes_seconds=t_stokes, seconds=secs, status=st,
               mflups=updates / secs / 1e6,
               counts={s: r["status"].count(s) for s in set(r["status"])},
               cells=[dict(tau=c["tau"], diameter=c["diameter"], re_target=c["re_target"],
                           re_p=float(x), delta_rho=c["delta_rho"], K_stokes=float(k0),
                           K_app=float(k1), steps=int(n), status=s)
                      for c, x, k0, k1, n, s in zip(cells, re, K, r["K_D"], r["steps"],
                                                     r["status"])])
    log(f"[batch] main run {secs:.1f} s, {out['mflups']:.0f} MFLUPS, statuses {out['counts']}")
    return out


def speed(n_cells=256, edge=64, seed=4, steps=100, shape=None, packs=False, log=print,
          device=None):
    """The study's batch under its Stokes forcing (or, with packs, the
    warm-start benchmark's random packs of 8-27 spheres at tau 0.8, seed 5),
    stepped `steps` times from rest with every cell running: ms per step of
    all cells.  shape =
    (wavefronts per block, z planes per block, solid-write mode) fixes the
    launch (then the only step launches are the timed ones, as a profiler
    should see them); by default the autotuner chooses it."""
    if packs:
        from . import warmstart_study

        drawn = warmstart_study.draw_packs(n_cells, edge, 5, warmstart_study.EVAL_SPHERES)
        cells = [dict(spheres=sp, tau=0.8, magic=3 / 16, delta_rho=1e-5) for sp, _ in drawn]
    else:
        cells = [dict(c, delta_rho=1e-7) for c in draw_cells(n_cells, seed, edge)[0]]
    b = lbm.Batch((edge, edge, edge), cells, wall="cli", storage="fp32", device=device)
    if shape:
        by, zp, mode = shape
        b.set_shape(by, zp)
        b.set_solid_writes(mode)
    else:
        by, zp, _ = b.autotune(steps=5)
    b.init_equilibrium()
    b.synchronize()
    t0 = time.perf_counter()
    b.step(steps)
    b.synchronize()
    ms = (time.perf_counter() - t0) / steps * 1e3
    out = dict(n_cells=n_cells, edge=edge, n_fluid=int(b.info.n_fluid), waves_per_block=by,
               z_planes_per_block=zp, solid_writes=b.solid_writes,
               tile=[b.info.tile_width, b.info.tile_height], steps=steps, ms_per_step=ms,
               mflups=b.info.n_fluid / ms / 1e3)
    b.close()
    log(f"[batch] {steps} steps of all cells: {ms:.4f} ms per step, {out['mflups']:.0f} MFLUPS")
    return out


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--cells", type=int, default=256)
    ap.add_argument("--edge", type=int, default=64)
    ap.add_argument("--seed", type=int, default=4)
    ap.add_argument("--max-steps", type=int, default=200000)
    ap.add_argument("--out", default=None)
    ap.add_argument("--speed", type=int, default=0, metavar="STEPS",
                    help="only time STEPS steps of the batch from rest")
    ap.add_argument("--shape", type=int, nargs=3, default=None, metavar=("WAVES", "ZPER", "MODE"),
                    help="launch shape for --speed (default: autotuned)")
    ap.add_argument("--packs", action="store_true",
                    help="--speed on the warm-start benchmark's packs of 8-27 spheres")
    a = ap.parse_args(argv)
    log = lambda s: print(s, flush=True)  # noqa: E731
    if a.speed > 0:
        res = speed(a.cells, a.edge, a.seed, a.speed, shape=a.shape, packs=a.packs, log=log)
    else:
        res = run(a.cells, a.edge, a.seed, max_steps=a.max_steps, log=log)
    txt = json.dumps(res)
    if a.out:
        open(a.out, "w").write(txt)
    else:
        print(txt)
    return 0


if __name__ == "__main__":
    sys.exit(main())
