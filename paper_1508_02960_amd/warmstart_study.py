"""Learned warm start: training fields from the batch solver, training of the
U-Net on the GPU, and cold- versus warm-start runs to a residual.

Training cells are periodic cubes of random overlapping spheres of one common
radius (1-4 spheres per 64^3 cell, porosity U[0.35, 0.6]); the evaluation
packs hold 8-27 spheres per 128^3 cell at the same porosities, so both sets
share the radius range (about 20-40 lattice units).  Only packs whose pore
space percolates in x are kept.  Every cell is solved in the Stokes regime
by the batch solver (TRT, Lambda = 3/16, CLI walls, FP32); with Lambda fixed
the steady TRT solution in the units of warmstart.fields_to_targets does not
depend on tau, so the training fields use tau = 1 (fast relaxation) and the
evaluation runs use tau = 0.8.

Several starts are compared on the same evaluation batch, each run by the
plain iteration to the residual tolerance: rest (g = 0), the linear density
profile of the pressure drop with u = 0, the network's velocity (its wall
layer at rest) with and without its density fluctuation, and the converged
fields themselves (the bound of any start from an equilibrium).  The
iteration decides the permeability in all of them.

    python -m paper_1508_02960_amd.warmstart_study train --out unet.npz
    python -m paper_1508_02960_amd.warmstart_study evaluate --weights unet.npz --out eval.json
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

from . import inputs, lbm, observables
from . import warmstart as W

TRAIN_SPHERES = (1, 4)
EVAL_SPHERES = (8, 27)
POROSITY = (0.35, 0.6)


def _log(msg: str) -> None:
    print(msg, flush=True)


# ------------------------------------------------------------------- packs

def fit_pack(draw, edge: int):
    """Common radius that gives the drawn porosity on the lattice, and the
    fluid mask: node p is solid iff its squared periodic distance to a
    centre is below r^2, so the solid count is a quantile of those squared
    distances (r^2 is placed midway between two of them)."""
    ax = np.arange(edge, dtype=np.float64)
    d2 = np.full((edge, edge, edge), np.inf)
    for cx, cy, cz in draw["centres"]:
        per = []
        for v in (cz, cy, cx):
            a = np.abs(ax - v)
            per.append(np.minimum(a, edge - a) ** 2)
        d2 = np.minimum(d2, per[0][:, None, None] + per[1][None, :, None] + per[2][None, None, :])
    flat = np.sort(d2.ravel())
    k = int(round((1.0 - draw["porosity"]) * flat.size))
    k = min(max(k, 1), flat.size - 1)
    r2 = 0.5 * (flat[k - 1] + flat[k])
    r = float(np.sqrt(r2))
    spheres = np.hstack([draw["centres"], np.full((len(draw["centres"]), 1), r)])
    return spheres, d2 >= r2


def draw_packs(n: int, edge: int, seed: int, n_range, phi_range=POROSITY):
    """n percolating packs: list of (spheres, fluid mask)."""
    out = []
    for dr in inputs.pack_draws(seed, edge, n_range, phi_range):
        if len(out) == n:
            break
        spheres, fluid = fit_pack(dr, edge)
        if W.percolates_x(fluid):
            out.append((spheres, fluid))
    return out


# ---------------------------------------------------------------- solving

def solve_stokes(packs, edge: int, tau: float, delta_rho: float, tol: float, max_steps: int,
                 device=None):
    """Steady fields of every pack by one batch run; returns targets
    (n, e, e, e, 4) float32, fluid masks (n, e, e, e) bool, results dict."""
    cells = [dict(spheres=sp, tau=tau, magic=3 / 16, delta_rho=delta_rho) for sp, _ in packs]
    b = lbm.Batch((edge, edge, edge), cells, wall="cli", storage="fp32", device=device)
    try:
        b.autotune(steps=5)
        b.run_to_residual(tol, max_steps)
        res = b.results()
        drho, u = b.macroscopic()
        fluid = b.mask() == 0
    finally:
        b.close()
    t = np.stack([W.fields_to_targets(drho[i], u[:, i], delta_rho, tau, fluid[i])
                  for i in range(len(packs))])
    return t, fluid, res


def training_set(n_cells: int, edge: int, seed: int, per_batch: int, tau: float,
                 delta_rho: float, tol: float, max_steps: int, device=None, log=_log,
                 time_limit: float = 1e30, n_range=TRAIN_SPHERES):
    """Device tensors (fluid uint8 (n, e, e, e), targets float32 (n, e, e, e, 4))
    of converged cells, from batches of per_batch cells with seeds seed, seed+1...
    Stops early (after a whole batch) once time_limit seconds have passed."""
    import torch

    dev = torch.device(device if device is not None else "cuda")
    fl, tg = [], []
    b = 0
    t_start = time.perf_counter()
    while sum(len(f) for f in fl) < n_cells:
        if b > 0 and time.perf_counter() - t_start > time_limit:
            log(f"[train-data] time limit: {sum(len(f) for f in fl)} cells")
            break
        t0 = time.perf_counter()
        want = min(per_batch, n_cells - sum(len(f) for f in fl))
        packs = draw_packs(want, edge, seed + b, n_range)
        t, fluid, res = solve_stokes(packs, edge, tau, delta_rho, tol, max_steps, device)
        ok = np.array([s == "converged" for s in res["status"]])
        fl.append(torch.from_numpy(fluid[ok].astype(np.uint8)).to(dev))
        tg.append(torch.from_numpy(t[ok]).to(dev))
        log(f"[train-data] batch {b}: {ok.sum()}/{len(ok)} converged, steps max "
            f"{int(res['steps'].max())}, K_D median {np.median(res['K_D']):.3g}, "
            f"{time.perf_counter() - t0:.1f} s")
        b += 1
    return torch.cat(fl)[:n_cells], torch.cat(tg)[:n_cells]


# --------------------------------------------------------------- training

def rel_errors(net, fluid, targets, minibatch: int = 4):
    """Relative L2 errors (velocity, density fluctuation) of the network on
    the given cells, over fluid nodes; targets in network output units."""
    torch = net.ctx.torch
    num = torch.zeros(2, dtype=torch.float64, device=net.ctx.dev)
    den = torch.zeros(2, dtype=torch.float64, device=net.ctx.dev)
    for i in range(0, len(fluid), minibatch):
        f = fluid[i:i + minibatch]
        out = net.forward(W.network_input(net.ctx, f))[..., :4].double()
        t = targets[i:i + minibatch].double()
        w = f.double()[..., None]
        e2 = (out - t) ** 2 * w
        t2 = t ** 2 * w
        num += torch.stack([e2[..., :3].sum(), e2[..., 3].sum()])
        den += torch.stack([t2[..., :3].sum(), t2[..., 3].sum()])
    r = (num / den).sqrt().cpu().numpy()
    return float(r[0]), float(r[1])


def train(net, fluid, targets, *, epochs: int, minibatch: int, lr: float, val_frac: float = 0.04,
          time_limit: float = 1e30, seed: int = 0, log=_log, checkpoint=None):
    """Adam on the weighted MSE over fluid nodes, cosine learning rate with
    a short warm-up; the last val_frac of the cells are held out.  targets
    are in target units; the network learns them divided by net.scale."""
    torch = net.ctx.torch
    n = len(fluid)
    n_val = max(1, int(round(val_frac * n))) if n > 1 else 0
    n_tr = n - n_val
    w = fluid[:n_tr].bool()[..., None]
    net.scale = float(torch.sqrt((targets[:n_tr, ..., :3] ** 2 * w).sum()
                                 / (3 * w.sum())).item())
    tn = targets / net.scale
    rng = np.random.default_rng(seed)
    steps_per_epoch = max(1, n_tr // minibatch)
    total = epochs * steps_per_epoch
    warm = min(100, total // 10 + 1)
    t0 = t_log = time.perf_counter()
    history = []
    step = 0
    for ep in range(epochs):
        perm = rng.permutation(n_tr)
        acc = torch.zeros((), dtype=torch.float64, device=net.ctx.dev)
        for j in range(steps_per_epoch):
            idx = torch.from_numpy(perm[j * minibatch:(j + 1) * minibatch]).to(net.ctx.dev)
            f = fluid[idx]
            out = net.forward(W.network_input(net.ctx, f))
            wt = f.float()
            loss, g = net.loss(out, tn[idx], wt, 4.0 * float(wt.sum().item()), sync=False)
            net.backward(g)
            # the schedule ends at the last step or at the time limit
            frac = min(1.0, max(step / max(total - 1, 1),
                                (time.perf_counter() - t0) / time_limit))
            rate = lr * min(1.0, (step + 1) / warm) * (0.05 + 0.95 * 0.5 * (1 + np.cos(np.pi * frac)))
            net.adam_step(rate)
            acc += loss
            step += 1
            if time.perf_counter() - t_log > 60:
                t_log = time.perf_counter()
                log(f"[train] epoch {ep} step {j + 1}/{steps_per_epoch}, "
                    f"{t_log - t0:.0f} s")
            if time.perf_counter() - t0 > time_limit:
                break
        train_loss = float(acc.item()) / max(1, j + 1)
        ev = rel_errors(net, fluid[n_tr:], tn[n_tr:]) if n_val else (float("nan"),) * 2
        el = time.perf_counter() - t0
        history.append(dict(epoch=ep, loss=train_loss, val_rel_u=ev[0], val_rel_p=ev[1],
                            seconds=el))
        log(f"[train] epoch {ep}: loss {train_loss:.4g}, held-out relative error u {ev[0]:.4f} "
            f"p {ev[1]:.4f}, {el:.0f} s")
        if checkpoint:
            net.save(checkpoint)
        if el > time_limit:
            log(f"[train] time limit reached after epoch {ep}")
            break
    return history


# ------------------------------------------------------------- evaluation

def _run(b, tol, max_steps, log, name):
    """Run the batch from its current state to tol; per-cell results."""
    t0 = time.perf_counter()
    st, steps, _ = b.run_to_residual(tol, max_steps)
    el = time.perf_counter() - t0
    r = b.results()
    out = dict(seconds=el, steps=r["steps"].tolist(), K_D=r["K_D"].tolist(), U=r["U"][:, 0].tolist(),
               status=r["status"])
    log(f"[eval] {name}: {el:.1f} s, steps median {np.median(r['steps']):.0f} "
        f"max {r['steps'].max()}, statuses {dict((s, r['status'].count(s)) for s in set(r['status']))}")
    return out


class _DeviceStart:
    """Start fields already on the device (Batch.init_equilibrium_device)."""

    def __init__(self, fields):
        self.fields = fields


def _init(b, start):
    """Initialise the batch from a start: host (drho, u) or _DeviceStart."""
    if isinstance(start, _DeviceStart):
        b.init_equilibrium_device(start.fields)
    else:
        b.init_equilibrium(*start)


def _trajectory(b, start, chunk, n_chunks):
    """Per-cell U_x after each of n_chunks runs of chunk steps from start
    (tolerance 0, so every cell runs the full chunk)."""
    _init(b, start)
    traj = []
    for _ in range(n_chunks):
        b.run_to_residual(0.0, chunk)
        traj.append(b.results()["U"][:, 0].copy())
    return np.array(traj)  # (n_chunks, n_cells)


def evaluate(nets, packs, edge: int, *, tau: float, delta_rho: float, tol: float, max_steps: int,
             device=None, log=_log, chunk: int = 0, n_chunks: int = 0,
             with_density: bool = False, controls: bool = True, two_grid: bool = False,
             direct: bool = True):
    """Starts of the same packs, each run to tol by the plain iteration:
    rest; linear density; the network's velocity (wall layer at rest) with
    the linear density; with with_density the same plus the network's
    density fluctuation; and, as the bound of any equilibrium-initialised warm start, the
    converged fields of the rest run.  Reports per-cell steps and K_D, wall
    times, the network's error against the converged fields and, with
    chunk > 0, |U_x / U_x* - 1| every chunk steps for each start.  nets is
    a network or a dict name -> network; the starts of a network named n
    are network_u[n] and network_u_rho[n] (no suffix for a single one).
    controls=False runs only the rest and network starts.  With two_grid
    each network also predicts on the half-resolution grid of every pack
    (warmstart.coarse_fluid), and the prediction interpolated back
    (warmstart.predict_two_grid) is the start network_u_2grid[n]; direct=False
    then leaves out the full-resolution starts."""
    if not isinstance(nets, dict):
        nets = {"": nets}
    cells = [dict(spheres=sp, tau=tau, magic=3 / 16, delta_rho=delta_rho) for sp, _ in packs]
    b = lbm.Batch((edge, edge, edge), cells, wall="cli", storage="fp32", device=device)
    out = dict(n_cells=len(packs), edge=edge, tau=tau, delta_rho=delta_rho, tol=tol)
    try:
        out["launch_shape"] = list(b.autotune(steps=5)[:2])
        fluid = b.mask() == 0
        lin = W.linear_density(fluid.shape, delta_rho, fluid)
        starts = {"rest": (None, None)}
        if controls:
            starts["linear_density"] = (lin, None)
        preds = {}
        for tag, net in nets.items():
            if direct or not two_grid:
                t0 = time.perf_counter()
                pred = np.stack([net.predict(fluid[i]) for i in range(len(packs))])
                out["predict_seconds" + tag] = time.perf_counter() - t0
                preds[tag] = pred
                wu = [W.warm_fields(pred[i], delta_rho, tau, fluid[i])
                      for i in range(len(packs))]
                starts["network_u" + tag] = (lin, np.stack([w[1] for w in wu], axis=1))
            if two_grid:
                # the whole start on the device, timed: coarse masks, network,
                # prolongation and the start fields
                ctx = net.ctx
                t0 = time.perf_counter()
                fine = ctx.f32(len(packs), edge, edge, edge, 4)
                for i, (sp, _) in enumerate(packs):
                    W.predict_two_grid_device(net, sp, edge, out=fine[i])
                fields = W.warm_fields_device(ctx, fine, fluid, delta_rho, tau)
                ctx.torch.cuda.synchronize()
                out["predict_seconds_2grid" + tag] = time.perf_counter() - t0
                preds["_2grid" + tag] = fine.cpu().numpy()
                starts["network_u_2grid" + tag] = _DeviceStart(fields)
            if with_density and tag in preds:
                wr = [W.warm_fields(preds[tag][i], delta_rho, tau, fluid[i], use_density=True)
                      for i in range(len(packs))]
                starts["network_u_rho" + tag] = (np.stack([w[0] for w in wr]),
                                                 np.stack([w[1] for w in wr], axis=1))
        conv = None
        extra = [("converged_fields", None)] if controls else []
        for name, start in list(starts.items()) + extra:
            if name == "converged_fields":
                start = conv
            _init(b, start)
            out[name] = _run(b, tol, max_steps, log, name)
            if name == "rest":
                drho, u = b.macroscopic()
                conv = (drho, u)
                for tag, pred in preds.items():
                    eu, ep, eU = [], [], []
                    for i in range(len(packs)):
                        t = W.fields_to_targets(drho[i], u[:, i], delta_rho, tau, fluid[i])
                        f = fluid[i]
                        eu.append(float(np.linalg.norm((pred[i][..., :3] - t[..., :3])[f])
                                        / np.linalg.norm(t[..., :3][f])))
                        ep.append(float(np.linalg.norm((pred[i][..., 3] - t[..., 3])[f])
                                        / np.linalg.norm(t[..., 3][f])))
                        eU.append(float((pred[i][..., 0] * f).sum() / (t[..., 0] * f).sum() - 1))
                    out["network_rel_error_u" + tag] = eu
                    out["network_rel_error_p" + tag] = ep
                    out["network_rel_error_U" + tag] = eU
        if chunk > 0:
            Ustar = np.array(out["rest"]["U"])
            for name in ["rest"] + (["converged_fields"] if controls else []) + [
                    n for n in starts if n.startswith("network_u") and "rho" not in n]:
                st = conv if name == "converged_fields" else starts[name]
                traj = _trajectory(b, st, chunk, n_chunks)
                out[name]["trajectory_rel_error"] = np.abs(traj / Ustar[None] - 1).tolist()
                out[name]["trajectory_chunk"] = chunk
    finally:
        b.close()
    cold = np.array(out["rest"]["steps"], float)
    kc = np.array(out["rest"]["K_D"])
    for name in [n for n in out if isinstance(out[n], dict) and "steps" in out[n] and n != "rest"]:
        s = np.array(out[name]["steps"], float)
        k = np.array(out[name]["K_D"])
        out[name]["step_ratio_median"] = float(np.median(s / cold))
        out[name]["step_ratio_mean"] = float(np.mean(s / cold))
        out[name]["total_step_ratio"] = float(s.sum() / cold.sum())
        out[name]["max_rel_K_diff"] = float(np.max(np.abs(k / kc - 1)))
    out["porosity"] = [float(f.mean()) for _, f in packs]
    out["radius"] = [float(sp[0, 3]) for sp, _ in packs]
    out["n_spheres"] = [int(len(sp)) for sp, _ in packs]
    return out


# -------------------------------------------------------------------- CLI

def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    sub = ap.add_subparsers(dest="cmd", required=True)
    tr = sub.add_parser("train")
    tr.add_argument("--cells", type=int, default=4096)
    tr.add_argument("--edge", type=int, default=64)
    tr.add_argument("--per-batch", type=int, default=256)
    tr.add_argument("--seed", type=int, default=5000)
    tr.add_argument("--tau", type=float, default=1.0)
    tr.add_argument("--delta-rho", type=float, default=1e-5)
    tr.add_argument("--tol", type=float, default=1e-6)
    tr.add_argument("--max-steps", type=int, default=50000)
    tr.add_argument("--widths", default="32,64,128,256")
    tr.add_argument("--spheres", default="1,4", help="sphere count range per cell")
    tr.add_argument("--epochs", type=int, default=8)
    tr.add_argument("--minibatch", type=int, default=4)
    tr.add_argument("--lr", type=float, default=1e-3)
    tr.add_argument("--time-limit", type=float, default=1e30)
    tr.add_argument("--data-time-limit", type=float, default=1e30)
    tr.add_argument("--out", required=True)
    tr.add_argument("--history")
    ev = sub.add_parser("evaluate")
    ev.add_argument("--weights", required=True, nargs="+",
                    help="network weights, as path or name=path")
    ev.add_argument("--with-density", action="store_true")
    ev.add_argument("--two-grid", action="store_true",
                    help="also start from each network's half-resolution prediction")
    ev.add_argument("--spheres", default="8,27", help="sphere count range per cell")
    ev.add_argument("--cells", type=int, default=64)
    ev.add_argument("--edge", type=int, default=128)
    ev.add_argument("--seed", type=int, default=5)
    ev.add_argument("--tau", type=float, default=0.8)
    ev.add_argument("--delta-rho", type=float, default=1e-5)
    ev.add_argument("--tol", type=float, default=1e-8)
    ev.add_argument("--max-steps", type=int, default=200000)
    ev.add_argument("--chunk", type=int, default=0)
    ev.add_argument("--n-chunks", type=int, default=0)
    ev.add_argument("--out", required=True)
    sp = sub.add_parser("speed")
    sp.add_argument("--edge", type=int, default=64)
    sp.add_argument("--minibatch", type=int, default=4)
    sp.add_argument("--steps", type=int, default=10)
    rp = sub.add_parser("report")
    rp.add_argument("--train", nargs="*", default=[], help="title=history.json")
    rp.add_argument("--eval", nargs="*", default=[], help="title=eval.json")
    rp.add_argument("--out", required=True)
    a = ap.parse_args(argv)
    if a.cmd == "speed":
        speed(a.edge, a.minibatch, a.steps)
        return 0
    if a.cmd == "report":
        parts = []
        for item in a.train:
            title, _, path = item.partition("=")
            with open(path) as fh:
                parts.append(report_training(json.load(fh), title))
        for item in a.eval:
            title, _, path = item.partition("=")
            with open(path) as fh:
                parts.append(report_eval(json.load(fh), title))
        with open(a.out, "w") as fh:
            fh.write("\n".join(parts))
        return 0
    if a.cmd == "train":
        t0 = time.perf_counter()
        fluid, targets = training_set(a.cells, a.edge, a.seed, a.per_batch, a.tau, a.delta_rho,
                                      a.tol, a.max_steps, time_limit=a.data_time_limit,
                                      n_range=tuple(int(v) for v in a.spheres.split(",")))
        gen = time.perf_counter() - t0
        _log(f"[train-data] {len(fluid)} cells in {gen:.0f} s")
        net = W.UNet(widths=tuple(int(v) for v in a.widths.split(",")), seed=a.seed)
        _log(f"[train] {net.n_params()} parameters")
        hist = train(net, fluid, targets, epochs=a.epochs, minibatch=a.minibatch, lr=a.lr,
                     time_limit=a.time_limit - gen, checkpoint=a.out)
        net.save(a.out)
        if a.history:
            with open(a.history, "w") as fh:
                json.dump(dict(cells=len(fluid), generate_seconds=gen, params=net.n_params(),
                               scale=net.scale, history=hist, args=vars(a)), fh, indent=1)
    else:
        nets = {}
        for w in a.weights:
            name, _, path = w.rpartition("=")
            nets[f"[{name}]" if name else ""] = W.UNet.load(path)
        packs = draw_packs(a.cells, a.edge, a.seed, tuple(int(v) for v in a.spheres.split(",")))
        res = evaluate(nets, packs, a.edge, tau=a.tau, delta_rho=a.delta_rho, tol=a.tol,
                       max_steps=a.max_steps, chunk=a.chunk, n_chunks=a.n_chunks,
                       with_density=a.with_density, two_grid=a.two_grid)
        res["params"] = {k: n.n_params() for k, n in nets.items()}
        with open(a.out, "w") as fh:
            json.dump(res, fh, indent=1)
        for name in [n for n in res if isinstance(res[n], dict) and "step_ratio_median" in res[n]]:
            _log(f"[eval] {name}: median step ratio {res[name]['step_ratio_median']:.3f}, "
                 f"total {res[name]['total_step_ratio']:.3f}, "
                 f"max |K/K_rest - 1| {res[name]['max_rel_K_diff']:.2e}")
    return 0



# ------------------------------------------------------------------ speed

def conv_flops(net, shape) -> float:
    """Multiply-add flops of one forward pass over (n, d, h, w) voxels:
    2 * 27 * c_in * c_out per output voxel of each convolution."""
    n, d, h, w = shape
    tot = 0.0
    levels = {id(c): l for l, c in enumerate(net.enc)}
    levels.update({id(c): 2 - j for j, c in enumerate(net.dec)})
    levels[id(net.head)] = 0
    for c in net.layers():
        m = n * (d >> levels[id(c)]) * (h >> levels[id(c)]) * (w >> levels[id(c)])
        tot += 2.0 * 27 * c.ci * c.co * m
    return tot


def speed(edge: int = 64, minibatch: int = 4, steps: int = 10, widths=(32, 64, 128, 256),
          log=_log):
    """Time forward and forward + backward + Adam training steps of the
    network on random masks (HIP events on torch's stream)."""
    import torch

    net = W.UNet(widths=widths, seed=0)
    rng = np.random.default_rng(0)
    fluid = (rng.uniform(size=(minibatch, edge, edge, edge)) > 0.4).astype(np.uint8)
    x = W.network_input(net.ctx, fluid)
    tgt = torch.zeros((minibatch, edge, edge, edge, 4), device=net.ctx.dev)
    wt = torch.from_numpy(fluid.astype(np.float32)).to(net.ctx.dev)
    norm = 4.0 * float(fluid.sum())

    def train_step():
        out = net.forward(x)
        _, g = net.loss(out, tgt, wt, norm, sync=False)
        net.backward(g)
        net.adam_step(1e-4)

    for _ in range(2):
        train_step()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        net.forward(x)
    e1.record()
    e1.synchronize()
    fwd_ms = e0.elapsed_time(e1) / steps
    e0.record()
    for _ in range(steps):
        train_step()
    e1.record()
    e1.synchronize()
    train_ms = e0.elapsed_time(e1) / steps
    f = conv_flops(net, (minibatch, edge, edge, edge))
    # backward: data gradient of every layer but the first, and weight gradients
    first = 2.0 * 27 * net.enc[0].ci * net.enc[0].co * minibatch * edge ** 3
    ftrain = 3 * f - first
    res = dict(edge=edge, minibatch=minibatch, params=net.n_params(), forward_ms=fwd_ms,
               train_ms=train_ms, forward_tflops=f / fwd_ms / 1e9,
               train_tflops=ftrain / train_ms / 1e9, forward_gflop=f / 1e9,
               train_gflop=ftrain / 1e9)
    log(f"[speed] {edge}^3 x {minibatch}: forward {fwd_ms:.2f} ms ({res['forward_tflops']:.1f} "
        f"TFLOP/s), train step {train_ms:.2f} ms ({res['train_tflops']:.1f} TFLOP/s)")
    return res


# ----------------------------------------------------------------- report

def steps_to_accuracy(traj, level: float, chunk: int) -> np.ndarray:
    """Per cell, the steps after which |U/U* - 1| stays below level (NaN if
    it is still above at the end of the trajectory)."""
    out = []
    for col in np.asarray(traj).T:
        above = np.nonzero(col >= level)[0]
        if len(above) == 0:
            out.append(chunk)
        elif above[-1] + 1 < len(col):
            out.append((above[-1] + 2) * chunk)
        else:
            out.append(np.nan)
    return np.array(out, float)


def report_eval(res: dict, title: str) -> str:
    """Markdown tables of one evaluation."""
    names = ["rest"] + [n for n in res if isinstance(res[n], dict) and "step_ratio_median" in res[n]]
    lines = [f"### {title}", "",
             f"{res['n_cells']} cells of {res['edge']}^3, {min(res['n_spheres'])}-{max(res['n_spheres'])} "
             f"spheres, porosity {min(res['porosity']):.2f}-{max(res['porosity']):.2f}, radius "
             f"{min(res['radius']):.1f}-{max(res['radius']):.1f}; tau {res['tau']}, delta_rho "
             f"{res['delta_rho']:g}, residual tolerance {res['tol']:g}; one batch run per start.  "
             "Network inference for all cells: " + ", ".join(
                 f"{res[k]:.1f} s" for k in res if k.startswith("predict_seconds")) + ".", "",
             "| start | wall time (s) | steps, median | steps / rest, median | total steps / rest "
             "| max \\|K_D / K_D(rest) - 1\\| |",
             "|---|---|---|---|---|---|"]
    for n in names:
        r = res[n]
        if n == "rest":
            lines.append(f"| rest | {r['seconds']:.1f} | {np.median(r['steps']):.0f} | 1 | 1 | 0 |")
        else:
            lines.append(f"| {n} | {r['seconds']:.1f} | {np.median(r['steps']):.0f} | "
                         f"{r['step_ratio_median']:.3f} | {r['total_step_ratio']:.3f} | "
                         f"{r['max_rel_K_diff']:.1e} |")
    traj = [n for n in names if "trajectory_rel_error" in res[n]]
    if traj:
        lines += ["", "Steps until the superficial velocity stays within a relative error of "
                  "U* (the converged rest-start value), median over cells:", "",
                  "| start | 1e-2 | 1e-3 | 1e-4 | 1e-5 |", "|---|---|---|---|---|"]
        for n in traj:
            c = res[n]["trajectory_chunk"]
            row = [f"{np.nanmedian(steps_to_accuracy(res[n]['trajectory_rel_error'], lv, c)):.0f}"
                   for lv in (1e-2, 1e-3, 1e-4, 1e-5)]
            lines.append(f"| {n} | " + " | ".join(row) + " |")
    errs = [k for k in res if k.startswith("network_rel_error_u")]
    if errs:
        lines += ["", "| network | relative L2 error of u, median | of the density fluctuation | "
                  "of U (mean flow), median \\|.\\| |", "|---|---|---|---|"]
        for k in errs:
            tag = k[len("network_rel_error_u"):] or "-"
            lines.append(f"| {tag} | {np.median(res[k]):.3f} | "
                         f"{np.median(res['network_rel_error_p' + k[len('network_rel_error_u'):]]):.3f} | "
                         f"{np.median(np.abs(res['network_rel_error_U' + k[len('network_rel_error_u'):]])):.3f} |")
    return "\n".join(lines) + "\n"


def report_training(hist: dict, title: str) -> str:
    h = hist["history"]
    a = hist["args"]
    return (f"### {title}\n\n{hist['cells']} cells of {a['edge']}^3 ({a.get('spheres', '1,4')} spheres), solved "
            f"to {a['tol']:g} at tau {a['tau']} in {hist['generate_seconds']:.0f} s; "
            f"{hist['params']} parameters, {len(h)} epochs of Adam (minibatch {a['minibatch']}, "
            f"lr {a['lr']:g}) in {h[-1]['seconds']:.0f} s; held-out relative error after the first "
            f"and last epoch: velocity {h[0]['val_rel_u']:.3f} -> {h[-1]['val_rel_u']:.3f}, "
            f"density fluctuation {h[0]['val_rel_p']:.3f} -> {h[-1]['val_rel_p']:.3f}.\n")


if __name__ == "__main__":
    sys.exit(main())
