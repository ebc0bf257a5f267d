#!/usr/bin/env python3
"""Throughput of the fused D3Q19 stream-and-collide hot path on one MI355X.

Workload (default): the 512^3 box of 2 x 2 x 2 simple-cubic cells of 256^3,
each holding one centred sphere of diameter 240 lattice units (porosity
0.569), D3Q19 TRT (Lambda = 6e-6, tau = 0.5005, the paper's settings for its
highest Reynolds numbers) with CLI interpolated bounce-back and the periodic
pressure drop, FP32 storage of the deviations f - w, FP64 mean-velocity
reductions every 100 steps.  One bench step is one time step of that
production loop.  Inputs are synthetic and seeded; all state is resident in
HBM when timing starts.

Prints one JSON line: metric, value (fluid-cell updates per second, in
millions), the roofline of the step kernel measured with HIP events on the
stream it runs on, next to attainable ceilings measured by plain streaming
kernels on the same GPU; the time to steady state from rest and from the
learned warm start on 128^3 random sphere packs; and the CPU oracle timed on
one 256^3 cell of the same geometry, single-threaded and on all cores.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "D3Q19 TRT MLUPS + %HBM roofline; time-to-steady-state (plain vs warm-start)"
HBM_PEAK_GBS = 8000.0
PROFILES = os.path.join(ROOT, "profiles")

WORKLOADS = {
    # name: (shape, sphere diameter, collision, wall, storage, tau, magic, delta_rho)
    "sc128_d100_trt_cli_fp32": ((128, 128, 128), 100.0, "trt", "cli", "fp32", 0.8, 3 / 16, 1.5e-4),
    "sc256_d200_trt_cli_fp32": ((256, 256, 256), 200.0, "trt", "cli", "fp32", 0.8, 3 / 16, 1.5e-4),
    "sc32_d24_trt_sbb_fp64": ((32, 32, 32), 24.0, "trt", "sbb", "fp64", 0.8, 3 / 16, 2.15e-6),
    "sc128_d100_trt_cli_fp16": ((128, 128, 128), 100.0, "trt", "cli", "fp16", 0.8, 3 / 16, 1.5e-4),
    "sc128_d100_trt_cli_bf16": ((128, 128, 128), 100.0, "trt", "cli", "bf16", 0.8, 3 / 16, 1.5e-4),
    "sc128_d100_mrt_cli_fp32": ((128, 128, 128), 100.0, "mrt", "cli", "fp32", 0.8, 3 / 16, 1.5e-4),
    # the 512^3 block at the pressure drop of the Re_p = 5812 target
    "sc512_d240x8_trt_cli_fp32": ((512, 512, 512), 240.0, "trt", "cli", "fp32", 0.5005, 6e-6,
                                  3.805e-5),
    "sc512_d240x8_trt_cli_fp16": ((512, 512, 512), 240.0, "trt", "cli", "fp16", 0.5005, 6e-6,
                                  3.805e-5),
    "sc512_d240x8_trt_cli_bf16": ((512, 512, 512), 240.0, "trt", "cli", "bf16", 0.5005, 6e-6,
                                  3.805e-5),
    "sc512_d240x8_mrt_cli_fp32": ((512, 512, 512), 240.0, "mrt", "cli", "fp32", 0.5005, 6e-6,
                                  3.805e-5),
    # the wall rules of Sec. 2.2.1 on the same block, at the Stokes-regime tau = 0.8 (throughput
    # does not depend on tau; some interpolated rules are not stable at tau = 0.5005)
    **{f"sc512_d240x8_trt_{w}_fp32": ((512, 512, 512), 240.0, "trt", w, "fp32", 0.8, 3 / 16,
                                      1e-5) for w in ("sbb", "libb", "qibb", "iebb", "mr")},
}
DEFAULT_WORKLOAD = "sc512_d240x8_trt_cli_fp32"


def workload_spheres(shape, dia):
    """One centred sphere per 256^3 cell (2 x 2 x 2 cells at 512^3)."""
    from paper_1508_02960_amd import inputs

    n = shape[0]
    if n > 256:
        return inputs.simple_cubic_array(n // 256, 256, dia)
    return inputs.centred_sphere(shape, dia)


def kernel_source_hash() -> str:
    from paper_1508_02960_amd.profiling import kernel_source_hash as h

    return h()


def stored_traffic(kernel: str, workload: str):
    """HBM bytes per step-kernel launch from committed rocprofv3 counters, or
    None if they were taken on a different kernel source or workload."""
    try:
        with open(os.path.join(PROFILES, f"{kernel}_{workload}_traffic.json")) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if (t.get("kernel_source_sha256_16") != kernel_source_hash() or t.get("workload") != workload
            or t.get("kernel") != kernel):
        return None
    return t.get("hbm_bytes_per_launch")


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def host_threads() -> int:
    """Threads for the all-core oracle run: OMP_NUM_THREADS when set (the CPU
    share of the GPU's host), else the visible cores."""
    env = os.environ.get("OMP_NUM_THREADS", "")
    return int(env) if env.isdigit() and int(env) > 0 else (os.cpu_count() or 1)


def cpu_baseline(wl, budget_s: float):
    """The FP64 CPU oracle on the same geometry: one 256^3 cell of the
    simple-cubic block (each cell of the 512^3 box is the same problem), or
    the whole box if it is smaller.  Whole steps, single-threaded and on all
    host threads, within about budget_s seconds in total."""
    import oracle

    oracle.build(force=False)
    shape, dia, coll, wall, _, tau, magic, drho = wl
    from paper_1508_02960_amd import inputs

    cell = tuple(min(n, 256) for n in shape)
    o = oracle.Oracle(cell, tau=tau, magic=magic, delta_rho=drho * cell[2] / shape[2],
                      collision=coll, wall=wall, spheres=inputs.centred_sphere(cell, dia))
    o.init()
    n_fluid = int((o.mask == 0).sum())

    def timed(threads, budget):
        oracle.set_threads(threads)
        t0 = time.perf_counter()
        o.step(1)
        per = time.perf_counter() - t0
        n_more = max(0, int(budget / max(per, 1e-9)) - 1)
        t1 = time.perf_counter()
        if n_more:
            o.step(n_more)
        total = per + (time.perf_counter() - t1)
        return 1 + n_more, total

    n_all = host_threads()
    s1, t1 = timed(1, budget_s / 2)
    sa, ta = timed(n_all, budget_s / 2)
    oracle.set_threads(1)
    one = n_fluid * s1 / t1 / 1e6
    return {"value": round(n_fluid * sa / ta / 1e6, 4), "unit": "MFLUPS", "cores": n_all,
            "kind": "oracle",
            "single_thread_value": round(one, 4),
            "cpu_model": cpu_model(), "nproc": os.cpu_count(),
            "sample": f"FP64 oracle steps of one {cell[2]}x{cell[1]}x{cell[0]} cell of the "
                      f"workload geometry ({n_fluid} fluid cells): {sa} steps on {n_all} threads "
                      f"in {ta:.1f} s, {s1} on one thread in {t1:.1f} s"}


def warm_start_leg(n_cells: int):
    """Time to steady state, plain vs learned warm start, on the evaluation
    packs of the warm-start study: n_cells random packs of 128^3 with 8-27
    overlapping spheres of one radius (porosity 0.35-0.6, pore space
    percolating in x, seed 5), TRT-CLI FP32 at tau 0.8, each start run by the
    batch solver to a 1e-8 residual.  The network is the stored one trained
    on 64^3 packs of 8-27 spheres; it predicts each 128^3 pack on the grid of
    half the resolution (its receptive field then spans the cell) and the
    prediction is interpolated back (two-grid start).  The warm start's time
    includes building the start on the device: coarse masks, network,
    prolongation and start fields (warm_setup_s)."""
    from paper_1508_02960_amd import warmstart, warmstart_study

    weights = os.path.join(ROOT, "paper_1508_02960_amd", "data", "unet64_dense_bf16.npz")
    net = warmstart.UNet.load(weights)
    packs = warmstart_study.draw_packs(n_cells, 128, 5, warmstart_study.EVAL_SPHERES)
    r = warmstart_study.evaluate(net, packs, 128, tau=0.8, delta_rho=1e-5, tol=1e-8,
                                 max_steps=400000, controls=False, two_grid=True, direct=False,
                                 log=lambda m: print(m, file=sys.stderr, flush=True))
    plain, warm = r["rest"], r["network_u_2grid"]
    return {
        "workload": f"{n_cells} random packs of 128^3 (8-27 spheres, porosity 0.35-0.6, seed 5), "
                    "TRT-CLI FP32, tau 0.8, residual 1e-8, one batch run per start; two-grid "
                    "start from the network trained on 64^3 packs of 8-27 spheres",
        "plain_s": round(plain["seconds"], 3),
        "warm_s": round(warm["seconds"] + r["predict_seconds_2grid"], 3),
        "warm_setup_s": round(r["predict_seconds_2grid"], 3),
        "plain_steps_median": float(np.median(plain["steps"])),
        "warm_steps_median": float(np.median(warm["steps"])),
        "step_ratio_median": round(warm["step_ratio_median"], 4),
        "total_step_ratio": round(warm["total_step_ratio"], 4),
        "max_rel_K_diff": warm["max_rel_K_diff"],
        "network_rel_error_u_median": round(float(np.median(r["network_rel_error_u_2grid"])), 4),
        "all_converged": all(s == "converged" for s in plain["status"] + warm["status"]),
    }


def ceiling_leg(dev, edge: int, nbytes: int = 4 << 30, reps: int = 10):
    """Attainable bandwidth of plain streaming kernels on this GPU
    (lbm_bandwidth_probe): read, write and copy of nbytes, and the step's
    19-plane pull pattern on an all-fluid periodic cube of the workload's
    edge (no flags, no collision).  GB/s of bytes moved, timed with HIP
    events on the stream the probes run on."""
    import torch

    from paper_1508_02960_amd import lbm

    stream = torch.cuda.current_stream(dev)

    def rate(kind, src, dst, n, moved):
        for _ in range(2):
            lbm.bandwidth_probe(kind, src, dst, n, stream)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            lbm.bandwidth_probe(kind, src, dst, n, stream)
        e1.record(stream)
        torch.cuda.synchronize()
        return round(moved / (e0.elapsed_time(e1) / reps * 1e-3) / 1e9, 1)

    out = {}
    a = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
    b = torch.zeros_like(a)
    out["read"] = rate("read", a, b, nbytes, nbytes)
    out["write"] = rate("write", None, b, nbytes, nbytes)
    out["copy"] = rate("copy", a, b, nbytes, 2 * nbytes)
    del a, b
    n = edge - edge % 16
    a = torch.full((19 * n ** 3,), 1e-3, dtype=torch.float32, device=dev)
    b = torch.zeros_like(a)
    out["gather19"] = rate("gather19", a, b, n, 2 * 19 * 4 * n ** 3)
    del a, b
    torch.cuda.empty_cache()
    out["bytes"] = {"read_write_copy": nbytes, "gather19_edge": n}
    return out


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--workload", default=DEFAULT_WORKLOAD, choices=sorted(WORKLOADS))
    ap.add_argument("--cpu-budget", type=float, default=30.0,
                    help="seconds of CPU oracle time for the cpu_baseline sample (0: skip)")
    ap.add_argument("--warm-cells", type=int, default=16,
                    help="128^3 packs for the plain vs warm-start comparison (0: skip)")
    ap.add_argument("--ceiling-gib", type=float, default=4.0,
                    help="GiB per buffer of the read/write/copy ceiling probes (0: skip)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(the step would shard by z slabs with halo exchange); run with --gpus 1.",
              file=sys.stderr)
        return 2

    import torch

    from paper_1508_02960_amd import inputs, lbm

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 2
    wl = WORKLOADS[args.workload]
    shape, dia, coll, wall, storage, tau, magic, drho = wl
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    d = lbm.Domain(shape, tau=tau, magic=magic, delta_rho=drho, collision=coll, wall=wall,
                   storage=storage, spheres=workload_spheres(shape, dia), device=dev,
                   check_interval=100)
    n_fluid, n_cells = d.n_fluid, d.ncell
    stream = d.stream
    # the step kernel this shape launches (two cells per lane for large 16-bit states)
    kernel = "step_pair_kernel" if d.step_shape()[2] else "step_kernel"
    print(f"[bench] workload {args.workload}: {n_cells} cells, {n_fluid} fluid, "
          f"{d.info.n_links} links, workspace {d.info.workspace_bytes / 2**30:.2f} GiB",
          file=sys.stderr, flush=True)

    # warm-up (also develops a non-trivial flow)
    d.step(args.warmup)
    d.synchronize()

    # timed region: K steps of the production loop (residual check every 100 steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    status, done, res = d.run_to_residual(0.0, args.steps)
    e1.record(stream)
    torch.cuda.synchronize()
    wall_s = time.perf_counter() - t0
    loop_ms = e0.elapsed_time(e1)
    assert done == args.steps, (status, done)
    U, vmax, _ = d.mean_velocity()
    if not np.isfinite(U[0]):
        print("[bench] non-finite state", file=sys.stderr)
        return 1

    # step-kernel timing: back-to-back launches bracketed by events on the
    # library's stream
    k_steps = max(args.steps, 200)
    k0 = torch.cuda.Event(enable_timing=True)
    k1 = torch.cuda.Event(enable_timing=True)
    k0.record(stream)
    d.step(k_steps)
    k1.record(stream)
    torch.cuda.synchronize()
    kernel_ms = k0.elapsed_time(k1) / k_steps

    ms_per_step = max(loop_ms, wall_s * 1e3) / args.steps
    value = n_fluid / (ms_per_step * 1e-3) / 1e6
    bpu = int(d.info.bytes_per_fluid_update)
    alg_bytes = n_fluid * bpu
    achieved = alg_bytes / (kernel_ms * 1e-3) / 1e9
    traffic = stored_traffic(kernel, args.workload)
    out = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "MFLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 6),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp32": "f32", "fp64": "f64", "fp16": "f16 storage, f32 compute",
                  "bf16": "bf16 storage, f32 compute"}[storage],
        "data": "synthetic",
        "config": {
            "workload": args.workload,
            "grid": list(shape[::-1]),
            "sphere_diameter": dia,
            "collision": coll, "wall": wall, "storage": storage,
            "tau": tau, "magic": magic, "delta_rho": drho,
            "fluid_cells": n_fluid, "cells": n_cells,
            "mlups_all_cells": round(n_cells / (ms_per_step * 1e-3) / 1e6, 2),
            "check_interval": 100,
            "parallelism": "single GPU",
        },
        "roofline": {
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "kernel": kernel,
            "kernel_ms": round(kernel_ms, 6),
            "algorithmic_bytes_per_launch": alg_bytes,
            "bytes_per_fluid_update": bpu,
        },
    }
    d.close()
    del d
    torch.cuda.empty_cache()
    if args.ceiling_gib > 0:
        print("[bench] ceiling probes", file=sys.stderr, flush=True)
        ceil = ceiling_leg(dev, shape[2], int(args.ceiling_gib * 2**30) // 16 * 16)
        out["roofline"]["ceiling"] = ceil
        out["roofline"]["frac_of_gather19"] = round(achieved / ceil["gather19"], 4)
        out["roofline"]["frac_of_copy"] = round(achieved / ceil["copy"], 4)
    if args.warm_cells > 0:
        print("[bench] time to steady state", file=sys.stderr, flush=True)
        out["time_to_steady_state"] = warm_start_leg(args.warm_cells)
    if args.cpu_budget > 0:
        print("[bench] cpu baseline", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(wl, args.cpu_budget)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
