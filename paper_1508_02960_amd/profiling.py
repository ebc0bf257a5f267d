"""rocprofv3 helpers: counter calibration with a plain copy and summaries.

    python -m paper_1508_02960_amd.profiling calib
        one plain device-to-device copy of 1 GiB, three times (run it under
        rocprofv3 --pmc FETCH_SIZE and --pmc WRITE_SIZE to get the factors
        that turn each counter into bytes)
    python -m paper_1508_02960_amd.profiling stats <kernel_stats.csv> <out.md> <command...>
        markdown table of a --kernel-trace --stats run
    python -m paper_1508_02960_amd.profiling traffic <fetch.csv> <write.csv>
        <calib_fetch.csv> <calib_write.csv> <kernel> <workload> <n_fluid>
        <bytes_per_update> <out.md> <out.json> <command...>
        HBM bytes per launch of <kernel> from the two counter runs, scaled by
        what the same counters read for the calibration copy.
"""
from __future__ import annotations

import csv
import hashlib
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCE = os.path.join(HERE, "csrc", "kernels.hpp")
CALIB_BYTES = 1 << 30


def kernel_source_hash() -> str:
    with open(KERNEL_SOURCE, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def calib() -> None:
    import torch

    a = torch.ones(CALIB_BYTES // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(f"calib: 3 device-to-device copies of {CALIB_BYTES} bytes")


def _counter_means(path: str):
    """{kernel name: mean counter value (KiB) per dispatch} of one --pmc run."""
    acc = {}
    with open(path) as f:
        for r in csv.DictReader(f):
            name = r["Kernel_Name"].split("(")[0].strip()
            acc.setdefault(name, []).append(float(r["Counter_Value"]))
    return {k: sum(v) / len(v) for k, v in acc.items()}, {k: len(v) for k, v in acc.items()}


def _calib_kernel(means):
    # the dispatch of the calibration copy: the kernel with the largest counter
    return max(means.items(), key=lambda kv: kv[1])


def stats(path: str, out: str, command: str) -> None:
    rows = list(csv.DictReader(open(path)))
    lines = ["# Kernel time summary", "", f"Command: `{command}`", "",
             "| kernel | calls | average (us) | min (us) | max (us) | share (%) |",
             "|---|---|---|---|---|---|"]
    for r in rows:
        lines.append(f"| {r['Name'][:60]} | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} | "
                     f"{float(r['MinNs']) / 1e3:.2f} | {float(r['MaxNs']) / 1e3:.2f} | "
                     f"{float(r['Percentage']):.2f} |")
    open(out, "w").write("\n".join(lines) + "\n")


def traffic(fetch, write, cfetch, cwrite, kernel, workload, n_fluid, bpu, out_md, out_json,
            command) -> None:
    fm, fc = _counter_means(fetch)
    wm, wc = _counter_means(write)
    cf_name, cf = _calib_kernel(_counter_means(cfetch)[0])
    cw_name, cw = _calib_kernel(_counter_means(cwrite)[0])
    f_factor = CALIB_BYTES / (cf * 1024.0)
    w_factor = CALIB_BYTES / (cw * 1024.0)
    kf = fm[kernel] * 1024.0 * f_factor
    kw = wm[kernel] * 1024.0 * w_factor
    alg = int(n_fluid) * int(bpu)
    rec = {
        "kernel": kernel, "workload": workload,
        "kernel_source_sha256_16": kernel_source_hash(),
        "fetch_bytes_per_launch": kf, "write_bytes_per_launch": kw,
        "hbm_bytes_per_launch": kf + kw,
        "algorithmic_bytes_per_launch": alg,
        "fetch_factor": f_factor, "write_factor": w_factor,
        "calibration_kernel": cf_name, "dispatches": fc[kernel],
        "command": command,
    }
    json.dump(rec, open(out_json, "w"), indent=1)
    lines = [f"# HBM traffic of `{kernel}` ({workload})", "",
             f"Command: `{command}`", "",
             "Counters are KiB per dispatch.  Each is scaled by what the same counter reads for "
             f"a plain copy of {CALIB_BYTES} bytes (`{cf_name}`): FETCH_SIZE x{f_factor:.3f}, "
             f"WRITE_SIZE x{w_factor:.3f}.", "",
             "| quantity | per launch |", "|---|---|",
             f"| FETCH_SIZE (raw KiB) | {fm[kernel]:.1f} |",
             f"| WRITE_SIZE (raw KiB) | {wm[kernel]:.1f} |",
             f"| read bytes (scaled) | {kf / 1e6:.2f} MB |",
             f"| written bytes (scaled) | {kw / 1e6:.2f} MB |",
             f"| total HBM traffic | {(kf + kw) / 1e6:.2f} MB |",
             f"| algorithmic bytes ({n_fluid} fluid cells x {bpu} B) | {alg / 1e6:.2f} MB |",
             f"| traffic / algorithmic | {(kf + kw) / alg:.3f} |",
             f"| kernel source sha256[:16] | {kernel_source_hash()} |"]
    open(out_md, "w").write("\n".join(lines) + "\n")


def main(argv) -> int:
    if not argv:
        print(__doc__)
        return 2
    cmd = argv[0]
    if cmd == "calib":
        calib()
    elif cmd == "stats":
        stats(argv[1], argv[2], " ".join(argv[3:]))
    elif cmd == "traffic":
        traffic(*argv[1:11], " ".join(argv[11:]))
    else:
        print(__doc__)
        return 2
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
