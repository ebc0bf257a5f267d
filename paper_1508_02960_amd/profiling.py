"""rocprofv3 helpers: kernel-time summaries and HBM traffic from byte counters.

    python -m paper_1508_02960_amd.profiling stats <kernel_stats.csv> <out.md> <command...>
        markdown table of a --kernel-trace --stats run
    python -m paper_1508_02960_amd.profiling traffic <fetch.csv> <write.csv> <probe_bytes>
        <kernel> <workload> <n_fluid> <bytes_per_update> <out.md> <out.json> <command...>
        HBM bytes per launch of <kernel> from a FETCH_SIZE run and a WRITE_SIZE run
        of bench.py.  The same runs hold the bandwidth probes of known byte counts
        (lbm_bandwidth_probe: read, write and copy of <probe_bytes> bytes); the
        read probe scales FETCH_SIZE to bytes, the write probe scales WRITE_SIZE,
        and the copy probe, read and written through both, checks both factors.
"""
from __future__ import annotations

import csv
import hashlib
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCES = [os.path.join(HERE, "csrc", f) for f in ("kernels.hpp", "step_impl.hpp")]


def kernel_source_hash() -> str:
    """sha256[:16] of the step kernels' source with comments and blank space
    removed, and of the compiler flags, so that counters stay attached to the
    code they measured."""
    import re

    from .build import HIPCC_FLAGS

    parts = []
    for path in KERNEL_SOURCES:
        src = open(path).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        src = re.sub(r"//[^\n]*", "", src)
        parts.append("\n".join(line.strip() for line in src.splitlines() if line.strip()))
    parts.append(" ".join(HIPCC_FLAGS))
    return hashlib.sha256("\n".join(parts).encode()).hexdigest()[:16]


def short_name(full: str) -> str:
    """Kernel name without namespace, template arguments and signature:
    'void lbm::step_kernel<float, 1, 1, false, true>(...)' -> 'step_kernel'."""
    n = full.replace("(anonymous namespace)::", "")
    n = n.split("(")[0].split("<")[0].strip()
    if n.startswith("void "):
        n = n[5:]
    return n.split("::")[-1]


def _counter_means(path: str):
    """{short kernel name: mean counter value (KiB) per dispatch} of one --pmc run."""
    acc = {}
    with open(path) as f:
        for r in csv.DictReader(f):
            acc.setdefault(short_name(r["Kernel_Name"]), []).append(float(r["Counter_Value"]))
    return {k: sum(v) / len(v) for k, v in acc.items()}, {k: len(v) for k, v in acc.items()}


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


def traffic(fetch, write, probe_bytes, kernel, workload, n_fluid, bpu, out_md, out_json,
            command) -> None:
    fm, fc = _counter_means(fetch)
    wm, wc = _counter_means(write)
    nb = float(probe_bytes)
    f_factor = nb / (fm["read_kernel"] * 1024.0)
    w_factor = nb / (wm["write_kernel"] * 1024.0)
    copy_read = fm["copy_kernel"] * 1024.0 * f_factor / nb
    copy_write = wm["copy_kernel"] * 1024.0 * w_factor / nb
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
        "copy_probe_read_over_bytes": copy_read, "copy_probe_write_over_bytes": copy_write,
        "probe_bytes": int(nb), "dispatches": fc[kernel],
        "command": command,
    }
    json.dump(rec, open(out_json, "w"), indent=1)
    lines = [f"# HBM traffic of `{kernel}` ({workload})", "",
             f"Command (run twice, with `--pmc FETCH_SIZE` and with `--pmc WRITE_SIZE`): "
             f"`{command}`", "",
             "Counters are KiB per dispatch of requests from the L2 caches to the memory side, "
             "which includes hits in the last-level (Infinity) cache, so they bound the HBM "
             "traffic from above.  They are scaled by what the same counters read for "
             f"the bandwidth probes of {int(nb)} bytes in the same runs: FETCH_SIZE x{f_factor:.3f} "
             f"(read probe), WRITE_SIZE x{w_factor:.3f} (write probe).  Check on the copy probe "
             f"(reads and writes {int(nb)} bytes): scaled reads {copy_read:.3f}x, scaled writes "
             f"{copy_write:.3f}x the bytes it moves.", "",
             "| quantity | per launch |", "|---|---|",
             f"| FETCH_SIZE (raw KiB) | {fm[kernel]:.1f} |",
             f"| WRITE_SIZE (raw KiB) | {wm[kernel]:.1f} |",
             f"| read bytes (scaled) | {kf / 1e6:.2f} MB |",
             f"| written bytes (scaled) | {kw / 1e6:.2f} MB |",
             f"| total memory-side traffic (HBM and last-level-cache hits) | {(kf + kw) / 1e6:.2f} MB |",
             f"| algorithmic bytes ({n_fluid} fluid cells x {bpu} B) | {alg / 1e6:.2f} MB |",
             f"| reads / algorithmic reads | {kf / (alg / 2):.3f} |",
             f"| writes / algorithmic writes | {kw / (alg / 2):.3f} |",
             f"| traffic / algorithmic | {(kf + kw) / alg:.3f} |",
             f"| dispatches averaged | {fc[kernel]} |",
             f"| kernel source sha256[:16] | {kernel_source_hash()} |"]
    open(out_md, "w").write("\n".join(lines) + "\n")


def main(argv) -> int:
    if not argv:
        print(__doc__)
        return 2
    cmd = argv[0]
    if cmd == "stats":
        stats(argv[1], argv[2], " ".join(argv[3:]))
    elif cmd == "traffic":
        traffic(*argv[1:10], " ".join(argv[10:]))
    else:
        print(__doc__)
        return 2
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
