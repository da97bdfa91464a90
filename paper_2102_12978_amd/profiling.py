"""Summaries of rocprofv3 output for the committed profile records.

    python -m paper_2102_12978_amd.profiling stats KERNEL_STATS_CSV --cmd "..."
        Markdown table of per-kernel call counts and durations.

    python -m paper_2102_12978_amd.profiling traffic --kernel NAME \
        --fetch CSV --write CSV --copy-fetch CSV --copy-write CSV \
        --copy-bytes BYTES --cells CELLS --cmd "..."
        HBM bytes per dispatch of NAME from FETCH_SIZE / WRITE_SIZE counter
        runs (KiB per dispatch), each scaled by what the same counter reads
        for a plain device copy of a known size. Printed as JSON.

Only reads CSV files; runs nothing on a device.
"""
import argparse
import csv
import hashlib
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2102_12978_amd", "csrc")
KERNEL_SRC = os.path.join(CSRC, "kernels_fused.hip")


def kernel_sha256_16(path=KERNEL_SRC):
    return hashlib.sha256(open(path, "rb").read()).hexdigest()[:16]


def source_of(kernel):
    """Source file of a kernel (by the name the counters carry): the two-step
    kernel, the one-step interior kernel, or the split frame kernels."""
    if "step2" in kernel:
        return os.path.join(CSRC, "kernels_step2.hip")
    if "split_" in kernel:
        return os.path.join(CSRC, "kernels_split.hip")
    return os.path.join(CSRC, "kernels_fused.hip")


def short_name(name):
    """Strip template arguments and namespaces: 'void a::b::f<4>(...)' -> 'f<4>'."""
    n = name.replace("(anonymous namespace)::", "").split("(")[0]
    if n.startswith("void "):
        n = n[5:]
    base, _, tmpl = n.partition("<")
    base = base.split("::")[-1]
    return base + ("<" + tmpl if tmpl else "")


def stats_markdown(path, cmd):
    rows = list(csv.DictReader(open(path)))
    out = [f"Command: `{cmd}`", "",
           "| kernel | calls | total ms | average us | min us | max us | % |",
           "|---|---|---|---|---|---|---|"]
    for r in rows:
        out.append(f"| {short_name(r['Name'])} | {r['Calls']} | "
                   f"{float(r['TotalDurationNs']) / 1e6:.2f} | {float(r['AverageNs']) / 1e3:.2f} | "
                   f"{float(r['MinNs']) / 1e3:.2f} | {float(r['MaxNs']) / 1e3:.2f} | "
                   f"{float(r['Percentage']):.2f} |")
    return "\n".join(out) + "\n"


def counter_per_dispatch(path, kernel, counter):
    """Mean counter value (KiB) over the dispatches whose name contains kernel."""
    vals = [float(r["Counter_Value"]) for r in csv.DictReader(open(path))
            if kernel in r["Kernel_Name"] and r["Counter_Name"].startswith(counter)]
    if not vals:
        raise SystemExit(f"no {counter} rows for a kernel named like {kernel!r} in {path}")
    return sum(vals) / len(vals), len(vals)


def largest_dispatch(path, counter):
    """Counter value (KiB) of the copy dispatches: the largest values in the file."""
    vals = sorted(float(r["Counter_Value"]) for r in csv.DictReader(open(path))
                  if r["Counter_Name"].startswith(counter))
    top = vals[-1]
    same = [v for v in vals if v > 0.9 * top]
    return sum(same) / len(same), len(same)


def traffic(a):
    f_kib, nf = counter_per_dispatch(a.fetch, a.kernel, "FETCH_SIZE")
    w_kib, nw = counter_per_dispatch(a.write, a.kernel, "WRITE_SIZE")
    cf_kib, _ = largest_dispatch(a.copy_fetch, "FETCH_SIZE")
    cw_kib, _ = largest_dispatch(a.copy_write, "WRITE_SIZE")
    f_scale = a.copy_bytes / (cf_kib * 1024.0)
    w_scale = a.copy_bytes / (cw_kib * 1024.0)
    read_b = f_kib * 1024.0 * f_scale
    write_b = w_kib * 1024.0 * w_scale
    return {
        "kernel": a.kernel,
        "kernel_sha256_16": kernel_sha256_16(source_of(a.kernel)),
        "command": a.cmd,
        "dispatches": {"fetch": nf, "write": nw},
        "fetch_kib_per_dispatch": round(f_kib, 1),
        "write_kib_per_dispatch": round(w_kib, 1),
        "copy_bytes": a.copy_bytes,
        "fetch_scale": round(f_scale, 4),
        "write_scale": round(w_scale, 4),
        "read_bytes_per_launch": round(read_b),
        "write_bytes_per_launch": round(write_b),
        "bytes_per_launch": round(read_b + write_b),
        "cells_per_launch": a.cells,
        "bytes_per_cell": round((read_b + write_b) / a.cells, 2) if a.cells else None,
    }


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="what", required=True)
    s = sub.add_parser("stats")
    s.add_argument("csv")
    s.add_argument("--cmd", required=True)
    t = sub.add_parser("traffic")
    for k in ("kernel", "fetch", "write", "copy_fetch", "copy_write", "cmd"):
        t.add_argument("--" + k.replace("_", "-"), dest=k, required=True)
    t.add_argument("--copy-bytes", dest="copy_bytes", type=int, required=True)
    t.add_argument("--cells", type=int, default=0)
    a = ap.parse_args(argv)
    if a.what == "stats":
        sys.stdout.write(stats_markdown(a.csv, a.cmd))
    else:
        print(json.dumps(traffic(a), indent=1))


if __name__ == "__main__":
    main()
