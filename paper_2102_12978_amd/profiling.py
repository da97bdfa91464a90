"""Summaries of rocprofv3 output for the committed profile records.

    python -m paper_2102_12978_amd.profiling stats KERNEL_STATS_CSV --cmd "..."
        Markdown table of per-kernel call counts and durations.

    python -m paper_2102_12978_amd.profiling traffic --kernel NAME [--grid N] \
        --fetch CSV --write CSV --copy-fetch CSV --copy-write CSV \
        --copy-bytes BYTES --cells CELLS --cmd "..."
        HBM bytes per dispatch of NAME from FETCH_SIZE / WRITE_SIZE counter
        runs (KiB per dispatch), each scaled by what the same counter reads
        for a plain device copy of a known size. Printed as JSON.

    python -m paper_2102_12978_amd.profiling table --row KERNEL[@GRID][=CELLS] ... \
        --fetch CSV --write CSV --copy-fetch CSV --copy-write CSV --copy-bytes BYTES \
        --cmd "..."
        The same for several kernels, as a markdown table.

    python -m paper_2102_12978_amd.profiling sum --name NAME --row KERNEL[@GRID] ... \
        --fetch CSV --write CSV --copy-fetch CSV --copy-write CSV --copy-bytes BYTES \
        --cells CELLS --cmd "..."
        Bytes of a group of launches made together (their sum), as JSON.

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
    """Source file of a kernel (by the name the counters carry): the two- or
    three-step kernel, the one-step interior kernel, or the split frame
    kernels."""
    if "step2" in kernel:
        return os.path.join(CSRC, "kernels_step2.hip")
    if "step3" in kernel:
        return os.path.join(CSRC, "kernels_step3.hip")
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


def pass_spans(trace_csv, kernel, size):
    """Launch groups of `size` consecutive dispatches (by dispatch id) of the
    kernels whose full name contains `kernel`, such as the four concurrent
    tile-class launches of a two-step pass: per group, first start to last
    end (ms). Returns (count, mean, min, max)."""
    rows = [r for r in csv.DictReader(open(trace_csv)) if kernel in r["Kernel_Name"]]
    rows.sort(key=lambda r: int(r["Dispatch_Id"]))
    spans = []
    for i in range(0, len(rows) - size + 1, size):
        g = rows[i:i + size]
        t0 = min(int(r["Start_Timestamp"]) for r in g)
        t1 = max(int(r["End_Timestamp"]) for r in g)
        spans.append((t1 - t0) / 1e6)
    if not spans:
        raise SystemExit(f"no dispatches of a kernel named like {kernel!r} in {trace_csv}")
    return len(spans), sum(spans) / len(spans), min(spans), max(spans)


def _matches(row, kernel, grid):
    name = short_name(row["Kernel_Name"])
    return (kernel == name or kernel in row["Kernel_Name"]) and \
        (grid is None or int(row["Grid_Size"]) == grid)


def counter_per_dispatch(path, kernel, counter, grid=None):
    """Mean counter value (KiB) over the dispatches of kernel (its short name,
    or a substring of the full name), optionally only those of one grid size
    (work-items): a launch shape when several ran under one name."""
    vals = [float(r["Counter_Value"]) for r in csv.DictReader(open(path))
            if _matches(r, kernel, grid) and r["Counter_Name"].startswith(counter)]
    if not vals:
        raise SystemExit(f"no {counter} rows for a kernel named like {kernel!r}"
                         f"{'' if grid is None else f' with grid {grid}'} in {path}")
    return sum(vals) / len(vals), len(vals)


def largest_dispatch(path, counter):
    """Counter value (KiB) of the copy dispatches: the largest values in the file."""
    vals = sorted(float(r["Counter_Value"]) for r in csv.DictReader(open(path))
                  if r["Counter_Name"].startswith(counter))
    top = vals[-1]
    same = [v for v in vals if v > 0.9 * top]
    return sum(same) / len(same), len(same)


def traffic(a):
    f_kib, nf = counter_per_dispatch(a.fetch, a.kernel, "FETCH_SIZE", a.grid)
    w_kib, nw = counter_per_dispatch(a.write, a.kernel, "WRITE_SIZE", a.grid)
    cf_kib, _ = largest_dispatch(a.copy_fetch, "FETCH_SIZE")
    cw_kib, _ = largest_dispatch(a.copy_write, "WRITE_SIZE")
    f_scale = a.copy_bytes / (cf_kib * 1024.0)
    w_scale = a.copy_bytes / (cw_kib * 1024.0)
    read_b = f_kib * 1024.0 * f_scale
    write_b = w_kib * 1024.0 * w_scale
    return {
        "kernel": a.kernel,
        "grid_size": a.grid,
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


def traffic_table(a):
    """Markdown table of HBM bytes per dispatch for several kernels."""
    out = [f"Command: `{a.cmd}`", "",
           f"Copy calibration: a {a.copy_bytes}-byte device copy; FETCH_SIZE and WRITE_SIZE "
           "(KiB per dispatch) are scaled by the copy's bytes over what each counter reads "
           "for it.", "",
           "| kernel | grid | dispatches | read MB | write MB | cells | B/cell |",
           "|---|---|---|---|---|---|---|"]
    for spec in a.row:
        spec, _, cells = spec.partition("=")
        kernel, _, grid = spec.partition("@")
        b = argparse.Namespace(kernel=kernel, grid=int(grid) if grid else None, fetch=a.fetch,
                               write=a.write, copy_fetch=a.copy_fetch, copy_write=a.copy_write,
                               copy_bytes=a.copy_bytes, cells=int(cells) if cells else 0,
                               cmd=a.cmd)
        t = traffic(b)
        out.append(f"| {kernel} | {grid or 'all'} | {t['dispatches']['fetch']} | "
                   f"{t['read_bytes_per_launch'] / 1e6:.1f} | "
                   f"{t['write_bytes_per_launch'] / 1e6:.1f} | {cells or '-'} | "
                   f"{t['bytes_per_cell'] if t['bytes_per_cell'] else '-'} |")
    return "\n".join(out) + "\n"


def traffic_sum(a):
    """HBM bytes of one launch group (several kernels launched together, such
    as the four tile classes of a two-step pass): the per-dispatch bytes of
    each row, and their sum. JSON."""
    rows, rd, wr = [], 0.0, 0.0
    for spec in a.row:
        kernel, _, grid = spec.partition("@")
        b = argparse.Namespace(kernel=kernel, grid=int(grid) if grid else None, fetch=a.fetch,
                               write=a.write, copy_fetch=a.copy_fetch, copy_write=a.copy_write,
                               copy_bytes=a.copy_bytes, cells=0, cmd=a.cmd)
        t = traffic(b)
        rows.append({"kernel": kernel, "grid_size": b.grid, "dispatches": t["dispatches"],
                     "read_bytes": t["read_bytes_per_launch"],
                     "write_bytes": t["write_bytes_per_launch"]})
        rd += t["read_bytes_per_launch"]
        wr += t["write_bytes_per_launch"]
        scale = (t["fetch_scale"], t["write_scale"])
    return {
        "kernel": a.name,
        "kernel_sha256_16": kernel_sha256_16(source_of(a.row[0].partition("@")[0])),
        "command": a.cmd,
        "copy_bytes": a.copy_bytes,
        "fetch_scale": scale[0],
        "write_scale": scale[1],
        "launches": rows,
        "read_bytes_per_launch": round(rd),
        "write_bytes_per_launch": round(wr),
        "bytes_per_launch": round(rd + wr),
        "cells_per_launch": a.cells,
        "bytes_per_cell": round((rd + wr) / a.cells, 2) if a.cells else None,
        # the tile shape the counters were taken with (rows, z chunk)
        "tile": ({"rows": int(a.tile.split(",")[0]), "zchunk": int(a.tile.split(",")[1])}
                 if a.tile else None),
    }


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="what", required=True)
    s = sub.add_parser("stats")
    s.add_argument("csv")
    s.add_argument("--cmd", required=True)
    s.add_argument("--pass-trace", default=None, help="kernel_trace.csv for launch-group spans")
    s.add_argument("--pass-kernel", default="step2_kernel")
    s.add_argument("--pass-size", type=int, default=4)
    t = sub.add_parser("traffic")
    for k in ("kernel", "fetch", "write", "copy_fetch", "copy_write", "cmd"):
        t.add_argument("--" + k.replace("_", "-"), dest=k, required=True)
    t.add_argument("--copy-bytes", dest="copy_bytes", type=int, required=True)
    t.add_argument("--cells", type=int, default=0)
    t.add_argument("--grid", type=int, default=None, help="only dispatches of this grid size")
    m = sub.add_parser("table")
    for k in ("fetch", "write", "copy_fetch", "copy_write", "cmd"):
        m.add_argument("--" + k.replace("_", "-"), dest=k, required=True)
    m.add_argument("--copy-bytes", dest="copy_bytes", type=int, required=True)
    m.add_argument("--row", action="append", required=True,
                   help="KERNEL[@GRID][=CELLS]: one table row")
    g = sub.add_parser("sum")
    for k in ("name", "fetch", "write", "copy_fetch", "copy_write", "cmd"):
        g.add_argument("--" + k.replace("_", "-"), dest=k, required=True)
    g.add_argument("--copy-bytes", dest="copy_bytes", type=int, required=True)
    g.add_argument("--cells", type=int, default=0)
    g.add_argument("--row", action="append", required=True, help="KERNEL[@GRID]")
    g.add_argument("--tile", default=None, help="ROWS,ZCHUNK of the profiled launches")
    a = ap.parse_args(argv)
    if a.what == "sum":
        print(json.dumps(traffic_sum(a), indent=1))
        return
    if a.what == "stats":
        sys.stdout.write(stats_markdown(a.csv, a.cmd))
        if a.pass_trace:
            n, mean, lo, hi = pass_spans(a.pass_trace, a.pass_kernel, a.pass_size)
            sys.stdout.write(f"\nLaunch groups of {a.pass_size} `{a.pass_kernel}` dispatches "
                             f"(consecutive dispatch ids; first start to last end): {n} "
                             f"groups, mean {mean:.4f} ms, min {lo:.4f} ms, max {hi:.4f} ms.\n")
    elif a.what == "traffic":
        print(json.dumps(traffic(a), indent=1))
    else:
        sys.stdout.write(traffic_table(a))


if __name__ == "__main__":
    main()
