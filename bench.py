"""Benchmark of the Bessel-antenna FDTD step on one MI355X.

One step = one leapfrog step of the whole hot path on the 768×768×256
(z fitted to 255) workload: E update + CPML + antenna E source, H update +
CPML + antenna H source, mid-plane ⟨E_y²⟩ accumulation. Inputs are resident
in HBM before timing. Prints one JSON line.

    python bench.py [--gpus 1] [--steps 1000] [--warmup 20] [--no-cpu]
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, 8 TB/s
BYTES_PER_CELL = 48            # read + write six FP32 field components
CSRC = os.path.join(ROOT, "paper_2102_12978_amd", "csrc")
# interior kernels: source file, committed PMC summary (one per tile shape
# where the name has {rows} and {zchunk}), cell-updates per cell and launch
KERNELS = {
    "step2_pass": ("kernels_step2.hip",
                   "step2_pass_768x768x255_rows{rows}_z{zchunk}_traffic.json", 2),
    "step3_pass": ("kernels_step3.hip",
                   "step3_pass_768x768x255_rows{rows}_z{zchunk}_traffic.json", 3),
    "fused_interior": ("kernels_fused.hip", "fused_interior_768x768x255_traffic.json", 1),
}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_hash(name):
    src = os.path.join(CSRC, KERNELS[name][0])
    return hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]


def measured_traffic(name, tile=None):
    """HBM bytes per launch of an interior kernel from the committed
    rocprofv3 PMC summary of its tile shape (rows, z chunk), or None when
    there is none or it was taken on another source."""
    fname = KERNELS[name][1]
    if "{" in fname:
        if not tile:
            return None
        fname = fname.format(rows=tile[0], zchunk=tile[1])
    try:
        t = json.load(open(os.path.join(ROOT, "profiles", fname)))
    except (OSError, ValueError):
        return None
    if t.get("kernel_sha256_16") != kernel_hash(name):
        return None
    rec = t.get("tile")
    if rec and tile and (rec["rows"], rec["zchunk"]) != tuple(tile):
        return None
    return t.get("bytes_per_launch")


def _oracle_leg(args):
    """One CPU leg (worker process): `steps` FP64 oracle steps of workload
    `name` (instances of the batch one after another). Returns (cells x steps,
    seconds)."""
    name, steps, per_instance = args
    from oracle import problem as P
    from oracle import yee as Y
    from paper_2102_12978_amd import workloads as W
    ws = W.batch64_instances() if name == "batch64" else [getattr(W, name)()]
    if per_instance is not None:
        ws = ws[:per_instance]
    upd, secs = 0, 0.0
    for w in ws:
        nz, dz = P.fit_periodic_z(W.WAVELENGTH, w.theta, w.dx, w.nz_hint)
        g = P.Grid(w.nx, w.ny, nz, w.dx, w.dx, dz, w.courant, P.BC_CPML, w.npml, w.grade,
                   w.sigma_scale, w.kappa_max, w.alpha_max)
        kind, a, b = w.ramp_args
        inj = P.Injector(W.WAVELENGTH, w.theta, w.order, w.e0, w.r_outer_cells * w.dx,
                         w.thickness_cells * w.dx, ramp_kind=kind, ramp_a=a, ramp_b=b)
        ant = P.build_antenna(g, inj)
        cp = P.cpml_tables(g)
        st = Y.zero_state(g)
        n = min(steps, w.steps)
        t0 = time.perf_counter()
        for _ in range(n):
            Y.step(st, g, cp, ant)
        secs += time.perf_counter() - t0
        upd += g.nx * g.ny * g.nz * n
    return upd, secs


# (workload, steps, instances) of each CPU leg: the 768x768x255 benchmark
# grid for the headline figure, and bounded samples of the other workloads.
CPU_LEGS = {
    "grid768": ("grid768", 3, None),
    "cube32": ("cube32", 200, None),
    "grad192": ("grad192", 100, None),
    "batch64": ("batch64", 5, 8),
}
CPU_LEGS_FULL = {
    "grid768": ("grid768", 20, None),
    "cube32": ("cube32", 200, None),
    "grad192": ("grad192", 1500, None),
    "batch64": ("batch64", 50, None),
}


def cpu_baseline(full=False):
    """The FP64 NumPy oracle timed on this host, one single-threaded process
    per leg (legs in parallel): the 768x768x255 grid (value) and samples of
    the 32^3, 192x192x61 and batch workloads (legs)."""
    from concurrent.futures import ProcessPoolExecutor
    legs = CPU_LEGS_FULL if full else CPU_LEGS
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count()
    workers = max(1, min(len(legs), avail))
    from concurrent.futures import as_completed
    res = {}
    with ProcessPoolExecutor(max_workers=workers) as ex:
        futs = {ex.submit(_oracle_leg, v): k for k, v in legs.items()}
        for f in as_completed(futs):
            res[futs[f]] = f.result()
            log(f"[bench] CPU leg {futs[f]}: {res[futs[f]][1]:.1f} s")
    out = {}
    for k, (name, steps, inst) in legs.items():
        upd, secs = res[k]
        out[k] = {"value": round(upd / secs / 1e9, 5), "unit": "Gcell-updates/s",
                  "steps": steps, "instances": inst, "seconds": round(secs, 1)}
    head = out["grid768"]
    return {"value": head["value"], "unit": "Gcell-updates/s", "cores": 1,
            "cores_available": avail, "kind": "oracle",
            "sample": f"{legs['grid768'][1]} full steps of the 768x768x255 grid in FP64 "
                      f"NumPy, one single-threaded process ({head['seconds']} s); other legs "
                      f"ran at the same time, one process each ({workers} processes)",
            "legs": out}


def batch_measure(torch, stream, steps=1000, warmup=20, graph_steps=20, tile=None):
    """The 64-instance seed-1 sweep: autotuned work shape, 20-step graphs,
    mid-plane ⟨E_y²⟩ over the last 5 periods of each instance, then the
    per-instance deviation from the analytic beam (report only)."""
    from paper_2102_12978_amd import _lib as L
    from paper_2102_12978_amd import analysis as A
    from paper_2102_12978_amd import workloads as W
    from paper_2102_12978_amd.batch import Batch
    ws = W.batch64_instances()
    b = Batch(ws, stream=stream.cuda_stream)
    if tile:
        # a fixed two-step tile (profiling runs: the same launches every run)
        cols, zc = None, None
        b.set_time_block(2, tile[0], tile[1])
    else:
        cols, zc = b.autotune(10)
    b.set_graph_steps(graph_steps)
    total = warmup + steps
    for q, w in enumerate(ws):
        b[q].set_diagnostics(b[q].nz // 2, total - w.window_steps, L.DIAG_EY2)
    b.step(warmup)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    b.step(steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    inf = b.info()
    chis = []
    for q, w in enumerate(ws):
        s = b[q]
        res = A.lobe_deviation(s.fluence(L.DIAG_EY2).astype(float),
                               s.analytic_ey2().astype(float), s.info().kr,
                               w.r_outer_cells - w.thickness_cells)
        chis.append(max(res["chi"][:3]) if res["chi"] else float("nan"))
    b.close()
    value = inf.cells * steps / (ms * 1e-3) / 1e9
    seq = sequential_measure(torch, stream, ws, steps=200)
    achieved = BYTES_PER_CELL * inf.cells * steps / (ms * 1e-3) / 1e9
    finite = [c for c in chis if c == c]
    return {
        "workload": "64 instances (seed 1): nx=ny~U{64..160}, nz fitted from U{48..64}, "
                    "theta in {5..30}deg, order 0..3, dx=lambda/20, 8-cell CPML",
        "instances": inf.count, "cells": inf.cells, "steps": steps, "warmup": warmup,
        "value": round(value, 2), "unit": "Gcell-updates/s",
        "ms_per_step": round(ms / steps, 4), "tile_cols": cols, "tile_zchunk": zc,
        "steps_per_pass": inf.time_block,
        "two_step_tile": {"rows": inf.tb_rows, "zchunk": inf.tb_zchunk,
                          "work_items_per_pair": inf.tb_items} if inf.time_block == 2 else None,
        "graph_steps": inf.graph_steps, "work_items": inf.work_items,
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "bytes_per_cell": BYTES_PER_CELL},
        "single_instance_runs": seq,
        "batch_over_single": round(value / seq["value"], 3),
        "analytic_chi_central_lobes": {
            "median_percent": round(100 * float(sorted(finite)[len(finite) // 2]), 2)
            if finite else None,
            "max_percent": round(100 * max(finite), 2) if finite else None,
            "note": "report only: thin 2-cell antennas, window after 1020 steps"},
    }


def sequential_measure(torch, stream, ws, steps=200, warmup=20):
    """The same 64 problems stepped one after another as plain single-domain
    forwards (fused kernel, autotuned tile and frame), for comparison with
    the batched launch: summed step time of each instance."""
    from paper_2102_12978_amd import _lib as L
    from paper_2102_12978_amd.solver import Solver
    total_ms, cells = 0.0, 0
    for w in ws:
        s = Solver.from_workload(w, kernel=L.KERNEL_FUSED, stream=stream.cuda_stream)
        s.set_workload_injector(w)
        s.autotune(2)
        s.set_diagnostics(s.nz // 2, 0, L.DIAG_EY2)
        s.step(warmup)
        torch.cuda.synchronize()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        s.step(steps)
        ev1.record(stream)
        torch.cuda.synchronize()
        total_ms += ev0.elapsed_time(ev1)
        cells += s.nx * s.ny * s.nz
        s.close()
    return {"value": round(cells * steps / (total_ms * 1e-3) / 1e9, 2), "unit": "Gcell-updates/s",
            "steps_each": steps, "ms_per_step_all": round(total_ms / steps, 4)}


def shard_measure(torch, stream, parts, steps=1000, warmup=20, reps=5):
    """One GPU's share of the 768×768×255 grid cut into `parts` z-slabs on a
    ring: 768×768×round(255/parts) planes, z periodic over the slab (the wrap
    stands in for the neighbour exchange, so no exchange is timed), same
    Δx, Δz, CPML, antenna and diagnostics as the whole grid (the antenna's
    axial phase does not close over the slab; the work per step does not
    depend on it). Autotuned like the headline leg; median of `reps` runs."""
    from paper_2102_12978_amd import _lib as L
    from paper_2102_12978_amd import workloads as W
    from paper_2102_12978_amd.solver import Solver
    w = W.grid768()
    (nx, ny, nz_full, dx, dy, dz), kw = Solver.workload_grid_args(w)
    nz = int(round(nz_full / parts))
    s = Solver(nx, ny, nz, dx, dy, dz, kernel=L.KERNEL_FUSED, stream=stream.cuda_stream, **kw)
    s.set_workload_injector(w, allow_z_misfit=True)
    s.autotune(3)
    s.set_diagnostics(nz // 2, 0, L.DIAG_EY2)
    s.step(warmup)
    torch.cuda.synchronize()
    runs = []
    for _ in range(reps):
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        ev0.record(stream)
        s.step(steps)
        ev1.record(stream)
        torch.cuda.synchronize()
        runs.append(ev0.elapsed_time(ev1))
    ms = sorted(runs)[len(runs) // 2] / steps
    it = s.info()
    cells = nx * ny * nz
    s.close()
    # what a pass would need from its ring neighbours, in component-planes
    # (derived from the planes a z chunk reads beyond its ends, not
    # measured): one step, H_x, H_y of the plane under the slab and E_x,
    # E_y of the one over it; a two-step pass, all six components of the
    # plane under the slab and H_x, H_y of the one under that, and all six
    # of the plane over it and all but E_z of the next; a three-step pass,
    # one whole plane more on each side
    plane_bytes = nx * ny * 4
    below, above = {1: (2, 2), 2: (8, 11), 3: (14, 17)}[it.time_block]
    return {
        "workload": f"768x768x{nz}: one of {parts} z-slabs of the 768x768x255 grid, z periodic "
                    "over the slab in place of the neighbour exchange",
        "cells": cells, "steps": steps, "repetitions": reps,
        "ms_per_step": round(ms, 5),
        "value": round(cells / (ms * 1e-3) / 1e9, 2), "unit": "Gcell-updates/s",
        "steps_per_pass": it.time_block,
        "tile_rows": it.tb_rows if it.time_block >= 2 else it.tile_rows,
        "tile_zchunk": it.tb_zchunk if it.time_block >= 2 else it.tile_zchunk,
        "halo_bytes_per_pass_from_below": below * plane_bytes,
        "halo_bytes_per_pass_from_above": above * plane_bytes,
    }


def adjoint_measure(torch, stream, reps=3):
    """Gradient cost on the differentiable workload (192×192×61, 1500 steps,
    checkpoints every 100, 256 sector weights): forward with checkpoints +
    reverse sweep, against a plain 1500-step forward of the same problem."""
    import numpy as np
    from paper_2102_12978_amd import _lib as L
    from paper_2102_12978_amd import workloads as W
    from paper_2102_12978_amd.adjoint import SectorSensitivity, central_lobe_target, on_axis
    w = W.grad192()
    amp, ph = W.sector_params(seed=2, sectors=256)
    sens = SectorSensitivity(w, stream=stream.cuda_stream)
    s = sens.solver
    s.autotune(3)        # the tile and steps per pass used by both timings
    A = on_axis(sens.intensity(np.ones(256), np.zeros(256)).astype(np.float64))
    region, j0sq = central_lobe_target(sens)
    target = A * j0sq

    def plain():
        s.set_sector_weights(amp, ph)
        s.reset()
        s.set_diagnostics(sens.plane, sens.window_begin, L.DIAG_EY2)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.step(sens.steps)
        ib = s.fluence(L.DIAG_EY2)          # synchronises
        return time.perf_counter() - t0, ib

    def grad():
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ib = sens.intensity(amp, ph).astype(np.float64)
        dl = np.where(region, 2.0 * (ib - target) / np.count_nonzero(region), 0.0)
        ga, gp = sens.backward(dl)
        return time.perf_counter() - t0, ga, gp

    plain()
    grad()
    t_plain = min(plain()[0] for _ in range(reps))
    t_grad = min(grad()[0] for _ in range(reps))
    inf = sens.adj.info()
    tb = s.info().time_block
    cells = s.nx * s.ny * s.nz
    sens.close()
    return {
        "workload": "192x192x64 (z fitted to 61), dx=lambda/20, theta=12deg, order 0, "
                    "256 sector amplitude/phase weights (seed 2), 1500 steps, checkpoints "
                    "every 100, loss on the mid-plane window-mean E_y^2",
        "cells": cells, "steps": sens.steps,
        "forward_ms": round(1e3 * t_plain, 2),
        "forward_plus_adjoint_ms": round(1e3 * t_grad, 2),
        "grad_over_forward": round(t_grad / t_plain, 3),
        "checkpoints": inf.checkpoints, "recompute_steps": inf.recompute_steps,
        "adjoint_device_bytes": inf.device_bytes,
        "forward_steps_per_pass": tb,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--reps", type=int, default=5,
                    help="timed runs of --steps steps; the median one gives the value")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-full", action="store_true",
                    help="CPU legs at their full lengths (minutes)")
    ap.add_argument("--no-tune", action="store_true", help="keep the default tile shape")
    ap.add_argument("--rows", type=int, default=0, help="fix the tile rows (skips autotune)")
    ap.add_argument("--zchunk", type=int, default=0, help="z chunk with --rows")
    ap.add_argument("--time-block", type=int, default=0,
                    help="fix the steps per pass (1, 2 or 3)")
    ap.add_argument("--tb-rows", type=int, default=4, help="two-/three-step kernel rows")
    ap.add_argument("--tb-zchunk", type=int, default=32, help="two-/three-step kernel z chunk")
    ap.add_argument("--no-batch", action="store_true", help="skip the 64-instance batch")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the gradient timing")
    ap.add_argument("--adjoint-reps", type=int, default=3,
                    help="timed repetitions of each gradient-cost leg (minimum taken)")
    ap.add_argument("--sequential-classes", action="store_true",
                    help="run the two-step boundary launches after the interior one instead "
                         "of beside it (times each launch alone; a measurement run)")
    ap.add_argument("--batch-graph-steps", type=int, default=20,
                    help="steps per captured graph in the batch leg (0: eager launches)")
    ap.add_argument("--no-step", action="store_true",
                    help="skip the single-domain leg (profiling runs of the other legs)")
    ap.add_argument("--batch-tile", default=None,
                    help="ROWS,ZCHUNK: run the batch with the two-step kernel at this tile "
                         "instead of autotuning")
    ap.add_argument("--shard", type=int, default=8,
                    help="also time one GPU's z-slab share of the grid cut into this many "
                         "slabs (0: skip)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the solver "
              "steps one domain on one GPU and has no multi-GPU path", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2102_12978_amd import _lib as L
    from paper_2102_12978_amd import workloads as W
    from paper_2102_12978_amd.solver import Solver

    torch.cuda.init()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    if args.no_step:
        out = {"metric": "Gcell-updates/s (Yee E+H+CPML+inject)", "value": None,
               "note": "single-domain leg skipped (--no-step, a profiling run)"}
    else:
        w = W.grid768()
        s = Solver.from_workload(w, kernel=L.KERNEL_FUSED, stream=stream.cuda_stream)
        s.set_workload_injector(w)
        cells = s.nx * s.ny * s.nz
        log(f"[bench] {w.name}: {s.nx}x{s.ny}x{s.nz} = {cells / 1e6:.1f} M cells")
        if args.rows:
            s.set_tile(args.rows, args.zchunk)
        elif not args.no_tune:
            rows, zc = s.autotune(3)
            it = s.info()
            log(f"[bench] autotuned: one-step tile rows={rows} zchunk={zc}; steps per pass "
                f"{it.time_block} (multi-step tile rows={it.tb_rows} zchunk={it.tb_zchunk})")
        if args.time_block:
            s.set_time_block(args.time_block, args.tb_rows, args.tb_zchunk)
        if args.sequential_classes:
            s.set_concurrency(False)
        s.set_diagnostics(s.nz // 2, 0, L.DIAG_EY2)
        s.step(args.warmup)
        torch.cuda.synchronize()
        info = s.info()

        # the headline: args.reps timed runs of exactly args.steps steps each,
        # no per-launch events; value from the median run
        runs = []
        for _ in range(args.reps):
            ev0 = torch.cuda.Event(enable_timing=True)
            ev1 = torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            ev0.record(stream)
            s.step(args.steps)
            ev1.record(stream)
            torch.cuda.synchronize()
            runs.append(ev0.elapsed_time(ev1))
        total_ms = sorted(runs)[len(runs) // 2]
        ms_per_step = total_ms / args.steps
        value = cells * args.steps / (total_ms * 1e-3) / 1e9
        log(f"[bench] {args.reps} x {args.steps} steps: " +
            ", ".join(f"{r:.1f}" for r in runs) + f" ms -> median {value:.1f} Gcell/s")

        # per-kernel launch times: one more run of args.steps steps with a HIP
        # event pair around every launch, on the solver's stream
        s.profile(True)
        torch.cuda.synchronize()
        s.step(args.steps)
        torch.cuda.synchronize()
        prof = s.profile_read()
        s.profile(False)
        log(f"[bench] kernels: {prof}")

        roof = None
        tb = info.time_block
        if tb in (2, 3) and f"step{tb}_interior" in prof:
            # Two- and three-step passes: the four tile-class launches of a
            # pass run concurrently (the boundary classes on side streams)
            # and the interior launch spans the pass, so the unit is the
            # pass: 48 B per cell-update, tb updates of every cell, over the
            # pass time of the timed runs (events on the solver's stream,
            # which forks and joins the side streams; a remainder of steps
            # that is not a whole pass runs as a shorter one and is counted
            # at the same rate per step). The per-kernel figures come from one
            # more run of the same passes with an event pair around each
            # launch on its own stream.
            kname = f"step{tb}_pass"
            pass_ms = total_ms / (args.steps / tb)
            upd = tb * cells
            bytes_launch = BYTES_PER_CELL * upd
            achieved = bytes_launch / (pass_ms * 1e-3) / 1e9
            ki = prof[f"step{tb}_interior"]
            int_ms = ki[1] / ki[0]
            int_bytes = BYTES_PER_CELL * tb * info.interior_cells
            int_gbs = int_bytes / (int_ms * 1e-3) / 1e9
            roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                    "traffic": measured_traffic(kname, (info.tb_rows, info.tb_zchunk)),
                    "kernel": kname,
                    "launch": f"one {'two' if tb == 2 else 'three'}-step pass: interior, "
                              "x-boundary, y-boundary and corner tile launches, " +
                              ("one after another" if args.sequential_classes else "concurrent"),
                    "avg_launch_ms": round(pass_ms, 5), "cells_per_launch": cells,
                    "cell_updates_per_launch": upd,
                    "algorithmic_bytes_per_launch": bytes_launch,
                    # bytes a pass must move at least: each field read and
                    # written once, whatever the steps it advances
                    "min_bytes_per_launch": BYTES_PER_CELL * cells,
                    "launches_ms": {k: round(v[1] / v[0], 5) for k, v in prof.items()
                                    if k.startswith(f"step{tb}_")},
                    "interior_launch": {
                        "avg_ms": round(int_ms, 5), "cells": info.interior_cells,
                        "cell_updates": tb * info.interior_cells,
                        "achieved": round(int_gbs, 1),
                        "frac": round(int_gbs / HBM_PEAK_GBS, 4)}}
        else:
            # one step per launch: the dominant kernel is the interior kernel
            kname = next((k for k in KERNELS if k in prof and KERNELS[k][2] == 1), None)
            if kname:
                kin = prof[kname]
                avg_ms = kin[1] / kin[0]
                ncell = info.interior_cells
                bytes_launch = BYTES_PER_CELL * ncell
                achieved = bytes_launch / (avg_ms * 1e-3) / 1e9
                roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                        "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                        "traffic": measured_traffic(kname), "kernel": kname,
                        "avg_launch_ms": round(avg_ms, 5), "cells_per_launch": ncell,
                        "cell_updates_per_launch": ncell,
                        "algorithmic_bytes_per_launch": bytes_launch}
        step_gbs = BYTES_PER_CELL * cells / (ms_per_step * 1e-3) / 1e9
        if roof:
            # what a kernel with no arithmetic reaches on the same GPU (context for frac)
            from paper_2102_12978_amd.hbm_copy import stream_ceiling
            ceil = stream_ceiling(stream=stream.cuda_stream)
            roof["stream_ceiling"] = ceil
            roof["frac_of_copy"] = round(roof["achieved"] / ceil["copy_gbs"], 4)
            log(f"[bench] streaming probe: {ceil}")
        out = {
            "metric": "Gcell-updates/s (Yee E+H+CPML+inject)",
            "value": round(value, 2),
            "unit": "Gcell-updates/s",
            "n_gpus": 1,
            "steps": args.steps,
            "warmup": args.warmup,
            "repetitions": args.reps,
            "ms_per_run": [round(r, 3) for r in runs],
            "ms_per_step": round(ms_per_step, 4),
            "higher_is_better": True,
            "scaling": "weak",
            "vs_baseline": None,
            "dtype": "f32",
            "data": "synthetic",
            "config": {"workload": "768x768x256 (z fitted to 255) Yee grid, dx=lambda/24, "
                                   "theta=20deg, order-2 Bessel antenna R=320dx, 16-cell CPML",
                       "cells": cells, "steps_per_pass": info.time_block,
                       "classes_concurrent": not args.sequential_classes,
                       "tile_rows": info.tb_rows if info.time_block >= 2 else info.tile_rows,
                       "tile_zchunk": info.tb_zchunk if info.time_block >= 2 else info.tile_zchunk},
            "step_hbm_fraction": round(step_gbs / HBM_PEAK_GBS, 4),
            "kernels_ms": {k: round(v[1] / v[0], 5) for k, v in prof.items()},
            "roofline": roof,
        }
        s.close()
    if args.shard > 1 and not args.no_step:
        log(f"[bench] z-slab share of {args.shard} ...")
        out["shard"] = shard_measure(torch, stream, args.shard)
        log(f"[bench] shard: {out['shard']}")
    if not args.no_batch:
        log("[bench] 64-instance batch ...")
        tile = tuple(int(v) for v in args.batch_tile.split(",")) if args.batch_tile else None
        out["batch"] = batch_measure(torch, stream, graph_steps=args.batch_graph_steps,
                                     tile=tile)
        log(f"[bench] batch: {out['batch']['value']} Gcell/s")
    if not args.no_adjoint:
        log("[bench] adjoint gradient cost ...")
        out["adjoint"] = adjoint_measure(torch, stream, max(1, args.adjoint_reps))
        log(f"[bench] adjoint: {out['adjoint']}")
    if not args.no_cpu:
        log("[bench] CPU oracle baseline ...")
        out["cpu_baseline"] = cpu_baseline(args.cpu_full)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
