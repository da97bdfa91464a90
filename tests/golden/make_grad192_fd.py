"""Writes grad192_fd_gradient.json: central finite differences (h = 1e-3) of the
192×192×61 intensity loss with respect to 8 sector amplitudes and 8 sector
phases, computed with the FP64 oracle only.

Problem: Δx = λ/20, θ = 12°, order 0, annulus R_B = 64Δx, δs = 2Δx, 16-cell
CPML, sin² ramp over 10 periods, 1500 steps, 256 sector weights drawn with
seed 2 (a = 1 + 0.05 N(0,1), then φ = 0.1 N(0,1)). Ī = mean of E_y² on the
middle plane over the last 5 periods (200 steps). Loss
L = mean over r < R_B − δs of (Ī − A J_0²(K r))², A = on-axis Ī of the run
with every weight equal to 1 (a constant). Probes: sectors 32 q + 5.

The scheme is linear in the source weights, so the E_y planes of a run with
one weight moved by ±h are the base run's planes plus the moved part times
that sector's response. Each sector's complex response V is taken from two
oracle runs with only that sector switched on (weight 1 and weight i);
every perturbed loss L(p ± h) is then evaluated in full from its planes and
differenced centrally. 18 oracle runs of 1500 steps in all.

    python tests/golden/make_grad192_fd.py [--procs 5]
"""
import argparse
import json
import math
import os
import sys
import time
from multiprocessing import Pool

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import fields as F          # noqa: E402
from oracle import problem as P         # noqa: E402
from oracle import yee as Y             # noqa: E402
from paper_2102_12978_amd import workloads as W   # noqa: E402

H = 1e-3
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "grad192_fd_gradient.json")


def setup():
    w = W.grad192()
    nz, dz = P.fit_periodic_z(W.WAVELENGTH, w.theta, w.dx, w.nz_hint)
    g = P.Grid(w.nx, w.ny, nz, w.dx, w.dx, dz, w.courant, P.BC_CPML, w.npml, w.grade,
               w.sigma_scale, w.kappa_max, w.alpha_max)
    return w, g


def window_planes(args):
    """E_y on the middle plane for every step of the window: [steps, ny, nx]."""
    amp, phase = args
    w, g = setup()
    inj = P.Injector(W.WAVELENGTH, w.theta, w.order, w.e0, w.r_outer_cells * w.dx,
                     w.thickness_cells * w.dx, ramp_kind=P.RAMP_SIN2, ramp_a=w.ramp_seconds,
                     sector_amp=np.asarray(amp), sector_phase=np.asarray(phase))
    ant = P.build_antenna(g, inj)
    d = Y.Diag(plane=g.nz // 2, window_begin=w.steps - w.window_steps)
    Y.run(g, w.steps, ant, diag=d, record_ey_plane=True)
    return np.array(d.planes)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--procs", type=int, default=5)
    a = ap.parse_args()
    w, g = setup()
    nsec = w.extra["sectors"]
    amp0, ph0 = W.sector_params(seed=2, sectors=nsec)
    sectors = W.fd_probe_sectors()
    jobs = [(np.ones(nsec), np.zeros(nsec)), (amp0, ph0)]
    for s in sectors:
        only = np.zeros(nsec)
        only[s] = 1.0
        jobs.append((only, np.zeros(nsec)))                 # weight 1  -> Re V
        jobs.append((only, np.where(only > 0, 0.5 * math.pi, 0.0)))   # weight i -> -Im V
    t0 = time.time()
    with Pool(a.procs) as pool:
        runs = pool.map(window_planes, jobs, chunksize=1)
    print(f"{len(jobs)} oracle runs in {time.time() - t0:.0f} s", flush=True)
    ny, nx = g.ny, g.nx
    jj, ii = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    r = np.hypot(ii - nx / 2.0, (jj + 0.5) * g.ry - ny * g.ry / 2.0)
    region = r < (w.r_outer_cells - w.thickness_cells)
    k = 2 * math.pi / w.ns
    j0sq = F.ey_mean_square(0, k, w.theta, 1.0, r) / (0.5 * math.cos(w.theta) ** 2)
    i_ref = np.mean(runs[0] ** 2, axis=0)
    A = 0.5 * (i_ref[ny // 2 - 1, nx // 2] + i_ref[ny // 2, nx // 2])
    target = A * j0sq
    base = runs[1]

    def loss(planes):
        ibar = np.mean(planes ** 2, axis=0)
        return float(np.mean((ibar[region] - target[region]) ** 2))

    fd_a, fd_p = [], []
    for q, s in enumerate(sectors):
        u1, u2 = runs[2 + 2 * q], runs[3 + 2 * q]      # Re V and -Im V
        a_s, p_s = amp0[s], ph0[s]

        def moved(da, dp):
            w_new = (a_s + da) * complex(math.cos(p_s + dp), math.sin(p_s + dp))
            dw = w_new - a_s * complex(math.cos(p_s), math.sin(p_s))
            return base + dw.real * u1 + dw.imag * u2    # Re{dw V}

        fd_a.append((loss(moved(H, 0.0)) - loss(moved(-H, 0.0))) / (2 * H))
        fd_p.append((loss(moved(0.0, H)) - loss(moved(0.0, -H))) / (2 * H))
    out = {
        "_recipe": "Central differences, h = 1e-3, of the 192² gradient workload's intensity loss; FP64 "
                   "oracle runs combined by linearity in the source weights. Written by "
                   "tests/golden/make_grad192_fd.py (oracle only).",
        "h": H, "sectors": sectors, "A_on_axis": float(A), "loss": loss(base),
        "grad_amp_fd": fd_a, "grad_phase_fd": fd_p,
        "grid": [g.nx, g.ny, g.nz], "steps": w.steps, "window_steps": w.window_steps,
    }
    json.dump(out, open(OUT, "w"), indent=1)
    print(json.dumps(out, indent=1))


if __name__ == "__main__":
    main()
