"""Turn a shared workload description into oracle inputs (test side only)."""
import math

import numpy as np

from oracle import problem as P
from paper_2102_12978_amd import workloads as W


def oracle_grid(w: W.Workload, bc=None, nz=None, dz=None):
    if nz is None:
        nz, dz = P.fit_periodic_z(W.WAVELENGTH, w.theta, w.dx, w.nz_hint)
    bc = w.bc if bc is None else bc
    return P.Grid(w.nx, w.ny, nz, w.dx, w.dx, dz, w.courant, bc,
                  w.npml if bc == P.BC_CPML else 0, w.grade, w.sigma_scale,
                  w.kappa_max, w.alpha_max)


def oracle_injector(w: W.Workload, amp=None, phase=None, e0=None):
    kind, a, b = w.ramp_args
    return P.Injector(W.WAVELENGTH, w.theta, w.order, w.e0 if e0 is None else e0,
                      w.r_outer_cells * w.dx, w.thickness_cells * w.dx,
                      ramp_kind=kind, ramp_a=a, ramp_b=b,
                      sector_amp=amp, sector_phase=phase, polarization=w.polarization)
