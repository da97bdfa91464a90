"""Shared helpers for the GPU parity tests: run a workload on both solvers."""
import numpy as np

from oracle import problem as P
from oracle import yee as Y
from paper_2102_12978_amd import _lib as L
from paper_2102_12978_amd import workloads as W
from paper_2102_12978_amd.solver import Solver
from tests import cases

COMPS = ("ex", "ey", "ez", "hx", "hy", "hz")
PSI = {L.PSI_EXY: "exy", L.PSI_EYX: "eyx", L.PSI_EZX: "ezx", L.PSI_EZY: "ezy",
       L.PSI_HXY: "hxy", L.PSI_HYX: "hyx", L.PSI_HZX: "hzx", L.PSI_HZY: "hzy"}


def rel_l2(gpu, ref):
    num = sum(float(np.sum((np.asarray(a, np.float64) - b) ** 2)) for a, b in zip(gpu, ref))
    den = sum(float(np.sum(np.asarray(b) ** 2)) for b in ref)
    return (num / den) ** 0.5 if den > 0 else num ** 0.5


def psi_slab(full, which, npml, nx, ny):
    """Oracle full-size ψ array -> the library's slab layout."""
    if which in (L.PSI_EYX, L.PSI_EZX, L.PSI_HYX, L.PSI_HZX):
        return np.concatenate([full[:, :, :npml], full[:, :, nx - npml:]], axis=2)
    return np.concatenate([full[:, :npml, :], full[:, ny - npml:, :]], axis=1)


def gpu_solver(w, kernel=L.KERNEL_FUSED, bc=None, rows=None, zchunk=0, inject=True, amp=None,
               phase=None):
    print(f"[gpu case] {w.name} kernel={kernel} bc={bc} rows={rows} zchunk={zchunk}",
          flush=True)
    s = Solver.from_workload(w, bc=bc, kernel=kernel)
    if rows is not None:
        s.set_tile(rows, zchunk)
    if inject:
        s.set_workload_injector(w, sector_amp=amp, sector_phase=phase)
    return s


def oracle_run(w, steps, bc=None, state=None, inject=True, diag=None, energy=False,
               amp=None, phase=None):
    g = cases.oracle_grid(w, bc=bc)
    ant = P.build_antenna(g, cases.oracle_injector(w, amp=amp, phase=phase)) if inject else None
    st = Y.run(g, steps, ant, state=state, diag=diag, want_energy=energy)
    return g, st


def random_start(w, bc, seed=0):
    """Seeded U(-1,1) fields (walls zeroed for PEC/CPML) for both solvers."""
    g = cases.oracle_grid(w, bc=bc)
    f = W.random_fields((g.nz, g.ny, g.nx), seed)
    st = Y.zero_state(g)
    for c, a in zip(COMPS, f):
        st.f[c] = a.astype(np.float32).astype(np.float64)
    if bc != P.BC_PERIODIC:
        for c in ("ex", "ey", "ez"):
            st.f[c][:, Y.held_mask(g, c)] = 0.0
    return g, st
