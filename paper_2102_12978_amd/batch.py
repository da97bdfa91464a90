"""Python handle around a batch of solver instances (include/fdtd.h,
fdtd_batch_*). Argument marshalling only."""
import ctypes
import math

from . import _lib as L
from . import workloads as W
from .solver import Solver, fit_periodic_z


class Batch:
    """Many independent Bessel-antenna problems advanced together.

    workloads: a list of Workload (grid, cone angle, order, annulus, CPML,
    ramp); each becomes one instance with its own z fit and antenna."""

    def __init__(self, workloads, stream=None, inject=True):
        self._lib = L.load()
        n = len(workloads)
        grids = (L.Grid * n)()
        injs = (L.Injector * n)()
        shapes = []
        for q, w in enumerate(workloads):
            nz, dz = fit_periodic_z(W.WAVELENGTH, w.theta, w.dx, w.nz_hint)
            npml = w.npml if w.bc == L.BC_CPML else 0
            grids[q] = L.Grid(nx=w.nx, ny=w.ny, nz=nz, dx=w.dx, dy=w.dx, dz=dz,
                              courant=w.courant, bc_xy=w.bc, cpml_cells=npml,
                              cpml_grade=w.grade, cpml_sigma_scale=w.sigma_scale,
                              cpml_kappa_max=w.kappa_max, cpml_alpha_max=w.alpha_max,
                              kernel=L.KERNEL_SPLIT, reserved=0, stream=None)
            kind, ra, rb = w.ramp_args
            injs[q] = L.Injector(wavelength=W.WAVELENGTH, theta=w.theta, order=w.order,
                                 ramp_kind=kind, e0=w.e0,
                                 r_outer=w.r_outer_cells * w.dx,
                                 thickness=w.thickness_cells * w.dx, axis_x=math.nan,
                                 axis_y=math.nan, ramp_a=ra, ramp_b=rb,
                                 n_sectors=0, polarization=w.polarization)
            shapes.append((w.nx, w.ny, nz, npml, w.dx, w.dx, dz))
        b = ctypes.c_void_p()
        rc = self._lib.fdtd_batch_create(n, grids, injs if inject else None, stream,
                                         ctypes.byref(b))
        if rc != L.OK:
            raise L.FdtdError(rc, self._lib.fdtd_batch_last_error(None).decode())
        self._b = b
        self.instances = [Solver._borrow(self._lib.fdtd_batch_instance(b, q), *shapes[q])
                          for q in range(n)]

    def _c(self, rc):
        if rc != L.OK:
            raise L.FdtdError(rc, self._lib.fdtd_batch_last_error(self._b).decode())

    def close(self):
        if getattr(self, "_b", None) is not None and self._b.value:
            for s in self.instances:
                s._ctx = None
            self._lib.fdtd_batch_destroy(self._b)
        self._b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __len__(self):
        return len(self.instances)

    def __getitem__(self, q):
        return self.instances[q]

    def step(self, n=1):
        self._c(self._lib.fdtd_batch_step(self._b, int(n)))

    def set_tile(self, cols, zchunk=0):
        self._c(self._lib.fdtd_batch_set_tile(self._b, int(cols), int(zchunk)))

    def set_kernel(self, kernel, rows=2):
        self._c(self._lib.fdtd_batch_set_kernel(self._b, int(kernel), int(rows)))

    def set_time_block(self, steps, rows=2, zchunk=16):
        self._c(self._lib.fdtd_batch_set_time_block(self._b, int(steps), int(rows), int(zchunk)))

    def set_graph_steps(self, steps):
        self._c(self._lib.fdtd_batch_set_graph_steps(self._b, int(steps)))

    def autotune(self, steps_per_trial=3):
        c = ctypes.c_int32()
        z = ctypes.c_int32()
        self._c(self._lib.fdtd_batch_autotune(self._b, int(steps_per_trial), ctypes.byref(c),
                                              ctypes.byref(z)))
        return c.value, z.value

    def info(self):
        inf = L.BatchInfo()
        self._c(self._lib.fdtd_batch_get_info(self._b, ctypes.byref(inf)))
        return inf
