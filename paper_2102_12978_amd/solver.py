"""Python handle around one solver context of the HIP library.

Argument marshalling only: every step, table and reduction runs in the
library (include/fdtd.h). Field and plane arrays come back as NumPy float32
arrays indexed [z][y][x].
"""
import ctypes
import math

import numpy as np

from . import _lib as L
from . import workloads as W


def _check(lib, ctx, rc):
    if rc != L.OK:
        msg = lib.fdtd_last_error(ctx)
        raise L.FdtdError(rc, msg.decode() if msg else "")


def fit_periodic_z(wavelength, theta, dx, nz_hint):
    lib = L.load()
    nz = ctypes.c_int32()
    dz = ctypes.c_double()
    rc = lib.fdtd_fit_periodic_z(wavelength, theta, dx, int(nz_hint), ctypes.byref(nz),
                                 ctypes.byref(dz))
    if rc != L.OK:
        raise L.FdtdError(rc, "fdtd_fit_periodic_z rejected its arguments")
    return nz.value, dz.value


def _fptr(a):
    return a.ctypes.data_as(L.c_float_p)


def _grid(nx, ny, nz, dx, dy, dz, courant, bc, cpml_cells, grade, sigma_scale, kappa_max,
          alpha_max, kernel, stream):
    return L.Grid(nx=nx, ny=ny, nz=nz, dx=dx, dy=dy, dz=dz, courant=courant, bc_xy=bc,
                  cpml_cells=cpml_cells, cpml_grade=grade, cpml_sigma_scale=sigma_scale,
                  cpml_kappa_max=kappa_max, cpml_alpha_max=alpha_max, kernel=kernel,
                  reserved=0, stream=stream)


def field_layout(nx, ny, nz, dx, dy, dz, courant=0.5, bc=L.BC_CPML, cpml_cells=0, grade=3.0,
                 sigma_scale=1.0, kappa_max=1.0, alpha_max=0.0):
    """(pitch, floats per parity) of the device field layout (fdtd_field_layout)."""
    lib = L.load()
    g = _grid(nx, ny, nz, dx, dy, dz, courant, bc, cpml_cells, grade, sigma_scale, kappa_max,
              alpha_max, L.KERNEL_AUTO, None)
    pitch = ctypes.c_int32()
    n = ctypes.c_int64()
    rc = lib.fdtd_field_layout(ctypes.byref(g), ctypes.byref(pitch), ctypes.byref(n))
    if rc != L.OK:
        raise L.FdtdError(rc, "fdtd_field_layout rejected the grid")
    return pitch.value, n.value


def antenna_points(w: W.Workload, n_sectors=0, bc=None):
    """Source points the library installs for workload w (fdtd_antenna_points;
    pure host call): int32 array [npoints, 4] of (component, i, j, sector),
    sector -1 without sector weights."""
    lib = L.load()
    nz, dz = fit_periodic_z(W.WAVELENGTH, w.theta, w.dx, w.nz_hint)
    bc = w.bc if bc is None else bc
    g = _grid(w.nx, w.ny, nz, w.dx, w.dx, dz, w.courant, bc,
              w.npml if bc == L.BC_CPML else 0, w.grade, w.sigma_scale, w.kappa_max,
              w.alpha_max, L.KERNEL_AUTO, None)
    kind, a, b = w.ramp_args
    ones = np.ones(max(1, n_sectors))
    zeros = np.zeros(max(1, n_sectors))
    inj = L.Injector(wavelength=W.WAVELENGTH, theta=w.theta, order=w.order, ramp_kind=kind,
                     e0=w.e0, r_outer=w.r_outer_cells * w.dx,
                     thickness=w.thickness_cells * w.dx, axis_x=math.nan, axis_y=math.nan,
                     ramp_a=a, ramp_b=b, n_sectors=n_sectors, polarization=w.polarization,
                     sector_amp=ones.ctypes.data_as(L.c_double_p),
                     sector_phase=zeros.ctypes.data_as(L.c_double_p), flags=0)
    count = ctypes.c_int64()
    rc = lib.fdtd_antenna_points(ctypes.byref(g), ctypes.byref(inj), None, 0,
                                 ctypes.byref(count))
    out = np.zeros((max(1, count.value), 4), dtype=np.int32)
    rc = lib.fdtd_antenna_points(ctypes.byref(g), ctypes.byref(inj),
                                 out.ctypes.data_as(L._I32P), count.value, ctypes.byref(count))
    if rc != L.OK:
        raise L.FdtdError(rc, "fdtd_antenna_points rejected its arguments")
    return out[:count.value]


class Solver:
    """dev_fields: None (the library allocates the fields) or the device
    addresses of two caller-owned parity buffers laid out as field_layout()
    says (fdtd_create_ext); the caller keeps them alive while the solver
    exists."""

    def __init__(self, nx, ny, nz, dx, dy, dz, courant=0.5, bc=L.BC_CPML, cpml_cells=0,
                 grade=3.0, sigma_scale=1.0, kappa_max=1.0, alpha_max=0.0,
                 kernel=L.KERNEL_AUTO, stream=None, dev_fields=None):
        self._lib = L.load()
        g = _grid(nx, ny, nz, dx, dy, dz, courant, bc, cpml_cells, grade, sigma_scale,
                  kappa_max, alpha_max, kernel, stream)
        ctx = ctypes.c_void_p()
        if dev_fields is None:
            rc = self._lib.fdtd_create(ctypes.byref(g), ctypes.byref(ctx))
        else:
            ptrs = (ctypes.c_void_p * 2)(int(dev_fields[0]), int(dev_fields[1]))
            rc = self._lib.fdtd_create_ext(ctypes.byref(g), ptrs, ctypes.byref(ctx))
        if rc != L.OK:
            raise L.FdtdError(rc, self._lib.fdtd_last_error(None).decode())
        self._ctx = ctx
        self._owned = True
        self.nx, self.ny, self.nz = nx, ny, nz
        self.npml = cpml_cells if bc == L.BC_CPML else 0
        self.dx, self.dy, self.dz = dx, dy, dz

    @classmethod
    def _borrow(cls, ctx, nx, ny, nz, npml, dx, dy, dz):
        """Handle of a context owned elsewhere (a batch instance); close()
        leaves it alone."""
        s = cls.__new__(cls)
        s._lib = L.load()
        s._ctx = ctypes.c_void_p(ctx)
        s._owned = False
        s.nx, s.ny, s.nz, s.npml = nx, ny, nz, npml
        s.dx, s.dy, s.dz = dx, dy, dz
        return s

    # -- construction from a shared workload description ------------------
    @staticmethod
    def workload_grid_args(w: W.Workload, bc=None):
        """Positional and keyword arguments of Solver / field_layout for a
        workload (z fitted to whole axial periods)."""
        nz, dz = fit_periodic_z(W.WAVELENGTH, w.theta, w.dx, w.nz_hint)
        bc = w.bc if bc is None else bc
        return ((w.nx, w.ny, nz, w.dx, w.dx, dz),
                dict(courant=w.courant, bc=bc, cpml_cells=w.npml if bc == L.BC_CPML else 0,
                     grade=w.grade, sigma_scale=w.sigma_scale, kappa_max=w.kappa_max,
                     alpha_max=w.alpha_max))

    @classmethod
    def from_workload(cls, w: W.Workload, bc=None, kernel=L.KERNEL_AUTO, stream=None,
                      dev_fields=None):
        args, kw = cls.workload_grid_args(w, bc)
        return cls(*args, kernel=kernel, stream=stream, dev_fields=dev_fields, **kw)

    def current_fields(self):
        """Device address of the parity buffer holding the current state."""
        ptr = ctypes.c_void_p()
        self._c(self._lib.fdtd_current_fields(self._ctx, ctypes.byref(ptr)))
        return ptr.value or 0

    def set_workload_injector(self, w: W.Workload, sector_amp=None, sector_phase=None,
                              allow_z_misfit=False):
        kind, a, b = w.ramp_args
        self.set_injector(W.WAVELENGTH, w.theta, w.order, w.e0, w.r_outer_cells * w.dx,
                          w.thickness_cells * w.dx, ramp_kind=kind, ramp_a=a, ramp_b=b,
                          sector_amp=sector_amp, sector_phase=sector_phase,
                          polarization=w.polarization, allow_z_misfit=allow_z_misfit)

    # -- API --------------------------------------------------------------
    def close(self):
        if getattr(self, "_ctx", None) is not None and self._ctx.value and self._owned:
            self._lib.fdtd_destroy(self._ctx)
        self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def _c(self, rc):
        _check(self._lib, self._ctx, rc)

    def set_injector(self, wavelength, theta, order, e0, r_outer, thickness,
                     ramp_kind=L.RAMP_SIN2, ramp_a=0.0, ramp_b=0.0, axis_x=math.nan,
                     axis_y=math.nan, sector_amp=None, sector_phase=None,
                     polarization=L.POL_X_TE, allow_z_misfit=False):
        inj = L.Injector(wavelength=wavelength, theta=theta, order=order, ramp_kind=ramp_kind,
                         e0=e0, r_outer=r_outer, thickness=thickness, axis_x=axis_x,
                         axis_y=axis_y, ramp_a=ramp_a, ramp_b=ramp_b, n_sectors=0,
                         polarization=polarization,
                         flags=L.INJ_ALLOW_Z_MISFIT if allow_z_misfit else 0)
        keep = []
        if sector_amp is not None:
            a = np.ascontiguousarray(sector_amp, dtype=np.float64)
            p = np.ascontiguousarray(sector_phase, dtype=np.float64)
            keep = [a, p]
            inj.n_sectors = len(a)
            inj.sector_amp = a.ctypes.data_as(L.c_double_p)
            inj.sector_phase = p.ctypes.data_as(L.c_double_p)
        self._c(self._lib.fdtd_set_injector(self._ctx, ctypes.byref(inj)))
        del keep

    def clear_injector(self):
        self._c(self._lib.fdtd_set_injector(self._ctx, None))

    def set_sector_weights(self, amp, phase):
        a = np.ascontiguousarray(amp, dtype=np.float64)
        p = np.ascontiguousarray(phase, dtype=np.float64)
        self._c(self._lib.fdtd_set_sector_weights(self._ctx, len(a),
                                                  a.ctypes.data_as(L.c_double_p),
                                                  p.ctypes.data_as(L.c_double_p)))

    def set_diagnostics(self, plane=-1, window_begin=0, mask=0):
        self._c(self._lib.fdtd_set_diagnostics(self._ctx, int(plane), int(window_begin),
                                               int(mask)))

    def step(self, n=1):
        self._c(self._lib.fdtd_step(self._ctx, int(n)))

    def step_static(self, n=1):
        """fdtd_step_static: the same steps with no allocation in the call."""
        self._c(self._lib.fdtd_step_static(self._ctx, int(n)))

    def fluence(self, quantity=L.DIAG_EY2):
        out = np.empty((self.ny, self.nx), dtype=np.float32)
        self._c(self._lib.fdtd_fluence(self._ctx, quantity, _fptr(out), out.size))
        return out

    def fluence_count(self):
        c = ctypes.c_int64()
        self._c(self._lib.fdtd_fluence_count(self._ctx, ctypes.byref(c)))
        return c.value

    def energy(self):
        w = ctypes.c_double()
        self._c(self._lib.fdtd_energy(self._ctx, ctypes.byref(w)))
        return w.value

    def state_shape(self, which):
        if which <= L.HZ:
            return (self.nz, self.ny, self.nx)
        if which in (L.PSI_EYX, L.PSI_EZX, L.PSI_HYX, L.PSI_HZX):
            return (self.nz, self.ny, 2 * self.npml)
        return (self.nz, 2 * self.npml, self.nx)

    def get_state(self, which):
        out = np.empty(self.state_shape(which), dtype=np.float32)
        self._c(self._lib.fdtd_get_state(self._ctx, which, _fptr(out), out.size))
        return out

    def set_state(self, which, arr):
        a = np.ascontiguousarray(arr, dtype=np.float32)
        if a.shape != self.state_shape(which):
            raise ValueError(f"shape {a.shape} != {self.state_shape(which)}")
        self._c(self._lib.fdtd_set_state(self._ctx, which, _fptr(a), a.size))

    def fields(self):
        return [self.get_state(c) for c in range(6)]

    def reset(self):
        self._c(self._lib.fdtd_reset(self._ctx))

    def info(self):
        inf = L.Info()
        self._c(self._lib.fdtd_get_info(self._ctx, ctypes.byref(inf)))
        return inf

    def analytic_ey2(self):
        out = np.empty((self.ny, self.nx), dtype=np.float32)
        self._c(self._lib.fdtd_analytic_ey2(self._ctx, _fptr(out), out.size))
        return out

    def set_tile(self, rows, zchunk=0):
        self._c(self._lib.fdtd_set_tile(self._ctx, rows, zchunk))

    def set_frame(self, kind, xalign=32, rows=2):
        self._c(self._lib.fdtd_set_frame(self._ctx, int(kind), int(xalign), int(rows)))

    def set_time_block(self, steps, rows=4, zchunk=0):
        """Steps per pass over the fields: 1, 2 (the two-step kernel) or 3
        (the three-step kernel), with tiles of `rows` rows and z chunks of
        `zchunk` planes."""
        self._c(self._lib.fdtd_set_time_block(self._ctx, int(steps), int(rows), int(zchunk)))

    def set_concurrency(self, on=True):
        """fdtd_set_concurrency: boundary launches beside the interior (True)
        or one after another (False)."""
        self._c(self._lib.fdtd_set_concurrency(self._ctx, 1 if on else 0))

    def profile(self, on=True):
        self._c(self._lib.fdtd_profile_enable(self._ctx, 1 if on else 0))

    def profile_read(self):
        arr = (L.KernelProfile * 16)()
        n = ctypes.c_int32()
        self._c(self._lib.fdtd_profile_read(self._ctx, arr, 16, ctypes.byref(n)))
        return {arr[i].name.decode(): (arr[i].launches, arr[i].total_ms)
                for i in range(min(n.value, 16))}

    def autotune(self, steps_per_trial=5):
        r = ctypes.c_int32()
        z = ctypes.c_int32()
        self._c(self._lib.fdtd_autotune(self._ctx, steps_per_trial, ctypes.byref(r),
                                        ctypes.byref(z)))
        return r.value, z.value
