"""Gradients of an intensity loss with respect to the antenna's sector
weights (include/fdtd.h, fdtd_adjoint_*), and the torch.autograd.Function
that exposes them. Argument marshalling only: the forward steps, the
checkpoints, the recomputation and the transposed steps run in the library.

    sens = SectorSensitivity(workload, checkpoint_every=100)
    I = SectorIntensity.apply(amp, phase, sens)     # [ny, nx] window mean of E_y²
    loss = ((I - target)[region] ** 2).mean()
    loss.backward()                                 # amp.grad, phase.grad
"""
import ctypes
import math

import numpy as np
import torch

from . import _lib as L
from . import workloads as W
from .solver import Solver, _fptr


class Adjoint:
    """fdtd_adjoint attached to a Solver (which it borrows)."""

    def __init__(self, solver: Solver, checkpoint_every=100):
        self.solver = solver
        self._lib = L.load()
        a = ctypes.c_void_p()
        rc = self._lib.fdtd_adjoint_create(solver._ctx, int(checkpoint_every), ctypes.byref(a))
        if rc != L.OK:
            raise L.FdtdError(rc, self._lib.fdtd_adjoint_last_error(None).decode())
        self._a = a

    def _c(self, rc):
        if rc != L.OK:
            raise L.FdtdError(rc, self._lib.fdtd_adjoint_last_error(self._a).decode())

    def close(self):
        if getattr(self, "_a", None) is not None and self._a.value:
            self._lib.fdtd_adjoint_destroy(self._a)
        self._a = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def forward(self, nsteps, plane, window_begin):
        self._c(self._lib.fdtd_adjoint_forward(self._a, int(nsteps), int(plane),
                                               int(window_begin)))

    def backward(self, dl_di, n_sectors):
        g = np.ascontiguousarray(dl_di, dtype=np.float32)
        ga = np.zeros(n_sectors)
        gp = np.zeros(n_sectors)
        self._c(self._lib.fdtd_adjoint_backward(self._a, _fptr(g), g.size, int(n_sectors),
                                                ga.ctypes.data_as(L.c_double_p),
                                                gp.ctypes.data_as(L.c_double_p)))
        return ga, gp

    def correlation(self):
        """Per-point G as complex [slot, component]."""
        n = self.info().antenna_columns
        out = np.zeros((n, 6, 2))
        self._c(self._lib.fdtd_adjoint_source_correlation(
            self._a, out.ctypes.data_as(L.c_double_p), out.size))
        return out[..., 0] + 1j * out[..., 1]

    def info(self):
        inf = L.AdjointInfo()
        self._c(self._lib.fdtd_adjoint_get_info(self._a, ctypes.byref(inf)))
        return inf

    def transpose(self, nsteps):
        """Source-free transposed steps on the λ state as it is."""
        self._c(self._lib.fdtd_adjoint_transpose(self._a, int(nsteps)))

    def get_state(self, which):
        out = np.empty(self.solver.state_shape(which), dtype=np.float32)
        self._c(self._lib.fdtd_adjoint_get_state(self._a, which, _fptr(out), out.size))
        return out

    def set_state(self, which, arr):
        a = np.ascontiguousarray(arr, dtype=np.float32)
        if a.shape != self.solver.state_shape(which):
            raise ValueError(f"shape {a.shape} != {self.solver.state_shape(which)}")
        self._c(self._lib.fdtd_adjoint_set_state(self._a, which, _fptr(a), a.size))


class SectorSensitivity:
    """A forward solver with an adjoint attached, for a workload whose antenna
    carries per-sector weights (workload.extra['sectors'])."""

    def __init__(self, w: W.Workload, checkpoint_every=None, n_sectors=None, stream=None,
                 plane=None, window_begin=None, steps=None, kernel=L.KERNEL_FUSED,
                 dev_fields=None):
        self.w = w
        self.n_sectors = n_sectors or w.extra.get("sectors", 256)
        self.every = checkpoint_every or w.extra.get("checkpoint_every", 100)
        self.steps = steps or w.steps
        self.window_begin = self.steps - w.window_steps if window_begin is None else window_begin
        self.solver = Solver.from_workload(w, kernel=kernel, stream=stream,
                                           dev_fields=dev_fields)
        ones = np.ones(self.n_sectors)
        self.solver.set_workload_injector(w, sector_amp=ones, sector_phase=0 * ones)
        self.plane = self.solver.nz // 2 if plane is None else plane
        self.adj = Adjoint(self.solver, self.every)

    def close(self):
        if getattr(self, "adj", None) is not None:
            self.adj.close()
            self.adj = None
        if getattr(self, "solver", None) is not None:
            self.solver.close()
            self.solver = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def intensity(self, amp, phase):
        """Forward run with checkpoints; returns Ī [ny, nx] (float32)."""
        self.solver.set_sector_weights(np.asarray(amp, np.float64),
                                       np.asarray(phase, np.float64))
        self.adj.forward(self.steps, self.plane, self.window_begin)
        return self.solver.fluence(L.DIAG_EY2)

    def forward_runs(self):
        """Number of forward runs so far (identifies the checkpoints held)."""
        return self.adj.info().forward_runs

    def backward(self, dl_di):
        return self.adj.backward(dl_di, self.n_sectors)

    def backward_of(self, run, amp, phase, dl_di):
        """Backward for the forward run `run` with weights (amp, phase): when
        another forward ran since (a second graph on the same sensitivity) or
        the weights were changed, the checkpoints belong to other weights, so
        that forward is run again first."""
        if self.forward_runs() != run:
            self.intensity(amp, phase)
        try:
            return self.backward(dl_di)
        except L.FdtdError as e:
            if e.code != L.ESTATE:
                raise
            self.intensity(amp, phase)
            return self.backward(dl_di)


class SectorIntensity(torch.autograd.Function):
    """(a_s, φ_s) -> Ī: the window-mean E_y² plane of the forward run.
    Backward is the library's adjoint sweep."""

    @staticmethod
    def forward(ctx, amp, phase, sens):
        a = amp.detach().cpu().double().numpy().copy()
        p = phase.detach().cpu().double().numpy().copy()
        ibar = sens.intensity(a, p)
        ctx.sens = sens
        ctx.dev = amp.device
        ctx.weights = (a, p)
        ctx.run = sens.forward_runs()
        return torch.from_numpy(ibar.astype(np.float64)).to(amp.device)

    @staticmethod
    def backward(ctx, grad_i):
        a, p = ctx.weights
        ga, gp = ctx.sens.backward_of(ctx.run, a, p, grad_i.detach().cpu().numpy())
        return (torch.from_numpy(ga).to(ctx.dev), torch.from_numpy(gp).to(ctx.dev), None)


def central_lobe_target(sens):
    """Config-4 loss pieces (both from the library): the region r < R_B - δs
    and J_0²(K r) at the E_y positions, from the analytic plane
    ½ E0² cos²θ J_0²(K r) divided by ½ E0² cos²θ."""
    w = sens.w
    ana = sens.solver.analytic_ey2().astype(np.float64)
    j0sq = ana / (0.5 * w.e0 ** 2 * math.cos(w.theta) ** 2)
    ny, nx = ana.shape
    jj, ii = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    r = np.hypot(ii - nx / 2.0, jj + 0.5 - ny / 2.0)
    region = r < (w.r_outer_cells - w.thickness_cells)
    return region, j0sq


def on_axis(ibar):
    """Mean of the two E_y positions next to the axis (y = ±½ at x = nx/2)."""
    ny, nx = ibar.shape
    return 0.5 * (float(ibar[ny // 2 - 1, nx // 2]) + float(ibar[ny // 2, nx // 2]))
