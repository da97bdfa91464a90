"""Pure-PyTorch FP64 forward of the Bessel-antenna Yee scheme, differentiated
by torch.autograd: an independent reference for the hand-written adjoint.

TEST INFRASTRUCTURE (see ``oracle/__init__``).

The time stepping is written here again with torch tensor operations (it
does not call ``oracle.yee``), following the paper's scheme (§4): E update
with backward differences of H̃, CPML memories ψ ← bψ + cΔ updated before
use in the slabs, PEC-held tangential E on the x = 0 and y = 0 walls, the E
soft source at t_{n+1}; then the H update with forward differences of E and
the H source at t_{n+3/2}; z periodic. The problem set-up (z fit, CPML
tables, antenna points with their unweighted amplitudes Ã, sectors, time
factors) comes from ``oracle.problem``. The sector weights w_s = a_s e^{iφ_s}
are leaf tensors, so the intensity plane and any loss built on it carry
exact reverse-mode gradients with respect to (a_s, φ_s).

Parity: pinned by its forward against ``oracle.yee.run`` and its gradient
against ``oracle.adjoint.intensity_loss_grad`` (tests/test_torch_ref.py).
"""
import numpy as np
import torch

from . import problem as P

AX = {"x": 2, "y": 1, "z": 0}
E_COMPS = ("ex", "ey", "ez")
H_COMPS = ("hx", "hy", "hz")
# (target, differenced field, axis, sign, CPML memory) of the curl terms
E_CURL = (("ex", "hz", "y", 1.0, "exy"), ("ex", "hy", "z", -1.0, None),
          ("ey", "hx", "z", 1.0, None), ("ey", "hz", "x", -1.0, "eyx"),
          ("ez", "hy", "x", 1.0, "ezx"), ("ez", "hx", "y", -1.0, "ezy"))
H_CURL = (("hx", "ez", "y", -1.0, "hxy"), ("hx", "ey", "z", 1.0, None),
          ("hy", "ex", "z", -1.0, None), ("hy", "ez", "x", 1.0, "hyx"),
          ("hz", "ey", "x", -1.0, "hzx"), ("hz", "ex", "y", 1.0, "hzy"))


def _shift(u, axis, by, periodic):
    """u at index - by along axis (by = +1: the previous cell), zero filled
    outside a non-periodic axis."""
    a = AX[axis]
    if periodic or axis == "z":
        return torch.roll(u, by, dims=a)
    out = torch.zeros_like(u)
    n = u.shape[a]
    src = [slice(None)] * 3
    dst = [slice(None)] * 3
    if by == 1:
        src[a], dst[a] = slice(0, n - 1), slice(1, n)
    else:
        src[a], dst[a] = slice(1, n), slice(0, n - 1)
    out[tuple(dst)] = u[tuple(src)]
    return out


class TorchYee:
    def __init__(self, g: P.Grid, inj: P.Injector):
        g.validate()
        self.g = g
        self.periodic = g.periodic_xy
        self.s = dict(zip("xyz", g.s))
        cp = P.cpml_tables(g)
        t = lambda a: torch.as_tensor(np.asarray(a, dtype=np.float64))   # noqa: E731
        self.coef = {}
        for axis, at_e, tabs in (("x", True, cp.xe), ("x", False, cp.xh),
                                 ("y", True, cp.ye), ("y", False, cp.yh)):
            b, c, kinv = (t(v) for v in tabs)
            shape = (1, 1, -1) if axis == "x" else (1, -1, 1)
            self.coef[(axis, at_e)] = (b.reshape(shape), c.reshape(shape), kinv.reshape(shape))
        self.held = {}
        for comp in E_COMPS:
            m = np.zeros((g.ny, g.nx), dtype=bool)
            if not self.periodic:
                if comp in ("ey", "ez"):
                    m[:, 0] = True
                if comp in ("ex", "ez"):
                    m[0, :] = True
            self.held[comp] = torch.as_tensor(m)[None]
        self.ant = P.build_antenna(g, inj)

    def _part(self, f, psi, terms, comps, at_e):
        new_f, new_psi = dict(f), dict(psi)
        for comp in comps:
            acc = f[comp]
            for tgt, src, axis, sign, pname in terms:
                if tgt != comp:
                    continue
                u = f[src]
                if at_e:
                    d = u - _shift(u, axis, 1, self.periodic)
                else:
                    d = _shift(u, axis, -1, self.periodic) - u
                if pname is None:
                    acc = acc + sign * self.s[axis] * d
                else:
                    b, c, kinv = self.coef[(axis, at_e)]
                    p_new = b * psi[pname] + c * d
                    if at_e:
                        p_new = torch.where(self.held[comp], psi[pname], p_new)
                    new_psi[pname] = p_new
                    acc = acc + sign * self.s[axis] * (kinv * d + p_new)
            if at_e:
                acc = torch.where(self.held[comp], f[comp], acc)
            new_f[comp] = acc
        return new_f, new_psi

    def _source(self, f, comps, t, weights):
        tf = complex(P.time_factor(self.ant, t))
        out = dict(f)
        for comp in comps:
            jj, ii = self.ant.idx[comp]
            if jj.size == 0:
                continue
            base = torch.as_tensor(self.ant.base[comp])
            sec = self.ant.sector[comp]
            w = weights[torch.as_tensor(sec)] if sec is not None else torch.ones(
                len(jj), dtype=torch.complex128)
            zph = torch.as_tensor(self.ant.zphase[comp])
            val = torch.real(zph[:, None] * (w * base)[None, :] * tf)       # [nz, npts]
            u = f[comp].clone()
            u[:, torch.as_tensor(jj), torch.as_tensor(ii)] += val
            out[comp] = u
        return out

    def intensity(self, amp, phase, nsteps, plane, window_begin):
        """Window mean of E_y² on one plane; amp, phase: FP64 leaf tensors."""
        g = self.g
        shape = (g.nz, g.ny, g.nx)
        f = {c: torch.zeros(shape, dtype=torch.float64) for c in E_COMPS + H_COMPS}
        psi = {name: torch.zeros(shape, dtype=torch.float64)
               for name in ("exy", "eyx", "ezx", "ezy", "hxy", "hyx", "hzx", "hzy")}
        weights = amp.to(torch.complex128) * torch.exp(1j * phase.to(torch.complex128))
        acc = torch.zeros((g.ny, g.nx), dtype=torch.float64)
        count = 0
        for n in range(nsteps):
            f, psi = self._part(f, psi, E_CURL, E_COMPS, True)
            f = self._source(f, E_COMPS, (n + 1.0) * g.dt, weights)
            if n >= window_begin:
                acc = acc + f["ey"][plane] ** 2
                count += 1
            f, psi = self._part(f, psi, H_CURL, H_COMPS, False)
            f = self._source(f, H_COMPS, (n + 1.5) * g.dt, weights)
        return acc / max(count, 1)
