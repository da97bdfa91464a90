"""Oracle values of single z-columns of a large grid, from small windows.

After s steps a cell depends only on cells within s of it in x and y (each
half step couples nearest neighbours), so the oracle reproduces the column
(j, i) exactly from a window of half-width s + 1 cut out of the initial
state: fields, CPML memories, the CPML coefficient rows and the antenna
points of the window, all at their global indices. The window is stepped as
if it were periodic in x and y; the wrap corrupts only its outer shell,
which cannot reach the centre within s steps. z is taken whole (periodic).
Windows must stay clear of the x = 0 and y = 0 walls (no held components
inside).
"""
from dataclasses import replace

import numpy as np

from oracle import problem as P
from oracle import yee as Y

X_SLAB = ("eyx", "ezx", "hyx", "hzx")


def _slab_col(i, n, npml):
    if i < npml:
        return i
    if i >= n - npml:
        return i - n + 2 * npml
    return -1


def psi_window(slab, name, g, xs, ys):
    """Full-size ψ window [nz, len(ys), len(xs)] from a slab-layout array."""
    out = np.zeros((g.nz, len(ys), len(xs)))
    if g.npml == 0:
        return out
    if name in X_SLAB:
        for a, i in enumerate(xs):
            c = _slab_col(i, g.nx, g.npml)
            if c >= 0:
                out[:, :, a] = slab[:, ys[0]:ys[-1] + 1, c]
    else:
        for b, j in enumerate(ys):
            r = _slab_col(j, g.ny, g.npml)
            if r >= 0:
                out[:, b, :] = slab[:, r, xs[0]:xs[-1] + 1]
    return out


def column(g, ant, fields, psi_slabs, i, j, s, n0=0):
    """Oracle E and H̃ columns at (j, i) after s steps from the given state.

    fields: comp -> [nz, ny, nx] arrays; psi_slabs: name -> slab arrays."""
    h = s + 1
    xs = list(range(i - h, i + h + 1))
    ys = list(range(j - h, j + h + 1))
    if xs[0] < 1 or ys[0] < 1 or xs[-1] >= g.nx or ys[-1] >= g.ny:
        raise ValueError("window must stay inside the grid and off the walls")
    gw = P.Grid(len(xs), len(ys), g.nz, g.dx, g.dy, g.dz, g.courant, P.BC_PERIODIC, 0,
                g.grade, g.sigma_scale, g.kappa_max, g.alpha_max)
    cp = P.cpml_tables(g)
    cpw = P.Cpml(xe=tuple(a[xs[0]:xs[-1] + 1] for a in cp.xe),
                 xh=tuple(a[xs[0]:xs[-1] + 1] for a in cp.xh),
                 ye=tuple(a[ys[0]:ys[-1] + 1] for a in cp.ye),
                 yh=tuple(a[ys[0]:ys[-1] + 1] for a in cp.yh))
    st = Y.zero_state(gw)
    for c in st.f:
        st.f[c] = np.asarray(fields[c][:, ys[0]:ys[-1] + 1, xs[0]:xs[-1] + 1], np.float64)
    for name in st.psi:
        st.psi[name] = psi_window(psi_slabs[name], name, g, xs, ys) if name in psi_slabs else \
            st.psi[name]
    st.n = n0
    antw = None
    if ant is not None:
        idx, amp, base, sector = {}, {}, {}, {}
        for comp, (jj, ii) in ant.idx.items():
            keep = (jj >= ys[0]) & (jj <= ys[-1]) & (ii >= xs[0]) & (ii <= xs[-1])
            idx[comp] = (jj[keep] - ys[0], ii[keep] - xs[0])
            amp[comp] = ant.amp[comp][keep]
            base[comp] = ant.base[comp][keep]
            sec = ant.sector.get(comp)
            sector[comp] = None if sec is None else sec[keep]
        antw = replace(ant, idx=idx, amp=amp, base=base, sector=sector)
    for _ in range(s):
        Y.step(st, gw, cpw, antw)
    return {c: st.f[c][:, h, h] for c in st.f}
