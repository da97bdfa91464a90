"""Comparison of a computed intensity plane with the analytic Bessel beam
(paper §5): the deviation χ at the lobe maxima inside the antenna.

The soft source couples an amplitude that is not E0, so one amplitude α is
fitted by least squares over the central lobes; then, at each lobe maximum
of the analytic profile along the ±x and ±y lines through the axis,
χ = | sqrt(⟨E_y²⟩/α) − sqrt(⟨E_y²⟩_ana) | / sqrt(⟨E_y²⟩_ana), the worst of the
four directions per lobe. Inputs are the solver's plane ⟨E_y²⟩ and the
library's analytic ½ E0² cos²θ J_m²(K r) at the same E_y positions
(fdtd_fluence / fdtd_analytic_ey2). Host-side post-processing only.
"""
import math

import numpy as np


def ey_radius(nx, ny, ry=1.0):
    """Offsets (x, y) and radius, in Δx, of the E_y positions (i, j+½) from
    the axis at the grid centre node (nx/2, ny/2)."""
    jj, ii = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    xs = ii - nx / 2.0
    ys = (jj + 0.5) * ry - ny * ry / 2.0
    return xs, ys, np.hypot(xs, ys)


def _line_maxima(ana, xs, ys, inside, direction):
    """Cells of the analytic plane's local maxima along one half-line from
    the axis, ordered by distance. Where two cells sit at the same distance
    along the line (the rows at y = ±½ for the x lines) the first stands for
    both."""
    dx, dy = direction
    along = xs * dx + ys * dy
    off = np.abs(xs * dy - ys * dx)
    sel = inside & (along >= 0) & (off <= 0.5 + 1e-9)
    idx = np.argwhere(sel)
    if len(idx) == 0:
        return []
    a_sel = along[sel]
    cells, seen = [], set()
    for o in np.argsort(a_sel, kind="stable"):
        key = round(float(a_sel[o]), 9)
        if key not in seen:
            seen.add(key)
            cells.append(tuple(idx[o]))
    vals = [ana[c] for c in cells]
    out = []
    for q in range(len(cells) - 1):   # the last cell may sit on a rising flank
        left = vals[q - 1] if q > 0 else -np.inf
        right = vals[q + 1]
        # the first cell counts as a maximum when the profile falls away from it
        if vals[q] > 0 and vals[q] >= left and vals[q] > right:
            out.append(cells[q])
    return out


def lobe_deviation(ey2, ana, kr, r_inner, ry=1.0, n_fit=3, margin=2.0):
    """χ per lobe (worst direction), α, and the lobe radii.

    ey2, ana: [ny, nx] planes; kr: transverse wavenumber K in 1/Δx;
    r_inner: inner antenna radius in Δx (lobes within r_inner - margin)."""
    ny, nx = ey2.shape
    xs, ys, r = ey_radius(nx, ny, ry)
    inside = r < r_inner - margin
    per_dir = [_line_maxima(ana, xs, ys, inside, d) for d in ((1, 0), (-1, 0), (0, 1), (0, -1))]
    nl = min(len(p) for p in per_dir)
    if nl == 0:
        return {"alpha": float("nan"), "radii": [], "chi": []}
    radii = [float(np.mean([r[p[q]] for p in per_dir])) for q in range(nl)]
    r_fit = radii[min(n_fit, nl) - 1] + 0.25 * 2 * math.pi / kr
    central = (r < r_inner) & (r < r_fit)
    alpha = float(np.sum(ey2[central] * ana[central]) / np.sum(ana[central] ** 2))
    chi = []
    for q in range(nl):
        worst = 0.0
        for p in per_dir:
            c = p[q]
            a = math.sqrt(ana[c])
            worst = max(worst, abs(math.sqrt(max(ey2[c], 0.0) / alpha) - a) / a)
        chi.append(worst)
    return {"alpha": alpha, "radii": radii, "chi": chi}
