"""Yee leapfrog with CPML, periodic z and the Bessel-antenna soft source.

TEST INFRASTRUCTURE (see ``oracle/__init__``). Plain NumPy, FP64, whole-array
slicing; no blocking, fusion or reordering beyond the scheme itself.

The scheme (paper §4: standard second-order Yee scheme, CPML on the x and y
faces, periodic boundary along the optical axis z, soft source on the
antenna points), in normalised units with H̃ = η0 H:

  E^{n+1} = E^n + S ∇_h × H̃^{n+1/2}          then E += E_B(t_{n+1}) on the antenna
  H̃^{n+3/2} = H̃^{n+1/2} - S ∇_e × E^{n+1}     then H̃ += H_B(t_{n+3/2}) on the antenna

Arrays are indexed [k, j, i] (z, y, x). Staggered positions (Yee cell, §4):
E_x (i+½, j, k), E_y (i, j+½, k), E_z (i, j, k+½), H_x (i, j+½, k+½),
H_y (i+½, j, k+½), H_z (i+½, j+½, k). Differences of H are backward (they
land on E positions), differences of E are forward (they land on H positions).

x/y boundary: PEC walls at x = 0, x = nx (y likewise) behind the CPML; the
tangential E on the x = 0 / y = 0 walls is never updated and values beyond
the last cell are zero. Test mode ``BC_PERIODIC`` wraps x and y as well.

CPML (Roden–Gedney form): inside a slab every S_d Δ_d(·) term becomes
S_d [(1/κ) Δ_d(·) + ψ] with ψ ← b ψ + c Δ_d(·) updated just before use.

Parity: pinned by the exact discrete plane-wave eigenmode (numerical
dispersion closed form), the discrete energy invariant, div H̃ and div E
invariance, linearity of the source, CPML absorption against a larger box, and
the analytic Bessel profile within the paper's deviation band (§5).
"""
from dataclasses import dataclass, field

import numpy as np

from . import problem as P

AXIS = {"x": 2, "y": 1, "z": 0}
E_COMPS = ("ex", "ey", "ez")
H_COMPS = ("hx", "hy", "hz")

# (updated component, differenced component, axis, sign, ψ name or None)
E_TERMS = (
    ("ex", "hz", "y", +1, "exy"), ("ex", "hy", "z", -1, None),
    ("ey", "hx", "z", +1, None), ("ey", "hz", "x", -1, "eyx"),
    ("ez", "hy", "x", +1, "ezx"), ("ez", "hx", "y", -1, "ezy"),
)
H_TERMS = (
    ("hx", "ez", "y", -1, "hxy"), ("hx", "ey", "z", +1, None),
    ("hy", "ex", "z", -1, None), ("hy", "ez", "x", +1, "hyx"),
    ("hz", "ey", "x", -1, "hzx"), ("hz", "ex", "y", +1, "hzy"),
)
PSI_NAMES = ("exy", "eyx", "ezx", "ezy", "hxy", "hyx", "hzx", "hzy")


@dataclass
class State:
    f: dict = field(default_factory=dict)     # six field components
    psi: dict = field(default_factory=dict)   # eight CPML memories (full size)
    n: int = 0                                # completed steps

    def copy(self):
        return State({k: v.copy() for k, v in self.f.items()},
                     {k: v.copy() for k, v in self.psi.items()}, self.n)


def zero_state(g: P.Grid) -> State:
    shp = (g.nz, g.ny, g.nx)
    return State({c: np.zeros(shp) for c in E_COMPS + H_COMPS},
                 {p: np.zeros(shp) for p in PSI_NAMES}, 0)


def back_diff(u, axis, periodic):
    """u(i) - u(i-1); u(-1) = 0 unless periodic."""
    a = AXIS[axis]
    if periodic or axis == "z":
        return u - np.roll(u, 1, axis=a)
    d = u.copy()
    sl_hi = [slice(None)] * 3
    sl_lo = [slice(None)] * 3
    sl_hi[a] = slice(1, None)
    sl_lo[a] = slice(None, -1)
    d[tuple(sl_hi)] -= u[tuple(sl_lo)]
    return d


def fwd_diff(u, axis, periodic):
    """u(i+1) - u(i); u(n) = 0 unless periodic."""
    a = AXIS[axis]
    if periodic or axis == "z":
        return np.roll(u, -1, axis=a) - u
    d = -u
    sl_hi = [slice(None)] * 3
    sl_lo = [slice(None)] * 3
    sl_hi[a] = slice(1, None)
    sl_lo[a] = slice(None, -1)
    d[tuple(sl_lo)] += u[tuple(sl_hi)]
    return d


def cpml_coeffs(cp: P.Cpml, axis, at_e):
    """(b, c, 1/κ) shaped to broadcast over [k, j, i]."""
    if axis == "x":
        b, c, kinv = cp.xe if at_e else cp.xh
        return b[None, None, :], c[None, None, :], kinv[None, None, :]
    b, c, kinv = cp.ye if at_e else cp.yh
    return b[None, :, None], c[None, :, None], kinv[None, :, None]


def held_mask(g: P.Grid, comp):
    """Boolean [j, i] mask of E components held at zero by the PEC walls."""
    m = np.zeros((g.ny, g.nx), dtype=bool)
    if g.periodic_xy or comp not in E_COMPS:
        return m
    if comp in ("ey", "ez"):
        m[:, 0] = True
    if comp in ("ex", "ez"):
        m[0, :] = True
    return m


def _update(st: State, g: P.Grid, cp: P.Cpml, terms, comps, at_e):
    s = dict(zip("xyz", g.s))
    diff = back_diff if at_e else fwd_diff
    for comp in comps:
        old = st.f[comp]
        acc = old.copy()
        touched = []
        for tgt, src, axis, sign, psi in terms:
            if tgt != comp:
                continue
            d = diff(st.f[src], axis, g.periodic_xy)
            if psi is None:
                acc += sign * s[axis] * d
            else:
                b, c, kinv = cpml_coeffs(cp, axis, at_e)
                p_new = b * st.psi[psi] + c * d
                touched.append((psi, st.psi[psi], p_new))
                acc += sign * s[axis] * (kinv * d + p_new)
        held = held_mask(g, comp)
        if held.any():
            acc[:, held] = old[:, held]
        st.f[comp] = acc
        for psi, p_old, p_new in touched:
            if held.any():
                p_new[:, held] = p_old[:, held]
            st.psi[psi] = p_new


def update_e(st, g, cp):
    """E^{n+1} = E^n + S ∇_h × H̃^{n+1/2} with CPML (no source)."""
    _update(st, g, cp, E_TERMS, E_COMPS, at_e=True)


def update_h(st, g, cp):
    """H̃^{n+3/2} = H̃^{n+1/2} - S ∇_e × E^{n+1} with CPML (no source)."""
    _update(st, g, cp, H_TERMS, H_COMPS, at_e=False)


def source_values(ant: P.Antenna, comp, t):
    """Soft-source values Re{w Ã e^{iβ z_c} f(t) e^{-iω(t-T0)}} on the antenna
    points of one component, shape [nz, npts] (§4 soft source)."""
    tf = P.time_factor(ant, t)
    return np.real(ant.zphase[comp][:, None] * (ant.amp[comp][None, :] * tf))


def add_source(st: State, ant: P.Antenna, comps, t):
    for comp in comps:
        jj, ii = ant.idx[comp]
        if jj.size:
            st.f[comp][:, jj, ii] += source_values(ant, comp, t)


def step(st: State, g: P.Grid, cp: P.Cpml, ant: P.Antenna = None, want_energy=False):
    """One leapfrog step n -> n+1 (E then H), soft sources included.

    Returns W^{n+1} = Σ (E^{n+1})² + Σ H̃^{n+1/2} · H̃^{n+3/2} when asked.
    """
    n = st.n
    update_e(st, g, cp)
    if ant is not None:
        add_source(st, ant, E_COMPS, (n + 1.0) * g.dt)
    h_old = {c: st.f[c].copy() for c in H_COMPS} if want_energy else None
    update_h(st, g, cp)
    if ant is not None:
        add_source(st, ant, H_COMPS, (n + 1.5) * g.dt)
    st.n = n + 1
    if want_energy:
        w = sum(float(np.sum(st.f[c] ** 2)) for c in E_COMPS)
        w += sum(float(np.sum(h_old[c] * st.f[c])) for c in H_COMPS)
        return w
    return None


@dataclass
class Diag:
    plane: int = 0
    window_begin: int = 0       # first step index n whose E^{n+1} is averaged
    count: int = 0
    sums: dict = field(default_factory=dict)   # 'ex2','ey2','ez2' -> [ny, nx]
    energy: list = field(default_factory=list)
    planes: list = field(default_factory=list)  # recorded E_y planes
    volume: bool = False        # also average E_y² over every plane

    def mean(self, key):
        return self.sums[key] / max(self.count, 1)


def run(g: P.Grid, nsteps, ant=None, state=None, diag: Diag = None,
        want_energy=False, record_ey_plane=False):
    """Advance ``nsteps`` steps; accumulate the §5 diagnostics on the way.

    Plane diagnostics: mean over the window of E_x², E_y², E_z² on plane k_d at
    their native positions (the intensity of §5 read as ⟨E_y²⟩).
    """
    g.validate()
    cp = P.cpml_tables(g)
    st = zero_state(g) if state is None else state
    if diag is not None and not diag.sums:
        diag.sums = {k: np.zeros((g.ny, g.nx)) for k in ("ex2", "ey2", "ez2")}
        if diag.volume:
            diag.sums["ey2_vol"] = np.zeros((g.nz, g.ny, g.nx))
    for _ in range(nsteps):
        n = st.n
        w = step(st, g, cp, ant, want_energy)
        if want_energy and diag is not None:
            diag.energy.append(w)
        if diag is not None and n >= diag.window_begin:
            k = diag.plane
            for comp in E_COMPS:
                diag.sums[comp + "2"] += st.f[comp][k] ** 2
            if diag.volume:
                diag.sums["ey2_vol"] += st.f["ey"] ** 2
            diag.count += 1
            if record_ey_plane:
                diag.planes.append(st.f["ey"][k].copy())
    return st


def energy(st: State, h_prev: dict):
    """W = Σ E² + Σ H̃_prev · H̃ (discrete invariant of the lossless scheme)."""
    w = sum(float(np.sum(st.f[c] ** 2)) for c in E_COMPS)
    return w + sum(float(np.sum(h_prev[c] * st.f[c])) for c in H_COMPS)


def div_h(st: State, g: P.Grid):
    """Discrete divergence of H̃ at cell centres (forward differences)."""
    rx, ry, rz = 1.0, g.ry, g.rz
    p = g.periodic_xy
    return (fwd_diff(st.f["hx"], "x", p) / rx + fwd_diff(st.f["hy"], "y", p) / ry
            + fwd_diff(st.f["hz"], "z", p) / rz)


def div_e(st: State, g: P.Grid):
    """Discrete divergence of E at the nodes (backward differences)."""
    p = g.periodic_xy
    return (back_diff(st.f["ex"], "x", p) + back_diff(st.f["ey"], "y", p) / g.ry
            + back_diff(st.f["ez"], "z", p) / g.rz)
