"""Problem set-up for the oracle: units, z fit, CPML profiles, antenna, time.

TEST INFRASTRUCTURE (see ``oracle/__init__``).

Normalised units: lengths in Δx, time in Δx/c, c = ε0 = μ0 = 1, H̃ = η0 H.
The Courant number S is c Δt / Δx, so Δt = S and the per-axis update factors
are S_x = S, S_y = S Δx/Δy, S_z = S Δx/Δz.

Readings of the paper taken here (each listed in the design notes):

* z periodicity (§4, sampling rule): the box holds p whole axial periods
  λ_z = λ / cos θ, p = max(1, round(nz_hint Δx / λ_z)), nz = round(p λ_z / Δx)
  and Δz = p λ_z / nz exactly; rounding is half-up on both solver sides.
* CPML (§4, the convolutional PML of Roden and Gedney): polynomial grading of
  order g over npml cells, σ_max = scale · 0.8 (g+1) Δx/Δ_d, κ grading to
  κ_max, α = α_max (1 - ρ), the recursive-convolution coefficients
  b = exp(-(σ/κ + α) Δt) and c = σ (b - 1)/(σ κ + κ² α); positions with zero
  depth carry b = c = 0 and 1/κ = 1 so ψ stays zero there.
* Antenna (§4, Fig. 3 and the soft source): a component location with
  R_B - δs < r ≤ R_B from the axis is a source point, tested at the
  component's own staggered position, for the whole periodic z length;
  tangential E on a PEC wall is never a source point.
* Time (§4, zeroth-order approximation): the injected value is
  Re{w Ã e^{iβz} f(t) e^{-iω(t - T0)}}; E is fed at t_{n+1} = (n+1)Δt and H
  at t_{n+3/2}, each at the time level of the field it is added to.

Parity: the z fit and the annulus membership are pinned by hand-computed
cases in the tests; CPML coefficients by the absorption test; the time factor
by the Gaussian-envelope FWHM the paper prints (§3.2).
"""
import math
from dataclasses import dataclass, field

import numpy as np

from . import fields

C_LIGHT = 299792458.0

BC_CPML, BC_PEC, BC_PERIODIC = 0, 1, 2
RAMP_SIN2, RAMP_GAUSS, RAMP_CW = 0, 1, 2


def round_half_up(x):
    return int(math.floor(x + 0.5))


def fit_periodic_z(wavelength, theta, dx, nz_hint):
    """Number of z cells and Δz for a box of whole axial periods (§4)."""
    lam_z = wavelength / math.cos(theta)
    p = max(1, round_half_up(nz_hint * dx / lam_z))
    nz = max(1, round_half_up(p * lam_z / dx))
    return nz, p * lam_z / nz


@dataclass
class Grid:
    nx: int
    ny: int
    nz: int
    dx: float
    dy: float
    dz: float
    courant: float = 0.5
    bc: int = BC_CPML
    npml: int = 0
    grade: float = 3.0
    sigma_scale: float = 1.0
    kappa_max: float = 1.0
    alpha_max: float = 0.0     # normalised: α Δx / (ε0 c)

    @property
    def ry(self):
        return self.dy / self.dx

    @property
    def rz(self):
        return self.dz / self.dx

    @property
    def dt(self):
        return self.courant

    @property
    def s(self):
        """(S_x, S_y, S_z)."""
        return (self.courant, self.courant / self.ry, self.courant / self.rz)

    @property
    def periodic_xy(self):
        return self.bc == BC_PERIODIC

    def validate(self):
        if min(self.nx, self.ny, self.nz) < 1:
            raise ValueError("grid sizes must be positive")
        sx, sy, sz = self.s
        if math.sqrt(sx * sx + sy * sy + sz * sz) >= 1.0:
            raise ValueError("Courant condition violated")
        if self.bc == BC_CPML:
            if self.npml < 1 or 2 * self.npml > min(self.nx, self.ny):
                raise ValueError("bad CPML thickness")
        elif self.npml != 0:
            raise ValueError("CPML cells given without CPML boundary")


def cpml_profile(n, npml, delta_ratio, grade, sigma_scale, kappa_max,
                 alpha_max, dt, half):
    """1-D CPML coefficient arrays (b, c, 1/κ) along one axis of n cells.

    ``half`` selects the positions i + 1/2 (derivatives of E, H positions)
    instead of i (derivatives of H, E positions). Depth ρ is measured from
    the interface x = npml (low face) or x = n - npml (high face), in cells.
    """
    b = np.zeros(n)
    c = np.zeros(n)
    kinv = np.ones(n)
    if npml <= 0:
        return b, c, kinv
    x = np.arange(n, dtype=np.float64) + (0.5 if half else 0.0)
    depth = np.maximum(np.maximum(npml - x, x - (n - npml)), 0.0)
    inside = depth > 0
    rho = depth[inside] / npml
    sigma_max = sigma_scale * 0.8 * (grade + 1.0) / delta_ratio
    sigma = sigma_max * rho ** grade
    kappa = 1.0 + (kappa_max - 1.0) * rho ** grade
    alpha = alpha_max * (1.0 - rho)
    bb = np.exp(-(sigma / kappa + alpha) * dt)
    den = sigma * kappa + kappa * kappa * alpha
    cc = np.where(den > 0, sigma * (bb - 1.0) / np.where(den > 0, den, 1.0), 0.0)
    b[inside] = bb
    c[inside] = cc
    kinv[inside] = 1.0 / kappa
    return b, c, kinv


@dataclass
class Cpml:
    """Per-axis CPML tables; ``xe`` = x derivatives at E positions (integer x),
    ``xh`` = x derivatives at H positions (half-integer x), same for y."""
    xe: tuple
    xh: tuple
    ye: tuple
    yh: tuple


def cpml_tables(g: Grid) -> Cpml:
    npml = g.npml if g.bc == BC_CPML else 0
    args = (g.grade, g.sigma_scale, g.kappa_max, g.alpha_max, g.dt)
    return Cpml(
        xe=cpml_profile(g.nx, npml, 1.0, *args, half=False),
        xh=cpml_profile(g.nx, npml, 1.0, *args, half=True),
        ye=cpml_profile(g.ny, npml, g.ry, *args, half=False),
        yh=cpml_profile(g.ny, npml, g.ry, *args, half=True),
    )


# Staggered positions (§4, soft-source indices; Yee cell): offsets in units
# of the cell along (x, y, z).
OFFSETS = {
    "ex": (0.5, 0.0, 0.0),
    "ey": (0.0, 0.5, 0.0),
    "ez": (0.0, 0.0, 0.5),
    "hx": (0.0, 0.5, 0.5),
    "hy": (0.5, 0.0, 0.5),
    "hz": (0.5, 0.5, 0.0),
}


@dataclass
class Injector:
    wavelength: float
    theta: float
    order: int
    e0: float
    r_outer: float
    thickness: float
    axis_x: float = float("nan")
    axis_y: float = float("nan")
    ramp_kind: int = RAMP_SIN2
    ramp_a: float = 0.0
    ramp_b: float = 0.0
    sector_amp: np.ndarray = None
    sector_phase: np.ndarray = None
    polarization: int = 0          # potential axis (0 x, 1 y, 2 z) + 3 for the TM pairing


@dataclass
class Antenna:
    """Source points per component: flat (j, i) index lists and the complex
    amplitude w·Ã at each, plus the per-plane phase e^{iβ z_c(k)}."""
    k: float
    beta: float
    omega: float
    idx: dict = field(default_factory=dict)      # comp -> (jj, ii)
    amp: dict = field(default_factory=dict)      # comp -> complex (npts,)
    base: dict = field(default_factory=dict)     # comp -> Ã without weight
    sector: dict = field(default_factory=dict)   # comp -> sector id or None
    zphase: dict = field(default_factory=dict)   # comp -> complex (nz,)
    t0: float = 0.0
    ramp_kind: int = RAMP_SIN2
    ramp_a: float = 0.0
    ramp_b: float = 0.0


def _held(comp, g: Grid, jj, ii):
    """Tangential E on the x = 0 or y = 0 PEC wall (never updated)."""
    m = np.zeros(jj.shape, dtype=bool)
    if g.periodic_xy:
        return m
    if comp in ("ey", "ez"):
        m |= ii == 0
    if comp in ("ex", "ez"):
        m |= jj == 0
    return m


def build_antenna(g: Grid, inj: Injector) -> Antenna:
    """Source point set and amplitudes (§4 antenna + §3.1 fields of the
    chosen potential and pairing; Π_x TE is the paper's y-polarised beam)."""
    assert inj.polarization in range(6)
    axis, tm = inj.polarization % 3, inj.polarization // 3
    ns = inj.wavelength / g.dx                   # cells per wavelength
    k = 2.0 * math.pi / ns
    ant = Antenna(k=k, beta=k * math.cos(inj.theta), omega=k)
    ax = (g.nx * 0.5) if math.isnan(inj.axis_x) else inj.axis_x / g.dx
    ay = (g.ny * 0.5 * g.ry) if math.isnan(inj.axis_y) else inj.axis_y / g.dx
    r_out = inj.r_outer / g.dx
    r_in = (inj.r_outer - inj.thickness) / g.dx
    nsec = 0 if inj.sector_amp is None else len(inj.sector_amp)
    jj_all, ii_all = np.meshgrid(np.arange(g.ny), np.arange(g.nx), indexing="ij")
    for ci, comp in enumerate(fields.COMPONENTS):
        ox, oy, oz = OFFSETS[comp]
        xc = (ii_all + ox) - ax
        yc = (jj_all + oy) * g.ry - ay
        r = np.hypot(xc, yc)
        sel = (r > r_in) & (r <= r_out)
        jj, ii = jj_all[sel], ii_all[sel]
        keep = ~_held(comp, g, jj, ii)
        jj, ii = jj[keep], ii[keep]
        xs, ys = (ii + ox) - ax, (jj + oy) * g.ry - ay
        amp = fields.amplitudes(axis, tm, inj.order, k, inj.theta, inj.e0, xs, ys)[ci]
        amp = np.asarray(amp, dtype=np.complex128).reshape(-1)
        ant.idx[comp] = (jj, ii)
        ant.base[comp] = amp
        if nsec:
            phi = np.mod(np.arctan2(ys, xs), 2.0 * math.pi)
            sec = np.minimum((phi * nsec / (2.0 * math.pi)).astype(np.int64), nsec - 1)
            w = np.asarray(inj.sector_amp)[sec] * np.exp(1j * np.asarray(inj.sector_phase)[sec])
            ant.sector[comp] = sec
            ant.amp[comp] = amp * w
        else:
            ant.sector[comp] = None
            ant.amp[comp] = amp
        zc = (np.arange(g.nz) + oz) * g.rz
        ant.zphase[comp] = np.exp(1j * ant.beta * zc)
    ant.ramp_kind = inj.ramp_kind
    tunit = C_LIGHT / g.dx                      # seconds -> Δx/c
    ant.ramp_a = inj.ramp_a * tunit
    ant.ramp_b = inj.ramp_b * tunit
    ant.t0 = ant.ramp_b if inj.ramp_kind == RAMP_GAUSS else 0.0
    return ant


def envelope(ant: Antenna, t):
    """Temporal envelope f(t) (§4 zeroth-order approximation; sin² ramp)."""
    t = np.asarray(t, dtype=np.float64)
    if ant.ramp_kind == RAMP_SIN2:
        tr = ant.ramp_a
        return np.where(t < tr, np.sin(0.5 * math.pi * t / tr) ** 2, 1.0)
    if ant.ramp_kind == RAMP_GAUSS:
        return np.exp(-((t - ant.ramp_b) / ant.ramp_a) ** 2)
    return np.ones_like(t)


def time_factor(ant: Antenna, t):
    """f(t) e^{-iω(t - T0)}."""
    return envelope(ant, t) * np.exp(-1j * ant.omega * (np.asarray(t) - ant.t0))
