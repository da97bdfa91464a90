"""Synthetic workloads and seeded inputs shared by the tests and the benchmark.

This module holds parameter values and random draws only; it contains none of
the method's arithmetic (no z fit, no CPML profile, no Bessel value). Both the
HIP solver and the CPU reference receive these plain numbers and derive
everything else on their own.

All configurations use λ = 800 nm, Courant number 0.5, E0 = 1, a sin² turn-on
ramp, CPML with polynomial grade 3, σ_max equal to the usual optimum
0.8 (g+1)/(η0 Δ), κ_max = 1 and a CFS pole α_max one tenth of the carrier
frequency (normalised α Δx/(ε0 c) = 0.1 · 2π/n_s).

The parameter sets follow the paper's workloads (§4, Table 1 and the sampling
rule; §5): a y-polarised order-m Bessel beam from a thin annulus, z-periodic
box of whole axial periods, CPML on x and y.
"""
import math
from dataclasses import dataclass, field, replace

import numpy as np

WAVELENGTH = 800e-9
C_LIGHT = 299792458.0
PERIOD = WAVELENGTH / C_LIGHT            # optical period, s

BC_CPML, BC_PEC, BC_PERIODIC = 0, 1, 2
RAMP_SIN2, RAMP_GAUSS, RAMP_CW = 0, 1, 2


@dataclass
class Workload:
    name: str
    nx: int
    ny: int
    nz_hint: int
    ns: float                  # cells per wavelength (Δx = λ/ns)
    theta_deg: float
    order: int
    r_outer_cells: float
    thickness_cells: float
    npml: int
    steps: int
    ramp_periods: float = 20.0
    courant: float = 0.5
    bc: int = BC_CPML
    e0: float = 1.0
    grade: float = 3.0
    sigma_scale: float = 1.0
    kappa_max: float = 1.0
    window_periods: float = 5.0
    ramp_kind: int = RAMP_SIN2
    polarization: int = 0              # potential axis (0 x, 1 y, 2 z) + 3 for TM
    pulse_t_fs: float = 0.0            # Gaussian envelope: T (fs)
    pulse_t0_fs: float = 0.0           # Gaussian envelope: peak time T0 (fs)
    extra: dict = field(default_factory=dict)

    @property
    def dx(self):
        return WAVELENGTH / self.ns

    @property
    def theta(self):
        return math.radians(self.theta_deg)

    @property
    def alpha_max(self):
        return 0.1 * 2.0 * math.pi / self.ns

    @property
    def ramp_seconds(self):
        return self.ramp_periods * PERIOD

    @property
    def ramp_args(self):
        """(kind, a, b) of the injector envelope in seconds: sin² turn-on
        (a = T_r) or Gaussian (a = T, b = T0)."""
        if self.ramp_kind == RAMP_GAUSS:
            return RAMP_GAUSS, self.pulse_t_fs * 1e-15, self.pulse_t0_fs * 1e-15
        return self.ramp_kind, self.ramp_seconds, 0.0

    @property
    def steps_per_period(self):
        return self.ns / self.courant

    @property
    def window_steps(self):
        return int(round(self.window_periods * self.steps_per_period))


def cube32():
    """32×32×32, Δx = λ/16, θ = 10°, m = 0, annulus 12Δx × 2Δx, 8-cell CPML, 200 steps."""
    return Workload("cube32_theta10_m0", 32, 32, 32, 16.0, 10.0, 0, 12.0, 2.0, 8, 200)


def grid256(order=0):
    """256×256×64 (z fitted), Δx = λ/20, θ = 15°, m = 0 or 1, annulus 100Δx, 2000 steps."""
    return Workload(f"grid256x256x64_theta15_m{order}", 256, 256, 64, 20.0, 15.0, order,
                    100.0, 2.0, 16, 2000)


def grid768():
    """768×768×256 (z fitted to 255), Δx = λ/24, θ = 20°, m = 2, annulus 320Δx, 1000 steps."""
    return Workload("grid768x768x256_theta20_m2", 768, 768, 256, 24.0, 20.0, 2, 320.0, 2.0,
                    16, 1000)


def batch64_instances(seed=1, count=64):
    """64 uneven instances: nx = ny ~ U{64..160}, nz_hint ~ U{48..64},
    θ ~ {5,10,15,20,25,30}°, m ~ U{0..3}; 8-cell CPML, R_B = 0.8 (nx/2 - 8) Δx."""
    rng = np.random.default_rng(seed)
    out = []
    for q in range(count):
        nx = int(rng.integers(64, 161))
        nzh = int(rng.integers(48, 65))
        th = float(rng.choice([5.0, 10.0, 15.0, 20.0, 25.0, 30.0]))
        m = int(rng.integers(0, 4))
        out.append(Workload(f"batch64_inst{q:02d}", nx, nx, nzh, 20.0, th, m,
                            0.8 * (nx / 2 - 8), 2.0, 8, 1000))
    return out


def batch_small(seed=3, count=5):
    """Small uneven instances for batch parity (the 64-instance batch recipe
    scaled down): nx = ny ~ U{40..72}, nz_hint ~ U{12..20}, θ ~ {10,15,20,25,30}°,
    m ~ U{0..3}; Δx = λ/16, 8-cell CPML, R_B = 0.8 (nx/2 - 8) Δx, 2-period
    ramp, 45 steps."""
    rng = np.random.default_rng(seed)
    out = []
    for q in range(count):
        nx = int(rng.integers(40, 73))
        nzh = int(rng.integers(12, 21))
        th = float(rng.choice([10.0, 15.0, 20.0, 25.0, 30.0]))
        m = int(rng.integers(0, 4))
        out.append(Workload(f"b_small{q}_{nx}_m{m}", nx, nx, nzh, 16.0, th, m,
                            0.8 * (nx / 2 - 8), 2.0, 8, 45, ramp_periods=2.0))
    return out


def grad192():
    """192×192×64 (z fitted), Δx = λ/20, θ = 12°, m = 0, annulus 64Δx, 1500 steps,
    checkpoints every 100 steps, 256 sector weights, 10-period ramp."""
    return Workload("grad192x192x64_theta12_m0", 192, 192, 64, 20.0, 12.0, 0, 64.0, 2.0,
                    16, 1500, ramp_periods=10.0,
                    extra={"checkpoint_every": 100, "sectors": 256})


def grad24():
    """24×24×(24 hint) copy of the 192² gradient workload for the autograd reference: Δx = λ/20,
    θ = 12°, m = 0, 4-cell CPML, R_B = 0.8 (12 - 4) Δx, δs = 2Δx, 300 steps,
    2.5-period ramp, window = last 5 periods, the same 256 seed-2 sector
    weights."""
    return Workload("grad24_theta12_m0", 24, 24, 24, 20.0, 12.0, 0, 6.4, 2.0, 4, 300,
                    ramp_periods=2.5, extra={"checkpoint_every": 100, "sectors": 256})


def sector_params(seed=2, sectors=256):
    """Initial sector amplitudes a = 1 + 0.05 N(0,1) and phases φ = 0.1 N(0,1)
    (amplitudes drawn first)."""
    rng = np.random.default_rng(seed)
    amp = 1.0 + 0.05 * rng.standard_normal(sectors)
    phase = 0.1 * rng.standard_normal(sectors)
    return amp, phase


def fd_probe_sectors():
    """The 16 finite-difference probes: amplitude and phase of sectors 32q + 5."""
    return [32 * q + 5 for q in range(8)]


def validation_run(order=0, n_perp=2, ns=16.0):
    """Paper-regime check (§4 Table 1 geometry scaled down): θ = 30°, n_s = 16
    (the paper's 20 on request), R_B = n_perp λ_xy, δs = 1 λ, 12-cell CPML,
    one axial period, 10-period ramp; the run lasts ramp + inward transit
    R_B/(c sin θ) + 6 periods."""
    th = 30.0
    lam_xy = ns / math.sin(math.radians(th))
    r_b = n_perp * lam_xy
    npml = 12
    n = int(2 * r_b) + 2 * npml
    transit = r_b / math.sin(math.radians(th))          # Δx units of time
    ramp_p = 10.0
    steps = int(round((ramp_p * ns + transit) / 0.5 + 6 * ns / 0.5))
    nz_hint = int(round(ns / math.cos(math.radians(th))))
    return Workload(f"v_theta30_m{order}_nperp{n_perp}_ns{int(ns)}", n, n, nz_hint, ns, th,
                    order, r_b, ns, npml, steps, ramp_periods=ramp_p)


def validation_v(order=0):
    """The validation run in the paper's regime (§4 Table 1 sampling rule,
    §5 band): θ = 25°, n_s = 20, N_perp = 2 (R_B = 2 λ_xy at the CPML
    interface), δs = 1 λ, 16-cell CPML, transverse points
    int(2 n_s N_perp / sin θ) + 2 N_PML = 221, z over two axial periods
    (44 cells), 20-period sin² ramp, 1700 steps (ramp 800 + inward transit
    R_B / (c sin θ) = 448 + a 200-step window + margin)."""
    th, ns, nperp, npml = 25.0, 20.0, 2, 16
    s = math.sin(math.radians(th))
    lam_xy = ns / s
    n = int(2 * ns * nperp / s) + 2 * npml
    nz_hint = int(round(2 * ns / math.cos(math.radians(th))))
    return Workload(f"v_theta25_m{order}_221", n, n, nz_hint, ns, th, order, nperp * lam_xy,
                    ns, npml, 1700)


# The paper's parameter sets (§4 Table 1): order m, cone angle θ (deg),
# antenna thickness δs (λ), N_parallel, N_perp.
TABLE1 = {
    "A": (0, 30.0, 1.0, 1, 4), "B": (1, 30.0, 1.0, 1, 4), "C": (2, 30.0, 1.0, 1, 4),
    "D": (0, 25.0, 1.0, 1, 4), "E": (0, 17.0, 1.0, 1, 4), "F": (0, 25.0, 2.0, 1, 4),
    "G": (0, 25.0, 3.0, 1, 4), "H": (0, 25.0, 1.0, 1, 3), "I": (0, 25.0, 1.0, 1, 2),
}
PULSE_T_FS, PULSE_T0_FS = 60.0, 180.0        # §5: T = 60 fs (100 fs FWHM), T0 = 180 fs
RUN_ABC_COMPARE_FS = 213.5                    # §5: snapshot time of runs A-C


def table1_run(name, ns=20, npml=6):
    """Run `name` of Table 1 (§4): n_s = 20 cells per λ, cubic cells, 6-cell
    CPML; transverse points int(2 n_s N_perp / sin θ) + 2 N_PML (the sampling
    rule of §4), outer radius R_B = N_perp λ_xy at the CPML interface,
    thickness δs; z periodic over 2 N_parallel axial periods (the z-fit
    replaces the rule's int() and z CPML cells); Gaussian envelope T = 60 fs,
    T0 = 180 fs (§5). The run lasts until the comparison time: 213.5 fs for
    runs A-C (§5), otherwise the whole optical period nearest to the peak
    time at the centre, T0 + R_B / (c sin θ)."""
    m, th, ds, npar, nperp = TABLE1[name]
    s = math.sin(math.radians(th))
    lam_xy = ns / s                                   # cells
    n = int(2 * ns * nperp / s) + 2 * npml
    nz_hint = int(round(2 * npar * ns / math.cos(math.radians(th))))
    if name in "ABC":
        t_cmp = RUN_ABC_COMPARE_FS * 1e-15
    else:
        t_peak = PULSE_T0_FS * 1e-15 + nperp * lam_xy * (WAVELENGTH / ns) / (C_LIGHT * s)
        t_cmp = round(t_peak / PERIOD) * PERIOD
    steps = int(round(t_cmp / PERIOD * ns / 0.5))
    return Workload(f"table1_{name}_m{m}_theta{th:g}_ds{ds:g}_nperp{nperp}", n, n, nz_hint,
                    float(ns), th, m, nperp * lam_xy, ds * ns, npml, steps,
                    ramp_kind=RAMP_GAUSS, pulse_t_fs=PULSE_T_FS, pulse_t0_fs=PULSE_T0_FS,
                    extra={"run": name, "compare_s": t_cmp})


def parity_gauss():
    """Gaussian-envelope parity case: 120×96×(20 hint), Δx = λ/14, θ = 25°,
    m = 1, R_B = 30Δx, δs = 4Δx, 10-cell CPML, T = 2 periods peaking at
    T0 = 3 periods, 84 steps (three periods)."""
    per_fs = PERIOD * 1e15
    return Workload("p_gauss_120x96x20_theta25_m1", 120, 96, 20, 14.0, 25.0, 1, 30.0, 4.0, 10,
                    84, ramp_kind=RAMP_GAUSS, pulse_t_fs=2 * per_fs, pulse_t0_fs=3 * per_fs)


def random_fields(shape, seed=0):
    """Six U(-1, 1) fields in the order Ex, Ey, Ez, Hx, Hy, Hz, each [nz, ny, nx]."""
    rng = np.random.default_rng(seed)
    return [rng.uniform(-1.0, 1.0, size=shape) for _ in range(6)]


def random_state_vectors(shape_f, shapes_psi, seed):
    """Random fields and CPML memories for transpose (dot-product) tests."""
    rng = np.random.default_rng(seed)
    f = [rng.standard_normal(shape_f) for _ in range(6)]
    p = [rng.standard_normal(s) for s in shapes_psi]
    return f, p


def parity_mid():
    """Several fused-kernel segments plus a frame: 300×150×(24 hint), 10-cell
    CPML, θ = 25°, m = 1, antenna of radius 60Δx crossing interior and frame,
    40 steps."""
    return Workload("p_300x150x24_theta25_m1", 300, 150, 24, 14.0, 25.0, 1, 60.0, 3.0, 10, 40,
                    ramp_periods=2.0)


def parity_thick():
    """A thick antenna filling whole tiles: 200×180×(16 hint), 10-cell CPML,
    θ = 25°, m = 2, Δx = λ/14, annulus from r = 40 to R_B = 78 cells (two
    cells short of the y CPML, reaching x- and y-boundary tiles), 30 steps."""
    return Workload("p_thick_200x180x16_theta25_m2", 200, 180, 16, 14.0, 25.0, 2, 78.0, 38.0, 10,
                    30, ramp_periods=2.0)


def parity_wide():
    """Seven fused segments (two workgroups of four x-adjacent wavefronts, the
    second one short): 540×80×(16 hint), 10-cell CPML, θ = 22°, m = 1,
    antenna of radius 30Δx across the workgroup boundary at x = 288, 40 steps."""
    return Workload("p_540x80x16_theta22_m1", 540, 80, 16, 14.0, 22.0, 1, 30.0, 3.0, 10, 40,
                    ramp_periods=2.0)


def parity_small():
    """Several-tile case with ragged edges: 100×72×(40 hint), source in the
    interior, 16-cell CPML, θ = 18°, m = 1, 60 steps."""
    return Workload("p_100x72x40_theta18_m1", 100, 72, 40, 14.0, 18.0, 1, 26.0, 3.0,
                    10, 60, ramp_periods=2.0)
