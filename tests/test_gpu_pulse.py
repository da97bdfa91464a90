"""The paper's own validation (§4 Table 1, §5): Gaussian-pulse antenna runs
A-I on the HIP solver against the FP64 quadrature of the Bessel pulse (§3.2).

Each run injects the zeroth-order field (the CW beam times
f(t) = exp(-(t - T0)²/T²), T = 60 fs, T0 = 180 fs) from the annulus of
Table 1 and stops at the comparison time (213.5 fs for runs A-C, the whole
period nearest to the peak time at the centre otherwise). On the z = 0 plane
the local amplitude |E_y| = sqrt(E_y(t)² + E_y(t + period/4)²) is formed from
two snapshots a quarter period apart, on both sides, at the E_y positions.
One amplitude α (the soft source's coupling) is fitted over the central
lobes; χ = | |E_y|/√α - |E_y^ana| | / |E_y^ana| at the lobe maxima of the
analytic amplitude along the four half-lines through the axis inside the
inner radius (worst direction per lobe).

The analytic pulse peaks (its T0) when the antenna's pulse peaks on the
axis, T0 + R_B/(c sin θ): the zeroth-order antenna emits the envelope f(t)
on the annulus, and the energy reaches the axis along the cone after
R_B/(c sin θ).

Gates: |E_x|² below 1e-3 |E_y|² everywhere (§5: E_x is orders of magnitude
below E_y); χ below 3 % at the first two lobe maxima (§5: below 3 % on the
central lobes) for every run but E, the smallest cone angle, where §5 also
reports the lobes building up less well. Reported: χ at every lobe.

Also gated (except E): χ below 3 % at every lobe against a model of what the
zeroth-order antenna builds, J_m(K r) times the mean of the inward and
outward envelopes f(t - (R_mid ∓ r)/(c sin θ)) (R_mid the mid-radius of the
annulus). The antenna's envelope converges on the axis at c sin θ, while the
§3.2 pulse's envelope is nearly uniform across the antenna: that difference,
not the solver, is what makes χ against the pulse grow towards the antenna.
"""
import math

import numpy as np
import pytest

from oracle import pulse as PU
from paper_2102_12978_amd import _lib as L
from paper_2102_12978_amd import analysis as A
from paper_2102_12978_amd import workloads as W
from paper_2102_12978_amd.solver import Solver

pytestmark = pytest.mark.gpu

def _axis_peak(w):
    """Time (Δx/c) at which the antenna's pulse peaks on the axis."""
    tunit = w.dx / W.C_LIGHT
    return w.pulse_t0_fs * 1e-15 / tunit + w.r_outer_cells / math.sin(w.theta)


def _amplitude_planes(w):
    print(f"[gpu case] {w.name}: {w.nx}x{w.ny}, {w.steps} steps", flush=True)
    s = Solver.from_workload(w, kernel=L.KERNEL_FUSED)
    s.set_workload_injector(w)
    q = int(round(w.steps_per_period / 4))
    s.step(w.steps)
    ey0 = s.get_state(L.EY)[0].astype(np.float64)
    ex0 = s.get_state(L.EX)[0].astype(np.float64)
    s.step(q)
    ey1 = s.get_state(L.EY)[0].astype(np.float64)
    info = s.info()
    s.close()
    a0 = _analytic_plane(w, w.steps * w.courant)
    a1 = _analytic_plane(w, (w.steps + q) * w.courant)
    return ey0 ** 2 + ey1 ** 2, a0 ** 2 + a1 ** 2, ex0, ey0, info


def _analytic_plane(w, t):
    """Quadrature E_y at the E_y positions (i, j + 1/2) of the z = 0 plane at
    time t (Δx/c). The formula depends on the azimuth only through e^{imφ},
    so the integral is taken once per distinct radius (at φ = 0)."""
    xs, ys, r = A.ey_radius(w.nx, w.ny)
    tunit = w.dx / W.C_LIGHT
    T, T0 = w.pulse_t_fs * 1e-15 / tunit, _axis_peak(w)
    ru, inv = np.unique(r, return_inverse=True)
    prof = PU.ey_pulse_complex(w.order, w.theta, 2 * math.pi / w.ns, T, T0, ru, 0.0, 0.0, t,
                               nodes=48)
    return (prof[inv].reshape(r.shape) * np.exp(1j * w.order * np.arctan2(ys, xs))).real


@pytest.mark.parametrize("run", list("ABCDEFGHI"))
def test_table1_run_against_bessel_pulse(run):
    w = W.table1_run(run)
    amp2, ana2, ex0, ey0, info = _amplitude_planes(w)
    assert np.isfinite(amp2).all()
    r_in = w.r_outer_cells - w.thickness_cells
    res = A.lobe_deviation(amp2, ana2, info.kr, r_in)
    chi = [100 * c for c in res["chi"]]
    model = A.lobe_deviation(amp2, _model_amp2(w, info.kr), info.kr, r_in)
    ex_ratio = float((ex0 ** 2).max() / (ey0 ** 2).max())
    print(f"  run {run}: m={w.order} theta={w.theta_deg:g} ds={w.thickness_cells / w.ns:g}λ "
          f"R_B={w.r_outer_cells:.1f}Δx t={w.extra['compare_s'] * 1e15:.1f} fs; "
          f"alpha={res['alpha']:.4g}; max Ex²/max Ey²={ex_ratio:.2e}; chi % at lobes: " +
          ", ".join(f"{c:.2f}" for c in chi) + "; against the envelope model: " +
          ", ".join(f"{100 * c:.2f}" for c in model["chi"]), flush=True)
    assert res["alpha"] > 0 and len(chi) >= 2
    assert ex_ratio < 1e-3
    if run != "E":
        assert max(chi[:2]) < 3.0, chi
        assert max(model["chi"]) < 0.03, model["chi"]


def _model_amp2(w, kr):
    """Squared amplitude of the zeroth-order antenna's beam at the two
    snapshot times: J_m(K r)² times the squared mean of the inward and
    outward envelopes (Gaussian f of the §4 antenna) at each radius."""
    xs, ys, r = A.ey_radius(w.nx, w.ny)
    from scipy.special import jv
    tunit = w.dx / W.C_LIGHT
    T, T0 = w.pulse_t_fs * 1e-15 / tunit, w.pulse_t0_fs * 1e-15 / tunit
    r_mid = w.r_outer_cells - 0.5 * w.thickness_cells
    s = math.sin(w.theta)
    q = int(round(w.steps_per_period / 4))
    out = np.zeros_like(r)
    for n in (w.steps, w.steps + q):
        t = n * w.courant
        env = 0.5 * (np.exp(-((t - T0 - (r_mid - r) / s) / T) ** 2) +
                     np.exp(-((t - T0 - (r_mid + r) / s) / T) ** 2))
        out += 0.5 * (jv(w.order, kr * r) * env) ** 2
    return out
