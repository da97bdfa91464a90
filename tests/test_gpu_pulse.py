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

Gates, from §5: χ below 7 % at every lobe maximum inside the antenna
(runs A-C: 0.01-7 %) and below 3 % on the three central lobes of the m = 0
runs A (two lobes for m = 1, 2: B, C); the thick antenna G below 3 % on its
central lobes (the paper: about 1.5 %); E_x far below E_y (§5: four orders).
The other runs are reported.
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

GATED = {"A": 3, "B": 2, "C": 2, "G": 3}   # run -> central lobes held below 3 %


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
    T, T0 = w.pulse_t_fs * 1e-15 / tunit, w.pulse_t0_fs * 1e-15 / tunit
    ru, inv = np.unique(r, return_inverse=True)
    prof = PU.ey_pulse_complex(w.order, w.theta, 2 * math.pi / w.ns, T, T0, ru, 0.0, 0.0, t,
                               nodes=48)
    return (prof[inv].reshape(r.shape) * np.exp(1j * w.order * np.arctan2(ys, xs))).real


@pytest.mark.parametrize("run", list("ABCDEFGHI"))
def test_table1_run_against_bessel_pulse(run):
    w = W.table1_run(run)
    amp2, ana2, ex0, ey0, info = _amplitude_planes(w)
    assert np.isfinite(amp2).all()
    res = A.lobe_deviation(amp2, ana2, info.kr, w.r_outer_cells - w.thickness_cells)
    chi = [100 * c for c in res["chi"]]
    ex_ratio = float(np.abs(ex0).max() / np.abs(ey0).max())
    print(f"  run {run}: m={w.order} theta={w.theta_deg:g} ds={w.thickness_cells / w.ns:g}λ "
          f"R_B={w.r_outer_cells:.1f}Δx t={w.extra['compare_s'] * 1e15:.1f} fs; "
          f"alpha={res['alpha']:.4g}; |Ex|max/|Ey|max={ex_ratio:.2e}; chi % at lobes: " +
          ", ".join(f"{c:.2f}" for c in chi), flush=True)
    assert res["alpha"] > 0 and len(chi) >= 2
    assert ex_ratio < 1e-3
    if run in GATED:
        assert max(chi[:GATED[run]]) < 3.0, chi
    if run in "ABC":
        assert max(chi) < 7.0, chi
