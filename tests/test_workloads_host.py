"""The workload recipes against the paper's parameter sets and sampling rule.

The run boxes, antenna radii and run lengths below are worked out by hand
from §4 (Table 1 and the sampling rule that follows it) and §5 (the Gaussian
envelope and the comparison times), so a slip in a recipe (a sin for a cos,
N_par for N_perp, a dropped CPML term) fails here on the CPU before any GPU
run uses it.
"""
import json
import math
import os

import pytest

from oracle import problem as P
from paper_2102_12978_amd import workloads as W

HERE = os.path.dirname(__file__)
GOLD = json.load(open(os.path.join(HERE, "golden", "paper_values.json")))

# run: (N_xy, z planes, outer radius in cells, steps to the comparison time)
#  N_xy = int(2 n_s N_perp / sin θ) + 2 N_PML with n_s = 20, N_PML = 6;
#  z: 2 N_par axial periods λ/cos θ at Δx = λ/20, rounded to whole cells;
#  R_B = N_perp λ/sin θ; steps = comparison time / (Δt = Δx / 2c).
#  A-C compare at 213.5 fs (80.01 periods); the others at the whole period
#  nearest 180 fs + R_B/(c sin θ): θ = 25°, N_perp 4: 67.45 + 22.39 -> 90;
#  θ = 17°: 67.45 + 46.79 -> 114; N_perp 3: 67.45 + 16.80 -> 84;
#  N_perp 2: 67.45 + 11.20 -> 79 periods.
EXPECTED = {
    "A": (332, 46, 160.0, 3200), "B": (332, 46, 160.0, 3200), "C": (332, 46, 160.0, 3200),
    "D": (390, 44, 189.29, 3600), "E": (559, 42, 273.62, 4560),
    "F": (390, 44, 189.29, 3600), "G": (390, 44, 189.29, 3600),
    "H": (295, 44, 141.97, 3360), "I": (201, 44, 94.65, 3160),
}


def test_table1_parameter_sets_are_the_printed_ones():
    gold = GOLD["table1"]["runs"]
    assert sorted(W.TABLE1) == sorted(gold)
    for name, (m, th, ds, npar, nperp) in W.TABLE1.items():
        g = gold[name]
        assert (m, th, ds, npar, nperp) == (g["m"], g["theta_deg"], g["ds_lambda"], g["n_par"],
                                            g["n_perp"]), name


@pytest.mark.parametrize("name", sorted(EXPECTED))
def test_table1_run_box_follows_sampling_rule(name):
    n_xy, nz, r_b, steps = EXPECTED[name]
    w = W.table1_run(name)
    m, th, ds, npar, nperp = W.TABLE1[name]
    assert w.ns == GOLD["table1"]["n_s"] and w.npml == GOLD["table1"]["n_pml"]
    assert (w.nx, w.ny) == (n_xy, n_xy)
    assert w.order == m and w.theta_deg == th
    assert w.r_outer_cells == pytest.approx(r_b, abs=0.01)
    assert w.thickness_cells == ds * w.ns
    # the antenna's outer edge sits on the CPML interface: the width inside
    # the CPML is 2 R_B cut to whole cells
    assert 0.0 <= 2 * w.r_outer_cells - (w.nx - 2 * w.npml) < 1.0
    assert w.steps == steps
    assert w.ramp_kind == W.RAMP_GAUSS
    assert (w.pulse_t_fs, w.pulse_t0_fs) == (60.0, 180.0)
    nz_fit, dz = P.fit_periodic_z(W.WAVELENGTH, w.theta, w.dx, w.nz_hint)
    assert nz_fit == nz
    # two whole axial periods per N_par, the cells cubic to within the
    # rounding of the box to whole cells
    lam_z = W.WAVELENGTH / math.cos(w.theta)
    assert nz_fit * dz == pytest.approx(2 * npar * lam_z, rel=1e-12)
    assert abs(dz / w.dx - 1.0) <= 0.5 / nz


def test_table1_comparison_times():
    # §5 compares runs A-C at 213.5 fs; the recipe keeps that time exactly
    for name in "ABC":
        assert W.table1_run(name).extra["compare_s"] == pytest.approx(213.5e-15, rel=1e-12)
    # the others end on a whole optical period
    for name in "DEFGHI":
        t = W.table1_run(name).extra["compare_s"] / W.PERIOD
        assert t == pytest.approx(round(t), abs=1e-9)


def test_gaussian_envelope_matches_printed_fwhm():
    # the amplitude exp(-t^2/T^2) has FWHM 2 T sqrt(ln 2): 60 fs gives 100 fs
    g = GOLD["gaussian_fwhm"]
    kind, a, b = W.table1_run("D").ramp_args
    assert kind == W.RAMP_GAUSS and b == pytest.approx(180e-15)
    assert a == pytest.approx(g["T_fs"] * 1e-15)
    assert 2 * a * math.sqrt(math.log(2)) == pytest.approx(g["fwhm_fs"] * 1e-15, rel=0.005)


@pytest.mark.parametrize("m", [0, 1, 2])
def test_validation_run_v_recipe(m):
    # θ = 25°, n_s = 20, N_perp = 2, 16-cell CPML: int(40 * 2 / 0.42262) + 32 = 221,
    # R_B = 2 * 20 / sin 25° = 94.65 cells, δs = 1 λ = 20 cells, two axial
    # periods = 44 planes, 1700 steps (800 ramp + 448 inward transit + window)
    w = W.validation_v(m)
    assert (w.nx, w.ny, w.npml) == (221, 221, 16)
    assert w.order == m and w.theta_deg == 25.0 and w.ns == 20.0
    assert w.r_outer_cells == pytest.approx(94.65, abs=0.01)
    assert w.thickness_cells == 20.0
    assert w.steps == 1700 and w.ramp_kind == W.RAMP_SIN2 and w.ramp_periods == 20.0
    ramp_steps = w.ramp_periods * w.steps_per_period
    transit_steps = w.r_outer_cells / math.sin(w.theta) / w.courant
    assert ramp_steps == 800 and transit_steps == pytest.approx(448, abs=0.5)
    assert w.steps >= ramp_steps + transit_steps + 200
    assert P.fit_periodic_z(W.WAVELENGTH, w.theta, w.dx, w.nz_hint)[0] == 44
    assert 0.0 <= 2 * w.r_outer_cells - (w.nx - 2 * w.npml) < 1.0


def test_headline_grid_sizes():
    # the step benchmark's box: 768 x 768 cells, 256 planes asked, whole
    # axial periods at θ = 20°, Δx = λ/24 give 255 planes
    w = W.grid768()
    assert (w.nx, w.ny, w.ns, w.theta_deg, w.order) == (768, 768, 24.0, 20.0, 2)
    nz, dz = P.fit_periodic_z(W.WAVELENGTH, w.theta, w.dx, w.nz_hint)
    assert nz == 255
    assert nz * dz == pytest.approx(10 * W.WAVELENGTH / math.cos(w.theta), rel=1e-12)
