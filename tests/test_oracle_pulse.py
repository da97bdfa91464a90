"""Pins of the oracle's Bessel pulse (paper §3.2) against closed forms, the
fronts the paper describes, the CW beam and an independent quadrature."""
import math

import numpy as np
from scipy.special import jv, jvp

from oracle import fields as F
from oracle import pulse as PU

TH = math.radians(25.0)
NS = 20.0
W0 = 2 * math.pi / NS          # carrier, 1/(Δx/c)


def test_on_axis_m0_is_the_gaussian_pulse_moving_at_c_over_cos_theta():
    """On the axis J_0 = 1 and the spectrum integral is the Gaussian
    envelope: E_y = -E0 cos θ exp(-τ²/T²) cos(ω0 τ), τ = t - T0 - z cos θ."""
    T, T0 = 450.0, 1350.0
    z = np.array([0.0, 7.0, -30.0, 200.0])
    t = np.linspace(800.0, 2000.0, 37)[:, None]
    got = PU.ey_pulse(0, TH, W0, T, T0, 0.0, 0.0, z[None, :], t, e0=1.3)
    tau = t - T0 - z[None, :] * math.cos(TH)
    want = -1.3 * math.cos(TH) * np.exp(-(tau / T) ** 2) * np.cos(W0 * tau)
    assert np.max(np.abs(got - want)) < 1e-13


def test_on_axis_higher_orders_vanish():
    for m in (1, 2, 3):
        v = PU.ey_pulse_complex(m, TH, W0, 300.0, 900.0, 0.0, 0.0, 3.0, np.linspace(0, 2000, 11))
        assert np.max(np.abs(v)) < 1e-15


def test_first_order_narrow_band_expansion():
    """Expanding J_m(ω a) to first order about ω0 (a = r sin θ): the
    integral is G(τ)[J_m(a ω0) - (2iτ/T²) a J_m'(a ω0)] e^{imφ} with
    G = e^{-iω0 τ} e^{-τ²/T²}; the remainder is O((a/T)²)."""
    T, T0 = 2000.0, 0.0
    rng = np.random.default_rng(5)
    for m in (0, 1, 2):
        x, y = rng.uniform(-60, 60, 20), rng.uniform(-60, 60, 20)
        t = rng.uniform(-T, T, 20)
        got = PU.ey_pulse_complex(m, TH, W0, T, T0, x, y, 0.0, t)
        r, phi = np.hypot(x, y), np.arctan2(y, x)
        a = r * math.sin(TH)
        tau = t - T0
        g = np.exp(-1j * W0 * tau) * np.exp(-(tau / T) ** 2)
        want = -math.cos(TH) * np.exp(1j * m * phi) * g * (
            jv(m, a * W0) - 2j * tau / T ** 2 * a * jvp(m, a * W0))
        bound = 3 * (a / T) ** 2 * (1 + 2 * (tau / T) ** 2) + 1e-12
        assert np.all(np.abs(got - want) <= bound), np.max(np.abs(got - want) / bound)


def test_envelope_fronts_travel_at_c_over_sin_theta():
    """Away from the axis the pulse is two conical fronts whose envelopes
    peak where t - T0 = ±r sin θ / c (§3.2: the waves move at ±c / sin θ
    across the transverse plane)."""
    T, T0 = 120.0, 0.0
    for r in (600.0, 900.0):
        a = r * math.sin(TH)
        t = np.linspace(-2 * a, 2 * a, 8001)
        env = np.abs(PU.ey_pulse_complex(0, TH, W0, T, T0, r, 0.0, 0.0, t, nodes=120))
        left = t < 0
        tl = t[left][np.argmax(env[left])]
        tr = t[~left][np.argmax(env[~left])]
        assert abs(tl + a) < 0.05 * T and abs(tr - a) < 0.05 * T, (tl, tr, a)


def test_long_pulse_limit_is_the_cw_beam():
    """T → ∞: the spectrum is a delta at ω0 and the pulse is the §3.1 beam
    Re{Ã_y e^{i(βz - ω0 (t - T0))}} with Ã_y from the CW field module."""
    rng = np.random.default_rng(6)
    x, y, z = rng.uniform(-80, 80, 30), rng.uniform(-80, 80, 30), rng.uniform(-20, 20, 30)
    t = rng.uniform(0, 100, 30)
    for m in (0, 1, 2):
        got = PU.ey_pulse(m, TH, W0, 1e7, 0.0, x, y, z, t)
        ay = F.te_x_amplitudes(m, W0, TH, 1.0, x, y)[1]
        want = (ay * np.exp(1j * (W0 * math.cos(TH) * z - W0 * t))).real
        assert np.max(np.abs(got - want)) < 1e-9


def test_quadrature_against_dense_trapezoid():
    T, T0 = 300.0, 700.0
    m = 1
    x, y, z = np.array([3.0, -40.0, 71.5]), np.array([-9.0, 12.5, 30.0]), np.array([0.0, 5.0, -2.0])
    t = np.array([650.0, 900.0, 1100.0])
    got = PU.ey_pulse_complex(m, TH, W0, T, T0, x, y, z, t)
    om = np.linspace(W0 - 14 / T, W0 + 14 / T, 20001)
    spec = T / (2 * math.sqrt(math.pi)) * np.exp(-(T * (om - W0)) ** 2 / 4)
    for q in range(3):
        r, phi = math.hypot(x[q], y[q]), math.atan2(y[q], x[q])
        f = spec * jv(m, om * math.sin(TH) * r) * np.exp(
            1j * om * (math.cos(TH) * z[q] - (t[q] - T0)))
        want = -math.cos(TH) * np.exp(1j * m * phi) * np.trapezoid(f, om)
        assert abs(got[q] - want) < 1e-10
