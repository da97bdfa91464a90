"""Pins of the analytic Bessel-beam module (paper §3.1, §3.2) — CPU only.

The pins are independent of the oracle's formulas: Maxwell's equations checked
with finite differences of the full 3-D complex field, ∇×Π checked with finite
differences of the Hertz potential itself, and numbers printed in the paper.
"""
import json
import math
import os

import numpy as np
import pytest
from scipy.optimize import brentq

from oracle import fields as F
from oracle import problem as P

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))

# 6th-order central first-derivative weights at offsets ±1, ±2, ±3 (times 1/h)
_W6 = (3.0 / 4.0, -3.0 / 20.0, 1.0 / 60.0)


def _d(fun, p, axis, h):
    acc = 0.0
    for q, wq in enumerate(_W6, start=1):
        e = np.zeros(3)
        e[axis] = q * h
        acc = acc + wq * (fun(p + e) - fun(p - e))
    return acc / h


def _field3d(m, k, theta, e0):
    beta = k * math.cos(theta)

    def comp(ci):
        def f(p):
            a = F.te_x_amplitudes(m, k, theta, e0, np.array([p[0]]), np.array([p[1]]))[ci]
            return complex(np.asarray(a).reshape(-1)[0]) * np.exp(1j * beta * p[2])
        return f
    return [comp(ci) for ci in range(6)]


def _curl(fx, fy, fz, p, h):
    return np.array([
        _d(fz, p, 1, h) - _d(fy, p, 2, h),
        _d(fx, p, 2, h) - _d(fz, p, 0, h),
        _d(fy, p, 0, h) - _d(fx, p, 1, h),
    ])


def _div(fx, fy, fz, p, h):
    return _d(fx, p, 0, h) + _d(fy, p, 1, h) + _d(fz, p, 2, h)


@pytest.mark.parametrize("m", [0, 1, 2, 3])
@pytest.mark.parametrize("theta_deg", [10.0, 25.0, 40.0])
def test_te_fields_satisfy_maxwell(m, theta_deg):
    """curl E = i k H, curl H = -i k E, div E = div H = 0 (e^{-iωt}, c = 1)."""
    k = 2 * math.pi / 16.0
    theta = math.radians(theta_deg)
    ex, ey, ez, hx, hy, hz = _field3d(m, k, theta, 1.3)
    rng = np.random.default_rng(7 + m)
    pts = [np.array([0.0, 0.0, 0.3])] + [rng.uniform(-40, 40, 3) for _ in range(6)]
    h = 0.02
    for p in pts:
        e = np.array([f(p) for f in (ex, ey, ez)])
        hh = np.array([f(p) for f in (hx, hy, hz)])
        scale = k * (np.linalg.norm(e) + np.linalg.norm(hh)) + 1e-6 * k
        assert np.linalg.norm(_curl(ex, ey, ez, p, h) - 1j * k * hh) / scale < 1e-9
        assert np.linalg.norm(_curl(hx, hy, hz, p, h) + 1j * k * e) / scale < 1e-9
        assert abs(_div(ex, ey, ez, p, h)) / scale < 1e-9
        assert abs(_div(hx, hy, hz, p, h)) / scale < 1e-9


@pytest.mark.parametrize("m", [0, 1, 2])
def test_printed_q_r_are_curls_of_hertz_potential(m):
    """Q and R printed for Π_x (§3.1) are ∇×Π and ∇×Q for Π ∝ e^{+iβz}."""
    k = 2 * math.pi / 20.0
    theta = math.radians(25.0)
    beta = k * math.cos(theta)

    def pi_x(p):
        return complex(F.hertz_x(m, k, theta, p[0], p[1], p[2]))

    def zero(p):
        return 0.0

    def q_comp(ci):
        def f(p):
            q, _ = F.qr_x(m, k, theta, np.array([p[0]]), np.array([p[1]]))
            return complex(np.asarray(q[ci]).reshape(-1)[0]) * np.exp(1j * beta * p[2])
        return f

    def r_comp(ci):
        def f(p):
            _, r = F.qr_x(m, k, theta, np.array([p[0]]), np.array([p[1]]))
            return complex(np.asarray(r[ci]).reshape(-1)[0]) * np.exp(1j * beta * p[2])
        return f

    rng = np.random.default_rng(11)
    h = 0.02
    for p in [rng.uniform(-30, 30, 3) for _ in range(5)]:
        q_fd = _curl(pi_x, zero, zero, p, h)
        q = np.array([q_comp(c)(p) for c in range(3)])
        r_fd = _curl(q_comp(0), q_comp(1), q_comp(2), p, h)
        r = np.array([r_comp(c)(p) for c in range(3)])
        assert np.linalg.norm(q_fd - q) / (k * np.linalg.norm(q) + 1e-30) < 1e-9
        assert np.linalg.norm(r_fd - r) / (k * np.linalg.norm(r) + 1e-30) < 1e-9


@pytest.mark.parametrize("theta_deg", [10.0, 17.0, 25.0, 30.0])
def test_on_axis_factor_is_minus_cos_theta(theta_deg):
    """§3.2: the order-0 E_y on the axis carries -cos θ (E0 = 1)."""
    theta = math.radians(theta_deg)
    k = 2 * math.pi / 20.0
    ey = F.te_x_amplitudes(0, k, theta, 1.0, np.array([0.0]), np.array([0.0]))[1]
    want = GOLDEN["on_axis_factor"]["value_over_cos_theta"] * math.cos(theta)
    assert abs(complex(ey[0]) - want) < 1e-14


def test_central_spot_radius_matches_paper():
    """§1: r0 = 0.383 λ / sin θ for the zeroth-order beam."""
    k = 2 * math.pi      # λ = 1
    theta = math.radians(20.0)
    r0 = brentq(lambda r: F.qr_x(0, k, theta, np.array([r]), np.array([0.0]))[0][1][0].imag,
                0.2 / math.sin(theta), 0.6 / math.sin(theta))
    assert round(r0 * math.sin(theta), 3) == GOLDEN["central_spot_radius_m0"]["value"]
    ms = F.ey_mean_square(0, k, theta, 1.0, np.array([r0]))
    assert ms[0] < 1e-25


def test_mean_square_is_half_amplitude_squared():
    """⟨E_y²⟩ = ½|Ẽ_y|², and |Ẽ_y| = E0 cos θ |J_m| for every m."""
    k = 2 * math.pi / 20.0
    theta = math.radians(25.0)
    rng = np.random.default_rng(3)
    x, y = rng.uniform(-50, 50, 20), rng.uniform(-50, 50, 20)
    for m in range(4):
        ey = F.te_x_amplitudes(m, k, theta, 2.0, x, y)[1]
        ms = F.ey_mean_square(m, k, theta, 2.0, np.hypot(x, y))
        np.testing.assert_allclose(ms, 0.5 * np.abs(ey) ** 2, rtol=1e-13, atol=1e-30)
        # brute-force average of the real field over one period
        t = np.linspace(0, 2 * math.pi, 64, endpoint=False)
        real = np.real(ey[:, None] * np.exp(-1j * t[None, :]))
        np.testing.assert_allclose(np.mean(real ** 2, axis=1), ms, rtol=1e-12, atol=1e-30)


def test_gaussian_envelope_fwhm_matches_paper():
    """§3.2: T = 60 fs gives FWHM = 2 T sqrt(ln 2) ≈ 100 fs of exp(-t²/T²)."""
    gold = GOLDEN["gaussian_fwhm"]
    dx = 50e-9
    tunit = dx / P.C_LIGHT
    ant = P.Antenna(k=1.0, beta=1.0, omega=1.0, ramp_kind=P.RAMP_GAUSS,
                    ramp_a=gold["T_fs"] * 1e-15 / tunit, ramp_b=180e-15 / tunit)
    half = lambda t: float(P.envelope(ant, t)) - 0.5
    lo = brentq(half, 0.0, ant.ramp_b)
    hi = brentq(half, ant.ramp_b, 3 * ant.ramp_b)
    fwhm_fs = (hi - lo) * tunit * 1e15
    assert abs(fwhm_fs - gold["fwhm_fs"]) < 0.5


def test_snapshot_times_are_whole_periods():
    """§5: 26.7, 106.8, 213.5 fs are 10, 40, 80 periods of λ = 0.8 µm."""
    gold = GOLDEN["snapshot_times"]
    period_fs = gold["wavelength_um"] * 1e-6 / P.C_LIGHT * 1e15
    for t, n in zip(gold["times_fs"], gold["periods"]):
        assert round(t / period_fs) == n
        assert abs(t - n * period_fs) < 0.1      # printed to 0.1 fs


def test_sin2_ramp_is_smooth_turn_on():
    ant = P.Antenna(k=1.0, beta=1.0, omega=1.0, ramp_kind=P.RAMP_SIN2, ramp_a=100.0)
    t = np.array([0.0, 50.0, 100.0, 150.0])
    np.testing.assert_allclose(P.envelope(ant, t), [0.0, 0.5, 1.0, 1.0], atol=1e-15)


def _pot_fd(axis, m, k, theta):
    """Components of Π = ê_axis J_m e^{imφ} e^{iβz} as functions of a point."""
    def psi(p):
        return complex(F.hertz_x(m, k, theta, p[0], p[1], p[2]))

    def zero(p):
        return 0.0
    return [psi if c == axis else zero for c in range(3)]


@pytest.mark.parametrize("axis", [1, 2])
@pytest.mark.parametrize("m", [0, 1, 2])
def test_printed_q_r_of_pi_y_and_pi_z_are_curls(axis, m):
    """Q and R printed for Π_y and Π_z (§3.1) are ∇×Π and ∇×Q."""
    k = 2 * math.pi / 20.0
    theta = math.radians(25.0)
    beta = k * math.cos(theta)

    def comp(which, ci):
        def f(p):
            qr = F.QR[axis](m, k, theta, np.array([p[0]]), np.array([p[1]]))[which]
            return complex(np.asarray(qr[ci]).reshape(-1)[0]) * np.exp(1j * beta * p[2])
        return f

    pot = _pot_fd(axis, m, k, theta)
    rng = np.random.default_rng(13 + axis)
    h = 0.02
    for p in [rng.uniform(-30, 30, 3) for _ in range(5)]:
        q_fd = _curl(*pot, p, h)
        q = np.array([comp(0, c)(p) for c in range(3)])
        r_fd = _curl(comp(0, 0), comp(0, 1), comp(0, 2), p, h)
        r = np.array([comp(1, c)(p) for c in range(3)])
        assert np.linalg.norm(q_fd - q) / (k * np.linalg.norm(q) + 1e-30) < 1e-9
        assert np.linalg.norm(r_fd - r) / (k * np.linalg.norm(r) + 1e-30) < 1e-9


@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("tm", [0, 1])
@pytest.mark.parametrize("m", [0, 1, 3])
def test_every_mode_satisfies_maxwell(axis, tm, m):
    """TE and TM pairings of the three potentials: curl E = i k H,
    curl H = -i k E, div E = div H = 0."""
    k = 2 * math.pi / 16.0
    theta = math.radians(22.0)
    beta = k * math.cos(theta)

    def comp(ci):
        def f(p):
            a = F.amplitudes(axis, tm, m, k, theta, 0.7, np.array([p[0]]), np.array([p[1]]))[ci]
            return complex(np.asarray(a).reshape(-1)[0]) * np.exp(1j * beta * p[2])
        return f
    ex, ey, ez, hx, hy, hz = [comp(c) for c in range(6)]
    rng = np.random.default_rng(31 + 3 * axis + tm)
    h = 0.02
    for p in [rng.uniform(-35, 35, 3) for _ in range(4)]:
        e = np.array([f(p) for f in (ex, ey, ez)])
        hh = np.array([f(p) for f in (hx, hy, hz)])
        scale = k * (np.linalg.norm(e) + np.linalg.norm(hh)) + 1e-6 * k
        assert np.linalg.norm(_curl(ex, ey, ez, p, h) - 1j * k * hh) / scale < 1e-9
        assert np.linalg.norm(_curl(hx, hy, hz, p, h) + 1j * k * e) / scale < 1e-9
        assert abs(_div(ex, ey, ez, p, h)) / scale < 1e-9
        assert abs(_div(hx, hy, hz, p, h)) / scale < 1e-9


def test_pi_z_order0_is_radial_tm_and_azimuthal_te():
    """§3.1: Π_z gives purely radial (TM, E from R) or azimuthal (TE, E from
    Q) polarisation for m = 0."""
    k = 2 * math.pi / 20.0
    theta = math.radians(25.0)
    rng = np.random.default_rng(17)
    x, y = rng.uniform(-60, 60, 40), rng.uniform(-60, 60, 40)
    phi = np.arctan2(y, x)
    ex, ey, ez = F.amplitudes(2, 1, 0, k, theta, 1.0, x, y)[:3]
    e_phi = -np.sin(phi) * ex + np.cos(phi) * ey
    assert np.max(np.abs(e_phi)) < 1e-15 * max(1.0, np.max(np.abs(ex)))
    assert np.max(np.abs(ex) + np.abs(ey)) > 1e-3
    ex, ey, ez = F.amplitudes(2, 0, 0, k, theta, 1.0, x, y)[:3]
    e_r = np.cos(phi) * ex + np.sin(phi) * ey
    assert np.max(np.abs(e_r)) < 1e-15 and np.max(np.abs(ez)) == 0.0
    assert np.max(np.abs(ex) + np.abs(ey)) > 1e-3


@pytest.mark.parametrize("tm", [0, 1])
@pytest.mark.parametrize("m", [0, 1, 2])
def test_pi_y_is_pi_x_turned_by_a_quarter(tm, m):
    """Turning Π_x by +90° about z gives e^{-imπ/2} Π_y, so every field of
    Π_y is the turned field of Π_x times e^{imπ/2}."""
    k = 2 * math.pi / 18.0
    theta = math.radians(20.0)
    rng = np.random.default_rng(19)
    x, y = rng.uniform(-50, 50, 30), rng.uniform(-50, 50, 30)
    fy = F.amplitudes(1, tm, m, k, theta, 1.0, x, y)
    fx = F.amplitudes(0, tm, m, k, theta, 1.0, y, -x)      # at R^{-1} p
    ph = np.exp(1j * m * math.pi / 2)
    for o in (0, 3):   # E then H: (vx, vy, vz) -> (-vy, vx, vz)
        np.testing.assert_allclose(fy[o + 0], -ph * fx[o + 1], atol=1e-14)
        np.testing.assert_allclose(fy[o + 1], ph * fx[o + 0], atol=1e-14)
        np.testing.assert_allclose(fy[o + 2], ph * fx[o + 2], atol=1e-14)
