"""Analytic Bessel-beam fields (paper §3.1, Bessel's solutions) — oracle side.

TEST INFRASTRUCTURE (see ``oracle/__init__``).

Reading of the paper used here (it is stated once and pinned by tests):

* Hertz potential polarised along x, order m (§3.1, the Π_x potential):
  Π = x̂ J_m(K r) e^{i m φ} e^{i β z} with the harmonic time factor e^{-iωt}
  (the convention §3.1 announces for the E/H solution pairs). The Q and R
  vectors printed for Π_x are exactly ∇×Π and ∇×∇×Π for this z factor.
* Dispersion / cone angle (§3.1): β² + K² = k², K = k sin θ, β = k cos θ.
* TE pairing (§3.1, TE/TM normalisation, TE case) in normalised units
  (c = ε0 = μ0 = 1, H̃ = η0 H): Ẽ = i (E0/k) Q and H̃ = (E0/k²) R. The factor i
  is the one that the E2 = i k0 Q solution carries; with it the pair obeys
  ∇×Ẽ = i k H̃ and ∇×H̃ = -i k Ẽ and the on-axis E_y of the m = 0 beam is
  -E0 cos θ, the sign and factor of the Bessel-pulse formula of §3.2.
* The real field is Re{Ã(x, y) e^{i(βz - ω(t - T0))}} f(t).

Parity: pinned by the Maxwell-residual tests (finite-difference curls of the
3-D complex field), by finite-difference curls of Π itself, and by the values
printed in the paper (first zero of the m = 0 intensity at 0.383 λ/sin θ,
on-axis factor -cos θ).
"""
import numpy as np
from scipy.special import jv

COMPONENTS = ("ex", "ey", "ez", "hx", "hy", "hz")


def _u(nu, kr, phi):
    """J_nu(K r) e^{i nu phi} for integer nu (negative orders through scipy)."""
    return jv(nu, kr) * np.exp(1j * nu * phi)


def hertz_x(m, k, theta, x, y, z):
    """Potential value J_m(K r) e^{i m φ} e^{i β z} (§3.1); the three potentials
    Π_x, Π_y, Π_z carry it along x̂, ŷ or ẑ."""
    K = k * np.sin(theta)
    beta = k * np.cos(theta)
    r = np.hypot(x, y)
    phi = np.arctan2(y, x)
    return _u(m, K * r, phi) * np.exp(1j * beta * z)


def qr_x(m, k, theta, x, y):
    """Transverse parts of Q = ∇×Π and R = ∇×∇×Π for Π_x (§3.1, Π_x case).

    Returns (Q, R), each a tuple of three complex arrays (x, y, z components),
    without the common factor e^{iβz} (and without e^{imφ} pulled out: the
    azimuthal factors are included in each Bessel term).
    """
    K = k * np.sin(theta)
    beta = k * np.cos(theta)
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    r = np.hypot(x, y)
    phi = np.arctan2(y, x)
    kr = K * r
    um = _u(m, kr, phi)
    up1, um1 = _u(m + 1, kr, phi), _u(m - 1, kr, phi)
    up2, um2 = _u(m + 2, kr, phi), _u(m - 2, kr, phi)
    q = (np.zeros_like(um),
         1j * beta * um,
         K / 2j * (up1 + um1))
    rr = ((k * k + beta * beta) / 2 * um + K * K / 4 * (up2 + um2),
          1j * K * K / 4 * (um2 - up2),
          1j * beta * K / 2 * (um1 - up1))
    return q, rr


def qr_y(m, k, theta, x, y):
    """Q = ∇×Π and R = ∇×∇×Π for Π_y (§3.1, Π_y case), as printed; same
    conventions as qr_x."""
    K = k * np.sin(theta)
    beta = k * np.cos(theta)
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    r = np.hypot(x, y)
    phi = np.arctan2(y, x)
    kr = K * r
    um = _u(m, kr, phi)
    up1, um1 = _u(m + 1, kr, phi), _u(m - 1, kr, phi)
    up2, um2 = _u(m + 2, kr, phi), _u(m - 2, kr, phi)
    q = (-1j * beta * um,
         np.zeros_like(um),
         -K / 2 * (up1 - um1))
    rr = (1j * K * K / 4 * (um2 - up2),
          (k * k + beta * beta) / 2 * um - K * K / 4 * (up2 + um2),
          -beta * K / 2 * (up1 + um1))
    return q, rr


def qr_z(m, k, theta, x, y):
    """Q = ∇×Π and R = ∇×∇×Π for Π_z (§3.1, Π_z case), as printed; same
    conventions as qr_x."""
    K = k * np.sin(theta)
    beta = k * np.cos(theta)
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    r = np.hypot(x, y)
    phi = np.arctan2(y, x)
    kr = K * r
    um = _u(m, kr, phi)
    up1, um1 = _u(m + 1, kr, phi), _u(m - 1, kr, phi)
    q = (1j * K / 2 * (up1 + um1),
         K / 2 * (up1 - um1),
         np.zeros_like(um))
    rr = (-1j * beta * K / 2 * (up1 - um1),
          -beta * K / 2 * (up1 + um1),
          K * K * um)
    return q, rr


QR = {0: qr_x, 1: qr_y, 2: qr_z}


def amplitudes(axis, tm, m, k, theta, e0, x, y):
    """Complex amplitudes (Ex, Ey, Ez, Hx, Hy, Hz) of the Π_axis beam.

    TE pairing (E ∝ Q, the E2/H2 solution): Ẽ = i (E0/k) Q, H̃ = (E0/k²) R.
    TM pairing (E ∝ R, the E1/H1 solution): Ẽ = (E0/k²) R, H̃ = -i (E0/k) Q.
    Both follow from ∇×Q = R and ∇×R = k² Q with ∇×Ẽ = i k H̃ (e^{-iωt},
    c = 1, H̃ = η0 H); the TE case is the reading stated in the header."""
    q, rr = QR[axis](m, k, theta, x, y)
    if tm:
        e = tuple(e0 / (k * k) * rc for rc in rr)
        h = tuple(-1j * e0 / k * qc for qc in q)
    else:
        e = tuple(1j * e0 / k * qc for qc in q)
        h = tuple(e0 / (k * k) * rc for rc in rr)
    return e + h


def te_x_amplitudes(m, k, theta, e0, x, y):
    """Complex amplitudes (Ex, Ey, Ez, Hx, Hy, Hz) of the TE Π_x beam.

    §3.1 TE normalisation under the reading in the module header:
    Ẽ = i (E0/k) Q, H̃ = (E0/k²) R. Coordinates are relative to the beam axis.
    """
    q, rr = qr_x(m, k, theta, x, y)
    e = tuple(1j * e0 / k * qc for qc in q)
    h = tuple(e0 / (k * k) * rc for rc in rr)
    return e + h


def ey_mean_square(m, k, theta, e0, r):
    """Time average of E_y² of the CW beam: ½ E0² cos²θ J_m²(K r).

    |Ẽ_y| = E0 cos θ |J_m(K r)| for every m, so the mean of the squared real
    field over a period is half its square (used for the intensity
    comparison of §5).
    """
    K = k * np.sin(theta)
    return 0.5 * e0 * e0 * np.cos(theta) ** 2 * jv(m, K * np.asarray(r)) ** 2
