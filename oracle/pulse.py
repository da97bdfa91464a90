"""Analytic Bessel pulse (paper §3.2, the Bessel-pulse formula) by FP64
quadrature — oracle side.

TEST INFRASTRUCTURE (see ``oracle/__init__``).

§3.2 builds a pulse by summing the monochromatic beam of §3.1 over a
Gaussian spectrum F(ω) = T/(2√π) exp(-T²(ω - ω0)²/4) (so ∫F dω = 1 and the
time-domain envelope is exp(-t²/T²)); every frequency keeps the cone angle θ,
so its transverse and axial wavenumbers are ω sin θ / c and ω cos θ / c.
Under the convention of ``fields`` (harmonic factor e^{-iωt}, axial factor
e^{+iβz}, on-axis E_y of the m = 0 beam equal to -E0 cos θ) the y component
of the y-polarised order-m pulse is

    E_y(x, y, z, t) = Re{ -E0 cos θ e^{imφ}
                          ∫ dω F(ω) J_m(ω sin θ r / c) e^{i(ω cos θ z / c - ω(t - T0))} },

which at T → ∞ is the CW beam of ``fields.te_x_amplitudes`` and on the axis
(m = 0) the Gaussian pulse -E0 cos θ exp(-τ²/T²) cos(ω0 τ), τ = t - T0 - z cos θ/c.

Units follow ``problem``: lengths in Δx, time in Δx/c, c = 1.

The integral is evaluated with Gauss-Hermite quadrature in u = T(ω - ω0)/2,
whose weight e^{-u²} is exactly the spectrum: ∫ F g dω = π^{-1/2} ∫ e^{-u²}
g(ω0 + 2u/T) du.

Parity: pinned by the on-axis closed form (m = 0, any z: the axial peak
travels at c / cos θ), the vanishing on-axis field for m ≥ 1, the
first-order narrow-band expansion, the envelope maxima at t - T0 = ±r sin θ/c
away from the axis (the ±c / sin θ fronts of §3.2 Fig. 2), the T → ∞ limit
against ``fields``, and a dense trapezoid rule over ω.
"""
import numpy as np
from scipy.special import jv


def ey_pulse_complex(m, theta, omega0, T, T0, x, y, z, t, e0=1.0, nodes=80):
    """Complex analytic signal whose real part is the pulse's E_y.

    m: order; theta: cone angle (rad); omega0: carrier angular frequency
    (1/(Δx/c)); T, T0: envelope width and peak time (Δx/c); x, y, z, t:
    broadcastable arrays (Δx, Δx/c) relative to the beam axis."""
    u, wts = np.polynomial.hermite.hermgauss(nodes)
    x, y, z, t = np.broadcast_arrays(*(np.asarray(v, dtype=np.float64) for v in (x, y, z, t)))
    r = np.hypot(x, y)
    phi = np.arctan2(y, x)
    tau = t - T0 - z * np.cos(theta)
    s = np.sin(theta)
    acc = np.zeros(r.shape, dtype=np.complex128)
    for ui, wi in zip(u, wts):
        om = omega0 + 2.0 * ui / T
        acc += wi * jv(m, om * s * r) * np.exp(-1j * om * tau)
    acc /= np.sqrt(np.pi)
    return -e0 * np.cos(theta) * np.exp(1j * m * phi) * acc


def ey_pulse(m, theta, omega0, T, T0, x, y, z, t, e0=1.0, nodes=80):
    """E_y of the order-m Bessel pulse (real field)."""
    return ey_pulse_complex(m, theta, omega0, T, T0, x, y, z, t, e0=e0, nodes=nodes).real
