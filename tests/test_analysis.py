"""Host-side comparison with the analytic beam (paper §5 deviation χ):
checked on planes built from SciPy's Bessel function, CPU only."""
import math

import numpy as np
import pytest
from scipy.special import jn_zeros, jnp_zeros, jv

from paper_2102_12978_amd import analysis as A


def _plane(m, nx=160, ny=160, ns=16.0, theta_deg=30.0):
    k = 2 * math.pi / ns
    K = k * math.sin(math.radians(theta_deg))
    xs, ys, r = A.ey_radius(nx, ny)
    return 0.5 * math.cos(math.radians(theta_deg)) ** 2 * jv(m, K * r) ** 2, K, r


@pytest.mark.parametrize("m", [0, 1, 2, 3])
def test_exact_plane_has_zero_deviation(m):
    ana, K, r = _plane(m)
    res = A.lobe_deviation(2.5 * ana, ana, K, 60.0)
    assert res["alpha"] == pytest.approx(2.5, rel=1e-12)
    assert max(res["chi"]) < 1e-12
    # lobe radii: the extrema of J_m — the axis and the zeros of J_1 for
    # m = 0 (J_0' = -J_1), the zeros of J_m' otherwise — within a cell
    expect = [0.0] + list(jn_zeros(1, 12) / K) if m == 0 else list(jnp_zeros(m, 12) / K)
    expect = [x for x in expect if x < 57.0]   # a maximum needs a cell beyond it
    assert len(res["radii"]) == len(expect)
    assert np.allclose(res["radii"], expect, atol=1.0)


def test_single_lobe_perturbation():
    """Scaling the second ring by 1.04 in ⟨E_y²⟩ gives χ ≈ 2 % there."""
    ana, K, r = _plane(0)
    res0 = A.lobe_deviation(ana, ana, K, 60.0)
    r1, r2 = res0["radii"][1], res0["radii"][2]
    ring = (r > 0.5 * (res0["radii"][0] + r1)) & (r < 0.5 * (r1 + r2))
    ey2 = np.where(ring, 1.04 * ana, ana)
    res = A.lobe_deviation(ey2, ana, K, 60.0, n_fit=1)
    assert res["chi"][0] < 1e-9
    assert res["chi"][1] == pytest.approx(math.sqrt(1.04) - 1.0, rel=1e-9)
