"""Pins of the oracle Yee solver — CPU only.

Each pin is something the mathematics fixes independently of the oracle's
code: the exact discrete plane-wave eigenmode (numerical dispersion closed
form), the discrete energy invariant, div∘curl = 0, linearity, a brute-force
single step, hand-computed z fits, a brute-force antenna membership, and CPML
absorption against a larger reflection-free box.
"""
import math

import numpy as np
import pytest

from oracle import fields as F
from oracle import problem as P
from oracle import yee as Y
from paper_2102_12978_amd import workloads as W
from tests import cases

OFFS = P.OFFSETS


def _positions(g, comp):
    ox, oy, oz = OFFS[comp]
    k, j, i = np.meshgrid(np.arange(g.nz), np.arange(g.ny), np.arange(g.nx), indexing="ij")
    return (i + ox) * 1.0, (j + oy) * g.ry, (k + oz) * g.rz


def _plane_wave(g, p_int, pol):
    """Exact discrete eigenmode of the periodic Yee scheme.

    With every component sampled at its own staggered position, the centred
    differences act on e^{iκ·x} as i K̃ with K̃_d = (2/Δ_d) sin(κ_d Δ_d / 2),
    so the leapfrog admits E = E0 e^{i(κ·x - ωt)}, H̃ = H0 e^{i(κ·x - ωt)} with
    E0 ⊥ K̃, Ω H0 = K̃ × E0 and Ω = (2/Δt) sin(ωΔt/2) = |K̃|.
    """
    deltas = np.array([1.0, g.ry, g.rz])
    n = np.array([g.nx, g.ny, g.nz])
    kap = 2 * np.pi * np.asarray(p_int) / (n * deltas)
    kt = 2.0 / deltas * np.sin(kap * deltas / 2)
    e0 = np.asarray(pol, dtype=float)
    e0 = e0 - kt * (e0 @ kt) / (kt @ kt)
    om = np.linalg.norm(kt)
    omega = 2.0 / g.dt * math.asin(g.dt * om / 2)
    h0 = np.cross(kt, e0) / om

    def state(n_e):
        st = Y.zero_state(g)
        for ci, comp in enumerate(("ex", "ey", "ez")):
            x, y, z = _positions(g, comp)
            st.f[comp] = np.real(e0[ci] * np.exp(1j * (kap[0] * x + kap[1] * y + kap[2] * z
                                                      - omega * n_e * g.dt)))
        for ci, comp in enumerate(("hx", "hy", "hz")):
            x, y, z = _positions(g, comp)
            st.f[comp] = np.real(h0[ci] * np.exp(1j * (kap[0] * x + kap[1] * y + kap[2] * z
                                                      - omega * (n_e + 0.5) * g.dt)))
        return st
    return state, omega


@pytest.mark.parametrize("p_int,pol", [
    ((1, 0, 0), (0, 1, 0.3)),
    ((0, 2, 0), (1, 0, 0.5)),
    ((0, 0, 1), (1, 0.4, 0)),
    ((2, -1, 1), (0.3, 1.0, -0.7)),
    ((3, 2, -2), (1.0, -0.2, 0.5)),
])
def test_plane_wave_eigenmode_dispersion(p_int, pol):
    g = P.Grid(12, 10, 8, 1.0, 1.1, 1.0154, courant=0.45, bc=P.BC_PERIODIC)
    g.validate()
    state, omega = _plane_wave(g, p_int, pol)
    st = state(0)
    Y.run(g, 200, state=st)
    want = state(200)
    scale = max(np.abs(want.f[c]).max() for c in want.f)
    for c in want.f:
        assert np.abs(st.f[c] - want.f[c]).max() / scale < 1e-11, c
    # the continuum ω would be off by the numerical dispersion: make sure the
    # test can tell them apart
    assert abs(omega - np.linalg.norm(2 * np.pi * np.asarray(p_int) /
                                      (np.array([12, 10, 8]) * np.array([1.0, 1.1, 1.0154])))) > 1e-4


def _random_state(g, seed, zero_walls):
    st = Y.zero_state(g)
    fields = W.random_fields((g.nz, g.ny, g.nx), seed)
    for c, f in zip(Y.E_COMPS + Y.H_COMPS, fields):
        st.f[c] = f
    if zero_walls:
        for c in Y.E_COMPS:
            st.f[c][:, Y.held_mask(g, c)] = 0.0
    return st


@pytest.mark.parametrize("bc", [P.BC_PERIODIC, P.BC_PEC])
def test_discrete_energy_invariant(bc):
    """W^n = Σ(E^n)² + Σ H̃^{n-1/2}·H̃^{n+1/2} is exact for the lossless scheme."""
    g = P.Grid(16, 12, 10, 1.0, 1.0, 1.0154, courant=0.5, bc=bc)
    st = _random_state(g, 0, zero_walls=(bc == P.BC_PEC))
    cp = P.cpml_tables(g)
    ws = [Y.step(st, g, cp, None, want_energy=True) for _ in range(200)]
    ws = np.array(ws)
    assert np.abs(ws - ws[0]).max() / abs(ws[0]) < 1e-12
    # and the scheme is not trivially static
    assert np.abs(st.f["ex"]).max() > 0.1


def test_divergence_invariants():
    """div∘curl = 0: div H̃ and div E stay at their initial values."""
    g = P.Grid(16, 12, 10, 1.0, 1.0, 1.0154, courant=0.5, bc=P.BC_PERIODIC)
    st = _random_state(g, 0, zero_walls=False)
    dh0, de0 = Y.div_h(st, g), Y.div_e(st, g)
    Y.run(g, 200, state=st)
    assert np.abs(Y.div_h(st, g) - dh0).max() < 1e-11
    assert np.abs(Y.div_e(st, g) - de0).max() < 1e-11
    # H̃ = curl_d A starts and stays divergence free
    a = _random_state(g, 5, zero_walls=False)
    st2 = Y.zero_state(g)
    p = True
    st2.f["hx"] = Y.fwd_diff(a.f["ez"], "y", p) / g.ry - Y.fwd_diff(a.f["ey"], "z", p) / g.rz
    st2.f["hy"] = Y.fwd_diff(a.f["ex"], "z", p) / g.rz - Y.fwd_diff(a.f["ez"], "x", p)
    st2.f["hz"] = Y.fwd_diff(a.f["ey"], "x", p) - Y.fwd_diff(a.f["ex"], "y", p) / g.ry
    assert np.abs(Y.div_h(st2, g)).max() < 1e-12
    Y.run(g, 100, state=st2)
    assert np.abs(Y.div_h(st2, g)).max() < 1e-11


def test_z_fit_hand_cases():
    """§4 periodic z: whole axial periods; values worked out by hand."""
    lam = 800e-9
    # 32³ grid: λ_z = 16/cos10° = 16.2469 cells, p = round(32/16.2469) = 2, nz = round(32.494) = 32
    nz, dz = P.fit_periodic_z(lam, math.radians(10), lam / 16, 32)
    assert nz == 32 and abs(dz / (lam / 16) - 2 * 16 / math.cos(math.radians(10)) / 32) < 1e-14
    # 256² grid: λ_z = 20.7055, p = 3, nz = round(62.116) = 62
    assert P.fit_periodic_z(lam, math.radians(15), lam / 20, 64)[0] == 62
    # 768² grid: λ_z = 25.5404, p = 10, nz = round(255.40) = 255
    assert P.fit_periodic_z(lam, math.radians(20), lam / 24, 256)[0] == 255
    # tiny hint never gives zero periods
    assert P.fit_periodic_z(lam, math.radians(30), lam / 16, 1)[0] == 18
    for th, ns, hint in [(10, 16, 32), (15, 20, 64), (20, 24, 256), (12, 20, 64), (5, 20, 50)]:
        nz, dz = P.fit_periodic_z(lam, math.radians(th), lam / ns, hint)
        beta = 2 * math.pi / lam * math.cos(math.radians(th))
        periods = beta * nz * dz / (2 * math.pi)
        assert abs(periods - round(periods)) < 1e-9


def test_antenna_membership_brute_force():
    """Annulus membership per component against an explicit double loop."""
    w = W.parity_small()
    g = cases.oracle_grid(w)
    ant = P.build_antenna(g, cases.oracle_injector(w))
    ax, ay = g.nx / 2.0, g.ny * g.ry / 2.0
    r_out, r_in = w.r_outer_cells, w.r_outer_cells - w.thickness_cells
    for comp in F.COMPONENTS:
        ox, oy, _ = OFFS[comp]
        want = set()
        for j in range(g.ny):
            for i in range(g.nx):
                r = math.hypot(i + ox - ax, (j + oy) * g.ry - ay)
                if r_in < r <= r_out:
                    want.add((j, i))
        got = set(zip(ant.idx[comp][0].tolist(), ant.idx[comp][1].tolist()))
        assert got == want, comp
        assert len(got) > 100


def test_first_step_brute_force():
    """From rest, E^1 is exactly the E source at t_1 and H̃^{3/2} = -S curl E^1 + H source."""
    w = W.parity_small()
    w.nx, w.ny = 72, 64
    w.r_outer_cells = 20.0
    g = cases.oracle_grid(w)
    inj = cases.oracle_injector(w)
    inj.ramp_kind = P.RAMP_CW
    ant = P.build_antenna(g, inj)
    st = Y.run(g, 1, ant)
    k = 2 * math.pi / w.ns
    beta = k * math.cos(w.theta)
    ax, ay = g.nx / 2.0, g.ny * g.ry / 2.0
    r_out, r_in = w.r_outer_cells, w.r_outer_cells - w.thickness_cells

    def src(comp, t):
        ci = F.COMPONENTS.index(comp)
        ox, oy, oz = OFFS[comp]
        out = np.zeros((g.nz, g.ny, g.nx))
        for j in range(g.ny):
            for i in range(g.nx):
                x, y = i + ox - ax, (j + oy) * g.ry - ay
                if not (r_in < math.hypot(x, y) <= r_out):
                    continue
                a = complex(np.asarray(F.te_x_amplitudes(w.order, k, w.theta, 1.0,
                                                         np.array([x]), np.array([y]))[ci])[0])
                for kk in range(g.nz):
                    out[kk, j, i] = (a * np.exp(1j * (beta * (kk + oz) * g.rz - k * t))).real
        return out

    for comp in ("ex", "ey", "ez"):
        np.testing.assert_allclose(st.f[comp], src(comp, g.dt), rtol=0, atol=1e-14)
    e1 = {c: src(c, g.dt) for c in ("ex", "ey", "ez")}
    s = g.s

    def dfx(u):   # forward differences with zero beyond the last cell
        return np.concatenate([u[:, :, 1:], np.zeros_like(u[:, :, :1])], axis=2) - u

    def dfy(u):
        return np.concatenate([u[:, 1:, :], np.zeros_like(u[:, :1, :])], axis=1) - u

    def dfz(u):
        return np.roll(u, -1, axis=0) - u
    # no CPML term touches the annulus here: it lies in the interior
    hx = -(s[1] * dfy(e1["ez"]) - s[2] * dfz(e1["ey"])) + src("hx", 1.5 * g.dt)
    hy = -(s[2] * dfz(e1["ex"]) - s[0] * dfx(e1["ez"])) + src("hy", 1.5 * g.dt)
    hz = -(s[0] * dfx(e1["ey"]) - s[1] * dfy(e1["ex"])) + src("hz", 1.5 * g.dt)
    for comp, want in (("hx", hx), ("hy", hy), ("hz", hz)):
        np.testing.assert_allclose(st.f[comp], want, rtol=0, atol=1e-14)


def test_source_linearity_and_superposition():
    w = W.parity_small()
    w.steps = 30
    g = cases.oracle_grid(w)
    a1 = Y.run(g, w.steps, P.build_antenna(g, cases.oracle_injector(w, e0=1.0)))
    a2 = Y.run(g, w.steps, P.build_antenna(g, cases.oracle_injector(w, e0=2.0)))
    for c in a1.f:
        np.testing.assert_allclose(a2.f[c], 2 * a1.f[c], rtol=0,
                                   atol=1e-13 * np.abs(a1.f[c]).max())
    # (random start, no source) + (rest, source) = (random start, source)
    r0 = _random_state(g, 3, zero_walls=True)
    free = Y.run(g, w.steps, state=r0.copy())
    both = Y.run(g, w.steps, P.build_antenna(g, cases.oracle_injector(w)), state=r0.copy())
    for c in a1.f:
        np.testing.assert_allclose(both.f[c], free.f[c] + a1.f[c], rtol=0, atol=1e-12)


def _blob_run(n, npml, bc, steps):
    g = P.Grid(n, n, 2, 1.0, 1.0, 1.0, courant=0.5, bc=bc, npml=npml, grade=3.0,
               sigma_scale=1.0, kappa_max=1.0, alpha_max=0.1 * 2 * math.pi / 20)
    st = Y.zero_state(g)
    c = n / 2.0
    i = np.arange(n)
    r2 = (i[None, :] - c) ** 2 + (i[:, None] - c) ** 2
    st.f["ez"][:] = np.exp(-r2 / (2 * 3.0 ** 2))[None]
    Y.run(g, steps, state=st)
    return st


def test_cpml_absorbs_against_larger_box():
    """A z-invariant pulse leaves a 64² box through 12-cell CPML; what comes
    back is compared with a 384² PEC box whose walls are out of reach."""
    steps = 160               # t = 80: the pulse reaches the CPML and returns
    small = _blob_run(64, 12, P.BC_CPML, steps)
    big = _blob_run(384, 0, P.BC_PEC, steps)
    o = (384 - 64) // 2
    inner = slice(12, 52)
    ez_s = small.f["ez"][:, inner, inner]
    ez_b = big.f["ez"][:, o + 12:o + 52, o + 12:o + 52]
    refl = np.abs(ez_s - ez_b).max()
    assert refl < 1e-5, refl         # measured 2.3e-7 (pulse peak 1)
    # without the absorber the PEC walls reflect strongly
    pec = _blob_run(64, 0, P.BC_PEC, steps)
    assert np.abs(pec.f["ez"][:, inner, inner] - ez_b).max() > 1e3 * refl
