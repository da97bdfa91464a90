"""Pins of the oracle's transposed step and intensity-loss gradient — CPU only.

The transpose is checked against the forward step by the dot-product identity
⟨F x, y⟩ = ⟨x, Fᵀ y⟩ (random x, y including CPML memories and wall values),
and the full gradient against central finite differences of the loss.
"""
import math

import numpy as np
import pytest

from oracle import adjoint as A
from oracle import problem as P
from oracle import yee as Y


def _rand_state(g, rng):
    st = Y.zero_state(g)
    for c in st.f:
        st.f[c] = rng.standard_normal(st.f[c].shape)
    for p in st.psi:
        st.psi[p] = rng.standard_normal(st.psi[p].shape)
    return st


@pytest.mark.parametrize("bc,npml", [(P.BC_PERIODIC, 0), (P.BC_PEC, 0), (P.BC_CPML, 4)])
@pytest.mark.parametrize("nsteps", [1, 4])
def test_dot_product_identity(bc, npml, nsteps):
    g = P.Grid(20, 16, 6, 1.0, 1.1, 1.0154, courant=0.5, bc=bc, npml=npml,
               grade=3.0, sigma_scale=1.0, kappa_max=1.7, alpha_max=0.05)
    g.validate()
    cp = P.cpml_tables(g)
    rng = np.random.default_rng(42 + npml + nsteps)
    x = _rand_state(g, rng)
    y = _rand_state(g, rng)
    fx = x.copy()
    for _ in range(nsteps):
        Y.step(fx, g, cp)
    fty = y.copy()
    for _ in range(nsteps):
        A.adjoint_step(fty, g, cp)
    lhs = A.inner(fx, y)
    rhs = A.inner(x, fty)
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + abs(rhs)), (lhs, rhs)


def _tiny_problem(nsec=16):
    ns = 8.0
    theta = math.radians(30.0)
    dx = 800e-9 / ns
    nz, dz = P.fit_periodic_z(800e-9, theta, dx, 9)
    g = P.Grid(24, 24, nz, dx, dx, dz, courant=0.5, bc=P.BC_CPML, npml=4,
               grade=3.0, sigma_scale=1.0, kappa_max=1.0, alpha_max=0.1 * 2 * math.pi / ns)
    rng = np.random.default_rng(9)
    amp = 1.0 + 0.05 * rng.standard_normal(nsec)
    ph = 0.1 * rng.standard_normal(nsec)
    inj = P.Injector(800e-9, theta, 0, 1.0, 8 * dx, 2 * dx, ramp_kind=P.RAMP_SIN2,
                     ramp_a=3 * 800e-9 / P.C_LIGHT, sector_amp=amp, sector_phase=ph)
    i = np.arange(g.nx)
    r = np.hypot(i[None, :] - g.nx / 2, (np.arange(g.ny)[:, None] + 0.5) - g.ny / 2)
    region = r < 6.0
    target = 0.05 * np.exp(-(r / 3.0) ** 2)
    return g, inj, region, target


def test_gradient_matches_central_differences():
    g, inj, region, target = _tiny_problem()
    nsteps, wb, plane = 60, 40, g.nz // 2
    loss, _, ga, gp, _ = A.intensity_loss_grad(g, inj, nsteps, plane, wb, target, region)
    assert np.abs(ga).max() > 0 and np.abs(gp).max() > 0
    h = 1e-4

    def loss_at(amp, ph):
        inj2 = P.Injector(**{**inj.__dict__, "sector_amp": amp, "sector_phase": ph})
        ant = P.build_antenna(g, inj2)
        d = Y.Diag(plane=plane, window_begin=wb)
        Y.run(g, nsteps, ant, diag=d)
        res = np.where(region, d.mean("ey2") - target, 0.0)
        return float(np.sum(res ** 2) / np.count_nonzero(region))

    assert abs(loss_at(inj.sector_amp, inj.sector_phase) - loss) < 1e-15 + 1e-12 * loss
    for s in (0, 3, 7, 12):
        e = np.zeros_like(inj.sector_amp)
        e[s] = h
        fd_a = (loss_at(inj.sector_amp + e, inj.sector_phase)
                - loss_at(inj.sector_amp - e, inj.sector_phase)) / (2 * h)
        fd_p = (loss_at(inj.sector_amp, inj.sector_phase + e)
                - loss_at(inj.sector_amp, inj.sector_phase - e)) / (2 * h)
        scale = np.abs(ga).max() + np.abs(gp).max()
        assert abs(fd_a - ga[s]) < 1e-6 * scale, (s, fd_a, ga[s])
        assert abs(fd_p - gp[s]) < 1e-6 * scale, (s, fd_p, gp[s])
