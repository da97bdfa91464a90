"""Exact transpose of one oracle Yee step, and the gradient of an intensity loss.

TEST INFRASTRUCTURE (see ``oracle/__init__``).

The step of ``oracle.yee`` is linear in the state x = (E, H̃, ψ_E, ψ_H) plus
the antenna source, so reverse-mode differentiation is the transposed step run
backwards in time. Written from the forward definition term by term:

  forward term (E part):  ψ' = b ψ + c Δ,   E' = E + s·S_d·((1/κ) Δ + ψ'),  Δ = D_b H
  its transpose:          μ = s·S_d·λ_E',  λ_Δ = ((1/κ) + c) μ + c λ_ψ',
                          λ_ψ = b (μ + λ_ψ'),  λ_H += D_bᵀ λ_Δ = -D_f λ_Δ

(and the same with D_f / D_b swapped for the H part). Components held by the
PEC walls are not updated forward, so their terms are masked out here.

Gradient of a loss on the time-averaged intensity plane with respect to the
per-sector antenna weights w_s = a_s e^{iφ_s} (which multiply Ã, §4): with
G = Σ_n Σ_k λ(k) e^{iβ z(k)} T(t_n) accumulated at every antenna point,
dL/da_s = Σ_{pts∈s} Re{e^{iφ_s} Ã G} and dL/dφ_s = -Σ_{pts∈s} Im{w_s Ã G}.

Parity: pinned by the dot-product identity ⟨F x, y⟩ = ⟨x, Fᵀ y⟩ against the
forward step and by central finite differences of the full loss.
"""
import numpy as np

from . import problem as P
from . import yee as Y


def _adj_part(lam, g, cp, terms, comps, at_e):
    """Transpose of the E part (at_e) or H part of the forward step.

    ``lam`` holds λ for the output of that part and is overwritten with λ for
    its input."""
    s = dict(zip("xyz", g.s))
    # the differenced component's adjoint receives -D_f (λ_Δ) for an E part
    # (backward differences forward) and -D_b (λ_Δ) for an H part.
    diff_t = Y.fwd_diff if at_e else Y.back_diff
    new_psi = {}
    contrib = {}
    for comp in comps:
        held = Y.held_mask(g, comp)
        upd = (~held).astype(np.float64)[None, :, :]
        lam_out = lam.f[comp]
        for tgt, src, axis, sign, psi in terms:
            if tgt != comp:
                continue
            mu = upd * sign * s[axis] * lam_out
            if psi is None:
                lam_d = mu
            else:
                b, c, kinv = Y.cpml_coeffs(cp, axis, at_e)
                lp = lam.psi[psi]
                lam_d = upd * ((kinv + c) * mu + c * lp)
                new_psi[psi] = upd * b * (mu + lp) + (1.0 - upd) * lp
            contrib.setdefault(src, []).append(-diff_t(lam_d, axis, g.periodic_xy))
    for src, parts in contrib.items():
        lam.f[src] = lam.f[src] + sum(parts)
    lam.psi.update(new_psi)


def adjoint_h_part(lam, g, cp):
    _adj_part(lam, g, cp, Y.H_TERMS, Y.H_COMPS, at_e=False)


def adjoint_e_part(lam, g, cp):
    _adj_part(lam, g, cp, Y.E_TERMS, Y.E_COMPS, at_e=True)


def adjoint_step(lam: Y.State, g: P.Grid, cp: P.Cpml):
    """λ^n = Fᵀ λ^{n+1} for the source-free step F (H part reversed first)."""
    adjoint_h_part(lam, g, cp)
    adjoint_e_part(lam, g, cp)
    return lam


def inner(a: Y.State, b: Y.State):
    """Euclidean inner product over all fields and CPML memories."""
    s = sum(float(np.sum(a.f[c] * b.f[c])) for c in a.f)
    return s + sum(float(np.sum(a.psi[p] * b.psi[p])) for p in a.psi)


def _accumulate(G, lam, ant, comps, t):
    tf = P.time_factor(ant, t)
    for comp in comps:
        jj, ii = ant.idx[comp]
        if jj.size:
            vals = lam.f[comp][:, jj, ii]                       # [nz, npts]
            G[comp] += tf * np.sum(vals * ant.zphase[comp][:, None], axis=0)


def intensity_loss_grad(g: P.Grid, inj: P.Injector, nsteps, plane, window_begin,
                        target, region):
    """Forward run, L = mean_region (Ī - target)², and dL/d(a_s, φ_s).

    Ī = mean over steps n ≥ window_begin of E_y^{n+1}² on plane k = ``plane``.
    Returns (L, Ī, dL/da, dL/dφ, per-point G by component).
    """
    ant = P.build_antenna(g, inj)
    cp = P.cpml_tables(g)
    diag = Y.Diag(plane=plane, window_begin=window_begin)
    Y.run(g, nsteps, ant, diag=diag, record_ey_plane=True)
    ibar = diag.mean("ey2")
    nreg = float(np.count_nonzero(region))
    resid = np.where(region, ibar - target, 0.0)
    loss = float(np.sum(resid ** 2) / nreg)
    dl_di = 2.0 * resid / nreg
    planes = diag.planes
    count = diag.count
    lam = Y.zero_state(g)
    G = {c: np.zeros(len(ant.idx[c][0]), dtype=np.complex128) for c in ant.idx}
    for n in range(nsteps - 1, -1, -1):
        if n >= window_begin:
            e_y = planes[n - window_begin]
            lam.f["ey"][plane] += dl_di * 2.0 * e_y / count
        _accumulate(G, lam, ant, Y.H_COMPS, (n + 1.5) * g.dt)
        adjoint_h_part(lam, g, cp)
        _accumulate(G, lam, ant, Y.E_COMPS, (n + 1.0) * g.dt)
        adjoint_e_part(lam, g, cp)
    nsec = len(inj.sector_amp)
    ga = np.zeros(nsec)
    gp = np.zeros(nsec)
    for comp in ant.idx:
        sec = ant.sector[comp]
        if sec is None or sec.size == 0:
            continue
        a = np.asarray(inj.sector_amp)[sec]
        ph = np.asarray(inj.sector_phase)[sec]
        prod = ant.base[comp] * G[comp]
        np.add.at(ga, sec, np.real(np.exp(1j * ph) * prod))
        np.add.at(gp, sec, -np.imag(a * np.exp(1j * ph) * prod))
    return loss, ibar, ga, gp, G
