"""The transposed step and the sector gradient on the GPU.

* Transposition: ⟨F x, y⟩ = ⟨x, Fᵀ y⟩ with the GPU forward step F and the
  GPU transposed step, random x and y including CPML memories and wall
  values (FP32: relative gap ≤ 1e-5), on the split path and on a grid where
  the fused interior kernel runs.
* The transposed step against the oracle's (FP64) from the same λ, element
  by element (relative L2 ≤ 1e-4).
* The sector gradient (forward with checkpoints, reverse sweep with
  recomputation) against the oracle's reverse-mode gradient (≤ 1e-3 of the
  largest component), and the autograd.Function end to end.
"""
import math

import numpy as np
import pytest
import torch

from oracle import adjoint as OA
from oracle import problem as P
from oracle import yee as Y
from paper_2102_12978_amd import _lib as L
from paper_2102_12978_amd import workloads as W
from paper_2102_12978_amd.adjoint import Adjoint, SectorIntensity, SectorSensitivity
from tests import cases
from tests import gpu_cases as GC

pytestmark = pytest.mark.gpu

IDS = list(range(6)) + list(GC.PSI)


def _shapes(s):
    return {q: s.state_shape(q) for q in IDS if q < 6 or s.npml > 0}


def _dot(a, b):
    return sum(float(np.dot(a[q].astype(np.float64).ravel(), b[q].astype(np.float64).ravel()))
               for q in a)


def _small(bc=L.BC_CPML):
    w = W.Workload("adj_40x36", 40, 36, 12, 14.0, 25.0, 1, 12.0, 2.0, 6 if bc == L.BC_CPML else 0,
                   10, bc=bc)
    return w


@pytest.mark.parametrize("bc", [L.BC_PERIODIC, L.BC_PEC, L.BC_CPML])
@pytest.mark.parametrize("nsteps", [1, 3])
def test_dot_product_identity(bc, nsteps):
    w = _small(bc)
    s = GC.gpu_solver(w, kernel=L.KERNEL_SPLIT, bc=bc, inject=False)
    adj = Adjoint(s)
    rng = np.random.default_rng(7 + bc + nsteps)
    sh = _shapes(s)
    x = {q: rng.standard_normal(v).astype(np.float32) for q, v in sh.items()}
    y = {q: rng.standard_normal(v).astype(np.float32) for q, v in sh.items()}
    for q, v in x.items():
        s.set_state(q, v)
    s.step(nsteps)
    fx = {q: s.get_state(q) for q in sh}
    for q, v in y.items():
        adj.set_state(q, v)
    adj.transpose(nsteps)
    fty = {q: adj.get_state(q) for q in sh}
    lhs, rhs = _dot(fx, y), _dot(x, fty)
    gap = abs(lhs - rhs) / (abs(lhs) + abs(rhs))
    print(f"  <Fx,y> = {lhs:.8e}, <x,F^T y> = {rhs:.8e}, gap {gap:.1e}", flush=True)
    assert gap < 1e-5
    adj.close()
    s.close()


@pytest.mark.parametrize("bc", [L.BC_CPML, L.BC_PEC])
def test_dot_product_identity_fused_grid(bc):
    """parity_mid grid: the forward step runs the fused interior kernel, and
    the transposed step runs it too (negated S) with the transposed-CPML
    kernels on the frame around it."""
    w = W.parity_mid()
    s = GC.gpu_solver(w, kernel=L.KERNEL_FUSED, bc=bc, inject=False)
    adj = Adjoint(s)
    rng = np.random.default_rng(11)
    sh = _shapes(s)
    x = {q: rng.standard_normal(v).astype(np.float32) for q, v in sh.items()}
    y = {q: rng.standard_normal(v).astype(np.float32) for q, v in sh.items()}
    for q, v in x.items():
        s.set_state(q, v)
    s.step(2)
    fx = {q: s.get_state(q) for q in sh}
    for q, v in y.items():
        adj.set_state(q, v)
    adj.transpose(2)
    fty = {q: adj.get_state(q) for q in sh}
    lhs, rhs = _dot(fx, y), _dot(x, fty)
    gap = abs(lhs - rhs) / (abs(lhs) + abs(rhs))
    print(f"  gap {gap:.1e}", flush=True)
    assert gap < 1e-5
    adj.close()
    s.close()


@pytest.mark.parametrize("bc", [L.BC_CPML, L.BC_PEC])
def test_transpose_decomposition_matches_whole_grid_kernels(bc):
    """The transposed step on a fused-kernel context (interior kernel with
    negated S + transposed-CPML kernels on the frame) against the
    transposed-CPML kernels over the whole grid (split-kernel context), from
    the same seeded λ, three steps."""
    w = W.parity_mid()
    sf = GC.gpu_solver(w, kernel=L.KERNEL_FUSED, bc=bc, inject=False)
    ss = GC.gpu_solver(w, kernel=L.KERNEL_SPLIT, bc=bc, inject=False)
    af, as_ = Adjoint(sf), Adjoint(ss)
    rng = np.random.default_rng(31)
    sh = _shapes(sf)
    for q, v in sh.items():
        y = rng.standard_normal(v).astype(np.float32)
        af.set_state(q, y)
        as_.set_state(q, y)
    af.transpose(3)
    as_.transpose(3)
    worst = 0.0
    for q in sh:
        a, b = af.get_state(q).astype(np.float64), as_.get_state(q).astype(np.float64)
        rel = float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))
        worst = max(worst, rel)
    print(f"  fused-context vs whole-grid transpose: worst rel-L2 {worst:.1e}", flush=True)
    assert worst < 1e-6
    for x in (af, as_, sf, ss):
        x.close()


def _slab_to_full(arr, which, npml, nx, ny):
    if which in (L.PSI_EYX, L.PSI_EZX, L.PSI_HYX, L.PSI_HZX):
        full = np.zeros((arr.shape[0], ny, nx))
        full[:, :, :npml] = arr[:, :, :npml]
        full[:, :, nx - npml:] = arr[:, :, npml:]
    else:
        full = np.zeros((arr.shape[0], ny, nx))
        full[:, :npml, :] = arr[:, :npml, :]
        full[:, ny - npml:, :] = arr[:, npml:, :]
    return full


def test_transposed_step_matches_oracle():
    w = _small()
    s = GC.gpu_solver(w, kernel=L.KERNEL_SPLIT, inject=False)
    adj = Adjoint(s)
    g = cases.oracle_grid(w)
    cp = P.cpml_tables(g)
    rng = np.random.default_rng(3)
    lam = Y.zero_state(g)
    for q, c in enumerate(GC.COMPS):
        v = rng.standard_normal((g.nz, g.ny, g.nx)).astype(np.float32)
        adj.set_state(q, v)
        lam.f[c] = v.astype(np.float64)
    for q, name in GC.PSI.items():
        v = rng.standard_normal(s.state_shape(q)).astype(np.float32)
        adj.set_state(q, v)
        lam.psi[name] = _slab_to_full(v.astype(np.float64), q, g.npml, g.nx, g.ny)
    adj.transpose(2)
    for _ in range(2):
        OA.adjoint_step(lam, g, cp)
    GC.assert_parity([adj.get_state(q) for q in range(6)], [lam.f[c] for c in GC.COMPS],
                     "lambda fields")
    GC.assert_parity([adj.get_state(q) for q in GC.PSI],
                     [GC.psi_slab(lam.psi[n], q, g.npml, g.nx, g.ny) for q, n in GC.PSI.items()],
                     "lambda psi")
    adj.close()
    s.close()


def _grad_problem():
    """48×48, θ = 30°, m = 0, 16 sectors with seeded weights, 90 steps,
    window of the last 30, checkpoints every 25 steps (the window spans two
    segments, the last one short)."""
    w = W.Workload("adj_48_m0", 48, 48, 10, 12.0, 30.0, 0, 12.0, 2.0, 6, 90, ramp_periods=2.0,
                   extra={"sectors": 16, "checkpoint_every": 25})
    rng = np.random.default_rng(21)
    amp = 1.0 + 0.05 * rng.standard_normal(16)
    ph = 0.1 * rng.standard_normal(16)
    return w, amp, ph


def _target(ny, nx):
    jj, ii = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    r = np.hypot(ii - nx / 2.0, jj + 0.5 - ny / 2.0)
    return r < 9.0, 1e-3 * np.exp(-(r / 4.0) ** 2)


def test_gradient_matches_oracle():
    w, amp, ph = _grad_problem()
    sens = SectorSensitivity(w, window_begin=60)
    ibar = sens.intensity(amp, ph).astype(np.float64)
    region, target = _target(*ibar.shape)
    nreg = np.count_nonzero(region)
    dl = np.where(region, 2.0 * (ibar - target) / nreg, 0.0)
    ga, gp = sens.backward(dl)
    inf = sens.adj.info()
    print(f"  checkpoints {inf.checkpoints}, recomputed steps {inf.recompute_steps}", flush=True)
    assert inf.checkpoints == 4 and inf.recompute_steps == 40
    g = cases.oracle_grid(w)
    inj = cases.oracle_injector(w, amp=amp, phase=ph)
    loss, ibar_o, ga_o, gp_o, _ = OA.intensity_loss_grad(g, inj, w.steps, sens.plane, 60,
                                                         target, region)
    assert GC.rel_l2([ibar], [ibar_o]) < 1e-4
    scale = max(np.abs(ga_o).max(), np.abs(gp_o).max())
    err = max(np.abs(ga - ga_o).max(), np.abs(gp - gp_o).max()) / scale
    print(f"  sector gradient vs oracle: max error {err:.1e} of the largest component",
          flush=True)
    assert err < 1e-3
    # a second backward from the same forward gives the same gradient
    ga2, gp2 = sens.backward(dl)
    assert np.array_equal(ga, ga2) and np.array_equal(gp, gp2)
    sens.close()


def test_autograd_function():
    w, amp, ph = _grad_problem()
    sens = SectorSensitivity(w, window_begin=60)
    a = torch.tensor(amp, requires_grad=True)
    p = torch.tensor(ph, requires_grad=True)
    ibar = SectorIntensity.apply(a, p, sens)
    region, target = _target(*ibar.shape)
    reg = torch.from_numpy(region)
    loss = ((ibar - torch.from_numpy(target))[reg] ** 2).mean()
    loss.backward()
    dl = np.where(region, 2.0 * (ibar.detach().numpy() - target) / region.sum(), 0.0)
    ga, gp = sens.backward(dl)
    assert np.allclose(a.grad.numpy(), ga, rtol=1e-6, atol=1e-30)
    assert np.allclose(p.grad.numpy(), gp, rtol=1e-6, atol=1e-30)
    sens.close()


def _grad192_loss_grad(sens, amp, ph, A):
    from paper_2102_12978_amd.adjoint import central_lobe_target
    region, j0sq = central_lobe_target(sens)
    a = torch.tensor(amp, requires_grad=True)
    p = torch.tensor(ph, requires_grad=True)
    ibar = SectorIntensity.apply(a, p, sens)
    reg = torch.from_numpy(region)
    loss = ((ibar - A * torch.from_numpy(j0sq))[reg] ** 2).mean()
    loss.backward()
    return loss.item(), a.grad.numpy(), p.grad.numpy(), region, j0sq


def test_torch_reference_24():
    """24×24×20 copy of the differentiable workload (300 steps, 256 seed-2
    sector weights, loss against A J_0²): GPU adjoint vs torch.autograd
    through the pure-PyTorch FP64 forward."""
    from oracle import torch_ref as T
    from paper_2102_12978_amd.adjoint import on_axis
    w = W.grad24()
    amp, ph = W.sector_params(seed=2, sectors=256)
    sens = SectorSensitivity(w)
    print(f"[gpu case] {w.name}: {sens.steps} steps, window from {sens.window_begin}", flush=True)
    A = on_axis(sens.intensity(np.ones(256), np.zeros(256)).astype(np.float64))
    loss, ga, gp, region, j0sq = _grad192_loss_grad(sens, amp, ph, A)
    g = cases.oracle_grid(w)
    ref = T.TorchYee(g, cases.oracle_injector(w, amp=amp, phase=ph))
    a2 = torch.tensor(amp, requires_grad=True)
    p2 = torch.tensor(ph, requires_grad=True)
    ib2 = ref.intensity(a2, p2, sens.steps, sens.plane, sens.window_begin)
    reg = torch.from_numpy(region)
    loss2 = ((ib2 - A * torch.from_numpy(j0sq))[reg] ** 2).mean()
    loss2.backward()
    scale = max(a2.grad.abs().max().item(), p2.grad.abs().max().item())
    err = max(np.abs(ga - a2.grad.numpy()).max(), np.abs(gp - p2.grad.numpy()).max()) / scale
    print(f"  loss GPU {loss:.6e} vs torch {loss2.item():.6e}; gradient error {err:.1e}",
          flush=True)
    assert abs(loss - loss2.item()) <= 1e-4 * loss2.item()
    assert err < 1e-3
    sens.close()


def test_grad192_gradient_vs_finite_differences():
    """192×192×61, 1500 steps, checkpoints every 100: adjoint gradients at 8
    amplitudes and 8 phases (sectors 32 q + 5) against FP64 central
    differences (h = 1e-3) stored by tests/golden/make_grad192_fd.py."""
    import json
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "grad192_fd_gradient.json")
    fd = json.load(open(path))
    w = W.grad192()
    amp, ph = W.sector_params(seed=2, sectors=256)
    sens = SectorSensitivity(w)
    print(f"[gpu case] {w.name}: {sens.steps} steps, checkpoints every {sens.every}", flush=True)
    loss, ga, gp, _, _ = _grad192_loss_grad(sens, amp, ph, fd["A_on_axis"])
    inf = sens.adj.info()
    assert inf.checkpoints == 15 and inf.recompute_steps == 200
    sec = fd["sectors"]
    got = np.concatenate([ga[sec], gp[sec]])
    ref = np.concatenate([fd["grad_amp_fd"], fd["grad_phase_fd"]])
    err = np.abs(got - ref).max() / np.abs(ref).max()
    print(f"  loss {loss:.6e} (FP64 {fd['loss']:.6e}); max gradient error {err:.1e} of the "
          f"largest; per probe " + ", ".join(f"{x:.1e}" for x in np.abs(got - ref) /
                                             np.abs(ref)), flush=True)
    assert abs(loss - fd["loss"]) <= 1e-4 * fd["loss"]
    assert err < 1e-3
    sens.close()


def test_adjoint_refuses_calls_out_of_order_and_bad_arguments():
    """ESTATE: backward before a forward, a forward context without an
    antenna. EINVAL: empty runs, a window outside the run, a plane outside
    the grid, a dL/dI of the wrong size, a wrong sector count, a negative
    transpose count. The context stays usable after every refusal."""
    w = W.Workload("adj_120_m0", 120, 120, 10, 12.0, 30.0, 0, 40.0, 2.0, 6, 90,
                   ramp_periods=2.0, extra={"sectors": 16, "checkpoint_every": 25})
    sens = SectorSensitivity(w, window_begin=60)
    adj, s = sens.adj, sens.solver
    nxy = s.nx * s.ny

    def code(fn, *args):
        with pytest.raises(L.FdtdError) as e:
            fn(*args)
        return e.value.code

    assert code(adj.backward, np.zeros((s.ny, s.nx)), 16) == L.ESTATE
    assert code(adj.forward, 0, sens.plane, 0) == L.EINVAL
    assert code(adj.forward, 90, sens.plane, 90) == L.EINVAL
    assert code(adj.forward, 90, s.nz, 60) == L.EINVAL
    assert code(adj.forward, 90, -1, 60) == L.EINVAL
    assert code(adj.transpose, -1) == L.EINVAL
    ibar = sens.intensity(np.ones(16), np.zeros(16))
    assert ibar.shape == (s.ny, s.nx)
    assert code(adj.backward, np.zeros(nxy - 1), 16) == L.EINVAL
    assert code(adj.backward, np.zeros(nxy), 8) == L.EINVAL
    ga, gp = sens.backward(np.full((s.ny, s.nx), 1e-3))
    assert np.all(np.isfinite(ga)) and np.all(np.isfinite(gp)) and np.any(ga != 0)
    sens.close()
    # an adjoint on a context without an antenna cannot run its forward
    bare = GC.gpu_solver(w, inject=False)
    a2 = Adjoint(bare, 25)
    assert code(a2.forward, 90, bare.nz // 2, 60) == L.ESTATE
    a2.close()
    bare.close()


def test_adjoint_refuses_a_changed_antenna_and_outlives_its_context():
    """The checkpoints belong to the antenna of the last forward: after
    fdtd_set_sector_weights or fdtd_set_injector (here a smaller annulus)
    the backward refuses with ESTATE and changes nothing; a new forward makes
    it usable again, with the gradient of a fresh run bit for bit. Destroying
    the forward context first detaches the adjoint: its calls return ESTATE
    and it can still be destroyed."""
    w = W.Workload("adj_120_m0", 120, 120, 10, 12.0, 30.0, 0, 40.0, 2.0, 6, 90,
                   ramp_periods=2.0, extra={"sectors": 16, "checkpoint_every": 25})
    amp, ph = W.sector_params(seed=5, sectors=16)
    dl = np.full((120, 120), 1e-3)
    ref = SectorSensitivity(w, window_begin=60)
    ref.intensity(amp, ph)
    ga0, gp0 = ref.backward(dl)
    ref.close()

    sens = SectorSensitivity(w, window_begin=60)
    adj, s = sens.adj, sens.solver

    def code(fn, *args):
        with pytest.raises(L.FdtdError) as e:
            fn(*args)
        return e.value.code

    sens.intensity(amp, ph)
    s.set_sector_weights(np.ones(16), np.zeros(16))
    assert code(sens.backward, dl) == L.ESTATE
    sens.intensity(amp, ph)
    small = W.Workload("adj_120_small", 120, 120, 10, 12.0, 30.0, 0, 20.0, 2.0, 6, 90,
                       ramp_periods=2.0)
    s.set_workload_injector(small, sector_amp=np.ones(16), sector_phase=np.zeros(16))
    assert code(sens.backward, dl) == L.ESTATE
    s.set_workload_injector(w, sector_amp=np.ones(16), sector_phase=np.zeros(16))
    sens.intensity(amp, ph)
    ga, gp = sens.backward(dl)
    assert np.array_equal(ga, ga0) and np.array_equal(gp, gp0)
    # the forward context destroyed before its adjoint
    s.close()
    assert code(adj.forward, 90, 5, 60) == L.ESTATE
    assert code(adj.backward, dl, 16) == L.ESTATE
    assert code(adj.transpose, 1) == L.ESTATE
    assert code(adj.get_state, L.EX) == L.ESTATE
    adj.close()
    sens.adj = None
    sens.solver = None


def test_autograd_two_graphs_on_one_sensitivity():
    """Two SectorIntensity graphs on one sensitivity: the second forward
    replaces the checkpoints, so the first graph's backward runs its own
    forward again; both gradients equal those of single-graph runs."""
    w = W.Workload("adj_120_m0", 120, 120, 10, 12.0, 30.0, 0, 40.0, 2.0, 6, 90,
                   ramp_periods=2.0, extra={"sectors": 16, "checkpoint_every": 25})
    sens = SectorSensitivity(w, window_begin=60)
    pa = [W.sector_params(seed=q, sectors=16) for q in (7, 8)]

    def grad_of(a, p, sv):
        at = torch.tensor(a, requires_grad=True)
        pt = torch.tensor(p, requires_grad=True)
        return at, pt, (SectorIntensity.apply(at, pt, sv) ** 2).sum()

    singles = []
    for a, p in pa:
        at, pt, loss = grad_of(a, p, sens)
        loss.backward()
        singles.append((at.grad.numpy().copy(), pt.grad.numpy().copy()))
    g1 = grad_of(*pa[0], sens)
    g2 = grad_of(*pa[1], sens)
    g1[2].backward()
    g2[2].backward()
    for (at, pt, _), (ga, gp) in zip((g1, g2), singles):
        assert np.array_equal(at.grad.numpy(), ga) and np.array_equal(pt.grad.numpy(), gp)
    sens.close()
