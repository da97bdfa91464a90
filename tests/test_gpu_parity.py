"""GPU parity: the HIP solver (through the C ABI) against the FP64 oracle.

Tolerance: relative L2 over all six field components ≤ 1e-4 (FP32 solver
against an FP64 reference on the same seeded inputs), and per component a
relative L2 and a max-abs bound against the component's own size (with a
floor; tests/gpu_cases.py states the bars and their derivation); the eight
CPML memories are compared the same way.
"""
import math

import numpy as np
import pytest

from oracle import problem as P
from oracle import yee as Y
from paper_2102_12978_amd import _lib as L
from paper_2102_12978_amd import workloads as W
from tests import cases
from tests import gpu_cases as GC

pytestmark = pytest.mark.gpu
TOL = 1e-4


def _compare(s, st, g, psi=True):
    rel = GC.assert_parity(s.fields(), [st.f[c] for c in GC.COMPS], "fields")
    if psi and g.bc == P.BC_CPML:
        gp, rp = [], []
        for which, name in GC.PSI.items():
            gp.append(s.get_state(which))
            rp.append(GC.psi_slab(st.psi[name], which, g.npml, g.nx, g.ny))
        GC.assert_parity(gp, rp, "psi")
    return rel


@pytest.mark.parametrize("kernel", [L.KERNEL_SPLIT, L.KERNEL_FUSED])
def test_cube32_forward(kernel):
    """32³, Δx = λ/16, θ = 10°, m = 0, annulus 12Δx, 8-cell CPML, 200 steps."""
    w = W.cube32()
    s = GC.gpu_solver(w, kernel=kernel)
    s.step(w.steps)
    g, st = GC.oracle_run(w, w.steps)
    _compare(s, st, g)
    s.close()


@pytest.mark.parametrize("kernel", [L.KERNEL_SPLIT, L.KERNEL_FUSED])
def test_gaussian_envelope(kernel):
    """The paper's Gaussian envelope f(t) = exp(-(t - T0)²/T²) with the phase
    referred to T0 (§4, zeroth-order approximation): 120×96, θ = 25°, m = 1,
    T = 2 periods, T0 = 3 periods, 84 steps through the peak."""
    w = W.parity_gauss()
    s = GC.gpu_solver(w, kernel=kernel)
    s.step(w.steps)
    g, st = GC.oracle_run(w, w.steps)
    _compare(s, st, g)
    s.close()


@pytest.mark.parametrize("rows,zchunk", [(4, 0), (8, 0), (4, 7), (8, 9)])
def test_fused_interior_frame_and_fixup(rows, zchunk):
    """300×150: three fused segments, ragged frame, z chunks that do not
    divide nz, 10-cell CPML, an antenna crossing interior and frame."""
    w = W.parity_mid()
    s = GC.gpu_solver(w, kernel=L.KERNEL_FUSED, rows=rows, zchunk=zchunk)
    s.step(w.steps)
    g, st = GC.oracle_run(w, w.steps)
    _compare(s, st, g)
    s.close()


@pytest.mark.parametrize("rows,zchunk", [(4, 0), (8, 5)])
def test_fused_partial_workgroup(rows, zchunk):
    """540×80: a full and a short group of x-adjacent wavefronts; halo values
    cross wavefronts through LDS inside a group and through memory between
    groups, with antenna points on both sides of the group boundary."""
    w = W.parity_wide()
    s = GC.gpu_solver(w, kernel=L.KERNEL_FUSED, rows=rows, zchunk=zchunk)
    s.step(w.steps)
    g, st = GC.oracle_run(w, w.steps)
    _compare(s, st, g)
    s.close()


def test_fused_partial_workgroup_random_start():
    """Random fields everywhere (walls zeroed) on the 540×80 grid, so every
    lane-0 / lane-63 halo value is nonzero from the first step."""
    w = W.parity_wide()
    w.steps = 12
    g, st0 = GC.random_start(w, P.BC_CPML, seed=6)
    s = GC.gpu_solver(w, kernel=L.KERNEL_FUSED, rows=4, zchunk=0)
    for i, c in enumerate(GC.COMPS):
        s.set_state(i, st0.f[c])
    s.step(w.steps)
    _, st = GC.oracle_run(w, w.steps, state=st0)
    _compare(s, st, g)
    s.close()


def test_ragged_small_grid():
    """100×72: too small for an interior, all cells go through the frame."""
    w = W.parity_small()
    for kernel in (L.KERNEL_SPLIT, L.KERNEL_FUSED):
        s = GC.gpu_solver(w, kernel=kernel)
        s.step(w.steps)
        g, st = GC.oracle_run(w, w.steps)
        _compare(s, st, g)
        s.close()


@pytest.mark.parametrize("bc", [P.BC_PERIODIC, P.BC_PEC])
@pytest.mark.parametrize("kernel", [L.KERNEL_SPLIT, L.KERNEL_FUSED])
def test_random_start_no_source(bc, kernel):
    """Seed-0 U(-1,1) fields, no source: periodic box (the 32³ random run)
    and PEC walls. Checks the fields, the energy invariant and div H."""
    w = W.cube32()
    g, st0 = GC.random_start(w, bc)
    s = GC.gpu_solver(w, kernel=kernel, bc=bc, inject=False)
    for i, c in enumerate(GC.COMPS):
        s.set_state(i, st0.f[c])
    s.set_diagnostics(-1, 0, L.DIAG_ENERGY)
    dh0 = Y.div_h(st0, g)
    st = st0.copy()
    cp = P.cpml_tables(g)
    w_ref = []
    energies = []
    for _ in range(w.steps):
        w_ref.append(Y.step(st, g, cp, None, want_energy=True))
        s.step(1)
        energies.append(s.energy())
    _compare(s, st, g, psi=False)
    w_ref = np.array(w_ref)
    energies = np.array(energies)
    drift = np.abs(energies - energies[0]).max() / abs(energies[0])
    print(f"  energy drift (FP32 solver) = {drift:.2e}; oracle drift = "
          f"{np.abs(w_ref - w_ref[0]).max() / abs(w_ref[0]):.1e}", flush=True)
    assert drift < 1e-5
    assert np.abs(energies - w_ref).max() / abs(w_ref[0]) < 1e-5
    gst = Y.zero_state(g)
    for i, c in enumerate(GC.COMPS):
        gst.f[c] = s.get_state(i).astype(np.float64)
    ddiv = np.abs(Y.div_h(gst, g) - dh0).max()
    print(f"  max |div H - div H0| = {ddiv:.2e}", flush=True)
    assert ddiv < 1e-4
    s.close()


def test_random_start_with_source_and_cpml():
    """Random start (walls zeroed) plus the antenna and CPML: the general
    state including nonzero CPML memories from the first step."""
    w = W.parity_mid()
    g, st0 = GC.random_start(w, P.BC_CPML, seed=4)
    s = GC.gpu_solver(w, kernel=L.KERNEL_FUSED)
    for i, c in enumerate(GC.COMPS):
        s.set_state(i, st0.f[c])
    s.step(w.steps)
    _, st = GC.oracle_run(w, w.steps, state=st0)
    _compare(s, st, g)
    s.close()


def test_plane_diagnostics_and_energy():
    """⟨E_x²⟩, ⟨E_y²⟩, ⟨E_z²⟩ on the mid plane over a window, and W^n."""
    w = W.parity_mid()
    g = cases.oracle_grid(w)
    plane, wb = g.nz // 2, 25
    s = GC.gpu_solver(w, kernel=L.KERNEL_FUSED, rows=4, zchunk=9)
    s.set_diagnostics(plane, wb, L.DIAG_EX2 | L.DIAG_EY2 | L.DIAG_EZ2 | L.DIAG_ENERGY)
    s.step(w.steps)
    d = Y.Diag(plane=plane, window_begin=wb)
    _, st = GC.oracle_run(w, w.steps, diag=d, energy=True)
    assert s.fluence_count() == d.count == w.steps - wb
    for q, key in ((L.DIAG_EX2, "ex2"), (L.DIAG_EY2, "ey2"), (L.DIAG_EZ2, "ez2")):
        rel = GC.rel_l2([s.fluence(q)], [d.mean(key)])
        print(f"  {key} rel-L2 = {rel:.2e}", flush=True)
        assert rel <= TOL
    e = s.energy()
    print(f"  energy {e:.9e} vs {d.energy[-1]:.9e}", flush=True)
    assert abs(e - d.energy[-1]) <= 1e-4 * abs(d.energy[-1])
    s.close()


def test_divergence_reported():
    """A non-finite value planted (from the host) on the diagnostic plane
    makes both readbacks report FDTD_EUNSTABLE instead of returning NaN."""
    w = W.parity_small()
    g = cases.oracle_grid(w)
    plane = g.nz // 2
    s = GC.gpu_solver(w, kernel=L.KERNEL_FUSED, rows=4, zchunk=0)
    s.set_diagnostics(plane, 0, L.DIAG_EY2 | L.DIAG_ENERGY)
    s.step(2)
    assert np.isfinite(s.fluence(L.DIAG_EY2)).all() and np.isfinite(s.energy())
    ey = s.get_state(L.EY)
    ey[plane, g.ny // 2, g.nx // 2] = np.nan
    s.set_state(L.EY, ey)
    s.step(1)
    for read in (lambda: s.fluence(L.DIAG_EY2), s.energy):
        with pytest.raises(L.FdtdError) as e:
            read()
        assert e.value.code == L.EUNSTABLE
    s.close()


def test_fused_equals_split():
    """The fused interior kernel forms every cell, its segment-boundary
    columns included, with the split kernels' expressions: the states agree
    bit for bit (fields and CPML memories)."""
    w = W.parity_mid()
    a = GC.gpu_solver(w, kernel=L.KERNEL_SPLIT)
    b = GC.gpu_solver(w, kernel=L.KERNEL_FUSED, rows=8, zchunk=0)
    c = GC.gpu_solver(w, kernel=L.KERNEL_FUSED, rows=4, zchunk=5)
    for s in (a, b, c):
        s.step(w.steps)
    for which in list(range(6)) + list(GC.PSI):
        ref = a.get_state(which).view(np.uint32)
        for s in (b, c):
            bad = int(np.count_nonzero(s.get_state(which).view(np.uint32) != ref))
            print(f"  array {which}: {bad} cells differ", flush=True) if bad else None
            assert bad == 0
    for s in (a, b, c):
        s.close()


def test_state_roundtrip_and_reset():
    w = W.parity_small()
    s = GC.gpu_solver(w, kernel=L.KERNEL_FUSED)
    rng = np.random.default_rng(5)
    for which in list(range(6)) + list(GC.PSI):
        a = rng.standard_normal(s.state_shape(which)).astype(np.float32)
        s.set_state(which, a)
        assert np.array_equal(s.get_state(which), a)
    s.reset()
    assert s.info().step == 0
    assert all(np.count_nonzero(s.get_state(c)) == 0 for c in range(6))
    s.close()


def test_autotune_leaves_state_alone():
    """Autotune between steps 20 and 21: the run then matches the oracle, and
    an untuned run bit for bit (every tile, frame and time-block choice gives
    the same bits), fields and CPML memories."""
    w = W.parity_mid()
    s = GC.gpu_solver(w, kernel=L.KERNEL_FUSED)
    r = GC.gpu_solver(w, kernel=L.KERNEL_FUSED)
    s.step(20)
    rows, zc = s.autotune(2)
    inf = s.info()
    print(f"  autotune picked rows={rows} zchunk={zc} time_block={inf.time_block} "
          f"tb_rows={inf.tb_rows} tb_zchunk={inf.tb_zchunk}", flush=True)
    assert rows in (4, 8)
    s.step(w.steps - 20)
    r.step(w.steps)
    for q in list(range(6)) + (list(GC.PSI) if s.npml > 0 else []):
        a, b = s.get_state(q), r.get_state(q)
        assert np.array_equal(a.view(np.uint32), b.view(np.uint32)), f"array {q}"
    g, st = GC.oracle_run(w, w.steps)
    _compare(s, st, g)
    s.close()
    r.close()


def test_z_misfit_needs_the_flag_and_matches_the_oracle():
    """A box three planes longer than the whole-period fit (a fractional
    number of axial periods): the antenna is refused without
    FDTD_INJ_ALLOW_Z_MISFIT, and with it the run (the injected phase jumps at
    the z wrap) matches the oracle on the same box."""
    from paper_2102_12978_amd.solver import Solver
    w = W.parity_small()
    nz_fit, dz = P.fit_periodic_z(W.WAVELENGTH, w.theta, w.dx, w.nz_hint)
    nz = nz_fit + 3
    args, kw = Solver.workload_grid_args(w)
    s = Solver(w.nx, w.ny, nz, w.dx, w.dx, dz, kernel=L.KERNEL_FUSED, **kw)
    with pytest.raises(L.FdtdError) as e:
        s.set_workload_injector(w)
    assert e.value.code == L.EINVAL and "axial periods" in str(e.value)
    s.set_workload_injector(w, allow_z_misfit=True)
    print(f"[gpu case] {w.name}: nz {nz} instead of {nz_fit}", flush=True)
    s.step(w.steps)
    g = cases.oracle_grid(w, nz=nz, dz=dz)
    ant = P.build_antenna(g, cases.oracle_injector(w))
    st = Y.run(g, w.steps, ant)
    _compare(s, st, g)
    s.close()


@pytest.mark.parametrize("nx,ny,nz,bc,npml", [(2, 2, 1, P.BC_PERIODIC, 0), (2, 2, 1, P.BC_PEC, 0),
                                             (3, 5, 2, P.BC_PEC, 0), (4, 4, 1, P.BC_CPML, 1),
                                             (5, 3, 2, P.BC_CPML, 1)])
def test_degenerate_grids(nx, ny, nz, bc, npml):
    """The smallest grids the library accepts (2×2×1; one-cell CPML on
    4 and 3 cells; one plane, so the z neighbours are the plane itself):
    no interior, the split kernels take every cell. A zero-step call changes
    nothing, a negative one is refused, and seven steps from a seeded random
    start match the oracle, CPML memories included."""
    from paper_2102_12978_amd.solver import Solver
    w = W.Workload(f"tiny_{nx}x{ny}x{nz}", nx, ny, nz, 16.0, 10.0, 0, 1.0, 0.5, npml, 7, bc=bc)
    g = cases.oracle_grid(w, bc=bc, nz=nz, dz=w.dx)
    st = Y.zero_state(g)
    for c, a in zip(GC.COMPS, W.random_fields((nz, ny, nx), 4)):
        st.f[c] = a.astype(np.float32).astype(np.float64)
    if bc != P.BC_PERIODIC:
        for c in ("ex", "ey", "ez"):
            st.f[c][:, Y.held_mask(g, c)] = 0.0
    print(f"[gpu case] {w.name} bc={bc} npml={npml}", flush=True)
    s = Solver(nx, ny, nz, w.dx, w.dx, w.dx, courant=w.courant, bc=bc, cpml_cells=npml,
               grade=w.grade, sigma_scale=w.sigma_scale, kappa_max=w.kappa_max,
               alpha_max=w.alpha_max, kernel=L.KERNEL_FUSED)
    assert s.info().interior_cells == 0
    for i, c in enumerate(GC.COMPS):
        s.set_state(i, st.f[c].astype(np.float32))
    before = [s.get_state(i) for i in range(6)]
    s.step(0)
    assert s.info().step == 0
    assert all(np.array_equal(b, s.get_state(i)) for i, b in enumerate(before))
    with pytest.raises(L.FdtdError) as e:
        s.step(-1)
    assert e.value.code == L.EINVAL
    cp = P.cpml_tables(g)
    for _ in range(7):
        Y.step(st, g, cp, None)
    s.step(7)
    assert s.info().step == 7
    _compare(s, st, g, psi=npml > 0)
    s.close()


def test_source_linearity_on_gpu():
    w = W.parity_small()
    w.steps = 30
    a = GC.gpu_solver(w)
    w2 = W.parity_small()
    w2.steps = 30
    w2.e0 = 2.0
    b = GC.gpu_solver(w2)
    a.step(30)
    b.step(30)
    rel = GC.rel_l2(b.fields(), [2.0 * x.astype(np.float64) for x in a.fields()])
    assert rel < 1e-6
    a.close()
    b.close()


@pytest.mark.parametrize("xalign,rows,zchunk,frows", [(32, 4, 0, 2), (64, 4, 7, 4), (64, 8, 9, 2),
                                                      (32, 8, 16, 4)])
def test_fused_frame(xalign, rows, zchunk, frows):
    """The frame stepped by the fused boundary-tile kernel (one launch over
    the 64 x 4 tiles that hold frame cells): 300×150, antenna across interior
    and frame, z chunks that do not divide nz; against the oracle (fields and
    CPML memories) and against the split-kernel frame."""
    w = W.parity_mid()
    s = GC.gpu_solver(w, kernel=L.KERNEL_FUSED, rows=rows, zchunk=zchunk)
    s.set_frame(L.FRAME_FUSED, xalign, frows)
    inf = s.info()
    assert inf.frame == L.FRAME_FUSED and inf.xalign == xalign and inf.frame_rows == frows
    s.step(w.steps)
    g, st = GC.oracle_run(w, w.steps)
    _compare(s, st, g)
    r = GC.gpu_solver(w, kernel=L.KERNEL_FUSED, rows=rows, zchunk=zchunk)
    r.step(w.steps)
    rel = GC.rel_l2(s.fields(), [x.astype(np.float64) for x in r.fields()])
    print(f"  fused frame vs split frame rel-L2 = {rel:.2e}", flush=True)
    assert rel < 1e-5
    s.close()
    r.close()


@pytest.mark.parametrize("maker", [W.cube32, W.parity_small, W.parity_gauss])
def test_fused_frame_small_grids(maker):
    """Grids with no interior or a small one: the fused frame covers the
    whole grid or a ragged ring (PEC walls, CPML corners, lanes past nx)."""
    w = maker()
    s = GC.gpu_solver(w, kernel=L.KERNEL_FUSED)
    s.set_frame(L.FRAME_FUSED, 64, 4 if maker is W.cube32 else 2)
    s.step(w.steps)
    g, st = GC.oracle_run(w, w.steps)
    _compare(s, st, g)
    s.close()


def test_fused_frame_diagnostics_and_energy():
    w = W.parity_mid()
    g = cases.oracle_grid(w)
    plane, wb = g.nz // 2, 25
    s = GC.gpu_solver(w, kernel=L.KERNEL_FUSED, rows=4, zchunk=9)
    s.set_frame(L.FRAME_FUSED, 64)
    s.set_diagnostics(plane, wb, L.DIAG_EX2 | L.DIAG_EY2 | L.DIAG_EZ2 | L.DIAG_ENERGY)
    s.step(w.steps)
    d = Y.Diag(plane=plane, window_begin=wb)
    _, st = GC.oracle_run(w, w.steps, diag=d, energy=True)
    for q, key in ((L.DIAG_EX2, "ex2"), (L.DIAG_EY2, "ey2"), (L.DIAG_EZ2, "ez2")):
        rel = GC.rel_l2([s.fluence(q)], [d.mean(key)])
        print(f"  {key} rel-L2 = {rel:.2e}", flush=True)
        assert rel <= TOL
    e = s.energy()
    print(f"  energy {e:.9e} vs {d.energy[-1]:.9e}", flush=True)
    assert abs(e - d.energy[-1]) <= 1e-4 * abs(d.energy[-1])
    s.close()


@pytest.mark.parametrize("pol,order", [(L.POL_Y_TE, 1), (L.POL_Z_TE, 0), (L.POL_X_TM, 2),
                                       (L.POL_Y_TM, 1), (L.POL_Z_TM, 0), (L.POL_Z_TE, 2)])
def test_polarisations(pol, order):
    """The other potentials and pairings of §3.1 (Π_y, Π_z; TE and TM),
    including the m = 0 azimuthal (Π_z TE) and radial (Π_z TM) beams, on the
    300×150 grid with the antenna across interior and frame."""
    from dataclasses import replace
    w = replace(W.parity_mid(), polarization=pol, order=order,
                name=f"p_300x150x24_pol{pol}_m{order}")
    s = GC.gpu_solver(w, kernel=L.KERNEL_FUSED, rows=4, zchunk=7)
    s.step(w.steps)
    g, st = GC.oracle_run(w, w.steps)
    _compare(s, st, g)
    s.close()


def test_forward_calls_refuse_bad_arguments():
    """Every refusal is an error code with a message and changes nothing:
    diagnostics outside the grid or with unknown bits, fluence and state
    buffers of the wrong length or kind, sector weights without sectors or
    of the wrong count, the energy before it was enabled."""
    import ctypes
    w = W.parity_small()
    s = GC.gpu_solver(w, kernel=L.KERNEL_FUSED)
    lib, ctx = s._lib, s._ctx

    def code(fn, *args):
        with pytest.raises(L.FdtdError) as e:
            fn(*args)
        assert str(e.value)
        return e.value.code

    assert code(s.set_diagnostics, s.nz, 0, L.DIAG_EY2) == L.EINVAL
    assert code(s.set_diagnostics, -2, 0, 0) == L.EINVAL
    assert code(s.set_diagnostics, 0, -1, L.DIAG_EY2) == L.EINVAL
    assert code(s.set_diagnostics, 0, 0, 1 << 4) == L.EINVAL
    assert code(s.set_diagnostics, -1, 0, L.DIAG_EY2) == L.EINVAL
    assert code(s.energy) == L.ESTATE
    s.set_diagnostics(s.nz // 2, 0, L.DIAG_EY2)
    s.step(3)
    small = np.empty(s.nx * s.ny - 1, dtype=np.float32)
    p = small.ctypes.data_as(L.c_float_p)
    assert lib.fdtd_fluence(ctx, L.DIAG_EY2, p, small.size) == L.EINVAL
    assert lib.fdtd_fluence(ctx, 3, p, s.nx * s.ny) == L.EINVAL
    assert lib.fdtd_get_state(ctx, L.EY, p, small.size) == L.EINVAL
    assert lib.fdtd_get_state(ctx, 99, p, small.size) == L.EINVAL
    assert lib.fdtd_set_state(ctx, L.EY, p, small.size) == L.EINVAL
    assert code(s.set_sector_weights, np.ones(4), np.zeros(4)) == L.EINVAL
    # the run goes on as if nothing had been asked
    ref = GC.gpu_solver(w, kernel=L.KERNEL_FUSED)
    ref.set_diagnostics(s.nz // 2, 0, L.DIAG_EY2)
    ref.step(3)
    s.step(4)
    ref.step(4)
    assert all(np.array_equal(a, b) for a, b in zip(s.fields(), ref.fields()))
    assert np.array_equal(s.fluence(L.DIAG_EY2), ref.fluence(L.DIAG_EY2))
    s.close()
    ref.close()
    bare = GC.gpu_solver(w, kernel=L.KERNEL_FUSED, inject=False)
    assert code(bare.set_sector_weights, np.ones(4), np.zeros(4)) == L.ESTATE
    bare.close()
