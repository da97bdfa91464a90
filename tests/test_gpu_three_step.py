"""Three-step kernel over the whole grid (fdtd_set_time_block(ctx, 3, ...)).

Every cell, walls and CPML included, is computed with the one-step kernels'
expressions in the same order, so a three-step run must equal a one-step
run bit for bit: fields, CPML memories and the plane sums. Step counts that
are not multiples of three end with a pair or a single step. The cases
cross several 58-cell tiles and row groups (interior, x boundary, y
boundary and corner launches), z chunks that do and do not divide nz,
sources, CPML and PEC walls, seeded random starts, the smallest grids the
library accepts and the 768x768x255 benchmark grid; two cases are also
checked against the FP64 oracle."""
from dataclasses import replace

import numpy as np
import pytest

from paper_2102_12978_amd import _lib as L
from paper_2102_12978_amd import workloads as W
from tests import cases
from tests import gpu_cases as GC

pytestmark = pytest.mark.gpu


def _solvers(w, rows, zchunk, inject=True, bc=None):
    one = GC.gpu_solver(w, kernel=L.KERNEL_FUSED, bc=bc, rows=4, zchunk=0, inject=inject)
    three = GC.gpu_solver(w, kernel=L.KERNEL_FUSED, bc=bc, rows=4, zchunk=0, inject=inject)
    three.set_time_block(3, rows, zchunk)
    assert three.info().time_block == 3
    return one, three


def _arrays(s):
    return list(range(6)) + (list(GC.PSI) if s.npml > 0 else [])


def _assert_identical(one, other, label):
    for q in _arrays(one):
        a, b = one.get_state(q), other.get_state(q)
        bad = np.count_nonzero(a.view(np.uint32) != b.view(np.uint32))
        if bad:
            idx = np.argwhere(a.view(np.uint32) != b.view(np.uint32))[:4]
            print(f"  {label}: array {q}: {bad} cells differ, first {idx.tolist()}", flush=True)
        assert bad == 0, f"{label}: array {q}"


def _random_start(solvers, seed):
    rng = np.random.default_rng(seed)
    s0 = solvers[0]
    for q in _arrays(s0):
        a = rng.uniform(-1.0, 1.0, size=s0.state_shape(q)).astype(np.float32)
        if q in (L.EX, L.EY, L.EZ):
            # E held on the x = 0 / y = 0 walls
            if q in (L.EY, L.EZ):
                a[:, :, 0] = 0.0
            if q in (L.EX, L.EZ):
                a[:, 0, :] = 0.0
        for s in solvers:
            s.set_state(q, a)


@pytest.mark.parametrize("rows,zchunk,steps", [(4, 0, 39), (2, 0, 41), (4, 5, 40), (2, 7, 13),
                                                (4, 16, 3), (2, 4, 2)])
def test_bit_identical_with_source(rows, zchunk, steps):
    w = W.parity_mid()
    one, three = _solvers(w, rows, zchunk)
    g = cases.oracle_grid(w)
    for s in (one, three):
        s.set_diagnostics(g.nz // 2, 5, L.DIAG_EX2 | L.DIAG_EY2 | L.DIAG_EZ2)
        s.step(steps)
    assert three.info().step == steps
    _assert_identical(one, three, f"rows={rows} zchunk={zchunk} steps={steps}")
    assert one.fluence_count() == three.fluence_count() == max(0, steps - 5)
    for q in (L.DIAG_EX2, L.DIAG_EY2, L.DIAG_EZ2):
        assert np.array_equal(one.fluence(q), three.fluence(q))
    one.close()
    three.close()


@pytest.mark.parametrize("maker,rows,zchunk", [(W.parity_wide, 4, 5), (W.parity_wide, 2, 0),
                                               (W.grad192, 4, 16), (W.parity_gauss, 2, 3)])
def test_bit_identical_random_start(maker, rows, zchunk):
    w = maker()
    one, three = _solvers(w, rows, zchunk)
    _random_start((one, three), seed=17)
    for s in (one, three):
        s.step(6)
    _assert_identical(one, three, f"{w.name} rows={rows} zchunk={zchunk}")
    # and on from there: a triple and a single step
    for s in (one, three):
        s.step(4)
    _assert_identical(one, three, f"{w.name} +4 steps")
    one.close()
    three.close()


def test_bit_identical_pec_walls():
    """PEC walls instead of CPML (no memories; E held on the x = 0 / y = 0
    walls): random start, antenna on, 7 steps (two triples and a single)."""
    w = W.parity_mid()
    one, three = _solvers(w, 4, 9, bc=L.BC_PEC)
    assert three.npml == 0 and three.info().time_block == 3
    _random_start((one, three), seed=5)
    for s in (one, three):
        s.step(7)
    _assert_identical(one, three, "PEC walls")
    one.close()
    three.close()


def test_against_oracle():
    w = W.parity_mid()
    s = GC.gpu_solver(w, kernel=L.KERNEL_FUSED, rows=4, zchunk=0)
    s.set_time_block(3, 4, 0)
    s.step(w.steps)
    g, st = GC.oracle_run(w, w.steps)
    GC.assert_parity(s.fields(), [st.f[c] for c in GC.COMPS], f"three-step {w.steps} steps")
    s.close()


@pytest.mark.parametrize("rows,zchunk", [(2, 0), (4, 5)])
def test_thick_antenna_fills_tiles(rows, zchunk):
    """An annulus 38 cells thick reaching the x- and y-boundary tiles: whole
    tiles take the source on every lane and row of every stage. The
    three-step run equals the one-step run bit for bit, and (rows 2) the
    FP64 oracle within the parity bars."""
    w = W.parity_thick()
    one, three = _solvers(w, rows, zchunk)
    assert one.info().n_slots > 10000
    for s in (one, three):
        s.step(w.steps)
    _assert_identical(one, three, f"thick antenna rows={rows} zchunk={zchunk}")
    if rows == 2:
        g, st = GC.oracle_run(w, w.steps)
        GC.assert_parity(three.fields(), [st.f[c] for c in GC.COMPS], "thick antenna, three-step")
    one.close()
    three.close()


@pytest.mark.parametrize("pol,order,rows", [(L.POL_Y_TE, 1, 2), (L.POL_Z_TE, 0, 4),
                                            (L.POL_X_TM, 2, 2), (L.POL_Y_TM, 1, 4),
                                            (L.POL_Z_TM, 0, 2), (L.POL_Z_TE, 2, 4)])
def test_polarisations_bit_identical(pol, order, rows):
    """The other potentials and pairings of §3.1 put their sources on other
    components: every component's amplitude goes through the LDS copy at
    every stage, and the three-step run equals the one-step run bit for
    bit."""
    w = replace(W.parity_mid(), polarization=pol, order=order,
                name=f"p_300x150x24_pol{pol}_m{order}")
    one, three = _solvers(w, rows, 5)
    for s in (one, three):
        s.step(w.steps)
    _assert_identical(one, three, f"polarisation {pol} m={order} rows={rows}")
    one.close()
    three.close()


def test_fallbacks():
    """Energy diagnostic on and the split kernel: triples run as single
    steps, with the same results; a grid with no wall-free tile runs triples
    through the boundary launches alone."""
    w = W.parity_mid()
    one, three = _solvers(w, 4, 0)
    g = cases.oracle_grid(w)
    for s in (one, three):
        s.set_diagnostics(g.nz // 2, 0, L.DIAG_EY2 | L.DIAG_ENERGY)
        s.step(10)
    assert one.energy() == three.energy()
    _assert_identical(one, three, "energy on")
    one.close()
    three.close()
    w0 = W.cube32()
    w0.steps = 12
    one, three = _solvers(w0, 4, 0)
    assert three.info().interior_cells == 0 and three.info().time_block == 3
    for s in (one, three):
        s.step(w0.steps)
    _assert_identical(one, three, "small grid")
    one.close()
    three.close()
    s = GC.gpu_solver(w, kernel=L.KERNEL_SPLIT)
    s.set_time_block(3, 2, 0)
    r = GC.gpu_solver(w, kernel=L.KERNEL_SPLIT)
    for x in (s, r):
        x.step(6)
    _assert_identical(r, s, "split kernel")
    s.close()
    r.close()


def test_benchmark_grid_bit_identical():
    """768x768x255 (the benchmark grid): random fields and CPML memories,
    antenna on, six steps with the three-step kernel (4 rows, z chunks of
    32) against six one-step launches."""
    w = W.grid768()
    one, three = _solvers(w, 4, 32)
    print(f"  {w.name}: random state", flush=True)
    _random_start((one, three), seed=23)
    for s in (one, three):
        s.step(6)
    _assert_identical(one, three, "768 grid")
    one.close()
    three.close()


@pytest.mark.parametrize("nx,ny,nz,bc,npml", [(2, 2, 1, L.BC_PEC, 0), (3, 5, 2, L.BC_PEC, 0),
                                             (4, 4, 1, L.BC_CPML, 1), (5, 3, 2, L.BC_CPML, 1),
                                             (59, 17, 3, L.BC_CPML, 2), (130, 70, 5, L.BC_CPML, 3)])
def test_bit_identical_small_and_ragged_grids(nx, ny, nz, bc, npml):
    """The smallest grids the library accepts and ragged ones (a 59-cell row
    of one tile and one lane, 130 cells over three tiles, partial row groups,
    one plane), from a seeded random start with every CPML memory random:
    eight steps (two triples and a pair) equal eight one-step launches."""
    from paper_2102_12978_amd.solver import Solver
    print(f"[gpu case] three-step {nx}x{ny}x{nz} bc={bc} npml={npml}", flush=True)
    w = W.Workload(f"tiny_{nx}x{ny}x{nz}", nx, ny, nz, 16.0, 10.0, 0, 1.0, 0.5, npml, 8, bc=bc)
    mk = lambda: Solver(nx, ny, nz, w.dx, w.dx, w.dx, courant=w.courant, bc=bc,
                        cpml_cells=npml, grade=w.grade, sigma_scale=w.sigma_scale,
                        kappa_max=w.kappa_max, alpha_max=w.alpha_max, kernel=L.KERNEL_FUSED)
    one, three = mk(), mk()
    three.set_time_block(3, 4, 0)
    _random_start((one, three), seed=9)
    for s in (one, three):
        s.step(8)
    _assert_identical(one, three, f"{nx}x{ny}x{nz}")
    one.close()
    three.close()


def test_rows_two_and_antenna_across_boundary_tiles():
    """Two rows per wavefront and an antenna crossing every launch class
    (300x150, 10-cell CPML, R_B = 60): 21 steps equal one-step runs, and the
    result matches the FP64 oracle."""
    w = W.parity_mid()
    w.steps = 21
    one, three = _solvers(w, 2, 7)
    for s in (one, three):
        s.step(w.steps)
    _assert_identical(one, three, "rows 2, z chunk 7")
    g, st = GC.oracle_run(w, w.steps)
    GC.assert_parity(three.fields(), [st.f[c] for c in GC.COMPS], "three-step rows 2")
    one.close()
    three.close()


def test_boundary_launches_in_order_equal_concurrent():
    """fdtd_set_concurrency(0) runs the three boundary launches after the
    interior one on the context's stream: the same state bit for bit as the
    default concurrent launches."""
    w = W.parity_mid()
    a, b = (GC.gpu_solver(w, kernel=L.KERNEL_FUSED, rows=4, zchunk=0) for _ in range(2))
    for s in (a, b):
        s.set_time_block(3, 2, 8)
    b.set_concurrency(False)
    _random_start((a, b), seed=5)
    for s in (a, b):
        s.step(12)
    _assert_identical(a, b, "in order vs concurrent")
    for s in (a, b):
        s.close()


def test_gradient_with_three_step_forward():
    """The adjoint's checkpointed forward runs through fdtd_step, so with the
    three-step kernel its segments of 25 steps run as triples and a single
    step (plane records run one step per launch); the intensity and the
    sector gradient equal those of the one-step forward bit for bit."""
    from paper_2102_12978_amd.adjoint import SectorSensitivity
    w = W.Workload("adj_120_m0", 120, 120, 10, 12.0, 30.0, 0, 40.0, 2.0, 6, 90,
                   ramp_periods=2.0, extra={"sectors": 16, "checkpoint_every": 25})
    rng = np.random.default_rng(21)
    amp = 1.0 + 0.05 * rng.standard_normal(16)
    ph = 0.1 * rng.standard_normal(16)
    out = []
    for tb in (1, 3):
        sens = SectorSensitivity(w, window_begin=60)
        if tb == 3:
            sens.solver.set_time_block(3, 4, 0)
            assert sens.solver.info().time_block == 3
        ibar = sens.intensity(amp, ph)
        dl = 1e-3 * np.cos(np.arange(ibar.size, dtype=np.float64)).reshape(ibar.shape)
        ga, gp = sens.backward(dl)
        out.append((ibar, ga, gp))
        sens.close()
    (i1, a1, p1), (i2, a2, p2) = out
    assert np.array_equal(i1, i2)
    assert np.array_equal(a1, a2) and np.array_equal(p1, p2)


def test_no_buffer_and_bad_arguments():
    """Three-step passes allocate nothing (device_bytes unchanged after
    selecting them and stepping), and tile shapes the kernel does not have
    are refused with FDTD_EINVAL, leaving the selection as it was."""
    w = W.parity_mid()
    s = GC.gpu_solver(w, kernel=L.KERNEL_FUSED)
    s.step(2)
    b0 = s.info().device_bytes
    s.set_time_block(3, 2, 8)
    s.step(6)
    inf = s.info()
    assert inf.device_bytes == b0 and inf.time_block == 3 and inf.step == 8
    for args in ((3, 8, 0), (3, 3, 0), (3, 2, -1), (3, 2, 10**6)):
        with pytest.raises(L.FdtdError) as e:
            s.set_time_block(*args)
        assert e.value.code == L.EINVAL
    inf = s.info()
    assert (inf.time_block, inf.tb_rows, inf.tb_zchunk) == (3, 2, 8)
    s.close()
