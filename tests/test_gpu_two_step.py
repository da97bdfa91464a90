"""Two-step kernel over the whole grid (temporal blocking, fdtd_set_time_block).

Every cell, walls and CPML included, is computed with the one-step kernels'
expressions in the same order, so a two-step run must equal a one-step run
bit for bit: fields, CPML memories and the plane sums. The cases cross
several 60-cell tiles and row groups (interior, x boundary, y boundary and
corner launches), z chunks that do and do not divide nz, odd step counts
(the last step runs alone), sources, CPML and PEC walls, seeded random
starts, the smallest grids the library accepts and the 768x768x255
benchmark grid; one case is also checked against the FP64 oracle."""
import numpy as np
import pytest

from paper_2102_12978_amd import _lib as L
from paper_2102_12978_amd import workloads as W
from tests import cases
from tests import gpu_cases as GC

pytestmark = pytest.mark.gpu



def _solvers(w, rows, zchunk, inject=True, bc=None):
    one = GC.gpu_solver(w, kernel=L.KERNEL_FUSED, bc=bc, rows=4, zchunk=0, inject=inject)
    two = GC.gpu_solver(w, kernel=L.KERNEL_FUSED, bc=bc, rows=4, zchunk=0, inject=inject)
    two.set_time_block(2, rows, zchunk)
    assert two.info().time_block == 2
    return one, two


def _arrays(w, s=None):
    npml = s.npml if s is not None else w.npml
    return list(range(6)) + (list(GC.PSI) if npml > 0 else [])


def _assert_identical(one, two, w, label):
    for q in _arrays(w, one):
        a, b = one.get_state(q), two.get_state(q)
        bad = np.count_nonzero(a.view(np.uint32) != b.view(np.uint32))
        if bad:
            idx = np.argwhere(a.view(np.uint32) != b.view(np.uint32))[:4]
            print(f"  {label}: array {q}: {bad} cells differ, first {idx.tolist()}", flush=True)
        assert bad == 0, f"{label}: array {q}"


def _random_start(solvers, w, seed):
    rng = np.random.default_rng(seed)
    s0 = solvers[0]
    for q in _arrays(w, s0):
        a = rng.uniform(-1.0, 1.0, size=s0.state_shape(q)).astype(np.float32)
        if q in (L.EX, L.EY, L.EZ):
            # E held on the x = 0 / y = 0 walls
            if q in (L.EY, L.EZ):
                a[:, :, 0] = 0.0
            if q in (L.EX, L.EZ):
                a[:, 0, :] = 0.0
        for s in solvers:
            s.set_state(q, a)


@pytest.mark.parametrize("rows,zchunk,steps", [(4, 0, 40), (2, 0, 41), (4, 5, 40), (2, 7, 13),
                                                (4, 16, 2)])
def test_bit_identical_with_source(rows, zchunk, steps):
    w = W.parity_mid()
    one, two = _solvers(w, rows, zchunk)
    g = cases.oracle_grid(w)
    for s in (one, two):
        s.set_diagnostics(g.nz // 2, 5, L.DIAG_EX2 | L.DIAG_EY2 | L.DIAG_EZ2)
        s.step(steps)
    assert two.info().step == steps
    _assert_identical(one, two, w, f"rows={rows} zchunk={zchunk} steps={steps}")
    assert one.fluence_count() == two.fluence_count() == max(0, steps - 5)
    for q in (L.DIAG_EX2, L.DIAG_EY2, L.DIAG_EZ2):
        assert np.array_equal(one.fluence(q), two.fluence(q))
    one.close()
    two.close()


@pytest.mark.parametrize("maker,rows,zchunk", [(W.parity_wide, 4, 5), (W.parity_wide, 2, 0),
                                               (W.grad192, 4, 16), (W.parity_gauss, 2, 3)])
def test_bit_identical_random_start(maker, rows, zchunk):
    w = maker()
    one, two = _solvers(w, rows, zchunk)
    _random_start((one, two), w, seed=17)
    for s in (one, two):
        s.step(6)
    _assert_identical(one, two, w, f"{w.name} rows={rows} zchunk={zchunk}")
    # and on from there, with the parities of the two runs now swapped once
    for s in (one, two):
        s.step(3)
    _assert_identical(one, two, w, f"{w.name} +3 steps")
    one.close()
    two.close()


def test_bit_identical_pec_walls():
    """PEC walls instead of CPML (no memories; E held on the x = 0 / y = 0
    walls): random start, antenna on, odd step count."""
    w = W.parity_mid()
    one, two = _solvers(w, 4, 9, bc=L.BC_PEC)
    assert two.npml == 0 and two.info().time_block == 2
    _random_start((one, two), w, seed=5)
    for s in (one, two):
        s.step(7)
    _assert_identical(one, two, w, "PEC walls")
    one.close()
    two.close()


def test_gradient_with_two_step_forward():
    """The adjoint's checkpointed forward runs through fdtd_step, so with
    the two-step kernel it runs in pairs (segments of 25 steps end with a
    single step); the intensity and the sector gradient equal those of the
    one-step forward bit for bit."""
    from paper_2102_12978_amd.adjoint import SectorSensitivity
    w = W.Workload("adj_120_m0", 120, 120, 10, 12.0, 30.0, 0, 40.0, 2.0, 6, 90,
                   ramp_periods=2.0, extra={"sectors": 16, "checkpoint_every": 25})
    rng = np.random.default_rng(21)
    amp = 1.0 + 0.05 * rng.standard_normal(16)
    ph = 0.1 * rng.standard_normal(16)
    out = []
    for tb in (1, 2):
        sens = SectorSensitivity(w, window_begin=60)
        if tb == 2:
            sens.solver.set_time_block(2, 4, 0)
            assert sens.solver.info().time_block == 2
        ibar = sens.intensity(amp, ph)
        dl = 1e-3 * np.cos(np.arange(ibar.size, dtype=np.float64)).reshape(ibar.shape)
        ga, gp = sens.backward(dl)
        out.append((ibar, ga, gp))
        sens.close()
    (i1, a1, p1), (i2, a2, p2) = out
    assert np.array_equal(i1, i2)
    assert np.array_equal(a1, a2) and np.array_equal(p1, p2)


def test_against_oracle():
    w = W.parity_mid()
    s = GC.gpu_solver(w, kernel=L.KERNEL_FUSED, rows=4, zchunk=0)
    s.set_time_block(2, 4, 0)
    s.step(w.steps)
    g, st = GC.oracle_run(w, w.steps)
    GC.assert_parity(s.fields(), [st.f[c] for c in GC.COMPS], f"two-step {w.steps} steps")
    s.close()


@pytest.mark.parametrize("rows,zchunk", [(2, 0), (4, 5)])
def test_thick_antenna_fills_tiles(rows, zchunk):
    """An annulus 38 cells thick reaching the x- and y-boundary tiles: whole
    tiles take the source on every lane and row, so every stage reads its
    amplitudes from the tile's LDS copy. The two-step run equals the
    one-step run bit for bit, and (rows 2) the FP64 oracle within the parity
    bars."""
    w = W.parity_thick()
    one, two = _solvers(w, rows, zchunk)
    assert one.info().n_slots > 10000
    for s in (one, two):
        s.step(w.steps)
    _assert_identical(one, two, w, f"thick antenna rows={rows} zchunk={zchunk}")
    if rows == 2:
        g, st = GC.oracle_run(w, w.steps)
        GC.assert_parity(two.fields(), [st.f[c] for c in GC.COMPS], "thick antenna, two-step")
    one.close()
    two.close()


@pytest.mark.parametrize("pol,order,rows", [(L.POL_Y_TE, 1, 2), (L.POL_Z_TE, 0, 4),
                                            (L.POL_X_TM, 2, 2), (L.POL_Y_TM, 1, 4),
                                            (L.POL_Z_TM, 0, 2), (L.POL_Z_TE, 2, 4)])
def test_polarisations_bit_identical(pol, order, rows):
    """The other potentials and pairings of §3.1 put their sources on other
    components (H_z for Π_z TE, E_z for Π_z TM, ...): every component's
    amplitude goes through the LDS copy, and the two-step run equals the
    one-step run (checked against the oracle in the parity tests) bit for
    bit."""
    from dataclasses import replace
    w = replace(W.parity_mid(), polarization=pol, order=order,
                name=f"p_300x150x24_pol{pol}_m{order}")
    one, two = _solvers(w, rows, 5)
    for s in (one, two):
        s.step(w.steps)
    _assert_identical(one, two, w, f"polarisation {pol} m={order} rows={rows}")
    one.close()
    two.close()


def test_fallbacks():
    """Energy diagnostic on and the split kernel: pairs run as single steps,
    with the same results; a grid with no wall-free tile runs pairs through
    the boundary launches alone."""
    w = W.parity_mid()
    one, two = _solvers(w, 4, 0)
    g = cases.oracle_grid(w)
    for s in (one, two):
        s.set_diagnostics(g.nz // 2, 0, L.DIAG_EY2 | L.DIAG_ENERGY)
        s.step(10)
    assert one.energy() == two.energy()
    _assert_identical(one, two, w, "energy on")
    one.close()
    two.close()
    w0 = W.cube32()
    w0.steps = 12
    one, two = _solvers(w0, 4, 0)
    # no tile of this grid is free of walls and CPML: every pair runs the
    # boundary launches only
    assert two.info().interior_cells == 0 and two.info().time_block == 2
    for s in (one, two):
        s.step(w0.steps)
    _assert_identical(one, two, w0, "small grid")
    one.close()
    two.close()
    s = GC.gpu_solver(w, kernel=L.KERNEL_SPLIT)
    s.set_time_block(2, 2, 0)
    r = GC.gpu_solver(w, kernel=L.KERNEL_SPLIT)
    for x in (s, r):
        x.step(6)
    _assert_identical(r, s, w, "split kernel")
    s.set_time_block(1, 4, 0)
    assert s.info().time_block == 1
    s.close()
    r.close()


def test_bad_arguments():
    w = W.parity_small()
    s = GC.gpu_solver(w, kernel=L.KERNEL_FUSED)
    for args in ((4, 4, 0), (0, 4, 0), (2, 8, 0), (2, 4, -1), (2, 4, 10**6)):
        with pytest.raises(L.FdtdError) as e:
            s.set_time_block(*args)
        assert e.value.code == L.EINVAL
    s.close()


def test_benchmark_grid_bit_identical():
    """768x768x255 (the benchmark grid): random fields and CPML memories,
    antenna on, four steps with the two-step kernel (4 rows, z chunks of 32)
    against four one-step launches."""
    w = W.grid768()
    one, two = _solvers(w, 4, 32)
    print(f"  {w.name}: random state", flush=True)
    _random_start((one, two), w, seed=23)
    for s in (one, two):
        s.step(4)
    _assert_identical(one, two, w, "768 grid")
    one.close()
    two.close()


def test_device_bytes_accounting():
    """The two-step kernel needs no buffer of its own: fdtd_set_time_block
    and an autotune call leave device_bytes as they were (the fused frame
    trials may grow the tile list and partial sums by a few tens of kB).
    Regrown time tables replace their old bytes, not add to them. The
    profiler stays attached across autotune."""
    w = W.parity_mid()
    s = GC.gpu_solver(w, kernel=L.KERNEL_FUSED)
    s.step(2)
    b0 = s.info().device_bytes
    for _ in range(3):
        s.set_time_block(2, 4, 0)
        assert s.info().device_bytes == b0
        s.set_time_block(1, 4, 0)
        assert s.info().device_bytes == b0
    s.profile(True)
    s.autotune(2)
    inf = s.info()
    extra = inf.device_bytes - b0
    print(f"  autotune: time_block {inf.time_block}, {extra} B of trial buffers kept", flush=True)
    assert 0 <= extra < 1 << 20
    # the trials run untimed and the profiler is back afterwards
    s.step(2)
    prof = s.profile_read()
    assert sum(v[0] for v in prof.values()) > 0
    s.profile(False)
    # past the time tables' first capacity, twice: the E and H tables (two
    # complex floats, 16 B per step) grow at most to twice the steps asked
    # for, and only the last size counts
    before = s.info().device_bytes
    s.step(1200)
    s.step(1200)
    upto = s.info().step
    grown = s.info().device_bytes - before
    print(f"  time tables grew by {grown} B up to step {upto}", flush=True)
    assert 0 < grown <= 16 * 2 * upto
    s.close()


@pytest.mark.parametrize("nx,ny,nz,bc,npml", [(2, 2, 1, L.BC_PEC, 0), (3, 5, 2, L.BC_PEC, 0),
                                             (4, 4, 1, L.BC_CPML, 1), (5, 3, 2, L.BC_CPML, 1),
                                             (61, 17, 3, L.BC_CPML, 2), (130, 70, 5, L.BC_CPML, 3)])
def test_bit_identical_small_and_ragged_grids(nx, ny, nz, bc, npml):
    """The smallest grids the library accepts and ragged ones (a 61-cell row
    of one tile and one lane, 130 cells over three tiles, partial row groups,
    one plane), from a seeded random start with every CPML memory random:
    seven steps in pairs equal seven one-step launches."""
    from paper_2102_12978_amd.solver import Solver
    print(f"[gpu case] two-step {nx}x{ny}x{nz} bc={bc} npml={npml}", flush=True)
    w = W.Workload(f"tiny_{nx}x{ny}x{nz}", nx, ny, nz, 16.0, 10.0, 0, 1.0, 0.5, npml, 7, bc=bc)
    mk = lambda: Solver(nx, ny, nz, w.dx, w.dx, w.dx, courant=w.courant, bc=bc,
                        cpml_cells=npml, grade=w.grade, sigma_scale=w.sigma_scale,
                        kappa_max=w.kappa_max, alpha_max=w.alpha_max, kernel=L.KERNEL_FUSED)
    one, two = mk(), mk()
    two.set_time_block(2, 4, 0)
    _random_start((one, two), w, seed=9)
    for s in (one, two):
        s.step(7)
    _assert_identical(one, two, w, f"{nx}x{ny}x{nz}")
    one.close()
    two.close()


def test_rows_two_and_antenna_across_boundary_tiles():
    """Two rows per wavefront and an antenna crossing every launch class
    (300x150, 10-cell CPML, R_B = 60): 20 steps equal one-step runs, and the
    result matches the FP64 oracle."""
    w = W.parity_mid()
    w.steps = 20
    one, two = _solvers(w, 2, 7)
    for s in (one, two):
        s.step(w.steps)
    _assert_identical(one, two, w, "rows 2, z chunk 7")
    g, st = GC.oracle_run(w, w.steps)
    GC.assert_parity(two.fields(), [st.f[c] for c in GC.COMPS], "two-step rows 2")
    one.close()
    two.close()


def test_boundary_launches_in_order_equal_concurrent():
    """fdtd_set_concurrency(0) runs the three boundary launches after the
    interior one on the context's stream: the same state bit for bit as the
    default concurrent launches; values other than 0 and 1 are refused."""
    w = W.parity_mid()
    a, b = (GC.gpu_solver(w, kernel=L.KERNEL_FUSED, rows=4, zchunk=0) for _ in range(2))
    for s in (a, b):
        s.set_time_block(2, 2, 8)
    b.set_concurrency(False)
    with pytest.raises(L.FdtdError) as e:
        b._c(b._lib.fdtd_set_concurrency(b._ctx, 2))
    assert e.value.code == L.EINVAL
    _random_start((a, b), w, seed=5)
    for s in (a, b):
        s.step(12)
    _assert_identical(a, b, w, "in order vs concurrent")
    for s in (a, b):
        s.close()
