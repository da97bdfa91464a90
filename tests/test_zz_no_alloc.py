"""fdtd_step_static (the stepping entry point that allocates nothing) against
fdtd_step through the C ABI: fields, CPML memories, plane sums and the
energy must agree bit for bit, on two calls in a row on two grids, the
second smaller (the shared static scratch keeps the first call's
contents), with the energy diagnostic (its partial sums in the static
scratch) and with the two- and three-step kernels; steps past the time tables and a
grid whose energy partials exceed the static scratch are refused without
stepping."""
import numpy as np
import pytest

from paper_2102_12978_amd import _lib as L
from paper_2102_12978_amd import workloads as W
from paper_2102_12978_amd.solver import Solver
from tests import gpu_cases as GC

pytestmark = pytest.mark.gpu


def _pair(w, time_block):
    out = []
    for _ in range(2):
        s = GC.gpu_solver(w, kernel=L.KERNEL_FUSED)
        if time_block > 1:
            s.set_time_block(time_block, 2, 8)
        out.append(s)
    return out


def _same_state(a, b, npml):
    ids = list(range(6)) + (list(GC.PSI) if npml > 0 else [])
    for q in ids:
        x, y = a.get_state(q), b.get_state(q)
        assert np.array_equal(x.view(np.uint32), y.view(np.uint32)), q


@pytest.mark.parametrize("time_block", [1, 2, 3])
def test_static_step_equals_step_on_two_grids(time_block):
    """300x150 then the smaller 100x72 grid, each stepped through both entry
    points: energy diagnostic on (one step per launch, partials in the
    static scratch), then off for 13 more steps (pairs with time_block 2,
    triples and a single step with time_block 3)."""
    for w in (W.parity_mid(), W.parity_small()):
        ref, st = _pair(w, time_block)
        for s in (ref, st):
            s.set_diagnostics(s.nz // 2, 4, L.DIAG_EY2 | L.DIAG_ENERGY)
        ref.step(9)
        st.step_static(9)
        assert ref.energy() == st.energy()
        for s in (ref, st):
            s.set_diagnostics(s.nz // 2, 4, L.DIAG_EY2)
        ref.step(13)
        st.step_static(13)
        assert st.info().step == ref.info().step == 22
        _same_state(ref, st, ref.npml)
        assert ref.fluence_count() == st.fluence_count()
        assert np.array_equal(ref.fluence(L.DIAG_EY2), st.fluence(L.DIAG_EY2))
        ref.close()
        st.close()


def test_static_step_refusals():
    w = W.parity_small()
    s = GC.gpu_solver(w, kernel=L.KERNEL_FUSED)
    before = s.get_state(L.EY)
    with pytest.raises(L.FdtdError) as e:
        s.step_static(5000)          # past the time tables built with the antenna
    assert e.value.code == L.ESTATE
    with pytest.raises(L.FdtdError) as e:
        s.step_static(-1)
    assert e.value.code == L.EINVAL
    assert s.info().step == 0 and np.array_equal(before, s.get_state(L.EY))
    s.close()
    # 512^3 with z chunks of one plane: more energy partials than the scratch
    big = Solver(512, 512, 512, 25e-9, 25e-9, 25e-9, courant=0.5, bc=L.BC_CPML, cpml_cells=16,
                 alpha_max=0.1, kernel=L.KERNEL_FUSED)
    big.set_tile(4, 1)
    big.set_diagnostics(256, 0, L.DIAG_ENERGY)
    with pytest.raises(L.FdtdError) as e:
        big.step_static(1)
    assert e.value.code == L.EINVAL and big.info().step == 0
    big.close()
