"""The windowed oracle column (tests/window.py) equals the full oracle run:
random fields and CPML memories, antenna on, columns in the interior, on
the CPML slabs and corners, on the antenna ring. CPU only."""
import numpy as np

from oracle import problem as P
from oracle import yee as Y
from paper_2102_12978_amd import workloads as W
from tests import cases
from tests import gpu_cases as GC
from tests import window as WN


def test_window_columns_equal_full_run():
    w = W.parity_mid()
    g = cases.oracle_grid(w)
    ant = P.build_antenna(g, cases.oracle_injector(w))
    rng = np.random.default_rng(1)
    st = Y.zero_state(g)
    for c in st.f:
        st.f[c] = rng.uniform(-1, 1, st.f[c].shape)
    for c in ("ex", "ey", "ez"):
        st.f[c][:, Y.held_mask(g, c)] = 0.0
    for name in st.psi:
        m = np.zeros((g.ny, g.nx), bool)
        if name in WN.X_SLAB:
            m[:, :g.npml] = m[:, g.nx - g.npml:] = True
        else:
            m[:g.npml, :] = m[g.ny - g.npml:, :] = True
        st.psi[name] = rng.uniform(-1, 1, st.psi[name].shape) * m[None]
    fields = {c: st.f[c].copy() for c in st.f}
    slabs = {name: GC.psi_slab(st.psi[name], q, g.npml, g.nx, g.ny) for q, name in GC.PSI.items()}
    ref = st.copy()
    cp = P.cpml_tables(g)
    for _ in range(3):
        Y.step(ref, g, cp, ant)
    for (i, j) in [(5, 5), (31, 16), (32, 17), (96, 60), (150, 75), (290, 140), (200, 20)]:
        col = WN.column(g, ant, fields, slabs, i, j, 3)
        for c in col:
            assert np.array_equal(col[c], ref.f[c][:, j, i]), (i, j, c)
