"""Parity at the benchmark's full size: 768×768×255, Δx = λ/24, θ = 20°,
order 2, annulus 320Δx, 16-cell CPML, in the launch shape the benchmark
times (one three-step pass: 2 rows per wavefront, z chunks of 32, the four
tile classes concurrent) and in the one-step shape (fused interior kernel,
4 rows per wavefront, z chunks of 16, split frame).

From a seeded random state (fields U(-1,1), random CPML memories, E held at
the walls zeroed) and with the antenna on, three steps run on the GPU; then
whole z-columns at sampled (x, y) positions are compared with the FP64
oracle, each computed exactly from a small window of the same initial state
(tests/window.py). The columns sit on interior segment and row-group
boundaries of both shapes (x0 - 1 / x0, last / first row of a group; the
three-step segments start at x = 36 + 58 k), on the interior's edge and
the frame or boundary tiles next to it, in the CPML slabs and corners, and
on the antenna ring; every z plane of each column is compared, so every
z-chunk boundary is crossed."""
import numpy as np
import pytest

from oracle import problem as P
from oracle import yee as Y
from paper_2102_12978_amd import _lib as L
from paper_2102_12978_amd import workloads as W
from tests import cases
from tests import gpu_cases as GC
from tests import window as WN

pytestmark = pytest.mark.gpu

COLUMNS = [(95, 100), (96, 101), (32, 17), (31, 16), (735, 748), (736, 749), (400, 20),
           (400, 21), (8, 400), (760, 400), (400, 760), (5, 5), (762, 762), (704, 384),
           (384, 64), (610, 610), (159, 383), (160, 384),
           # three-step shape: x-boundary / interior segment edges (36, 732),
           # an interior segment edge (94), the first and last interior rows
           # of the row groups at 2 rows per wavefront (24, 743)
           (35, 300), (36, 301), (93, 200), (94, 201), (731, 500), (732, 501), (400, 23),
           (401, 24), (402, 743), (403, 744)]


@pytest.mark.parametrize("shape", ["three-step", "one-step"])
def test_large_grid_sampled_columns(shape):
    w = W.grid768()
    steps = 3
    s = GC.gpu_solver(w, kernel=L.KERNEL_FUSED, rows=4, zchunk=16)
    if shape == "three-step":
        s.set_time_block(3, 2, 32)
    g = cases.oracle_grid(w)
    ant = P.build_antenna(g, cases.oracle_injector(w))
    rng = np.random.default_rng(7)
    fields = {}
    for q, c in enumerate(GC.COMPS):
        a = rng.uniform(-1.0, 1.0, size=(g.nz, g.ny, g.nx)).astype(np.float32)
        if c in ("ex", "ey", "ez"):
            a[:, Y.held_mask(g, c)] = 0.0
        s.set_state(q, a)
        fields[c] = a
    slabs = {}
    for q, name in GC.PSI.items():
        a = rng.uniform(-1.0, 1.0, size=s.state_shape(q)).astype(np.float32)
        s.set_state(q, a)
        slabs[name] = a
    print(f"  random state set; {steps} steps, {shape} launch shape", flush=True)
    s.step(steps)
    got = {c: s.get_state(q) for q, c in enumerate(GC.COMPS)}
    s.close()
    num = den = 0.0
    worst = 0.0
    for (i, j) in COLUMNS:
        ref = WN.column(g, ant, fields, slabs, i, j, steps)
        for c in GC.COMPS:
            d = got[c][:, j, i].astype(np.float64) - ref[c]
            num += float(np.sum(d * d))
            den += float(np.sum(ref[c] ** 2))
            worst = max(worst, float(np.abs(d).max()))
    rel = (num / den) ** 0.5
    print(f"  {len(COLUMNS)} columns x {g.nz} planes x 6 components: rel-L2 {rel:.2e}, "
          f"max |diff| {worst:.2e}", flush=True)
    assert rel <= 1e-5 and worst <= 1e-5


@pytest.mark.parametrize("time_block", [1, 2, 3])
def test_component_beyond_4_gib(time_block):
    """A grid whose field components exceed 4 GiB (2048×1024×536, 1.12 G
    cells, 54 GB of fields): planes past 512 lie beyond 32-bit byte offsets,
    so the fused kernel takes 64-bit plane bases (the two- and three-step
    kernels always do). Random fields in windows around sampled columns
    (zero elsewhere), antenna on, three steps (one pair and a single step
    with time_block 2, one pass with time_block 3); whole columns (every
    plane) against the windowed FP64 oracle."""
    w = W.Workload("big_2048x1024x536_theta20_m1", 2048, 1024, 540, 24.0, 20.0, 1, 400.0, 2.0,
                   16, 3)
    steps = 3
    g = cases.oracle_grid(w)
    assert g.nz * g.ny * 2048 * 4 > (1 << 32)
    # antenna ring, interior, frame, and the two-step kernel's tile boundary
    # (x = 632), rectangle edges (x 32 / 2015, y 18 / 1005) and the last,
    # left-shifted tile (x 1956); the three-step kernel's segment edges
    # (x = 38 + 58 k: 618, and 2010, where its last segment starts)
    cols = [(1024 - 399, 512), (1024 + 399, 512), (1024, 512 + 399), (700, 300), (64, 700),
            (2040, 1010), (1500, 16), (1024, 512), (632, 400), (32, 600), (2015, 777),
            (1956, 1005), (1300, 18), (618, 450), (2010, 820)]
    h = steps + 2
    s = GC.gpu_solver(w, kernel=L.KERNEL_FUSED, rows=4, zchunk=16)
    if time_block == 2:
        s.set_time_block(2, 4, 32)
    if time_block == 3:
        s.set_time_block(3, 2, 32)
    ant = P.build_antenna(g, cases.oracle_injector(w))
    rng = np.random.default_rng(11)
    fields = {}
    for q, c in enumerate(GC.COMPS):
        a = np.zeros((g.nz, g.ny, g.nx), dtype=np.float32)
        for (i, j) in cols:
            a[:, j - h:j + h + 1, i - h:i + h + 1] = rng.uniform(
                -1.0, 1.0, size=(g.nz, 2 * h + 1, 2 * h + 1))
        if c in ("ex", "ey", "ez"):
            a[:, Y.held_mask(g, c)] = 0.0
        s.set_state(q, a)
        fields[c] = a
    print(f"  {w.name}: nz={g.nz}, component {g.nz * g.ny * g.nx * 4 / 2**30:.2f} GiB; "
          f"state set, {steps} steps", flush=True)
    s.step(steps)
    num = den = worst = 0.0
    got = {}
    for q, c in enumerate(GC.COMPS):
        full = s.get_state(q)
        got[c] = {ij: full[:, ij[1], ij[0]].astype(np.float64) for ij in cols}
        del full
    s.close()
    for (i, j) in cols:
        ref = WN.column(g, ant, fields, {}, i, j, steps)
        for c in GC.COMPS:
            d = got[c][(i, j)] - ref[c]
            num += float(np.sum(d * d))
            den += float(np.sum(ref[c] ** 2))
            worst = max(worst, float(np.abs(d).max()))
    rel = (num / den) ** 0.5
    print(f"  {len(cols)} columns x {g.nz} planes x 6 components: rel-L2 {rel:.2e}, "
          f"max |diff| {worst:.2e}", flush=True)
    assert rel <= 1e-5 and worst <= 1e-5
