"""Batched instances (fdtd_batch_*): every instance of a batch must evolve
exactly as the same problem run alone through the split kernels (the batch
kernels share the per-cell code), and match the FP64 oracle to 1e-4
relative L2. Graph replays, eager steps, odd step counts and autotuning
must not change a bit."""
import numpy as np
import pytest

from paper_2102_12978_amd import _lib as L
from paper_2102_12978_amd import workloads as W
from paper_2102_12978_amd.batch import Batch
from tests import gpu_cases as GC

pytestmark = pytest.mark.gpu


def _single(w, steps, plane=None, wb=0):
    s = GC.gpu_solver(w, kernel=L.KERNEL_SPLIT)
    if plane is not None:
        s.set_diagnostics(plane, wb, L.DIAG_EY2 | L.DIAG_EX2)
    s.step(steps)
    out = s.fields()
    fl = (s.fluence(L.DIAG_EY2), s.fluence(L.DIAG_EX2), s.fluence_count()) if plane is not None \
        else None
    s.close()
    return out, fl


def _same(a, b):
    return all(np.array_equal(x, y) for x, y in zip(a, b))


@pytest.mark.parametrize("kernel", [L.KERNEL_FUSED, L.KERNEL_SPLIT])
def test_batch_equals_single_split_runs(kernel):
    ws = W.batch_small()
    print(f"[gpu case] batch of {len(ws)}: " + ", ".join(w.name for w in ws), flush=True)
    b = Batch(ws)
    b.set_kernel(kernel)
    b.set_graph_steps(20)
    b.step(45)            # two graph replays, then five direct steps (odd: parity flips)
    for q, w in enumerate(ws):
        ref, _ = _single(w, 45)
        got = b[q].fields()
        rel = GC.rel_l2(got, [x.astype(np.float64) for x in ref])
        print(f"  {w.name}: rel-L2 vs single split run = {rel:.1e}", flush=True)
        assert _same(got, ref), w.name
    b.close()


def test_batch_matches_oracle():
    ws = W.batch_small()[:3]
    b = Batch(ws)
    b.step(45)
    for q, w in enumerate(ws):
        g, st = GC.oracle_run(w, 45)
        GC.assert_parity(b[q].fields(), [st.f[c] for c in GC.COMPS], w.name)
    b.close()


def test_graph_replays_equal_direct_launches():
    ws = W.batch_small()
    a = Batch(ws)
    a.set_graph_steps(0)
    a.step(50)
    b = Batch(ws)
    b.set_graph_steps(8)
    for n in (7, 17, 3, 23):   # graphs start at both parities and at several counter values
        b.step(n)
    assert a.info().step == b.info().step == 50
    for q in range(len(ws)):
        assert _same(a[q].fields(), b[q].fields()), ws[q].name
    a.close()
    b.close()


def test_autotune_leaves_state_alone():
    ws = W.batch_small()
    a = Batch(ws)
    a.step(10)
    cols, zc = a.autotune(2)
    print(f"  batch autotune picked kernel={a.info().kernel} cols={cols} zchunk={zc}", flush=True)
    assert cols in (0, 64, 128, 256) and zc in (0, 32, 16, 8, 4, 1)
    a.step(30)
    b = Batch(ws)
    b.step(40)
    for q in range(len(ws)):
        assert _same(a[q].fields(), b[q].fields()), ws[q].name
    a.close()
    b.close()


@pytest.mark.parametrize("kernel,cols,zchunk,rows", [(L.KERNEL_SPLIT, 64, 5, 2),
                                                     (L.KERNEL_SPLIT, 128, 0, 2),
                                                     (L.KERNEL_SPLIT, 256, 1, 2),
                                                     (L.KERNEL_FUSED, 64, 5, 2),
                                                     (L.KERNEL_FUSED, 64, 0, 4)])
def test_tile_shapes_agree(kernel, cols, zchunk, rows):
    ws = W.batch_small()
    a = Batch(ws)
    a.set_kernel(kernel, rows)
    a.set_tile(cols, zchunk)
    a.step(24)
    for q, w in enumerate(ws):
        ref, _ = _single(w, 24)
        assert _same(a[q].fields(), ref), w.name
    a.close()


def test_batch_plane_diagnostics():
    ws = W.batch_small()[:3]
    b = Batch(ws)
    planes = []
    for q in range(len(ws)):
        plane = b[q].nz // 2
        planes.append(plane)
        b[q].set_diagnostics(plane, 30, L.DIAG_EY2 | L.DIAG_EX2)
    b.step(45)
    for q, w in enumerate(ws):
        _, (ey2, ex2, count) = _single(w, 45, plane=planes[q], wb=30)
        assert b[q].fluence_count() == count == 15
        assert np.array_equal(b[q].fluence(L.DIAG_EY2), ey2)
        assert np.array_equal(b[q].fluence(L.DIAG_EX2), ex2)
    b.close()


def test_instances_refuse_direct_stepping():
    ws = W.batch_small()[:2]
    b = Batch(ws)
    lib = L.load()
    ctx = b[0]._ctx
    assert lib.fdtd_step(ctx, 1) == L.ESTATE
    assert lib.fdtd_reset(ctx) == L.ESTATE
    assert lib.fdtd_destroy(ctx) == L.ESTATE
    assert lib.fdtd_set_tile(ctx, 4, 0) == L.ESTATE
    assert lib.fdtd_set_time_block(ctx, 2, 4, 0) == L.ESTATE
    assert lib.fdtd_set_frame(ctx, L.FRAME_SPLIT, 32, 2) == L.ESTATE
    assert lib.fdtd_autotune(ctx, 2, None, None) == L.ESTATE
    assert lib.fdtd_batch_instance(b._b, 2) is None
    assert lib.fdtd_batch_set_tile(b._b, 96, 0) == L.EINVAL
    assert lib.fdtd_batch_set_graph_steps(b._b, 3) == L.EINVAL
    b.close()


def test_batch64_sampled_instances():
    """The 64 seed-1 instances (48.5 M cells) in the benchmark's launch
    configuration (autotuned shape, 20-step graphs); instances 0, 21 and 63
    must equal their single split runs bit for bit after 24 steps."""
    ws = W.batch64_instances()
    b = Batch(ws)
    cols, zc = b.autotune(1)
    b.set_graph_steps(20)
    inf = b.info()
    print(f"  batch: {inf.count} instances, {inf.cells / 1e6:.2f} M cells, kernel={inf.kernel} "
          f"cols={cols} zchunk={zc}, "
          f"{inf.work_items} work items, {inf.blocks} workgroups", flush=True)
    assert inf.count == 64 and inf.cells == 48_492_676   # sum of nx ny nz after the z fits
    b.step(24)
    for q in (0, 21, 63):
        ref, _ = _single(ws[q], 24)
        assert _same(b[q].fields(), ref), ws[q].name
    b.close()


def test_single_instance_batch_and_step_counts():
    """A batch of one instance equals its single split run; zero steps
    change nothing and a negative count is refused."""
    w = W.batch_small()[0]
    b = Batch([w])
    b.set_graph_steps(20)
    before = b[0].fields()
    b.step(0)
    assert b.info().step == 0
    assert _same(before, b[0].fields())
    with pytest.raises(L.FdtdError) as e:
        b.step(-1)
    assert e.value.code == L.EINVAL
    b.step(23)            # one graph replay and three direct steps
    ref, _ = _single(w, 23)
    assert _same(b[0].fields(), ref)
    b.close()


@pytest.mark.parametrize("rows,zchunk,graph", [(2, 16, 20), (4, 5, 8), (2, 0, 0)])
def test_two_step_batch_equals_single_runs(rows, zchunk, graph):
    """fdtd_batch_set_time_block(2): pairs of steps of every instance run the
    whole-grid two-step kernel (four tile-class launches per pair, walls and
    CPML included); graph replays, eager pairs and an odd last step; fields
    and the plane sums equal the single split runs bit for bit."""
    ws = W.batch_small()
    b = Batch(ws)
    b.set_time_block(2, rows, zchunk)
    b.set_graph_steps(graph)
    inf = b.info()
    print(f"  two-step batch rows={rows} zchunk={zchunk} graph={graph}: "
          f"{inf.tb_items} work items per pair", flush=True)
    assert inf.time_block == 2 and inf.tb_items > 0
    planes = []
    for q in range(len(ws)):
        planes.append(b[q].nz // 2)
        b[q].set_diagnostics(planes[q], 30, L.DIAG_EY2 | L.DIAG_EX2)
    b.step(21)
    b.step(24)
    for q, w in enumerate(ws):
        ref, (ey2, ex2, count) = _single(w, 45, plane=planes[q], wb=30)
        assert _same(b[q].fields(), ref), w.name
        assert b[q].fluence_count() == count == 15
        assert np.array_equal(b[q].fluence(L.DIAG_EY2), ey2)
        assert np.array_equal(b[q].fluence(L.DIAG_EX2), ex2)
    b.close()


def test_two_step_batch_refuses_bad_arguments():
    ws = W.batch_small()[:2]
    b = Batch(ws)
    lib = L.load()
    for args in ((3, 2, 0), (2, 3, 0), (2, 2, -1)):
        assert lib.fdtd_batch_set_time_block(b._b, *args) == L.EINVAL
    assert b.info().time_block == 1
    b.close()
