"""Fields in caller-owned device memory (fdtd_create_ext): two torch tensors
hold the two field parities. A run on them equals a run on library-owned
buffers bit for bit (one-, two- and three-step passes, antenna on, CPML memories
included); the current-state buffer read through torch equals fdtd_get_state;
the library zeroes the buffers at create and leaves them alive at destroy;
buffers the kernels could not use are rejected on the host."""
import numpy as np
import pytest
import torch

from paper_2102_12978_amd import _lib as L
from paper_2102_12978_amd import workloads as W
from paper_2102_12978_amd.solver import Solver, field_layout
from tests import cases
from tests import gpu_cases as GC

pytestmark = pytest.mark.gpu


def _arrays(s):
    return list(range(6)) + (list(GC.PSI) if s.npml > 0 else [])


def _external(w, kernel=L.KERNEL_FUSED):
    args, kw = Solver.workload_grid_args(w)
    pitch, n = field_layout(*args, **kw)
    assert pitch % 64 == 0 and pitch >= w.nx
    assert n == 6 * args[2] * args[1] * pitch
    bufs = [torch.full((n,), float("nan"), dtype=torch.float32, device="cuda")
            for _ in range(2)]
    torch.cuda.synchronize()
    print(f"[gpu case] {w.name}: external fields, {n} floats per parity, pitch {pitch}",
          flush=True)
    s = Solver(*args, kernel=kernel, dev_fields=(bufs[0].data_ptr(), bufs[1].data_ptr()), **kw)
    s.set_workload_injector(w)
    return s, bufs, pitch


def _assert_identical(a, b, label):
    for q in _arrays(a):
        x, y = a.get_state(q), b.get_state(q)
        assert np.array_equal(x.view(np.uint32), y.view(np.uint32)), f"{label}: array {q}"


def _check_view(s, bufs, pitch, label):
    """The buffer fdtd_current_fields names is one of the caller's and holds
    the state fdtd_get_state returns."""
    ptr = s.current_fields()
    ptrs = [b.data_ptr() for b in bufs]
    assert ptr in ptrs, label
    torch.cuda.synchronize()
    f = bufs[ptrs.index(ptr)].view(6, s.nz, s.ny, pitch)[:, :, :, :s.nx].cpu().numpy()
    for c in range(6):
        assert np.array_equal(f[c].view(np.uint32), s.get_state(c).view(np.uint32)), \
            f"{label}: component {c}"


def test_external_fields_bit_identical():
    w = W.parity_mid()
    s, bufs, pitch = _external(w)
    r = GC.gpu_solver(w, kernel=L.KERNEL_FUSED)
    g = cases.oracle_grid(w)
    # zeroed at create (the NaN fill is gone)
    torch.cuda.synchronize()
    assert all(int(torch.count_nonzero(b)) == 0 for b in bufs)
    for x in (s, r):
        x.set_diagnostics(g.nz // 2, 5, L.DIAG_EY2)
        x.step(13)
    _assert_identical(s, r, "one-step, 13 steps")
    _check_view(s, bufs, pitch, "one-step")
    for x in (s, r):
        x.set_time_block(2, 4, 0)
        x.step(9)
    assert s.info().time_block == 2
    _assert_identical(s, r, "two-step pairs, 22 steps")
    _check_view(s, bufs, pitch, "two-step")
    for x in (s, r):
        x.set_time_block(3, 2, 8)
        x.step(10)
    assert s.info().time_block == 3
    _assert_identical(s, r, "three-step passes, 32 steps")
    _check_view(s, bufs, pitch, "three-step")
    assert np.array_equal(s.fluence(L.DIAG_EY2), r.fluence(L.DIAG_EY2))
    # the two field buffers are not counted as the library's memory
    assert s.info().device_bytes < r.info().device_bytes
    s.close()
    r.close()
    # still the caller's after destroy
    bufs[0].fill_(1.0)
    torch.cuda.synchronize()
    assert float(bufs[0].sum()) == float(bufs[0].numel())


def test_external_fields_reset_and_set_state():
    """fdtd_reset clears the caller's buffers; fdtd_set_state writes into
    them."""
    w = W.parity_small()
    s, bufs, pitch = _external(w)
    s.step(6)
    s.reset()
    torch.cuda.synchronize()
    assert all(int(torch.count_nonzero(b)) == 0 for b in bufs)
    rng = np.random.default_rng(3)
    a = rng.uniform(-1, 1, size=s.state_shape(L.EY)).astype(np.float32)
    s.set_state(L.EY, a)
    _check_view(s, bufs, pitch, "set_state")
    s.close()


def test_external_fields_rejected():
    w = W.parity_mid()
    args, kw = Solver.workload_grid_args(w)
    pitch, n = field_layout(*args, **kw)
    a = torch.zeros(n, dtype=torch.float32, device="cuda")
    b = torch.zeros(n, dtype=torch.float32, device="cuda")
    small = torch.zeros(16, dtype=torch.float32, device="cuda")
    host_raw = np.zeros(n + 64, dtype=np.float32)
    host = host_raw[(-host_raw.ctypes.data) % 256 // 4:]   # 256-byte aligned host memory
    assert host.ctypes.data % 256 == 0
    assert n * 4 > (4 << 20)   # the small tensor's allocation is far shorter
    cases_ = [
        ((a.data_ptr() + 4, b.data_ptr()), "aligned"),
        ((a.data_ptr(), a.data_ptr()), "overlap"),
        ((0, b.data_ptr()), "NULL"),
        ((a.data_ptr(), small.data_ptr()), "ends before"),
        ((host.ctypes.data, b.data_ptr()), "device memory"),
    ]
    for ptrs, frag in cases_:
        with pytest.raises(L.FdtdError) as e:
            Solver(*args, dev_fields=ptrs, **kw)
        assert e.value.code == L.EINVAL, frag
        assert frag in str(e.value), (frag, str(e.value))
    # the buffers were not written
    torch.cuda.synchronize()
    assert int(torch.count_nonzero(a)) == 0 and int(torch.count_nonzero(b)) == 0


def test_gradient_on_external_fields():
    """The adjoint (checkpointed forward through fdtd_step, reverse sweep)
    on a context whose fields live in torch tensors gives the intensity and
    the sector gradient of a library-owned context bit for bit."""
    from paper_2102_12978_amd.adjoint import SectorSensitivity
    w = W.Workload("adj_120_m0", 120, 120, 10, 12.0, 30.0, 0, 40.0, 2.0, 6, 90,
                   ramp_periods=2.0, extra={"sectors": 16, "checkpoint_every": 25})
    rng = np.random.default_rng(21)
    amp = 1.0 + 0.05 * rng.standard_normal(16)
    ph = 0.1 * rng.standard_normal(16)
    args, kw = Solver.workload_grid_args(w)
    pitch, n = field_layout(*args, **kw)
    bufs = [torch.zeros(n, dtype=torch.float32, device="cuda") for _ in range(2)]
    torch.cuda.synchronize()
    out = []
    for dev in (None, (bufs[0].data_ptr(), bufs[1].data_ptr())):
        print(f"[gpu case] {w.name}: gradient, external fields {dev is not None}", flush=True)
        sens = SectorSensitivity(w, window_begin=60, dev_fields=dev)
        ibar = sens.intensity(amp, ph)
        dl = 1e-3 * np.cos(np.arange(ibar.size, dtype=np.float64)).reshape(ibar.shape)
        ga, gp = sens.backward(dl)
        out.append((ibar, ga, gp))
        sens.close()
    (i1, a1, p1), (i2, a2, p2) = out
    assert np.array_equal(i1, i2)
    assert np.array_equal(a1, a2) and np.array_equal(p1, p2)
