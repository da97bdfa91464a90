"""Host-side checks of the HIP library that need no GPU: it loads, exports
every symbol the header declares, and its pure host logic (periodic z fit,
argument validation) behaves."""
import ctypes
import math

import numpy as np
import pytest

from oracle import problem as P
from paper_2102_12978_amd import _lib as L
from paper_2102_12978_amd.solver import Solver, field_layout, fit_periodic_z


def test_library_exports_every_declared_symbol():
    lib = L.load()
    declared = L.declared_symbols()
    assert len(declared) >= 19
    for name in declared:
        assert hasattr(lib, name), name
    assert lib.fdtd_version().startswith(b"besselfdtd")


@pytest.mark.parametrize("theta_deg,ns,hint", [(10, 16, 32), (15, 20, 64), (20, 24, 256),
                                               (12, 20, 64), (5, 20, 48), (30, 20, 64),
                                               (25, 16, 18), (30, 16, 1)])
def test_fit_periodic_z_matches_reference(theta_deg, ns, hint):
    lam = 800e-9
    nz, dz = fit_periodic_z(lam, math.radians(theta_deg), lam / ns, hint)
    nz_o, dz_o = P.fit_periodic_z(lam, math.radians(theta_deg), lam / ns, hint)
    assert nz == nz_o
    assert abs(dz - dz_o) <= 1e-15 * dz_o


def test_fit_periodic_z_rejects_bad_arguments():
    lib = L.load()
    nz, dz = ctypes.c_int32(), ctypes.c_double()
    for args in [(800e-9, 0.0, 5e-8, 10), (800e-9, math.pi / 2, 5e-8, 10),
                 (-1.0, 0.3, 5e-8, 10), (800e-9, 0.3, 0.0, 10), (800e-9, 0.3, 5e-8, 0)]:
        assert lib.fdtd_fit_periodic_z(*args, ctypes.byref(nz), ctypes.byref(dz)) == L.EINVAL
    assert lib.fdtd_fit_periodic_z(800e-9, 0.3, 5e-8, 10, None, None) == L.EINVAL


@pytest.mark.parametrize("kw,frag", [
    (dict(courant=0.7), "Courant"),
    (dict(cpml_cells=17), "cpml_cells"),
    (dict(cpml_cells=0), "cpml_cells"),
    (dict(bc=L.BC_PEC, cpml_cells=4), "cpml_cells must be 0"),
    (dict(bc=7), "bc_xy"),
    (dict(nx=1), "grid sizes"),
    (dict(dz=-1.0), "cell sizes"),
    (dict(kernel=9), "kernel"),
])
def test_create_validates_before_touching_the_gpu(kw, frag):
    args = dict(nx=32, ny=32, nz=32, dx=5e-8, dy=5e-8, dz=5.07e-8, courant=0.5,
                bc=L.BC_CPML, cpml_cells=8)
    args.update(kw)
    with pytest.raises(L.FdtdError) as e:
        Solver(**args)
    assert e.value.code == L.EINVAL
    assert frag in str(e.value)


def test_null_arguments_are_rejected():
    lib = L.load()
    assert lib.fdtd_create(None, None) == L.EINVAL
    ctx = ctypes.c_void_p()
    assert lib.fdtd_create(None, ctypes.byref(ctx)) == L.EINVAL
    assert ctx.value is None
    assert lib.fdtd_destroy(None) == L.OK
    assert lib.fdtd_step(None, 1) == L.EINVAL
    assert lib.fdtd_get_info(None, None) == L.EINVAL


@pytest.mark.parametrize("nx,ny,nz,pitch", [(32, 32, 32, 64), (65, 40, 7, 128),
                                             (768, 768, 255, 768), (130, 64, 1, 192)])
def test_field_layout(nx, ny, nz, pitch):
    """Rows padded to 256 bytes; one parity is the six components back to
    back (pure host function)."""
    p, n = field_layout(nx, ny, nz, 5e-8, 5e-8, 5.07e-8, cpml_cells=8)
    assert p == pitch
    assert n == 6 * nz * ny * pitch


def test_external_field_entry_points_validate_on_the_host():
    lib = L.load()
    ctx = ctypes.c_void_p()
    g = L.Grid(nx=32, ny=32, nz=32, dx=5e-8, dy=5e-8, dz=5.07e-8, courant=0.7, bc_xy=L.BC_CPML,
               cpml_cells=8, cpml_grade=3.0, cpml_sigma_scale=1.0, cpml_kappa_max=1.0,
               cpml_alpha_max=0.0, kernel=L.KERNEL_AUTO, reserved=0, stream=None)
    pitch, n = ctypes.c_int32(), ctypes.c_int64()
    assert lib.fdtd_field_layout(ctypes.byref(g), ctypes.byref(pitch), ctypes.byref(n)) == L.EINVAL
    g.courant = 0.5
    assert lib.fdtd_field_layout(ctypes.byref(g), None, ctypes.byref(n)) == L.EINVAL
    assert lib.fdtd_field_layout(None, ctypes.byref(pitch), ctypes.byref(n)) == L.EINVAL
    assert lib.fdtd_create_ext(ctypes.byref(g), None, ctypes.byref(ctx)) == L.EINVAL
    assert b"dev_fields" in lib.fdtd_last_error(None)
    assert ctx.value is None
    ptr = ctypes.c_void_p()
    assert lib.fdtd_current_fields(None, ctypes.byref(ptr)) == L.EINVAL
    # the grid is validated before any pointer or the GPU is looked at
    with pytest.raises(L.FdtdError) as e:
        Solver(32, 32, 32, 5e-8, 5e-8, 5.07e-8, courant=0.7, cpml_cells=8,
               dev_fields=(256, 512))
    assert e.value.code == L.EINVAL and "Courant" in str(e.value)


def test_batch_create_rejects_empty_batches_on_the_host():
    lib = L.load()
    out = ctypes.c_void_p()
    assert lib.fdtd_batch_create(0, None, None, None, ctypes.byref(out)) == L.EINVAL
    assert out.value is None
    assert b"count" in lib.fdtd_batch_last_error(None)
    assert lib.fdtd_batch_create(-3, None, None, None, ctypes.byref(out)) == L.EINVAL
    assert lib.fdtd_batch_step(None, 1) == L.EINVAL


def test_stream_probe_validates_before_touching_the_gpu():
    lib = L.load()
    ms, gbs = ctypes.c_double(), ctypes.c_double()
    bad = [(3, 1 << 20, 5), (-1, 1 << 20, 5), (0, 0, 5), (0, (1 << 20) + 4, 5), (0, 1 << 20, 0),
           (0, 1 << 20, 1001)]
    for kind, nbytes, reps in bad:
        assert lib.fdtd_stream_probe(kind, nbytes, reps, None, ctypes.byref(ms),
                                     ctypes.byref(gbs)) == L.EINVAL
    assert lib.fdtd_stream_probe(0, 1 << 20, 5, None, None, None) == L.EINVAL


def test_frame_and_batch_setters_reject_null_handles():
    lib = L.load()
    assert lib.fdtd_set_frame(None, L.FRAME_FUSED, 32, 2) == L.EINVAL
    assert lib.fdtd_batch_set_kernel(None, L.KERNEL_FUSED, 2) == L.EINVAL
    assert lib.fdtd_batch_set_tile(None, 256, 1) == L.EINVAL


def test_polarisation_constants_match_the_header():
    text = open(L.HEADER).read()
    for name, value in (("FDTD_POL_X_TE", L.POL_X_TE), ("FDTD_POL_Y_TE", L.POL_Y_TE),
                        ("FDTD_POL_Z_TE", L.POL_Z_TE), ("FDTD_POL_X_TM", L.POL_X_TM),
                        ("FDTD_POL_Y_TM", L.POL_Y_TM), ("FDTD_POL_Z_TM", L.POL_Z_TM),
                        ("FDTD_FRAME_SPLIT", L.FRAME_SPLIT), ("FDTD_FRAME_FUSED", L.FRAME_FUSED),
                        ("FDTD_INJ_ALLOW_Z_MISFIT", L.INJ_ALLOW_Z_MISFIT)):
        assert f"#define {name} {value}" in text, name


def test_time_block_setter_rejects_null_handle():
    lib = L.load()
    assert lib.fdtd_set_time_block(None, 2, 4, 0) == L.EINVAL
    assert lib.fdtd_set_concurrency(None, 1) == L.EINVAL


# ctypes structure -> C type name in include/fdtd.h
_STRUCTS = (("Grid", "fdtd_grid"), ("Injector", "fdtd_injector"), ("Info", "fdtd_info"),
            ("KernelProfile", "fdtd_kernel_profile"), ("BatchInfo", "fdtd_batch_info"),
            ("AdjointInfo", "fdtd_adjoint_info"))


def test_ctypes_structures_match_the_header_layout(tmp_path):
    """Size and every field offset of the binding's structures equal what a
    C compiler makes of include/fdtd.h."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    lines = ['#include <stddef.h>', '#include <stdio.h>', f'#include "{L.HEADER}"',
             'int main(void) {']
    for py, c in _STRUCTS:
        cls = getattr(L, py)
        lines.append(f'  printf("{py} size %zu\\n", sizeof({c}));')
        for fname, _ in cls._fields_:
            lines.append(f'  printf("{py} {fname} %zu\\n", offsetof({c}, {fname}));')
    lines += ['  return 0;', '}']
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c99", "-o", str(exe), str(src)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    got = {}
    for line in out.splitlines():
        py, key, val = line.split()
        got[(py, key)] = int(val)
    for py, _ in _STRUCTS:
        cls = getattr(L, py)
        assert got[(py, "size")] == ctypes.sizeof(cls), py
        for fname, _ in cls._fields_:
            assert got[(py, fname)] == getattr(cls, fname).offset, (py, fname)
