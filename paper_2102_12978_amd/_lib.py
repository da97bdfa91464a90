"""ctypes view of the C ABI declared in include/fdtd.h (argument marshalling only)."""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("BESSELFDTD_LIB") or os.path.join(HERE, "lib", "libbesselfdtd.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "fdtd.h")

OK, EINVAL, ENOMEM, EDEVICE, ESTATE, EUNSTABLE = 0, -1, -2, -3, -4, -5
BC_CPML, BC_PEC, BC_PERIODIC = 0, 1, 2
RAMP_SIN2, RAMP_GAUSS, RAMP_CW = 0, 1, 2
KERNEL_AUTO, KERNEL_SPLIT, KERNEL_FUSED = 0, 1, 2
FRAME_SPLIT, FRAME_FUSED = 0, 1
POL_X_TE, POL_Y_TE, POL_Z_TE, POL_X_TM, POL_Y_TM, POL_Z_TM = range(6)
INJ_ALLOW_Z_MISFIT = 1
EX, EY, EZ, HX, HY, HZ = range(6)
PSI_EXY, PSI_EYX, PSI_EZX, PSI_EZY, PSI_HXY, PSI_HYX, PSI_HZX, PSI_HZY = range(6, 14)
DIAG_EX2, DIAG_EY2, DIAG_EZ2, DIAG_ENERGY = 1, 2, 4, 8

c_double_p = ctypes.POINTER(ctypes.c_double)
c_float_p = ctypes.POINTER(ctypes.c_float)


class Grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("dx", ctypes.c_double), ("dy", ctypes.c_double), ("dz", ctypes.c_double),
                ("courant", ctypes.c_double), ("bc_xy", ctypes.c_int32),
                ("cpml_cells", ctypes.c_int32), ("cpml_grade", ctypes.c_double),
                ("cpml_sigma_scale", ctypes.c_double), ("cpml_kappa_max", ctypes.c_double),
                ("cpml_alpha_max", ctypes.c_double), ("kernel", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("stream", ctypes.c_void_p)]


class Injector(ctypes.Structure):
    _fields_ = [("wavelength", ctypes.c_double), ("theta", ctypes.c_double),
                ("order", ctypes.c_int32), ("ramp_kind", ctypes.c_int32),
                ("e0", ctypes.c_double), ("r_outer", ctypes.c_double),
                ("thickness", ctypes.c_double), ("axis_x", ctypes.c_double),
                ("axis_y", ctypes.c_double), ("ramp_a", ctypes.c_double),
                ("ramp_b", ctypes.c_double), ("n_sectors", ctypes.c_int32),
                ("polarization", ctypes.c_int32), ("sector_amp", c_double_p),
                ("sector_phase", c_double_p), ("flags", ctypes.c_int32)]


class Info(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("pitch", ctypes.c_int32), ("sx", ctypes.c_double), ("sy", ctypes.c_double),
                ("sz", ctypes.c_double), ("k", ctypes.c_double), ("beta", ctypes.c_double),
                ("kr", ctypes.c_double), ("omega", ctypes.c_double),
                ("n_source", ctypes.c_int32 * 6), ("n_slots", ctypes.c_int32),
                ("kernel", ctypes.c_int32), ("tile_rows", ctypes.c_int32),
                ("tile_zchunk", ctypes.c_int32), ("step", ctypes.c_int64),
                ("device_bytes", ctypes.c_int64), ("interior_cells", ctypes.c_int64),
                ("frame", ctypes.c_int32), ("xalign", ctypes.c_int32),
                ("frame_rows", ctypes.c_int32), ("time_block", ctypes.c_int32),
                ("tb_rows", ctypes.c_int32), ("tb_zchunk", ctypes.c_int32)]


class KernelProfile(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 48), ("launches", ctypes.c_int64),
                ("total_ms", ctypes.c_double)]


class BatchInfo(ctypes.Structure):
    _fields_ = [("count", ctypes.c_int32), ("tile_cols", ctypes.c_int32),
                ("tile_zchunk", ctypes.c_int32), ("work_items", ctypes.c_int32),
                ("blocks", ctypes.c_int32), ("graph_steps", ctypes.c_int32),
                ("cells", ctypes.c_int64), ("step", ctypes.c_int64),
                ("device_bytes", ctypes.c_int64), ("kernel", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("time_block", ctypes.c_int32),
                ("tb_rows", ctypes.c_int32), ("tb_zchunk", ctypes.c_int32),
                ("tb_items", ctypes.c_int32)]


class AdjointInfo(ctypes.Structure):
    _fields_ = [("checkpoint_every", ctypes.c_int32), ("checkpoints", ctypes.c_int32),
                ("antenna_columns", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("forward_steps", ctypes.c_int64), ("recompute_steps", ctypes.c_int64),
                ("device_bytes", ctypes.c_int64), ("forward_runs", ctypes.c_int64)]


_CTX = ctypes.c_void_p
_ADJ = ctypes.c_void_p
_BATCH = ctypes.c_void_p
_I32P = ctypes.POINTER(ctypes.c_int32)
_SIGS = {
    "fdtd_version": (ctypes.c_char_p, []),
    "fdtd_fit_periodic_z": (ctypes.c_int, [ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                           ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                           c_double_p]),
    "fdtd_antenna_points": (ctypes.c_int, [ctypes.POINTER(Grid), ctypes.POINTER(Injector),
                                           _I32P, ctypes.c_int64,
                                           ctypes.POINTER(ctypes.c_int64)]),
    "fdtd_create": (ctypes.c_int, [ctypes.POINTER(Grid), ctypes.POINTER(_CTX)]),
    "fdtd_create_ext": (ctypes.c_int, [ctypes.POINTER(Grid), ctypes.POINTER(ctypes.c_void_p),
                                       ctypes.POINTER(_CTX)]),
    "fdtd_field_layout": (ctypes.c_int, [ctypes.POINTER(Grid), ctypes.POINTER(ctypes.c_int32),
                                         ctypes.POINTER(ctypes.c_int64)]),
    "fdtd_current_fields": (ctypes.c_int, [_CTX, ctypes.POINTER(ctypes.c_void_p)]),
    "fdtd_destroy": (ctypes.c_int, [_CTX]),
    "fdtd_last_error": (ctypes.c_char_p, [_CTX]),
    "fdtd_set_injector": (ctypes.c_int, [_CTX, ctypes.POINTER(Injector)]),
    "fdtd_set_sector_weights": (ctypes.c_int, [_CTX, ctypes.c_int32, c_double_p, c_double_p]),
    "fdtd_set_diagnostics": (ctypes.c_int, [_CTX, ctypes.c_int32, ctypes.c_int64,
                                            ctypes.c_uint32]),
    "fdtd_step": (ctypes.c_int, [_CTX, ctypes.c_int64]),
    "fdtd_step_static": (ctypes.c_int, [_CTX, ctypes.c_int64]),
    "fdtd_fluence": (ctypes.c_int, [_CTX, ctypes.c_uint32, c_float_p, ctypes.c_int64]),
    "fdtd_fluence_count": (ctypes.c_int, [_CTX, ctypes.POINTER(ctypes.c_int64)]),
    "fdtd_energy": (ctypes.c_int, [_CTX, c_double_p]),
    "fdtd_get_state": (ctypes.c_int, [_CTX, ctypes.c_int32, c_float_p, ctypes.c_int64]),
    "fdtd_set_state": (ctypes.c_int, [_CTX, ctypes.c_int32, c_float_p, ctypes.c_int64]),
    "fdtd_reset": (ctypes.c_int, [_CTX]),
    "fdtd_get_info": (ctypes.c_int, [_CTX, ctypes.POINTER(Info)]),
    "fdtd_analytic_ey2": (ctypes.c_int, [_CTX, c_float_p, ctypes.c_int64]),
    "fdtd_set_tile": (ctypes.c_int, [_CTX, ctypes.c_int32, ctypes.c_int32]),
    "fdtd_autotune": (ctypes.c_int, [_CTX, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                     ctypes.POINTER(ctypes.c_int32)]),
    "fdtd_set_frame": (ctypes.c_int, [_CTX, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]),
    "fdtd_set_time_block": (ctypes.c_int, [_CTX, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]),
    "fdtd_set_concurrency": (ctypes.c_int, [_CTX, ctypes.c_int32]),
    "fdtd_profile_enable": (ctypes.c_int, [_CTX, ctypes.c_int32]),
    "fdtd_profile_read": (ctypes.c_int, [_CTX, ctypes.POINTER(KernelProfile), ctypes.c_int32,
                                         ctypes.POINTER(ctypes.c_int32)]),
    "fdtd_adjoint_create": (ctypes.c_int, [_CTX, ctypes.c_int32, ctypes.POINTER(_ADJ)]),
    "fdtd_adjoint_destroy": (ctypes.c_int, [_ADJ]),
    "fdtd_adjoint_last_error": (ctypes.c_char_p, [_ADJ]),
    "fdtd_adjoint_forward": (ctypes.c_int, [_ADJ, ctypes.c_int64, ctypes.c_int32,
                                            ctypes.c_int64]),
    "fdtd_adjoint_backward": (ctypes.c_int, [_ADJ, c_float_p, ctypes.c_int64, ctypes.c_int32,
                                             c_double_p, c_double_p]),
    "fdtd_adjoint_source_correlation": (ctypes.c_int, [_ADJ, c_double_p, ctypes.c_int64]),
    "fdtd_adjoint_transpose": (ctypes.c_int, [_ADJ, ctypes.c_int64]),
    "fdtd_adjoint_get_state": (ctypes.c_int, [_ADJ, ctypes.c_int32, c_float_p, ctypes.c_int64]),
    "fdtd_adjoint_set_state": (ctypes.c_int, [_ADJ, ctypes.c_int32, c_float_p, ctypes.c_int64]),
    "fdtd_adjoint_get_info": (ctypes.c_int, [_ADJ, ctypes.POINTER(AdjointInfo)]),
    "fdtd_batch_create": (ctypes.c_int, [ctypes.c_int32, ctypes.POINTER(Grid),
                                         ctypes.POINTER(Injector), ctypes.c_void_p,
                                         ctypes.POINTER(_BATCH)]),
    "fdtd_batch_destroy": (ctypes.c_int, [_BATCH]),
    "fdtd_batch_last_error": (ctypes.c_char_p, [_BATCH]),
    "fdtd_batch_instance": (_CTX, [_BATCH, ctypes.c_int32]),
    "fdtd_batch_step": (ctypes.c_int, [_BATCH, ctypes.c_int64]),
    "fdtd_batch_set_tile": (ctypes.c_int, [_BATCH, ctypes.c_int32, ctypes.c_int32]),
    "fdtd_batch_set_graph_steps": (ctypes.c_int, [_BATCH, ctypes.c_int32]),
    "fdtd_batch_set_time_block": (ctypes.c_int, [_BATCH, ctypes.c_int32, ctypes.c_int32,
                                                 ctypes.c_int32]),
    "fdtd_batch_set_kernel": (ctypes.c_int, [_BATCH, ctypes.c_int32, ctypes.c_int32]),
    "fdtd_batch_autotune": (ctypes.c_int, [_BATCH, ctypes.c_int32, _I32P, _I32P]),
    "fdtd_batch_get_info": (ctypes.c_int, [_BATCH, ctypes.POINTER(BatchInfo)]),
    "fdtd_stream_probe": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int64, ctypes.c_int32,
                                         ctypes.c_void_p, c_double_p, c_double_p]),
}

_lib = None


class FdtdError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"besselfdtd error {code}: {msg}")
        self.code = code


def load():
    """Load the in-tree HIP library; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -c 'import __graft_entry__ as g; g.build()'`")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def declared_symbols():
    """Function names declared in include/fdtd.h."""
    import re
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(fdtd_[a-z0-9_]+)\s*\(", text)))
