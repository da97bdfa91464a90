"""besselfdtd: MI355X (gfx950) FDTD solver for the Bessel-antenna method.

The solver runs in the HIP library ``lib/libbesselfdtd.so`` (C ABI in
``include/fdtd.h``); this package only marshals arguments. Importing a
solver class loads the library and raises if it has not been built.
"""
from . import workloads
from ._lib import (BC_CPML, BC_PEC, BC_PERIODIC, DIAG_ENERGY, DIAG_EX2, DIAG_EY2, DIAG_EZ2,
                   KERNEL_AUTO, KERNEL_FUSED, KERNEL_SPLIT, RAMP_CW, RAMP_GAUSS, RAMP_SIN2,
                   FdtdError)


def __getattr__(name):
    if name in ("Solver", "fit_periodic_z"):
        from . import solver
        return getattr(solver, name)
    raise AttributeError(name)
