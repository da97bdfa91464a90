"""FP64 CPU reference implementation (the oracle) of the Bessel-antenna FDTD method.

TEST INFRASTRUCTURE. Only the test suite, the smoke check in ``__graft_entry__``
and the ``cpu_baseline`` leg of ``bench.py`` may import this package. The HIP
solver never calls it, and it shares no code, tables or constants with the HIP
solver: every quantity here (z fit, CPML profiles, Bessel amplitudes, time
factors) is recomputed from the paper in plain NumPy/SciPy double precision.

Modules
-------
``fields``    analytic Bessel-beam fields of the Hertz potential (paper §3.1)
``problem``   units, periodic z fit, CPML profiles, antenna point set and
              time factors (paper §4)
``yee``       second-order Yee leapfrog with CPML, z-periodic boundary and the
              soft-source injection (paper §4), plus the diagnostics (§5)
``pulse``     the Bessel pulse of §3.2 (Gaussian spectrum) by quadrature
``adjoint``   the exact transpose of one ``yee`` step (for the gradient path)
``torch_ref`` a pure-PyTorch FP64 forward used as an autograd reference

Parity status of each function is stated in its module header.
"""
