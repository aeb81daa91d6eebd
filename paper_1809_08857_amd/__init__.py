"""MI355X (gfx950) geometric-multigrid engine for the elliptic solves of
fluid streamer simulation: the variable-permittivity Poisson equation and
the three screened (Helmholtz) radiative-transfer equations.

All arithmetic runs in the HIP kernels of ``libmg.so`` (sources in
``csrc/``, C ABI in ``include/mg.h``); ``mg`` is its ctypes binding.
"""
from . import mg  # noqa: F401
