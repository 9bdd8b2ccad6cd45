"""MI355X (gfx950) DOLINC explicit-residual library: Python binding.

The compute path is ``libdolinc.so`` (hand-written HIP kernels behind the C
ABI declared in ``include/dolinc.h``); this package only marshals arguments.
"""
from .binding import (DolincError, Solver, load, make_params, mesh_prepare)  # noqa: F401
