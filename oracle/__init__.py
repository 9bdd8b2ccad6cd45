"""FP64 CPU oracle for the DOLINC explicit residual (arXiv 2404.08952).

TEST INFRASTRUCTURE ONLY.  A plain, slow, obviously-correct NumPy
implementation written from the paper; it shares no code with the HIP path.
Only the test suite, the smoke check and the benchmark's CPU-baseline leg
may import it.  The product path (``paper_2404_08952_amd``) never does.

Modules
-------
geometry  textbook FV geometry; face scalars d, omega, g (Sec. 2.2)
scheme    Gauss-linear gradient (Sec. 2.3), DOLINC differentials, far-cell
          inversion (eq:diffDLC and its one-sided forms), eq:coeff
          reconstruction (Sec. 2.4)
flux      upwind / Godunov-Burgers / Rusanov / HLLC
limiter   Van Leer state, classical sensor, blend
positivity  per-cell scaling of the face-side states (shock workloads)
solver    residual, SSP-RK3, conservation and error norms
"""
from . import flux, geometry, limiter, positivity, scheme, solver  # noqa: F401
from .geometry import Geometry, geometry as compute_geometry  # noqa: F401
from .solver import residual, rk_step, ssp_rk3  # noqa: F401
