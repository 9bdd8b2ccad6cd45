"""Observed order of the GPU path on 2-D Burgers (u0 = 0.5 + 0.25 sin 2 pi
(x + y), flux along (1, 1), before the shock) on regular triangle and quad
meshes: second order, the bound of one flux evaluation per face for a
nonlinear flux in more than one dimension, for USR3 and CSR4 alike.  On the
mixed, jittered meshes of the Burgers workload the same schemes lose order
or stability (reported by the bench's sweep, not asserted here)."""
import math

import numpy as np
import pytest

from synth import configs, fields
from synth import mesh as M

pytestmark = pytest.mark.gpu


def _error(n, split, scheme):
    from paper_2404_08952_amd import Solver
    m = M.periodic_2d(n, n, split=split, diagonal="main")
    U0 = fields.cell_averages(m, fields.burgers_diag(0.0), n_pts=4)
    dt0 = configs.nominal_dt(m, "burgers", U0, 0.4, simplex=True)
    steps = int(math.ceil(0.05 / dt0))
    s = Solver(m, pde="burgers", scheme=scheme, flux="upwind")
    U = s.to_internal(U0)
    s.advance(U, 0.05 / steps, steps)
    u = s.to_external(U)[:, 0]
    V = s.geometry()["V"].cpu().numpy()[s.perm]
    s.close()
    ex = fields.cell_averages(m, fields.burgers_diag(0.05), n_pts=4)[:, 0]
    return math.sqrt(np.sum(V * (u - ex) ** 2) / np.sum(V))


@pytest.mark.parametrize("scheme", ["USR3", "CSR4"])
@pytest.mark.parametrize("split", [1.0, 0.0], ids=["triangles", "quads"])
def test_second_order_on_regular_meshes(split, scheme):
    e = [_error(n, split, scheme) for n in (32, 64, 128)]
    orders = np.log2(np.array(e[:-1]) / np.array(e[1:]))
    assert np.all(orders > 1.8), (e, orders)
