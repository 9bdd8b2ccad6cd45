"""Single-step reconstruction on a graded boundary-layer mesh (Sec. 3.1):
cell averages of the Blasius velocity on quadrilateral rows growing away
from the wall, face values from one reconstruction, compared with the exact
velocity at the face centres.  Test code only (oracle side and helpers for
the GPU side)."""
from __future__ import annotations

import numpy as np

from oracle import boundary as OB
from oracle import scheme as OS
from synth import fields
from synth import mesh as M

NX, LENGTH, H1, HEIGHT, X0 = 24, 1.0, 0.05, 12.0, 1.0
GROWTHS = (1.1, 1.2, 1.3, 1.4, 1.5)
# wall: the velocity vanishes (Dirichlet); top: far field (zero gradient)
BCS = {2: (OB.DIRICHLET, [0.0]), 3: (OB.ZERO_GRADIENT,)}

_BLASIUS = None


def blasius():
    global _BLASIUS
    if _BLASIUS is None:
        _BLASIUS = fields.Blasius()
    return _BLASIUS


def case(growth):
    """(mesh, extended mesh, cell averages [n, 2] of (u, v), exact face values [n_faces, 2])."""
    m = M.boundary_layer_2d(NX, LENGTH, H1, growth, HEIGHT)
    X = OB.extend(m)
    fn = blasius().field(X0)
    U = fields.cell_averages(m, fn, n_pts=6)
    return m, X, U, fn(X.geo.xf)


def measured_faces(X):
    """Faces between two interior cells, parallel to the wall, at least three
    columns away from the x seam (the field is not periodic in x)."""
    nc = X.n_cells
    own, nei = X.mesh.owner, X.mesh.neighbour
    col = lambda c: np.floor(X.geo.xc[c, 0] / (LENGTH / NX)).astype(int)  # noqa: E731
    inner = nei < nc
    co, cn = col(own), col(np.minimum(nei, nc - 1))
    away = (co >= 3) & (co <= NX - 4) & (cn >= 3) & (cn <= NX - 4)
    along = np.abs(X.geo.S[:, 1]) > np.abs(X.geo.S[:, 0])
    return inner & away & along


def oracle_face_states(X, U1, scheme):
    """Oracle UL, UR [n_faces] of one scalar field U1 [n_cells]."""
    nc = X.n_cells
    Ue = np.zeros((X.mesh.n_cells, 1))
    Ue[:nc, 0] = U1
    G = OB.cell_derivs(X, Ue, OS.scheme_order(scheme), BCS, euler=False)
    UL, UR, _ = OS.face_states(X.mesh, X.geo, G[0], scheme, G)
    return UL[:, 0], UR[:, 0]


def rel_error(UL, UR, exact, sel):
    """Relative L2 error of both sides' face values over the selected faces."""
    num = np.sum((UL[sel] - exact[sel]) ** 2) + np.sum((UR[sel] - exact[sel]) ** 2)
    return float(np.sqrt(num / (2.0 * np.sum(exact[sel] ** 2))))
