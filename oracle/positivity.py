"""Oracle: positivity of the cell averages for the Euler equations (FP64).

Test infrastructure only.  Not in the paper (its Euler runs need none); a
reading added for the shock workloads, in the manner of the positivity
limiters of Zhang and Shu (J. Comput. Phys. 2010) and Perthame and Shu
(1996): the semi-discrete update of a cell is written as a convex
combination of first-order Lax-Friedrichs updates, each admissible.

For cell c with face-side states U_{c,f} (after the reconstruction, the blend
and the face-side rule for non-positive density or pressure) and area
weights a_f = |S_f| / sum_f' |S_f'|, let

    U*(theta) = U_c - theta * sum_f a_f (U_{c,f} - U_c).

Then U_c = 1/2 U*(theta) + 1/2 sum_f a_f U^theta_{c,f} with the scaled states
U^theta_{c,f} = U_c + theta (U_{c,f} - U_c).  With a flux of
Lax-Friedrichs type (lambda at least the face's wave speeds) one forward
Euler step from these states is admissible when U* and every U^theta_{c,f}
are and dt lambda sum_f |S_f| / V_c <= 1/2; SSP-RK3 is a convex
combination of such steps.  theta_c is the largest theta in [0, 1] with
rho*(theta) >= delta rho_c and p*(theta) >= delta p_c (delta = 1e-6): 1 when
theta = 1 already qualifies, else the smaller of the linear root for the
density and the first positive root of the quadratic

    f(theta) = rho* (E* - k) - |m*|^2 / 2,   k = delta p_c / (gamma - 1),

for the pressure (the admissible states form a convex set, so the admissible
theta form an interval that contains 0).  Every face-side state of cell c is
then replaced by U^theta_c.
"""
from __future__ import annotations

import numpy as np

from . import flux as _flux

DELTA = 1e-6


def theta_cell(Uc, dbar, gamma):
    """theta_c per cell from the cell states Uc [nc, 5] and the area-weighted
    mean face increments dbar [nc, 5] (sum_f a_f (U_{c,f} - U_c))."""
    rho, m, E = Uc[:, 0], Uc[:, 1:4], Uc[:, 4]
    _r, _v, _E, p = _flux.euler_primitives(Uc, gamma)
    drho, dm, dE = dbar[:, 0], dbar[:, 1:4], dbar[:, 4]
    k = DELTA * p / (gamma - 1.0)
    # U*(1)
    r1, m1, E1 = rho - drho, m - dm, E - dE
    ok1 = (r1 >= DELTA * rho) & (r1 * (E1 - k) - 0.5 * np.sum(m1 * m1, 1) >= 0.0)
    th = np.ones_like(rho)
    # density: rho - theta drho = delta rho
    th_r = np.where(drho > 0.0, (1.0 - DELTA) * rho / np.where(drho > 0.0, drho, 1.0), np.inf)
    # pressure: f(theta) = A theta^2 + B theta + C, C > 0
    A = drho * dE - 0.5 * np.sum(dm * dm, 1)
    B = -rho * dE - drho * (E - k) + np.sum(m * dm, 1)
    C = rho * (E - k) - 0.5 * np.sum(m * m, 1)
    disc = np.maximum(B * B - 4.0 * A * C, 0.0)
    q = -0.5 * (B + np.where(B >= 0.0, 1.0, -1.0) * np.sqrt(disc))
    with np.errstate(divide="ignore", invalid="ignore"):
        r_a = np.where(A != 0.0, q / A, np.inf)
        r_b = np.where(q != 0.0, C / q, np.inf)
    r_a = np.where(r_a > 0.0, r_a, np.inf)
    r_b = np.where(r_b > 0.0, r_b, np.inf)
    th_p = np.minimum(r_a, r_b)
    th_low = np.minimum(np.minimum(th_r, th_p), 1.0)
    return np.where(ok1, th, th_low)


def scale_face_states(mesh, geo, U, UL, UR, gamma):
    """The face-side states after the positivity scaling of both cells, and
    theta per cell."""
    nc = mesh.n_cells
    P, N = mesh.owner, mesh.neighbour
    area = np.linalg.norm(geo.S, axis=1)
    tot = np.bincount(P, area, nc) + np.bincount(N, area, nc)
    eL = UL - U[P]
    eR = UR - U[N]
    dbar = np.zeros_like(U)
    for v in range(U.shape[1]):
        dbar[:, v] = (np.bincount(P, area * eL[:, v], nc) + np.bincount(N, area * eR[:, v], nc)) / tot
    th = theta_cell(U, dbar, gamma)
    return U[P] + th[P][:, None] * eL, U[N] + th[N][:, None] * eR, th
