"""Oracle: semi-discrete residual, SSP-RK3 and diagnostics (FP64).

Test infrastructure only.

Residual of the finite-volume update on cell averages (Sec. 2.2, Sec. 3);
with params["positivity"] the face-side states of the Euler equations are
scaled per cell first (positivity.py):
    R_P = -V_P^-1 sum_{f of P} sigma_{P,f} F_f,   sigma = +1 owner, -1 neighbour,
with F_f the numerical flux of the reconstructed face states.  Time
integration is the third-order TVD (SSP) Runge-Kutta method named in Sec. 3:
    U1 = U + dt R(U);  U2 = 3/4 U + 1/4 (U1 + dt R(U1));
    U' = 1/3 U + 2/3 (U2 + dt R(U2)).
"""
from __future__ import annotations

import numpy as np

from . import flux as _flux
from . import limiter as _lim
from . import positivity as _pos
from . import scheme as _sch
from .geometry import geometry  # noqa: F401  (re-exported)


def n_vars(params, dim):
    return dim + 2 if params["pde"] == "euler" else 1


def _positivity_fallback(UL, UR, U, mesh, gamma):
    """Euler: a face side whose state has rho <= 0 or p <= 0 uses the cell value."""
    rL, _v, _E, pL = _flux.euler_primitives(UL, gamma)
    rR, _v, _E, pR = _flux.euler_primitives(UR, gamma)
    badL = ~((rL > 0.0) & (pL > 0.0))
    badR = ~((rR > 0.0) & (pR > 0.0))
    UL = np.where(badL[:, None], U[mesh.owner], UL)
    UR = np.where(badR[:, None], U[mesh.neighbour], UR)
    return UL, UR


def face_flux(mesh, geo, U, params, theta=None):
    scheme = params["scheme"]
    order = max(_sch.scheme_order(scheme), 1 if theta is not None else 0)
    G = _sch.cell_derivs(mesh, geo, U, order)
    UL, UR, G = _sch.face_states(mesh, geo, U, scheme, G)
    if theta is not None:
        LL, LR = _lim.limited_states(mesh, geo, U, G[1])
        UL, UR = _lim.blend(UL, UR, LL, LR, np.asarray(theta, dtype=np.float64), mesh)
    pde = params["pde"]
    if pde == "advection":
        return _flux.upwind(UL, UR, geo.S, params.get("adv_vel", (1.0, 0.5, 0.0)))
    if pde == "burgers":
        return _flux.godunov_burgers(UL, UR, geo.S, params.get("burgers_dir", (1.0, 1.0, 0.0)))
    gamma = params.get("gamma", 1.4)
    UL, UR = _positivity_fallback(UL, UR, U, mesh, gamma)
    if params.get("positivity"):
        UL, UR, _th = _pos.scale_face_states(mesh, geo, U, UL, UR, gamma)
    if params["flux"] == "rusanov":
        return _flux.rusanov(UL, UR, geo.S, gamma)
    if params["flux"] == "hllc":
        return _flux.hllc(UL, UR, geo.S, gamma)
    raise ValueError(params["flux"])


def accumulate(mesh, geo, F):
    nc = mesh.n_cells
    R = np.zeros((nc, F.shape[1]))
    for v in range(F.shape[1]):
        R[:, v] = -(np.bincount(mesh.owner, weights=F[:, v], minlength=nc) -
                    np.bincount(mesh.neighbour, weights=F[:, v], minlength=nc)) / geo.V
    return R


def residual(mesh, geo, U, params, theta=None):
    U = np.asarray(U, dtype=np.float64).reshape(mesh.n_cells, -1)
    return accumulate(mesh, geo, face_flux(mesh, geo, U, params, theta))


def ssp_rk3(U, dt, rhs):
    """One SSP-RK3 step of dU/dt = rhs(U)."""
    U1 = U + dt * rhs(U)
    U2 = 0.75 * U + 0.25 * (U1 + dt * rhs(U1))
    return U / 3.0 + (2.0 / 3.0) * (U2 + dt * rhs(U2))


def rk_step(mesh, geo, U, dt, params, theta=None):
    return ssp_rk3(np.asarray(U, dtype=np.float64), dt,
                   lambda X: residual(mesh, geo, X, params, theta))


def conserved_totals(geo, U):
    return (geo.V[:, None] * U).sum(0)


def error_norms(geo, U, Uexact):
    """Volume-weighted L1 and L2 norms of cell-average errors, per variable."""
    e = U - Uexact
    Vt = geo.V.sum()
    L1 = (geo.V[:, None] * np.abs(e)).sum(0) / Vt
    L2 = np.sqrt((geo.V[:, None] * e * e).sum(0) / Vt)
    return L1, L2
