"""Oracle: numerical fluxes through a face with area vector S (owner -> neighbour).

Test infrastructure only.  Every flux returns the face-integrated flux F . S.
* advection (Sec. 3.2): upwind, F = (a.S) U_L if a.S >= 0 else (a.S) U_R.
* Burgers (Sec. 3.3) along a fixed direction b: the Godunov flux of the
  scalar flux f(u) = u^2/2 (b.S): min of f over [U_L, U_R] if U_L <= U_R,
  else max over [U_R, U_L].
* Euler (Sec. 3.4): local Lax-Friedrichs (Rusanov) with the largest |u_n| + c
  of the two states; HLLC (Toro) with Davis wave-speed estimates.
"""
from __future__ import annotations

import numpy as np


def upwind(UL, UR, S, a):
    an = S @ np.asarray(a[: S.shape[1]], dtype=np.float64)
    return np.where((an >= 0.0)[:, None], an[:, None] * UL, an[:, None] * UR)


def godunov_burgers(UL, UR, S, b):
    s = S @ np.asarray(b[: S.shape[1]], dtype=np.float64)
    uL, uR = UL[:, 0], UR[:, 0]

    def f(u):
        return 0.5 * u * u * s
    fL, fR, f0 = f(uL), f(uR), np.zeros_like(s)
    lo = np.minimum(uL, uR)
    hi = np.maximum(uL, uR)
    has0 = (lo <= 0.0) & (hi >= 0.0)
    fmin = np.minimum(fL, fR)
    fmax = np.maximum(fL, fR)
    fmin = np.where(has0, np.minimum(fmin, f0), fmin)
    fmax = np.where(has0, np.maximum(fmax, f0), fmax)
    return np.where(uL <= uR, fmin, fmax)[:, None]


def euler_primitives(U, gamma):
    rho = U[:, 0]
    D = U.shape[1] - 2
    vel = U[:, 1:1 + D] / rho[:, None]
    E = U[:, 1 + D]
    p = (gamma - 1.0) * (E - 0.5 * rho * np.sum(vel * vel, 1))
    return rho, vel, E, p


def euler_flux_n(U, n, gamma):
    """Physical Euler flux dotted with the (not necessarily unit) vector n."""
    rho, vel, E, p = euler_primitives(U, gamma)
    un = np.sum(vel * n, 1)
    F = np.empty_like(U)
    D = U.shape[1] - 2
    F[:, 0] = rho * un
    F[:, 1:1 + D] = rho[:, None] * vel * un[:, None] + p[:, None] * n
    F[:, 1 + D] = (E + p) * un
    return F


def rusanov(UL, UR, S, gamma):
    area = np.linalg.norm(S, axis=1)
    n = S / area[:, None]
    rL, vL, _EL, pL = euler_primitives(UL, gamma)
    rR, vR, _ER, pR = euler_primitives(UR, gamma)
    cL = np.sqrt(gamma * pL / rL)
    cR = np.sqrt(gamma * pR / rR)
    lam = np.maximum(np.abs(np.sum(vL * n, 1)) + cL, np.abs(np.sum(vR * n, 1)) + cR)
    FL = euler_flux_n(UL, S, gamma)
    FR = euler_flux_n(UR, S, gamma)
    return 0.5 * (FL + FR) - 0.5 * (lam * area)[:, None] * (UR - UL)


def hllc(UL, UR, S, gamma):
    area = np.linalg.norm(S, axis=1)
    n = S / area[:, None]
    D = UL.shape[1] - 2
    rL, vL, EL, pL = euler_primitives(UL, gamma)
    rR, vR, ER, pR = euler_primitives(UR, gamma)
    cL = np.sqrt(gamma * pL / rL)
    cR = np.sqrt(gamma * pR / rR)
    qL = np.sum(vL * n, 1)
    qR = np.sum(vR * n, 1)
    SL = np.minimum(qL - cL, qR - cR)
    SR = np.maximum(qL + cL, qR + cR)
    Ss = (pR - pL + rL * qL * (SL - qL) - rR * qR * (SR - qR)) / (rL * (SL - qL) - rR * (SR - qR))
    FL = euler_flux_n(UL, n, gamma)
    FR = euler_flux_n(UR, n, gamma)

    def star(r, v, E, p, q, Sk):
        fac = r * (Sk - q) / (Sk - Ss)
        Us = np.empty((r.shape[0], D + 2))
        Us[:, 0] = fac
        Us[:, 1:1 + D] = fac[:, None] * (v + (Ss - q)[:, None] * n)
        Us[:, 1 + D] = fac * (E / r + (Ss - q) * (Ss + p / (r * (Sk - q))))
        return Us
    UsL = star(rL, vL, EL, pL, qL, SL)
    UsR = star(rR, vR, ER, pR, qR, SR)
    F = np.where((SL >= 0.0)[:, None], FL,
                 np.where((Ss >= 0.0)[:, None], FL + SL[:, None] * (UsL - UL),
                          np.where((SR > 0.0)[:, None], FR + SR[:, None] * (UsR - UR), FR)))
    return F * area[:, None]
