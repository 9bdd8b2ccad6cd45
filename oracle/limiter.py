"""Oracle: limited second-order face state, classical sensor and the blend.

Test infrastructure only.
* Van Leer limited state, written with the method's quantities: in a frame
  where cell 0 is upwind and cell 1 downwind, Delta = phi_1 - phi_0 and the
  upwind difference s = phi_0^(1) - Delta (= g (phi_0 - phi_-1) by the
  first inversion formula, Sec. 2.3, and the ENO3 divided difference,
  Sec. 2.4).  The limited state is phi_0 + L with the increment
  L = (1 - omega_0) psi Delta, psi Delta = 2 s Delta / (s + Delta) when
  s Delta > 0, else 0 (Van Leer's limiter in the gradient-ratio form
  r = s / Delta; symmetric, psi(1/r) = psi(r) / r), and |L| capped at |Delta|
  so that the face state stays between the two cell values.  On a face with
  omega_0 >= 1/2 (uniform cells, or the face nearer the upwind cell) Van
  Leer's psi < 2 keeps it there by itself; where the downwind cell is the
  nearer one, (1 - omega_0) psi can reach 2 (1 - omega_0) > 1 and the
  uncapped state would overshoot the downwind value.
* Sensor: beta = |s - Delta| / (|s| + |Delta| + eps) per face side and
  sensed variable; a cell takes the largest beta over the faces on which it
  is the upwind cell.  theta = clip((beta_hi - beta) / (beta_hi - beta_lo)).
* Blend: U = theta_f U_high + (1 - theta_f) U_limited, theta_f = min over the
  two cells of the face.
"""
from __future__ import annotations

import numpy as np

BETA_LO = 0.6
BETA_HI = 0.9


def vanleer_psi(r):
    r = np.asarray(r, dtype=np.float64)
    return np.where(r > 0.0, 2.0 * r / (1.0 + r), 0.0)


def vanleer_increment(s, delta):
    prod = s * delta
    safe = np.where(prod > 0.0, s + delta, 1.0)
    return np.where(prod > 0.0, 2.0 * prod / safe, 0.0)


def limited_increment(s, delta, w_down):
    """(1 - omega_0) psi Delta with w_down = 1 - omega_0 (the downwind cell's
    interpolation weight), its magnitude capped at |Delta|."""
    inc = w_down * vanleer_increment(s, delta)
    return np.where(np.abs(inc) > np.abs(delta), delta, inc)


def limited_states(mesh, geo, U, G1):
    """Van Leer limited (U_L, U_R) per face."""
    P, N = mesh.owner, mesh.neighbour
    w = geo.omega[:, None]
    dL = U[N] - U[P]
    sL = 2.0 * np.einsum("fva,fa->fv", G1[P], geo.d) - dL
    UL = U[P] + limited_increment(sL, dL, 1.0 - w)
    dR = U[P] - U[N]
    sR = 2.0 * np.einsum("fva,fa->fv", G1[N], -geo.d) - dR
    UR = U[N] + limited_increment(sR, dR, w)
    return UL, UR


def sensed_vars(n_v):
    return [0] if n_v == 1 else [0, n_v - 1]


def face_beta(phi0, phi1, d0):
    """beta for one frame: cell 0 upwind, d0 = phi_0^(1)."""
    delta = phi1 - phi0
    s = d0 - delta
    eps = 1e-8 * (np.abs(phi0) + np.abs(phi1)) + 1e-30
    return np.abs(s - delta) / (np.abs(s) + np.abs(delta) + eps)


def classical_theta(mesh, geo, U, G1):
    P, N = mesh.owner, mesh.neighbour
    beta = np.zeros(mesh.n_cells)
    for v in sensed_vars(U.shape[1]):
        bP = face_beta(U[P, v], U[N, v], 2.0 * np.einsum("fa,fa->f", G1[P, v], geo.d))
        bN = face_beta(U[N, v], U[P, v], 2.0 * np.einsum("fa,fa->f", G1[N, v], -geo.d))
        np.maximum.at(beta, P, bP)
        np.maximum.at(beta, N, bN)
    return np.clip((BETA_HI - beta) / (BETA_HI - BETA_LO), 0.0, 1.0), beta


def blend(UHL, UHR, ULL, ULR, theta, mesh):
    tf = np.minimum(theta[mesh.owner], theta[mesh.neighbour])[:, None]
    return tf * UHL + (1.0 - tf) * ULL, tf * UHR + (1.0 - tf) * ULR
