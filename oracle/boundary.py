"""Oracle: non-coupled boundaries through auxiliary cells (Sec. 2.6).

Test infrastructure only (FP64, plain NumPy); the product path never imports it.

The paper keeps the low-order treatment of Dirichlet and Neumann boundaries:
the boundary-face value follows from the condition, and the inversion gives
an auxiliary cell O on the far side of the face whose value makes the linear
interpolation between the boundary cell C and O return that face value:
    T_O = T_C + 2 (T_f - T_C).
Its Neumann example: with the outward normal gradient q and the distance
d_fC from the cell centre to the face centre, T_f = T_C + q d_fC, so that
(T_O - T_C) / (2 d_fC) = q again.

Readings taken here (the paper gives the values only):
* O is the mirror image of C in the face plane (through x_f, normal n):
  x_O = x_C + 2 ((x_f - x_C).n) n, V_O = V_C, so the face is midway
  (omega = 1/2, g = 1) and d = x_O - x_C is normal to the face; d_fC is the
  normal distance (x_f - x_C).n.  With d along n the auxiliary field is the
  exact mirror image of the cell's, so a slip wall passes no mass even on
  skewed cells.
* Conditions: Dirichlet (face value given), Neumann (outward normal
  gradient given), zero gradient (Neumann with q = 0, the transmissive end
  of a shock tube) and, for the Euler equations, a slip wall (density and
  energy copied, momentum reflected in the face plane).
* The DOLINC differentials of O are those of the field continued across the
  face by the same rule: with R = I - 2 n n^T the reflection in the face
  plane (n the outward unit normal),
    symmetric conditions (zero gradient, Neumann, slip wall):
        grad O = R grad C,  hess O = R hess C R,
        and for the momentum of a slip wall (a reflected vector field)
        grad m_O = R (grad m_C) R, hess m_O,i = sum_k R_ik R hess m_C,k R;
    Dirichlet (the field continued antisymmetrically about T_f):
        grad O = -R grad C,  hess O = -R hess C R.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import flux as _flux
from . import geometry as _geom
from . import limiter as _lim
from . import scheme as _sch

ZERO_GRADIENT, DIRICHLET, NEUMANN, SLIP_WALL = 0, 1, 2, 3


@dataclass
class Extended:
    mesh: object            # mesh with one auxiliary cell per boundary face appended
    geo: object
    n_cells: int            # interior cells
    ghost_cell: np.ndarray  # [nb] boundary cell C of auxiliary cell n_cells + k
    ghost_face: np.ndarray  # [nb] its boundary face
    patch: np.ndarray       # [nb]
    normal: np.ndarray      # [nb, dim] outward unit normal
    dist: np.ndarray        # [nb] (x_f - x_C).n


def extend(mesh):
    """Append the auxiliary cells and their geometry."""
    from synth.mesh import Mesh
    bf = np.nonzero(mesh.neighbour < 0)[0]
    nc = mesh.n_cells
    nei = mesh.neighbour.astype(np.int64).copy()
    nei[bf] = nc + np.arange(bf.size)
    ext = Mesh(mesh.dim, mesh.nodes, mesh.face_ptr, mesh.face_nodes, mesh.owner.astype(np.int32),
               nei.astype(np.int32), mesh.shift, nc + bf.size, mesh.lengths, dict(mesh.info))
    S, xf, fan_c = _geom.face_geometry(ext)
    with np.errstate(divide="ignore", invalid="ignore"):
        V, xc = _geom.cell_geometry(ext, S, xf, fan_c)
    C = mesh.owner[bf].astype(np.int64)
    n = S[bf] / np.linalg.norm(S[bf], axis=1)[:, None]
    dist = np.einsum("ka,ka->k", xf[bf] - xc[C], n)
    V[nc:] = V[C]
    xc[nc:] = xc[C] + 2.0 * dist[:, None] * n
    d, omega, g = _geom.face_scalars(ext, xc, xf)
    geo = _geom.Geometry(S, xf, V, xc, d, omega, g)
    return Extended(ext, geo, nc, C, bf, mesh.patch[bf].astype(np.int64), n, dist)


def _reflections(X):
    n = X.normal
    return np.eye(n.shape[1])[None] - 2.0 * n[:, :, None] * n[:, None, :]     # [nb, d, d]


def _bc_of(X, bcs, nv):
    """Per auxiliary cell: type and value vector (defaults: zero gradient)."""
    typ = np.zeros(X.ghost_cell.size, dtype=np.int64)
    val = np.zeros((X.ghost_cell.size, nv))
    for p, spec in (bcs or {}).items():
        sel = X.patch == p
        typ[sel] = spec[0]
        if len(spec) > 1 and spec[1] is not None:
            val[sel] = np.asarray(spec[1], dtype=np.float64)
    return typ, val


def fill_values(X, U, bcs, euler):
    """U [n_cells + nb, nv]: auxiliary rows from the boundary conditions."""
    nc, C = X.n_cells, X.ghost_cell
    nv = U.shape[1]
    typ, val = _bc_of(X, bcs, nv)
    UC = U[C]
    Tf = UC.copy()                                                   # zero gradient
    Tf = np.where((typ == DIRICHLET)[:, None], val, Tf)
    Tf = np.where((typ == NEUMANN)[:, None], UC + val * X.dist[:, None], Tf)
    UO = UC + 2.0 * (Tf - UC)
    if euler:
        wall = typ == SLIP_WALL
        R = _reflections(X)
        mom = np.einsum("kij,kj->ki", R, UC[:, 1:1 + R.shape[1]])
        UO[wall, 1:1 + R.shape[1]] = mom[wall]
    U[nc:] = UO
    return U


def fill_grad(X, G, bcs, euler):
    """G [n_cells + nb, nv, dim]: auxiliary rows (gradient of each variable)."""
    nc, C = X.n_cells, X.ghost_cell
    typ, _ = _bc_of(X, bcs, G.shape[1])
    R = _reflections(X)
    GC = G[C]
    GO = np.einsum("kab,kvb->kva", R, GC)                             # R grad
    GO = np.where((typ == DIRICHLET)[:, None, None], -GO, GO)
    if euler:
        wall = typ == SLIP_WALL
        D = R.shape[1]
        J = np.einsum("kia,kab,kbj->kij", R, GC[:, 1:1 + D], R)       # R (grad m) R
        GO[wall, 1:1 + D] = J[wall]
    G[nc:] = GO
    return G


def fill_hess(X, H, bcs, euler):
    """H [n_cells + nb, nv, dim, dim]: auxiliary rows (second derivatives)."""
    nc, C = X.n_cells, X.ghost_cell
    typ, _ = _bc_of(X, bcs, H.shape[1])
    R = _reflections(X)
    HC = H[C]
    HO = np.einsum("kac,kvcd,kdb->kvab", R, HC, R)
    HO = np.where((typ == DIRICHLET)[:, None, None, None], -HO, HO)
    if euler:
        wall = typ == SLIP_WALL
        D = R.shape[1]
        Hm = np.einsum("kij,kac,kjcd,kdb->kiab", R, R, HC[:, 1:1 + D], R)
        HO[wall, 1:1 + D] = Hm[wall]
    H[nc:] = HO
    return H


def cell_derivs(X, U, order, bcs, euler):
    """U, G1, G2 on the extended mesh with every auxiliary row from the
    boundary conditions (each derivative after the rows it is built from)."""
    U = fill_values(X, U, bcs, euler)
    G = [U]
    if order >= 1:
        G1 = _sch.gauss_linear(X.mesh, X.geo, U)
        G.append(fill_grad(X, G1, bcs, euler))
    if order >= 2:
        G2 = _sch.gauss_linear(X.mesh, X.geo, G[1])
        G.append(fill_hess(X, G2, bcs, euler))
    return G


def residual(X, U, params, bcs, theta=None):
    """R = dU/dt for the interior cells (U [n_cells, nv])."""
    U = np.asarray(U, dtype=np.float64).reshape(X.n_cells, -1)
    nv = U.shape[1]
    euler = params["pde"] == "euler"
    Ue = np.zeros((X.mesh.n_cells, nv))
    Ue[:X.n_cells] = U
    scheme = params["scheme"]
    order = max(_sch.scheme_order(scheme), 1 if theta is not None else 0)
    G = cell_derivs(X, Ue, order, bcs, euler)
    UL, UR, G = _sch.face_states(X.mesh, X.geo, G[0], scheme, G)
    if theta is not None:
        th = np.concatenate([theta, np.asarray(theta)[X.ghost_cell]])
        LL, LR = _lim.limited_states(X.mesh, X.geo, G[0], G[1])
        UL, UR = _lim.blend(UL, UR, LL, LR, th, X.mesh)
    pde = params["pde"]
    if pde == "advection":
        F = _flux.upwind(UL, UR, X.geo.S, params.get("adv_vel", (1.0, 0.5, 0.0)))
    elif pde == "burgers":
        F = _flux.godunov_burgers(UL, UR, X.geo.S, params.get("burgers_dir", (1.0, 1.0, 0.0)))
    else:
        gamma = params.get("gamma", 1.4)
        rL, _v, _E, pL = _flux.euler_primitives(UL, gamma)
        rR, _v, _E, pR = _flux.euler_primitives(UR, gamma)
        UL = np.where((~((rL > 0) & (pL > 0)))[:, None], G[0][X.mesh.owner], UL)
        UR = np.where((~((rR > 0) & (pR > 0)))[:, None], G[0][X.mesh.neighbour], UR)
        F = (_flux.rusanov if params["flux"] == "rusanov" else _flux.hllc)(UL, UR, X.geo.S, gamma)
    nc = X.n_cells
    R = np.zeros((nc, nv))
    own, nei = X.mesh.owner, X.mesh.neighbour
    inner = nei < nc
    for v in range(nv):
        R[:, v] = -(np.bincount(own, weights=F[:, v], minlength=nc) -
                    np.bincount(nei[inner], weights=F[inner, v], minlength=nc)) / X.geo.V[:nc]
    return R


def rk_step(X, U, dt, params, bcs, theta=None):
    from .solver import ssp_rk3
    return ssp_rk3(np.asarray(U, dtype=np.float64), dt, lambda Y: residual(X, Y, params, bcs, theta))
