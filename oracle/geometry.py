"""Oracle: mesh geometry and the per-face scalars of the method (FP64).

Test infrastructure only: a slow, plain reference that nothing on the product
path may import.

Geometry is textbook finite-volume geometry (the paper does not spell it out):
* 2-D face (edge a->b): area vector S = (t_y, -t_x), t = b - a; centre = midpoint.
* 3-D face: triangle fan about the vertex average c; S = sum of the triangle
  area vectors; centre = triangle centroids weighted by triangle area.
* Cell: volume and centroid from the simplices (x_e, c, p_k, p_k+1) with x_e
  the mean of the cell's face centres (2-D: triangles (x_e, a, b)).

Face scalars follow Sec. 2.2: d = x_N - x_P (centre-to-centre vector),
omega = |x_N - x_f| / (|x_P - x_f| + |x_N - x_f|) (the linear-interpolation
weight of the owner) and the growth rate g = omega / (1 - omega)
= |x_N - x_f| / |x_f - x_P|.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class Geometry:
    S: np.ndarray      # [nf, d] area vector, owner -> neighbour
    xf: np.ndarray     # [nf, d] face centre (owner frame)
    V: np.ndarray      # [nc]
    xc: np.ndarray     # [nc, d]
    d: np.ndarray      # [nf, d] x_N (+ shift) - x_P
    omega: np.ndarray  # [nf]
    g: np.ndarray      # [nf]


def _faces_by_size(mesh):
    cnt = np.diff(mesh.face_ptr)
    for m in np.unique(cnt):
        fs = np.nonzero(cnt == m)[0]
        base = mesh.face_ptr[fs]
        P = np.stack([mesh.nodes[mesh.face_nodes[base + k]] for k in range(m)], 1)
        yield fs, P


def face_geometry(mesh):
    """S, face centre and the fan centre (vertex average) of every face."""
    nf, d = mesh.n_faces, mesh.dim
    S = np.zeros((nf, d))
    xf = np.zeros((nf, d))
    fan_c = np.zeros((nf, d))
    for fs, P in _faces_by_size(mesh):
        if d == 2:
            t = P[:, 1] - P[:, 0]
            S[fs] = np.stack([t[:, 1], -t[:, 0]], 1)
            xf[fs] = 0.5 * (P[:, 0] + P[:, 1])
            fan_c[fs] = xf[fs]
            continue
        m = P.shape[1]
        c = P.mean(axis=1)
        Ssum = np.zeros((len(fs), 3))
        asum = np.zeros(len(fs))
        cen = np.zeros((len(fs), 3))
        for k in range(m):
            q1, q2 = P[:, k], P[:, (k + 1) % m]
            s = 0.5 * np.cross(q1 - c, q2 - c)
            a = np.linalg.norm(s, axis=1)
            Ssum += s
            asum += a
            cen += a[:, None] * (c + q1 + q2) / 3.0
        S[fs] = Ssum
        xf[fs] = cen / asum[:, None]
        fan_c[fs] = c
    return S, xf, fan_c


def _half_faces(mesh):
    """(face, cell, sign, translation) for both sides of every face."""
    nf = mesh.n_faces
    f = np.concatenate([np.arange(nf), np.arange(nf)])
    cell = np.concatenate([mesh.owner, mesh.neighbour]).astype(np.int64)
    sgn = np.concatenate([np.ones(nf), -np.ones(nf)])
    tr = np.concatenate([np.zeros_like(mesh.shift), -mesh.shift])
    return f, cell, sgn, tr


def cell_geometry(mesh, S, xf, fan_c):
    nc, d = mesh.n_cells, mesh.dim
    hf, hc, hs, ht = _half_faces(mesh)
    nface = np.bincount(hc, minlength=nc).astype(np.float64)
    xe = np.stack([np.bincount(hc, weights=xf[hf, a] + ht[:, a], minlength=nc)
                   for a in range(d)], 1) / nface[:, None]
    V = np.zeros(nc)
    mom = np.zeros((nc, d))
    nf = mesh.n_faces
    for fs, P in _faces_by_size(mesh):
        m = P.shape[1]
        for side in (0, 1):
            if side == 0:
                cells = mesh.owner[fs].astype(np.int64)
                Q = P
                fc = fan_c[fs]
            else:
                cells = mesh.neighbour[fs].astype(np.int64)
                Q = P[:, ::-1] - mesh.shift[fs][:, None, :]
                fc = fan_c[fs] - mesh.shift[fs]
            e = xe[cells]
            if d == 2:
                a, b = Q[:, 0], Q[:, 1]
                v = 0.5 * ((a[:, 0] - e[:, 0]) * (b[:, 1] - e[:, 1]) -
                           (a[:, 1] - e[:, 1]) * (b[:, 0] - e[:, 0]))
                V += np.bincount(cells, weights=v, minlength=nc)
                cen = (e + a + b) / 3.0
                for ax in range(d):
                    mom[:, ax] += np.bincount(cells, weights=v * cen[:, ax], minlength=nc)
                continue
            for k in range(m):
                q1, q2 = Q[:, k], Q[:, (k + 1) % m]
                v = np.einsum("ij,ij->i", fc - e, np.cross(q1 - e, q2 - e)) / 6.0
                V += np.bincount(cells, weights=v, minlength=nc)
                cen = (e + fc + q1 + q2) / 4.0
                for ax in range(d):
                    mom[:, ax] += np.bincount(cells, weights=v * cen[:, ax], minlength=nc)
    del nf
    return V, mom / V[:, None]


def face_scalars(mesh, xc, xf):
    """d, omega, g per face (Sec. 2.2, the growth-rate and weight equations)."""
    xP = xc[mesh.owner]
    xN = xc[mesh.neighbour] + mesh.shift
    d = xN - xP
    dP = np.linalg.norm(xP - xf, axis=1)
    dN = np.linalg.norm(xN - xf, axis=1)
    omega = dN / (dP + dN)
    g = omega / (1.0 - omega)
    return d, omega, g


def geometry(mesh):
    S, xf, fan_c = face_geometry(mesh)
    V, xc = cell_geometry(mesh, S, xf, fan_c)
    d, omega, g = face_scalars(mesh, xc, xf)
    return Geometry(S, xf, V, xc, d, omega, g)
