"""Shared helpers for the GPU parity tests (test code only)."""
from __future__ import annotations

import numpy as np

from synth import mesh as M
from synth.mesh import Mesh


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (den if den > 0 else 1.0)


def oracle_params(p):
    """Keyword params of the binding -> oracle params dict."""
    out = dict(pde=p["pde"], scheme=p["scheme"], flux=p.get("flux", "upwind"), gamma=p.get("gamma", 1.4),
               adv_vel=p.get("adv_vel", (1.0, 0.5, 0.0)), burgers_dir=p.get("burgers_dir", (1.0, 1.0, 0.0)))
    return out


def submesh(mesh: Mesh, seeds, rings):
    """Cells within ``rings`` face-rings of ``seeds`` plus every face of them.

    Cells reached only through those faces become ghost cells whose face set
    is incomplete; quantities are exact for cells deep enough inside.
    Returns (sub, old_index_of_sub_cell).
    """
    nc = mesh.n_cells
    own, nei = mesh.owner.astype(np.int64), mesh.neighbour.astype(np.int64)
    inside = np.zeros(nc, dtype=bool)
    inside[np.asarray(seeds)] = True
    for _ in range(rings):
        fr = inside[own] | inside[nei]
        inside[own[fr]] = True
        inside[nei[fr]] = True
    fsel = np.nonzero(inside[own] | inside[nei])[0]
    cells = np.unique(np.concatenate([own[fsel], nei[fsel]]))
    new = -np.ones(nc, dtype=np.int64)
    new[cells] = np.arange(cells.size)
    cnt = np.diff(mesh.face_ptr)[fsel]
    ptr = np.zeros(fsel.size + 1, dtype=np.int64)
    np.cumsum(cnt, out=ptr[1:])
    idx = np.concatenate([np.arange(mesh.face_ptr[f], mesh.face_ptr[f + 1]) for f in fsel]) if fsel.size else \
        np.zeros(0, dtype=np.int64)
    sub = Mesh(mesh.dim, mesh.nodes, ptr, mesh.face_nodes[idx], new[own[fsel]].astype(np.int32),
               new[nei[fsel]].astype(np.int32), mesh.shift[fsel], int(cells.size), mesh.lengths, dict(mesh.info))
    return sub, cells, fsel


def small_meshes():
    """A spread of small periodic meshes with ragged partition tails."""
    return {
        "tri2d": M.periodic_2d(12, 10, jitter=0.2, seed=1, split=1.0, diagonal="main", perm_seed=3),
        "mixed2d": M.periodic_2d(14, 13, jitter=0.25, seed=2, split=0.5, diagonal="seeded",
                                 pentagon_frac=0.1, perm_seed=4),
        "tet3d": M.periodic_3d(5, 4, 3, jitter=0.2, seed=5, kinds=M.KUHN6, perm_seed=6),
        "hex3d": M.periodic_3d(7, 6, 5, jitter=0.2, seed=7, perm_seed=8),
        "mixed3d": M.periodic_3d(6, 5, 5, jitter=0.2, seed=9, kinds=M.mixed_kinds(6, 5, 5, 0.4, seed=10),
                                 perm_seed=11),
    }
