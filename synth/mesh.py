"""Seeded synthetic periodic meshes in face-addressed (owner/neighbour) form.

The finite-volume storage model the method is written for is the
face-addressed unstructured mesh: a cell learns about its neighbours only
through the faces it shares with them (Sec. 2.1, Fig. meshTopo).  This module
produces such meshes; it holds none of the method's arithmetic (no geometry
integrals, gradients, coefficients or fluxes).

Conventions shared by every generator
-------------------------------------
* ``nodes`` are *unwrapped* lattice nodes: periodic boundaries duplicate the
  nodes of the opposite side, and duplicated nodes carry the same jitter, so
  each cell is geometrically compact in its own frame.
* A face is listed once.  Its node list is given in the owner's frame and
  ordered so that the right-hand normal points from owner to neighbour
  (2-D: for the edge a->b the normal is (t_y, -t_x) with t = b - a;
  3-D: (p1 - p0) x (p2 - p0) for a planar face).
* ``shift[f]`` translates the neighbour's geometry into the owner's frame
  (zero for faces that do not cross a periodic boundary).
* Every face has two cells: all generated domains are fully periodic.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from itertools import permutations

import numpy as np


@dataclass
class Mesh:
    dim: int
    nodes: np.ndarray          # [n_nodes, dim] float64
    face_ptr: np.ndarray       # [n_faces + 1] int64
    face_nodes: np.ndarray     # [face_ptr[-1]] int32
    owner: np.ndarray          # [n_faces] int32
    neighbour: np.ndarray      # [n_faces] int32
    shift: np.ndarray          # [n_faces, dim] float64
    n_cells: int
    lengths: tuple             # periodic box size per axis
    info: dict = field(default_factory=dict)
    # boundary faces: neighbour = -1 and patch[f] >= 0 (the owner is the
    # adjacent cell, the face normal points out of the domain); None when
    # every face is interior or periodic
    patch: np.ndarray | None = None

    @property
    def n_faces(self) -> int:
        return int(self.owner.shape[0])

    @property
    def n_nodes(self) -> int:
        return int(self.nodes.shape[0])

    def permuted(self, new_of_old: np.ndarray) -> "Mesh":
        """The same mesh with cells relabelled ``c -> new_of_old[c]``."""
        p = np.asarray(new_of_old, dtype=np.int64)
        info = dict(self.info)
        if "parent_hex" in info:
            ph = np.empty_like(info["parent_hex"])
            ph[p] = info["parent_hex"]
            info["parent_hex"] = ph
        nei = np.where(self.neighbour >= 0, p[np.maximum(self.neighbour, 0)], -1)
        return Mesh(self.dim, self.nodes, self.face_ptr, self.face_nodes,
                    p[self.owner].astype(np.int32), nei.astype(np.int32),
                    self.shift, self.n_cells, self.lengths, info, self.patch)


def bounded(mesh: Mesh, axis: int = 0) -> Mesh:
    """Open the periodic direction ``axis`` of a lattice mesh made by
    ``periodic_2d`` / ``periodic_3d`` (before any permutation): every face
    that wrapped around becomes two boundary faces, one per end of the
    lattice, each owned by the cell next to it with its normal pointing out of
    the domain (the copy has its nodes moved to the other end's node layer
    and reversed).  Patch 2 axis is the end at the origin, 2 axis + 1 the far
    end."""
    n = mesh.info["lattice"]
    NX = n[0] + 1
    NY = n[1] + 1
    stride = (1, NX, NX * NY)[axis]
    wrap = mesh.shift[:, axis] != 0.0
    fi = np.nonzero(wrap)[0]
    cnt = np.diff(mesh.face_ptr)
    new_nodes, new_cnt = [], []
    # shift > 0: the owner is the last cell and the face sits on the far node
    # layer; shift < 0: the owner is the first cell, face on the origin layer
    high = mesh.shift[fi, axis] > 0
    for f, hi in zip(fi, high):
        nodes = mesh.face_nodes[mesh.face_ptr[f]:mesh.face_ptr[f + 1]].astype(np.int64)
        moved = nodes - n[axis] * stride if hi else nodes + n[axis] * stride
        new_nodes.append(moved[::-1])
        new_cnt.append(cnt[f])
    owner = np.concatenate([mesh.owner, mesh.neighbour[fi]]).astype(np.int32)
    neigh = mesh.neighbour.copy()
    neigh[fi] = -1
    neigh = np.concatenate([neigh, np.full(fi.size, -1, dtype=np.int32)]).astype(np.int32)
    patch = np.full(owner.size, -1, dtype=np.int32)
    patch[fi] = np.where(high, 2 * axis + 1, 2 * axis)
    patch[mesh.n_faces:] = np.where(high, 2 * axis, 2 * axis + 1)
    shift = np.concatenate([mesh.shift, np.zeros((fi.size, mesh.dim))])
    shift[fi] = 0.0
    lens = np.concatenate([cnt, np.asarray(new_cnt, dtype=np.int64)])
    ptr = np.zeros(lens.size + 1, dtype=np.int64)
    np.cumsum(lens, out=ptr[1:])
    fn = np.concatenate([mesh.face_nodes] + [x.astype(np.int32) for x in new_nodes]).astype(np.int32)
    info = dict(mesh.info)
    info["open_axis"] = axis
    return Mesh(mesh.dim, mesh.nodes, ptr, fn, owner, neigh, shift, mesh.n_cells, mesh.lengths, info, patch)


def graded_spacing(h1, growth, height):
    """Node coordinates 0 .. height whose spacings grow geometrically from
    h1 by the factor growth (the last cell absorbs the remainder, merged into
    its neighbour when it would be thinner than half of it)."""
    ys = [0.0]
    h = h1
    while ys[-1] + h < height:
        ys.append(ys[-1] + h)
        h *= growth
    if len(ys) > 2 and height - ys[-1] < 0.5 * (ys[-1] - ys[-2]):
        ys[-1] = height
    else:
        ys.append(height)
    return np.asarray(ys)


def boundary_layer_2d(nx, length, h1, growth, height):
    """Quadrilateral boundary-layer mesh: nx uniform columns over [0, length]
    (periodic in x) and rows growing away from the wall y = 0 by the factor
    growth from the first height h1 up to height; y is open (patch 2: the
    wall, patch 3: the top)."""
    ys = graded_spacing(h1, growth, height)
    m = periodic_2d(nx, ys.size - 1, lengths=(length, height), ycoords=ys)
    return bounded(m, 1)


def _lattice_coords(n, L, coords):
    if coords is None:
        return np.linspace(0.0, L, n + 1)
    c = np.asarray(coords, dtype=np.float64)
    if c.shape != (n + 1,) or abs(c[0]) > 0 or abs(c[-1] - L) > 1e-12 * max(1.0, L):
        raise ValueError("coords must have n+1 entries running from 0 to L")
    return c


def _jitter(rng, shape, dim, amp):
    if amp == 0.0:
        return np.zeros(shape + (dim,))
    return rng.uniform(-amp, amp, size=shape + (dim,))


# ---------------------------------------------------------------------------
# 2-D: periodic quadrilateral lattice, optional triangle splits and pentagons
# ---------------------------------------------------------------------------

def periodic_2d(nx, ny, lengths=(1.0, 1.0), jitter=0.0, seed=0, split=0.0,
                split_seed=None, diagonal="main", pentagon_frac=0.0, perm_seed=None,
                xcoords=None, ycoords=None):
    """Periodic 2-D mesh from an ``nx`` x ``ny`` quad lattice.

    jitter        : every lattice node moves by U(-jitter*h, +jitter*h) per axis
                    (h = mean spacing along that axis); periodic images share it.
    split         : fraction of quads cut into two triangles (1.0 = all).
    diagonal      : "main" cuts along (i,j)-(i+1,j+1); "seeded" picks per quad.
    pentagon_frac : fraction of the unsplit quads merged with one adjacent
                    triangle into a pentagon (merges never cross the boundary).
    perm_seed     : if given, cells are listed in a seeded random order.
    """
    if nx < 2 or ny < 2:
        raise ValueError("need at least 2 cells per periodic direction")
    Lx, Ly = lengths
    xs = _lattice_coords(nx, Lx, xcoords)
    ys = _lattice_coords(ny, Ly, ycoords)
    rng = np.random.default_rng(seed)
    jit = _jitter(rng, (ny, nx), 2, 1.0) * np.array([jitter * Lx / nx, jitter * Ly / ny])

    I, J = np.meshgrid(np.arange(nx + 1), np.arange(ny + 1), indexing="xy")
    nodes = np.stack([xs[I], ys[J]], axis=-1) + jit[J % ny, I % nx]
    nodes = nodes.reshape(-1, 2)

    def nid(i, j):
        return i + (nx + 1) * j

    srng = np.random.default_rng(split_seed if split_seed is not None else seed + 1)
    do_split = srng.random((ny, nx)) < split
    if diagonal == "main":
        diag_main = np.ones((ny, nx), dtype=bool)
    elif diagonal == "seeded":
        diag_main = srng.random((ny, nx)) < 0.5
    else:
        raise ValueError(diagonal)

    cells = []       # CCW lists of (i, j) lattice coordinates
    kind = []        # 0 quad, 1 triangle
    quad_at = {}
    tri_at = {}
    for j in range(ny):
        for i in range(nx):
            c00, c10, c11, c01 = (i, j), (i + 1, j), (i + 1, j + 1), (i, j + 1)
            if not do_split[j, i]:
                quad_at[(i, j)] = len(cells)
                cells.append([c00, c10, c11, c01]); kind.append(0)
            elif diag_main[j, i]:
                tri_at[(i, j)] = (len(cells), len(cells) + 1)
                cells.append([c00, c10, c11]); kind.append(1)
                cells.append([c00, c11, c01]); kind.append(1)
            else:
                tri_at[(i, j)] = (len(cells), len(cells) + 1)
                cells.append([c00, c10, c01]); kind.append(1)
                cells.append([c10, c11, c01]); kind.append(1)

    n_pent = 0
    if pentagon_frac > 0.0 and quad_at:
        prng = np.random.default_rng((split_seed if split_seed is not None else seed + 1) + 7919)
        keys = sorted(quad_at)
        order = prng.permutation(len(keys))
        target = int(round(pentagon_frac * len(keys)))
        used = set()
        dead = set()
        for q in order:
            if n_pent >= target:
                break
            i, j = keys[q]
            qc = quad_at[(i, j)]
            A = cells[qc]
            for k in range(4):
                u, v = A[k], A[(k + 1) % 4]
                # neighbouring lattice quad across edge u->v (outward side)
                di, dj = v[1] - u[1], -(v[0] - u[0])
                ni, nj = i + di, j + dj
                if not (0 <= ni < nx and 0 <= nj < ny) or (ni, nj) not in tri_at:
                    continue
                hit = None
                for tc in tri_at[(ni, nj)]:
                    if tc in used:
                        continue
                    B = cells[tc]
                    for m in range(3):
                        if B[m] == v and B[(m + 1) % 3] == u:
                            hit = (tc, B[(m + 2) % 3])
                if hit is None:
                    continue
                tc, third = hit
                cells[qc] = [A[(k + 1) % 4], A[(k + 2) % 4], A[(k + 3) % 4], A[k], third]
                kind[qc] = 2
                used.add(tc)
                dead.add(tc)
                n_pent += 1
                break
        if dead:
            keep = [c for c in range(len(cells)) if c not in dead]
            cells = [cells[c] for c in keep]
            kind = [kind[c] for c in keep]

    # half-edges and matching
    hc, ha, hb = [], [], []
    for c, poly in enumerate(cells):
        m = len(poly)
        for k in range(m):
            hc.append(c); ha.append(poly[k]); hb.append(poly[(k + 1) % m])
    hc = np.array(hc, dtype=np.int64)
    ha = np.array(ha, dtype=np.int64)
    hb = np.array(hb, dtype=np.int64)
    pa = (ha[:, 0] % nx) + nx * (ha[:, 1] % ny)
    pb = (hb[:, 0] % nx) + nx * (hb[:, 1] % ny)
    dd = hb - ha                      # in {-1,0,1}^2 (+ unchanged by wrap)
    fwd = (pa < pb) | ((pa == pb) & ((dd[:, 0] > 0) | ((dd[:, 0] == 0) & (dd[:, 1] > 0))))
    k1 = np.where(fwd, pa, pb)
    k2 = np.where(fwd, pb, pa)
    s = np.where(fwd, 1, -1)
    key = ((k1 * (nx * ny) + k2) * 3 + (s * dd[:, 0] + 1)) * 3 + (s * dd[:, 1] + 1)
    order = np.lexsort((~fwd, key))
    ks = key[order]
    if ks.size % 2 or not np.all(ks[0::2] == ks[1::2]):
        raise RuntimeError("2-D mesh: unmatched half-edges")
    h_own = order[0::2]
    h_nei = order[1::2]
    owner = hc[h_own]
    neigh = hc[h_nei]
    a_own = ha[h_own]
    b_own = hb[h_own]
    b_nei = hb[h_nei]           # neighbour's half-edge runs b->a, so its end is a
    face_nodes = np.stack([nid(a_own[:, 0], a_own[:, 1]), nid(b_own[:, 0], b_own[:, 1])], 1)
    lat = (a_own - b_nei).astype(np.float64)
    shift = np.stack([lat[:, 0] / nx * Lx, lat[:, 1] / ny * Ly], 1)

    n_cells = len(cells)
    kinds = np.array(kind)
    info = {"n_tri": int((kinds == 1).sum()), "n_quad": int((kinds == 0).sum()),
            "n_pent": int((kinds == 2).sum()), "lattice": (nx, ny)}
    mesh = Mesh(2, nodes, np.arange(0, 2 * len(owner) + 1, 2, dtype=np.int64),
                face_nodes.reshape(-1).astype(np.int32), owner.astype(np.int32),
                neigh.astype(np.int32), shift, n_cells, (Lx, Ly), info)
    if perm_seed is not None:
        mesh = mesh.permuted(np.random.default_rng(perm_seed).permutation(n_cells))
    return mesh


# ---------------------------------------------------------------------------
# 3-D: periodic hex lattice with per-hex split types
# ---------------------------------------------------------------------------
# Hex corner b = bx + 2*by + 4*bz sits at (bx, by, bz) of the unit cube.
# Side s = 2*a + (0 minus | 1 plus) is the hex face normal to axis a.
# On a lattice face normal to a, (u, v) = ((a+1)%3, (a+2)%3); its corners are
# c00, c10, c11, c01 and every split uses the diagonal c00-c11, so splits of
# neighbouring hexes always conform.  Piece 0 = whole quad, piece 1 =
# (c00, c10, c11), piece 2 = (c00, c11, c01).

HEX, KUHN6, PRISM_X, PRISM_Y, PRISM_Z = 0, 1, 2, 3, 4


def _corner(bits):
    return bits[0] + 2 * bits[1] + 4 * bits[2]


def _face_corners(a, side_plus):
    u, v = (a + 1) % 3, (a + 2) % 3
    out = []
    for (du, dv) in ((0, 0), (1, 0), (1, 1), (0, 1)):
        b = [0, 0, 0]
        b[a] = 1 if side_plus else 0
        b[u] = du
        b[v] = dv
        out.append(_corner(b))
    return out  # CCW about +e_a


_CUBE = np.array([[b & 1, (b >> 1) & 1, (b >> 2) & 1] for b in range(8)], dtype=np.float64)


def _orient_outward(poly, centre):
    p = _CUBE[poly]
    c = p.mean(0)
    n = np.zeros(3)
    for k in range(len(poly)):
        n += np.cross(p[k] - c, p[(k + 1) % len(poly)] - c)
    return list(poly) if np.dot(n, c - centre) > 0 else list(poly[::-1])


def _local_topology(kind):
    """Sub-cells of one hex: (faces per sub-cell, boundary lookup, internal faces)."""
    if kind == HEX:
        subs = [list(range(8))]
    elif kind == KUHN6:
        subs = []
        for perm in permutations(range(3)):
            b = [0, 0, 0]
            path = [_corner(b)]
            for ax in perm:
                b[ax] = 1
                path.append(_corner(b))
            subs.append(path)
    else:
        a = kind - PRISM_X
        corners0 = {}
        corners1 = {}
        u, v = (a + 1) % 3, (a + 2) % 3
        for (du, dv) in ((0, 0), (1, 0), (1, 1), (0, 1)):
            b = [0, 0, 0]; b[u] = du; b[v] = dv
            corners0[(du, dv)] = _corner(b)
            b[a] = 1
            corners1[(du, dv)] = _corner(b)
        t1 = [(0, 0), (1, 0), (1, 1)]
        t2 = [(0, 0), (1, 1), (0, 1)]
        subs = [[corners0[t] for t in t1] + [corners1[t] for t in t1],
                [corners0[t] for t in t2] + [corners1[t] for t in t2]]
    faces_of = []
    for sc in subs:
        centre = _CUBE[sc].mean(0)
        if kind == HEX:
            fl = [_face_corners(a, sp) for a in range(3) for sp in (False, True)]
        elif kind == KUHN6:
            fl = [[sc[i] for i in range(4) if i != skip] for skip in range(4)]
        else:
            fl = [sc[0:3], sc[3:6]]
            for k in range(3):
                fl.append([sc[k], sc[(k + 1) % 3], sc[3 + (k + 1) % 3], sc[3 + k]])
        faces_of.append([_orient_outward(f, centre) for f in fl])
    # classify faces
    lookup = -np.ones((6, 3), dtype=np.int64)
    internal = {}
    for si, fl in enumerate(faces_of):
        for f in fl:
            P = _CUBE[f]
            side = None
            for a in range(3):
                if np.all(P[:, a] == 0):
                    side = 2 * a
                elif np.all(P[:, a] == 1):
                    side = 2 * a + 1
            if side is None:
                key = tuple(sorted(f))
                internal.setdefault(key, []).append((si, f))
                continue
            a = side // 2
            fc = _face_corners(a, side % 2 == 1)
            if len(f) == 4:
                lookup[side, :] = si
            else:
                t1 = {fc[0], fc[1], fc[2]}
                piece = 1 if set(f) == t1 else 2
                lookup[side, piece] = si
    ints = []
    for key, lst in internal.items():
        assert len(lst) == 2, (kind, key)
        (sa, fa), (sb, _fb) = lst
        ints.append((sa, sb, fa))
    return len(subs), lookup, ints


_TOPO = {k: _local_topology(k) for k in (HEX, KUHN6, PRISM_X, PRISM_Y, PRISM_Z)}


def periodic_3d(nx, ny=None, nz=None, lengths=(1.0, 1.0, 1.0), jitter=0.0, seed=0,
                kinds=None, coords=(None, None, None), perm_seed=None):
    """Periodic 3-D mesh from an ``nx`` x ``ny`` x ``nz`` hex lattice.

    kinds : per-hex split type array of shape (nz, ny, nx) with values HEX,
            KUHN6 (6 tetrahedra about the main diagonal), PRISM_{X,Y,Z}
            (2 prisms along that axis); a scalar applies to every hex.
            Lattice faces next to a split hex are cut into two triangles,
            which turns neighbouring hexes or prisms into polyhedra.
    """
    ny = nx if ny is None else ny
    nz = nx if nz is None else nz
    n = (nx, ny, nz)
    if min(n) < 2:
        raise ValueError("need at least 2 cells per periodic direction")
    L = np.asarray(lengths, dtype=np.float64)
    axes = [_lattice_coords(n[a], L[a], coords[a]) for a in range(3)]
    rng = np.random.default_rng(seed)
    h = L / np.array(n)
    jit = _jitter(rng, (nz, ny, nx), 3, 1.0) * (jitter * h)

    NX, NY, NZ = nx + 1, ny + 1, nz + 1
    kk, jj, ii = np.meshgrid(np.arange(NZ), np.arange(NY), np.arange(NX), indexing="ij")
    nodes = np.stack([axes[0][ii], axes[1][jj], axes[2][kk]], -1)
    nodes = nodes + jit[kk % nz, jj % ny, ii % nx]
    nodes = nodes.reshape(-1, 3)
    del kk, jj, ii

    if kinds is None:
        kinds = HEX
    kinds = np.broadcast_to(np.asarray(kinds, dtype=np.int8), (nz, ny, nx)).reshape(-1)
    nsub = np.array([_TOPO[k][0] for k in range(5)], dtype=np.int64)
    base = np.zeros(nx * ny * nz + 1, dtype=np.int64)
    np.cumsum(nsub[kinds], out=base[1:])
    n_cells = int(base[-1])
    lookup = np.stack([_TOPO[k][1] for k in range(5)])           # [5, 6, 3]
    needs = np.zeros((5, 6), dtype=bool)
    needs[KUHN6, :] = True
    for a in range(3):
        needs[PRISM_X + a, 2 * a:2 * a + 2] = True

    hex_idx = np.arange(nx * ny * nz, dtype=np.int64)
    hi = hex_idx % nx
    hj = (hex_idx // nx) % ny
    hk = hex_idx // (nx * ny)
    hijk = np.stack([hi, hj, hk], 1)

    def node_id(ijk):
        return (ijk[..., 0] + NX * (ijk[..., 1] + NY * ijk[..., 2])).astype(np.int64)

    f_nodes, f_ptrlen, f_own, f_nei, f_shift = [], [], [], [], []
    for a in range(3):
        u, v = (a + 1) % 3, (a + 2) % 3
        plus = hijk                                        # hex on the + side
        minus = hijk.copy()
        minus[:, a] = (minus[:, a] - 1) % n[a]
        wrap = plus[:, a] == 0
        h_plus = hex_idx
        h_minus = minus[:, 0] + nx * (minus[:, 1] + ny * minus[:, 2])
        k_plus = kinds[h_plus]
        k_minus = kinds[h_minus]
        split = needs[k_minus, 2 * a + 1] | needs[k_plus, 2 * a]
        # face corner lattice coords in the owner (= minus hex) frame
        org = minus.copy()
        org[:, a] = minus[:, a] + 1
        cuv = {}
        for (du, dv) in ((0, 0), (1, 0), (1, 1), (0, 1)):
            q = org.copy()
            q[:, u] += du
            q[:, v] += dv
            cuv[(du, dv)] = node_id(q)
        sh = np.zeros((nx * ny * nz, 3))
        sh[wrap, a] = L[a]
        for piece, corners in ((0, ((0, 0), (1, 0), (1, 1), (0, 1))),
                               (1, ((0, 0), (1, 0), (1, 1))),
                               (2, ((0, 0), (1, 1), (0, 1)))):
            sel = ~split if piece == 0 else split
            if not np.any(sel):
                continue
            own = base[h_minus[sel]] + lookup[k_minus[sel], 2 * a + 1, piece]
            nei = base[h_plus[sel]] + lookup[k_plus[sel], 2 * a, piece]
            f_own.append(own)
            f_nei.append(nei)
            f_nodes.append(np.stack([cuv[c][sel] for c in corners], 1))
            f_ptrlen.append(np.full(int(sel.sum()), len(corners), dtype=np.int64))
            f_shift.append(sh[sel])
    # faces inside split hexes
    for k in (KUHN6, PRISM_X, PRISM_Y, PRISM_Z):
        hs = np.nonzero(kinds == k)[0]
        if hs.size == 0:
            continue
        for (sa, sb, f) in _TOPO[k][2]:
            f_own.append(base[hs] + sa)
            f_nei.append(base[hs] + sb)
            cols = []
            for b in f:
                q = hijk[hs] + _CUBE[b].astype(np.int64)
                cols.append(node_id(q))
            f_nodes.append(np.stack(cols, 1))
            f_ptrlen.append(np.full(hs.size, len(f), dtype=np.int64))
            f_shift.append(np.zeros((hs.size, 3)))

    owner = np.concatenate(f_own)
    neigh = np.concatenate(f_nei)
    lens = np.concatenate(f_ptrlen)
    face_ptr = np.zeros(owner.size + 1, dtype=np.int64)
    np.cumsum(lens, out=face_ptr[1:])
    fn = np.empty(int(face_ptr[-1]), dtype=np.int32)
    off = 0
    for blk in f_nodes:
        m = blk.size
        fn[off:off + m] = blk.reshape(-1)
        off += m
    shift = np.concatenate(f_shift)
    counts = np.bincount(kinds, minlength=5)
    parent = np.repeat(np.arange(nx * ny * nz, dtype=np.int32), nsub[kinds])
    info = {"lattice": n, "n_hex_unsplit": int(counts[HEX]), "n_hex_kuhn": int(counts[KUHN6]),
            "n_hex_prism": int(counts[PRISM_X:].sum()), "parent_hex": parent}
    mesh = Mesh(3, nodes, face_ptr, fn, owner.astype(np.int32), neigh.astype(np.int32),
                shift, n_cells, tuple(float(x) for x in L), info)
    if perm_seed is not None:
        mesh = mesh.permuted(np.random.default_rng(perm_seed).permutation(n_cells))
    return mesh


def mixed_kinds(nx, ny=None, nz=None, split_frac=0.3, seed=0):
    """Seeded split pattern: ``split_frac`` of hexes split, half into 6
    tetrahedra and half into 2 prisms along a seeded axis."""
    ny = nx if ny is None else ny
    nz = nx if nz is None else nz
    rng = np.random.default_rng(seed)
    r = rng.random((nz, ny, nx))
    ax = rng.integers(0, 3, size=(nz, ny, nx))
    k = np.full((nz, ny, nx), HEX, dtype=np.int8)
    k[r < split_frac * 0.5] = KUHN6
    prism = (r >= split_frac * 0.5) & (r < split_frac)
    k[prism] = (PRISM_X + ax[prism]).astype(np.int8)
    return k
