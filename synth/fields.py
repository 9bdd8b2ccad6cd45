"""Seeded initial data and closed-form solutions on ``synth.mesh`` meshes.

Holds no arithmetic of the finite-volume method itself.  Cell averages of a
closed-form field are obtained by splitting each cell into simplices (a
triangle fan about each face's vertex average, closed at an interior point of
the cell) and integrating with collapsed (Duffy) Gauss-Legendre rules.
"""
from __future__ import annotations

import numpy as np

GAMMA = 1.4


# --------------------------------------------------------------------------
# cell simplices
# --------------------------------------------------------------------------

def _interior_points(mesh):
    """A point inside each cell: the mean of its faces' vertex averages."""
    d = mesh.dim
    fc = np.zeros((mesh.n_faces, d))
    cnt = np.diff(mesh.face_ptr)
    idx = np.repeat(np.arange(mesh.n_faces), cnt)
    for a in range(d):
        fc[:, a] = np.bincount(idx, weights=mesh.nodes[mesh.face_nodes, a],
                               minlength=mesh.n_faces) / cnt
    acc = np.zeros((mesh.n_cells, d))
    two = mesh.neighbour >= 0  # boundary faces have one cell
    nei = mesh.neighbour[two]
    num = np.bincount(mesh.owner, minlength=mesh.n_cells) + np.bincount(nei, minlength=mesh.n_cells)
    for a in range(d):
        acc[:, a] = (np.bincount(mesh.owner, weights=fc[:, a], minlength=mesh.n_cells) +
                     np.bincount(nei, weights=fc[two, a] - mesh.shift[two, a], minlength=mesh.n_cells))
    return acc / num[:, None], fc


def cell_simplices(mesh):
    """Positively oriented simplices tiling every cell.

    Returns (verts [n_s, dim+1, dim], cell [n_s]).  In 3-D each face is fanned
    into triangles about its vertex average; each triangle is closed into a
    tetrahedron with the cell's interior point.
    """
    d = mesh.dim
    centre, fcen = _interior_points(mesh)
    cnt = np.diff(mesh.face_ptr)
    out_v, out_c = [], []
    for m in np.unique(cnt):
        fs = fs0 = np.nonzero(cnt == m)[0]
        base = mesh.face_ptr[fs]
        P = np.stack([mesh.nodes[mesh.face_nodes[base + k]] for k in range(m)], 1)  # [nf,m,d]
        for side in (0, 1):
            if side == 0:
                cells = mesh.owner[fs]
                Q = P
                fcs = fcen[fs]
            else:
                fs = fs[mesh.neighbour[fs] >= 0]
                P = P[mesh.neighbour[fs0] >= 0]
                cells = mesh.neighbour[fs]
                Q = P[:, ::-1, :] - mesh.shift[fs][:, None, :]
                fcs = fcen[fs] - mesh.shift[fs]
            c = centre[cells]
            if d == 2:
                out_v.append(np.stack([c, Q[:, 0], Q[:, 1]], 1))
                out_c.append(cells)
            else:
                for k in range(m):
                    out_v.append(np.stack([c, fcs, Q[:, k], Q[:, (k + 1) % m]], 1))
                    out_c.append(cells)
    return np.concatenate(out_v), np.concatenate(out_c)


def _gauss01(n):
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w


def simplex_rule(dim, n):
    """Barycentric points [q, dim+1] and weights [q] on the unit-measure simplex."""
    x, w = _gauss01(n)
    if dim == 2:
        X, Y = np.meshgrid(x, x, indexing="ij")
        W = np.outer(w, w) * (1 - X)
        s, t = X, Y * (1 - X)
        lam = np.stack([1 - s - t, s, t], -1).reshape(-1, 3)
        return lam, 2.0 * W.reshape(-1)
    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
    W = w[:, None, None] * w[None, :, None] * w[None, None, :] * (1 - X) ** 2 * (1 - Y)
    s = X
    t = Y * (1 - X)
    r = Z * (1 - X) * (1 - Y)
    lam = np.stack([1 - s - t - r, s, t, r], -1).reshape(-1, 4)
    return lam, 6.0 * W.reshape(-1)


def cell_averages(mesh, fn, n_pts=4, chunk=200_000):
    """Volume averages of ``fn(x) -> [n, n_v]`` over every cell (FP64)."""
    verts, cells = cell_simplices(mesh)
    d = mesh.dim
    lam, w = simplex_rule(d, n_pts)
    acc = None
    vol = np.zeros(mesh.n_cells)
    for s0 in range(0, verts.shape[0], chunk):
        V = verts[s0:s0 + chunk]
        C = cells[s0:s0 + chunk]
        E = V[:, 1:, :] - V[:, :1, :]
        meas = np.abs(np.linalg.det(E)) / (2.0 if d == 2 else 6.0)
        pts = np.einsum("qk,skd->sqd", lam, V)                # [s, q, d]
        vals = fn(pts.reshape(-1, d))
        vals = vals.reshape(pts.shape[0], pts.shape[1], -1)
        integ = np.einsum("sqv,q->sv", vals, w) * meas[:, None]
        if acc is None:
            acc = np.zeros((mesh.n_cells, integ.shape[1]))
        for v in range(integ.shape[1]):
            acc[:, v] += np.bincount(C, weights=integ[:, v], minlength=mesh.n_cells)
        vol += np.bincount(C, weights=meas, minlength=mesh.n_cells)
    return acc / vol[:, None]


def cell_points(mesh):
    """A representative interior point per cell (for point-sampled data)."""
    return _interior_points(mesh)[0]


def parent_hex_points(mesh):
    """Corner average of each cell's parent lattice hex (3-D lattice meshes):
    a cheap sample point for large meshes (exact centre for unsplit hexes
    up to jitter curvature, the parent's centre for split cells)."""
    nx, ny, nz = mesh.info["lattice"]
    h = mesh.info["parent_hex"].astype(np.int64)
    i, j, k = h % nx, (h // nx) % ny, h // (nx * ny)
    NX, NY = nx + 1, ny + 1
    out = np.zeros((h.size, 3))
    for dk in (0, 1):
        for dj in (0, 1):
            for di in (0, 1):
                out += mesh.nodes[(i + di) + NX * ((j + dj) + NY * (k + dk))]
    return out / 8.0


# --------------------------------------------------------------------------
# closed-form fields
# --------------------------------------------------------------------------

def sine2d(a=(1.0, 0.5), t=0.0):
    a = np.asarray(a, dtype=np.float64)

    def f(x):
        y = x - a[None, : x.shape[1]] * t
        return (np.sin(2 * np.pi * y[:, 0]) * np.sin(2 * np.pi * y[:, 1]))[:, None]
    return f


def sine1d(L=1.0, a=1.0, t=0.0):
    def f(x):
        return np.sin(2 * np.pi * (x[:, 0] - a * t) / L)[:, None]
    return f


def burgers_diag(t=0.0, mean=0.5, amp=0.25):
    """Solution of u_t + div(u^2/2 (1,1)) = 0 with u0 = mean + amp sin(2 pi (x+y)).

    Along characteristics x+y moves with speed 2u, so u = u0(xi - 2 u t),
    xi = x + y; solved by Newton (valid before the shock time).
    """
    def f(x):
        xi = x[:, 0] + x[:, 1]
        u = mean + amp * np.sin(2 * np.pi * xi)
        for _ in range(60):
            arg = 2 * np.pi * (xi - 2 * u * t)
            g = u - mean - amp * np.sin(arg)
            dg = 1.0 + amp * np.cos(arg) * 2 * np.pi * 2 * t
            du = g / dg
            u = u - du
            if np.max(np.abs(du)) < 1e-15:
                break
        return u[:, None]
    return f


class Blasius:
    """The laminar flat-plate boundary layer (Blasius): f''' + f f'' / 2 = 0,
    f(0) = f'(0) = 0, f'(inf) = 1, solved by shooting on f''(0) with an
    adaptive Runge-Kutta integrator (rtol 1e-12).  With eta = y / sqrt(nu x / U)
    the velocity is u = U f'(eta), v = sqrt(nu U / x) (eta f' - f) / 2.
    (Input data only: the plate flow is the workload of the single-step
    reconstruction study, not part of the finite-volume method.)"""

    def __init__(self, eta_max=15.0):
        from scipy.integrate import solve_ivp
        from scipy.optimize import brentq

        def rhs(_eta, y):
            return [y[1], y[2], -0.5 * y[0] * y[2]]

        def shoot(s, dense=False):
            return solve_ivp(rhs, (0.0, eta_max), [0.0, 0.0, s], method="DOP853", rtol=1e-12, atol=1e-14,
                             dense_output=dense)

        self.fpp0 = brentq(lambda s: shoot(s).y[1, -1] - 1.0, 0.2, 0.5, xtol=1e-15)
        self._sol = shoot(self.fpp0, dense=True).sol
        self.eta_max = eta_max

    def f_and_fp(self, eta):
        eta = np.asarray(eta, dtype=np.float64)
        e = np.clip(eta, 0.0, self.eta_max)
        y = self._sol(e.ravel())
        f, fp = y[0].reshape(e.shape), y[1].reshape(e.shape)
        # beyond eta_max: f' = 1, f grows linearly
        f = np.where(eta > self.eta_max, f + (eta - self.eta_max), f)
        return f, fp

    def velocity(self, x, y, nu=1.0, U=1.0):
        """(u, v) at plate distance x > 0 and wall distance y >= 0."""
        d = np.sqrt(nu * x / U)
        eta = y / d
        f, fp = self.f_and_fp(eta)
        return U * fp, 0.5 * np.sqrt(nu * U / x) * (eta * fp - f)

    def field(self, x0=1.0):
        """fn(points) -> [n, 2] (u, v), the lattice's x measured from x0."""
        def fn(pts):
            u, v = self.velocity(x0 + pts[:, 0], pts[:, 1])
            return np.stack([u, v], axis=1)
        return fn


def prim_to_cons(rho, vel, p, gamma=GAMMA):
    E = p / (gamma - 1.0) + 0.5 * rho * np.sum(vel * vel, axis=-1)
    return np.concatenate([rho[:, None], rho[:, None] * vel, E[:, None]], 1)


def isentropic_vortex(t=0.0, strength=5.0, centre=(5.0, 5.0), vinf=(1.0, 1.0, 0.0),
                      box=10.0, gamma=GAMMA):
    """Convected isentropic vortex (axis along z), conserved variables."""
    vinf = np.asarray(vinf, dtype=np.float64)

    def f(x):
        cx = centre[0] + vinf[0] * t
        cy = centre[1] + vinf[1] * t
        dx = x[:, 0] - cx
        dy = x[:, 1] - cy
        dx -= box * np.round(dx / box)
        dy -= box * np.round(dy / box)
        r2 = dx * dx + dy * dy
        e = np.exp(0.5 * (1.0 - r2))
        du = strength / (2 * np.pi) * e
        T = 1.0 - (gamma - 1.0) * strength ** 2 / (8 * gamma * np.pi ** 2) * e * e
        rho = T ** (1.0 / (gamma - 1.0))
        p = rho * T
        vel = np.stack([vinf[0] - du * dy, vinf[1] + du * dx,
                        np.full_like(dx, vinf[2])], 1)
        return prim_to_cons(rho, vel, p, gamma)
    return f


def taylor_green(mach=0.1, gamma=GAMMA):
    p0 = 1.0 / (gamma * mach * mach)

    def f(x):
        X, Y, Z = x[:, 0], x[:, 1], x[:, 2]
        vel = np.stack([np.sin(X) * np.cos(Y) * np.cos(Z),
                        -np.cos(X) * np.sin(Y) * np.cos(Z), np.zeros_like(X)], 1)
        p = p0 + (np.cos(2 * X) + np.cos(2 * Y)) * (np.cos(2 * Z) + 2.0) / 16.0
        return prim_to_cons(np.ones_like(X), vel, p, gamma)
    return f


def sod_slab(gamma=GAMMA):
    """High state (1, 0, 1) where |x - 0.5| < 0.25, low (0.125, 0, 0.1) elsewhere."""
    def f(x):
        inside = np.abs(x[:, 0] - 0.5) < 0.25
        rho = np.where(inside, 1.0, 0.125)
        p = np.where(inside, 1.0, 0.1)
        return prim_to_cons(rho, np.zeros((x.shape[0], 3)), p, gamma)
    return f


def blast(gamma=GAMMA, radius=0.2, centre=(0.5, 0.5, 0.5)):
    def f(x):
        r = np.linalg.norm(x - np.asarray(centre)[None, :], axis=1)
        p = np.where(r < radius, 10.0, 0.1)
        return prim_to_cons(np.ones(x.shape[0]), np.zeros((x.shape[0], 3)), p, gamma)
    return f


def max_wave_speed(pde, U, gamma=GAMMA, vel=None):
    """Largest characteristic speed of the state (for a CFL time step)."""
    if pde == "advection":
        return float(np.linalg.norm(vel))
    if pde == "burgers":
        return float(np.max(np.abs(U[:, 0])) * np.sqrt(2.0))
    rho = U[:, 0]
    v = U[:, 1:4] / rho[:, None]
    p = (gamma - 1.0) * (U[:, 4] - 0.5 * rho * np.sum(v * v, 1))
    c = np.sqrt(gamma * p / rho)
    return float(np.max(np.linalg.norm(v, axis=1) + c))


# --------------------------------------------------------------------------
# exact solution of the 1-D Riemann problem for an ideal gas (textbook)
# --------------------------------------------------------------------------

def riemann_exact(left, right, xi, gamma=GAMMA):
    """Exact Riemann solution sampled at similarity coordinates xi = x / t.

    left, right: (rho, u, p).  Returns (rho, u, p) arrays.  Newton iteration
    on the star pressure with the shock / rarefaction pressure functions.
    """
    rL, uL, pL = left
    rR, uR, pR = right
    cL = np.sqrt(gamma * pL / rL)
    cR = np.sqrt(gamma * pR / rR)
    g1 = (gamma - 1.0) / (2.0 * gamma)
    g2 = (gamma + 1.0) / (2.0 * gamma)

    def fk(p, r, pk, ck):
        if p > pk:
            A = 2.0 / ((gamma + 1.0) * r)
            B = (gamma - 1.0) / (gamma + 1.0) * pk
            q = np.sqrt(A / (p + B))
            return (p - pk) * q, q * (1.0 - 0.5 * (p - pk) / (B + p))
        pr = p / pk
        return 2.0 * ck / (gamma - 1.0) * (pr ** g1 - 1.0), pr ** (-g2) / (r * ck)

    p = max(1e-8, 0.5 * (pL + pR))
    for _ in range(100):
        fL, dL = fk(p, rL, pL, cL)
        fR, dR = fk(p, rR, pR, cR)
        dp = (fL + fR + uR - uL) / (dL + dR)
        p = max(1e-10, p - dp)
        if abs(dp) < 1e-15 * p:
            break
    fL, _ = fk(p, rL, pL, cL)
    fR, _ = fk(p, rR, pR, cR)
    us = 0.5 * (uL + uR) + 0.5 * (fR - fL)
    xi = np.asarray(xi, dtype=np.float64)
    rho = np.empty_like(xi)
    u = np.empty_like(xi)
    pp = np.empty_like(xi)
    gm = (gamma - 1.0) / (gamma + 1.0)
    for side, (rk, uk, pk, ck, sgn) in enumerate(((rL, uL, pL, cL, -1.0), (rR, uR, pR, cR, 1.0))):
        sel = (xi < us) if side == 0 else (xi >= us)
        x = xi[sel]
        if p > pk:                                   # shock
            Ssh = uk + sgn * ck * np.sqrt(g2 * p / pk + g1)
            rs = rk * (p / pk + gm) / (gm * p / pk + 1.0)
            outer = (x < Ssh) if sgn < 0 else (x > Ssh)
            rho[sel] = np.where(outer, rk, rs)
            u[sel] = np.where(outer, uk, us)
            pp[sel] = np.where(outer, pk, p)
        else:                                        # rarefaction
            cs = ck * (p / pk) ** g1
            head = uk + sgn * ck
            tail = us + sgn * cs
            rs = rk * (p / pk) ** (1.0 / gamma)
            fan_u = 2.0 / (gamma + 1.0) * (-sgn * ck + (gamma - 1.0) / 2.0 * uk + x)
            fan_c = 2.0 / (gamma + 1.0) * (ck - sgn * (gamma - 1.0) / 2.0 * (uk - x))
            fan_r = rk * (fan_c / ck) ** (2.0 / (gamma - 1.0))
            fan_p = pk * (fan_c / ck) ** (2.0 * gamma / (gamma - 1.0))
            if sgn < 0:
                outer, inner = x <= head, x >= tail
            else:
                outer, inner = x >= head, x <= tail
            rho[sel] = np.where(outer, rk, np.where(inner, rs, fan_r))
            u[sel] = np.where(outer, uk, np.where(inner, us, fan_u))
            pp[sel] = np.where(outer, pk, np.where(inner, p, fan_p))
    return rho, u, pp


def sod_slab_exact(x, t, gamma=GAMMA):
    """(rho, u, p) of the periodic Sod slab (high state on |x - 0.5| < 0.25)
    before the waves of its two Riemann problems meet (t < 0.14)."""
    hi = (1.0, 0.0, 1.0)
    lo = (0.125, 0.0, 0.1)
    x = np.asarray(x, dtype=np.float64)
    right = x >= 0.5
    out = [np.empty_like(x) for _ in range(3)]
    r = riemann_exact(hi, lo, (x[right] - 0.75) / t, gamma)
    # the left problem is the mirror image of the right one
    q = riemann_exact(hi, lo, (0.25 - x[~right]) / t, gamma)
    for k in range(3):
        out[k][right] = r[k]
        out[k][~right] = -q[k] if k == 1 else q[k]
    return tuple(out)


# --------------------------------------------------------------------------
# reference solution of the spherical blast: 1-D radial Euler on a fine grid
# --------------------------------------------------------------------------

def radial_euler(init, r_max, n, t_end, alpha=2, gamma=GAMMA, cfl=0.4):
    """Symmetric Euler flow in r (alpha = 0 planar, 2 spherical) to t_end.

    Finite volumes on n shells of [0, r_max]: MUSCL with minmod slopes of
    (rho, u, p), HLL flux with Davis speeds, SSP-RK3, time step from the CFL
    number.  Shell volumes (r+^(a+1) - r-^(a+1)) / (a+1), face areas r^a; the
    pressure force on the shell's curved sides is p (A+ - A-), so a gas at
    rest and uniform pressure stays at rest exactly.  Mirror condition at
    r = 0, zero-gradient state at r_max.  init(r) -> (rho, u, p) at the
    shell centres.  Returns (centres, rho, u, p)."""
    h = r_max / n
    rf = np.arange(n + 1) * h
    rc = 0.5 * (rf[:-1] + rf[1:])
    A = rf ** alpha
    V = (rf[1:] ** (alpha + 1) - rf[:-1] ** (alpha + 1)) / (alpha + 1)
    dA = A[1:] - A[:-1]
    rho, u, p = (np.asarray(q, dtype=np.float64).copy() for q in init(rc))
    U = np.stack([rho, rho * u, p / (gamma - 1.0) + 0.5 * rho * u * u])

    def prim(U):
        r = U[0]
        v = U[1] / r
        return r, v, (gamma - 1.0) * (U[2] - 0.5 * r * v * v)

    def minmod(a, b):
        return np.where(a * b > 0, np.sign(a) * np.minimum(np.abs(a), np.abs(b)), 0.0)

    def rhs(U):
        r, v, pr = prim(U)
        W = np.stack([r, v, pr])
        # two ghost shells each side: mirror at r = 0, copies at r_max
        Wg = np.concatenate([W[:, 1::-1], W, W[:, -1:], W[:, -1:]], axis=1)
        Wg[1, :2] *= -1.0
        s = minmod(Wg[:, 1:-1] - Wg[:, :-2], Wg[:, 2:] - Wg[:, 1:-1])   # slopes of shells -1 .. n
        WL = Wg[:, 1:-2] + 0.5 * s[:, :-1]                              # faces 0 .. n
        WR = Wg[:, 2:-1] - 0.5 * s[:, 1:]

        def flux(W):
            r, v, pr = W
            E = pr / (gamma - 1.0) + 0.5 * r * v * v
            return np.stack([r * v, r * v * v + pr, (E + pr) * v]), np.stack([r, r * v, E])

        FL, UL = flux(WL)
        FR, UR = flux(WR)
        cL = np.sqrt(gamma * WL[2] / WL[0])
        cR = np.sqrt(gamma * WR[2] / WR[0])
        sL = np.minimum(WL[1] - cL, WR[1] - cR)
        sR = np.maximum(WL[1] + cL, WR[1] + cR)
        Fh = (sR * FL - sL * FR + sL * sR * (UR - UL)) / (sR - sL)
        F = np.where(sL >= 0, FL, np.where(sR <= 0, FR, Fh))
        R = -(A[1:] * F[:, 1:] - A[:-1] * F[:, :-1]) / V
        R[1] += pr * dA / V
        return R, float(np.max(np.abs(v) + np.sqrt(gamma * pr / r)))

    t = 0.0
    while t < t_end:
        R1, smax = rhs(U)
        dt = min(cfl * h / smax, t_end - t)
        U1 = U + dt * R1
        U2 = 0.75 * U + 0.25 * (U1 + dt * rhs(U1)[0])
        U = U / 3.0 + 2.0 / 3.0 * (U2 + dt * rhs(U2)[0])
        t += dt
    r, v, pr = prim(U)
    return rc, r, v, pr


def blast_reference(t, n=8000, r_max=0.5, gamma=GAMMA, radius=0.2):
    """Radial profile of the spherical blast (rho 1 at rest, p 10 inside
    radius, 0.1 outside) at time t, valid in the sphere r < r_max while its
    outgoing shock stays inside (t <= 0.05: the shock is near r = 0.3).
    Returns a function of r -> (rho, u, p) by linear interpolation."""
    def init(r):
        return np.ones_like(r), np.zeros_like(r), np.where(r < radius, 10.0, 0.1)
    rc, rho, u, p = radial_euler(init, r_max, n, t, alpha=2, gamma=gamma)

    def at(r):
        r = np.asarray(r, dtype=np.float64)
        return tuple(np.interp(r, rc, q) for q in (rho, u, p))
    return at
