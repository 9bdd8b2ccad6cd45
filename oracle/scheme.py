"""Oracle: DOLINC differentials, far-cell inversion and k-th order reconstruction.

Test infrastructure only (FP64, plain NumPy); the product path never imports it.

Steps, in the paper's order:
1. Gauss-linear ("central differencing") gradient, Sec. 2.3:
   grad(phi)_P = V_P^-1 sum_f S_f^(P) (omega_f phi_P + (1 - omega_f) phi_N).
   Applying it again to each gradient component gives the second-order tensor.
2. DOLINC differentials of the two face-adjacent cells (Sec. 2.3, definition
   of the DOLINC differential): phi_n^(m) = 2^m (grad^m phi)_n : d^(x m),
   with d the centre-to-centre vector of the face being reconstructed.
3. Far-cell inversion with the two recursions of Sec. 2.3 (eq:diffDLC and the
   two one-sided forms before it), applied step by step:
     right:  phi_{n+2}^(m) = g (phi_n^(m) + g^n phi_{n+1}^(m+1)) + (1-g) phi_{n+1}^(m)
     left:   phi_{n-1}^(m) = g^-1 (phi_{n+1}^(m) - g^n phi_n^(m+1)) + (1-g^-1) phi_n^(m)
4. Reconstruction on the retrieved template with the coefficients of
   eq:coeff (Sec. 2.4), evaluated numerically on cell widths g^j.
   ENO3 and WENO5 (end of Sec. 2.4) retrieve cells -2..2 and choose among
   (ENO: Harten's rule on the printed DOLINC undivided differences) or
   weight (WENO: Jiang-Shu smoothness indicators, linear weights that
   reproduce the 5-cell coefficients) the three 3-cell stencils; the
   quadratics are fitted to the retrieved cell averages directly.
The right state comes from the same steps in the mirrored (N -> P) frame:
cells swap, d -> -d and g -> 1/g.
"""
from __future__ import annotations

import numpy as np

SCHEMES = {"FOU": (1, 0), "CD2": (2, 0), "USR3": (3, 1), "CSR4": (4, 1), "USR4": (4, 2), "USR5": (5, 2),
           "CSR6": (6, 2)}


# ------------------------------------------------------------------ step 1
def gauss_linear(mesh, geo, phi):
    """phi [nc, ...] -> gradient [nc, ..., dim] (natural face-order sums)."""
    P, N = mesh.owner, mesh.neighbour
    w = geo.omega.reshape((-1,) + (1,) * (phi.ndim - 1))
    phif = w * phi[P] + (1.0 - w) * phi[N]
    flat = phif.reshape(mesh.n_faces, -1)
    out = np.zeros((mesh.n_cells, flat.shape[1], mesh.dim))
    for a in range(mesh.dim):
        contrib = flat * geo.S[:, a:a + 1]
        for k in range(flat.shape[1]):
            out[:, k, a] = (np.bincount(P, weights=contrib[:, k], minlength=mesh.n_cells) -
                            np.bincount(N, weights=contrib[:, k], minlength=mesh.n_cells))
    out /= geo.V[:, None, None]
    return out.reshape(phi.shape + (mesh.dim,))


# ------------------------------------------------------------------ step 4 coefficients
def shu_coefficients(widths, r):
    """eq:coeff: reconstruction weights c_rj at the right edge of cell i.

    widths [..., k]: widths of cells i-r .. i-r+k-1.  Returns [..., k].
    """
    widths = np.asarray(widths, dtype=np.float64)
    k = widths.shape[-1]
    xb = np.concatenate([np.zeros(widths.shape[:-1] + (1,)), np.cumsum(widths, -1)], -1)
    xface = xb[..., r + 1]
    c = np.zeros(widths.shape)
    for j in range(k):
        tot = np.zeros(widths.shape[:-1])
        for m in range(j + 1, k + 1):
            num = np.zeros(widths.shape[:-1])
            for l in range(k + 1):
                if l == m:
                    continue
                prod = np.ones(widths.shape[:-1])
                for q in range(k + 1):
                    if q != m and q != l:
                        prod = prod * (xface - xb[..., q])
                num = num + prod
            den = np.ones(widths.shape[:-1])
            for l in range(k + 1):
                if l != m:
                    den = den * (xb[..., m] - xb[..., l])
            tot = tot + num / den
        c[..., j] = tot * widths[..., j]
    return c


def growth_widths(g, k, r):
    """Widths g^j of template cells j = -r .. k-r-1 under a constant growth rate."""
    g = np.asarray(g, dtype=np.float64)
    return np.stack([g ** j for j in range(-r, k - r)], -1)


# ------------------------------------------------------------------ step 2
def differentials(G, d, order):
    """phi^(m) for m = 0..order of one cell: G = [phi, G1, G2] (cell values)."""
    out = [G[0]]
    if order >= 1:
        out.append(2.0 * np.einsum("f...a,fa->f...", G[1], d))
    if order >= 2:
        out.append(4.0 * np.einsum("f...ab,fa,fb->f...", G[2], d, d))
    return out


# ------------------------------------------------------------------ step 3
def invert(table, g, lo, hi):
    """Extend {phi_0^(m), phi_1^(m)} to cells lo..hi with the recursions.

    table: dict (n, m) -> values for n in {0, 1}.  Returns the dict extended
    with every (n, m) the recursions can reach for lo <= n <= hi.
    """
    t = dict(table)
    gb = g.reshape((-1,) + (1,) * (next(iter(t.values())).ndim - 1))
    mmax = max(m for (_n, m) in t)
    n = 1
    while n + 1 <= hi:                    # phi_{n+1} from cells n-1, n
        for m in range(0, mmax + 1):
            if (n - 1, m) in t and (n, m + 1) in t and (n, m) in t:
                t[(n + 1, m)] = gb * (t[(n - 1, m)] + gb ** (n - 1) * t[(n, m + 1)]) + \
                    (1.0 - gb) * t[(n, m)]
        n += 1
    n = 0
    while n - 1 >= lo:                    # phi_{n-1} from cells n, n+1
        for m in range(0, mmax + 1):
            if (n + 1, m) in t and (n, m + 1) in t and (n, m) in t:
                t[(n - 1, m)] = (t[(n + 1, m)] - gb ** n * t[(n, m + 1)]) / gb + \
                    (1.0 - 1.0 / gb) * t[(n, m)]
        n -= 1
    return t


def one_side(G0, G1c, d, g, scheme):
    """Face value at the right edge of cell 0 from cells 0 (upwind) and 1.

    G0, G1c: lists [phi, grad, grad2] of cells 0 and 1 gathered per face.
    """
    k, r = SCHEMES[scheme]
    order = scheme_order(scheme)
    D0 = differentials(G0, d, order)
    D1 = differentials(G1c, d, order)
    table = {}
    for m in range(order + 1):
        table[(0, m)] = D0[m]
        table[(1, m)] = D1[m]
    t = invert(table, g, -r, k - r - 1)
    c = shu_coefficients(growth_widths(g, k, r), r)
    out = np.zeros_like(G0[0])
    cb = c.reshape(c.shape[:1] + (1,) * (G0[0].ndim - 1) + c.shape[1:])
    for j in range(k):
        out = out + cb[..., j] * t[(j - r, 0)]
    return out


def cell_derivs(mesh, geo, U, order):
    G = [U]
    if order >= 1:
        G.append(gauss_linear(mesh, geo, U))
    if order >= 2:
        G.append(gauss_linear(mesh, geo, G[1]))
    return G


def scheme_order(scheme):
    """DOLINC order: the highest differential the far cells need.  Cell -n
    (n >= 1) needs phi^(n) of the upwind cell; cell 1 + n needs phi^(n) of
    the downwind cell.  ENO3 and WENO5 choose among, or weight, the three
    3-cell stencils inside cells -2..2, so they are second-order DOLINC
    schemes (end of Sec. 2.4)."""
    if scheme in NONLINEAR:
        return 2
    k, r = SCHEMES[scheme]
    return max(0, r, k - r - 2)


# ------------------------------------------------------------------ ENO3 / WENO5 (Sec. 2.4)
NONLINEAR = ("ENO3", "WENO5")
WENO_EPS = 1e-6   # the paper gives no value; the classical choice of Jiang and Shu
ENO_TIE = 1e-10   # relative margin below which two ENO candidates count as tied


def substencil_polys(g, r):
    """Quadratic p(x) = a0 + a1 x + a2 x^2 whose averages over the cells
    -r .. 2-r (widths g^j, cell 0 = [0, 1]) are the given cell values.

    Returns M [F, 3, 3] with (a0, a1, a2) = M @ (phi_-r, .., phi_{2-r})."""
    g = np.atleast_1d(np.asarray(g, dtype=np.float64))
    F = g.shape[0]
    widths = np.stack([g ** j for j in range(-r, 3 - r)], -1)        # [F, 3]
    left = np.zeros((F, 4))                                          # cell edges
    left[:, 1:] = np.cumsum(widths, -1)
    left -= left[:, r:r + 1]                                         # cell 0 starts at 0
    A = np.zeros((F, 3, 3))
    for j in range(3):
        a, b = left[:, j], left[:, j + 1]
        for q in range(3):                                           # average of x^q
            A[:, j, q] = (b ** (q + 1) - a ** (q + 1)) / ((q + 1) * (b - a))
    return np.linalg.inv(A)


def substencil_values_and_smoothness(t, g):
    """For r = 0, 1, 2 (stencils {0,1,2}, {-1,0,1}, {-2,-1,0}): the value of
    p_r at the right edge of cell 0 and the Jiang-Shu smoothness indicator
    beta_r = int_0^1 (p_r')^2 dx + int_0^1 (p_r'')^2 dx (cell 0 has unit
    width in the growth-scaled frame).  t: retrieved cells -2..2."""
    q, beta = [], []
    for r in range(3):
        M = substencil_polys(g, r)
        cells = np.stack([t[(j, 0)] for j in range(-r, 3 - r)], 1)     # [F, 3, ...]
        a = np.einsum("fij,fj...->fi...", M, cells)                    # [F, 3, ...]
        q.append(a[:, 0] + a[:, 1] + a[:, 2])
        # p' = a1 + 2 a2 x; int_0^1 p'^2 = a1^2 + 2 a1 a2 + 4/3 a2^2; p'' = 2 a2
        beta.append(a[:, 1] ** 2 + 2.0 * a[:, 1] * a[:, 2] + (4.0 / 3.0) * a[:, 2] ** 2 + 4.0 * a[:, 2] ** 2)
    return q, beta


def weno5_linear_weights(g):
    """d_r with sum_r d_r (3-cell coefficients of stencil r) = the 5-cell
    coefficients of eq:coeff (k = 5, r = 2), solved by least squares over
    the five cells (the system is consistent for every g)."""
    g = np.atleast_1d(np.asarray(g, dtype=np.float64))
    gu, back = np.unique(g, return_inverse=True)                     # weights depend on g only
    c5 = shu_coefficients(growth_widths(gu, 5, 2), 2)                 # cells -2..2
    A = np.zeros((gu.shape[0], 5, 3))
    for r in range(3):
        c3 = shu_coefficients(growth_widths(gu, 3, r), r)             # cells -r..2-r
        A[:, 2 - r:5 - r, r] = c3
    d = np.stack([np.linalg.lstsq(A[f], c5[f], rcond=None)[0] for f in range(gu.shape[0])])
    back = back.reshape(-1)
    return d[back], A[back], c5[back]


def eno3_select(t, g):
    """Harten's stencil choice with the DOLINC-form undivided differences of
    Sec. 2.4: first between {-1,0} and {0,1}, then between the two 3-cell
    extensions of the winner.  The upwind candidate wins only when its
    magnitude is smaller by more than a relative ENO_TIE (ties, which the
    mirror symmetry of a boundary produces exactly, go to the downwind
    candidate whatever the rounding).  Returns r in {0, 1, 2} per face."""
    gb = g.reshape((-1,) + (1,) * (t[(0, 0)].ndim - 1))
    p = {j: t[(j, 0)] for j in range(-2, 3)}
    left2 = gb * (p[0] - p[-1])
    right2 = p[1] - p[0]
    d3_m2 = gb ** 2 * (p[0] - (1.0 + gb) * p[-1] + gb * p[-2])       # {-2,-1,0}
    d3_m1 = p[1] - (1.0 + gb) * p[0] + gb * p[-1]                     # {-1,0,1}
    d3_0 = gb ** -2 * (p[2] - (1.0 + gb) * p[1] + gb * p[0])          # {0,1,2}
    keep = 1.0 - ENO_TIE
    go_left = np.abs(left2) < keep * np.abs(right2)
    r_if_left = np.where(np.abs(d3_m2) < keep * np.abs(d3_m1), 2, 1)
    r_if_right = np.where(np.abs(d3_m1) < keep * np.abs(d3_0), 1, 0)
    return np.where(go_left, r_if_left, r_if_right)


def nonlinear_side(G0, G1c, d, g, scheme):
    """ENO3 / WENO5 face value at the right edge of cell 0 (upwind)."""
    D0 = differentials(G0, d, 2)
    D1 = differentials(G1c, d, 2)
    table = {}
    for m in range(3):
        table[(0, m)] = D0[m]
        table[(1, m)] = D1[m]
    t = invert(table, g, -2, 2)
    q, beta = substencil_values_and_smoothness(t, g)
    if scheme == "ENO3":
        r = eno3_select(t, g)
        return np.where(r == 0, q[0], np.where(r == 1, q[1], q[2]))
    dl, _A, _c5 = weno5_linear_weights(g)
    shape = (-1,) + (1,) * (q[0].ndim - 1)
    alpha = [dl[:, k].reshape(shape) / (WENO_EPS + beta[k]) ** 2 for k in range(3)]
    tot = alpha[0] + alpha[1] + alpha[2]
    return (alpha[0] * q[0] + alpha[1] * q[1] + alpha[2] * q[2]) / tot


def face_states(mesh, geo, U, scheme, G=None):
    """High-order (U_L, U_R) on every face: L from the owner side, R mirrored."""
    order = scheme_order(scheme)
    if G is None:
        G = cell_derivs(mesh, geo, U, order)
    P, N = mesh.owner, mesh.neighbour
    GP = [x[P] for x in G]
    GN = [x[N] for x in G]
    side = nonlinear_side if scheme in NONLINEAR else one_side
    UL = side(GP, GN, geo.d, geo.g, scheme)
    UR = side(GN, GP, -geo.d, 1.0 / geo.g, scheme)
    return UL, UR, G
