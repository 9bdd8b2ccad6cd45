"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test ties the oracle to something other than itself: values printed in
the paper, closed forms, identities that hold for any data, textbook special
cases and brute force.  All run on the CPU.
"""
import os

import numpy as np
import pytest

from oracle import flux as OF
from oracle import geometry as OG
from oracle import limiter as OL
from oracle import scheme as OS
from oracle import solver as SV
from synth import configs, fields
from synth import mesh as M

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- coefficients
def test_coefficients_uniform_constants():
    """g = 1 constants printed in Sec. 2.4 (USR3: -1/6, 5/6, 1/3; CSR4:
    -1/12, 7/12, 7/12, -1/12) and the textbook 5th/6th-order ones."""
    one = np.array([1.0])
    exp = {"USR3": [-1 / 6, 5 / 6, 1 / 3], "CSR4": [-1 / 12, 7 / 12, 7 / 12, -1 / 12],
           "USR5": np.array([2, -13, 47, 27, -3]) / 60,
           "CSR6": np.array([1, -8, 37, 37, -8, 1]) / 60, "CD2": [0.5, 0.5]}
    for sch, ref in exp.items():
        k, r = OS.SCHEMES[sch]
        c = OS.shu_coefficients(OS.growth_widths(one, k, r), r)[0]
        np.testing.assert_allclose(c, ref, rtol=0, atol=1e-14)


def test_coefficients_printed_closed_forms():
    """eq:coeff on widths g^j equals the closed forms printed for USR3 and CSR4."""
    g = np.array([0.3, 0.7, 0.999, 1.0, 1.001, 1.5, 2.5, 4.0])
    G = lambda n: sum(g ** i for i in range(n))  # noqa: E731  (sum form of G_n)
    c3 = OS.shu_coefficients(OS.growth_widths(g, 3, 1), 1)
    ref3 = np.stack([-g ** 3 / (G(2) * G(3)), g * (1 + 2 * g + 2 * g * g) / (G(2) * G(3)),
                     1 / G(3)], 1)
    np.testing.assert_allclose(c3, ref3, rtol=1e-12, atol=1e-13)
    c4 = OS.shu_coefficients(OS.growth_widths(g, 4, 1), 1)
    den = G(3) * G(4)
    ref4 = np.stack([-g ** 5 / den, g * g * (1 + 2 * g + 2 * g * g + 2 * g ** 3) / den,
                     (2 + 2 * g + 2 * g * g + g ** 3) / den, -1 / den], 1)
    np.testing.assert_allclose(c4, ref4, rtol=1e-12, atol=1e-13)


@pytest.mark.parametrize("k,r", [(2, 0), (3, 1), (4, 1), (5, 2), (6, 2)])
def test_coefficients_polynomial_exact(k, r):
    """Cell averages of x^p, p < k, reconstruct the point value at the face
    on an arbitrary non-uniform template (brute force over random widths)."""
    rng = np.random.default_rng(k * 10 + r)
    w = rng.uniform(0.3, 2.0, size=(50, k))
    c = OS.shu_coefficients(w, r)
    xb = np.concatenate([np.zeros((50, 1)), np.cumsum(w, 1)], 1)
    xf = xb[:, r + 1]
    for p in range(k):
        avg = (xb[:, 1:] ** (p + 1) - xb[:, :-1] ** (p + 1)) / ((p + 1) * w)
        np.testing.assert_allclose((c * avg).sum(1), xf ** p, rtol=1e-11, atol=1e-11)
    np.testing.assert_allclose(c.sum(1), 1.0, atol=1e-13)


def test_cd2_is_linear_interpolation():
    """k = 2 reduces to linear interpolation with the distance weight omega."""
    g = np.array([0.4, 1.0, 2.2])
    c = OS.shu_coefficients(OS.growth_widths(g, 2, 0), 0)
    omega = g / (1 + g)
    np.testing.assert_allclose(c, np.stack([omega, 1 - omega], 1), atol=1e-14)


# ---------------------------------------------------------------- inversion
def _graded_line(n, g, dim=3):
    return configs.line_1d(n, widths=g ** np.arange(n), dim=dim)


def _columns(mesh, geo, n):
    order = np.argsort(geo.xc[:, 0], kind="stable")
    col = np.empty(mesh.n_cells, dtype=np.int64)
    per = mesh.n_cells // n
    col[order] = np.arange(mesh.n_cells) // per
    return col


def _x_faces(mesh, geo, col, i):
    sel = (np.abs(geo.S[:, 1:]).max(1) < 1e-14) & (col[mesh.owner] == i) & \
          (col[mesh.neighbour] == i + 1)
    return np.nonzero(sel)[0]


@pytest.mark.parametrize("g", [0.5, 0.7, 1.0, 1.5, 3.0])
def test_inversion_recovers_far_cells(g):
    """eq:diffDLC and its one-sided forms recover phi_-2, phi_-1, phi_2, phi_3
    exactly (any data) on a constant-growth line of cells."""
    n = 14
    mesh = _graded_line(n, g)
    geo = OG.geometry(mesh)
    col = _columns(mesh, geo, n)
    rng = np.random.default_rng(int(g * 100))
    ucol = rng.normal(size=n)
    U = ucol[col][:, None]
    G = OS.cell_derivs(mesh, geo, U, 2)
    i = 6
    for f in _x_faces(mesh, geo, col, i):
        P, N = mesh.owner[[f]], mesh.neighbour[[f]]
        D0 = OS.differentials([x[P] for x in G], geo.d[[f]], 2)
        D1 = OS.differentials([x[N] for x in G], geo.d[[f]], 2)
        tab = {(0, m): D0[m] for m in range(3)}
        tab.update({(1, m): D1[m] for m in range(3)})
        t = OS.invert(tab, geo.g[[f]], -2, 3)
        scale = np.abs(ucol).max() * max(g, 1 / g) ** 3
        for j in (-2, -1, 2, 3):
            assert abs(t[(j, 0)][0, 0] - ucol[i + j]) < 1e-13 * scale


@pytest.mark.parametrize("scheme", ["USR3", "CSR4", "USR5", "CSR6"])
@pytest.mark.parametrize("g", [0.8, 1.0, 1.25])
def test_dolinc_equals_classical_reconstruction(scheme, g):
    """On constant growth the DOLINC face value equals the classical
    reconstruction with the real far cells ("entirely equivalent", Sec. 2.4),
    and reproduces polynomials of degree < k exactly."""
    n = 16
    mesh = _graded_line(n, g)
    geo = OG.geometry(mesh)
    col = _columns(mesh, geo, n)
    k, r = OS.SCHEMES[scheme]
    rng = np.random.default_rng(3)
    ucol = rng.normal(size=n)
    U = ucol[col][:, None]
    UL, UR, _ = OS.face_states(mesh, geo, U, scheme)
    i = 7
    w = g ** np.arange(n)
    c = OS.shu_coefficients(w[i - r:i - r + k][None, :], r)[0]
    faces = _x_faces(mesh, geo, col, i)
    assert faces.size == 4
    ref = (c * ucol[i - r:i - r + k]).sum()
    np.testing.assert_allclose(UL[faces, 0], ref, rtol=0, atol=1e-12)
    # mirrored frame: upwind cell i+1, template reversed
    wr = w[::-1]
    jr = n - 1 - (i + 1)
    cr = OS.shu_coefficients(wr[jr - r:jr - r + k][None, :], r)[0]
    refR = (cr * ucol[::-1][jr - r:jr - r + k]).sum()
    np.testing.assert_allclose(UR[faces, 0], refR, rtol=0, atol=1e-12)
    # polynomial data: exact face values
    xb = np.concatenate([[0.0], np.cumsum(w)])
    for p in range(k):
        avg = (xb[1:] ** (p + 1) - xb[:-1] ** (p + 1)) / ((p + 1) * w)
        UL, _UR, _ = OS.face_states(mesh, geo, avg[col][:, None], scheme)
        np.testing.assert_allclose(UL[faces, 0], xb[i + 1] ** p, rtol=1e-10, atol=1e-10)


def test_polynomial_exact_on_graded_tensor_mesh():
    """3-D tensor-product mesh with a constant growth rate per axis: every
    y-face away from the periodic seam reproduces a cubic in y (CSR4)."""
    n = 12
    wy = 1.2 ** np.arange(n)
    yb = np.concatenate([[0.0], np.cumsum(wy)])
    mesh = M.periodic_3d(3, n, 3, lengths=(1.0, yb[-1], 1.0),
                         coords=(None, yb, None))
    geo = OG.geometry(mesh)
    j = np.searchsorted(yb, geo.xc[:, 1]) - 1
    avg = (yb[1:] ** 4 - yb[:-1] ** 4) / (4 * wy) - 2 * (yb[1:] ** 2 - yb[:-1] ** 2) / (2 * wy)
    U = avg[j][:, None]
    UL, UR, _ = OS.face_states(mesh, geo, U, "CSR4")
    yf = geo.xf[:, 1]
    sel = (np.abs(geo.S[:, [0, 2]]).max(1) < 1e-14) & (yf > yb[3] - 1e-9) & (yf < yb[n - 3] + 1e-9)
    assert sel.sum() > 0
    exact = yf[sel] ** 3 - 2 * yf[sel]
    np.testing.assert_allclose(UL[sel, 0], exact, rtol=1e-10, atol=1e-9)
    np.testing.assert_allclose(UR[sel, 0], exact, rtol=1e-10, atol=1e-9)


# ---------------------------------------------------------------- gradient
def test_gradient_closure_and_uniform_central_difference():
    mesh = M.periodic_3d(4, jitter=0.25, seed=5, kinds=M.mixed_kinds(4, split_frac=0.5, seed=6))
    geo = OG.geometry(mesh)
    G = OS.gauss_linear(mesh, geo, np.full((mesh.n_cells, 2), 3.7))
    assert np.abs(G).max() < 1e-12
    mesh = M.periodic_3d(5, 4, 3, lengths=(1.0, 2.0, 0.5))
    geo = OG.geometry(mesh)
    U = np.sin(2 * np.pi * geo.xc[:, :1])
    G = OS.gauss_linear(mesh, geo, U)
    h = 1.0 / 5
    cd = (np.sin(2 * np.pi * (geo.xc[:, 0] + h)) - np.sin(2 * np.pi * (geo.xc[:, 0] - h))) / (2 * h)
    np.testing.assert_allclose(G[:, 0, 0], cd, atol=1e-12)
    assert np.abs(G[:, 0, 1:]).max() < 1e-12


def test_geometry_closed_and_exact_volumes():
    for mesh in (M.periodic_2d(6, 5, jitter=0.25, seed=2, split=0.5, diagonal="seeded",
                               pentagon_frac=0.1),
                 M.periodic_3d(4, jitter=0.2, seed=3, kinds=M.mixed_kinds(4, split_frac=0.6, seed=4))):
        geo = OG.geometry(mesh)
        nc = mesh.n_cells
        for a in range(mesh.dim):
            clo = np.bincount(mesh.owner, weights=geo.S[:, a], minlength=nc) - \
                np.bincount(mesh.neighbour, weights=geo.S[:, a], minlength=nc)
            assert np.abs(clo).max() < 1e-14
        assert abs(geo.V.sum() - np.prod(mesh.lengths)) < 1e-13
        assert geo.V.min() > 0
    # a single tetrahedron's centroid is the vertex mean: check on Kuhn tets
    mesh = M.periodic_3d(3, kinds=M.KUHN6)
    geo = OG.geometry(mesh)
    np.testing.assert_allclose(geo.V, 1.0 / (27 * 6), rtol=1e-13)


# ---------------------------------------------------------------- time / conservation
def test_ssp_rk3_amplification():
    """y' = lam y: one step multiplies by 1 + z + z^2/2 + z^3/6 (z = lam dt)."""
    for z in (-0.3, 0.5j, -1.0 + 0.7j):
        y = SV.ssp_rk3(np.array([1.0 + 0j]), 1.0, lambda u: z * u)
        assert abs(y[0] - (1 + z + z * z / 2 + z ** 3 / 6)) < 1e-15


def test_table1_sine_advection():
    """1-D sine advection over one period reproduces the paper's Table 1
    errors and orders (CD2, USR3, CSR4).  Time is integrated exactly: the
    residual of a uniform periodic line is circulant, so each Fourier mode
    evolves with exp(lambda t)."""
    tab = np.loadtxt(os.path.join(GOLDEN, "table1_sine_advection.txt"))
    for col, sch in ((1, "CD2"), (2, "USR3"), (3, "CSR4")):
        errs = []
        for N in tab[:5, 0].astype(int):
            mesh = configs.line_1d(N, dim=2)
            geo = OG.geometry(mesh)
            c = np.floor(geo.xc[:, 0] * N + 1e-9).astype(int)
            p = dict(pde="advection", flux="upwind", adv_vel=(1.0, 0.0, 0.0), scheme=sch)
            R = SV.residual(mesh, geo, (c == 0).astype(float)[:, None], p)[:, 0]
            a = np.bincount(c, weights=R, minlength=N) / np.bincount(c, minlength=N)
            lam = np.fft.fft(a)
            U0 = fields.cell_averages(mesh, fields.sine1d(), n_pts=8)[:, 0]
            u0 = np.bincount(c, weights=U0, minlength=N) / np.bincount(c, minlength=N)
            uT = np.real(np.fft.ifft(np.exp(lam) * np.fft.fft(u0)))
            errs.append(np.sqrt(np.mean((uT - u0) ** 2)))
        errs = np.array(errs)
        ratio = errs / tab[:5, col]
        assert abs(ratio[0] - 1) < 0.10, (sch, ratio)
        assert np.all(np.abs(ratio[2:] - 1) < 0.02), (sch, ratio)
        orders = np.log2(errs[:-1] / errs[1:])
        printed = np.log2(tab[:4, col] / tab[1:5, col])
        assert np.all(np.abs(orders[1:] - printed[1:]) < 0.05), (sch, orders, printed)


@pytest.mark.parametrize("pde", ["advection", "burgers", "euler"])
def test_conservation_and_free_stream(pde):
    mesh = M.periodic_3d(3, jitter=0.2, seed=9, kinds=M.mixed_kinds(3, split_frac=0.5, seed=2)) \
        if pde == "euler" else M.periodic_2d(6, 6, jitter=0.25, seed=1, split=0.5,
                                             diagonal="seeded", pentagon_frac=0.1)
    geo = OG.geometry(mesh)
    rng = np.random.default_rng(0)
    if pde == "euler":
        p = dict(pde="euler", scheme="USR5", flux="hllc", gamma=1.4)
        U = fields.prim_to_cons(1 + 0.1 * rng.random(mesh.n_cells),
                                0.3 * rng.normal(size=(mesh.n_cells, 3)),
                                1 + 0.1 * rng.random(mesh.n_cells))
        Uinf = np.tile(fields.prim_to_cons(np.array([1.2]), np.array([[0.3, -0.2, 0.5]]),
                                           np.array([2.0])), (mesh.n_cells, 1))
    else:
        p = dict(pde=pde, scheme="USR3", flux="upwind", adv_vel=(1.0, 0.5, 0.0))
        U = 0.5 + 0.2 * rng.random((mesh.n_cells, 1))
        Uinf = np.full((mesh.n_cells, 1), 0.7)
    Un = SV.rk_step(mesh, geo, U, 1e-3, p)
    tot0 = SV.conserved_totals(geo, U)
    tot1 = SV.conserved_totals(geo, Un)
    scale = (geo.V[:, None] * np.abs(U)).sum(0)
    assert np.all(np.abs(tot1 - tot0) <= 20 * np.finfo(float).eps * scale)
    R = SV.residual(mesh, geo, Uinf, p)
    assert np.abs(R).max() < 1e-13 * np.abs(Uinf).max() / geo.V.min() ** (1 / mesh.dim)


def test_csr4_orientation_invariance():
    """CSR4's template is symmetric: U_L from the owner side equals U_R from
    the neighbour side on any mesh and any data."""
    mesh = M.periodic_3d(3, jitter=0.2, seed=4, kinds=M.KUHN6)
    geo = OG.geometry(mesh)
    U = np.random.default_rng(1).normal(size=(mesh.n_cells, 2))
    UL, UR, _ = OS.face_states(mesh, geo, U, "CSR4")
    np.testing.assert_allclose(UL, UR, rtol=1e-12, atol=1e-12)


# ---------------------------------------------------------------- fluxes
def test_fluxes_consistency_and_textbook_cases():
    rng = np.random.default_rng(0)
    S = rng.normal(size=(20, 3))
    U = fields.prim_to_cons(1 + rng.random(20), rng.normal(size=(20, 3)), 1 + rng.random(20))
    phys = OF.euler_flux_n(U, S, 1.4)
    np.testing.assert_allclose(OF.rusanov(U, U, S, 1.4), phys, rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(OF.hllc(U, U, S, 1.4), phys, rtol=1e-12, atol=1e-12)
    # stationary contact: HLLC is exact (pressure flux only)
    UL = fields.prim_to_cons(np.array([1.0]), np.zeros((1, 3)), np.array([1.0]))
    UR = fields.prim_to_cons(np.array([0.2]), np.zeros((1, 3)), np.array([1.0]))
    Sx = np.array([[2.0, 0.0, 0.0]])
    np.testing.assert_allclose(OF.hllc(UL, UR, Sx, 1.4), [[0, 2.0, 0, 0, 0]], atol=1e-14)
    # supersonic: both fluxes upwind
    UL = fields.prim_to_cons(np.array([1.0]), np.array([[5.0, 0.3, 0.0]]), np.array([1.0]))
    UR = fields.prim_to_cons(np.array([0.5]), np.array([[4.0, 0.0, 0.1]]), np.array([0.7]))
    np.testing.assert_allclose(OF.hllc(UL, UR, Sx, 1.4), OF.euler_flux_n(UL, Sx, 1.4), rtol=1e-13)
    # Godunov Burgers: shock, rarefaction through 0, upwind cases (s = 1)
    b = (1.0, 1.0, 0.0)
    S1 = np.array([[1.0, 0.0]])
    cases = [(1.0, 0.5, 0.5), (-1.0, 2.0, 0.0), (0.3, 0.9, 0.045), (-0.9, -0.3, 0.045),
             (0.5, -0.5, 0.125), (0.2, -0.8, 0.32)]
    for uL, uR, ref in cases:
        F = OF.godunov_burgers(np.array([[uL]]), np.array([[uR]]), S1, b)
        assert abs(F[0, 0] - ref) < 1e-15, (uL, uR)
    # upwind advection
    F = OF.upwind(np.array([[2.0]]), np.array([[3.0]]), np.array([[1.0, -4.0]]), (1.0, 0.5, 0.0))
    assert F[0, 0] == -3.0


def test_vanleer_limiter_properties():
    r = np.linspace(0.01, 20, 200)
    psi = OL.vanleer_psi(r)
    np.testing.assert_allclose(OL.vanleer_psi(1 / r), psi / r, rtol=1e-14)
    assert psi.min() >= 0 and psi.max() <= 2
    assert np.all(OL.vanleer_psi(-r) == 0)
    delta = np.linspace(-2, 2, 41)
    s = 0.7 * delta
    np.testing.assert_allclose(OL.vanleer_increment(s, delta),
                               np.where(delta != 0, OL.vanleer_psi(s / np.where(delta == 0, 1, delta)) * delta, 0))


def _sod_l1(flux, N, scheme="FOU"):
    mesh = configs.line_1d(N, dim=3)
    geo = OG.geometry(mesh)
    U = fields.sod_slab()(geo.xc)
    p = dict(pde="euler", scheme=scheme, flux=flux, gamma=1.4)
    n = int(np.ceil(0.1 / (0.4 / N / fields.max_wave_speed("euler", U))))
    for _ in range(n):
        U = SV.rk_step(mesh, geo, U, 0.1 / n, p)
    return np.mean(np.abs(U[:, 0] - fields.sod_slab_exact(geo.xc[:, 0], 0.1)[0]))


def test_sod_converges_to_exact_riemann_solution():
    """First-order Rusanov and HLLC converge to the exact Sod solution
    (textbook Riemann solver); HLLC is the less dissipative of the two."""
    r1, r2 = _sod_l1("rusanov", 100), _sod_l1("rusanov", 200)
    h1, h2 = _sod_l1("hllc", 100), _sod_l1("hllc", 200)
    assert r2 < 0.03 and h2 < 0.025
    assert r2 < 0.85 * r1 and h2 < 0.8 * h1
    assert h2 < r2


def test_hllc_star_flux_is_physical_flux_of_star_state():
    """In the subsonic star region the HLLC flux must equal the Euler flux of a
    state moving with the contact speed S* under the common star pressure
    p* = p_L + rho_L (S_L - q_L)(S* - q_L), its energy fixed by the
    Rankine-Hugoniot condition of the energy equation across S_L."""
    rng = np.random.default_rng(7)
    n = np.array([[0.6, -0.8, 0.0]])
    for _ in range(20):
        UL = fields.prim_to_cons(np.array([1 + rng.random()]), 0.2 * rng.normal(size=(1, 3)),
                                 np.array([1 + rng.random()]))
        UR = fields.prim_to_cons(np.array([0.5 + rng.random()]), 0.2 * rng.normal(size=(1, 3)),
                                 np.array([0.5 + rng.random()]))
        rL, vL, EL, pL = OF.euler_primitives(UL, 1.4)
        rR, vR, _ER, pR = OF.euler_primitives(UR, 1.4)
        cL, cR = np.sqrt(1.4 * pL / rL), np.sqrt(1.4 * pR / rR)
        qL, qR = (vL * n).sum(1), (vR * n).sum(1)
        SL = min(qL - cL, qR - cR)
        SR = max(qL + cL, qR + cR)
        Ss = (pR - pL + rL * qL * (SL - qL) - rR * qR * (SR - qR)) / (rL * (SL - qL) - rR * (SR - qR))
        if not (SL < 0 <= Ss):
            continue
        ps = pL + rL * (SL - qL) * (Ss - qL)
        rs = rL * (SL - qL) / (SL - Ss)
        vs = vL + (Ss - qL) * n
        F = OF.hllc(UL, UR, n, 1.4)[0]
        Es = ((SL - qL) * EL - pL * qL + ps * Ss) / (SL - Ss)
        np.testing.assert_allclose(F[0], rs * Ss, rtol=1e-12, atol=1e-13)
        np.testing.assert_allclose(F[1:4], rs * vs[0] * Ss + ps * n[0], rtol=1e-12, atol=1e-13)
        np.testing.assert_allclose(F[4], (Es + ps) * Ss, rtol=1e-12, atol=1e-13)


# ---------------------------------------------------------------- ENO3 / WENO5
def test_weno5_linear_weights_uniform_and_consistent():
    """Uniform mesh: the textbook weights (3/10, 6/10, 1/10) for the stencils
    {0,1,2}, {-1,0,1}, {-2,-1,0}; on graded meshes the weighted 3-cell
    coefficients reproduce the 5-cell ones of eq:coeff exactly, the weights
    stay positive and sum to one."""
    d, A, c5 = OS.weno5_linear_weights(np.array([1.0]))
    assert np.allclose(d[0], [0.3, 0.6, 0.1], atol=1e-13)
    g = np.array([0.5, 0.8, 1.25, 1.7, 2.0])
    d, A, c5 = OS.weno5_linear_weights(g)
    assert np.abs(np.einsum("fij,fj->fi", A, d) - c5).max() < 1e-12
    assert np.all(d > 0) and np.allclose(d.sum(1), 1.0, atol=1e-13)
    # closed form of the outer weights (middle one by the sum)
    den = (g ** 2 + 1) * (g ** 4 + g ** 3 + g ** 2 + g + 1)
    assert np.allclose(d[:, 0], (g ** 2 + g + 1) / den, rtol=1e-12)
    assert np.allclose(d[:, 2], g ** 6 / den, rtol=1e-12)


def test_smoothness_indicators_uniform_jiang_shu():
    """g = 1: beta_r equal the Jiang-Shu closed forms
    13/12 (second difference)^2 + 1/4 (one-sided first difference)^2."""
    rng = np.random.default_rng(3)
    v = rng.normal(size=(7, 5))                    # cells -2..2 per row
    t = {(j, 0): v[:, j + 2] for j in range(-2, 3)}
    q, beta = OS.substencil_values_and_smoothness(t, np.ones(7))
    a, b, c, d, e = (v[:, k] for k in range(5))    # phi_-2 .. phi_2
    js = [13 / 12 * (c - 2 * d + e) ** 2 + 1 / 4 * (3 * c - 4 * d + e) ** 2,
          13 / 12 * (b - 2 * c + d) ** 2 + 1 / 4 * (b - d) ** 2,
          13 / 12 * (a - 2 * b + c) ** 2 + 1 / 4 * (a - 4 * b + 3 * c) ** 2]
    for r in range(3):
        assert np.allclose(beta[r], js[r], rtol=1e-12, atol=1e-13)
    # and the textbook face values of the three stencils
    qs = [(2 * c + 5 * d - e) / 6, (-b + 5 * c + 2 * d) / 6, (2 * a - 7 * b + 11 * c) / 6]
    for r in range(3):
        assert np.allclose(q[r], qs[r], rtol=1e-12, atol=1e-13)


@pytest.mark.parametrize("g", [0.6, 1.0, 1.45])
def test_eno_weno_exact_for_quadratics(g):
    """Cell averages of a quadratic on a constant-growth template: every
    3-cell stencil reproduces the face value, so ENO3 and WENO5 do for any
    stencil choice and any nonlinear weights; all beta_r coincide and WENO5
    falls back to the linear weights."""
    gg = np.array([g])
    edges = np.concatenate([[0.0], np.cumsum([g ** j for j in range(-2, 3)])])
    edges -= edges[2]                             # cell 0 = [0, 1]
    poly = np.polynomial.Polynomial([0.3, -1.2, 0.7])
    prim = poly.integ()
    avg = [(prim(edges[j + 1]) - prim(edges[j])) / (edges[j + 1] - edges[j]) for j in range(5)]
    t = {(j, 0): np.array([avg[j + 2]]) for j in range(-2, 3)}
    q, beta = OS.substencil_values_and_smoothness(t, gg)
    for r in range(3):
        assert abs(q[r][0] - poly(1.0)) < 1e-12
    assert np.ptp([b[0] for b in beta]) < 1e-11
    r = OS.eno3_select(t, gg)
    assert r.shape == (1,)


def test_eno3_avoids_a_jump():
    """A step between cells 0 and 1: ENO3 takes the upwind stencil
    {-2,-1,0}; a step between cells -1 and 0: the downwind {0,1,2}."""
    for step_at, want in ((1, 2), (0, 0)):
        t = {(j, 0): np.array([1.0 if j >= step_at else 0.0]) for j in range(-2, 3)}
        assert int(OS.eno3_select(t, np.array([1.0]))[0]) == want


def _sine_advection_error(N, scheme, cfl, theta=False):
    mesh = configs.line_1d(N, dim=2)
    geo = OG.geometry(mesh)
    c = np.floor(geo.xc[:, 0] * N + 1e-9).astype(int)
    U0 = fields.cell_averages(mesh, fields.sine1d(), n_pts=8)
    p = dict(pde="advection", flux="upwind", adv_vel=(1.0, 0.0, 0.0), scheme=scheme)
    nsteps = int(np.ceil(N / cfl))
    th = np.zeros(mesh.n_cells) if theta else None
    U = U0.copy()
    for _ in range(nsteps):
        U = SV.rk_step(mesh, geo, U, 1.0 / nsteps, p, theta=th)
    cnt = np.bincount(c, minlength=N)
    u = np.bincount(c, weights=U[:, 0], minlength=N) / cnt
    u0 = np.bincount(c, weights=U0[:, 0], minlength=N) / cnt
    return np.sqrt(np.mean((u - u0) ** 2))


def test_table2_sine_advection_nonoscillatory():
    """1-D sine advection over one period, SSP-RK3 at a small CFL number,
    against the paper's Table 2: ENO3, WENO5 and the Van Leer TVD scheme
    (theta = 0 everywhere) within a few per cent, and their orders."""
    tab = np.loadtxt(os.path.join(GOLDEN, "table2_sine_advection.txt"))
    cases = (("ENO3", 3, 0.1, False, (0.04, 0.03)), ("WENO5", 4, 0.05, False, (0.03, 0.02)),
             ("CD2", 1, 0.1, True, (0.06, 0.02)))
    for sch, col, cfl, th, (tol0, tol) in cases:
        Ns = tab[:3, 0].astype(int)
        errs = np.array([_sine_advection_error(N, sch, cfl, th) for N in Ns])
        ratio = errs / tab[:3, col]
        assert abs(ratio[0] - 1) < tol0, (sch, ratio)
        assert np.all(np.abs(ratio[1:] - 1) < tol), (sch, ratio)
        orders = np.log2(errs[:-1] / errs[1:])
        printed = np.log2(tab[:2, col] / tab[1:3, col])
        assert np.all(np.abs(orders - printed) < 0.1), (sch, orders, printed)


def test_csr6_design_order_on_sine_advection():
    """CSR6 (k = 6, the central second-order DOLINC scheme of Sec. 2.4) on
    the 1-D sine advection with exact time integration (as for Table 1):
    sixth-order error decay, and at every N below CSR4's error."""
    errs = {}
    for sch in ("CSR4", "CSR6"):
        errs[sch] = []
        for N in (20, 40, 80):
            mesh = configs.line_1d(N, dim=2)
            geo = OG.geometry(mesh)
            c = np.floor(geo.xc[:, 0] * N + 1e-9).astype(int)
            p = dict(pde="advection", flux="upwind", adv_vel=(1.0, 0.0, 0.0), scheme=sch)
            R = SV.residual(mesh, geo, (c == 0).astype(float)[:, None], p)[:, 0]
            a = np.bincount(c, weights=R, minlength=N) / np.bincount(c, minlength=N)
            lam = np.fft.fft(a)
            U0 = fields.cell_averages(mesh, fields.sine1d(), n_pts=8)[:, 0]
            u0 = np.bincount(c, weights=U0, minlength=N) / np.bincount(c, minlength=N)
            uT = np.real(np.fft.ifft(np.exp(lam) * np.fft.fft(u0)))
            errs[sch].append(np.sqrt(np.mean((uT - u0) ** 2)))
    e6 = np.array(errs["CSR6"])
    orders = np.log2(e6[:-1] / e6[1:])
    assert np.all(np.abs(orders - 6.0) < 0.15), orders
    assert np.all(e6 < np.array(errs["CSR4"]))
