"""Pins of the oracle's blend parts against values fixed by hand or by the
mathematics (not by re-running the oracle's own formulas):

* the classical sensor on a uniform line, where the Gauss-linear gradient is
  the central difference and beta reduces to a closed form in the cell values;
* the face weight theta_f = min(theta_P, theta_N) on a two-valued theta;
* the Van Leer limited state on a graded line (g != 1): exact for linear data
  on both sides of every face, and bounded by the two cell values;
* the positivity fallback, face side by face side;
* the indicator's chain-rule channels (grad p, grad |rho u|) against finite
  differences of the closed-form fields, and hand values of the statistics.
"""
from types import SimpleNamespace

import numpy as np
import pytest

from oracle import geometry as OG
from oracle import indicator as OI
from oracle import limiter as OL
from oracle import scheme as OS
from oracle import solver as SV
from synth import configs, fields
from synth import mesh as M

GAMMA = 1.4


def _line(n):
    mesh = configs.line_1d(n, dim=3)
    geo = OG.geometry(mesh)
    i = np.floor(geo.xc[:, 0] * n + 1e-9).astype(int)
    return mesh, geo, i


def _euler(rho, p, n):
    return fields.prim_to_cons(np.asarray(rho, float), np.zeros((n, 3)), np.asarray(p, float))


# ---------------------------------------------------------------- classical sensor
def _beta_line(phi):
    """beta of cell i of a uniform periodic line: the central-difference
    gradient makes the DOLINC differential phi_{i+1} - phi_{i-1}, so on both
    x-faces s - Delta = 2 phi_i - phi_{i-1} - phi_{i+1} and
    |s| + |Delta| = |phi_i - phi_{i-1}| + |phi_{i+1} - phi_i|; the transverse
    faces have s = Delta = 0."""
    a, c = np.roll(phi, 1), np.roll(phi, -1)
    num = np.abs(2 * phi - a - c)
    den = np.abs(phi - a) + np.abs(c - phi)
    return np.where(den > 0, num / np.where(den > 0, den, 1.0), 0.0)


def test_classical_sensor_closed_form_on_uniform_line():
    n = 24
    mesh, geo, i = _line(n)
    rng = np.random.default_rng(3)
    rho_line = 1.0 + 0.3 * rng.random(n)
    p_line = np.full(n, 0.8)
    U = _euler(rho_line[i], p_line[i], mesh.n_cells)
    th, beta = OL.classical_theta(mesh, geo, U, OS.gauss_linear(mesh, geo, U))
    b = _beta_line(rho_line)
    np.testing.assert_allclose(beta, b[i], rtol=1e-6, atol=1e-12)
    np.testing.assert_allclose(th, np.clip((0.9 - b[i]) / 0.3, 0.0, 1.0), rtol=1e-5, atol=1e-6)
    assert (b > 0.9).any() and (b < 0.6).any() and ((b > 0.6) & (b < 0.9)).any()


def test_classical_sensor_hand_values():
    """Quadratic density rho = 1 + 10 (x - x0)^2 (cell averages: centre values
    + 10 h^2 / 12) on a uniform line: a cell at distance t h from x0 has
    2 phi_i - phi_(i-1) - phi_(i+1) = -20 h^2 and first differences
    10 h^2 |2t -+ 1|, so beta = 2 / (|2t - 1| + |2t + 1|): 1 / (2t) for
    |t| >= 1/2, 1 inside.  With x0 = 0.6 h left of the centre of cell 10:
    cell 10 (t = 0.6) beta = 5/6, theta = (0.9 - 5/6) / 0.3 = 2/9; cell 9
    (t = -0.4) beta = 1, theta = 0; cell 7 (t = -2.4) beta = 5/24, theta = 1.
    A density step gives beta = 1 (theta = 0) on the two cells at each jump
    and 0 (theta = 1) elsewhere; a pressure step at constant density is
    sensed through rho E."""
    n = 24
    h = 1.0 / n
    mesh, geo, i = _line(n)
    xc = (np.arange(n) + 0.5) * h
    x0 = xc[10] - 0.6 * h
    rho = 1.0 + 10.0 * (xc - x0) ** 2 + 10.0 * h * h / 12.0
    U = _euler(rho[i], np.full(mesh.n_cells, 1.0), mesh.n_cells)
    th, beta = OL.classical_theta(mesh, geo, U, OS.gauss_linear(mesh, geo, U))
    cell = lambda k: np.nonzero(i == k)[0]  # noqa: E731
    np.testing.assert_allclose(beta[cell(10)], 5.0 / 6.0, rtol=2e-6)
    np.testing.assert_allclose(th[cell(10)], 2.0 / 9.0, rtol=2e-5)
    np.testing.assert_allclose(beta[cell(9)], 1.0, rtol=2e-6)
    np.testing.assert_allclose(th[cell(9)], 0.0)
    np.testing.assert_allclose(beta[cell(7)], 5.0 / 24.0, rtol=2e-6)
    np.testing.assert_allclose(th[cell(7)], 1.0)
    # density jumps between cells 1|2 and 11|12
    rho = np.where((np.arange(n) >= 2) & (np.arange(n) < 12), 1.0, 0.25)
    U = _euler(rho[i], np.full(mesh.n_cells, 1.0), mesh.n_cells)
    th, beta = OL.classical_theta(mesh, geo, U, OS.gauss_linear(mesh, geo, U))
    jump = np.isin(i, (1, 2, 11, 12))
    np.testing.assert_allclose(th[jump], 0.0)
    np.testing.assert_allclose(th[~jump], 1.0)
    # pressure jumps between cells 5|6 and 17|18 at constant density
    p = np.where((np.arange(n) >= 6) & (np.arange(n) < 18), 2.0, 1.0)
    U = _euler(np.full(mesh.n_cells, 1.0), p[i], mesh.n_cells)
    th, _ = OL.classical_theta(mesh, geo, U, OS.gauss_linear(mesh, geo, U))
    jump = np.isin(i, (5, 6, 17, 18))
    np.testing.assert_allclose(th[jump], 0.0)
    np.testing.assert_allclose(th[~jump], 1.0)


def test_classical_sensor_each_cell_takes_its_own_frames():
    """beta of a cell comes from the frames where that cell is cell 0: on a
    line whose values make beta differ from cell to cell, every cell's beta
    is its own closed-form value (not its neighbour's), whichever of its
    faces it owns."""
    n = 16
    mesh, geo, i = _line(n)
    rho = np.array([1.0, 1.1, 1.3, 1.35, 1.5, 1.9, 2.0, 2.05, 2.3, 2.25, 2.0, 1.6, 1.3, 1.2, 1.1, 1.05])
    U = _euler(rho[i], np.full(mesh.n_cells, 1.0), mesh.n_cells)
    _th, beta = OL.classical_theta(mesh, geo, U, OS.gauss_linear(mesh, geo, U))
    b = _beta_line(rho)
    np.testing.assert_allclose(beta, b[i], rtol=1e-6, atol=1e-12)
    assert np.unique(np.round(b, 6)).size >= 8


# ---------------------------------------------------------------- blend weight
def test_face_weight_is_min_of_the_two_cells():
    """theta_f = min(theta_P, theta_N): with theta (0.3, 0.8) every face
    between the two cells takes 0.3 on both sides; (1, 0) gives the limited
    states alone."""
    mesh = SimpleNamespace(owner=np.array([0, 1]), neighbour=np.array([1, 0]))
    UHL, UHR = np.array([[1.0], [2.0]]), np.array([[3.0], [4.0]])
    ULL, ULR = np.array([[10.0], [20.0]]), np.array([[30.0], [40.0]])
    L, R = OL.blend(UHL, UHR, ULL, ULR, np.array([0.3, 0.8]), mesh)
    np.testing.assert_allclose(L[:, 0], [0.3 * 1 + 0.7 * 10, 0.3 * 2 + 0.7 * 20])
    np.testing.assert_allclose(R[:, 0], [0.3 * 3 + 0.7 * 30, 0.3 * 4 + 0.7 * 40])
    L, R = OL.blend(UHL, UHR, ULL, ULR, np.array([1.0, 0.0]), mesh)
    np.testing.assert_allclose(L, ULL)
    np.testing.assert_allclose(R, ULR)


def test_two_valued_theta_limits_the_interface_faces():
    """theta = 1 on the left half of a line and 0 on the right: the residual of
    a cell whose faces all touch theta = 1 cells is the high-order one, a cell
    on the interface sees limited faces."""
    n = 20
    mesh, geo, i = _line(n)
    rho = 1.0 + 0.2 * np.sin(2 * np.pi * (np.arange(n) + 0.5) / n)
    U = _euler(rho[i], np.full(mesh.n_cells, 1.0), mesh.n_cells)
    params = dict(pde="euler", scheme="USR3", flux="rusanov", gamma=GAMMA)
    th = np.where(i < 10, 1.0, 0.0)
    R_blend = SV.residual(mesh, geo, U, params, theta=th)
    R_high = SV.residual(mesh, geo, U, params, theta=np.ones(mesh.n_cells))
    R_low = SV.residual(mesh, geo, U, params, theta=np.zeros(mesh.n_cells))
    deep_left = np.isin(i, (2, 3, 4, 5, 6, 7))
    deep_right = np.isin(i, (12, 13, 14, 15, 16, 17))
    np.testing.assert_allclose(R_blend[deep_left], R_high[deep_left], rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(R_blend[deep_right], R_low[deep_right], rtol=1e-13, atol=1e-15)
    # cell 9's right face is limited on both sides (min rule)
    c9 = i == 9
    assert np.abs(R_blend[c9, 0] - R_high[c9, 0]).max() > 1e-6


# ---------------------------------------------------------------- limited state on a graded line
def _graded_line(n, growth):
    w = growth ** np.arange(n)
    xb = np.concatenate([[0.0], np.cumsum(w)])
    mesh = M.periodic_3d(n, 2, 2, lengths=(xb[-1], 1.0, 1.0), coords=(xb, None, None))
    return mesh, OG.geometry(mesh), xb


@pytest.mark.parametrize("growth", [1.3, 0.7])
def test_vanleer_state_exact_for_linear_data_on_graded_line(growth):
    """On a line of constant growth g != 1 a linear field has r = 1, psi = 1,
    and the limited state phi_0 + (1 - omega_0) Delta is the face value on
    both sides of every x-face away from the periodic seam (omega_0 is the
    upwind cell's weight, g/(1+g) from the owner and 1/(1+g) from the
    neighbour)."""
    n = 14
    mesh, geo, xb = _graded_line(n, growth)
    x = geo.xc[:, 0]
    U = (2.0 + 0.5 * x)[:, None]
    G1 = OS.gauss_linear(mesh, geo, U)
    UL, UR = OL.limited_states(mesh, geo, U, G1)
    xf = geo.xf[:, 0]
    sel = (np.abs(geo.S[:, 0]) > 0) & (xf > xb[2] - 1e-9) & (xf < xb[n - 2] + 1e-9)
    assert sel.sum() >= 4 * (n - 5)
    assert np.abs(geo.omega[sel] - 0.5).min() > 0.05
    np.testing.assert_allclose(UL[sel, 0], 2.0 + 0.5 * xf[sel], rtol=1e-12)
    np.testing.assert_allclose(UR[sel, 0], 2.0 + 0.5 * xf[sel], rtol=1e-12)


def test_vanleer_state_hand_values_on_graded_face():
    """Hand values of the increment: Van Leer's psi Delta = 2 s Delta /
    (s + Delta) (s = 2, Delta = 3: 2.4), weighted by the downwind cell's
    interpolation weight (2/3 on a face twice as far from the upwind centre:
    1.6) and capped at Delta where the weighted value would pass it
    (s = 30: 2/3 * 180/33 = 3.64 > 3); on a uniform face (weight 1/2) the cap
    never acts; opposite signs give the first-order state."""
    s, delta = 2.0, 3.0
    inc = OL.vanleer_increment(np.array([s]), np.array([delta]))[0]
    assert inc == pytest.approx(2 * s * delta / (s + delta))
    # omega_0 = 1/3: (2/3) * 2.4 = 1.6 < 3, kept
    assert OL.limited_increment(np.array([s]), np.array([delta]), 2.0 / 3.0)[0] == pytest.approx(1.6)
    # a steep upwind side, s = 30: psi Delta = 180/33; with w_down = 2/3 it is 3.64 > Delta = 3: capped
    assert OL.limited_increment(np.array([30.0]), np.array([3.0]), 2.0 / 3.0)[0] == 3.0
    assert OL.limited_increment(np.array([-30.0]), np.array([-3.0]), 2.0 / 3.0)[0] == -3.0
    # uniform face (w_down = 1/2): psi < 2 never reaches the cap
    assert OL.limited_increment(np.array([30.0]), np.array([3.0]), 0.5)[0] == pytest.approx(0.5 * 180 / 33)
    # opposite signs: first order
    assert OL.limited_increment(np.array([-1.0]), np.array([3.0]), 0.9)[0] == 0.0


@pytest.mark.parametrize("growth", [0.6, 1.0, 1.6])
def test_vanleer_state_between_the_cell_values(growth):
    """Random data on a graded line and on a jittered mixed mesh: every
    limited face state lies between the two cell values of its face."""
    rng = np.random.default_rng(11)
    mesh, geo, _xb = _graded_line(12, growth)
    meshes = [(mesh, geo)]
    jm = M.periodic_3d(4, jitter=0.25, seed=5, kinds=M.mixed_kinds(4, split_frac=0.5, seed=6))
    meshes.append((jm, OG.geometry(jm)))
    for mesh, geo in meshes:
        U = rng.random((mesh.n_cells, 2)) ** 3
        G1 = OS.gauss_linear(mesh, geo, U)
        UL, UR = OL.limited_states(mesh, geo, U, G1)
        lo = np.minimum(U[mesh.owner], U[mesh.neighbour]) - 1e-15
        hi = np.maximum(U[mesh.owner], U[mesh.neighbour]) + 1e-15
        for X in (UL, UR):
            assert np.all(X >= lo) and np.all(X <= hi)


# ---------------------------------------------------------------- positivity fallback
def test_positivity_fallback_each_side():
    """A face side whose reconstructed rho or p is not positive takes its own
    cell's value (owner for U_L, neighbour for U_R); the other side keeps its
    state."""
    mesh = SimpleNamespace(owner=np.array([0, 1, 0]), neighbour=np.array([1, 2, 2]))
    U = np.stack([fields.prim_to_cons(np.array([r]), np.array([[0.1 * r, 0.0, 0.0]]), np.array([p]))[0]
                  for r, p in ((1.0, 1.0), (0.5, 0.4), (2.0, 3.0))])
    good = fields.prim_to_cons(np.array([0.7, 0.8, 0.9]), np.zeros((3, 3)), np.array([0.6, 0.7, 0.8]))
    neg_rho = good.copy()
    neg_rho[:, 0] = -0.1
    neg_p = good.copy()
    neg_p[:, 4] = 0.01  # kinetic energy 0, p = 0.4 * 0.01 > 0; make it negative below
    neg_p[:, 1] = 2.0   # |m|^2 / (2 rho) > E: p < 0
    # face 0: left bad (rho), right good; face 1: left good, right bad (p); face 2: both bad
    UL = np.stack([neg_rho[0], good[1], neg_p[2]])
    UR = np.stack([good[0], neg_p[1], neg_rho[2]])
    L, R = SV._positivity_fallback(UL, UR, U, mesh, GAMMA)
    np.testing.assert_array_equal(L[0], U[0])
    np.testing.assert_array_equal(R[0], good[0])
    np.testing.assert_array_equal(L[1], good[1])
    np.testing.assert_array_equal(R[1], U[2])
    np.testing.assert_array_equal(L[2], U[0])
    np.testing.assert_array_equal(R[2], U[2])


# ---------------------------------------------------------------- indicator channels and statistics
def _lin_state(x):
    """Linear conserved fields with a non-symmetric momentum gradient."""
    rho = 1.2 + 0.3 * x[:, 0] - 0.2 * x[:, 1] + 0.1 * x[:, 2]
    Mg = np.array([[0.4, -0.3, 0.2], [0.5, 0.1, -0.6], [-0.2, 0.7, 0.3]])
    m = np.array([0.3, -0.2, 0.25])[None, :] + x @ Mg.T
    E = 3.0 + 0.6 * x[:, 0] + 0.4 * x[:, 1] - 0.5 * x[:, 2]
    return np.concatenate([rho[:, None], m, E[:, None]], 1)


def _p_and_mag(U):
    rho, m, E = U[:, 0], U[:, 1:4], U[:, 4]
    return (GAMMA - 1.0) * (E - 0.5 * np.sum(m * m, 1) / rho), np.linalg.norm(m, axis=1)


def test_feature_channels_chain_rule_on_linear_conserved_fields():
    """With linear conserved variables the Gauss-linear gradient is exact on
    a uniform lattice away from the seam, so the chain-rule gradients of p and
    |rho u| at a cell equal the derivatives of the closed-form p(x) and
    |m(x)| at its centre (central finite differences, step 1e-5)."""
    n = 6
    mesh = M.periodic_3d(n)
    geo = OG.geometry(mesh)
    x = geo.xc
    U = _lin_state(x)
    q, gq = OI.channels(U, OS.gauss_linear(mesh, geo, U), GAMMA)
    inner = np.all((x > 1.0 / n) & (x < 1.0 - 1.0 / n), axis=1)
    assert inner.sum() == (n - 2) ** 3
    eps = 1e-5
    for a in range(3):
        e = np.zeros(3)
        e[a] = eps
        pp, mp = _p_and_mag(_lin_state(x + e))
        pm, mm = _p_and_mag(_lin_state(x - e))
        np.testing.assert_allclose(gq[inner, 1, a], ((pp - pm) / (2 * eps))[inner], rtol=1e-7, atol=1e-9)
        np.testing.assert_allclose(gq[inner, 3, a], ((mp - mm) / (2 * eps))[inner], rtol=1e-7, atol=1e-9)
        np.testing.assert_allclose(gq[inner, 0, a], ((_lin_state(x + e) - _lin_state(x - e))[:, 0] /
                                                      (2 * eps))[inner], rtol=1e-8)
    p0, m0 = _p_and_mag(U)
    np.testing.assert_allclose(q[:, 1], p0, rtol=1e-13)
    np.testing.assert_allclose(q[:, 3], m0, rtol=1e-13)
    np.testing.assert_allclose(q[:, 2], U[:, 4], rtol=1e-15)


def test_feature_statistics_hand_values():
    """Linear density on an 8^3 lattice (still fluid, p = 1): on every inner
    cell g0 = 2 h 0.01 = 0.0025 on the x, y, z faces, |Delta| = 0.00125 on all
    six, so f1 = 0.0025 / (rho + 0.00125) and f6 = 0 (s = Delta).  A density
    bump b = 0.5 on one cell of a uniform field: there Delta = -b on all six
    faces and g0 = 0 (central difference), so s = b, beta = 1 on every face:
    f3 = f4 = 1 (a mean, not the sum 6), f5 = s Delta / Delta^2 = -1, and with
    scale = rho + mean |Delta| = 1.5 + 0.5 = 2: f6 = |s - Delta| / scale =
    0.5, f2 = 0.25, f1 = 0."""
    n = 8
    h = 1.0 / n
    mesh = M.periodic_3d(n)
    geo = OG.geometry(mesh)
    x = geo.xc
    rho = 1.0 + 0.01 * (x[:, 0] + x[:, 1] + x[:, 2])
    U = _euler(rho, np.ones(mesh.n_cells), mesh.n_cells)
    F = OI.features(mesh, geo, U, OS.gauss_linear(mesh, geo, U), GAMMA)
    inner = np.all((x > h) & (x < 1 - h), axis=1)
    np.testing.assert_allclose(F[inner, 0], 2 * h * 0.01 / (rho[inner] + 0.01 * h + 1e-8), rtol=1e-9)
    np.testing.assert_allclose(F[inner, 5], 0.0, atol=1e-9)
    np.testing.assert_allclose(F[inner, 3], 0.0, atol=1e-9)
    U = _euler(np.ones(mesh.n_cells), np.ones(mesh.n_cells), mesh.n_cells)
    c0 = int(np.argmin(np.linalg.norm(x - 0.5 - h / 2, axis=1)))
    U[c0, 0] += 0.5
    F = OI.features(mesh, geo, U, OS.gauss_linear(mesh, geo, U), GAMMA)
    np.testing.assert_allclose(F[c0, 0], 0.0, atol=1e-12)           # f1
    np.testing.assert_allclose(F[c0, 1], 0.5 / 2.0, rtol=1e-7)      # f2
    np.testing.assert_allclose(F[c0, 2], 1.0, rtol=1e-7)            # f3 max beta
    np.testing.assert_allclose(F[c0, 3], 1.0, rtol=1e-7)            # f4 mean beta
    np.testing.assert_allclose(F[c0, 4], -1.0, rtol=1e-7)           # f5 = s Delta / Delta^2 = -1
    np.testing.assert_allclose(F[c0, 5], 1.0 / 2.0, rtol=1e-7)      # f6
