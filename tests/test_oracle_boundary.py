"""Pins of the oracle's non-coupled boundaries (auxiliary cells, Sec. 2.6).

The paper's Neumann example, the exactness of the face value and of the
gradient for linear data, free-stream preservation, and the 1-D Sod and Lax
shock tubes of Sec. 3.4 against the exact Riemann solution (with the paper's
observation that WENO5 with the local Lax-Friedrichs flux is sharper than
the Van Leer TVD scheme).
"""
import numpy as np
import pytest

from oracle import boundary as OB
from synth import fields
from synth import mesh as M


def _line(n=8, jitter=0.0, seed=0):
    return M.bounded(M.periodic_3d(n, 2, 2, lengths=(1.0, 0.25, 0.25), jitter=jitter, seed=seed), 0)


def test_auxiliary_geometry():
    """Auxiliary cells mirror their boundary cell in the face plane:
    omega = 1/2 and g = 1 on boundary faces, d along the normal, V_O = V_C;
    the interior geometry is that of the periodic mesh."""
    per = M.periodic_3d(8, 2, 2, lengths=(1.0, 0.25, 0.25), jitter=0.2, seed=3)
    m = M.bounded(per, 0)
    X = OB.extend(m)
    from oracle import geometry as OG
    gp = OG.geometry(per)
    nc = X.n_cells
    assert np.allclose(X.geo.V[:nc], gp.V, rtol=1e-13)
    assert np.allclose(X.geo.xc[:nc], gp.xc, rtol=1e-13)
    bf = X.ghost_face
    assert np.allclose(X.geo.omega[bf], 0.5) and np.allclose(X.geo.g[bf], 1.0)
    rel = X.geo.xc[nc:] - X.geo.xf[bf]
    assert np.allclose(rel, np.einsum("kab,kb->ka", np.eye(3)[None] - 2 * X.normal[:, :, None] * X.normal[:, None, :],
                                      X.geo.xc[X.ghost_cell] - X.geo.xf[bf]))
    dn = X.geo.d[bf] / np.linalg.norm(X.geo.d[bf], axis=1)[:, None]
    assert np.allclose(np.abs(np.einsum("ka,ka->k", dn, X.normal)), 1.0)
    assert np.allclose(X.geo.V[nc:], X.geo.V[X.ghost_cell])
    # outward normals (the jittered boundary faces are not exactly planar)
    assert np.all(X.normal[X.patch == 1, 0] > 0.9) and np.all(X.normal[X.patch == 0, 0] < -0.9)


def test_neumann_worked_example_and_dirichlet():
    """Sec. 2.6: T_f = T_C + q d_fC, T_O = T_C + 2 (T_f - T_C), and the
    normal gradient recovered from T_O and T_C is q; a Dirichlet value is
    returned by the linear interpolation between C and O."""
    m = _line()
    X = OB.extend(m)
    nc = X.n_cells
    rng = np.random.default_rng(1)
    U = np.zeros((X.mesh.n_cells, 1))
    U[:nc, 0] = rng.normal(size=nc)
    q, Tf = 0.7, -1.3
    bcs = {1: (OB.NEUMANN, [q]), 0: (OB.DIRICHLET, [Tf])}
    U = OB.fill_values(X, U, bcs, euler=False)
    for k in range(X.ghost_cell.size):
        C, O = X.ghost_cell[k], nc + k
        if X.patch[k] == 1:
            T_f = U[C, 0] + q * X.dist[k]
            assert abs(U[O, 0] - (U[C, 0] + 2 * (T_f - U[C, 0]))) < 1e-14
            assert abs((U[O, 0] - U[C, 0]) / (2 * X.dist[k]) - q) < 1e-12
        else:
            w = X.geo.omega[X.ghost_face[k]]
            assert abs(w * U[C, 0] + (1 - w) * U[O, 0] - Tf) < 1e-14


def test_linear_field_gradient_exact_with_dirichlet_values():
    """Linear data with Dirichlet values taken from the field itself: the
    auxiliary values are the field at the mirrored centres, so the
    Gauss-linear gradient is exact in every boundary cell too (graded
    spacing, growth 1.3, where the interior gradient is exact)."""
    xs = np.concatenate([[0.0], np.cumsum(1.3 ** np.arange(8))])
    m = M.bounded(M.periodic_3d(8, 2, 2, lengths=(xs[-1], 0.25, 0.25), coords=(xs, None, None)), 0)
    X = OB.extend(m)
    nc = X.n_cells
    # one patch per boundary face, so each face gets the field's own value;
    # the field varies along the open axis only (y and z are periodic)
    Xp = OB.Extended(X.mesh, X.geo, nc, X.ghost_cell, X.ghost_face, np.arange(X.ghost_cell.size),
                     X.normal, X.dist)
    b2 = np.array([0.8, 0.0, 0.0])
    U = np.zeros((X.mesh.n_cells, 1))
    U[:nc, 0] = 2.0 + X.geo.xc[:nc] @ b2
    bcs = {k: (OB.DIRICHLET, [2.0 + X.geo.xf[f] @ b2]) for k, f in enumerate(X.ghost_face)}
    G = OB.cell_derivs(Xp, U, 1, bcs, euler=False)
    assert np.allclose(G[1][:nc, 0], b2[None, :], atol=1e-12)
    assert G[0].shape[0] == X.mesh.n_cells


@pytest.mark.parametrize("scheme", ["USR3", "CSR4", "USR5", "WENO5", "ENO3"])
def test_free_stream_with_boundaries(scheme):
    """A uniform flow through zero-gradient ends (jittered mesh) and along
    planar slip walls stays uniform (residual at rounding level)."""
    per = M.periodic_3d(6, 4, 3, jitter=0.2, seed=7)
    m = M.bounded(per, 0)
    X = OB.extend(m)
    U = fields.prim_to_cons(np.full(m.n_cells, 1.2), np.tile([0.4, 0.1, -0.2], (m.n_cells, 1)),
                            np.full(m.n_cells, 0.9))
    for flux in ("rusanov", "hllc"):
        R = OB.residual(X, U, dict(pde="euler", scheme=scheme, flux=flux), {})
        assert np.abs(R).max() < 1e-12, (scheme, flux, np.abs(R).max())
    # planar slip walls (unjittered mesh) with the flow along them
    m = M.bounded(M.periodic_3d(6, 4, 3), 0)
    X = OB.extend(m)
    U2 = fields.prim_to_cons(np.full(m.n_cells, 1.2), np.tile([0.0, 0.3, -0.2], (m.n_cells, 1)),
                             np.full(m.n_cells, 0.9))
    R = OB.residual(X, U2, dict(pde="euler", scheme=scheme, flux="hllc"), {0: (OB.SLIP_WALL,), 1: (OB.SLIP_WALL,)})
    assert np.abs(R).max() < 1e-11, (scheme, np.abs(R).max())


SOD = ((1.0, 0.0, 1.0), (0.125, 0.0, 0.1), 0.2)
LAX = ((0.445, 0.698, 3.528), (0.5, 0.0, 0.571), 0.16)


def shock_tube(N, prob, scheme, tvd=False, cfl=0.3):
    left_state, right_state, T = prob
    m = M.bounded(M.periodic_3d(N, 2, 2, lengths=(1.0, 0.02, 0.02)), 0)
    X = OB.extend(m)
    x = X.geo.xc[:X.n_cells, 0]
    lft = x < 0.5
    prim = [np.where(lft, a, b) for a, b in zip(left_state, right_state)]
    vel = np.zeros((m.n_cells, 3))
    vel[:, 0] = prim[1]
    U = fields.prim_to_cons(prim[0], vel, prim[2])
    smax = 4.5 if prob is LAX else 2.5
    steps = int(np.ceil(T * N * smax / cfl))
    th = np.zeros(m.n_cells) if tvd else None
    par = dict(pde="euler", scheme=scheme, flux="rusanov")
    for _ in range(steps):
        U = OB.rk_step(X, U, T / steps, par, {}, th)
    ex = fields.riemann_exact(left_state, right_state, (x - 0.5) / T)
    return np.mean(np.abs(U[:, 0] - ex[0])), U


def test_sod_and_lax_tubes_against_exact_solution():
    """Zero-gradient ends, local Lax-Friedrichs flux (Sec. 3.4): WENO5 is
    within a small L1 distance of the exact density and sharper than the
    Van Leer TVD scheme on both problems (the paper's observation)."""
    for prob, tol in ((SOD, 0.009), (LAX, 0.024)):
        e_w, U = shock_tube(100, prob, "WENO5")
        e_t, _ = shock_tube(100, prob, "CD2", tvd=True)
        assert np.isfinite(U).all()
        assert e_w < tol, (prob, e_w)
        assert e_w < e_t, (prob, e_w, e_t)


def test_slip_wall_reflects_like_the_mirrored_riemann_problem():
    """Uniform flow into a slip wall: the wall acts as the mirror state, so
    the solution is the Riemann problem (rho, u, p) | (rho, -u, p) centred on
    the wall (a reflected shock)."""
    N, T = 80, 0.25
    state = (1.0, 0.5, 1.0)
    m = M.bounded(M.periodic_3d(N, 2, 2, lengths=(1.0, 0.02, 0.02)), 0)
    X = OB.extend(m)
    x = X.geo.xc[:X.n_cells, 0]
    vel = np.zeros((m.n_cells, 3))
    vel[:, 0] = state[1]
    U = fields.prim_to_cons(np.full(m.n_cells, state[0]), vel, np.full(m.n_cells, state[2]))
    steps = int(np.ceil(T * N * 3.0 / 0.3))
    par = dict(pde="euler", scheme="WENO5", flux="rusanov")
    bcs = {0: (OB.ZERO_GRADIENT,), 1: (OB.SLIP_WALL,)}
    for _ in range(steps):
        U = OB.rk_step(X, U, T / steps, par, bcs)
    ex = fields.riemann_exact(state, (state[0], -state[1], state[2]), (x - 1.0) / T)
    near = x > 0.5
    # smeared shock and the usual wall-heating dip next to the wall
    assert np.mean(np.abs(U[near, 0] - ex[0][near])) < 0.02
    assert np.mean(np.abs(U[near, 1] - ex[0][near] * ex[1][near])) < 0.02
    # a wall that let the flow through would leave rho = 1 everywhere
    assert U[x > 0.95, 0].min() > 1.4


def test_slip_walls_pass_no_mass_on_skewed_cells():
    """Walls at both open ends of a jittered mesh: the auxiliary field is the
    mirror image of each wall cell's, so with a linear reconstruction (which
    commutes with the reflection) the residual's mass and energy totals
    vanish.  WENO5 reconstructs the Cartesian momentum component by
    component, which commutes with the reflection only for walls normal to a
    coordinate axis: checked on planar walls.  (ENO3 is not checked: at a
    wall its two candidate stencils tie exactly in exact arithmetic, and the
    rounding of omega = 1/2 decides each side's choice independently.)"""
    rng = np.random.default_rng(4)
    cases = (("USR5", "hllc", 0.25), ("USR3", "hllc", 0.25), ("CSR4", "rusanov", 0.25), ("WENO5", "rusanov", 0.0))
    for scheme, flux, jit in cases:
        m = M.bounded(M.periodic_3d(6, 4, 3, jitter=jit, seed=9), 0)
        X = OB.extend(m)
        rho = 1.0 + 0.2 * rng.random(m.n_cells)
        U = fields.prim_to_cons(rho, 0.3 * rng.normal(size=(m.n_cells, 3)), 1.0 + 0.2 * rng.random(m.n_cells))
        R = OB.residual(X, U, dict(pde="euler", scheme=scheme, flux=flux), {0: (OB.SLIP_WALL,), 1: (OB.SLIP_WALL,)})
        tot = (X.geo.V[:X.n_cells, None] * R).sum(0)
        scale = (X.geo.V[:X.n_cells, None] * np.abs(R)).sum(0)
        assert abs(tot[0]) < 1e-13 * scale[0] and abs(tot[4]) < 1e-13 * scale[4], (scheme, tot, scale)
