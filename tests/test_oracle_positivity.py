"""Pins of the oracle's positivity scaling of the face-side states (shock
workloads; Zhang-Shu style, not in the paper): hand values of theta for
density-, energy- and momentum-driven cases, the convex decomposition it
rests on, and its guarantee: one forward Euler step within the stated time
step keeps every cell admissible on states where the plain scheme does
not."""
import numpy as np

from oracle import flux as OF
from oracle import geometry as OG
from oracle import positivity as OP
from oracle import scheme as OS
from oracle import solver as SV
from synth import fields
from synth import mesh as M

G = 1.4
D = OP.DELTA


def _theta(Uc, dbar):
    return OP.theta_cell(np.array([Uc], float), np.array([dbar], float), G)[0]


def test_theta_hand_values():
    rest = [1.0, 0.0, 0.0, 0.0, 2.5]                     # rho 1, p 1
    # small increments: U*(1) admissible, theta = 1
    assert _theta(rest, [0.5, 0.1, 0.0, 0.0, 0.3]) == 1.0
    # density: U*(1) has rho = -0.5; rho* = delta rho_c at theta = (1 - delta) / 1.5
    # (the pressure's root, 1 / 1.5, is larger)
    np.testing.assert_allclose(_theta(rest, [1.5, 0, 0, 0, 0]), (1 - D) / 1.5, rtol=1e-14)
    # energy: f(theta) = 2.5 - k - 3 theta, k = delta p_c / (gamma - 1)
    k = D * 1.0 / 0.4
    np.testing.assert_allclose(_theta(rest, [0, 0, 0, 0, 3.0]), (2.5 - k) / 3.0, rtol=1e-14)
    # momentum: m* = (3 theta, 0, 0), f(theta) = 2.5 - k - 4.5 theta^2
    np.testing.assert_allclose(_theta(rest, [0, -3.0, 0, 0, 0]), np.sqrt((2.5 - k) / 4.5), rtol=1e-13)
    # momentum of 2: U*(1) keeps p = 0.4 (2.5 - 2) = 0.2: theta = 1
    assert _theta(rest, [0, -2.0, 0, 0, 0]) == 1.0


def _violent(n, rng):
    rho = np.exp(rng.normal(scale=1.6, size=n))
    p = np.exp(rng.normal(scale=1.6, size=n))
    return fields.prim_to_cons(rho, 0.8 * rng.normal(size=(n, 3)), p)


def test_decomposition_and_admissible_parts():
    """U_c = U*/2 + sum_f a_f U^theta_{c,f} / 2 exactly, with U* and every
    scaled face-side state admissible."""
    mesh = M.periodic_3d(4, jitter=0.25, seed=5, kinds=M.mixed_kinds(4, split_frac=0.5, seed=6))
    geo = OG.geometry(mesh)
    U = _violent(mesh.n_cells, np.random.default_rng(3))
    UL, UR, _ = OS.face_states(mesh, geo, U, "USR5")
    UL, UR = SV._positivity_fallback(UL, UR, U, mesh, G)
    SL, SR, th = OP.scale_face_states(mesh, geo, U, UL, UR, G)
    assert (th < 1).sum() > 10 and th.min() >= 0
    nc = mesh.n_cells
    P, N = mesh.owner, mesh.neighbour
    area = np.linalg.norm(geo.S, axis=1)
    tot = np.bincount(P, area, nc) + np.bincount(N, area, nc)
    mean_face = np.stack([(np.bincount(P, area * SL[:, v], nc) + np.bincount(N, area * SR[:, v], nc)) / tot
                          for v in range(5)], 1)
    Ustar = 2.0 * U - mean_face            # from U_c = U*/2 + mean/2
    r, _v, _E, p = OF.euler_primitives(Ustar, G)
    rc, _v, _E, pc = OF.euler_primitives(U, G)
    assert np.all(r >= (D - 1e-9) * rc) and np.all(p >= (D - 1e-9) * pc)
    for X in (SL, SR):
        r, _v, _E, p = OF.euler_primitives(X, G)
        assert np.all(r > 0) and np.all(p > 0)


def test_forward_euler_step_stays_admissible():
    """Rusanov flux, one forward Euler step at dt lambda sum |S| / V = 1/2
    from states spread over three decades: with the scaling every cell stays
    admissible; without it some cells lose positivity (so the test has
    teeth)."""
    mesh = M.periodic_3d(5, jitter=0.25, seed=8, kinds=M.mixed_kinds(5, split_frac=0.5, seed=9))
    geo = OG.geometry(mesh)
    nc = mesh.n_cells
    area = np.linalg.norm(geo.S, axis=1)
    ssum = np.bincount(mesh.owner, area, nc) + np.bincount(mesh.neighbour, area, nc)
    lost = 0
    for seed in range(6):
        U = _violent(nc, np.random.default_rng(20 + seed))
        base = dict(pde="euler", scheme="USR3", flux="rusanov", gamma=G)
        # the largest wave speed any face state or cell can carry
        UL, UR, _ = OS.face_states(mesh, geo, U, "USR3")
        UL, UR = SV._positivity_fallback(UL, UR, U, mesh, G)
        lam = 0.0
        for X in (UL, UR, U):
            r, v, _E, p = OF.euler_primitives(X, G)
            lam = max(lam, float(np.max(np.linalg.norm(v, axis=1) + np.sqrt(G * p / r))))
        dt = 0.5 * float(np.min(geo.V / ssum)) / lam
        with np.errstate(all="ignore"):
            U1 = U + dt * SV.residual(mesh, geo, U, dict(base, positivity=True))
            U0 = U + dt * SV.residual(mesh, geo, U, base)
        r, _v, _E, p = OF.euler_primitives(U1, G)
        assert np.all(r > 0) and np.all(p > 0), seed
        r0, _v, _E, p0 = OF.euler_primitives(U0, G)
        lost += int(np.sum(~((r0 > 0) & (p0 > 0))))
    assert lost > 0


def test_smooth_flow_untouched():
    """On a smooth state the face-side states stay close to their cells:
    theta = 1 and the residual equals the plain one."""
    mesh = M.periodic_3d(6, jitter=0.2, seed=2)
    geo = OG.geometry(mesh)
    U = fields.isentropic_vortex(box=1.0, strength=1.0, centre=(0.5, 0.5))(geo.xc)
    p = dict(pde="euler", scheme="USR5", flux="hllc", gamma=G)
    np.testing.assert_array_equal(SV.residual(mesh, geo, U, dict(p, positivity=True)), SV.residual(mesh, geo, U, p))
