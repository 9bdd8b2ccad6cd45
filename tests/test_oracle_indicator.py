"""Pins of the indicator oracle: backprop against finite differences, Adam
against its first-step property, bfloat16 rounding against hand-worked
cases and the features against closed-form special cases."""
import numpy as np

from oracle import geometry as OG
from oracle import indicator as OI
from oracle import scheme as OS
from synth import fields
from synth import mesh as M


def test_backprop_matches_finite_differences():
    rng = np.random.default_rng(0)
    p = OI.xavier_init(1) + 0.05 * rng.normal(size=OI.N_PARAMS)
    X = rng.normal(size=(7, OI.N_IN))
    y = rng.random(7)
    _loss, g = OI.loss_and_grad(p, X, y)
    idx = rng.choice(OI.N_PARAMS, 60, replace=False)
    h = 1e-6
    for i in idx:
        e = np.zeros(OI.N_PARAMS)
        e[i] = h
        fd = (OI.loss_and_grad(p + e, X, y)[0] - OI.loss_and_grad(p - e, X, y)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1e-3, abs(fd)) + 1e-10, (i, fd, g[i])


def test_adam_first_step_moves_by_lr_sign():
    rng = np.random.default_rng(1)
    p = rng.normal(size=50)
    g = np.sign(rng.normal(size=50)) * (0.5 + rng.random(50))  # |g| >> eps
    p1, m, v = OI.adam_step(p, g, np.zeros(50), np.zeros(50), 1, lr=1e-3)
    np.testing.assert_allclose(p1 - p, -1e-3 * np.sign(g), rtol=1e-6)
    np.testing.assert_allclose(m, 0.1 * g)
    np.testing.assert_allclose(v, 0.001 * g * g)


def test_bf16_rounding_cases():
    one = 1.0
    cases = [(one, one), (one + 2 ** -8, one), (one + 3 * 2 ** -8, one + 2 ** -6),
             (one + 2 ** -8 + 2 ** -20, one + 2 ** -7), (-2.5, -2.5), (0.0, 0.0),
             (3.0e-3, 0.0030059814453125)]
    for x, ref in cases:
        assert OI.bf16_round(np.array([x]))[0] == ref, (x, OI.bf16_round(np.array([x]))[0])


def test_network_special_values():
    p = np.zeros(OI.N_PARAMS)
    p[-1] = 0.7
    th, _ = OI.forward(p, np.random.default_rng(2).normal(size=(5, OI.N_IN)))
    np.testing.assert_allclose(th, 1 / (1 + np.exp(-0.7)))


def test_features_uniform_and_linear_fields():
    mesh = M.periodic_3d(8)
    geo = OG.geometry(mesh)
    U = np.tile(fields.prim_to_cons(np.array([1.3]), np.array([[0.2, -0.1, 0.4]]), np.array([0.9])),
                (mesh.n_cells, 1))
    G1 = OS.gauss_linear(mesh, geo, U)
    F = OI.features(mesh, geo, U, G1)
    assert np.abs(F).max() < 1e-6   # rounding-level gradients of a constant field
    # linear density, still fluid, constant pressure: on a uniform lattice
    # the DOLINC differential equals twice the jump, so s = Delta, beta = 0
    # and the gradient ratio r = 1 away from the periodic seam
    x = geo.xc
    rho = 1.0 + 0.01 * (x[:, 0] + x[:, 1] + x[:, 2])
    U = fields.prim_to_cons(rho, np.zeros((mesh.n_cells, 3)), np.full(mesh.n_cells, 1.0))
    G1 = OS.gauss_linear(mesh, geo, U)
    F = OI.features(mesh, geo, U, G1)
    inner = np.all((x > 1 / 8) & (x < 7 / 8), axis=1)      # away from the seam
    assert inner.sum() == 216
    np.testing.assert_allclose(F[inner, 2], 0.0, atol=1e-9)   # max beta (rho)
    np.testing.assert_allclose(F[inner, 4], 1.0, atol=1e-9)   # min r (rho)
    np.testing.assert_allclose(F[inner, 1], 0.01 / 8 / (rho[inner] + 0.01 / 8), rtol=1e-6)
    # a local density maximum makes s and Delta opposite: beta = 1
    U2 = U.copy()
    c0 = np.argmin(np.linalg.norm(x - 0.5 - 1 / 12, axis=1))
    U2[c0, 0] += 0.5
    U2[c0, 4] += 0.0
    F2 = OI.features(mesh, geo, U2, OS.gauss_linear(mesh, geo, U2))
    assert F2[c0, 2] > 0.99


def test_ratio_feature_clip():
    """On a uniform lattice the Gauss gradient is the central difference, so
    a cell with neighbours a, c along x and value b has, on its +x face,
    r = s Delta / Delta^2 = (b - a) / (c - b) (s = 2 d.grad - Delta); its
    -x face gives (b - c) / (a - b) and its y and z faces (Delta = 0) give 0.
    (a, b, c) = (1.0, 1.1, 1.0 + 0.1 / 3): r = -1.5, the minimum feature.
    (a, b, c) = (1.0, 1.1, 1.075): r = -4, clipped to -2."""
    n = 6
    mesh = M.periodic_3d(n)
    geo = OG.geometry(mesh)
    i = np.floor(geo.xc[:, 0] * n + 1e-9).astype(int)
    for c_val, want in ((1.0 + 0.1 / 3.0, -1.5), (1.075, -2.0)):
        row = {1: 1.0, 2: 1.1, 3: c_val}
        rho = np.array([row.get(k, 1.0) for k in i])
        U = fields.prim_to_cons(rho, np.zeros((mesh.n_cells, 3)), np.full(mesh.n_cells, 1.0))
        F = OI.features(mesh, geo, U, OS.gauss_linear(mesh, geo, U))
        sel = i == 2
        np.testing.assert_allclose(F[sel, 4], want, atol=1e-9)   # min r of the density channel
