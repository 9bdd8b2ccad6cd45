"""Non-coupled boundaries through auxiliary cells (Sec. 2.6) through the C ABI
against the FP64 oracle (oracle/boundary.py): element-wise FP64 residuals and
RK steps with every boundary type, the FP32 stage error, and the 1-D shock
tubes of Sec. 3.4 and a reflecting wall against exact Riemann solutions.
"""
import numpy as np
import pytest

from oracle import boundary as OB
from synth import fields
from synth import mesh as M

from .helpers import oracle_params
from .test_gpu_parity import FP32_REF, _close, _euler_state, _group_errors
from .test_oracle_boundary import LAX, SOD

pytestmark = pytest.mark.gpu

KIND = {OB.ZERO_GRADIENT: "zero_gradient", OB.DIRICHLET: "dirichlet", OB.NEUMANN: "neumann",
        OB.SLIP_WALL: "slip_wall"}

MESHES = {
    "hex3d": lambda: M.bounded(M.periodic_3d(7, 6, 5, jitter=0.2, seed=7), 0),
    "mixed3d": lambda: M.bounded(M.periodic_3d(6, 5, 4, jitter=0.2, seed=11,
                                               kinds=M.mixed_kinds(6, 5, 4, split_frac=0.5, seed=12)), 0),
    "tri2d": lambda: M.bounded(M.periodic_2d(12, 10, jitter=0.2, seed=1, split=1.0, diagonal="main"), 0),
    "mixed2d": lambda: M.bounded(M.periodic_2d(14, 13, jitter=0.25, seed=2, split=0.5, diagonal="seeded",
                                               pentagon_frac=0.1), 0),
}

CASES = [
    ("hex3d", dict(pde="euler", scheme="USR5", flux="hllc"), {0: (OB.ZERO_GRADIENT,), 1: (OB.SLIP_WALL,)}),
    ("hex3d", dict(pde="euler", scheme="WENO5", flux="rusanov"), {0: (OB.SLIP_WALL,), 1: (OB.SLIP_WALL,)}),
    ("mixed3d", dict(pde="euler", scheme="USR3", flux="rusanov"),
     {0: (OB.DIRICHLET, [1.1, 0.2, 0.0, 0.1, 2.6]), 1: (OB.NEUMANN, [0.3, -0.1, 0.2, 0.0, 0.5])}),
    ("mixed3d", dict(pde="euler", scheme="CSR4", flux="hllc"), {0: (OB.ZERO_GRADIENT,), 1: (OB.ZERO_GRADIENT,)}),
    ("tri2d", dict(pde="advection", scheme="USR5"), {0: (OB.DIRICHLET, [0.7]), 1: (OB.NEUMANN, [-0.4])}),
    ("mixed2d", dict(pde="burgers", scheme="ENO3"), {0: (OB.NEUMANN, [0.5]), 1: (OB.DIRICHLET, [0.2])}),
    ("mixed2d", dict(pde="advection", scheme="CSR4"), {0: (OB.ZERO_GRADIENT,), 1: (OB.DIRICHLET, [-0.3])}),
]
IDS = [f"{n}-{k['pde']}-{k['scheme']}-{'-'.join(KIND[b[0]] for b in v.values())}" for n, k, v in CASES]


@pytest.fixture(scope="module")
def meshes():
    out = {}
    for k, f in MESHES.items():
        m = f()
        out[k] = (m, OB.extend(m))
    return out


def _solver(mesh, bcs, **kw):
    from paper_2404_08952_amd import Solver
    s = Solver(mesh, **kw)
    for p, spec in bcs.items():
        s.set_boundary(p, KIND[spec[0]], spec[1] if len(spec) > 1 else None)
    return s


def _state(mesh, kw, rng):
    if kw["pde"] == "euler":
        return _euler_state(mesh.n_cells, rng)
    if kw["pde"] == "burgers":
        return 0.5 + 0.3 * rng.normal(size=(mesh.n_cells, 1))
    return rng.normal(size=(mesh.n_cells, 1))


@pytest.mark.parametrize("name,kw,bcs", CASES, ids=IDS)
def test_residual_parity(name, kw, bcs, meshes):
    mesh, X = meshes[name]
    U = _state(mesh, kw, np.random.default_rng(21))
    ref = OB.residual(X, U, oracle_params(kw), bcs)
    # full states, and each face side about its own cell (the auxiliary
    # cells are ordinary rows to it)
    for extra in ({}, dict(u_ref=FP32_REF)):
        s = _solver(mesh, bcs, **kw, **extra)
        R = s.to_external(s.residual(s.to_internal(U)))
        for v in range(ref.shape[1]):
            _close(R[:, v], ref[:, v])
        s.close()


@pytest.mark.parametrize("name,kw,bcs", [CASES[0], CASES[2], CASES[5]], ids=[IDS[0], IDS[2], IDS[5]])
def test_rk_step_parity(name, kw, bcs, meshes):
    mesh, X = meshes[name]
    U = _state(mesh, kw, np.random.default_rng(22))
    s = _solver(mesh, bcs, **kw)
    Ud = s.to_internal(U)
    ref = U.copy()
    for _ in range(3):
        s.rk_step(Ud, 1e-3)
        ref = OB.rk_step(X, ref, 1e-3, oracle_params(kw), bcs)
    _close(s.to_external(Ud), ref)


@pytest.mark.parametrize("name,kw,bcs", CASES, ids=IDS)
def test_fp32_stage_error(name, kw, bcs, meshes):
    mesh, X = meshes[name]
    U = _state(mesh, kw, np.random.default_rng(23)).astype(np.float32).astype(np.float64)
    s = _solver(mesh, bcs, precision="fp32", **kw, u_ref=FP32_REF)
    R32 = s.to_external(s.residual(s.to_internal(U)))
    ref = OB.residual(X, U, oracle_params(kw), bcs)
    errs = _group_errors(R32, ref)
    assert max(errs) <= 1e-5, errs


def test_slip_walls_conserve_mass_and_energy():
    """Closed box in x (slip walls at both ends): mass and energy totals are
    conserved to round-off over 20 steps; x-momentum is not (wall pressure)."""
    mesh = MESHES["hex3d"]()
    U = _euler_state(mesh.n_cells, np.random.default_rng(24))
    s = _solver(mesh, {0: (OB.SLIP_WALL,), 1: (OB.SLIP_WALL,)}, pde="euler", scheme="USR5", flux="hllc")
    Ud = s.to_internal(U)
    d0 = s.diagnostics(Ud)
    s.advance(Ud, 2e-3, 20)
    d1 = s.diagnostics(Ud)
    assert abs(d1[0] - d0[0]) < 1e-12 * abs(d0[0])
    assert abs(d1[4] - d0[4]) < 1e-12 * abs(d0[4])
    assert d1[-1] == 0


def _tube(N, prob, scheme, precision="fp64", tvd=False, cfl=0.3):
    left_state, right_state, T = prob
    mesh = M.bounded(M.periodic_3d(N, 2, 2, lengths=(1.0, 0.02, 0.02)), 0)
    X = OB.extend(mesh)
    x = X.geo.xc[:X.n_cells, 0]
    lft = x < 0.5
    prim = [np.where(lft, a, b) for a, b in zip(left_state, right_state)]
    vel = np.zeros((mesh.n_cells, 3))
    vel[:, 0] = prim[1]
    U0 = fields.prim_to_cons(prim[0], vel, prim[2])
    kw = dict(pde="euler", scheme=scheme, flux="rusanov", precision=precision)
    if tvd:
        kw["blend"] = "theta"
    if precision == "fp32":
        kw["u_ref"] = FP32_REF
    s = _solver(mesh, {}, **kw)
    if tvd:
        s.set_theta(s.torch.zeros(s.n_rows, dtype=s.torch.float32, device=s.device))
    smax = 4.5 if prob is LAX else 2.5
    steps = int(np.ceil(T * N * smax / cfl))
    Ud = s.to_internal(U0)
    s.advance(Ud, T / steps, steps)
    U = s.to_external(Ud)
    ex = fields.riemann_exact(left_state, right_state, (x - 0.5) / T)
    return np.mean(np.abs(U[:, 0] - ex[0])), U


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_sod_and_lax_tubes(precision):
    """Sec. 3.4's 1-D Riemann problems with zero-gradient ends and the local
    Lax-Friedrichs flux: WENO5 close to the exact density, sharper than the
    Van Leer TVD scheme; at N = 50 the FP64 GPU run matches the oracle."""
    for prob, tol in ((SOD, 0.009), (LAX, 0.024)):
        e_w, U = _tube(100, prob, "WENO5", precision)
        e_t, _ = _tube(100, prob, "CD2", precision, tvd=True)
        assert np.isfinite(U).all()
        assert e_w < tol and e_w < e_t, (precision, prob, e_w, e_t)
    if precision == "fp64":
        from .test_oracle_boundary import shock_tube
        e_o, Uo = shock_tube(50, SOD, "WENO5")
        e_g, Ug = _tube(50, SOD, "WENO5")
        _close(Ug, Uo, rtol=1e-9, afloor=1e-11)


def test_reflecting_wall_on_gpu():
    """Uniform flow into a slip wall: the mirrored Riemann problem's exact
    reflected shock, within the same bounds as the oracle."""
    N, T = 80, 0.25
    state = (1.0, 0.5, 1.0)
    mesh = M.bounded(M.periodic_3d(N, 2, 2, lengths=(1.0, 0.02, 0.02)), 0)
    X = OB.extend(mesh)
    x = X.geo.xc[:X.n_cells, 0]
    vel = np.zeros((mesh.n_cells, 3))
    vel[:, 0] = state[1]
    U0 = fields.prim_to_cons(np.full(mesh.n_cells, state[0]), vel, np.full(mesh.n_cells, state[2]))
    s = _solver(mesh, {0: (OB.ZERO_GRADIENT,), 1: (OB.SLIP_WALL,)}, pde="euler", scheme="WENO5", flux="rusanov")
    steps = int(np.ceil(T * N * 3.0 / 0.3))
    Ud = s.to_internal(U0)
    s.advance(Ud, T / steps, steps)
    U = s.to_external(Ud)
    ex = fields.riemann_exact(state, (state[0], -state[1], state[2]), (x - 1.0) / T)
    near = x > 0.5
    assert np.mean(np.abs(U[near, 0] - ex[0][near])) < 0.02
    assert U[x > 0.95, 0].min() > 1.4


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_theta_blend_with_boundaries(precision, meshes):
    """Blend with given per-cell weights next to walls and a Dirichlet inflow:
    the auxiliary cells take their boundary cell's weight."""
    mesh, X = meshes["mixed3d"]
    rng = np.random.default_rng(25)
    U = _euler_state(mesh.n_cells, rng)
    if precision == "fp32":
        U = U.astype(np.float32).astype(np.float64)
    theta = rng.random(mesh.n_cells).astype(np.float32)
    bcs = {0: (OB.DIRICHLET, [1.05, 0.1, 0.0, 0.0, 2.5]), 1: (OB.SLIP_WALL,)}
    kw = dict(pde="euler", scheme="USR5", flux="hllc")
    extra = dict(u_ref=FP32_REF) if precision == "fp32" else {}
    s = _solver(mesh, bcs, blend="theta", precision=precision, **kw, **extra)
    th = np.zeros(s.n_rows, dtype=np.float32)
    th[s.perm] = theta
    s.set_theta(s.torch.from_numpy(th).to(s.device))
    R = s.to_external(s.residual(s.to_internal(U)))
    ref = OB.residual(X, U, oracle_params(kw), bcs, theta=theta.astype(np.float64))
    if precision == "fp64":
        for v in range(ref.shape[1]):
            _close(R[:, v], ref[:, v])
    else:
        assert max(_group_errors(R, ref)) <= 1e-5


def test_learned_blend_with_boundaries(meshes):
    """The learned blend next to a Dirichlet inflow and slip walls (FP64):
    the stage (network on the context's second stream, auxiliary cells'
    weights rewritten after it joins) equals, bit for bit, the residual with
    the weights network(features(U)) given explicitly, and matches the oracle
    fed those weights."""
    from paper_2404_08952_amd.training import WEIGHTS
    mesh, X = meshes["mixed3d"]
    rng = np.random.default_rng(26)
    U = _euler_state(mesh.n_cells, rng)
    bcs = {0: (OB.DIRICHLET, [1.05, 0.1, 0.0, 0.0, 2.5]), 1: (OB.SLIP_WALL,)}
    kw = dict(pde="euler", scheme="USR5", flux="hllc")
    sl = _solver(mesh, bcs, blend="learned", precision="fp64", **kw)
    sl.mlp_set(np.load(WEIGHTS))
    st = _solver(mesh, bcs, blend="theta", precision="fp64", **kw)
    Ui = sl.to_internal(U)
    sl.residual(sl.to_internal(_euler_state(mesh.n_cells, rng)))   # other weights left behind
    R = sl.residual(Ui)
    th = sl.mlp_forward(sl.features(Ui, fp32=False)[1])
    st.set_theta(th)
    Rt = st.residual(Ui)
    assert sl.torch.equal(R, Rt)
    theta = th.cpu().numpy()[:sl.n_rows][sl.perm].astype(np.float64)
    ref = OB.residual(X, U, oracle_params(kw), bcs, theta=theta)
    Re = sl.to_external(R)
    for v in range(ref.shape[1]):
        _close(Re[:, v], ref[:, v])
    sl.close()
    st.close()
