"""The positivity rule on the GPU path: a face side whose reconstructed
density or pressure is not positive takes its own cell's value (the same
rule in the oracle).  States with density and pressure spread over three
decades make the high-order reconstruction undershoot on many face sides of
both orientations; the FP64 path must match the oracle element by element
(states after the rule, fluxes, residual), and the FP32 reference-state form
must take the same decisions and stay within the stage tolerance.  The
states are chosen so that every reconstructed density and pressure is at
least 1e-3 of its scale away from zero, so the two precisions decide alike.
"""
import numpy as np
import pytest

from oracle import flux as OF
from oracle import geometry as OG
from oracle import scheme as OS
from oracle import solver as SV
from synth import fields

from .helpers import oracle_params, rel_l2, small_meshes

pytestmark = pytest.mark.gpu

MESHES = small_meshes()
GAMMA = 1.4


def _violent_state(n, rng):
    rho = np.exp(rng.normal(scale=1.6, size=n))
    p = np.exp(rng.normal(scale=1.6, size=n))
    vel = 0.5 * rng.normal(size=(n, 3))
    return fields.prim_to_cons(rho, vel, p)


def _case(mesh, geo, scheme):
    """First seed whose reconstructed densities and pressures all keep a
    margin of 1e-3 (relative to the face's cell values) from zero, with
    fallbacks on both sides of many faces."""
    for seed in range(40):
        U = _violent_state(mesh.n_cells, np.random.default_rng(100 + seed))
        U = U.astype(np.float32).astype(np.float64)
        UL, UR, _ = OS.face_states(mesh, geo, U, scheme)
        rL, _v, _E, pL = OF.euler_primitives(UL, GAMMA)
        rR, _v, _E, pR = OF.euler_primitives(UR, GAMMA)
        _r, _v, _E, pc = OF.euler_primitives(U, GAMMA)
        rs = np.maximum(U[mesh.owner, 0], U[mesh.neighbour, 0])
        ps = np.maximum(pc[mesh.owner], pc[mesh.neighbour])
        margin = min(np.abs(rL / rs).min(), np.abs(rR / rs).min(), np.abs(pL / ps).min(), np.abs(pR / ps).min())
        badL = ~((rL > 0) & (pL > 0))
        badR = ~((rR > 0) & (pR > 0))
        if margin > 1e-3 and badL.sum() >= 8 and badR.sum() >= 8:
            return U, badL, badR
    raise AssertionError("no seed gives a clear positivity case")


def _solver(mesh, **kw):
    from paper_2404_08952_amd import Solver
    return Solver(mesh, **kw)


@pytest.mark.parametrize("name,scheme,flux", [("mixed3d", "USR5", "hllc"), ("hex3d", "USR3", "rusanov"),
                                              ("tet3d", "USR5", "rusanov")])
def test_positivity_fallback_fp64(name, scheme, flux):
    mesh = MESHES[name]
    geo = OG.geometry(mesh)
    U, badL, badR = _case(mesh, geo, scheme)
    kw = dict(pde="euler", scheme=scheme, flux=flux)
    s = _solver(mesh, **kw)
    Ud = s.to_internal(U)
    UL, UR, F = (x.cpu().numpy() for x in s.face_states(Ud))
    rL, rR, _ = OS.face_states(mesh, geo, U, scheme)
    rL, rR = SV._positivity_fallback(rL, rR, U, mesh, GAMMA)
    scale = np.abs(U).max()
    np.testing.assert_allclose(UL, rL, rtol=1e-10, atol=1e-12 * scale)
    np.testing.assert_allclose(UR, rR, rtol=1e-10, atol=1e-12 * scale)
    # the fallen-back sides are exactly their cells' values
    np.testing.assert_array_equal(UL[badL], U[mesh.owner[badL]])
    np.testing.assert_array_equal(UR[badR], U[mesh.neighbour[badR]])
    ref_F = SV.face_flux(mesh, geo, U, oracle_params(kw))
    np.testing.assert_allclose(F, ref_F, rtol=1e-10, atol=1e-12 * np.abs(ref_F).max())
    R = s.to_external(s.residual(Ud))
    ref = SV.residual(mesh, geo, U, oracle_params(kw))
    np.testing.assert_allclose(R, ref, rtol=1e-10, atol=1e-12 * np.abs(ref).max())
    s.close()


@pytest.mark.parametrize("form", ["cell", "constant"])
@pytest.mark.parametrize("name,scheme,flux", [("mixed3d", "USR5", "hllc"), ("hex3d", "USR3", "rusanov")])
def test_positivity_fallback_fp32_reference_state(name, scheme, flux, form):
    mesh = MESHES[name]
    geo = OG.geometry(mesh)
    U, badL, badR = _case(mesh, geo, scheme)
    kw = dict(pde="euler", scheme=scheme, flux=flux)
    uref = tuple(float(x) for x in U.mean(0)) if form == "constant" else "cell"
    s = _solver(mesh, precision="fp32", u_ref=uref, **kw)
    Ud = s.to_internal(U)
    UL, UR, _F = (x.cpu().numpy().astype(np.float64) for x in s.face_states(Ud))
    rL, rR, _ = OS.face_states(mesh, geo, U, scheme)
    rL, rR = SV._positivity_fallback(rL, rR, U, mesh, GAMMA)
    # same decisions: the sides that fell back hold their cells' values
    # (to the rounding of U - U_ref + U_ref in FP32)
    tol = 4 * np.finfo(np.float32).eps * 2 * np.abs(U).max()
    assert np.abs(UL[badL] - U[mesh.owner[badL]]).max() <= tol
    assert np.abs(UR[badR] - U[mesh.neighbour[badR]]).max() <= tol
    assert rel_l2(UL, rL) <= 1e-5 and rel_l2(UR, rR) <= 1e-5
    R = s.to_external(s.residual(Ud))
    ref = SV.residual(mesh, geo, U, oracle_params(kw))
    errs = [rel_l2(R[:, 0], ref[:, 0]), rel_l2(R[:, 1:4], ref[:, 1:4]), rel_l2(R[:, 4], ref[:, 4])]
    assert max(errs) <= 1e-5, errs
    s.close()


# ---------------------------------------------------------------- positivity of the cell averages
@pytest.mark.parametrize("name,scheme,flux,blend", [("mixed3d", "USR3", "rusanov", "theta"),
                                                    ("mixed3d", "USR5", "hllc", "none"),
                                                    ("tet3d", "CSR4", "rusanov", "none")])
def test_cell_positivity_scaling_fp64(name, scheme, flux, blend):
    """The per-cell scaling of the face-side states (params positivity): FP64
    residual and exported face states equal the oracle's element by element
    on states where many cells are scaled."""
    from oracle import positivity as OP
    mesh = MESHES[name]
    geo = OG.geometry(mesh)
    U, _bl, _br = _case(mesh, geo, scheme)
    kw = dict(pde="euler", scheme=scheme, flux=flux)
    rng = np.random.default_rng(7)
    theta = rng.random(mesh.n_cells).astype(np.float32) if blend == "theta" else None
    s = _solver(mesh, **kw, blend=blend, positivity=True)
    if theta is not None:
        th = np.empty_like(theta)
        th[s.perm] = theta
        s.set_theta(s.torch.from_numpy(th).to(s.device))
    th64 = None if theta is None else theta.astype(np.float64)
    Ud = s.to_internal(U)
    R = s.to_external(s.residual(Ud))
    ref = SV.residual(mesh, geo, U, dict(oracle_params(kw), positivity=True), theta=th64)
    np.testing.assert_allclose(R, ref, rtol=1e-10, atol=1e-12 * np.abs(ref).max())
    # the scaling acts: it changes the residual of many cells
    plain = SV.residual(mesh, geo, U, oracle_params(kw), theta=th64)
    assert (np.abs(plain - ref).max(1) > 1e-6 * np.abs(ref).max()).sum() > 10
    UL, UR, _F = (x.cpu().numpy() for x in s.face_states(Ud))
    G = OS.cell_derivs(mesh, geo, U, max(OS.scheme_order(scheme), 1))
    rL, rR, _ = OS.face_states(mesh, geo, U, scheme, G)
    if th64 is not None:
        from oracle import limiter as OL
        LL, LR = OL.limited_states(mesh, geo, U, G[1])
        rL, rR = OL.blend(rL, rR, LL, LR, th64, mesh)
    rL, rR = SV._positivity_fallback(rL, rR, U, mesh, GAMMA)
    rL, rR, _t = OP.scale_face_states(mesh, geo, U, rL, rR, GAMMA)
    scale = np.abs(U).max()
    np.testing.assert_allclose(UL, rL, rtol=1e-10, atol=1e-12 * scale)
    np.testing.assert_allclose(UR, rR, rtol=1e-10, atol=1e-12 * scale)
    s.close()


def test_cell_positivity_scaling_fp32_cell_form():
    mesh = MESHES["mixed3d"]
    geo = OG.geometry(mesh)
    U, _bl, _br = _case(mesh, geo, "USR5")
    kw = dict(pde="euler", scheme="USR5", flux="hllc")
    s = _solver(mesh, precision="fp32", u_ref="cell", positivity=True, **kw)
    R = s.to_external(s.residual(s.to_internal(U)))
    ref = SV.residual(mesh, geo, U, dict(oracle_params(kw), positivity=True))
    errs = [rel_l2(R[:, 0], ref[:, 0]), rel_l2(R[:, 1:4], ref[:, 1:4]), rel_l2(R[:, 4], ref[:, 4])]
    assert max(errs) <= 1e-5, errs
    s.close()


def test_cell_positivity_refused_where_not_built():
    from paper_2404_08952_amd import binding as B
    from synth import mesh as M
    with pytest.raises(B.DolincError) as e:
        _solver(MESHES["tri2d"], pde="advection", scheme="USR3", positivity=True)
    assert e.value.status in (B.EUNSUPPORTED, B.EINVAL)
    with pytest.raises(B.DolincError) as e:
        _solver(MESHES["hex3d"], pde="euler", scheme="USR3", flux="rusanov", u_ref=(1, 0, 0, 0, 2.5),
                positivity=True)
    assert e.value.status == B.EUNSUPPORTED
    bm = M.bounded(M.periodic_3d(4, 3, 3), 0)
    with pytest.raises(B.DolincError) as e:
        _solver(bm, pde="euler", scheme="USR3", flux="rusanov", positivity=True)
    assert e.value.status == B.EUNSUPPORTED
    # the constant reference state is Euler-only (the cell form is not)
    with pytest.raises(B.DolincError) as e:
        _solver(MESHES["tri2d"], pde="advection", scheme="USR3", u_ref=(1, 0, 0, 0, 0))
    assert e.value.status == B.EUNSUPPORTED
    _solver(MESHES["tri2d"], pde="advection", scheme="USR3", u_ref="cell").close()
