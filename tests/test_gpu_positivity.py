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
