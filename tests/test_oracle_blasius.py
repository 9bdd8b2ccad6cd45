"""Pins of the graded-mesh reconstruction study (Sec. 3.1) on the oracle.

The input generator is pinned to the textbook Blasius solution; the oracle's
single-step DOLINC reconstruction of the boundary-layer velocity then shows
the paper's two observations: the global error grows with the mesh growth
rate (fewer, wider cells over the same layer), and raising the order from
the third-order USR3 to the fourth-order CSR4 (and on to USR5 and CSR6)
lowers it considerably on every graded mesh.  (The paper's figures give no
values to compare with; the comparison with non-DOLINC gradient schemes is
not part of this build.)
"""
import numpy as np
import pytest
from scipy.optimize import brentq

from synth import mesh as M

from . import graded_study as GS


def test_blasius_profile_textbook_values():
    """f''(0) = 0.33206, f' = 0.99 at eta = 4.91, displacement thickness
    1.7208 (Blasius' flat-plate solution)."""
    b = GS.blasius()
    assert abs(b.fpp0 - 0.33206) < 1e-5
    e99 = brentq(lambda e: b.f_and_fp(np.array([e]))[1][0] - 0.99, 1.0, 10.0)
    assert abs(e99 - 4.91) < 0.01
    f, fp = b.f_and_fp(np.array([10.0]))
    assert abs(fp[0] - 1.0) < 1e-7 and abs((10.0 - f[0]) - 1.7208) < 1e-4
    # v at the edge: (eta f' - f) / 2 -> 0.8604 sqrt(nu U / x)
    assert abs(0.5 * (10.0 * fp[0] - f[0]) - 0.8604) < 1e-3


def test_graded_mesh_layout():
    """Rows grow by the stated factor from the wall (the last one absorbs the
    remainder) and the wall and top are the two open patches."""
    ys = M.graded_spacing(0.05, 1.5, 12.0)
    h = np.diff(ys)
    assert abs(h[0] - 0.05) < 1e-15 and np.allclose(h[1:-1] / h[:-2], 1.5)
    assert ys[-1] == 12.0 and h[-1] >= 0.5 * h[-2]
    m = M.boundary_layer_2d(GS.NX, GS.LENGTH, 0.05, 1.5, 12.0)
    assert set(np.unique(m.patch[m.patch >= 0])) == {2, 3}
    assert (m.patch == 2).sum() == GS.NX and (m.patch == 3).sum() == GS.NX


@pytest.fixture(scope="module")
def errors():
    out = {}
    for r in GS.GROWTHS:
        _m, X, U, ex = GS.case(r)
        sel = GS.measured_faces(X)
        for comp in (0, 1):
            for sch in ("CD2", "USR3", "CSR4", "USR5", "CSR6"):
                UL, UR = GS.oracle_face_states(X, U[:, comp], sch)
                out[(r, comp, sch)] = GS.rel_error(UL, UR, ex[:, comp], sel)
    return out


@pytest.mark.parametrize("comp", [0, 1], ids=["u", "v"])
def test_error_grows_with_growth_rate(errors, comp):
    for sch in ("USR3", "CSR4", "USR5", "CSR6"):
        e = [errors[(r, comp, sch)] for r in GS.GROWTHS]
        assert e[-1] > 10 * e[0], (sch, e)
        assert all(e[i + 1] > e[i] for i in range(2)), (sch, e)  # 1.1 -> 1.2 -> 1.3


@pytest.mark.parametrize("comp", [0, 1], ids=["u", "v"])
def test_higher_order_dolinc_is_more_accurate_on_every_graded_mesh(errors, comp):
    for r in GS.GROWTHS:
        e = [errors[(r, comp, s)] for s in ("CD2", "USR3", "CSR4", "USR5", "CSR6")]
        assert all(e[i + 1] < e[i] for i in range(len(e) - 1)), (r, e)
        assert e[2] < 0.7 * e[1], (r, e)  # USR3 -> CSR4
