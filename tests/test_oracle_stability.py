"""Linear stability of the oracle's semi-discrete operator from its
spectrum: the evidence for the schemes the tetrahedral and mixed workloads
run with.

The DOLINC inversion assumes a constant growth rate between neighbouring
cells (Sec. 2.2), and the paper names low accuracy on tetrahedral and hybrid
grids as the method's limitation (Conclusions).  On jittered simplicial and
mixed meshes the growth rate varies from face to face.  The tests below take
the matrix L of dU/dt = L U for linear advection with the upwind flux
(columns from the oracle's residual of unit vectors) and report
max Re(lambda) in units of |a| / h, h = (mean cell volume)^(1/dim): a
positive value grows without bound at any time step.  The spectrum itself is
pinned first on a uniform line, where USR3 is the kappa = 1/3 upwind-biased
scheme with a closed-form symbol.
"""
import numpy as np

from oracle import geometry as OG
from oracle import solver as SV
from synth import mesh as M


def _operator(mesh, scheme, vel):
    geo = OG.geometry(mesh)
    n = mesh.n_cells
    E = np.eye(n)
    p = dict(pde="advection", scheme=scheme, flux="upwind", adv_vel=vel)
    L = np.stack([SV.residual(mesh, geo, E[:, j:j + 1], p)[:, 0] for j in range(n)], 1)
    return L, np.mean(geo.V) ** (1.0 / mesh.dim)


def _max_re(mesh, scheme, vel):
    L, h = _operator(mesh, scheme, vel)
    return np.linalg.eigvals(L).real.max() * h / np.linalg.norm(vel)


def test_uniform_line_usr3_symbol():
    """Uniform periodic lines of n cells, a = 1 along them (a 16 x 2 x 2
    lattice: four uncoupled lines): USR3's face value is
    (-u_{i-1} + 5 u_i + 2 u_{i+1}) / 6, so mode k of each line has
    lambda h / a = -[(1 - cos t)^2 / 3 + i (8 sin t - sin 2t) / 6], t = 2 pi k / n."""
    n = 16
    mesh = M.periodic_3d(n, 2, 2, lengths=(1.0, 2.0 / n, 2.0 / n))
    L, _h = _operator(mesh, "USR3", (1.0, 0.0, 0.0))
    ev = np.linalg.eigvals(L) / n
    t = 2 * np.pi * np.arange(n) / n
    ref = np.tile(-((1 - np.cos(t)) ** 2 / 3 + 1j * (8 * np.sin(t) - np.sin(2 * t)) / 6), 4)
    np.testing.assert_allclose(np.sort(ev.real), np.sort(ref.real), atol=1e-12)
    np.testing.assert_allclose(np.sort(ev.imag), np.sort(ref.imag), atol=1e-12)


def test_jittered_tetrahedra():
    """The vortex workload's mesh recipe (Kuhn tetrahedra, +-0.2 h jitter):
    the central CSR4 state and the second-order USR5 template have growing
    modes; USR3 none above round-off -- the workload runs USR3."""
    mesh = M.periodic_3d(4, jitter=0.2, seed=21, kinds=M.KUHN6)
    vel = (1.0, 0.5, 0.3)
    assert _max_re(mesh, "CSR4", vel) > 0.2
    assert _max_re(mesh, "USR5", vel) > 0.03
    assert _max_re(mesh, "USR3", vel) < 1e-10


def test_unjittered_tetrahedra():
    """Unjittered Kuhn tetrahedra: CSR4 has no growing mode (a central
    scheme on a lattice), while USR3 has a weak global one,
    Re lambda = +0.004 to +0.009 |a| / h depending on the direction (and
    USR5 a stronger one): less than e^0.3 over the vortex run's 200 steps."""
    mesh = M.periodic_3d(4, jitter=0.0, kinds=M.KUHN6)
    vel = (1.0, 0.5, 0.3)
    assert _max_re(mesh, "CSR4", vel) < 1e-10
    assert 1e-3 < _max_re(mesh, "USR3", vel) < 2e-2
    assert _max_re(mesh, "USR5", vel) > 0.02


def test_jittered_hexahedra():
    mesh = M.periodic_3d(4, jitter=0.2, seed=21)
    vel = (1.0, 0.5, 0.3)
    assert _max_re(mesh, "USR3", vel) < 1e-10
    assert _max_re(mesh, "USR5", vel) < 1e-10
    assert _max_re(mesh, "CSR4", vel) > 0.02


def test_mixed_2d_jittered_usr3_mode_on_triangles():
    """The 2-D Burgers workload's recipe (half the quads split, 5 % pentagons,
    +-0.25 h jitter) at 24^2: USR3 has a growing mode localised on a few
    jittered triangles (its largest component sits on a three-face cell),
    CSR4 a far stronger one.  Without the jitter USR3 has none (CSR4 still
    has); with jitter but no triangles neither does USR3.  (Not every
    realisation has such a triangle: the 16^2 mesh of the same recipe has
    none.)"""
    vel = (0.5, 0.5, 0.0)
    kw = dict(seed=11, split_seed=12, diagonal="seeded")
    mesh = M.periodic_2d(24, 24, jitter=0.25, split=0.5, pentagon_frac=0.05, **kw)
    L, h = _operator(mesh, "USR3", vel)
    ev, V = np.linalg.eig(L)
    i = np.argmax(ev.real)
    assert ev[i].real * h / np.linalg.norm(vel) > 0.05
    faces = np.bincount(mesh.owner, minlength=mesh.n_cells) + np.bincount(mesh.neighbour, minlength=mesh.n_cells)
    assert faces[np.argmax(np.abs(V[:, i]))] == 3
    assert _max_re(mesh, "CSR4", vel) > 1.0
    reg = M.periodic_2d(24, 24, jitter=0.0, split=0.5, pentagon_frac=0.05, **kw)
    assert _max_re(reg, "USR3", vel) < 1e-10
    assert _max_re(reg, "CSR4", vel) > 0.1
    quads = M.periodic_2d(24, 24, jitter=0.25, split=0.0, **kw)
    assert _max_re(quads, "USR3", vel) < 1e-10
