"""The five synthetic workloads and the small pin meshes, seeded.

Each workload mirrors a test problem shape from the paper's results section
(2-D advection, 2-D Burgers, 3-D Euler) on periodic unstructured meshes; the
paper's own data sets are not available, so these stand in for them.  Sizes
are lattice counts; ``n`` overrides the lattice size for scaled-down copies.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import fields
from .mesh import KUHN6, HEX, mixed_kinds, periodic_2d, periodic_3d


@dataclass
class Case:
    name: str
    mesh: object
    params: dict
    U0: np.ndarray
    dt: float
    steps: int
    exact: object = None           # callable t -> field fn (or None)
    info: dict = field(default_factory=dict)


def nominal_dt(mesh, pde, U, cfl, vel=None, simplex=False):
    """CFL time step from the lattice spacing and the fastest wave of U.

    h_eff = h / dim on hex/quad lattices and h / (dim + 1) on simplex
    lattices, h being the smallest lattice spacing.
    """
    lat = mesh.info["lattice"]
    h = min(L / n for L, n in zip(mesh.lengths, lat))
    h_eff = h / (mesh.dim + 1 if simplex else mesh.dim)
    lam = fields.max_wave_speed(pde, U, vel=vel)
    return cfl * h_eff / lam


def _steps_to(t_end, dt):
    n = int(np.ceil(t_end / dt - 1e-12))
    return n, t_end / n


def advection_2d(n=32, jitter=0.2, seed=1, perm_seed=2, scheme="USR3", t_end=0.1,
                 cfl=0.5, quad_pts=5):
    """2-D linear advection, a = (1, 0.5), u0 = sin(2 pi x) sin(2 pi y)."""
    mesh = periodic_2d(n, n, jitter=jitter, seed=seed, split=1.0, diagonal="main",
                       perm_seed=perm_seed)
    vel = np.array([1.0, 0.5])
    U0 = fields.cell_averages(mesh, fields.sine2d(vel, 0.0), n_pts=quad_pts)
    dt0 = nominal_dt(mesh, "advection", U0, cfl, vel=vel, simplex=True)
    steps, dt = _steps_to(t_end, dt0)
    params = dict(pde="advection", scheme=scheme, flux="upwind", adv_vel=(1.0, 0.5, 0.0))
    return Case("advection2d", mesh, params, U0, dt, steps,
                exact=lambda t: fields.sine2d(vel, t))


def burgers_2d(n=256, jitter=0.25, seed=11, split_seed=12, perm_seed=13, scheme="USR3",
               t_end=0.05, cfl=0.5, quad_pts=4, pentagon_frac=0.05):
    """2-D Burgers along (1,1), u0 = 0.5 + 0.25 sin(2 pi (x + y)), mixed cells."""
    mesh = periodic_2d(n, n, jitter=jitter, seed=seed, split=0.5, split_seed=split_seed,
                       diagonal="seeded", pentagon_frac=pentagon_frac, perm_seed=perm_seed)
    U0 = fields.cell_averages(mesh, fields.burgers_diag(0.0), n_pts=quad_pts)
    dt0 = nominal_dt(mesh, "burgers", U0, cfl, simplex=True)
    steps, dt = _steps_to(t_end, dt0)
    params = dict(pde="burgers", scheme=scheme, flux="upwind")
    return Case("burgers2d", mesh, params, U0, dt, steps, exact=lambda t: fields.burgers_diag(t))


# free stream of the vortex workload (rho, rho u, rho v, rho w, rho E)
VORTEX_REF = (1.0, 1.0, 1.0, 0.0, 1.0 / 0.4 + 1.0)


def vortex_3d(n=64, jitter=0.2, seed=21, perm_seed=22, scheme="CSR4", flux="rusanov",
              steps=200, cfl=0.4, quad_pts=3, point_ic=False):
    """3-D Euler isentropic vortex in [0,10]^3 on Kuhn-split tetrahedra."""
    mesh = periodic_3d(n, lengths=(10.0, 10.0, 10.0), jitter=jitter, seed=seed, kinds=KUHN6,
                       perm_seed=perm_seed)
    fn = fields.isentropic_vortex(0.0)
    U0 = fn(fields.cell_points(mesh)) if point_ic else fields.cell_averages(mesh, fn, n_pts=quad_pts)
    dt = nominal_dt(mesh, "euler", U0, cfl, simplex=True)
    params = dict(pde="euler", scheme=scheme, flux=flux, gamma=fields.GAMMA)
    return Case("vortex3d", mesh, params, U0, dt, steps,
                exact=lambda t: fields.isentropic_vortex(t))


def shocks_3d(n=200, jitter=0.2, seed=31, split_seed=32, perm_seed=33, problem="sod",
              scheme="USR3", flux="rusanov", cfl=0.4, speed_margin=2.0):
    """3-D Euler Sod slab or spherical blast on a mixed hex/tet/prism mesh.

    The fixed time step uses ``speed_margin`` times the initial fastest wave:
    behind the shocks |u| + c grows (Sod: from 1.18 to about 2.2)."""
    mesh = periodic_3d(n, jitter=jitter, seed=seed, kinds=mixed_kinds(n, split_frac=0.3,
                       seed=split_seed), perm_seed=perm_seed)
    fn = fields.sod_slab() if problem == "sod" else fields.blast()
    U0 = fn(fields.cell_points(mesh))
    dt0 = nominal_dt(mesh, "euler", U0, cfl, simplex=True) / speed_margin
    t_end = 0.1 if problem == "sod" else 0.05
    steps, dt = _steps_to(t_end, dt0)
    params = dict(pde="euler", scheme=scheme, flux=flux, gamma=fields.GAMMA)
    return Case("shocks3d_" + problem, mesh, params, U0, dt, steps)


# reference state of the Taylor-Green workload at Mach 0.1 (rest, p0 = 1 / (gamma M^2))
TGV_REF = (1.0, 0.0, 0.0, 0.0, 1.0 / (1.4 * 0.01) / 0.4)


def taylor_green_3d(n=288, jitter=0.2, seed=41, perm_seed=42, scheme="USR5", flux="hllc",
                    steps=100, cfl=0.4, mach=0.1):
    """3-D Euler Taylor-Green vortex at Mach 0.1 in [0, 2 pi]^3 on jittered hexes."""
    L = 2 * np.pi
    mesh = periodic_3d(n, lengths=(L, L, L), jitter=jitter, seed=seed, kinds=HEX,
                       perm_seed=perm_seed)
    U0 = fields.taylor_green(mach)(fields.parent_hex_points(mesh))
    dt = nominal_dt(mesh, "euler", U0, cfl)
    params = dict(pde="euler", scheme=scheme, flux=flux, gamma=fields.GAMMA)
    return Case("taylor_green3d", mesh, params, U0, dt, steps)


def line_1d(n, L=1.0, widths=None, jitter=0.0, seed=0, dim=3):
    """A 1-D problem as an n x 2 (x 2) periodic slab; optional graded x widths."""
    coords = None
    if widths is not None:
        w = np.asarray(widths, dtype=np.float64)
        coords = np.concatenate([[0.0], np.cumsum(w)])
        coords *= L / coords[-1]
        coords[-1] = L
    if dim == 2:
        return periodic_2d(n, 2, lengths=(L, 1.0), jitter=jitter, seed=seed, xcoords=coords)
    return periodic_3d(n, 2, 2, lengths=(L, 1.0, 1.0), jitter=jitter, seed=seed,
                       coords=(coords, None, None))
