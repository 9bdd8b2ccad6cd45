"""The 1-D radial Euler solver that scores the spherical blast.

Pinned to what fixes it independently of itself: in planar geometry it
converges to the exact Riemann solution of Sod's problem; in spherical
geometry it conserves mass and energy to round-off (no wave reaches the
outer shell by t = 0.05) and keeps a gas at rest and uniform pressure at
rest exactly (the pressure force on a shell's curved sides balances the
face pressures)."""
import numpy as np

from synth import fields


def _sod(r):
    left = r < 0.5
    return np.where(left, 1.0, 0.125), np.zeros_like(r), np.where(left, 1.0, 0.1)


def test_planar_sod_converges_to_exact():
    errs = []
    for n in (400, 800):
        rc, rho, u, p = fields.radial_euler(_sod, 1.0, n, 0.2, alpha=0)
        ex = fields.riemann_exact((1.0, 0.0, 1.0), (0.125, 0.0, 0.1), (rc - 0.5) / 0.2)
        errs.append(np.mean(np.abs(rho - ex[0])))
        assert np.mean(np.abs(p - ex[2])) < 3e-3
    assert errs[0] < 3e-3 and errs[1] < 0.7 * errs[0], errs


def test_spherical_blast_conserves_mass_and_energy():
    n, gamma = 400, 1.4
    rc, rho, u, p = fields.radial_euler(
        lambda r: (np.ones_like(r), np.zeros_like(r), np.where(r < 0.2, 10.0, 0.1)), 0.5, n, 0.05)
    rf = np.arange(n + 1) * (0.5 / n)
    V = (rf[1:] ** 3 - rf[:-1] ** 3) / 3.0
    E0 = np.sum(V * np.where(rc < 0.2, 10.0, 0.1)) / (gamma - 1.0)
    assert abs(np.sum(V * rho) - 0.5 ** 3 / 3.0) < 1e-13
    assert abs(np.sum(V * (p / (gamma - 1.0) + 0.5 * rho * u * u)) - E0) < 1e-13 * E0
    # an outgoing shock near r = 0.3, the outer shells undisturbed
    shock = rc[np.argmax(np.abs(np.diff(rho)))]
    assert 0.27 < shock < 0.33
    assert np.all(rho[rc > 0.4] == 1.0) and np.all(p[rc > 0.4] == 0.1)


def test_rest_state_stays_at_rest():
    rc, rho, u, p = fields.radial_euler(
        lambda r: (np.ones_like(r), np.zeros_like(r), np.full_like(r, 0.7)), 0.5, 100, 0.02)
    assert np.max(np.abs(u)) < 1e-14 and np.max(np.abs(p - 0.7)) < 1e-13 and np.max(np.abs(rho - 1)) < 1e-13
