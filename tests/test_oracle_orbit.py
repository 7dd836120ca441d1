"""Pins of the orbit oracle (CPU only): Kepler invariants, fourth-order convergence, period, and the
complex-step gradient against central finite differences."""
import numpy as np

import srp_inputs as si
from oracle import orbit


def kepler_run(dt, n_steps):
    sc = si.meo_orbit(n_steps=n_steps, dt=dt)
    F = np.zeros((2 * n_steps + 1, 3))
    z, zs = orbit.rk4(sc.z0, sc.mu, sc.mass, dt, n_steps, F, sc.R, keep=True)
    return sc, zs


def test_circular_orbit_invariants_and_period():
    sc, zs = kepler_run(60.0, 720)
    r = np.linalg.norm(zs[:, :3], axis=1)
    v = np.linalg.norm(zs[:, 3:], axis=1)
    E = 0.5 * v ** 2 - sc.mu / r
    assert np.abs(r / r[0] - 1).max() < 1e-9
    assert np.abs(E / E[0] - 1).max() < 1e-9
    period = 2 * np.pi * np.sqrt(26_560_000.0 ** 3 / sc.mu)
    assert abs(period - 43077.8) < 0.5
    # after exactly one period (60 s steps do not divide it: compare with the analytic position)
    n = 718
    t = n * 60.0
    u = 2 * np.pi * t / period
    i = np.deg2rad(55.0)
    r_ref = 26_560_000.0 * np.array([np.cos(u), np.sin(u) * np.cos(i), np.sin(u) * np.sin(i)])
    assert np.linalg.norm(zs[n, :3] - r_ref) < 0.1  # RK4 truncation at 60 s steps: ~2 cm per orbit


def test_fourth_order_convergence():
    T = 36000.0
    errs = []
    for dt in (240.0, 120.0, 60.0):
        n = int(T / dt)
        sc, zs = kepler_run(dt, n)
        period = 2 * np.pi * np.sqrt(26_560_000.0 ** 3 / sc.mu)
        u = 2 * np.pi * T / period
        i = np.deg2rad(55.0)
        r_ref = 26_560_000.0 * np.array([np.cos(u), np.sin(u) * np.cos(i), np.sin(u) * np.sin(i)])
        errs.append(np.linalg.norm(zs[-1, :3] - r_ref))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 12 < r1 < 20 and 12 < r2 < 20, errs


def test_complex_step_gradient_vs_central_differences():
    """With negligible gravity the final position is linear in the forces and the loss quadratic, so
    central differences are exact up to rounding (tight); with gravity they carry O(h^2) and the
    rounding of the 26,560 km position (looser)."""
    n = 40
    sc = si.meo_orbit(n_steps=n, dt=60.0)
    rng = np.random.default_rng(0)
    F = 1e-4 * rng.standard_normal((2 * n + 1, 3))
    for mu, h, tol in ((1.0, 1e-2, 1e-8), (sc.mu, 1e-3, 3e-6)):
        r_t = orbit.rk4(sc.z0, mu, sc.mass, sc.dt, n, F * 1.3, sc.R)[:3] + 10.0
        g = orbit.grad_forces(sc.z0, mu, sc.mass, sc.dt, n, F, sc.R, r_t)
        for (k, c) in [(0, 0), (5, 1), (41, 2), (2 * n - 1, 1), (2 * n, 0)]:
            Fp = F.copy()
            Fp[k, c] += h
            Fm = F.copy()
            Fm[k, c] -= h
            Lp = orbit.final_position_loss(orbit.rk4(sc.z0, mu, sc.mass, sc.dt, n, Fp, sc.R), r_t)
            Lm = orbit.final_position_loss(orbit.rk4(sc.z0, mu, sc.mass, sc.dt, n, Fm, sc.R), r_t)
            fd = (Lp - Lm) / (2 * h)
            assert abs(fd - g[k, c]) <= tol * abs(g).max(), (mu, k, c, fd, g[k, c])
        # the force of the last stage time enters only the last velocity update, never a position
        assert not g[2 * n].any() and g[2 * n - 1].all()
