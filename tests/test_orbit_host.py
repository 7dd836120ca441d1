"""Host orbit integration of libsrp (srp_orbit_rk4 / srp_orbit_rk4_adjoint, CPU FP64) against the
orbit oracle: trajectory and the complex-step gradient with respect to every stage-time force."""
import os

import numpy as np
import pytest

import srp_inputs as si
from oracle import orbit

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if not os.path.exists(os.path.join(ROOT, "paper_2602_10712_amd", "libsrp.so")):
    pytest.skip("libsrp.so not built", allow_module_level=True)

from paper_2602_10712_amd import _binding as B  # noqa: E402


@pytest.mark.parametrize("n_steps,ckpt", [(1440, 60), (97, 10), (5, 7), (1, 1)])
def test_rk4_and_adjoint_match_oracle(n_steps, ckpt):
    sc = si.meo_orbit(n_steps=n_steps, dt=60.0)
    rng = np.random.default_rng(n_steps)
    F = 2e-5 * rng.standard_normal((2 * n_steps + 1, 3)) + np.array([1e-5, -2e-5, 3e-5])
    zf, zs = B.srp_orbit_rk4(sc.z0, sc.mu, sc.mass, sc.dt, n_steps, F, sc.R, keep_states=True)
    zf_ref, zs_ref = orbit.rk4(sc.z0, sc.mu, sc.mass, sc.dt, n_steps, F, sc.R, keep=True)
    assert np.abs(zs - zs_ref)[:, :3].max() < 1e-6 and np.abs(zs - zs_ref)[:, 3:].max() < 1e-9
    r_t = zf_ref[:3] + np.array([120.0, -40.0, 15.0])
    if n_steps <= 97:
        ref, z_cs = orbit.grad_forces(sc.z0, sc.mu, sc.mass, sc.dt, n_steps, F, sc.R, r_t, return_final=True)
        rows = np.arange(2 * n_steps + 1)
    else:
        # full day: complex step on a sample of stage times (memory)
        rows = np.array([0, 1, 2, 777, 1500, 2879, 2880])
        ref = np.zeros((len(rows), 3))
        for q, k in enumerate(rows):
            for c in range(3):
                Fc = F.astype(np.complex128)
                Fc[k, c] += 1e-30j
                z = orbit.rk4(sc.z0.astype(np.complex128), sc.mu, sc.mass, sc.dt, n_steps, Fc, sc.R)
                ref[q, c] = orbit.final_position_loss(z, r_t).imag / 1e-30
                z_cs = z.real
    # both sides differentiate L = |r_N - r_t|^2 at the same final state (the seed is an input)
    g_final = np.concatenate([2 * (z_cs[:3] - r_t), np.zeros(3)])
    gF, gz0 = B.srp_orbit_rk4_adjoint(sc.z0, sc.mu, sc.mass, sc.dt, n_steps, F, sc.R, g_final, ckpt)
    assert np.abs(gF[rows] - ref).max() <= 1e-10 * np.abs(gF).max()
    # the gradient with respect to the initial state: central differences in position
    h = 1e-2
    zp = sc.z0.copy()
    zp[0] += h
    zm = sc.z0.copy()
    zm[0] -= h
    Lp = orbit.final_position_loss(orbit.rk4(zp, sc.mu, sc.mass, sc.dt, n_steps, F, sc.R), r_t)
    Lm = orbit.final_position_loss(orbit.rk4(zm, sc.mu, sc.mass, sc.dt, n_steps, F, sc.R), r_t)
    assert abs((Lp - Lm) / (2 * h) - gz0[0]) <= 1e-5 * max(abs(gz0[0]), 1.0)


def test_orbit_invalid_arguments():
    sc = si.meo_orbit(n_steps=2)
    F = np.zeros((5, 3))
    with pytest.raises(B.SRPError):
        B.srp_orbit_rk4(np.zeros(6), sc.mu, sc.mass, sc.dt, 2, F, sc.R)
    with pytest.raises(B.SRPError):
        B.srp_orbit_rk4(sc.z0, sc.mu, -1.0, sc.dt, 2, F, sc.R)
    with pytest.raises(B.SRPError):
        B.srp_orbit_rk4_adjoint(sc.z0, sc.mu, sc.mass, sc.dt, 2, F, sc.R, np.zeros(6), 0)
