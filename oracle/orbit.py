"""Oracle: orbit integration -- TEST INFRASTRUCTURE ONLY.

Translational part of the paper's state equation (Sec. 3.4.1, Eq. ODE): dr/dt = v,
dv/dt = m^-1 T^T F + o(z), integrated with the classic fourth-order Runge-Kutta method in double
precision (Sec. 3.4.1, "Implementation"), o = point-mass gravity.  The force table holds the
body-frame force at every distinct stage time t_k = k h / 2 and R_k rotates it to inertial axes.

The gradient of a loss of the final state with respect to every entry of the force table is
obtained by complex-step differentiation of this same integrator (Squire & Trapp 1998): one complex
perturbation i*eps per table entry, all propagated together, dL/dF = Im(L)/eps, exact to rounding
because RK4 and the loss are analytic (|r| is written as sqrt(r . r)).
"""
from __future__ import annotations

import numpy as np


def accel(r, mu):
    rr = np.sqrt((r * r).sum(-1, keepdims=True))
    return -mu * r / rr ** 3


def rk4(z0, mu, mass, dt, n_steps, F, R, keep=False):
    """F [2n+1][...][3] body-frame forces (extra middle axes broadcast: batched trajectories),
    R [2n+1][3][3]; z0 [..., 6].  Returns the final state (and all states if keep)."""
    z = np.array(z0, dtype=np.result_type(z0, F, np.float64), copy=True)
    states = [z.copy()] if keep else None

    def f(z, k):
        a = accel(z[..., :3], mu) + np.einsum("ij,...j->...i", R[k], F[k]) / mass
        return np.concatenate([z[..., 3:], a], -1)

    for n in range(n_steps):
        k1 = f(z, 2 * n)
        k2 = f(z + 0.5 * dt * k1, 2 * n + 1)
        k3 = f(z + 0.5 * dt * k2, 2 * n + 1)
        k4 = f(z + dt * k3, 2 * n + 2)
        z = z + dt / 6.0 * (k1 + 2.0 * k2 + 2.0 * k3 + k4)
        if keep:
            states.append(z.copy())
    return (z, np.array(states)) if keep else z


def final_position_loss(z, r_target):
    d = z[..., :3] - r_target
    return (d * d).sum(-1)


def grad_forces(z0, mu, mass, dt, n_steps, F, R, r_target, eps=1e-30, return_final=False):
    """dL/dF [2n+1][3] for L = |r_N - r_target|^2 by complex-step differentiation (and, with
    return_final, the final state of the same complex-arithmetic run, real part)."""
    F = np.asarray(F, dtype=np.float64)
    S = F.shape[0]
    m = 3 * S
    Fc = np.broadcast_to(F[:, None, :], (S, m, 3)).astype(np.complex128).copy()
    idx = np.arange(m)
    Fc[idx // 3, idx, idx % 3] += 1j * eps
    zc = np.broadcast_to(np.asarray(z0, dtype=np.complex128), (m, 6)).copy()
    zN = rk4(zc, mu, mass, dt, n_steps, Fc, R)
    L = final_position_loss(zN, r_target)
    g = (L.imag / eps).reshape(S, 3)
    return (g, zN[0].real.copy()) if return_final else g
