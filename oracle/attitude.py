"""Oracle: 13-D orbit and attitude integration -- TEST INFRASTRUCTURE ONLY.

The paper's state equation (Sec. 3.4.1, Eq. ODE) for the state z = (r, v, q, w):
  dr/dt = v,
  dv/dt = m^-1 R(q) F(s_body, design) + o(r),      o(r) = -mu r / |r|^3 (point-mass gravity),
  dq/dt = 1/2 Omega(w) q,
  dw/dt = I^-1 (tau(s_body, design) - w x (I w)),
with s_body = R(q)^T s the Sun direction in the body frame, integrated with the classic RK4 method
in double precision (Sec. 3.4.1, "Implementation").  The cylinder eclipse model the paper names
(Montenbruck & Gill) switches the radiation off where the spacecraft is behind the Earth and
inside the cylinder of radius R_E along the Sun direction: nu = 0 when r . s < 0 and
|r - (r . s) s| < R_E, else 1; force and torque are multiplied by nu.

Conventions (readings; the paper does not fix them):
  * q = (q0, q1, q2, q3), scalar first; R(q) rotates body vectors to inertial ones; the state
    quaternion is not renormalised between steps and R is formed from q / |q|;
  * w is the angular velocity in the body frame, so dq/dt = 1/2 q (x) (0, w) (quaternion product);
  * s is the unit vector toward the Sun, fixed in the inertial frame.

The force-and-torque model is a callback model(s_body [B][3], design [B][k]) -> (F [B][3],
tau [B][3]) in the body frame; `mlp_model` wraps the oracle network (oracle.mlp, BF16 emulation)
the way the GPU path uses it: input [s_body as float32, design], outputs scaled by force_scale
(first three) and torque_scale (next three).
"""
from __future__ import annotations

import numpy as np

from . import mlp as _mlp


def rot(q):
    """R(q / |q|) for q [..., 4] scalar first: body -> inertial."""
    q = np.asarray(q, dtype=np.float64)
    q = q / np.sqrt((q * q).sum(-1, keepdims=True))
    q0, q1, q2, q3 = q[..., 0], q[..., 1], q[..., 2], q[..., 3]
    R = np.empty(q.shape[:-1] + (3, 3))
    R[..., 0, 0] = 1 - 2 * (q2 * q2 + q3 * q3)
    R[..., 0, 1] = 2 * (q1 * q2 - q0 * q3)
    R[..., 0, 2] = 2 * (q1 * q3 + q0 * q2)
    R[..., 1, 0] = 2 * (q1 * q2 + q0 * q3)
    R[..., 1, 1] = 1 - 2 * (q1 * q1 + q3 * q3)
    R[..., 1, 2] = 2 * (q2 * q3 - q0 * q1)
    R[..., 2, 0] = 2 * (q1 * q3 - q0 * q2)
    R[..., 2, 1] = 2 * (q2 * q3 + q0 * q1)
    R[..., 2, 2] = 1 - 2 * (q1 * q1 + q2 * q2)
    return R


def quat_mul(a, b):
    """Hamilton product a (x) b, scalar first."""
    a0, av = a[..., :1], a[..., 1:]
    b0, bv = b[..., :1], b[..., 1:]
    return np.concatenate([a0 * b0 - (av * bv).sum(-1, keepdims=True), a0 * bv + b0 * av + np.cross(av, bv)], -1)


def shadow(r, sun, earth_radius):
    """Cylinder eclipse factor nu [B] (1 lit, 0 in shadow); earth_radius 0 disables it."""
    if earth_radius <= 0:
        return np.ones(r.shape[:-1])
    along = r @ sun
    perp = r - along[..., None] * sun
    dark = (along < 0) & ((perp * perp).sum(-1) < earth_radius * earth_radius)
    return np.where(dark, 0.0, 1.0)


def deriv(z, design, model, mu, mass, inertia, inertia_inv, sun, earth_radius):
    r, v, q, w = z[:, 0:3], z[:, 3:6], z[:, 6:10], z[:, 10:13]
    R = rot(q)
    s_body = np.einsum("bji,j->bi", R, sun)  # R^T s
    F, tau = model(s_body, design)
    nu = shadow(r, sun, earth_radius)[:, None]
    rr = np.sqrt((r * r).sum(-1, keepdims=True))
    acc = -mu * r / rr ** 3 + nu * np.einsum("bij,bj->bi", R, F) / mass
    wq = np.concatenate([np.zeros_like(w[:, :1]), w], -1)
    dq = 0.5 * quat_mul(q, wq)
    Iw = w @ inertia.T
    dw = (nu * tau - np.cross(w, Iw)) @ inertia_inv.T
    return np.concatenate([v, acc, dq, dw], -1)


def rk4(z0, design, model, *, mu, mass, inertia, sun, dt, n_steps, earth_radius=0.0, keep=False, steps_per_design=0):
    """z0 [B][13], design [B][k]; returns z_N [B][13] (and all states [n+1][B][13] if keep).
    With steps_per_design = L > 0 the design changes over time: design [S][B][k], and step n (all
    four of its stages) uses row min(n // L, S - 1)."""
    z = np.array(z0, dtype=np.float64, copy=True).reshape(-1, 13)
    B = z.shape[0]
    sched = np.asarray(design, dtype=np.float64)
    sched = sched.reshape(-1, B, sched.shape[-1]) if steps_per_design > 0 else sched.reshape(1, B, -1)
    inertia = np.asarray(inertia, dtype=np.float64).reshape(3, 3)
    inertia_inv = np.linalg.inv(inertia)
    sun = np.asarray(sun, dtype=np.float64)
    states = [z.copy()] if keep else None
    for n in range(n_steps):
        seg = min(n // steps_per_design, len(sched) - 1) if steps_per_design > 0 else 0
        args = (sched[seg], model, mu, mass, inertia, inertia_inv, sun, earth_radius)
        k1 = deriv(z, *args)
        k2 = deriv(z + 0.5 * dt * k1, *args)
        k3 = deriv(z + 0.5 * dt * k2, *args)
        k4 = deriv(z + dt * k3, *args)
        z = z + dt / 6.0 * (k1 + 2.0 * k2 + 2.0 * k3 + k4)
        if keep:
            states.append(z.copy())
    return (z, np.array(states)) if keep else z


def mlp_model(layers, force_scale, torque_scale, emulate=True):
    """The network as force-and-torque model: x = [float32(s_body), design]."""
    def model(s_body, design):
        x = np.concatenate([_mlp.f32(s_body), np.asarray(design, dtype=np.float64)], -1)
        y, _ = _mlp.forward(layers, x, emulate=emulate)
        return force_scale * y[:, 0:3], torque_scale * y[:, 3:6]
    return model
