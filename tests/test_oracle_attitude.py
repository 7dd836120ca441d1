"""Pins of the oracle's 13-D integrator (paper Sec. 3.4.1, Eq. ODE: position, velocity, quaternion,
angular velocity; RK4 in FP64; cylinder eclipse), independent of the GPU path:

  * rotation: R(q) for an axis-angle quaternion is the right-handed rotation; R(a (x) b) = R(a) R(b);
  * torque-free axisymmetric body: the body-frame rates follow the closed-form precession, and the
    error falls ~16x when the step halves (fourth order);
  * torque-free asymmetric body (full inertia tensor): inertial angular momentum R(q) I w and
    kinetic energy are conserved to the integrator's order -- a wrong sign of the quaternion rate
    or a transposed rotation breaks this at O(1);
  * constant body torque from rest about a principal axis: w = tau t / I, q = q0 (x) rotation by
    tau t^2 / (2 I) about that axis;
  * no rotation, no torque, constant body force: the translational part equals the pinned 6-D
    integrator (oracle/orbit.py) with the constant attitude;
  * a force along the body-frame Sun direction acts the same on a spinning and a still body
    (s_body = R^T s and R F cancel);
  * cylinder eclipse: a straight pass behind the Earth loses the radiation for exactly the time
    inside the shadow cylinder (to one step), a pass on the Sun side never does.
"""
import numpy as np
import pytest

from oracle import attitude as att
from oracle import orbit as orb
from oracle import mlp as omlp

MU = 3.986004418e14
RE = 6378137.0


def axis_quat(axis, phi):
    axis = np.asarray(axis, dtype=np.float64) / np.linalg.norm(axis)
    return np.concatenate([[np.cos(phi / 2)], np.sin(phi / 2) * axis])


def zero_model(s, d):
    return np.zeros_like(s), np.zeros_like(s)


def state(r, v, q, w):
    return np.concatenate([r, v, q, w])[None]


def test_rotation_conventions():
    R = att.rot(axis_quat([0, 0, 1], 0.3))
    assert np.allclose(R @ [1, 0, 0], [np.cos(0.3), np.sin(0.3), 0], atol=1e-15)
    R = att.rot(axis_quat([1, 0, 0], 0.4))
    assert np.allclose(R @ [0, 1, 0], [0, np.cos(0.4), np.sin(0.4)], atol=1e-15)
    rng = np.random.default_rng(1)
    a, b = rng.normal(size=4), rng.normal(size=4)
    a /= np.linalg.norm(a)
    b /= np.linalg.norm(b)
    assert np.allclose(att.rot(att.quat_mul(a, b)), att.rot(a) @ att.rot(b), atol=1e-14)
    # non-unit quaternions give the rotation of their direction
    assert np.allclose(att.rot(3.0 * a), att.rot(a), atol=1e-15)


def precession_error(dt, T=600.0):
    I1, I3 = 100.0, 160.0
    w0 = np.array([0.03, -0.01, 0.05])
    n = int(round(T / dt))
    z0 = state([4e7, 0, 0], [0, 3157.0, 0], [1, 0, 0, 0], w0)
    z = att.rk4(z0, np.zeros((1, 0)), zero_model, mu=MU, mass=500.0, inertia=np.diag([I1, I1, I3]),
                sun=np.array([1.0, 0, 0]), dt=dt, n_steps=n)
    lam = (I3 - I1) / I1 * w0[2]
    c = (w0[0] + 1j * w0[1]) * np.exp(1j * lam * T)
    ref = np.array([c.real, c.imag, w0[2]])
    return np.abs(z[0, 10:13] - ref).max()


def test_axisymmetric_precession_closed_form_and_order():
    e1, e2, e3 = precession_error(10.0), precession_error(5.0), precession_error(1.25)
    assert e3 < 1e-8  # |w| ~ 0.06 rad/s, precession 0.03 rad/s
    assert 14 < e1 / e2 < 19


def invariants(z, I):
    R = att.rot(z[:, 6:10])
    w = z[:, 10:13]
    H = np.einsum("bij,bj->bi", R, w @ I.T)
    T = 0.5 * (w * (w @ I.T)).sum(-1)
    return H, T


def drift(dt, I, w0, q0, T=900.0):
    z0 = state([3e7, 1e6, 0], [0, 3600.0, 200.0], q0, w0)
    n = int(round(T / dt))
    zN = att.rk4(z0, np.zeros((1, 0)), zero_model, mu=MU, mass=800.0, inertia=I, sun=np.array([0, 1.0, 0]),
                 dt=dt, n_steps=n)
    H0, T0 = invariants(z0, I)
    H1, T1 = invariants(zN, I)
    return np.linalg.norm(H1 - H0) / np.linalg.norm(H0), abs(T1 - T0)[0] / T0[0]


def test_asymmetric_body_conserves_inertial_momentum_and_energy():
    I = np.array([[120.0, 4.0, -2.0], [4.0, 210.0, 6.0], [-2.0, 6.0, 310.0]])
    w0 = np.array([0.04, 0.03, -0.02])
    q0 = axis_quat([0.3, -0.5, 0.8], 1.1)
    h1, t1 = drift(3.0, I, w0, q0)
    h2, t2 = drift(1.5, I, w0, q0)
    h3, t3 = drift(0.75, I, w0, q0)
    assert h3 < 1e-8 and t3 < 1e-9  # |w| ~ 0.05 rad/s over 900 s
    assert 12 < h1 / h2 < 20 and 12 < h2 / h3 < 20  # fourth order (energy falls faster still)
    assert t1 / t2 > 12 and t2 / t3 > 12


def spin_up(dt, T=400.0):
    Ia, tau = 250.0, 0.02
    I = np.diag([180.0, Ia, 320.0])
    q0 = axis_quat([1, 2, 3], 0.7)
    z0 = state([5e7, 0, 0], [0, 2800.0, 0], q0, [0, 0, 0])

    def model(s, d):
        t = np.zeros_like(s)
        t[:, 1] = tau
        return np.zeros_like(s), t

    z = att.rk4(z0, np.zeros((1, 0)), model, mu=MU, mass=500.0, inertia=I, sun=np.array([1.0, 0, 0]), dt=dt,
                n_steps=int(round(T / dt)))
    w_err = np.abs(z[0, 10:13] - [0, tau * T / Ia, 0]).max()
    q_ref = att.quat_mul(q0, axis_quat([0, 1, 0], tau * T * T / (2 * Ia)))
    return w_err, np.abs(z[0, 6:10] - q_ref).max()


def test_constant_torque_spin_up():
    (w1, q1), (w2, q2) = spin_up(2.0), spin_up(1.0)
    assert w1 < 1e-16 and w2 < 1e-16  # w is linear in t: RK4 is exact
    assert q2 < 1e-9  # 6.4 rad turned, final rate 0.032 rad/s
    assert 12 < q1 / q2 < 20


def test_translation_reduces_to_pinned_orbit_integrator():
    q0 = axis_quat([0.2, 0.9, -0.4], 2.2)
    F_body = np.array([3e-5, -1e-5, 2e-5])
    r0, v0 = np.array([2.656e7, 0, 0]), np.array([0, 3873.96, 0])
    n, dt = 200, 60.0
    z = att.rk4(state(r0, v0, q0, [0, 0, 0]), np.zeros((1, 0)),
                lambda s, d: (np.broadcast_to(F_body, s.shape).copy(), np.zeros_like(s)), mu=MU, mass=1000.0,
                inertia=np.diag([1.0, 2.0, 3.0]), sun=np.array([0, 0, 1.0]), dt=dt, n_steps=n)
    F = np.broadcast_to(F_body, (2 * n + 1, 3))
    R = np.broadcast_to(att.rot(q0), (2 * n + 1, 3, 3))
    ref = orb.rk4(np.concatenate([r0, v0]), MU, 1000.0, dt, n, F, R)
    assert np.allclose(z[0, :6], ref, rtol=1e-13, atol=0)
    assert np.array_equal(z[0, 6:10], q0)


def test_sun_direction_force_is_attitude_independent():
    sun = np.array([0.6, 0.0, 0.8])
    r0, v0 = np.array([0, 2.656e7, 0]), np.array([-3873.96, 0, 0])

    def model(s, d):
        return 4e-5 * s, np.zeros_like(s)

    kw = dict(mu=MU, mass=1000.0, inertia=np.diag([300.0, 200.0, 100.0]), sun=sun, dt=30.0, n_steps=240)
    still = att.rk4(state(r0, v0, [1, 0, 0, 0], [0, 0, 0]), np.zeros((1, 0)), model, **kw)
    spin = att.rk4(state(r0, v0, axis_quat([1, -1, 2], 0.5), [0.02, -0.05, 0.03]), np.zeros((1, 0)), model, **kw)
    free = att.rk4(state(r0, v0, [1, 0, 0, 0], [0, 0, 0]), np.zeros((1, 0)), zero_model, **kw)
    effect = np.linalg.norm(still[0, :3] - free[0, :3])
    assert effect > 0.5  # metres of displacement from the radiation force
    assert np.linalg.norm(spin[0, :3] - still[0, :3]) <= 1e-8 * effect


@pytest.mark.parametrize("side", [-1.0, 1.0])
def test_cylinder_eclipse_straight_pass(side):
    a, v, dt = 1e-6, 7000.0, 10.0
    T = 6 * RE / v
    n = int(np.ceil(T / dt))
    r0 = np.array([side * 2 * RE, -3 * RE, 0.0])

    def model(s, d):
        return -a * 1000.0 * s, np.zeros_like(s)  # a push away from the Sun

    z = att.rk4(state(r0, [0, v, 0], [1, 0, 0, 0], [0, 0, 0]), np.zeros((1, 0)), model, mu=1e-30, mass=1000.0,
                inertia=np.eye(3), sun=np.array([1.0, 0, 0]), dt=dt, n_steps=n, earth_radius=RE)
    t_end = n * dt
    lit = t_end - (2 * RE / v if side < 0 else 0.0)
    assert abs(-z[0, 3] - a * lit) <= 2 * a * dt
    assert abs(z[0, 4] - v) < 1e-9


def test_mlp_model_inputs_and_scales():
    layers = omlp.unpack(omlp.init_params(5, 16, 2, 6, seed=3), 5, 16, 2, 6)
    s = np.array([[0.6, 0.0, 0.8], [0.0, -1.0, 0.0]])
    d = np.array([[0.25, -0.5], [1.0, 0.0]])
    F, tau = att.mlp_model(layers, 2.0, 3.0)(s, d)
    y, _ = omlp.forward(layers, np.concatenate([s, d], 1), emulate=True)
    assert np.array_equal(F, 2.0 * y[:, :3]) and np.array_equal(tau, 3.0 * y[:, 3:])


def test_design_schedule_segments():
    """A schedule of identical rows is the constant design; a schedule switches at step boundaries:
    running its first segment alone and restarting from that state with the second gives the same
    end state."""
    layers = omlp.unpack(omlp.init_params(5, 16, 2, 6, seed=4), 5, 16, 2, 6)
    model = att.mlp_model(layers, 3e-5, 1e-5)
    z0 = state([2.656e7, 0, 0], [0, 3873.96, 0], axis_quat([1, 2, 2], 0.4), [0.01, -0.02, 0.005])
    kw = dict(mu=MU, mass=1000.0, inertia=np.diag([300.0, 200.0, 100.0]), sun=np.array([0.6, 0.0, 0.8]), dt=30.0)
    d1, d2 = np.array([[0.3, -0.7]]), np.array([[-0.9, 0.2]])
    const = att.rk4(z0, d1, model, n_steps=20, **kw)
    same = att.rk4(z0, np.stack([d1, d1]), model, n_steps=20, steps_per_design=10, **kw)
    assert np.array_equal(const, same)
    sched = att.rk4(z0, np.stack([d1, d2]), model, n_steps=20, steps_per_design=10, **kw)
    half = att.rk4(z0, d1, model, n_steps=10, **kw)
    rest = att.rk4(half, d2, model, n_steps=10, **kw)
    assert np.array_equal(sched, rest)
    assert not np.array_equal(sched, const)
    # past the last row the schedule holds it
    longer = att.rk4(z0, np.stack([d1, d2]), model, n_steps=25, steps_per_design=10, **kw)
    assert np.array_equal(longer, att.rk4(rest, d2, model, n_steps=5, **kw))
