"""Pins of the oracle's gradient functions (CPU only).

  * the reflectance adjoint against central finite differences of the oracle forward (with the
    counters and the specular-sampling probabilities frozen the estimator is a polynomial in the
    reflectances, so central differences are exact up to rounding and an O(h^2) term);
  * the frozen-visibility estimator equals the forward at the reference design;
  * for a hinged plate the frozen-visibility estimator IS the flat-plate closed form at every
    angle, so its derivative matches the closed form's.
"""
import numpy as np
import pytest

import oracle
import srp_inputs as si
from oracle.design import apply_hinges

C = 299792458.0
PHI = 1361.0


def loss(res, gF, gT):
    return float((res.force * gF).sum() + (res.torque * gT).sum())


def test_rho_adjoint_matches_central_differences():
    m = si.box_wing()
    rs, rd = si.materials(m.n_tris, 1)
    rs = (0.05 + 0.8 * rs).astype(np.float32)  # both reflectances in [0.05, 0.45]
    rd = (0.05 + 0.8 * rd).astype(np.float32)
    ps = oracle.default_pspec(rs, rd)
    sun = si.fibonacci_dirs(8)
    rng = np.random.default_rng(0)
    gF = rng.standard_normal((8, 3))
    gT = rng.standard_normal((8, 3))
    kw = dict(nu=48, nv=48, bounces=3, seed=4, p_spec=ps)
    g_rs, g_rd = oracle.trace_adjoint_rho(m.verts, m.tris, rs, rd, sun, gF, gT, **kw)
    h = 1e-3
    for f in range(m.n_tris):
        for which, g in ((0, g_rs), (1, g_rd)):
            a = [rs.copy(), rd.copy()]
            b = [rs.copy(), rd.copy()]
            a[which][f] = np.float32(a[which][f] + h)
            b[which][f] = np.float32(b[which][f] - h)
            hp = float(a[which][f]) - float(b[which][f])
            Lp = loss(oracle.trace(m.verts, m.tris, a[0], a[1], sun, **kw), gF, gT)
            Lm = loss(oracle.trace(m.verts, m.tris, b[0], b[1], sun, **kw), gF, gT)
            fd = (Lp - Lm) / hp
            assert abs(fd - g[f]) <= 1e-6 * max(abs(fd), 1e-3 * np.abs(g).max()), (f, which, fd, g[f])
    # the bounces matter: some facets receive light from other facets
    res = oracle.trace(m.verts, m.tris, rs, rd, sun, records=True, **kw)
    assert (res.hit_prim[..., 1] >= 0).any()


def test_frozen_estimator_equals_forward_at_reference():
    m = si.meo_satellite(bus_n=6, cyl_sides=16, panel_n=4, dish_rings=8, dish_sectors=16, strut_sides=6)
    rs, rd = si.materials(m.n_tris, 2)
    ang = np.array([0.3, -0.2])
    V0 = apply_hinges(m.verts, m.vert_hinge, m.hinge_origin, m.hinge_axis, ang)
    sun = si.fibonacci_dirs(6)
    fr = oracle.frames(V0, sun, 40, 40)
    kw = dict(nu=40, nv=40, bounces=3, seed=9)
    ref = oracle.trace(V0, m.tris, rs, rd, sun, frames_in=fr, records=True, **kw)
    F, T = oracle.trace_frozen(V0, V0, m.tris, rs, rd, sun, ref.hit_prim, fr, **kw)
    assert np.allclose(F, ref.force, rtol=1e-10, atol=1e-10 * np.abs(ref.force).max())
    assert np.allclose(T, ref.torque, rtol=1e-10, atol=1e-10 * np.abs(ref.torque).max())


def hinged_plate():
    """1.2 x 0.8 plate in z = 0 (x in [-0.6, 0.6], y in [0.2, 1.0]) on a hinge along +x through the
    origin, facing +z."""
    v, t = si.quad_grid((-0.6, 0.2, 0.0), (1.2, 0, 0), (0, 0.8, 0), 1, 1)
    return si.Mesh(verts=v, tris=t.astype(np.int32), vert_hinge=np.zeros(len(v), np.int32),
                   hinge_origin=np.zeros((1, 3)), hinge_axis=np.array([[1.0, 0, 0]]), group=np.zeros(2, np.int32))


def plate_closed_form(theta, rs, rd, sun):
    n = np.array([0.0, -np.sin(theta), np.cos(theta)])  # normal after rotating by theta about +x
    s_hat = -sun
    c = float(s_hat @ -n)
    return PHI * 0.96 * c / C * ((1 - rs) * s_hat + 2 * (rs * c + rd / 3) * (-n))


@pytest.mark.parametrize("theta0", [0.0, 0.35])
def test_frozen_estimator_plate_hinge_closed_form(theta0):
    m = hinged_plate()
    rs = np.full(2, 0.3, np.float32)
    rd = np.full(2, 0.25, np.float32)
    sun = np.array([[0.0, 0.0, 1.0]])
    V0 = apply_hinges(m.verts, m.vert_hinge, m.hinge_origin, m.hinge_axis, [theta0])
    nu, nv = 60, 40
    fr = oracle.frames(V0, sun, nu, nv)
    kw = dict(nu=nu, nv=nv, bounces=1, jitter=False)
    ref = oracle.trace(V0, m.tris, rs, rd, sun, frames_in=fr, records=True, **kw)
    assert (ref.hit_prim[0, :, 0] >= 0).all()
    for dth in (0.0, 1e-3, -2e-2, 0.1):
        V = apply_hinges(m.verts, m.vert_hinge, m.hinge_origin, m.hinge_axis, [theta0 + dth])
        F, _ = oracle.trace_frozen(V, V0, m.tris, rs, rd, sun, ref.hit_prim, fr, **kw)
        cf = plate_closed_form(theta0 + dth, float(rs[0]), float(rd[0]), sun[0])
        assert np.allclose(F[0], cf, rtol=1e-10, atol=1e-12 * np.abs(cf).max()), dth
