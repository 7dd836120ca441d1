"""Pins of the Phong lobes of the oracle's surface-sampling estimator (CPU only).

The materials follow the modified Phong BRDF rho_d/pi + rho_s (m + 2)/(2 pi) ((r.o)+)^m about the
mirror direction r of the arriving light (Lafortune and Willems 1994); a specular event samples the
lobe (BRDF importance sampling) or, with the plain-MC option, the hemisphere.  Every pin compares
the Monte Carlo estimate with a value computed here without it, within 5 standard errors:

  * a plate lit at normal incidence: the lobe's reflected momentum per unit incident momentum is
    rho_s (m + 2)/(m + 3) along the normal (closed form), so the force is
    -(Phi A / c)(1 + 2 rho_d / 3 + rho_s (m + 2)/(m + 3)) n; m infinite is the mirror's 1;
  * a plate lit obliquely: the lobe is cut by the horizon; its momentum comes from a 2-D quadrature
    of the BRDF here (scipy), both sampling options;
  * glossy sunlight gathered by next-event estimation: a black plate facing a sunlit Phong plate
    receives the momentum of the lobe's light, a 4-D quadrature over the two plates;
  * a glossy continuation: sunlit Lambertian plate -> unlit Phong plate -> black plate, a 6-D
    quadrature over the three plates (plus the direct Lambertian light, 4-D).
"""
import numpy as np
import pytest
from scipy import integrate

import oracle
import srp_inputs as si

PHI, C = 1361.0, 299792458.0


def _square(center, normal, size, up=(0.0, 0.0, 1.0), n=1):
    """A one-sided square facing `normal` (two triangles per cell)."""
    normal = np.asarray(normal, float) / np.linalg.norm(normal)
    up = np.asarray(up, float)
    if abs(up @ normal) > 0.9:
        up = np.array([1.0, 0.0, 0.0])
    a = np.cross(up, normal)
    a /= np.linalg.norm(a)
    b = np.cross(normal, a)
    v, t = si.quad_grid(np.asarray(center) - 0.5 * size * (a + b), size * a, size * b, n, n)
    # quad_grid faces eu x ev = a x b = normal
    return v, t


def _mesh(parts):
    V, T, owner = [], [], []
    off = 0
    for k, (v, t) in enumerate(parts):
        V.append(v)
        T.append(t + off)
        owner += [k] * len(t)
        off += len(v)
    return np.concatenate(V), np.concatenate(T).astype(np.int32), np.array(owner)


def _grid_points(center, normal, size, k):
    """Midpoints of a k x k grid on the square (same frame as _square) and the cell area."""
    normal = np.asarray(normal, float) / np.linalg.norm(normal)
    up = np.array([0.0, 0.0, 1.0])
    if abs(up @ normal) > 0.9:
        up = np.array([1.0, 0.0, 0.0])
    a = np.cross(up, normal)
    a /= np.linalg.norm(a)
    b = np.cross(normal, a)
    s = (np.arange(k) + 0.5) / k - 0.5
    S, Tt = np.meshgrid(s, s, indexing="ij")
    P = np.asarray(center) + size * (S.ravel()[:, None] * a + Tt.ravel()[:, None] * b)
    return P, normal, (size / k) ** 2


def _lobe_momentum(theta_i, m, rho_s):
    """Reflected momentum per unit incident momentum of the Phong lobe for light arriving at angle
    theta_i from the normal z (propagation p = (sin, 0, -cos)): rho_s (m+2)/(2 pi) int o ((r.o)+)^m
    cos(theta_o) d omega over the upper hemisphere, r = (sin, 0, cos)."""
    r = np.array([np.sin(theta_i), 0.0, np.cos(theta_i)])

    def comp(c):
        def f(ph, th):
            o = np.array([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)])
            return o[c] * max(0.0, r @ o) ** m * np.cos(th) * np.sin(th)
        return integrate.dblquad(f, 0.0, np.pi / 2, 0.0, 2 * np.pi, epsabs=1e-11, epsrel=1e-10)[0]
    return rho_s * (m + 2) / (2 * np.pi) * np.array([comp(0), comp(1), comp(2)])


def _estimate(V, T, rs, rd, sun, phong, n, bounces, sampling=0, seed=3):
    r = oracle.surface_estimate(V, T, rs, rd, sun[None], n_samples=n, bounces=bounces, seed=seed, records=True,
                                sampling=sampling, phong=phong)
    return r


def _mean_se(sf, mask, n):
    x = np.where(mask[:, None], sf, 0.0)
    return x.sum(0) / n, x.std(0) / np.sqrt(n)


@pytest.mark.parametrize("m", [1.0, 8.0, 60.0, np.inf])
def test_plate_normal_incidence_closed_form(m):
    v, t = si.quad_grid((-0.5, -0.5, 0.0), (1, 0, 0), (0, 1, 0), 1, 1)
    rs = np.full(len(t), 0.6, np.float32)
    rd = np.full(len(t), 0.3, np.float32)
    n = 60000
    r = _estimate(v, t, rs, rd, np.array([0.0, 0.0, 1.0]), np.full(len(t), m, np.float32), n, 1)
    lobe = 1.0 if np.isinf(m) else (m + 2) / (m + 3)
    expect = -PHI / C * (1 + 2 * 0.3 / 3 + float(np.float32(0.6)) * lobe) * np.array([0, 0, 1.0])
    mean, se = _mean_se(r.sample_force[0], np.ones(n, bool), n)
    assert np.allclose(mean, r.force[0], rtol=1e-12, atol=1e-20)
    tol = 5 * se + 1e-12 * np.abs(expect).max()
    print(f"m={m}: {mean[2]:.6e} vs {expect[2]:.6e} (se {se[2]:.1e})")
    assert np.all(np.abs(mean - expect) <= tol)


@pytest.mark.parametrize("m,theta_deg,sampling", [(5.0, 50.0, 0), (20.0, 70.0, 0), (5.0, 50.0, 2)])
def test_plate_oblique_lobe_against_quadrature(m, theta_deg, sampling):
    """The horizon cuts the lobe; plain MC (uniform hemisphere) must agree as well."""
    v, t = si.quad_grid((-0.5, -0.5, 0.0), (1, 0, 0), (0, 1, 0), 1, 1)
    rs_v = 0.7
    rs = np.full(len(t), rs_v, np.float32)
    rd = np.zeros(len(t), np.float32)
    th = np.deg2rad(theta_deg)
    sun = np.array([-np.sin(th), 0.0, np.cos(th)])  # light propagates along (sin, 0, -cos)
    n = 200000
    r = _estimate(v, t, rs, rd, sun, np.full(len(t), m, np.float32), n, 1, sampling=sampling)
    p = -sun
    M = _lobe_momentum(th, m, float(np.float32(rs_v)))
    expect = PHI / C * np.cos(th) * 1.0 * (p - M)
    mean, se = _mean_se(r.sample_force[0], np.ones(n, bool), n)
    print(f"m={m} theta={theta_deg} sampling={sampling}: {mean} vs {expect} (se {se})")
    assert np.all(np.abs(mean - expect) <= 5 * se + 1e-15)


def _pair_quadrature(PA, nA, dA, PB, nB, dB, radiance):
    """Momentum flux absorbed by a black receiver B from the radiance leaving A: sum over point
    pairs of L(omega) cos_A cos_B / r^2 omega / c dA dB, omega the unit vector A -> B."""
    D = PB[None, :, :] - PA[:, None, :]
    r2 = (D ** 2).sum(-1)
    om = D / np.sqrt(r2)[..., None]
    ca = om @ nA
    cb = -(om @ nB)
    ok = (ca > 0) & (cb > 0)
    L = radiance(om)
    w = np.where(ok, L * ca * cb / r2, 0.0) * dA * dB / C
    return (w[..., None] * om).sum((0, 1))


def test_glossy_sunlight_gathered_by_next_event_estimation():
    """Black plate B faces a sunlit Phong plate A along A's mirror direction: the force on B is the
    momentum of A's lobe, B = 2."""
    m, rs_v = 20.0, 0.8
    sun = np.array([np.sin(np.pi / 6), 0.0, np.cos(np.pi / 6)])
    nA = np.array([0.0, 0.0, 1.0])
    r = -sun + 2 * (sun @ nA) * nA  # mirror direction of the sunlight's propagation
    cA, cB, size = np.zeros(3), 1.2 * r, 0.5
    vA, tA = _square(cA, nA, size)
    vB, tB = _square(cB, -r, size)
    V, T, owner = _mesh([(vA, tA), (vB, tB)])
    rs = np.where(owner == 0, rs_v, 0.0).astype(np.float32)
    rd = np.zeros(len(T), np.float32)
    ph = np.full(len(T), m, np.float32)
    n = 400000
    res = _estimate(V, T, rs, rd, sun, ph, n, 2)
    onB = owner[res.facet[0]] == 1
    mean, se = _mean_se(res.sample_force[0], onB, n)
    PA, nA_, dA = _grid_points(cA, nA, size, 40)
    PB, nB_, dB = _grid_points(cB, -r, size, 40)
    rsf = float(np.float32(rs_v))
    radiance = lambda om: rsf * (m + 2) / (2 * np.pi) * np.maximum(om @ r, 0.0) ** m * PHI * (sun @ nA)
    expect = _pair_quadrature(PA, nA_, dA, PB, nB_, dB, radiance)
    print(f"force on B: {mean} (se {se}) vs quadrature {expect}")
    assert np.all(np.abs(mean - expect) <= 5 * se + 2e-3 * np.abs(expect).max())


@pytest.mark.parametrize("sampling", [0, 2])
def test_glossy_continuation_three_plates(sampling):
    """Sunlit Lambertian plate A -> unlit Phong plate G -> black plate B (and A -> B directly), B = 3:
    the continuation at G samples the lobe about the mirror of the gathering direction (or, plain
    MC, the hemisphere).  The light that comes by way of G is isolated by running the same samples
    with G black (common random numbers: every other path is the same in both runs)."""
    m, rsG, rdA = 5.0, 0.9, 0.9
    sun = np.array([0.0, 0.0, 1.0])
    cA, nA, size = np.zeros(3), np.array([0.0, 0.0, 1.0]), 0.6
    # G stands upright (unlit: its normal is horizontal) and turns A's light sideways and up to B,
    # clear of the sunlight on A and of the line of sight A -> B
    cG = np.array([1.0, 0.0, 0.6])
    nG = np.array([-1.0, -0.6, 0.0]) / np.linalg.norm([-1.0, -0.6, 0.0])
    pAG = (cG - cA) / np.linalg.norm(cG - cA)  # propagation of A's light reaching G
    rG = pAG - 2 * (pAG @ nG) * nG
    cB = cG + 1.0 * rG
    nB = -rG
    assert nB @ sun <= 0.0 and nG @ sun <= 0.0
    vA, tA = _square(cA, nA, size)
    vG, tG = _square(cG, nG, size)
    vB, tB = _square(cB, nB, size)
    V, T, owner = _mesh([(vA, tA), (vG, tG), (vB, tB)])
    rs = np.where(owner == 1, rsG, 0.0).astype(np.float32)
    rd = np.where(owner == 0, rdA, 0.0).astype(np.float32)
    ph = np.full(len(T), m, np.float32)
    n = 600000
    res = _estimate(V, T, rs, rd, sun, ph, n, 3, sampling=sampling)
    onB = owner[res.facet[0]] == 2
    mean, se = _mean_se(res.sample_force[0], onB, n)
    res0 = _estimate(V, T, np.zeros_like(rs), rd, sun, ph, n, 3, sampling=sampling)
    assert np.array_equal(res0.facet, res.facet)
    mean_via, se_via = _mean_se(res.sample_force[0] - res0.sample_force[0], onB, n)
    k = 12
    PA, _, dA = _grid_points(cA, nA, size, k)
    PG, _, dG = _grid_points(cG, nG, size, k)
    PB, _, dB = _grid_points(cB, nB, size, k)
    rdf, rsf = float(np.float32(rdA)), float(np.float32(rsG))
    LA = rdf / np.pi * PHI * (sun @ nA)  # Lambertian radiance of A
    # A -> B directly
    direct = _pair_quadrature(PA, nA, dA, PB, nB, dB, lambda om: np.full(om.shape[:-1], LA))
    # A -> G -> B: irradiance at each G point from A, per direction, reflected by the lobe to B
    DAG = PG[None, :, :] - PA[:, None, :]
    r2 = (DAG ** 2).sum(-1)
    om1 = DAG / np.sqrt(r2)[..., None]
    ca = om1 @ nA
    cg = -(om1 @ nG)
    e = np.where((ca > 0) & (cg > 0), LA * ca * cg / r2, 0.0) * dA  # [A][G] irradiance pieces
    DGB = PB[None, :, :] - PG[:, None, :]
    r2b = (DGB ** 2).sum(-1)
    om2 = DGB / np.sqrt(r2b)[..., None]
    cg2 = om2 @ nG  # light leaves G's outward side along om2
    cb = -(om2 @ nB)
    geo = np.where((cg2 > 0) & (cb > 0), cg2 * cb / r2b, 0.0) * dG * dB  # [G][B]
    # mirror of each incoming propagation om1 about nG, and the lobe toward om2
    rr = om1 - 2 * (om1 @ nG)[..., None] * nG  # [A][G][3]
    lobe = np.einsum("agc,gbc->agb", rr, om2)  # [A][G][B]
    f = rsf * (m + 2) / (2 * np.pi) * np.maximum(lobe, 0.0) ** m
    w = np.einsum("ag,agb,gb->gb", e, f, geo) / C  # [G][B] momentum weights
    via = (w[..., None] * om2).sum((0, 1))
    expect = direct + via
    print(f"force on B: {mean} (se {se}) vs quadrature {expect} (direct {direct}); by way of G "
          f"{mean_via} (se {se_via}) vs {via}")
    assert np.all(np.abs(mean - expect) <= 5 * se + 5e-3 * np.abs(expect).max())
    assert np.all(np.abs(mean_via - via) <= 5 * se_via + 5e-3 * np.abs(via).max())


def test_phong_exponents_validated():
    v, t = si.quad_grid((-0.5, -0.5, 0.0), (1, 0, 0), (0, 1, 0), 1, 1)
    rs = np.full(len(t), 0.5, np.float32)
    rd = np.zeros(len(t), np.float32)
    for bad in (0.5, np.nan, -1.0):
        with pytest.raises(ValueError):
            oracle.surface_estimate(v, t, rs, rd, np.array([[0, 0, 1.0]]), n_samples=10, bounces=1,
                                    phong=np.full(len(t), bad, np.float32))
