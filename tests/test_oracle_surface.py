"""Pins of the oracle's surface-sampling estimator (paper Sec. 3.2, "Estimation": area-sampled
surface points, path-traced incoming light with next-event estimation toward the Sun, one sampled
outgoing event), independent of the GPU path:

  * plates: a black and a mirror plate give the closed form exactly (every sample deposits the
    same force density); a mixed plate's mean and its torque lever arm within 5 standard errors;
  * convex body: gathering rays escape, the mean matches the exact lit-facet sum;
  * mirror dihedral: sunlight whose first reflection is a mirror is not gathered, so two bounces
    give the single-bounce value of the ray-grid closed form (the estimator's stated limit);
  * Lambertian scenes with interreflection (dihedral, box-wing, 3 bounces): the mean agrees with
    the ray-grid estimator, which is the same expectation;
  * the result does not depend on the thread count;
  * the variance-reduction options of the paper's convergence study (stratified surface sampling,
    and plain MC with uniform hemisphere directions instead of the BRDF's cosine importance
    sampling): plates stay exact, every option is unbiased (convex body against the exact sum,
    Lambertian box-wing at 3 bounces against the ray grid, over independent seeds), and
    stratification cuts the variance of the estimate.
"""
import numpy as np
import pytest

import oracle
import srp_inputs as si

C = 299792458.0
PHI = 1361.0


def plate_force(area, cos_t, rho_s, rho_d, s_hat, n_hat):
    """(Phi A cos / c) [(1 - rho_s) s + 2 (rho_s cos + rho_d / 3) n]; s = propagation, n = inward."""
    return PHI * area * cos_t / C * ((1 - rho_s) * s_hat + 2 * (rho_s * cos_t + rho_d / 3) * n_hat)


def mean_and_se(x):
    x = np.asarray(x).reshape(-1, 3)
    return x.mean(0), x.std(0, ddof=1) / np.sqrt(len(x))


def lit_facet_sum(mesh, sun, rho_s, rho_d):
    V, T = mesh.verts, mesh.tris
    cr = np.cross(V[T[:, 1]] - V[T[:, 0]], V[T[:, 2]] - V[T[:, 0]])
    area = 0.5 * np.linalg.norm(cr, axis=1)
    n_out = cr / (2 * area[:, None])
    s_hat = -np.asarray(sun) / np.linalg.norm(sun)
    F = np.zeros(3)
    for f in range(len(T)):
        c = float(s_hat @ -n_out[f])
        if c > 0:
            F += plate_force(area[f], c, float(rho_s[f]), float(rho_d[f]), s_hat, -n_out[f])
    return F


@pytest.mark.parametrize("rho", [(0.0, 0.0), (1.0, 0.0)])
def test_black_and_mirror_plate_exact(rho):
    W, H, tilt = 2.0, 1.5, 35.0
    m = si.plate(W, H, tilt_deg=tilt)
    rs = np.full(2, rho[0], np.float32)
    rd = np.full(2, rho[1], np.float32)
    sun = np.array([[0.0, 0.0, 1.0]])
    res = oracle.surface_estimate(m.verts, m.tris, rs, rd, sun, n_samples=1000, bounces=3, seed=3, records=True,
                                  threads=2)
    a = np.deg2rad(tilt)
    n_out = np.array([0.0, -np.sin(a), np.cos(a)])
    ref = plate_force(W * H, np.cos(a), rho[0], rho[1], np.array([0.0, 0.0, -1.0]), -n_out)
    assert np.allclose(res.force[0], ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())
    assert np.all(res.lit[0] == 1) and np.all(res.hits[0] == -1) and not res.degen.any()


def test_mixed_plate_mean_and_lever_arm():
    W, H = 2.0, 1.0
    centre = np.array([0.7, -0.4, 0.3])
    com = np.array([-0.2, 0.1, 0.05])
    m = si.plate(W, H, center=centre, nu=3, nv=2)
    rs = np.full(m.n_tris, 0.3, np.float32)
    rd = np.full(m.n_tris, 0.45, np.float32)
    sun = np.array([0.3, -0.2, 1.0])
    sun /= np.linalg.norm(sun)
    N = 200000
    res = oracle.surface_estimate(m.verts, m.tris, rs, rd, sun[None], n_samples=N, bounces=2, seed=4, com=com,
                                  records=True, threads=4)
    ref = plate_force(W * H, sun[2], 0.3, 0.45, -sun, np.array([0.0, 0.0, -1.0]))
    mean, se = mean_and_se(res.sample_force[0])
    assert np.allclose(mean, res.force[0], rtol=1e-9, atol=0)  # same samples, other summation order
    assert np.all(np.abs(mean - ref) <= 5 * se + 1e-3 * np.abs(ref).max())
    # uniform points on the plate: the torque averages to (centre - com) x F
    tq_ref = np.cross(centre - com, ref)
    L = np.linalg.norm(centre - com) + np.hypot(W, H)
    assert np.linalg.norm(res.torque[0] - tq_ref) <= 0.01 * L * np.linalg.norm(ref)


def test_convex_body_matches_lit_facet_sum():
    m = si.icosphere(2, radius=1.3)
    rs, rd = si.materials(m.n_tris, 7)
    sun = np.array([0.2, 0.5, -0.84])
    sun /= np.linalg.norm(sun)
    res = oracle.surface_estimate(m.verts, m.tris, rs, rd, sun[None], n_samples=400000, bounces=3, seed=5,
                                  records=True, threads=4)
    assert np.all(res.hits == -1)  # gathering rays leave a convex body
    ref = lit_facet_sum(m, sun, rs, rd)
    mean, se = mean_and_se(res.sample_force[0])
    assert np.all(np.abs(mean - ref) <= 5 * se)


def test_mirror_dihedral_gathers_no_mirror_first_light():
    Lp, Hp = 2.0, 1.0
    m = si.dihedral(Lp, Hp)
    rs = np.ones(4, np.float32)
    rd = np.zeros(4, np.float32)
    sun = np.array([1.0, 1.0, 0.0]) / np.sqrt(2)
    unit = np.sqrt(2) * PHI * Lp * Hp / C * (-sun)  # ray-grid value at one bounce (two: twice this)
    res = oracle.surface_estimate(m.verts, m.tris, rs, rd, sun[None], n_samples=100000, bounces=2, seed=6,
                                  records=True, threads=4)
    mean, se = mean_and_se(res.sample_force[0])
    assert np.all(np.abs(mean - unit) <= 5 * se + 1e-12)
    assert np.linalg.norm(mean - 2 * unit) > 0.4 * np.linalg.norm(unit)
    assert np.all(res.lit[0] == 1)  # only direct light at x, never a lit gathered vertex


def test_lambertian_dihedral_matches_ray_grid():
    Lp, Hp = 2.0, 1.0
    m = si.dihedral(Lp, Hp)
    rs = np.zeros(4, np.float32)
    rd = np.full(4, 0.9, np.float32)
    sun = np.array([[0.8, 0.45, 0.4]])
    sun /= np.linalg.norm(sun)
    grid = oracle.trace(m.verts, m.tris, rs, rd, sun, nu=256, nv=256, bounces=2, seed=7, threads=4)
    res = oracle.surface_estimate(m.verts, m.tris, rs, rd, sun, n_samples=400000, bounces=2, seed=8, records=True,
                                  threads=4)
    mean, se = mean_and_se(res.sample_force[0])
    # the ray grid's own Monte Carlo error (256^2 jittered rays) is far below the sampling error here
    assert np.all(np.abs(mean - grid.force[0]) <= 5 * se + 2e-3 * np.abs(grid.force[0]).max())
    assert (res.lit[0] >= 2).any()  # gathered light does arrive (lit gathered vertices)


def test_mirror_after_diffuse_matches_ray_grid():
    """Dihedral with a mirror plate (x = 0, facing +x) the Sun does not light and a Lambertian
    plate (y = 0, facing +y) it does: every mirror reflection follows a diffuse one, so the gathered
    paths (mirror continuation at a gathered vertex) carry all the light of the ray grid."""
    Lp, Hp = 2.0, 1.0
    m = si.dihedral(Lp, Hp)
    rs = np.array([1.0, 1.0, 0.0, 0.0], np.float32)
    rd = np.array([0.0, 0.0, 0.95, 0.95], np.float32)
    sun = np.array([[-0.3, 0.9, 0.3]])
    sun /= np.linalg.norm(sun)
    grid = oracle.trace(m.verts, m.tris, rs, rd, sun, nu=256, nv=256, bounces=3, seed=12, threads=4)
    res = oracle.surface_estimate(m.verts, m.tris, rs, rd, sun, n_samples=400000, bounces=3, seed=13, records=True,
                                  threads=4)
    mean, se = mean_and_se(res.sample_force[0])
    assert np.all(np.abs(mean - grid.force[0]) <= 5 * se + 2e-3 * np.abs(grid.force[0]).max())
    # samples on the mirror plate that gather light reflected by the lit plate
    on_mirror = res.facet[0] < 2
    assert ((res.lit[0][on_mirror] & 2) != 0).any()


def test_lambertian_box_wing_matches_ray_grid_three_bounces():
    m = si.box_wing()
    rd = np.full(m.n_tris, 0.8, np.float32)
    rs = np.zeros(m.n_tris, np.float32)
    sun = si.fibonacci_dirs(3)
    grid = oracle.trace(m.verts, m.tris, rs, rd, sun, nu=256, nv=256, bounces=3, seed=9, threads=4)
    res = oracle.surface_estimate(m.verts, m.tris, rs, rd, sun, n_samples=200000, bounces=3, seed=10, records=True,
                                  threads=4)
    for j in range(len(sun)):
        mean, se = mean_and_se(res.sample_force[j])
        assert np.all(np.abs(mean - grid.force[j]) <= 5 * se + 2e-3 * np.abs(grid.force[j]).max())


def test_thread_count_independent():
    m = si.box_wing()
    rs, rd = si.materials(m.n_tris, 2)
    sun = si.fibonacci_dirs(2)
    a = oracle.surface_estimate(m.verts, m.tris, rs, rd, sun, n_samples=3000, bounces=3, seed=11, threads=1)
    b = oracle.surface_estimate(m.verts, m.tris, rs, rd, sun, n_samples=3000, bounces=3, seed=11, threads=5)
    assert np.array_equal(a.force, b.force) and np.array_equal(a.torque, b.torque)


def seed_estimates(mesh, rs, rd, sun, n, k, bounces, sampling):
    """k independent estimates (seeds 200..) of n samples each: [k][D][3]."""
    return np.array([oracle.surface_estimate(mesh.verts, mesh.tris, rs, rd, sun, n_samples=n, bounces=bounces,
                                             seed=200 + i, threads=4, sampling=sampling).force for i in range(k)])


@pytest.mark.parametrize("sampling", [1, 2, 3])
def test_sampling_options_keep_plates_exact(sampling):
    W, H, tilt = 2.0, 1.5, 35.0
    m = si.plate(W, H, tilt_deg=tilt)
    a = np.deg2rad(tilt)
    n_out = np.array([0.0, -np.sin(a), np.cos(a)])
    for rho in [(0.0, 0.0), (1.0, 0.0)]:
        rs = np.full(2, rho[0], np.float32)
        rd = np.full(2, rho[1], np.float32)
        res = oracle.surface_estimate(m.verts, m.tris, rs, rd, np.array([[0.0, 0.0, 1.0]]), n_samples=1000, bounces=3,
                                      seed=3, threads=2, sampling=sampling)
        ref = plate_force(W * H, np.cos(a), rho[0], rho[1], np.array([0.0, 0.0, -1.0]), -n_out)
        assert np.allclose(res.force[0], ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())


@pytest.mark.parametrize("sampling", [1, 2, 3])
def test_sampling_options_unbiased_on_convex_body(sampling):
    m = si.icosphere(2, radius=1.3)
    rs, rd = si.materials(m.n_tris, 7)
    sun = np.array([0.2, 0.5, -0.84])
    sun /= np.linalg.norm(sun)
    est = seed_estimates(m, rs, rd, sun[None], 20000, 12, 3, sampling)[:, 0]
    ref = lit_facet_sum(m, sun, rs, rd)
    se = est.std(0, ddof=1) / np.sqrt(len(est))
    assert np.all(np.abs(est.mean(0) - ref) <= 5 * se + 1e-6 * np.abs(ref).max())


@pytest.mark.parametrize("sampling", [2, 3])
def test_uniform_directions_unbiased_through_interreflection(sampling):
    m = si.box_wing()
    rd = np.full(m.n_tris, 0.8, np.float32)
    rs = np.zeros(m.n_tris, np.float32)
    sun = si.fibonacci_dirs(3)
    grid = oracle.trace(m.verts, m.tris, rs, rd, sun, nu=256, nv=256, bounces=3, seed=9, threads=4)
    est = seed_estimates(m, rs, rd, sun, 20000, 12, 3, sampling)
    se = est.std(0, ddof=1) / np.sqrt(len(est))
    assert np.all(np.abs(est.mean(0) - grid.force) <= 5 * se + 2e-3 * np.abs(grid.force).max())


def test_stratification_reduces_variance():
    m = si.icosphere(2, radius=1.3)
    rs, rd = si.materials(m.n_tris, 7)
    sun = np.array([[0.2, 0.5, -0.84]])
    sun /= np.linalg.norm(sun)
    var = {}
    for sampling in range(4):
        est = seed_estimates(m, rs, rd, sun, 4096, 24, 3, sampling)
        var[sampling] = ((est - est.mean(0)) ** 2).sum(-1).mean()
    print("variance by option:", var)
    assert var[1] < var[0] / 3 and var[3] < var[2] / 3  # stratified vs not (measured 8.6x, 4.9x)
    assert var[2] / var[1] > 4  # plain MC vs both (measured 10.5x)
