"""Pins of the oracle against what the paper and the mathematics fix (CPU only).

Each test checks the FP64 oracle against something other than itself:
  * Philox blocks against the rocRAND library implementation;
  * the flat-plate closed form (exact to rounding when the grid covers the plate exactly);
  * the plate's torque about the centre of mass (lever arm of the footprint centroid);
  * the sphere closed form (1 + 4 rho_d / 9) Phi pi R^2 / c via the exact sum over lit facets,
    and the traced estimate against that sum within its Monte Carlo error;
  * the 90-degree dihedral mirror (retro-reflection after exactly two hits);
  * the mean Lambertian momentum 2/3 n (Sec. 5.9) through sampled diffuse bounces;
  * closest-hit indices against a brute-force numpy.linalg.solve of the ray/plane systems;
  * invariants: linearity in Phi (bit-exact), rho = 0 (force along the light, independent of the
    bounce count), rotational equivariance with rotated caller frames, projected area of a cube.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
import srp_inputs as si

C = 299792458.0
PHI = 1361.0


def plate_force(area, cos_t, rho_s, rho_d, s_hat, n_hat):
    """F = (Phi A cos(theta) / c) [(1 - rho_s) s + 2 (rho_s cos(theta) + rho_d / 3) n]:
    s = propagation direction of the light, n = inward normal (cos(theta) = s . n > 0)."""
    return PHI * area * cos_t / C * ((1 - rho_s) * s_hat + 2 * (rho_s * cos_t + rho_d / 3) * n_hat)


def lit_facet_sum(mesh, sun, rho_s, rho_d):
    """Exact shadow-free force of a convex mesh: sum of the plate formula over lit facets."""
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


# --------------------------------------------------------------------------------------------
# Philox
# --------------------------------------------------------------------------------------------
def _rocrand_ref(blocks):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc) or not os.path.exists("/opt/rocm/include/rocrand/rocrand_philox4x32_10.h"):
        pytest.skip("rocRAND headers / hipcc not available")
    src = os.path.join(os.path.dirname(__file__), "native", "philox_rocrand.cpp")
    exe = os.path.join("/tmp", f"philox_rocrand_{os.getpid()}")
    subprocess.run([hipcc, "-O1", "-o", exe, src], check=True, capture_output=True)
    inp = "\n".join(" ".join(str(int(x)) for x in b) for b in blocks) + "\n"
    out = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True).stdout
    os.remove(exe)
    return np.array([[int(x) for x in line.split()] for line in out.strip().splitlines()], dtype=np.uint64)


def test_philox_matches_rocrand():
    rng = np.random.default_rng(11)
    blocks = []
    for i in range(64):
        c = rng.integers(0, 2 ** 32, 4, dtype=np.uint64)
        c[1] %= 2 ** 30  # keeps the library's element offset (4 * counter) inside 64 bits
        k = rng.integers(0, 2 ** 32, 2, dtype=np.uint64)
        blocks.append([*c, *k])
    blocks.append([0, 0, 0, 0, 0, 0])
    blocks.append([5, 7, 1, 3, 2, 0])
    ref = _rocrand_ref(blocks)
    for b, r in zip(blocks, ref):
        got = oracle.philox(b[:4], b[4:])
        assert np.array_equal(got.astype(np.uint64), r), (b, got, r)


def test_philox_uniformity_chi2():
    # 24-bit uniforms from consecutive pixel counters: chi^2 over 64 bins
    n = 20000
    u = np.array([oracle.philox([i, 3, 0, 0], [2, 0])[0] >> 8 for i in range(n)], dtype=np.float64) / 2 ** 24
    h, _ = np.histogram(u, bins=64, range=(0, 1))
    e = n / 64
    chi2 = ((h - e) ** 2 / e).sum()
    assert chi2 < 120  # 63 dof: p ~ 1e-5 threshold
    assert u.min() >= 0 and u.max() < 1


def test_basis_orthonormal_right_handed():
    rng = np.random.default_rng(0)
    ns = list(rng.standard_normal((200, 3))) + [np.array([0, 0, 1.0]), np.array([0, 0, -1.0]),
                                               np.array([1.0, 0, 0]), np.array([0, 1.0, 0]),
                                               np.array([0.0, 0.6, -0.8])]
    for n in ns:
        n = n / np.linalg.norm(n)
        b1, b2 = oracle.basis(n)
        M = np.stack([b1, b2, n])
        assert np.allclose(M @ M.T, np.eye(3), atol=1e-12)
        assert np.allclose(np.cross(b1, b2), n, atol=1e-12)


# --------------------------------------------------------------------------------------------
# plate
# --------------------------------------------------------------------------------------------
@pytest.mark.parametrize("tilt", [0.0, 25.0, 60.0])
@pytest.mark.parametrize("rho", [(0.0, 0.0), (0.3, 0.2), (0.5, 0.0), (0.0, 0.5), (0.9, 0.1)])
def test_plate_closed_form_exact(tilt, rho):
    W, H = 2.0, 1.5
    m = si.plate(W, H, tilt_deg=tilt)
    rs = np.full(2, rho[0], np.float32)
    rd = np.full(2, rho[1], np.float32)
    sun = np.array([[0.0, 0.0, 1.0]])  # Duff basis for d = -z: u = +x, v = -y -> grid == footprint
    res = oracle.trace(m.verts, m.tris, rs, rd, sun, nu=64, nv=48, bounces=1, jitter=False, seed=0, threads=2)
    a = np.deg2rad(tilt)
    n_out = np.array([0.0, -np.sin(a), np.cos(a)])
    s_hat = np.array([0.0, 0.0, -1.0])
    ref = plate_force(W * H, np.cos(a), float(rs[0]), float(rd[0]), s_hat, -n_out)
    assert np.allclose(res.force[0], ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())
    # torque about the COM: the pixel-centre hit points average to the plate centre (the origin)
    assert np.allclose(res.torque[0], 0.0, atol=1e-18)


def test_plate_torque_lever_arm():
    W, H = 2.0, 1.0
    centre = np.array([0.7, -0.4, 0.3])
    m = si.plate(W, H, center=centre)
    rs = np.full(2, 0.25, np.float32)
    rd = np.full(2, 0.35, np.float32)
    com = np.array([-0.2, 0.1, 0.05])
    res = oracle.trace(m.verts, m.tris, rs, rd, [[0, 0, 1.0]], nu=40, nv=20, bounces=1, jitter=False, com=com,
                       threads=2)
    ref_F = plate_force(W * H, 1.0, float(rs[0]), float(rd[0]), np.array([0, 0, -1.0]), np.array([0, 0, -1.0]))
    assert np.allclose(res.force[0], ref_F, rtol=1e-12, atol=0)
    assert np.allclose(res.torque[0], np.cross(centre - com, ref_F), rtol=1e-10, atol=1e-20)


def test_plate_oblique_caller_frame():
    """Arbitrary plate orientation; light in the plane of the normal and one edge, grid aligned
    with the rectangular footprint through a caller-supplied frame."""
    rng = np.random.default_rng(5)
    for trial in range(5):
        Q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
        a_dir, b_dir, n = Q[:, 0], Q[:, 1], np.cross(Q[:, 0], Q[:, 1])
        A, Bl = 1.3, 0.7
        p0 = rng.standard_normal(3) * 0.3
        verts = np.array([p0, p0 + A * a_dir, p0 + A * a_dir + Bl * b_dir, p0 + Bl * b_dir])
        tris = np.array([[0, 1, 2], [0, 2, 3]], dtype=np.int32)
        th = rng.uniform(0.1, 1.2)
        sun = np.cos(th) * n + np.sin(th) * a_dir  # toward the Sun, in span(n, a)
        d = -sun
        u = a_dir - (a_dir @ d) * d
        u /= np.linalg.norm(u)
        v = b_dir
        proj_u = (verts - p0) @ u
        proj_v = (verts - p0) @ v
        s0 = (verts @ d).min() - 0.1
        o0 = s0 * d + (p0 @ u + proj_u.min()) * u + (p0 @ v + proj_v.min()) * v
        nu, nv = 30, 20
        fr = np.concatenate([u, v, o0, [np.ptp(proj_u) / nu, np.ptp(proj_v) / nv, 0.0]])[None]
        rs = np.full(2, 0.4, np.float32)
        rd = np.full(2, 0.3, np.float32)
        res = oracle.trace(verts, tris, rs, rd, sun[None], nu=nu, nv=nv, bounces=1, jitter=False, frames_in=fr,
                           threads=2)
        ref = plate_force(A * Bl, np.cos(th), float(rs[0]), float(rd[0]), d, -n)
        assert np.allclose(res.force[0], ref, rtol=1e-11, atol=1e-11 * np.abs(ref).max()), trial


# --------------------------------------------------------------------------------------------
# sphere, convex bodies
# --------------------------------------------------------------------------------------------
def test_sphere_facet_sum_converges_to_closed_form():
    """The exact lit-facet sum of icospheres approaches (1 + 4 rho_d/9) Phi pi R^2 / c, and is
    independent of rho_s in the limit (specular reflection of a sphere cancels)."""
    R = 1.0
    sun = np.array([0.3, -0.5, 0.81])
    sun /= np.linalg.norm(sun)
    errs = []
    for level in (2, 3, 4):
        m = si.icosphere(level, R)
        T = m.n_tris
        for rs_v, rd_v in ((0.0, 0.5), (0.6, 0.2)):
            F = lit_facet_sum(m, sun, np.full(T, rs_v), np.full(T, rd_v))
            ref = (1 + 4 * rd_v / 9) * PHI * np.pi * R ** 2 / C * (-sun)
            errs.append((level, np.linalg.norm(F - ref) / np.linalg.norm(ref)))
    e = {lv: max(x for l2, x in errs if l2 == lv) for lv, _ in errs}
    assert e[4] < 2.5e-3 and e[3] < e[2] and e[4] < e[3]


def test_sphere_traced_matches_facet_sum_statistically():
    m = si.icosphere(2, 1.0)
    T = m.n_tris
    rs = np.full(T, 0.3, np.float32)
    rd = np.full(T, 0.4, np.float32)
    sun = np.array([[0.2, 0.4, -0.894]])
    sun /= np.linalg.norm(sun)
    exact = lit_facet_sum(m, sun[0], rs, rd)
    samples = []
    for seed in range(6):
        res = oracle.trace(m.verts, m.tris, rs, rd, sun, nu=96, nv=96, bounces=1, jitter=True, seed=seed)
        samples.append(res.force[0])
    samples = np.array(samples)
    mean = samples.mean(0)
    se = samples.std(0, ddof=1) / np.sqrt(len(samples))
    assert np.all(np.abs(mean - exact) < 5 * se + 1e-4 * np.abs(exact).max())
    # and the sphere closed form is within the tessellation error
    ref = (1 + 4 * 0.4 / 9) * PHI * np.pi / C * (-sun[0])
    assert np.linalg.norm(mean - ref) / np.linalg.norm(ref) < 0.03


def test_convex_bounces_unbiased_and_diffuse_two_thirds():
    """B = 2 samples the reflected direction (the light then escapes a convex body); its mean
    must equal the B = 1 expected recoil, which uses the Lambertian 2/3 n (Sec. 5.9)."""
    m = si.plate(1.0, 1.0)
    for rho in ((0.0, 1.0), (0.3, 0.4)):
        rs = np.full(2, rho[0], np.float32)
        rd = np.full(2, rho[1], np.float32)
        sun = np.array([[0.0, 0.0, 1.0]])
        f1 = oracle.trace(m.verts, m.tris, rs, rd, sun, nu=128, nv=128, bounces=1, jitter=True, seed=3,
                          records=True)
        f2 = oracle.trace(m.verts, m.tris, rs, rd, sun, nu=128, nv=128, bounces=2, jitter=True, seed=3,
                          records=True)
        per_ray = f2.ray_force[0]
        hit = f2.hit_prim[0, :, 0] >= 0
        per_ray = per_ray[hit]
        mean = per_ray.mean(0) * hit.sum()
        se = per_ray.std(0, ddof=1) / np.sqrt(hit.sum()) * hit.sum()
        assert np.all(np.abs(mean - f1.force[0]) < 5 * se + 1e-18), (rho, mean, f1.force[0], se)
        if rho == (0.0, 1.0):
            # deposit per ray: w d - w o'  =>  mean o' . n = 2/3 exactly in expectation
            w = PHI * (1.0 / 128) ** 2 / C
            o_n = (w * -1.0 - per_ray[:, 2]) / w  # d = -z, n = +z: F_z = -w - w o'_z
            assert abs(o_n.mean() - 2 / 3) < 5 * o_n.std() / np.sqrt(len(o_n))


# --------------------------------------------------------------------------------------------
# bounce logic: dihedral mirror
# --------------------------------------------------------------------------------------------
@pytest.mark.parametrize("bounces", [1, 2, 3])
def test_dihedral_retroreflection(bounces):
    Lp, Hp = 2.0, 1.0
    m = si.dihedral(Lp, Hp)
    rs = np.ones(4, np.float32)
    rd = np.zeros(4, np.float32)
    sun = np.array([1.0, 1.0, 0.0]) / np.sqrt(2)
    d = -sun
    u = np.array([1.0, -1.0, 0.0]) / np.sqrt(2)
    v = np.array([0.0, 0.0, 1.0])
    s0 = -np.sqrt(2) * Lp - 0.1
    o0 = s0 * d + (-Lp / np.sqrt(2)) * u
    nu, nv = 64, 16
    fr = np.concatenate([u, v, o0, [np.sqrt(2) * Lp / nu, Hp / nv, 0.0]])[None]
    res = oracle.trace(m.verts, m.tris, rs, rd, sun[None], nu=nu, nv=nv, bounces=bounces, jitter=False,
                       frames_in=fr, records=True, threads=2)
    unit = np.sqrt(2) * PHI * Lp * Hp / C * d
    ref = unit if bounces == 1 else 2 * unit
    assert np.allclose(res.force[0], ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())
    hp = res.hit_prim[0]
    plate_of = lambda tri: np.where(tri < 0, -1, tri // 2)
    p = plate_of(hp)
    assert np.all(p[:, 0] >= 0)
    if bounces >= 2:
        assert np.all(p[:, 1] >= 0) and np.all(p[:, 1] != p[:, 0])
    if bounces == 3:
        assert np.all(p[:, 2] == -1)
    assert not res.degen.any()


# --------------------------------------------------------------------------------------------
# closest hit vs brute-force linear solves
# --------------------------------------------------------------------------------------------
def test_closest_hit_matches_linear_solve():
    rng = np.random.default_rng(7)
    nt = 12
    centres = rng.uniform(-1, 1, (nt, 3))
    V = (centres[:, None, :] + rng.normal(0, 0.5, (nt, 3, 3))).reshape(-1, 3)
    T = np.arange(3 * nt, dtype=np.int32).reshape(nt, 3)
    sun = si.random_dirs(3, 1)
    rs = np.zeros(nt, np.float32)
    rd = np.zeros(nt, np.float32)
    nu = nv = 24
    res = oracle.trace(V, T, rs, rd, sun, nu=nu, nv=nv, bounces=1, jitter=True, seed=9, records=True, threads=2)
    fr = oracle.frames(V, sun, nu, nv)
    checked = 0
    for j in range(len(sun)):
        d = -sun[j]
        u, v, o0, du, dv = fr[j, :3], fr[j, 3:6], fr[j, 6:9], fr[j, 9], fr[j, 10]
        for p in range(nu * nv):
            i, k = p % nu, p // nu
            r = oracle.philox([p, j, 0, 0], [9, 0])
            a, b = (r[0] >> 8) / 2 ** 24, (r[1] >> 8) / 2 ** 24
            o = o0 + (i + a) * du * u + (k + b) * dv * v
            best, tbest, margin_ok = -1, np.inf, True
            for f in range(nt):
                p0, p1, p2 = V[T[f]]
                n = np.cross(p1 - p0, p2 - p0)
                if n @ d >= 0:
                    continue
                # o + t d = p0 + beta (p1 - p0) + gamma (p2 - p0)
                M = np.stack([-d, p1 - p0, p2 - p0], 1)
                t, beta, gamma = np.linalg.solve(M, o - p0)
                bary = min(beta, gamma, 1 - beta - gamma)
                if abs(bary) < 1e-9:
                    margin_ok = False
                if bary >= 0 and t > 0 and t < tbest:
                    if abs(t - tbest) < 1e-9:
                        margin_ok = False
                    best, tbest = f, t
            if margin_ok:
                assert res.hit_prim[j, p, 0] == best, (j, p)
                checked += 1
    assert checked > 0.99 * len(sun) * nu * nv


# --------------------------------------------------------------------------------------------
# invariants
# --------------------------------------------------------------------------------------------
def test_linear_in_flux_bit_exact():
    m = si.box_wing()
    rs, rd = si.materials(m.n_tris, 1)
    sun = si.fibonacci_dirs(8)
    a = oracle.trace(m.verts, m.tris, rs, rd, sun, nu=48, nv=48, bounces=3, flux=1361.0, seed=2)
    b = oracle.trace(m.verts, m.tris, rs, rd, sun, nu=48, nv=48, bounces=3, flux=2722.0, seed=2)
    assert np.array_equal(2 * a.force, b.force) and np.array_equal(2 * a.torque, b.torque)


def test_black_body_force_along_light_and_bounce_independent():
    m = si.box_wing()
    z = np.zeros(m.n_tris, np.float32)
    sun = si.fibonacci_dirs(6)
    a = oracle.trace(m.verts, m.tris, z, z, sun, nu=40, nv=40, bounces=1, seed=4)
    b = oracle.trace(m.verts, m.tris, z, z, sun, nu=40, nv=40, bounces=3, seed=4)
    assert np.array_equal(a.force, b.force)
    for j in range(len(sun)):
        F = a.force[j]
        assert np.allclose(F / np.linalg.norm(F), -sun[j], atol=1e-12)


def test_cube_projected_area_statistical():
    m = si.meo_satellite(bus_n=2, cyl_sides=8, panel_n=1, dish_rings=3, dish_sectors=8, strut_sides=4,
                         n_antennas=0)
    # keep only the bus (first 6 faces x 2 x 2 x 2 = 48 tris)
    T = m.tris[:48]
    z = np.zeros(48, np.float32)
    sun = np.array([0.48, 0.6, 0.64])
    sun /= np.linalg.norm(sun)
    V = m.verts
    cr = np.cross(V[T[:, 1]] - V[T[:, 0]], V[T[:, 2]] - V[T[:, 0]])
    area_proj = 0.5 * np.clip(cr @ sun, 0, None).sum()
    vals = []
    for seed in range(4):
        r = oracle.trace(V, T, z, z, sun[None], nu=80, nv=80, bounces=1, seed=seed)
        vals.append(np.linalg.norm(r.force[0]) * C / PHI)
    vals = np.array(vals)
    assert abs(vals.mean() - area_proj) < 5 * vals.std(ddof=1) / 2 + 1e-3 * area_proj


def test_rotational_equivariance_with_rotated_frames():
    # mirror-only materials: the Lambertian direction is drawn in a basis tied to the absolute
    # normal direction, so only the specular paths are exactly equivariant
    m = si.box_wing()
    rs, _ = si.materials(m.n_tris, 1)
    rd = np.zeros_like(rs)
    sun = si.fibonacci_dirs(5)
    nu = nv = 40
    fr = oracle.frames(m.verts, sun, nu, nv)
    base = oracle.trace(m.verts, m.tris, rs, rd, sun, nu=nu, nv=nv, bounces=3, seed=8, frames_in=fr)
    Q, _ = np.linalg.qr(np.random.default_rng(3).standard_normal((3, 3)))
    if np.linalg.det(Q) < 0:
        Q[:, 0] *= -1
    fr2 = fr.copy()
    for j in range(len(sun)):
        fr2[j, 0:3] = Q @ fr[j, 0:3]
        fr2[j, 3:6] = Q @ fr[j, 3:6]
        fr2[j, 6:9] = Q @ fr[j, 6:9]
    rot = oracle.trace(m.verts @ Q.T, m.tris, rs, rd, sun @ Q.T, nu=nu, nv=nv, bounces=3, seed=8, frames_in=fr2)
    assert np.allclose(rot.force, base.force @ Q.T, rtol=1e-9, atol=1e-9 * np.abs(base.force).max())
    assert np.allclose(rot.torque, base.torque @ Q.T, rtol=1e-9, atol=1e-9 * np.abs(base.torque).max())


def test_degeneracy_flags_shared_diagonal():
    """Pixel centres on the shared diagonal of a two-triangle plate are flagged, the others not."""
    m = si.plate(1.0, 1.0)
    z = np.full(2, 0.2, np.float32)
    nu = 16
    res = oracle.trace(m.verts, m.tris, z, z, [[0, 0, 1.0]], nu=nu, nv=nu, bounces=1, jitter=False, records=True)
    deg = res.degen[0, :, 0].reshape(nu, nu)  # [k][i]
    # u = +x, v = -y: pixel (i, k) centre at x = -0.5 + (i+.5)/16, y = 0.5 - (k+.5)/16;
    # the diagonal of quad_grid runs from (-0.5,-0.5) to (0.5,0.5): x = y  <=>  i + k = 15
    expect = np.zeros((nu, nu), bool)
    for i in range(nu):
        expect[nu - 1 - i, i] = True
    assert np.array_equal(deg.astype(bool), expect)


def test_frame_covers_mesh():
    m = si.meo_satellite()
    sun = si.fibonacci_dirs(16)
    fr = oracle.frames(m.verts, sun, 64, 32)
    for j in range(len(sun)):
        u, v, o0, du, dv = fr[j, :3], fr[j, 3:6], fr[j, 6:9], fr[j, 9], fr[j, 10]
        d = -sun[j]
        rel = m.verts - o0
        pu, pv, pd = rel @ u / du, rel @ v / dv, rel @ d
        assert pu.min() > -1e-9 and pu.max() < 64 + 1e-9
        assert pv.min() > -1e-9 and pv.max() < 32 + 1e-9
        assert pd.min() > 0
