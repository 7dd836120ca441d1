"""Pins of the oracle's degenerate-segment classification, its hit-point records and its
reflectance adjoint restricted to non-degenerate paths (CPU only).

A segment is degenerate when an FP32 evaluation could choose another closest hit than the FP64
one; the rules are stated in srp_oracle.c.  A primary segment's position uncertainty across the
ray is u = LAT * L; after an interaction at incidence cos(theta) it becomes u / cos(theta) + LAT L.
A primary ray meets a plane at incidence cos at a t uncertain by tau = (DEPTH L + u) / cos.  Each pin places single rays with
caller frames (one ray per "direction": pixel (0, 0) of a 1 x 1 grid, centre at a chosen point)
and compares the flags with the answer of plane geometry computed here, independently:
  * a cube seen face-on: flagged exactly where the ray passes within u of an edge of the lit
    face in the image plane (the face's own diagonal included, the side faces edge-on along the
    silhouette), never because of the unseen back face;
  * a lone plate: rays just inside or just outside its outer edges;
  * coincident layers: a two-sided sheet (opposite windings) is not a tie, a doubled sheet with
    the same winding always is; two parallel sheets tie below 2 tau apart and not above;
  * edges of a sheet behind the closest hit do not count;
  * a grazing plate is flagged;
  * an entry plane within tau of a lit facet, in front of it or just behind it, is flagged, one
    farther away is not;
  * the uncertainty grows at an interaction: after a 45-degree mirror, a ray meeting a second
    plate 1.5 u from its edge is flagged (u there is (sqrt(2) + 1) LAT L), one 3.5 u away is not.
Mutations of the rules (the edge or near rule without the factor L, back-facing layers counted
as ties, no growth of u at an interaction, degenerate paths kept in the adjoint) each fail a pin.
"""
import numpy as np

import oracle
import srp_inputs as si

Z = np.float32(0.2)


def scene_size(V):
    return 2.0 * np.linalg.norm(V - V.mean(0), axis=1).max()


def single_rays(points, sun, start_dist):
    """Caller frames [n][12] whose pixel-(0,0) centre (nu = nv = 1, no jitter) lies at
    points[i] + start_dist * sun (the ray then travels along -sun through points[i])."""
    sun = np.asarray(sun, float) / np.linalg.norm(sun)
    b1 = np.cross(sun, [1.0, 0, 0] if abs(sun[0]) < 0.9 else [0, 1.0, 0])
    b1 /= np.linalg.norm(b1)
    b2 = np.cross(sun, b1)
    h = 1e-3  # pixel size (the weight is irrelevant to the flags)
    fr = np.zeros((len(points), 12))
    for i, p in enumerate(points):
        o = np.asarray(p, float) + start_dist * sun
        fr[i, 0:3], fr[i, 3:6] = b1, b2
        fr[i, 6:9] = o - 0.5 * h * b1 - 0.5 * h * b2
        fr[i, 9] = fr[i, 10] = h
    return fr


def flags(mesh_v, mesh_t, points, sun, start_dist, bounces=1):
    n = len(points)
    fr = single_rays(points, sun, start_dist)
    sd = np.tile(np.asarray(sun, float) / np.linalg.norm(sun), (n, 1))
    z = np.full(len(mesh_t), Z, np.float32)
    res = oracle.trace(mesh_v, mesh_t, z, z, sd, nu=1, nv=1, bounces=bounces, jitter=False, frames_in=fr,
                       records=True)
    return res.degen[:, 0, 0].astype(bool), res.hit_prim[:, 0, 0]


def seg_dist(p, a, b):
    ab, ap = b - a, p - a
    s = np.clip(ap @ ab / (ab @ ab), 0.0, 1.0)
    return np.linalg.norm(a + s * ab - p)


def test_cube_face_on_edges_and_diagonal():
    faces = si.box_faces((-0.5, -0.5, -0.5), (0.5, 0.5, 0.5), 1)
    V = np.concatenate([f[0] for f in faces])
    T = np.concatenate([f[1] + 4 * i for i, f in enumerate(faces)]).astype(np.int32)
    L = scene_size(V)
    th = oracle.degen_thresholds()["lat"] * L
    # the lit face z = +0.5 (light along -z); its triangles' edges in the image plane (x, y)
    top = [t for t in T if np.allclose(V[t][:, 2], 0.5)]
    assert len(top) == 2
    edges = []
    for t in top:
        for a, b in ((0, 1), (1, 2), (2, 0)):
            edges.append((V[t[a], :2], V[t[b], :2]))
    rng = np.random.default_rng(5)
    pts = list(rng.uniform(-0.45, 0.45, (200, 2)))
    # points at chosen distances from the silhouette, the diagonal and the corners
    for off in (0.0, 0.3, 0.7, 1.5, 3.0, 30.0):
        d = off * th
        pts += [(0.5 - d, 0.13), (-0.5 + d, -0.21), (0.31, 0.5 - d), (-0.17, -0.5 + d), (0.5 - d, 0.5 - d)]
        pts += [(0.2 + d / np.sqrt(2), 0.2 - d / np.sqrt(2)), (-0.2 - d / np.sqrt(2), -0.2 + d / np.sqrt(2)),
                (0.2 - d / np.sqrt(2), 0.2 + d / np.sqrt(2))]
    pts = np.array(pts)
    dist = np.array([min(seg_dist(p, a, b) for a, b in edges) for p in pts])
    keep = (dist < 0.9 * th) | (dist > 1.1 * th)  # stay clear of the threshold itself
    pts, dist = pts[keep], dist[keep]
    P3 = np.column_stack([pts, np.full(len(pts), 0.5)])
    deg, hit = flags(V, T, P3, [0, 0, 1.0], 2.0)
    expect = dist < th
    assert expect.sum() >= 20 and (~expect).sum() >= 150
    assert np.array_equal(deg, expect), np.argwhere(deg != expect)[:5]
    # every ray hits the lit face (its two triangles), never the unseen one behind
    assert set(hit.tolist()) <= {int(np.flatnonzero((T == top[0]).all(1))[0]), int(np.flatnonzero((T == top[1]).all(1))[0])}


def test_plate_outer_edges():
    """A lone plate: its outer edges have no neighbour across them and no edge-on face beside them,
    so only the edge rule can flag a ray that passes just inside (a hit) or just outside (a miss)."""
    m = si.plate(3.0, 2.0)
    L = scene_size(m.verts)
    th = oracle.degen_thresholds()["lat"] * L
    pts, expect = [], []
    for off in (0.3, 0.7, 1.5, 3.0):
        for sgn in (-1.0, 1.0):  # inside, outside
            d = sgn * off * th
            pts += [(1.5 + d, 0.4, 0.0), (-1.5 - d, -0.3, 0.0), (0.55, 1.0 + d, 0.0), (-0.45, -1.0 - d, 0.0)]
            expect += [off < 1.0] * 4
    deg, hit = flags(m.verts, m.tris, pts, [0, 0, 1.0], 1.0)
    assert np.array_equal(deg, np.array(expect))
    assert ((hit >= 0) == np.tile(np.repeat([True, False], 4), 4)).all()


def test_coincident_layers():
    v, t = si.quad_grid((-1, -1, 0), (2, 0, 0), (0, 2, 0), 1, 1)  # faces +z
    L_single = scene_size(v)
    dt = oracle.degen_thresholds()
    tau = (dt["depth"] + dt["lat"]) * L_single  # normal incidence
    rng = np.random.default_rng(1)
    pts = np.column_stack([rng.uniform(-0.6, 0.6, (60, 2)), np.zeros(60)])
    pts = pts[np.abs(pts[:, 0] - pts[:, 1]) > 0.05]  # clear of the shared diagonal (x = y)
    # two-sided sheet: the back layer never faces the light, so no tie
    vb, tb = si.two_sided(v, t)
    V2 = np.concatenate([v, vb])
    T2 = np.concatenate([t, tb + len(v)]).astype(np.int32)
    deg, hit = flags(V2, T2, pts, [0, 0, 1.0], 1.0)
    assert not deg.any() and (hit < 2).all()
    # the same layer twice with the same winding: an exact tie everywhere (lower index wins)
    T3 = np.concatenate([t, t + len(v)]).astype(np.int32)
    deg, hit = flags(np.concatenate([v, v]), T3, pts, [0, 0, 1.0], 1.0)
    assert deg.all() and (hit < 2).all()
    # two parallel sheets dz apart: a tie below tau_f + tau_hit = 2 tau, distinct hits above
    for frac, tied in ((0.4, True), (0.75, True), (2.5, False)):
        dz = frac * 2 * tau  # L grows by dz/2 at most: well inside the margins
        v2 = v + np.array([0, 0, -dz])
        deg, hit = flags(np.concatenate([v, v2]), T3, pts, [0, 0, 1.0], 1.0)
        assert bool(deg.all()) == tied and not (deg.any() and not tied)
        assert (hit < 2).all()  # the upper sheet is closer either way


def test_edges_behind_the_hit_do_not_count():
    """A sheet behind the lit one, triangulated along the other diagonal: rays along its diagonal
    are not flagged (it lies beyond the closest hit), rays along the lit sheet's diagonal are."""
    v, t = si.quad_grid((-1, -1, 0), (2, 0, 0), (0, 2, 0), 1, 1)  # diagonal x = y, faces +z
    vb, tb = si.quad_grid((1, -1, -0.5), (0, 2, 0), (-2, 0, 0), 1, 1)  # diagonal x = -y, faces +z
    V = np.concatenate([v, vb])
    T = np.concatenate([t, tb + len(v)]).astype(np.int32)
    s = np.linspace(-0.6, 0.6, 13)
    s = s[np.abs(s) > 0.05]
    on_back = np.column_stack([s, -s, np.zeros(len(s))])
    on_front = np.column_stack([s, s, np.zeros(len(s))])
    deg, hit = flags(V, T, on_back, [0, 0, 1.0], 1.0)
    assert not deg.any() and (hit < 2).all()
    deg, hit = flags(V, T, on_front, [0, 0, 1.0], 1.0)
    assert deg.all()


def test_grazing_plate_flagged():
    graze = oracle.degen_thresholds()["graze"]
    for cos_t, grazing in ((0.5 * graze, True), (0.2, False)):
        tilt = np.rad2deg(np.arccos(cos_t))  # plate normal at angle tilt from the light
        m = si.plate(1.0, 1.0, tilt_deg=tilt)
        n = np.cross(m.verts[m.tris[0, 1]] - m.verts[m.tris[0, 0]], m.verts[m.tris[0, 2]] - m.verts[m.tris[0, 0]])
        n /= np.linalg.norm(n)
        # ray through the plate's centre region, away from the diagonal
        p = np.array([0.2, 0.0, 0.0]) + 0.0 * n
        sun = np.array([0, 0, 1.0])
        assert abs(n @ sun - cos_t) < 1e-9
        deg, hit = flags(m.verts, m.tris, [p], sun, 2.0)
        assert bool(deg[0]) == grazing
        assert hit[0] >= 0


def test_entry_plane_near_a_lit_facet():
    m = si.plate(4.0, 4.0)  # L = 5.7 m, so thresholds in metres differ from those in units of L
    L = scene_size(m.verts)
    dt = oracle.degen_thresholds()
    tau = (dt["depth"] + dt["lat"]) * L  # normal incidence
    p = [[0.25, -0.1, 0.0]]
    for h, flagged in ((0.4 * tau, True), (3.0 * tau, False)):
        deg, hit = flags(m.verts, m.tris, p, [0, 0, 1.0], h)
        assert bool(deg[0]) == flagged and hit[0] >= 0
        # the ray starting just behind the facet's plane misses it; an FP32 walk might not
        deg, hit = flags(m.verts, m.tris, p, [0, 0, 1.0], -h)
        assert bool(deg[0]) == flagged and hit[0] < 0


def test_hit_points_lie_on_the_hit_facets():
    m = si.box_wing()
    rs, rd = si.materials(m.n_tris, 1)
    sun = si.fibonacci_dirs(8)
    nu = nv = 48
    res = oracle.trace(m.verts, m.tris, rs, rd, sun, nu=nu, nv=nv, bounces=3, seed=4, records=True)
    fr = oracle.frames(m.verts, sun, nu, nv)
    V = m.verts
    L = scene_size(V)
    n_checked = 0
    for j in range(len(sun)):
        for q in range(nu * nv):
            for b in range(3):
                f = res.hit_prim[j, q, b]
                x = res.hit_x[j, q, b]
                if f < 0:
                    assert np.isnan(x).all()
                    continue
                v0, v1, v2 = V[m.tris[f]]
                n = np.cross(v1 - v0, v2 - v0)
                # on the plane and inside the triangle (barycentrics by least squares)
                assert abs((x - v0) @ n) / np.linalg.norm(n) < 1e-12 * L
                A = np.column_stack([v1 - v0, v2 - v0])
                uv = np.linalg.lstsq(A, x - v0, rcond=None)[0]
                assert uv.min() > -1e-9 and uv.sum() < 1 + 1e-9
                if b == 0:
                    # a primary hit lies on the pixel's ray: perpendicular offset from the frame
                    # origin matches the jittered pixel position within the pixel
                    u, v, o0, du, dv = fr[j, :3], fr[j, 3:6], fr[j, 6:9], fr[j, 9], fr[j, 10]
                    i, k = q % nu, q // nu
                    a, bb = (x - o0) @ u / du - i, (x - o0) @ v / dv - k
                    assert -1e-9 <= a <= 1 + 1e-9 and -1e-9 <= bb <= 1 + 1e-9
                n_checked += 1
    assert n_checked > 5000


def test_adjoint_without_degenerate_paths():
    """Leaving out degenerate paths: the mask equals the forward records' degenerate paths, and the
    full gradient is the masked one plus the gradient of the left-out paths alone."""
    m = si.meo_satellite(bus_n=6, cyl_sides=16, panel_n=4, dish_rings=6, dish_sectors=16)
    rs, rd = si.materials(m.n_tris, 1)
    sun = si.fibonacci_dirs(64)[[5, 40]]
    nu = nv = 48
    kw = dict(nu=nu, nv=nv, bounces=3, seed=9)
    gF = np.random.default_rng(2).standard_normal((2, 3))
    gT = np.random.default_rng(3).standard_normal((2, 3))
    full = oracle.trace_adjoint_rho(m.verts, m.tris, rs, rd, sun, gF, gT, **kw)
    gs, gd, mask = oracle.trace_adjoint_rho(m.verts, m.tris, rs, rd, sun, gF, gT, drop_degenerate=True, **kw)
    rec = oracle.trace(m.verts, m.tris, rs, rd, sun, records=True, **kw)
    assert np.array_equal(mask, rec.path_degenerate())
    assert 0 < mask.sum() < 0.2 * mask.size
    rest_s = np.zeros(m.n_tris)
    rest_d = np.zeros(m.n_tris)
    for j in range(2):
        pix = np.flatnonzero(mask[j])
        if len(pix) == 0:
            continue
        a, b = oracle.trace_adjoint_rho(m.verts, m.tris, rs, rd, sun[j:j + 1], gF[j:j + 1], gT[j:j + 1], pix=pix,
                                        dir_index_base=j, **kw)
        rest_s += a
        rest_d += b
    scale = np.abs(full[0]).max() + np.abs(full[1]).max()
    assert np.abs(gs + rest_s - full[0]).max() < 1e-12 * scale
    assert np.abs(gd + rest_d - full[1]).max() < 1e-12 * scale


def test_uncertainty_grows_at_an_interaction():
    """A mirror at 45 degrees (plane y + z = 0, facing +y+z) sends light travelling along -z off
    along +y to a plate in y = 2 facing -y whose lower edge lies at z = ze.  A primary ray at
    (x0, y0) leaves the mirror from (x0, y0, -y0) + eps n (eps = 1e-5 L) and meets the plate at
    z = -y0 + eps / sqrt(2), a distance delta above the edge.  The second segment carries
    u2 = u1 / cos(45) + LAT L, so delta = 1.5 u1 is flagged there while the primary segment is
    not, and delta = 3.5 u1 is flagged nowhere."""
    vm, tm = si.quad_grid((-1, -1, 1), (2, 0, 0), (0, 2, -2), 1, 1)  # mirror, faces +y+z
    ze = -0.2
    vb, tb = si.quad_grid((-1, 2, ze), (2, 0, 0), (0, 0, 2), 1, 1)    # plate, faces -y
    V = np.concatenate([vm, vb])
    T = np.concatenate([tm, tb + len(vm)]).astype(np.int32)
    L = scene_size(V)
    u1 = oracle.degen_thresholds()["lat"] * L
    u2 = u1 * np.sqrt(2.0) + u1
    assert np.isclose(oracle.degeneracy_uncertainty(L, [np.sqrt(0.5)])[1], u2)
    eps = 1e-5 * L
    pts, expect = [], []
    for frac, flagged in ((1.5, True), (3.5, False)):
        delta = frac * u1
        y0 = -(ze + delta) + eps / np.sqrt(2.0)
        pts.append((0.3, y0, -y0))
        expect.append(flagged)
    n = len(pts)
    fr = single_rays(pts, [0, 0, 1.0], 3.0)
    sd = np.tile([0, 0, 1.0], (n, 1))
    rs = np.array([1.0, 1.0, 0.0, 0.0], np.float32)  # mirror: rho_s = 1; plate: black
    rd = np.zeros(4, np.float32)
    res = oracle.trace(V, T, rs, rd, sd, nu=1, nv=1, bounces=2, jitter=False, frames_in=fr, records=True)
    assert (res.hit_prim[:, 0, 0] < 2).all() and (res.hit_prim[:, 0, 1] >= 2).all()
    # the second hit lies where the geometry above puts it
    for q in range(n):
        assert abs(res.hit_x[q, 0, 1, 2] - ze - (1.5, 3.5)[q] * u1) < 1e-3 * u1
    assert not res.degen[:, 0, 0].any()
    assert np.array_equal(res.degen[:, 0, 1].astype(bool), np.array(expect))
