"""Pins of the oracle's hinge-angle gradient split: the pathwise part (the frozen-visibility
estimator without footprint factor, each path at its image position with its facet sequence) and
the visibility-edge part by edge sampling (oracle_edge_term), against closed forms (CPU only).

  * an unoccluded hinged plate (light along -z, one bounce): the pathwise part is the derivative of
    the per-area deposit times the projected area, the edge part the deposit times the derivative
    of the projected area; together the derivative of the flat-plate closed form;
  * the same plate half behind a fixed absorbing plate: the edge part is the deposit times the
    derivative of the VISIBLE projected area, which the hidden stretch of the moving edge does not
    change;
  * two-sided sheets and shared edges count once; an edge on the hinge line contributes nothing;
  * the box-wing at three bounces (panels shadowed by the bus, reflections): pathwise + edge agrees
    with a central difference of the full estimator over a fine jittered grid.
"""
import numpy as np

import oracle
import srp_inputs as si
from oracle.design import apply_hinges

PHI, C = 1361.0, 299792458.0


def plate_deposit(theta, rs, rd):
    """Force per unit projected area (N/m^2) of a plate with normal (0, -sin, cos) under light
    travelling along -z, one bounce: (Phi/c) [(1 - rs) s + 2 (rs c + rd/3) n_in], c = cos(theta)."""
    n_out = np.array([0.0, -np.sin(theta), np.cos(theta)])
    s_hat = np.array([0.0, 0.0, -1.0])
    c = float(s_hat @ -n_out)
    return PHI / C * ((1 - rs) * s_hat + 2 * (rs * c + rd / 3) * (-n_out))


def hinged_plate(extra=None):
    """Plate x in [-0.6, 0.6], y in [0.2, 1.0] at z = 0 facing +z, carried by hinge 0 (the x axis)."""
    v, t = si.quad_grid((-0.6, 0.2, 0.0), (1.2, 0, 0), (0, 0.8, 0), 1, 1)
    vh = np.zeros(len(v), np.int32)
    if extra is not None:
        ve, te = extra
        t = np.concatenate([t, te + len(v)])
        v = np.concatenate([v, ve])
        vh = np.concatenate([vh, np.full(len(ve), -1, np.int32)])
    return v, t.astype(np.int32), vh


def frozen_pathwise(V_of, tris, rs, rd, sun, fr, nu, nv, theta0, h=1e-6, **kw):
    """Central difference of the frozen-visibility estimator without footprint (the pathwise part)."""
    V0 = V_of(theta0)
    ref = oracle.trace(V0, tris, rs, rd, sun, nu=nu, nv=nv, frames_in=fr, records=True, **kw)
    out = []
    for sgn in (1, -1):
        F, T = oracle.trace_frozen(V_of(theta0 + sgn * h), V0, tris, rs, rd, sun, ref.hit_prim, fr, nu=nu, nv=nv,
                                   footprint=False, **kw)
        out.append(np.concatenate([F, T], 1))
    return (out[0] - out[1]) / (2 * h)


def test_unoccluded_plate_closed_form():
    v, t, vh = hinged_plate()
    rs = np.full(2, 0.3, np.float32)
    rd = np.full(2, 0.25, np.float32)
    sun = np.array([[0.0, 0.0, 1.0]])
    for theta0 in (0.0, 0.4):
        V_of = lambda th: apply_hinges(v, vh, [[0, 0, 0]], [[1.0, 0, 0]], [th])
        V0 = V_of(theta0)
        fr = oracle.frames(V0, sun, 60, 40)  # the grid covers the plate's image exactly
        kw = dict(bounces=1, jitter=False)
        path = frozen_pathwise(V_of, t, rs, rd, sun, fr, 60, 40, theta0, **kw)[0, :3]
        edge, n_edges = oracle.edge_term(V0, t, vh, [[0, 0, 0]], [[1.0, 0, 0]], rs, rd, sun, fr, bounces=1, samples=8)
        assert n_edges == 5  # four sides and the diagonal
        area = 0.96 * np.cos(theta0)
        h = 1e-6
        d_dep = (plate_deposit(theta0 + h, float(rs[0]), float(rd[0])) - plate_deposit(theta0 - h, float(rs[0]), float(rd[0]))) / (2 * h)
        dep = plate_deposit(theta0, float(rs[0]), float(rd[0]))
        assert np.allclose(path, area * d_dep, rtol=1e-6, atol=1e-6 * np.abs(area * d_dep).max())
        expect_edge = dep * (-0.96 * np.sin(theta0))
        scale = max(np.abs(dep).max() * 0.96, 1e-30)
        assert np.abs(edge[0, 0, :3] - expect_edge).max() <= 1e-9 * scale


def test_partially_occluded_plate():
    """A fixed absorbing square in front of the plate hides part of its far edge: only the visible
    part of the moving edge changes the force."""
    # occluder at z = 2, facing +z, covering x in [-0.2, 0.3], y in [0.5, 1.5] (rigid)
    vo, to = si.quad_grid((-0.2, 0.5, 2.0), (0.5, 0, 0), (0, 1.0, 0), 1, 1)
    v, t, vh = hinged_plate((vo, to))
    rs = np.array([0.3, 0.3, 0.0, 0.0], np.float32)
    rd = np.array([0.25, 0.25, 0.0, 0.0], np.float32)
    sun = np.array([[0.0, 0.0, 1.0]])
    theta0 = 0.4
    V0 = apply_hinges(v, vh, [[0, 0, 0]], [[1.0, 0, 0]], [theta0])
    fr = oracle.frames(V0, sun, 8, 8)
    # M = 4800 per edge puts the far edge's hidden stretch (x in [-0.2, 0.3]) on stratum boundaries
    edge, n_edges = oracle.edge_term(V0, t, vh, [[0, 0, 0]], [[1.0, 0, 0]], rs, rd, sun, fr, bounces=1, samples=4800)
    assert n_edges == 5
    dep = plate_deposit(theta0, float(rs[0]), float(rd[0]))
    # visible projected area: 1.2 x 0.8 cos - 0.5 x (cos - 0.5): derivative (-0.96 + 0.5) sin
    expect = dep * (-0.96 + 0.5) * np.sin(theta0)
    assert np.abs(edge[0, 0, :3] - expect).max() <= 1e-3 * np.abs(expect).max()
    # without the occluder the same edges give the full area change
    edge_free, _ = oracle.edge_term(V0[:4], t[:2], vh[:4], [[0, 0, 0]], [[1.0, 0, 0]], rs[:2], rd[:2], sun, fr,
                                    bounces=1, samples=4800)
    assert np.abs(edge_free[0, 0, :3] - dep * (-0.96) * np.sin(theta0)).max() <= 1e-3 * np.abs(dep).max() * 0.96


def test_two_sided_sheet_counts_edges_once():
    v, t, vh = hinged_plate()
    vb, tb = si.two_sided(v, t)
    V2 = np.concatenate([v, vb])
    T2 = np.concatenate([t, tb + len(v)]).astype(np.int32)
    vh2 = np.zeros(len(V2), np.int32)
    rs = np.full(4, 0.3, np.float32)
    rd = np.full(4, 0.25, np.float32)
    sun = np.array([[0.0, 0.0, 1.0]])
    V0 = apply_hinges(V2, vh2, [[0, 0, 0]], [[1.0, 0, 0]], [0.4])
    fr = oracle.frames(V0, sun, 8, 8)
    e2, n2 = oracle.edge_term(V0, T2, vh2, [[0, 0, 0]], [[1.0, 0, 0]], rs, rd, sun, fr, bounces=1, samples=16)
    e1, n1 = oracle.edge_term(V0[:4], t, vh2[:4], [[0, 0, 0]], [[1.0, 0, 0]], rs[:2], rd[:2], sun, fr, bounces=1,
                              samples=16)
    assert n2 == n1 == 5
    assert np.allclose(e2, e1, rtol=1e-12, atol=0)
    # a plate whose near edge lies on the hinge line: that edge does not move
    v3, t3 = si.quad_grid((-0.6, 0.0, 0.0), (1.2, 0, 0), (0, 0.8, 0), 1, 1)
    vh3 = np.zeros(4, np.int32)
    V3 = apply_hinges(v3, vh3, [[0, 0, 0]], [[1.0, 0, 0]], [0.4])
    fr3 = oracle.frames(V3, sun, 8, 8)
    e3, _ = oracle.edge_term(V3, t3.astype(np.int32), vh3, [[0, 0, 0]], [[1.0, 0, 0]], rs[:2], rd[:2], sun, fr3,
                             bounces=1, samples=16)
    dep = plate_deposit(0.4, float(rs[0]), float(rd[0]))
    assert np.abs(e3[0, 0, :3] - dep * (-0.96) * np.sin(0.4)).max() <= 1e-9 * np.abs(dep).max()


def test_box_wing_three_bounces_against_full_difference():
    """Box-wing with both panels hinged (the bus shadows them for some directions, light reflects
    between bus and panels): pathwise + edge against a central difference (h = 0.01) of the full
    estimator, both averaged over four jittered 1024^2 grids, for four sun directions.  The full
    difference itself carries the grid's sampling error of the swept strips (about 1 %), and the
    secondary-visibility edges are not in the estimate."""
    m = si.box_wing()
    rs, rd = si.materials(m.n_tris, 1)
    sun = si.fibonacci_dirs(32)[[3, 11, 19, 27]]
    ang0 = np.array([0.3, -0.25])
    V_of = lambda a: apply_hinges(m.verts, m.vert_hinge, m.hinge_origin, m.hinge_axis, a)
    V0 = V_of(ang0)
    nu = nv = 1024
    fr = oracle.frames(V0, sun, nu, nv)
    seeds = (4, 5, 6, 7)
    est = np.zeros((2, 4, 3))
    path_only = np.zeros((2, 4, 3))
    fd = np.zeros((2, 4, 3))
    for seed in seeds:
        kw = dict(bounces=3, seed=seed)
        ref = oracle.trace(V0, m.tris, rs, rd, sun, nu=nu, nv=nv, frames_in=fr, records=True, **kw)
        edge, _ = oracle.edge_term(V0, m.tris, m.vert_hinge, m.hinge_origin, m.hinge_axis, rs, rd, sun, fr,
                                   samples=512, **kw)
        for k in range(2):
            vals = []
            for sgn in (1, -1):
                a = ang0.copy()
                a[k] += sgn * 1e-6
                F, _ = oracle.trace_frozen(V_of(a), V0, m.tris, rs, rd, sun, ref.hit_prim, fr, nu=nu, nv=nv,
                                           footprint=False, **kw)
                vals.append(F)
            path = (vals[0] - vals[1]) / 2e-6
            path_only[k] += path / len(seeds)
            est[k] += (path + edge[:, k, :3]) / len(seeds)
            full = []
            for sgn in (1, -1):
                a = ang0.copy()
                a[k] += sgn * 0.01
                full.append(oracle.trace(V_of(a), m.tris, rs, rd, sun, nu=nu, nv=nv, frames_in=fr, **kw).force)
            fd[k] += (full[0] - full[1]) / 0.02 / len(seeds)
    for k in range(2):
        err = np.linalg.norm(est[k] - fd[k]) / np.linalg.norm(fd[k])
        err_path = np.linalg.norm(path_only[k] - fd[k]) / np.linalg.norm(fd[k])
        print(f"hinge {k}: pathwise + edge vs full difference rel {err:.3e} (pathwise alone {err_path:.3e})")
        assert err <= 0.02 and err < 0.25 * err_path


def _panel(n):
    """The hinged plate of hinged_plate() split into n x n quads (2 triangles each)."""
    v, t = si.quad_grid((-0.6, 0.2, 0.0), (1.2, 0, 0), (0, 0.8, 0), n, n)
    return v, t.astype(np.int32), np.zeros(len(v), np.int32)


def _on_rim(p):
    return np.isclose(p[0], -0.6) or np.isclose(p[0], 0.6) or np.isclose(p[1], 0.2) or np.isclose(p[1], 1.0)


def test_smooth_edges_are_the_flat_interior_ones():
    """Counts on an n x n panel: 2n(n+1) + n^2 moving edges, of which the 4n rim edges are kept and
    the 3n^2 - 2n interior ones (the integrand is continuous across them) are left out; a crease, a
    material boundary and a p_spec boundary keep theirs; the two layers of a two-sided sheet are
    checked each on its own."""
    from oracle.edges import moving_edges, smooth_edge_mask
    n = 4
    v, t, vh = _panel(n)
    rs = np.full(len(t), 0.3, np.float32)
    rd = np.full(len(t), 0.25, np.float32)
    edges = moving_edges(v, t, vh)
    smooth = smooth_edge_mask(v, t, vh, rs, rd)
    assert len(edges) == 2 * n * (n + 1) + n * n
    assert smooth.sum() == 3 * n * n - 2 * n
    for (a, b, _, _), s in zip(edges, smooth):
        assert s == (not (_on_rim(v[a]) and _on_rim(v[b]) and
                          (np.isclose(v[a][0], v[b][0]) or np.isclose(v[a][1], v[b][1]))))
    # per-facet materials: every edge is a material boundary
    rs_r, rd_r = si.materials(len(t), 2)
    assert not smooth_edge_mask(v, t, vh, rs_r, rd_r).any()
    # one interior facet with another p_spec: its three edges are kept
    ps = np.full(len(t), 0.5, np.float32)
    assert smooth_edge_mask(v, t, vh, rs, rd, ps).sum() == 3 * n * n - 2 * n
    ps[2 * (n + 1)] = 0.6  # a triangle of the quad at (1, 1), interior for n = 4
    assert smooth_edge_mask(v, t, vh, rs, rd, ps).sum() == 3 * n * n - 2 * n - 3
    # a crease along the middle row of vertices: the n edges on the fold line are kept
    vf = v.copy()
    vf[:, 2] = np.maximum(vf[:, 1] - 0.6, 0.0) * 0.5
    assert smooth_edge_mask(vf, t, vh, rs, rd).sum() == 3 * n * n - 2 * n - n
    # two-sided sheet: each layer pairs on its own side
    vb, tb = si.two_sided(v, t)
    V2 = np.concatenate([v, vb])
    T2 = np.concatenate([t, tb + len(v)]).astype(np.int32)
    vh2 = np.zeros(len(V2), np.int32)
    rs2 = np.concatenate([rs, np.full(len(t), 0.1, np.float32)])
    rd2 = np.concatenate([rd, np.full(len(t), 0.2, np.float32)])
    s2 = smooth_edge_mask(V2, T2, vh2, rs2, rd2)
    assert len(s2) == len(edges) and (s2 == smooth).all()
    # an interior edge that a rigid facet also contains, or that a second (crossing) plane of the
    # same hinge passes through, is kept
    e_in = int(np.flatnonzero(smooth)[0])
    a, b = edges[e_in][0], edges[e_in][1]
    top, bottom = (v[a] + v[b]) / 2 + [0, 0, 0.3], (v[a] + v[b]) / 2 - [0, 0, 0.3]
    V3 = np.concatenate([v, [top, bottom]])
    mat3 = lambda k: (np.append(rs, [0.3] * k).astype(np.float32), np.append(rd, [0.25] * k).astype(np.float32))
    T3 = np.concatenate([t, [[a, b, len(v)]]]).astype(np.int32)
    vh3 = np.concatenate([vh, [-1, -1]]).astype(np.int32)
    s3 = smooth_edge_mask(V3, T3, vh3, *mat3(1))
    assert s3.sum() == smooth.sum() - 1 and not s3[e_in]
    T4 = np.concatenate([t, [[a, b, len(v)], [b, a, len(v) + 1]]]).astype(np.int32)
    vh4 = np.concatenate([vh, [0, 0]]).astype(np.int32)
    s4 = smooth_edge_mask(V3, T4, vh4, *mat3(2))
    assert not s4[e_in] and s4.sum() == smooth.sum() - 1


def test_leaving_out_smooth_edges_changes_the_estimate_by_order_delta():
    """The subdivided plate half behind the absorbing square, one and three bounces: with and
    without the interior edges the force agrees to rounding and the torque within 1e-3 (the left-out
    terms are 2 delta x deposit per side pair, delta = 1e-5 L); the closed form of
    test_partially_occluded_plate holds for the reduced edge set."""
    v, t, vh = _panel(4)
    vo, to = si.quad_grid((-0.2, 0.5, 2.0), (0.5, 0, 0), (0, 1.0, 0), 1, 1)
    V = np.concatenate([v, vo])
    T = np.concatenate([t, to + len(v)]).astype(np.int32)
    VH = np.concatenate([vh, np.full(4, -1, np.int32)])
    rs = np.concatenate([np.full(len(t), 0.3, np.float32), np.zeros(2, np.float32)])
    rd = np.concatenate([np.full(len(t), 0.25, np.float32), np.zeros(2, np.float32)])
    theta0 = 0.4
    V0 = apply_hinges(V, VH, [[0, 0, 0]], [[1.0, 0, 0]], [theta0])
    sun = np.array([[0.0, 0.0, 1.0], [0.3, -0.2, 0.93]])
    sun /= np.linalg.norm(sun, axis=1)[:, None]
    fr = oracle.frames(V0, sun, 8, 8)
    for bounces in (1, 3):
        kw = dict(bounces=bounces, samples=64)
        full, _ = oracle.edge_term(V0, T, VH, [[0, 0, 0]], [[1.0, 0, 0]], rs, rd, sun, fr, drop_smooth=False, **kw)
        red, _ = oracle.edge_term(V0, T, VH, [[0, 0, 0]], [[1.0, 0, 0]], rs, rd, sun, fr, **kw)
        assert np.abs(full[..., :3] - red[..., :3]).max() <= 1e-12 * np.abs(full[..., :3]).max()
        assert np.abs(full[..., 3:] - red[..., 3:]).max() <= 1e-3 * np.abs(full[..., 3:]).max()
        assert np.abs(full[..., 3:] - red[..., 3:]).max() > 0.0  # the interior edges were left out
    red, _ = oracle.edge_term(V0, T, VH, [[0, 0, 0]], [[1.0, 0, 0]], rs, rd, sun[:1], fr[:1], bounces=1, samples=4800)
    dep = plate_deposit(theta0, 0.3, 0.25)
    expect = dep * (-0.96 + 0.5) * np.sin(theta0)
    assert np.abs(red[0, 0, :3] - expect).max() <= 1e-3 * np.abs(expect).max()
