"""GPU BVH build (srp_scene_build_gpu, linear BVH) against the host-built SAH tree.

The closest hit with its index tie-break does not depend on the tree, so a scene whose BVH was
rebuilt on the GPU must give bit-identical forces, torques, hit records and surface-estimator
results, also after a hinge change refits the new tree; the oracle agrees as for the SAH tree.
"""
import numpy as np
import pytest

import oracle
import srp_inputs as si
from oracle.design import apply_hinges

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def pair(mesh, rs, rd, angles=None):
    import paper_2602_10712_amd as p
    a = p.Scene.from_mesh(mesh)
    a.set_design(rs, rd, hinge_angles=angles)
    b = p.Scene.from_mesh(mesh)
    b.set_design(rs, rd, hinge_angles=angles)
    n_nodes, depth = p.srp_scene_build_gpu(b)
    return a, b, n_nodes, depth


def records(sc, sun, prm, pix):
    import paper_2602_10712_amd as p
    dev = torch.device("cuda")
    sd = torch.as_tensor(sun, dtype=torch.float64, device=dev).contiguous()
    px = torch.as_tensor(pix, dtype=torch.int64, device=dev)
    hp = torch.empty((len(sun), len(pix), prm.bounces), dtype=torch.int32, device=dev)
    rf = torch.empty((len(sun), len(pix), 3), dtype=torch.float32, device=dev)
    p.srp_trace_records(sc.handle, sd, prm, hp, rf, pix=px)
    torch.cuda.synchronize()
    return hp.cpu().numpy(), rf.cpu().numpy()


@pytest.mark.parametrize("full", [False, True])
def test_gpu_tree_gives_identical_traces(full):
    import paper_2602_10712_amd as p
    if full:
        m = si.meo_satellite()
    else:
        m = si.meo_satellite(bus_n=6, cyl_sides=16, panel_n=4, dish_rings=8, dish_sectors=16, strut_sides=6)
    rs, rd = si.materials(m.n_tris, 5)
    a, b, n_nodes, depth = pair(m, rs, rd, [0.1, -0.25])
    print(f"{m.n_tris} tris: GPU tree {n_nodes} nodes, depth {depth}; SAH tree {a.info()['n_nodes']} nodes, "
          f"depth {a.info()['depth']}")
    assert b.info()["n_nodes"] == n_nodes and b.info()["depth"] == depth
    sun = si.fibonacci_dirs(16)
    prm = p.TraceParams(nu=256, nv=256, bounces=3, seed=31)
    Fa, Ta = a.trace(sun, prm)
    Fb, Tb = b.trace(sun, prm)
    assert torch.equal(Fa, Fb) and torch.equal(Ta, Tb)
    pix = np.arange(0, 256 * 256, 37)
    ha, fa = records(a, sun, prm, pix)
    hb, fb = records(b, sun, prm, pix)
    assert np.array_equal(ha, hb) and np.array_equal(fa, fb)
    # the surface estimator's BVH walk
    dev = torch.device("cuda")
    sd = torch.as_tensor(sun, dtype=torch.float64, device=dev).contiguous()
    Ga = torch.empty((1, 16, 3), dtype=torch.float64, device=dev)
    Gb = torch.empty_like(Ga)
    p.srp_surface_estimate([a], sd, 4096, prm, Ga)
    p.srp_surface_estimate([b], sd, 4096, prm, Gb)
    torch.cuda.synchronize()
    assert torch.equal(Ga, Gb)
    # a hinge change refits each scene's own tree
    a.set_design(rs, rd, hinge_angles=[-0.3, 0.2])
    b.set_design(rs, rd, hinge_angles=[-0.3, 0.2])
    Fa, _ = a.trace(sun, prm)
    Fb, _ = b.trace(sun, prm)
    assert torch.equal(Fa, Fb)
    if not full:
        V = apply_hinges(m.verts, m.vert_hinge, m.hinge_origin, m.hinge_axis, [-0.3, 0.2])
        assert np.allclose(b.vertices(), V, rtol=0, atol=1e-12)
        ref = oracle.trace(V, m.tris, rs, rd, sun[:4], nu=256, nv=256, bounces=3, seed=31)
        rel = np.linalg.norm(Fb.cpu().numpy()[:4] - ref.force) / np.linalg.norm(ref.force)
        assert rel <= 1e-4
    a.close()
    b.close()


def test_statistics_follow_the_gpu_tree():
    """The instrumented host traversal reads the GPU-built records back: the same hits (segments per
    ray) as on the SAH tree, with the new tree's node counts."""
    import paper_2602_10712_amd as p
    m2 = si.meo_satellite(bus_n=6, cyl_sides=16, panel_n=4, dish_rings=8, dish_sectors=16, strut_sides=6)
    rs, rd = si.materials(m2.n_tris, 5)
    a, b, _, _ = pair(m2, rs, rd, [0.2, 0.1])
    sun = si.fibonacci_dirs(8)
    prm = p.TraceParams(nu=128, nv=128, bounces=3, seed=3)
    sa = p.ray_stats(a, sun, prm, n_dirs=8, pixel_stride=7)
    b.build_gpu()
    sb = p.ray_stats(b, sun, prm, n_dirs=8, pixel_stride=7)
    print(f"SAH tree: {sa['nodes_per_segment']:.2f} nodes/segment; GPU tree: {sb['nodes_per_segment']:.2f}")
    assert sa["segments_per_ray"] == sb["segments_per_ray"]
    assert sb["nodes_per_segment"] > 0
    a.close()
    b.close()


def test_gpu_build_small_mesh_refused():
    import paper_2602_10712_amd as p
    m = si.plate(1.0, 1.0)
    sc = p.Scene.from_mesh(m)
    with pytest.raises(p.SRPError) as e:
        p.srp_scene_build_gpu(sc)
    assert e.value.status == -5
    sc.close()


def _warp(V):
    """A smooth deformation close to the identity (no facet collapses)."""
    return V + 0.03 * np.stack([np.sin(1.3 * V[:, 1]), np.sin(0.7 * V[:, 2]), np.sin(0.9 * V[:, 0])], 1)


@pytest.mark.parametrize("gpu_tree", [False, True])
def test_device_refit_matches_a_fresh_build(gpu_tree):
    """A hinge change refits the boxes of the kept tree on the device (SAH tree from the host, or
    the GPU-built tree): traces and hit records are bit-identical to a scene built from scratch on
    the rotated vertices, whose closest hits do not depend on the tree."""
    import dataclasses
    import paper_2602_10712_amd as p
    m = si.meo_satellite()
    rs, rd = si.materials(m.n_tris, 6)
    ang = [0.45, -0.6]
    a = p.Scene.from_mesh(m)
    if gpu_tree:
        a.build_gpu()
    a.set_design(rs, rd, hinge_angles=ang)
    V = apply_hinges(m.verts, m.vert_hinge, m.hinge_origin, m.hinge_axis, ang)
    c = p.Scene.from_mesh(dataclasses.replace(m, verts=V))
    c.set_design(rs, rd)
    assert np.array_equal(a.vertices(), c.vertices())
    sun = si.fibonacci_dirs(32)
    prm = p.TraceParams(nu=256, nv=256, bounces=3, seed=17)
    Fa, Ta = a.trace(sun, prm)
    Fc, Tc = c.trace(sun, prm)
    assert torch.equal(Fa, Fc) and torch.equal(Ta, Tc)
    pix = np.arange(0, 256 * 256, 29)
    ha, fa = records(a, sun, prm, pix)
    hc, fc = records(c, sun, prm, pix)
    assert np.array_equal(ha, hc) and np.array_equal(fa, fc)
    a.close()
    c.close()


def test_set_vertices_refit_and_rebuild():
    """srp_scene_set_vertices: a new rest pose under the same hinge angles and materials, with the
    tree refitted on the device or rebuilt on the host, traces bit-identically to a scene created
    from the new pose; the oracle agrees on a small mesh; bad input leaves the scene as it was."""
    import dataclasses
    import paper_2602_10712_amd as p
    for full in (True, False):
        if full:
            m = si.meo_satellite()
        else:
            m = si.meo_satellite(bus_n=6, cyl_sides=16, panel_n=4, dish_rings=8, dish_sectors=16, strut_sides=6)
        rs, rd = si.materials(m.n_tris, 8)
        ang = [0.2, -0.35]
        W = _warp(m.verts)
        c = p.Scene.from_mesh(dataclasses.replace(m, verts=W))
        c.set_design(rs, rd, hinge_angles=ang)
        sun = si.fibonacci_dirs(16)
        prm = p.TraceParams(nu=256, nv=256, bounces=3, seed=23)
        Fc, Tc = c.trace(sun, prm)
        for rebuild in (False, True):
            a = p.Scene.from_mesh(m)
            a.set_design(rs, rd, hinge_angles=ang)
            a.set_vertices(W, rebuild=rebuild)
            assert np.array_equal(a.vertices(), c.vertices())
            Fa, Ta = a.trace(sun, prm)
            assert torch.equal(Fa, Fc) and torch.equal(Ta, Tc), (full, rebuild)
            # the hinge angles stay applied on top of the new rest pose
            a.set_design(rs, rd, hinge_angles=[0.0, 0.0])
            assert np.allclose(a.vertices(), W, rtol=0, atol=1e-12)
            a.close()
        if not full:
            Vw = apply_hinges(W, m.vert_hinge, m.hinge_origin, m.hinge_axis, ang)
            assert np.allclose(c.vertices(), Vw, rtol=0, atol=1e-12)
            ref = oracle.trace(Vw, m.tris, rs, rd, sun[:4], nu=256, nv=256, bounces=3, seed=23)
            rel = np.linalg.norm(Fc.cpu().numpy()[:4] - ref.force) / np.linalg.norm(ref.force)
            assert rel <= 1e-4
        c.close()
    # errors: size, mode, a non-finite vertex, a collapsed facet; the scene keeps its geometry
    a = p.Scene.from_mesh(m)
    a.set_design(rs, rd, hinge_angles=ang)
    V0 = a.vertices()
    F0, _ = a.trace(sun, prm)
    with pytest.raises(p.SRPError) as e:
        a.set_vertices(W[:-1])
    assert e.value.status == -1
    with pytest.raises(p.SRPError) as e:
        p.srp_scene_set_vertices(a.handle, W, mode=2)
    assert e.value.status == -1
    bad = W.copy()
    bad[5, 1] = np.nan
    with pytest.raises(p.SRPError) as e:
        a.set_vertices(bad)
    assert e.value.status == -4
    bad = W.copy()
    t0 = m.tris[3]
    bad[t0[1]] = bad[t0[0]]
    with pytest.raises(p.SRPError) as e:
        a.set_vertices(bad, rebuild=True)
    assert e.value.status == -4
    assert np.array_equal(a.vertices(), V0)
    F1, _ = a.trace(sun, prm)
    assert torch.equal(F0, F1)
    a.close()


def test_edge_terms_follow_tree_and_pose_changes():
    """Hinge gradients with visibility-edge terms under one material per part (the flat panels'
    interior edges skipped): bit-identical on the GPU-built tree and the SAH tree (the edge
    classification reads the facets' packed materials through the new record order), and after
    srp_scene_set_vertices with a tree refit or a host rebuild to a scene created from the new pose
    (the facet pairs of the moving edges are re-derived from the new rest pose)."""
    import dataclasses
    import paper_2602_10712_amd as p
    m = si.meo_satellite()
    rs, rd = si.design_materials(m, [0.1, -0.25, 0.2, 0.3, 0.1, 0.4, 0.25, 0.15])
    ang = [0.1, -0.25]
    sun = si.fibonacci_dirs(16)
    rng = np.random.default_rng(12)
    gF = rng.standard_normal((16, 3))
    gT = rng.standard_normal((16, 3))
    prm = p.TraceParams(nu=128, nv=128, bounces=3, seed=17, edge_samples=4)
    a, b, _, _ = pair(m, rs, rd, ang)
    ha = a.adjoint(sun, prm, gF, gT)[2]
    hb = b.adjoint(sun, prm, gF, gT)[2]
    h0 = a.adjoint(sun, p.TraceParams(nu=128, nv=128, bounces=3, seed=17), gF, gT)[2]
    torch.cuda.synchronize()
    print(f"hinge gradients: SAH tree {ha.cpu().numpy()}, GPU tree {hb.cpu().numpy()}, pathwise only "
          f"{h0.cpu().numpy()}")
    assert torch.equal(ha, hb)
    assert not torch.equal(ha, h0)
    W = _warp(m.verts)
    c = p.Scene.from_mesh(dataclasses.replace(m, verts=W))
    c.set_design(rs, rd, hinge_angles=ang)
    hc = c.adjoint(sun, prm, gF, gT)[2]
    for rebuild in (False, True):
        a.set_vertices(W, rebuild=rebuild)
        hw = a.adjoint(sun, prm, gF, gT)[2]
        torch.cuda.synchronize()
        assert torch.equal(hw, hc), rebuild
    for s in (a, b, c):
        s.close()
