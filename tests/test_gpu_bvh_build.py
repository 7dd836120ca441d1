"""GPU BVH build (srp_scene_build_gpu, linear BVH) against the host-built SAH tree.

The closest hit with its index tie-break does not depend on the tree, so a scene whose BVH was
rebuilt on the GPU must give bit-identical forces, torques, hit records and surface-estimator
results, also after a hinge change refits the new tree; the oracle agrees as for the SAH tree.
"""
import numpy as np
import pytest

import oracle
import srp_inputs as si

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
        ref = oracle.trace(b.vertices(), m.tris, rs, rd, sun[:4], nu=256, nv=256, bounces=3, seed=31)
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
