"""GPU surface-sampling estimator (srp_surface_estimate) vs the FP64 oracle, through the C ABI.

Same Philox counters on both sides, so the samples are the same:
  * per-sample records (facet, gathered facets, sunlit flags) identical wherever the oracle does not
    flag the sample degenerate; the sample mean's force and torque within 1e-4 relative L2;
  * the BVH walk and the brute-force test of every triangle give bit-identical results;
  * several designs in one call ("multi-world") equal each design's own call bit for bit;
  * ragged sample counts, one bounce, invalid arguments;
  * at the benchmark's sample count on the 20.6k-triangle satellite, the records of the first
    512 samples of each direction match the oracle;
  * the variance-reduction options (stratified surface, plain-MC hemisphere directions, both):
    records, force and torque against the oracle in each, BVH walk = brute force bit for bit.
"""
import numpy as np
import pytest

import oracle
import srp_inputs as si
from oracle.design import apply_hinges

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def run(scenes, sun, n, params, brute, records=True):
    import paper_2602_10712_amd as p
    dev = torch.device("cuda")
    S, D = len(scenes), len(sun)
    sd = torch.as_tensor(sun, dtype=torch.float64, device=dev).contiguous()
    F = torch.empty((S, D, 3), dtype=torch.float64, device=dev)
    T = torch.empty_like(F)
    rf = rl = rh = None
    if records:
        rf = torch.full((S, D, n), -7, dtype=torch.int32, device=dev)
        rl = torch.full((S, D, n), -7, dtype=torch.int32, device=dev)
        rh = torch.full((S, D, n, max(params.bounces - 1, 1)), -7, dtype=torch.int32, device=dev)
    p.srp_surface_estimate(scenes, sd, n, params, F, T, brute_force=brute, rec_facet=rf, rec_hits=rh, rec_lit=rl)
    torch.cuda.synchronize()
    out = {"F": F.cpu().numpy(), "T": T.cpu().numpy()}
    if records:
        out.update(facet=rf.cpu().numpy(), lit=rl.cpu().numpy(), hits=rh.cpu().numpy()[..., :params.bounces - 1])
    return out


def check_records(g, ref, bounces, min_ok=0.99):
    """Records identical on every sample the oracle does not flag; samples start on the surface, so
    their shadow and gathering rays sometimes begin within the position uncertainty of a
    neighbouring facet's edge (flagged); the flagged ones that still agree are reported."""
    ok = ref.degen == 0
    assert ok.mean() > min_ok, f"degenerate fraction {1 - ok.mean():.4f}"
    assert np.array_equal(g["facet"][ok], ref.facet[ok])
    assert np.array_equal(g["lit"][ok], ref.lit[ok])
    if bounces > 1:
        assert np.array_equal(g["hits"][ok], ref.hits[ok])
    same = (g["facet"] == ref.facet) & (g["lit"] == ref.lit)
    if bounces > 1:
        same &= (g["hits"] == ref.hits).all(-1)
    print(f"  flagged {1 - ok.mean():.4f}; of those, records differ in {(~same[~ok]).sum()} of {(~ok).sum()}")
    return 1 - ok.mean()


def make(mesh, rs, rd, angles=None):
    import paper_2602_10712_amd as p
    sc = p.Scene.from_mesh(mesh)
    sc.set_design(rs, rd, hinge_angles=angles)
    return sc


@pytest.mark.parametrize("bounces", [1, 3])
def test_box_wing_matches_oracle(bounces):
    import paper_2602_10712_amd as p
    m = si.box_wing()
    rs, rd = si.materials(m.n_tris, 1)
    sun = si.fibonacci_dirs(8)
    sc = make(m, rs, rd)
    n = 4096
    prm = p.TraceParams(bounces=bounces, seed=21)
    ref = oracle.surface_estimate(m.verts, m.tris, rs, rd, sun, n_samples=n, bounces=bounces, seed=21, records=True)
    for brute in (False, True):
        g = run([sc], sun, n, prm, brute)
        deg = check_records({k: v[0] for k, v in g.items()}, ref, bounces)
        assert rel_l2(g["F"][0], ref.force) <= 1e-4
        assert rel_l2(g["T"][0], ref.torque) <= 1e-4
        print(f"box-wing B={bounces} brute={brute}: degenerate {deg:.4f}")
    sc.close()


def test_meo_small_bvh_equals_brute_and_oracle():
    import paper_2602_10712_amd as p
    m = si.meo_satellite(bus_n=6, cyl_sides=16, panel_n=4, dish_rings=8, dish_sectors=16, strut_sides=6)
    rs, rd = si.materials(m.n_tris, 3)
    th = np.array([0.2, -0.3])
    sc = make(m, rs, rd, th)
    V = apply_hinges(m.verts, m.vert_hinge, m.hinge_origin, m.hinge_axis, th)
    assert np.allclose(sc.vertices(), V, rtol=0, atol=1e-12)
    sun = si.fibonacci_dirs(6)
    n = 1000  # not a multiple of the 256-sample workgroup
    prm = p.TraceParams(bounces=3, seed=22, design_index=4)
    a = run([sc], sun, n, prm, False)
    b = run([sc], sun, n, prm, True)
    for k in ("F", "T", "facet", "lit", "hits"):
        assert np.array_equal(a[k], b[k]), k
    ref = oracle.surface_estimate(V, m.tris, rs, rd, sun, n_samples=n, bounces=3, seed=22, design_index=4,
                                  com=m.com, records=True)
    deg = check_records({k: v[0] for k, v in a.items()}, ref, 3)
    assert rel_l2(a["F"][0], ref.force) <= 1e-4
    print(f"meo small: degenerate {deg:.4f}")
    sc.close()


def test_multi_world_equals_single_designs():
    import paper_2602_10712_amd as p
    scenes = []
    for k, n_t in enumerate([2500, 6000, 11000]):
        m = si.meo_variant(n_t)
        th = si.random_designs(1, seed=500 + k)[0]
        rs, rd = si.materials(m.n_tris, 600 + k)
        scenes.append(make(m, rs, rd, th[:2]))
    sun = si.fibonacci_dirs(5)
    n = 512
    prm = p.TraceParams(bounces=3, seed=23, design_index=10)
    for brute in (False, True):
        allg = run(scenes, sun, n, prm, brute)
        for s, sc in enumerate(scenes):
            one = run([sc], sun, n, p.TraceParams(bounces=3, seed=23, design_index=10 + s), brute)
            for key in ("F", "T", "facet", "lit", "hits"):
                assert np.array_equal(allg[key][s], one[key][0]), (brute, s, key)
    for sc in scenes:
        sc.close()


def test_invalid_arguments():
    import paper_2602_10712_amd as p
    m = si.box_wing()
    rs, rd = si.materials(m.n_tris, 1)
    sc = make(m, rs, rd)
    dev = torch.device("cuda")
    sun = torch.as_tensor(si.fibonacci_dirs(2), device=dev).contiguous()
    F = torch.empty((1, 2, 3), dtype=torch.float64, device=dev)
    with pytest.raises(p.SRPError):
        p.srp_surface_estimate([sc], sun, 0, p.TraceParams(bounces=2), F)
    with pytest.raises(p.SRPError):
        p.srp_surface_estimate([sc], sun, 16, p.TraceParams(bounces=9), F)
    rl = torch.zeros((1, 2, 16), dtype=torch.int32, device=dev)
    with pytest.raises(p.SRPError):  # records need the facet array
        p.srp_surface_estimate([sc], sun, 16, p.TraceParams(bounces=2), F, rec_lit=rl)
    sc.close()


def test_full_size_meo_records_match_oracle():
    import paper_2602_10712_amd as p
    m = si.meo_satellite()
    rs, rd = si.materials(m.n_tris, 1)
    sc = make(m, rs, rd, [0.0, 0.0])
    sun = si.fibonacci_dirs(1024)[::128].copy()  # 8 directions spread over the sphere
    n = 1 << 16
    prm = p.TraceParams(bounces=3, seed=24)
    g = run([sc], sun, n, prm, False)
    k = 512
    ref = oracle.surface_estimate(m.verts, m.tris, rs, rd, sun, n_samples=k, bounces=3, seed=24, records=True)
    sub = {key: g[key][0][:, :k] for key in ("facet", "lit", "hits")}
    deg = check_records(sub, ref, 3, min_ok=0.98)  # 1 cm antenna facets and dish slivers (measured 0.8 % flagged)
    print(f"full size: degenerate {deg:.4f}")
    assert np.all(np.isfinite(g["F"])) and np.abs(g["F"]).max() > 0
    sc.close()


@pytest.mark.parametrize("sampling", [1, 2, 3])
def test_sampling_options_match_oracle(sampling):
    import paper_2602_10712_amd as p
    m = si.meo_satellite(bus_n=6, cyl_sides=16, panel_n=4, dish_rings=8, dish_sectors=16, strut_sides=6)
    rs, rd = si.materials(m.n_tris, 3)
    sc = make(m, rs, rd, [0.1, 0.2])
    V = apply_hinges(m.verts, m.vert_hinge, m.hinge_origin, m.hinge_axis, [0.1, 0.2])
    assert np.allclose(sc.vertices(), V, rtol=0, atol=1e-12)
    sun = si.fibonacci_dirs(5)
    n = 1500  # ragged: not a multiple of the 256-sample workgroup
    prm = p.TraceParams(bounces=3, seed=25, design_index=2, sampling=sampling)
    a = run([sc], sun, n, prm, False)
    b = run([sc], sun, n, prm, True)
    for k in ("F", "T", "facet", "lit", "hits"):
        assert np.array_equal(a[k], b[k]), k
    ref = oracle.surface_estimate(V, m.tris, rs, rd, sun, n_samples=n, bounces=3, seed=25, design_index=2,
                                  com=m.com, records=True, sampling=sampling)
    deg = check_records({k: v[0] for k, v in a.items()}, ref, 3)
    assert rel_l2(a["F"][0], ref.force) <= 1e-4
    assert rel_l2(a["T"][0], ref.torque) <= 1e-4
    print(f"sampling {sampling}: degenerate {deg:.4f}")
    with pytest.raises(p.SRPError):
        p.srp_surface_estimate([sc], torch.as_tensor(sun, device="cuda"), 16, p.TraceParams(bounces=2, sampling=4),
                               torch.empty((1, 5, 3), dtype=torch.float64, device="cuda"))
    sc.close()


def test_phong_lobes_match_oracle():
    """Per-facet Phong exponents (srp_scene_set_phong; panels glossy with m from 2 to 200, the other
    facets mirrors or m = 1): records on the samples the oracle does not flag identical to the
    oracle's and force and torque within 1e-4, under lobe importance sampling and plain MC; the BVH
    walk equals brute force bit for bit.  Exponents below 1 are refused and leave the scene as it
    was; the ray-grid calls refuse a scene with lobes; set_phong(None) restores the mirrors."""
    import paper_2602_10712_amd as p
    m = si.meo_satellite(bus_n=6, cyl_sides=16, panel_n=4, dish_rings=8, dish_sectors=16, strut_sides=6)
    rs, rd = si.materials(m.n_tris, 7)
    rng = np.random.default_rng(8)
    ex = np.where(np.asarray(m.group) == si.PANEL, rng.uniform(2.0, 200.0, m.n_tris),
                  np.where(rng.uniform(size=m.n_tris) < 0.5, np.inf, 1.0)).astype(np.float32)
    th = np.array([0.25, -0.2])
    V = apply_hinges(m.verts, m.vert_hinge, m.hinge_origin, m.hinge_axis, th)
    sc = make(m, rs, rd, th)
    plain = make(m, rs, rd, th)
    sun = si.fibonacci_dirs(6)
    n = 2000
    mirror_ref = run([plain], sun, n, p.TraceParams(bounces=3, seed=41, design_index=2), False)
    sc.set_phong(ex)
    first = None
    for sampling in (0, 2):
        prm = p.TraceParams(bounces=3, seed=41, design_index=2, sampling=sampling)
        a = run([sc], sun, n, prm, False)
        b = run([sc], sun, n, prm, True)
        for k in ("F", "T", "facet", "lit", "hits"):
            assert np.array_equal(a[k], b[k]), (sampling, k)
        ref = oracle.surface_estimate(V, m.tris, rs, rd, sun, n_samples=n, bounces=3, seed=41, design_index=2,
                                      com=m.com, records=True, sampling=sampling, phong=ex)
        deg = check_records({k: v[0] for k, v in a.items()}, ref, 3, min_ok=0.98)
        ef, et = rel_l2(a["F"][0], ref.force), rel_l2(a["T"][0], ref.torque)
        print(f"Phong lobes, sampling {sampling}: force {ef:.2e}, torque {et:.2e}, flagged {deg:.4f}")
        assert ef <= 1e-4 and et <= 1e-4
        if sampling == 0:
            first = a
    # the lobes change the answer
    assert rel_l2(first["F"][0], mirror_ref["F"][0]) > 1e-3
    # ray-grid calls refuse the scene
    with pytest.raises(p.SRPError) as e:
        sc.trace(sun, p.TraceParams(nu=16, nv=16))
    assert e.value.status == -5
    # an exponent below 1 is refused and the scene keeps its lobes
    bad = ex.copy()
    bad[3] = 0.5
    with pytest.raises(p.SRPError) as e:
        sc.set_phong(bad)
    assert e.value.status == -1
    again = run([sc], sun, n, p.TraceParams(bounces=3, seed=41, design_index=2), False)
    assert np.array_equal(again["F"], first["F"])
    # the lobes survive a new design; None restores the mirrors
    sc.set_design(rs, rd, hinge_angles=th)
    again = run([sc], sun, n, p.TraceParams(bounces=3, seed=41, design_index=2), False)
    assert np.array_equal(again["F"], first["F"])
    sc.set_phong(None)
    back = run([sc], sun, n, p.TraceParams(bounces=3, seed=41, design_index=2), False)
    for k in ("F", "T", "facet", "lit", "hits"):
        assert np.array_equal(back[k], mirror_ref[k]), k
    sc.trace(sun, p.TraceParams(nu=16, nv=16))
    sc.close()
    plain.close()


def _mw_designs(n, seed):
    rng = np.random.default_rng(seed)
    ang = rng.uniform(-0.5, 0.5, (n, 2))
    cols = [ang]
    for g in range(3):
        rs = rng.uniform(0.0, 0.5, n)
        rd = rng.uniform(0.0, 0.5, n)
        mm = np.where(rng.uniform(size=n) < 0.3, np.inf, rng.uniform(1.0, 80.0, n))
        cols.append(np.stack([rs, rd, mm], 1))
    return np.concatenate(cols, 1).astype(np.float32)


def run_designs(sc, group, sun, dsg, K, prm, records=True):
    import paper_2602_10712_amd as p
    dev = torch.device("cuda")
    N = len(sun)
    sd = torch.as_tensor(sun, dtype=torch.float64, device=dev).contiguous()
    dd = torch.as_tensor(dsg, dtype=torch.float32, device=dev).contiguous()
    F = torch.empty((N, 3), dtype=torch.float64, device=dev)
    T = torch.empty_like(F)
    rf = rl = rh = None
    if records:
        rf = torch.full((N, K), -7, dtype=torch.int32, device=dev)
        rl = torch.full((N, K), -7, dtype=torch.int32, device=dev)
        rh = torch.full((N, K, max(prm.bounces - 1, 1)), -7, dtype=torch.int32, device=dev)
    p.srp_surface_designs(sc, group, 3, sd, dd, K, prm, F, T, rec_facet=rf, rec_hits=rh, rec_lit=rl)
    torch.cuda.synchronize()
    out = {"F": F.cpu().numpy(), "T": T.cpu().numpy()}
    if records:
        out.update(facet=rf.cpu().numpy(), lit=rl.cpu().numpy(), hits=rh.cpu().numpy()[..., :prm.bounces - 1])
    return out


def test_multi_world_designs_match_oracle():
    """srp_surface_designs (the paper's multi-world sampling: every pair of sun direction and design
    is its own world, turned from the rest pose, with its group materials and Phong exponents):
    records on the samples the oracle does not flag identical to the oracle's multi-world
    estimator and the per-pair forces and torques within 1e-4, under both sampling modes; pairs
    that all carry one design agree with srp_surface_estimate on a scene set to that design (same
    samples; turned rays against turned vertices); invalid designs are refused."""
    import paper_2602_10712_amd as p
    m = si.meo_satellite(bus_n=6, cyl_sides=16, panel_n=4, dish_rings=8, dish_sectors=16, strut_sides=6)
    group = np.asarray(m.group, dtype=np.int32)
    sc = p.Scene.from_mesh(m)
    N, K = 64, 96
    dsg = _mw_designs(N, 61)
    sun = si.random_dirs(N, seed=62)
    for sampling in (0, 2):
        prm = p.TraceParams(bounces=3, seed=51, dir_index_base=7, design_index=3, sampling=sampling)
        g = run_designs(sc, group, sun, dsg, K, prm)
        ref = oracle.surface_designs(m.verts, m.tris, m.vert_hinge, m.hinge_origin, m.hinge_axis, group, 3,
                                     dsg.astype(np.float64), sun, samples=K, bounces=3, seed=51, dir_index_base=7,
                                     design_index=3, sampling=sampling, com=m.com, records=True)
        deg = check_records(g, ref, 3, min_ok=0.98)
        ef, et = rel_l2(g["F"], ref.force), rel_l2(g["T"], ref.torque)
        print(f"multi-world, sampling {sampling}: per-pair force {ef:.2e}, torque {et:.2e}, flagged {deg:.4f}")
        assert ef <= 1e-4 and et <= 1e-4
    # one design in every pair = the single-design estimator on that design's scene
    th = dsg[5]
    one = np.tile(th, (N, 1))
    prm = p.TraceParams(bounces=3, seed=51, dir_index_base=7, design_index=3)
    g1 = run_designs(sc, group, sun, one, K, prm)
    mats = th[2:].reshape(3, 3)[group]
    single = make(m, mats[:, 0], mats[:, 1], th[:2].astype(np.float64))
    single.set_phong(mats[:, 2])
    g2 = run([single], sun, K, p.TraceParams(bounces=3, seed=51, dir_index_base=7, design_index=3), True)
    agree = (g1["facet"] == g2["facet"][0]) & (g1["lit"] == g2["lit"][0]) & (g1["hits"] == g2["hits"][0]).all(-1)
    e1 = rel_l2(g1["F"], g2["F"][0])
    print(f"one design: records agree on {agree.mean():.4f} of the samples, forces {e1:.2e} apart")
    assert agree.mean() >= 0.995 and e1 <= 1e-4
    # invalid designs, groups and sizes
    bad = dsg.copy()
    bad[3, 2] = 0.7
    bad[3, 3] = 0.5
    with pytest.raises(p.SRPError) as e:
        run_designs(sc, group, sun, bad, K, prm, records=False)
    assert e.value.status == -1
    bad = dsg.copy()
    bad[1, 7] = 0.5
    with pytest.raises(p.SRPError):
        run_designs(sc, group, sun, bad, K, prm, records=False)
    with pytest.raises(p.SRPError):
        run_designs(sc, np.full_like(group, 5), sun, dsg, K, prm, records=False)
    sc.close()
    single.close()
