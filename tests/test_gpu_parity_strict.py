"""Parity of the timed forward kernel at ray granularity, and the FP32 error the degeneracy rules
guard against (GPU vs the FP64 oracle, through the C ABI).

  * FP32 error of the hit points: the GPU's hit point of every non-degenerate segment against the
    oracle's, split into the offset across the segment (what decides which side of an edge a ray
    passes), along it (which of two nearby surfaces is closer) and normal to the hit facet.  The
    oracle's degeneracy rules give each segment a position uncertainty u (LAT L on primary rays,
    grown by 1/cos(theta) at each interaction) and a depth uncertainty of at least DEPTH L; every
    measured error must stay below a tenth of its margin: across <= u/10,
    along <= (DEPTH L + u)/(10 cos), normal <= DEPTH L/10.
  * The forward trace with a ray mask: with the oracle's degenerate paths left out, the reduced
    force and torque of k_trace (the grid-mode kernel bench.py times, culling included) equal the
    oracle's sum over the same rays, and so do the sums over seven disjoint classes of 8 x 8 tiles
    (each class traced with every other tile masked), on the small workload and on one direction
    of the benchmark launch itself.
Inputs reach the oracle only through its own design step (oracle.design.apply_hinges).
"""
import numpy as np
import pytest

import oracle
import srp_inputs as si
from oracle.design import apply_hinges

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

FORCE_BAR = 1e-5  # masked sums: only FP32 rounding separates the two sides (torque on the (L/2)|F| scale)


def _lib():
    import paper_2602_10712_amd as p
    return p


def rel_l2(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300))


def scene_size(V):
    return 2.0 * np.linalg.norm(V - V.mean(0), axis=1).max()


def torque_err(T, T_ref, F_ref, V):
    """Torque error on the scale a force of this size can produce, ||dT|| / ((L/2) ||F||) (a nearly
    symmetric body has a small net torque, so its relative error says little)."""
    return float(np.linalg.norm(np.asarray(T) - T_ref) / max(0.5 * scene_size(V) * np.linalg.norm(F_ref), 1e-300))


def hit_point_errors(gpu_x, orc, sun, V, tris):
    """On the hit segments of non-degenerate paths: the GPU hit point's offset from the oracle's
    across the segment and along it, the segment's incidence cosine at the hit, its position
    uncertainty u under the oracle's degeneracy model (base L, grown by 1/cos at each earlier
    interaction), and the offset normal to the hit facet's plane.  gpu_x, orc.hit_x: [D][P][B][3]."""
    L = scene_size(V)
    ok = ~orc.path_degenerate()
    hit = orc.hit_prim >= 0
    X = orc.hit_x
    D, P, B = orc.hit_prim.shape
    nrm = np.cross(V[tris[:, 1]] - V[tris[:, 0]], V[tris[:, 2]] - V[tris[:, 0]])
    nrm /= np.linalg.norm(nrm, axis=1)[:, None]
    d = np.empty_like(X)
    d[:, :, 0, :] = -np.asarray(sun, float)[:, None, :]
    if B > 1:
        seg = X[:, :, 1:, :] - X[:, :, :-1, :]
        with np.errstate(invalid="ignore", divide="ignore"):
            d[:, :, 1:, :] = seg / np.linalg.norm(seg, axis=-1, keepdims=True)
    n_hit = nrm[np.where(hit, orc.hit_prim, 0)]
    cos = -(d * n_hit).sum(-1)  # [D][P][B]
    th = oracle.degen_thresholds()
    u = np.empty((D, P, B))
    u[:, :, 0] = th["lat"] * L
    for b in range(1, B):
        u[:, :, b] = u[:, :, b - 1] / np.maximum(np.where(hit[:, :, b - 1], cos[:, :, b - 1], 1.0), th["graze"]) \
            + th["lat"] * L
    sel = ok[:, :, None] & hit
    delta = gpu_x.astype(np.float64)[sel] - X[sel]
    dd = d[sel]
    along = np.abs((delta * dd).sum(-1))
    across = np.linalg.norm(delta - (delta * dd).sum(-1, keepdims=True) * dd, axis=-1)
    normal = np.abs((delta * n_hit[sel]).sum(-1))
    return across, along, cos[sel], u[sel], normal


def tile_class(nu, nv, classes):
    """Class (0..classes-1) of the 8 x 8 wave tile of every pixel p = i + k nu."""
    i = np.arange(nu * nv) % nu
    k = np.arange(nu * nv) // nu
    tiles_x = (nu + 7) // 8
    return ((i // 8) + (k // 8) * tiles_x) % classes


def test_fp32_hit_point_error_and_masked_sums():
    p = _lib()
    m = si.meo_satellite()
    rs, rd = si.materials(m.n_tris, 1)
    ang = np.deg2rad([20.0, -20.0])
    V = apply_hinges(m.verts, m.vert_hinge, m.hinge_origin, m.hinge_axis, ang)
    L = scene_size(V)
    sun = si.fibonacci_dirs(1024)[::128]
    nu, nv, B = 96, 80, 3
    sc = p.Scene.from_mesh(m)
    sc.set_design(rs, rd, hinge_angles=ang)
    assert np.allclose(sc.vertices(), V, rtol=0, atol=1e-12)  # the library's design step
    params = p.TraceParams(nu=nu, nv=nv, bounces=B, jitter=1, seed=7)
    hp, rf, hx = sc.records(sun, params, points=True)
    torch.cuda.synchronize()
    orc = oracle.trace(V, m.tris, rs, rd, sun, nu=nu, nv=nv, bounces=B, seed=7, records=True)
    deg = orc.path_degenerate()
    seg_flag = orc.degen.astype(bool) & (orc.hit_prim >= 0)
    print(f"degenerate: paths {deg.mean():.2e}, hit segments {seg_flag.sum() / max((orc.hit_prim >= 0).sum(), 1):.2e}")
    ok = ~deg
    assert np.array_equal(hp.cpu().numpy()[ok], orc.hit_prim[ok])
    across, along, cos, u, normal = hit_point_errors(hx.cpu().numpy(), orc, sun, V, m.tris)
    depth = oracle.degen_thresholds()["depth"] * L
    print(f"FP32 hit-point error over {len(across)} segments (L = {L:.3f} m): across / u max {(across / u).max():.3f} "
          f"(absolute max {across.max() / L:.2e} L); along * cos / (DEPTH L + u) max "
          f"{(along * cos / (depth + u)).max():.3f}; normal to the facet / (DEPTH L) max {(normal / depth).max():.3f}")
    # the degeneracy rules assume errors at most a tenth of their margins: across the ray u, in t at
    # least (DEPTH L + u) / cos, off the facet's plane DEPTH L
    assert (across <= 0.1 * u).all()
    assert (along * cos <= 0.1 * (depth + u)).all()
    assert (normal <= 0.1 * depth).all()

    # k_trace (grid mode) with the degenerate paths masked out: reduced force and torque equal the
    # oracle's sum over the same rays
    mask = p.ray_mask_bits(deg)
    pm = p.TraceParams(nu=nu, nv=nv, bounces=B, jitter=1, seed=7, ray_mask=mask)
    F, T = sc.trace(sun, pm)
    torch.cuda.synchronize()
    o_F = (orc.ray_force * ok[..., None]).sum(1)
    o_T = (orc.ray_torque * ok[..., None]).sum(1)
    eF, eT = rel_l2(F.cpu().numpy(), o_F), torque_err(T.cpu().numpy(), o_T, o_F, V)
    print(f"masked k_trace: force rel L2 {eF:.2e}, torque error {eT:.2e}")
    assert eF <= FORCE_BAR and eT <= FORCE_BAR
    # seven disjoint tile classes, each traced alone
    cls = tile_class(nu, nv, 7)
    worst = 0.0
    for r in range(7):
        keep = ok & (cls == r)[None, :]
        pr = p.TraceParams(nu=nu, nv=nv, bounces=B, jitter=1, seed=7, ray_mask=p.ray_mask_bits(~keep))
        Fr, Tr = sc.trace(sun, pr)
        torch.cuda.synchronize()
        oF = (orc.ray_force * keep[..., None]).sum(1)
        oT = (orc.ray_torque * keep[..., None]).sum(1)
        e = max(rel_l2(Fr.cpu().numpy(), oF), torque_err(Tr.cpu().numpy(), oT, oF, V))
        worst = max(worst, e)
        assert e <= FORCE_BAR, (r, e)
    print(f"tile classes: worst rel L2 {worst:.2e}")
    # records honour the mask too: left-out paths record no hit and no force
    hp2, rf2 = sc.records(sun, pm)
    torch.cuda.synchronize()
    hp2, rf2 = hp2.cpu().numpy(), rf2.cpu().numpy()
    assert (hp2[deg] == -1).all() and (rf2[deg] == 0).all()
    assert np.array_equal(hp2[ok], orc.hit_prim[ok])
    sc.close()


def test_masked_sum_on_the_benchmark_launch():
    """The benchmark launch (20.6k tris, 1024 dirs x 1024^2 rays, 3 bounces, jitter seed 2) with one
    direction's degenerate paths masked out: that direction's force and torque equal the oracle's
    sum over its non-degenerate paths; every other direction is unchanged by the mask."""
    p = _lib()
    m = si.meo_satellite()
    rs, rd = si.materials(m.n_tris, 1)
    V = apply_hinges(m.verts, m.vert_hinge, m.hinge_origin, m.hinge_axis, [0.0, 0.0])
    sun = si.fibonacci_dirs(1024)
    G = 1024
    sc = p.Scene.from_mesh(m)
    sc.set_design(rs, rd, hinge_angles=[0.0, 0.0])
    j = 357
    orc = oracle.trace(V, m.tris, rs, rd, sun[j:j + 1], nu=G, nv=G, bounces=3, seed=2, dir_index_base=j,
                       records=True)
    deg = orc.path_degenerate()[0]
    ok = ~deg
    print(f"direction {j}: degenerate paths {deg.mean():.2e}")
    words = (G * G + 31) // 32
    mask = torch.zeros((1024, words), dtype=torch.int32, device="cuda")
    mask[j] = p.ray_mask_bits(deg[None, :])[0]
    F0, T0 = sc.trace(sun, p.TraceParams(nu=G, nv=G, bounces=3, jitter=1, seed=2))
    F1, T1 = sc.trace(sun, p.TraceParams(nu=G, nv=G, bounces=3, jitter=1, seed=2, ray_mask=mask))
    torch.cuda.synchronize()
    F0, T0, F1, T1 = (x.cpu().numpy() for x in (F0, T0, F1, T1))
    others = np.arange(1024) != j
    assert np.array_equal(F0[others], F1[others]) and np.array_equal(T0[others], T1[others])
    o_F = (orc.ray_force[0] * ok[:, None]).sum(0)
    o_T = (orc.ray_torque[0] * ok[:, None]).sum(0)
    eF, eT = rel_l2(F1[j], o_F), torque_err(T1[j], o_T, o_F, V)
    print(f"benchmark launch, direction {j}, degenerate paths masked: force rel L2 {eF:.2e}, torque {eT:.2e}; "
          f"unmasked vs the full oracle sum: force {rel_l2(F0[j], orc.force[0]):.2e}")
    assert eF <= FORCE_BAR and eT <= FORCE_BAR
    sc.close()


def test_ray_mask_rejected_where_unsupported():
    p = _lib()
    m = si.box_wing()
    sc = p.Scene.from_mesh(m)
    sc.set_design(*si.materials(m.n_tris, 1))
    sun = torch.as_tensor(si.fibonacci_dirs(2), device="cuda")
    mask = p.ray_mask_bits(np.zeros((2, 64), bool))
    prm = p.TraceParams(nu=8, nv=8, bounces=1, ray_mask=mask)
    F = torch.zeros((2, 3), dtype=torch.float64, device="cuda")
    with pytest.raises(p.SRPError) as e:
        p.srp_batch_trace([sc], sun, prm, F.reshape(1, 2, 3))
    assert e.value.status == -5
    sc.close()
