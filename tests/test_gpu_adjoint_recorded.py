"""The adjoint on recorded paths (srp_trace_recorded + srp_trace_adjoint_recorded) against the
walking replay (srp_trace_adjoint) and the FP64 oracle.

Bars:
  * forces and torques of the recorded forward equal to srp_trace's within 1e-7 per direction (a
    separate kernel, whose FP32 expressions the compiler may contract differently; measured ~5e-9);
  * hinge and reflectance gradients equal to the walking replay's within 1e-6 of the largest entry
    (each path adds the same terms; the two kernels sum them in different orders and the compiler
    may contract their FP32 expressions differently); covered on the 20k-triangle satellite with
    hinge angles, a ragged grid
    (250^2: partial 8 x 8 tiles), a direction count that is not a multiple of 8, culled tiles,
    with and without edge samples;
  * reflectance gradients vs the oracle's FP64 adjoint on the box-wing: relative L2 <= 1e-4;
  * a record is refused (SRP_EINVAL) after a design change, for other arguments, when too small,
    or when it is not the last one recorded; paths of more than 3 interactions are not recorded
    (SRP_EUNSUPPORTED).
"""
import numpy as np
import pytest

import oracle
import srp_inputs as si

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _lib():
    import paper_2602_10712_amd as p
    return p


def rel_l2(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("edge_samples", [0, 4])
def test_recorded_equals_replay_on_satellite(edge_samples):
    p = _lib()
    m = si.meo_satellite()
    rs, rd = si.materials(m.n_tris, 3)
    sc = p.Scene.from_mesh(m)
    sc.set_design(rs, rd, hinge_angles=[0.25, -0.35])
    D = 20
    sun = torch.as_tensor(si.random_dirs(D, seed=31), device="cuda").contiguous()
    rng = np.random.default_rng(32)
    gF = rng.standard_normal((D, 3))
    gT = rng.standard_normal((D, 3))
    params = p.TraceParams(nu=250, nv=250, bounces=3, seed=9, jitter=1, edge_samples=edge_samples)
    F0, T0 = sc.trace(sun, params)
    F1, T1, rec = sc.trace_recorded(sun, params)
    a_rs, a_rd, a_h = sc.adjoint(sun, params, gF, gT)
    b_rs, b_rd, b_h = sc.adjoint_recorded(rec, params, gF, gT)
    torch.cuda.synchronize()
    for a, b in ((F0, F1), (T0, T1)):  # two kernels: FP32 expressions may be contracted differently
        assert float(((a - b).norm(dim=1) / a.norm(dim=1)).max()) <= 1e-7
    ha, hb = a_h.cpu().numpy(), b_h.cpu().numpy()
    print(f"hinge gradients: walking replay {ha}, over the record {hb}, largest difference "
          f"{np.abs(ha - hb).max() / np.abs(ha).max():.2e} of the largest")
    assert np.abs(ha - hb).max() <= 1e-6 * np.abs(ha).max()
    for a, b in ((a_rs, b_rs), (a_rd, b_rd)):
        a = a.cpu().numpy()
        b = b.cpu().numpy()
        scale = np.abs(a).max()
        assert scale > 0
        assert np.abs(a - b).max() <= 1e-6 * scale
    print(f"edge samples {edge_samples}: record {rec.paths.numel() * 4 / 1e6:.1f} MB")


def test_recorded_rho_gradients_match_oracle_box_wing():
    p = _lib()
    m = si.box_wing()
    rs, rd = si.materials(m.n_tris, 1)
    sun = si.fibonacci_dirs(16)
    rng = np.random.default_rng(1)
    gF = rng.standard_normal((16, 3))
    gT = rng.standard_normal((16, 3))
    sc = p.Scene.from_mesh(m)
    sc.set_design(rs, rd)
    params = p.TraceParams(nu=96, nv=96, bounces=3, seed=5)
    _, _, rec = sc.trace_recorded(sun, params)
    grs, grd, _ = sc.adjoint_recorded(rec, params, gF, gT)
    torch.cuda.synchronize()
    o_rs, o_rd = oracle.trace_adjoint_rho(m.verts, m.tris, rs, rd, sun, gF, gT, nu=96, nv=96, bounces=3, seed=5)
    e = rel_l2(np.concatenate([grs.cpu().numpy(), grd.cpu().numpy()]), np.concatenate([o_rs, o_rd]))
    print(f"box-wing rho-gradient rel L2 (recorded paths) {e:.3e}")
    assert e <= 1e-4


def test_stale_or_foreign_records_are_refused():
    p = _lib()
    m = si.box_wing()
    rs, rd = si.materials(m.n_tris, 1)
    sc = p.Scene.from_mesh(m)
    sc.set_design(rs, rd, hinge_angles=[0.1, 0.0])
    sun = torch.as_tensor(si.fibonacci_dirs(8), device="cuda").contiguous()
    params = p.TraceParams(nu=64, nv=64, bounces=3, seed=5)
    gF = np.ones((8, 3))
    _, _, rec = sc.trace_recorded(sun, params)
    sc.adjoint_recorded(rec, params, gF)  # valid
    other = p.TraceParams(nu=64, nv=64, bounces=3, seed=6)
    with pytest.raises(p.SRPError):
        sc.adjoint_recorded(rec, other, gF)
    short = p.PathRecord(rec.sun_dirs, rec.frames, rec.paths[: rec.paths.numel() // 2])
    with pytest.raises(p.SRPError):
        sc.adjoint_recorded(short, params, gF)
    _, _, rec2 = sc.trace_recorded(sun, params)
    with pytest.raises(p.SRPError):
        sc.adjoint_recorded(rec, params, gF)  # not the last record
    sc.adjoint_recorded(rec2, params, gF)
    sc.set_design(rs, rd)  # same angles: materials re-packed, still a new scene state
    with pytest.raises(p.SRPError):
        sc.adjoint_recorded(rec2, params, gF)
    with pytest.raises(p.SRPError):
        p.srp_trace_recorded(sc.handle, sun, params, torch.empty((8, 3), dtype=torch.float64, device="cuda"),
                             None, torch.empty(16, dtype=torch.int32, device="cuda"))
    with pytest.raises(p.SRPError):  # a record holds three interactions per path
        sc.trace_recorded(sun, p.TraceParams(nu=64, nv=64, bounces=4, seed=5))
    torch.cuda.synchronize()
