"""srp_trace_noalloc (the forward trace with its workspace in the library's fixed device array)
against srp_trace, through the C ABI: bit-identical force and torque on two calls in a row, the
second smaller than the first, and an oversized request rejected before anything is enqueued."""
import numpy as np
import pytest

import srp_inputs as si

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _pair(p, sc, sun_np, params, with_torque=True):
    sun = torch.from_numpy(np.ascontiguousarray(sun_np)).cuda()
    D = sun.shape[0]
    F0 = torch.full((D, 3), np.nan, dtype=torch.float64, device="cuda")
    T0 = torch.full((D, 3), np.nan, dtype=torch.float64, device="cuda") if with_torque else None
    F1 = torch.full((D, 3), np.nan, dtype=torch.float64, device="cuda")
    T1 = torch.full((D, 3), np.nan, dtype=torch.float64, device="cuda") if with_torque else None
    p.srp_trace_noalloc(sc.handle, sun, params, F0, T0)
    p.srp_trace(sc.handle, sun, params, F1, T1)
    torch.cuda.synchronize()
    F0, F1 = F0.cpu().numpy(), F1.cpu().numpy()
    assert np.isfinite(F0).all() and np.abs(F0).max() > 0
    assert np.array_equal(F0, F1)
    if with_torque:
        assert np.array_equal(T0.cpu().numpy(), T1.cpu().numpy())
    return F0


def test_noalloc_matches_trace_two_calls():
    import paper_2602_10712_amd as p
    # call 1: the 20.6k-triangle satellite, 24 directions x 256^2, 3 bounces
    m = si.meo_satellite()
    rs, rd = si.materials(m.n_tris, 1)
    sat = p.Scene.from_mesh(m)
    sat.set_design(rs, rd, hinge_angles=np.deg2rad([15.0, -10.0]))
    params = p.TraceParams(nu=256, nv=256, bounces=3, jitter=1, seed=11)
    F_big = _pair(p, sat, si.fibonacci_dirs(24), params)
    print("satellite 24 dirs x 256^2 x 3: bit-identical; |F| max", np.abs(F_big).max())
    # call 2, smaller: box-wing, 5 directions x 37 x 23 pixels, 1 bounce, no torque output; the
    # array still holds the first call's partial sums
    bw = si.box_wing()
    rs2, rd2 = si.materials(bw.n_tris, 3)
    box = p.Scene.from_mesh(bw)
    box.set_design(rs2, rd2)
    params2 = p.TraceParams(nu=37, nv=23, bounces=1, jitter=1, seed=5)
    F_small = _pair(p, box, si.fibonacci_dirs(5), params2, with_torque=False)
    print("box-wing 5 dirs x 37 x 23 x 1: bit-identical; |F| max", np.abs(F_small).max())
    # and the large one again after the small one
    _pair(p, sat, si.fibonacci_dirs(24), params)
    sat.close()
    box.close()


def test_noalloc_rejects_oversized_trace():
    import paper_2602_10712_amd as p
    bw = si.box_wing()
    rs, rd = si.materials(bw.n_tris, 1)
    sc = p.Scene.from_mesh(bw)
    sc.set_design(rs, rd)
    D = 4096  # 4096 directions x 1024^2 pixels need ~54 MB of partial sums
    sun = torch.from_numpy(si.fibonacci_dirs(D)).cuda()
    F = torch.full((D, 3), 7.0, dtype=torch.float64, device="cuda")
    params = p.TraceParams(nu=1024, nv=1024, bounces=1, jitter=1, seed=1)
    with pytest.raises(p.SRPError) as ei:
        p.srp_trace_noalloc(sc.handle, sun, params, F)
    assert ei.value.status == -1 and "workspace" in str(ei.value)
    torch.cuda.synchronize()
    assert bool((F == 7.0).all())  # nothing was enqueued
    sc.close()
