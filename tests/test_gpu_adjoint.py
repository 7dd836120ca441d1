"""GPU adjoint (srp_trace_adjoint) vs the FP64 oracle, and the autograd Function.

Bars:
  * reflectance gradients vs the oracle's FP64 adjoint: relative L2 over the stacked [2][T] vector
    <= 1e-4 on the box-wing (FP32 per ray, FP64 atomics); on the 20k-triangle satellite <= 1e-4 with
    the oracle's degenerate paths left out on both sides (the oracle drops them, the GPU receives
    them as a ray mask), at 128^2 and on one direction of the benchmark's adjoint launch; the
    unmasked difference (degenerate paths that take another facet sequence on the GPU) is printed;
  * hinge gradients, pathwise part (no edge samples) vs central differences (h = 1e-4) of the
    oracle's frozen-visibility estimator without footprint factor: relative error <= 2e-3 per hinge;
  * a hinged plate: pathwise + visibility-edge parts match the derivative of the flat-plate
    closed form (the edge part carries the change of the plate's projected area).
"""
import numpy as np
import pytest

import oracle
import srp_inputs as si
from oracle.design import apply_hinges

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

C = 299792458.0
PHI = 1361.0


def _lib():
    import paper_2602_10712_amd as p
    return p


def rel_l2(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300))


def test_rho_gradients_box_wing():
    m = si.box_wing()
    rs, rd = si.materials(m.n_tris, 1)
    sun = si.fibonacci_dirs(16)
    rng = np.random.default_rng(1)
    gF = rng.standard_normal((16, 3))
    gT = rng.standard_normal((16, 3))
    p = _lib()
    sc = p.Scene.from_mesh(m)
    sc.set_design(rs, rd)
    params = p.TraceParams(nu=96, nv=96, bounces=3, seed=5)
    grs, grd, _ = sc.adjoint(sun, params, gF, gT)
    torch.cuda.synchronize()
    o_rs, o_rd = oracle.trace_adjoint_rho(m.verts, m.tris, rs, rd, sun, gF, gT, nu=96, nv=96, bounces=3, seed=5)
    g = np.concatenate([grs.cpu().numpy(), grd.cpu().numpy()])
    o = np.concatenate([o_rs, o_rd])
    e = rel_l2(g, o)
    print(f"box-wing rho-gradient rel L2 {e:.3e}")
    assert e <= 1e-4


def test_rho_gradients_meo_and_accumulation():
    m = si.meo_satellite()
    rs, rd = si.materials(m.n_tris, 1)
    sun = si.fibonacci_dirs(1024)[::256]
    rng = np.random.default_rng(2)
    gF = rng.standard_normal((4, 3))
    gT = rng.standard_normal((4, 3))
    p = _lib()
    sc = p.Scene.from_mesh(m)
    sc.set_design(rs, rd, hinge_angles=[0.2, -0.3])
    V = apply_hinges(m.verts, m.vert_hinge, m.hinge_origin, m.hinge_axis, [0.2, -0.3])
    params = p.TraceParams(nu=128, nv=128, bounces=3, seed=6)
    grs, grd, _ = sc.adjoint(sun, params, gF, gT)
    torch.cuda.synchronize()
    o_rs, o_rd, deg = oracle.trace_adjoint_rho(V, m.tris, rs, rd, sun, gF, gT, nu=128, nv=128, bounces=3, seed=6,
                                               drop_degenerate=True)
    pm = p.TraceParams(nu=128, nv=128, bounces=3, seed=6, ray_mask=p.ray_mask_bits(deg))
    mrs, mrd, _ = sc.adjoint(sun, pm, gF, gT)
    torch.cuda.synchronize()
    e = rel_l2(np.concatenate([mrs.cpu().numpy(), mrd.cpu().numpy()]), np.concatenate([o_rs, o_rd]))
    f_rs, f_rd = oracle.trace_adjoint_rho(V, m.tris, rs, rd, sun, gF, gT, nu=128, nv=128, bounces=3, seed=6)
    e_all = rel_l2(np.concatenate([grs.cpu().numpy(), grd.cpu().numpy()]), np.concatenate([f_rs, f_rd]))
    print(f"meo rho-gradient rel L2 {e:.3e} without the {deg.mean():.2e} degenerate paths; all paths {e_all:.3e}")
    assert e <= 1e-4
    # the outputs accumulate (+=): a second call on the same buffers doubles them
    dev = torch.device("cuda")
    a_rs = torch.zeros(m.n_tris, dtype=torch.float32, device=dev)
    a_rd = torch.zeros(m.n_tris, dtype=torch.float32, device=dev)
    sd = torch.as_tensor(sun, device=dev)
    gFd = torch.as_tensor(gF, device=dev)
    gTd = torch.as_tensor(gT, device=dev)
    for _ in range(2):
        p.srp_trace_adjoint(sc.handle, sd, params, gFd, gTd, a_rs, a_rd)
    torch.cuda.synchronize()
    assert rel_l2(a_rs.cpu().numpy(), 2 * grs.cpu().numpy()) <= 1e-6


def frozen_fd(m, V0, ang0, rs, rd, sun, fr, ref_hits, gF, gT, kw, h=1e-4):
    out = []
    for k in range(len(ang0)):
        Ls = []
        for sgn in (1, -1):
            a = np.array(ang0, dtype=np.float64)
            a[k] += sgn * h
            V = apply_hinges(m.verts, m.vert_hinge, m.hinge_origin, m.hinge_axis, a)
            F, T = oracle.trace_frozen(V, V0, m.tris, rs, rd, sun, ref_hits, fr, footprint=False, **kw)
            Ls.append((F * gF).sum() + (T * gT).sum())
        out.append((Ls[0] - Ls[1]) / (2 * h))
    return np.array(out)


def test_hinge_gradients_meo_vs_frozen_fd():
    m = si.meo_satellite()
    rs, rd = si.materials(m.n_tris, 3)
    ang0 = [0.3, -0.25]
    sun = si.fibonacci_dirs(1024)[[100, 350, 600, 900]]
    rng = np.random.default_rng(4)
    gF = rng.standard_normal((4, 3))
    gT = rng.standard_normal((4, 3))
    nu = nv = 96
    p = _lib()
    sc = p.Scene.from_mesh(m)
    sc.set_design(rs, rd, hinge_angles=ang0)
    V0 = apply_hinges(m.verts, m.vert_hinge, m.hinge_origin, m.hinge_axis, ang0)
    assert np.allclose(sc.vertices(), V0, atol=1e-12)
    fr = oracle.frames(V0, sun, nu, nv)
    params = p.TraceParams(nu=nu, nv=nv, bounces=3, seed=8, frame_mode=1)
    _, _, gh = sc.adjoint(sun, params, gF, gT, frames=fr)
    torch.cuda.synchronize()
    gh = gh.cpu().numpy()
    kw = dict(nu=nu, nv=nv, bounces=3, seed=8)
    ref = oracle.trace(V0, m.tris, rs, rd, sun, frames_in=fr, records=True, **kw)
    fd = frozen_fd(m, V0, ang0, rs, rd, sun, fr, ref.hit_prim, gF, gT, kw)
    err = np.abs(gh - fd) / np.abs(fd).max()
    print(f"hinge gradient (pathwise part) GPU {gh}, frozen-visibility FD {fd}, rel err {err}")
    assert np.all(err <= 2e-3)
    # the full finite difference (visibility changes included) differs by the visibility-edge part
    full = []
    for k in range(2):
        Ls = []
        for sgn in (1, -1):
            a = np.array(ang0)
            a[k] += sgn * 1e-3
            V = apply_hinges(m.verts, m.vert_hinge, m.hinge_origin, m.hinge_axis, a)
            r = oracle.trace(V, m.tris, rs, rd, sun, frames_in=fr, **kw)
            Ls.append((r.force * gF).sum() + (r.torque * gT).sum())
        full.append((Ls[0] - Ls[1]) / 2e-3)
    print(f"full finite difference (with visibility changes) {np.array(full)}; difference from the pathwise part "
          f"{np.array(full) - gh}")


@pytest.mark.parametrize("theta0", [0.0, 0.4])
def test_hinge_gradient_plate_closed_form(theta0):
    v, t = si.quad_grid((-0.6, 0.2, 0.0), (1.2, 0, 0), (0, 0.8, 0), 1, 1)
    m = si.Mesh(verts=v, tris=t.astype(np.int32), vert_hinge=np.zeros(len(v), np.int32),
                hinge_origin=np.zeros((1, 3)), hinge_axis=np.array([[1.0, 0, 0]]), group=np.zeros(2, np.int32))
    rs = np.full(2, 0.3, np.float32)
    rd = np.full(2, 0.25, np.float32)
    sun = np.array([[0.0, 0.0, 1.0]])
    p = _lib()
    sc = p.Scene.from_mesh(m)
    sc.set_design(rs, rd, hinge_angles=[theta0])
    V0 = apply_hinges(m.verts, m.vert_hinge, m.hinge_origin, m.hinge_axis, [theta0])
    assert np.allclose(sc.vertices(), V0, rtol=0, atol=1e-12)
    fr = oracle.frames(V0, sun, 60, 40)
    params = p.TraceParams(nu=60, nv=40, bounces=1, jitter=0, frame_mode=1, edge_samples=64)
    g_dir = np.array([[0.3, -0.8, 0.5]])
    _, _, gh = sc.adjoint(sun, params, g_dir, None, frames=fr)
    torch.cuda.synchronize()

    def cf(th):
        n = np.array([0.0, -np.sin(th), np.cos(th)])
        s_hat = np.array([0.0, 0.0, -1.0])
        c = float(s_hat @ -n)
        return PHI * 0.96 * c / C * ((1 - 0.3) * s_hat + 2 * (0.3 * c + float(rd[0]) / 3) * (-n))

    h = 1e-6
    d_cf = (cf(theta0 + h) - cf(theta0 - h)) / (2 * h)
    ref = float(g_dir[0] @ d_cf)
    assert abs(float(gh[0]) - ref) <= 1e-4 * abs(ref) + 1e-12, (float(gh[0]), ref)


def test_autograd_function_matches_adjoint():
    p = _lib()
    m = si.box_wing()
    rs0, rd0 = si.materials(m.n_tris, 5)
    sc = p.Scene.from_mesh(m)
    sun = si.fibonacci_dirs(8)
    params = p.TraceParams(nu=64, nv=64, bounces=3, seed=3)
    dev = torch.device("cuda")
    rs = torch.tensor(rs0, device=dev, requires_grad=True)
    rd = torch.tensor(rd0, device=dev, requires_grad=True)
    ang = torch.tensor([0.1, -0.2], dtype=torch.float64, requires_grad=True)
    F, T = p.srp_force(sc, sun, params, rs, rd, ang)
    w = torch.linspace(-1, 1, 24, dtype=torch.float64, device=dev).reshape(8, 3)
    L = (F * w).sum() + (T * w.flip(0)).sum()
    L.backward()
    grs, grd, gh = sc.adjoint(sun, params, w, w.flip(0).contiguous())
    torch.cuda.synchronize()
    assert torch.allclose(rs.grad, grs, rtol=1e-6, atol=0)
    assert torch.allclose(rd.grad, grd, rtol=1e-6, atol=0)
    assert torch.allclose(ang.grad, gh.cpu(), rtol=1e-9, atol=0)
    # forward values equal a plain trace of the same design
    F2, _ = sc.trace(sun, params)
    assert torch.equal(F.detach(), F2)


def test_adjoint_invalid_arguments():
    p = _lib()
    m = si.box_wing()
    sc = p.Scene.from_mesh(m)
    sc.set_design(*si.materials(m.n_tris, 1))
    with pytest.raises(p.SRPError):
        p.srp_trace_adjoint(sc.handle, torch.zeros((2, 3), dtype=torch.float64, device="cuda"),
                            p.TraceParams(nu=8, nv=8, bounces=9), torch.zeros((2, 3), dtype=torch.float64, device="cuda"))
    with pytest.raises(p.SRPError):
        p.srp_trace_adjoint(sc.handle, torch.zeros((2, 3), dtype=torch.float64, device="cuda"),
                            p.TraceParams(nu=8, nv=8), None)


def test_full_size_adjoint_sampled_direction():
    """The fwd+adjoint benchmark's adjoint launch (20.6k satellite, 1024 Fibonacci directions x 512^2
    rays, 3 bounces, jitter seed 2) with the cotangents nonzero on one direction only: the reflectance
    gradients are that direction's contribution and must match the oracle's FP64 adjoint of it."""
    m = si.meo_satellite()
    rs, rd = si.materials(m.n_tris, 1)
    p = _lib()
    sc = p.Scene.from_mesh(m)
    sc.set_design(rs, rd, hinge_angles=[0.0, 0.0])
    V = apply_hinges(m.verts, m.vert_hinge, m.hinge_origin, m.hinge_axis, [0.0, 0.0])
    sun = si.fibonacci_dirs(1024)
    j0 = 333
    rng = np.random.default_rng(3)
    gF = np.zeros((1024, 3))
    gT = np.zeros((1024, 3))
    gF[j0] = rng.standard_normal(3)
    gT[j0] = rng.standard_normal(3)
    params = p.TraceParams(nu=512, nv=512, bounces=3, jitter=1, seed=2)
    grs, grd, gh = sc.adjoint(sun, params, gF, gT)
    torch.cuda.synchronize()
    o_rs, o_rd, deg = oracle.trace_adjoint_rho(V, m.tris, rs, rd, sun[j0:j0 + 1], gF[j0:j0 + 1], gT[j0:j0 + 1],
                                               nu=512, nv=512, bounces=3, seed=2, dir_index_base=j0,
                                               drop_degenerate=True)
    # the same launch with direction j0's degenerate paths masked
    mask = torch.zeros((1024, 512 * 512 // 32), dtype=torch.int32, device="cuda")
    mask[j0] = p.ray_mask_bits(deg)[0]
    pm = p.TraceParams(nu=512, nv=512, bounces=3, jitter=1, seed=2, ray_mask=mask)
    mrs, mrd, _ = sc.adjoint(sun, pm, gF, gT)
    torch.cuda.synchronize()
    e = rel_l2(np.concatenate([mrs.cpu().numpy(), mrd.cpu().numpy()]), np.concatenate([o_rs, o_rd]))
    f_rs, f_rd = oracle.trace_adjoint_rho(V, m.tris, rs, rd, sun[j0:j0 + 1], gF[j0:j0 + 1], gT[j0:j0 + 1], nu=512,
                                          nv=512, bounces=3, seed=2, dir_index_base=j0)
    e_all = rel_l2(np.concatenate([grs.cpu().numpy(), grd.cpu().numpy()]), np.concatenate([f_rs, f_rd]))
    print(f"full-size adjoint, direction {j0}: rho-gradient rel L2 {e:.3e} without the {deg.mean():.2e} "
          f"degenerate paths; all paths {e_all:.3e}")
    assert e <= 1e-4
    assert np.isfinite(gh.cpu().numpy()).all()
