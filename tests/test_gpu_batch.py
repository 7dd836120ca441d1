"""Batched designs in one launch (srp_batch_trace): each design equals its own single-scene trace
with the same Philox design index, and a sampled design matches the oracle."""
import numpy as np
import pytest

import oracle
import srp_inputs as si
from oracle.design import apply_hinges

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def test_batch_matches_single_scene_traces_and_oracle():
    import paper_2602_10712_amd as p
    sizes = [2000, 5000, 9000, 14000, 20000, 26000, 33000, 41000, 50000]  # S = 9: not a multiple of 8
    rng = np.random.default_rng(8)
    scenes, meshes, designs = [], [], []
    for k, n in enumerate(sizes):
        m = si.meo_variant(n)
        th = si.random_designs(1, seed=100 + k)[0]
        rs, rd = si.materials(m.n_tris, seed=200 + k)
        sc = p.Scene.from_mesh(m)
        sc.set_design(rs, rd, hinge_angles=th[:2])
        scenes.append(sc)
        meshes.append((m, rs, rd, th))
    sun = si.fibonacci_dirs(16)
    sd = torch.as_tensor(sun, device="cuda")
    S, D = len(scenes), len(sun)
    prm = p.TraceParams(nu=64, nv=64, bounces=3, seed=4, design_index=10)
    F = torch.empty((S, D, 3), dtype=torch.float64, device="cuda")
    T = torch.empty((S, D, 3), dtype=torch.float64, device="cuda")
    p.srp_batch_trace(scenes, sd, prm, F, T)
    torch.cuda.synchronize()
    for s in range(S):
        ps = p.TraceParams(nu=64, nv=64, bounces=3, seed=4, design_index=10 + s)
        Fs, Ts = scenes[s].trace(sun, ps)
        torch.cuda.synchronize()
        assert rel_l2(F[s].cpu().numpy(), Fs.cpu().numpy()) <= 1e-6, s
        assert rel_l2(T[s].cpu().numpy(), Ts.cpu().numpy()) <= 1e-6, s
    s = 3
    m, rs, rd, th = meshes[s]
    V = apply_hinges(m.verts, m.vert_hinge, m.hinge_origin, m.hinge_axis, th[:2])
    ref = oracle.trace(V, m.tris, rs, rd, sun, nu=64, nv=64, bounces=3, seed=4, design_index=10 + s)
    assert rel_l2(F[s].cpu().numpy(), ref.force) <= 1e-4
    with pytest.raises(p.SRPError):
        p.srp_batch_trace(scenes, sd, p.TraceParams(nu=8, nv=8, frame_mode=1), F, T)
