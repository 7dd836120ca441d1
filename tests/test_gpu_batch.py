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


def test_full_size_batch_sampled():
    """The batched benchmark launch itself: 256 MEO-style variants (log-uniform 2k-50k tris, random
    hinges and materials), 256 Fibonacci directions x 512^2 rays, 3 bounces, one launch.  Sampled
    designs equal their single-scene traces; two directions of the smallest design match the oracle."""
    from concurrent.futures import ThreadPoolExecutor
    import paper_2602_10712_amd as p
    S, D, G = 256, 256, 512
    rng = np.random.default_rng(6)
    sizes = np.exp(rng.uniform(np.log(2000.0), np.log(50000.0), S)).astype(int)
    dsg = si.random_designs(S, seed=6)

    def make(k):
        m = si.meo_variant(int(sizes[k]))
        sc = p.Scene.from_mesh(m)
        rs, rd = si.materials(m.n_tris, 100 + k)
        sc.set_design(rs, rd, hinge_angles=dsg[k][:2])
        return sc, m, rs, rd

    with ThreadPoolExecutor(16) as ex:
        built = list(ex.map(make, range(S)))
    scenes = [b[0] for b in built]
    sun = si.fibonacci_dirs(D)
    sd = torch.as_tensor(sun, device="cuda")
    params = p.TraceParams(nu=G, nv=G, bounces=3, jitter=1, seed=2)
    F = torch.empty((S, D, 3), dtype=torch.float64, device="cuda")
    T = torch.empty_like(F)
    p.srp_batch_trace(scenes, sd, params, F, T)
    torch.cuda.synchronize()
    n_tris = np.array([b[1].n_tris for b in built])
    small = int(np.argmin(n_tris))
    for k in (small, int(np.argsort(n_tris)[S // 2]), int(np.argmax(n_tris)), 7, 200):
        pk = p.TraceParams(nu=G, nv=G, bounces=3, jitter=1, seed=2, design_index=k)
        Fs, Ts = scenes[k].trace(sd, pk)
        torch.cuda.synchronize()
        e = rel_l2(F[k].cpu().numpy(), Fs.cpu().numpy())
        print(f"[batch design {k}, {n_tris[k]} tris] vs single-scene trace: rel L2 {e:.2e}")
        assert e <= 1e-9
        assert rel_l2(T[k].cpu().numpy(), Ts.cpu().numpy()) <= 1e-9
    sc, m, rs, rd = built[small][0], built[small][1], built[small][2], built[small][3]
    V = apply_hinges(m.verts, m.vert_hinge, m.hinge_origin, m.hinge_axis, dsg[small][:2])
    assert np.allclose(sc.vertices(), V, rtol=0, atol=1e-12)
    for j in (17, 190):
        ref = oracle.trace(V, m.tris, rs, rd, sun[j:j + 1], nu=G, nv=G, bounces=3, seed=2, dir_index_base=j,
                           design_index=small)
        e = rel_l2(F[small, j:j + 1].cpu().numpy(), ref.force)
        print(f"[batch design {small}, direction {j}] vs oracle: force rel L2 {e:.2e}")
        assert e <= 1e-4
    for sc in scenes:
        sc.close()


def test_tiles_per_wave_and_autotuner():
    """tiles_per_wave changes only the launch shape: forces agree to FP32 summation order (single
    scene and batched, including the direction-major order of fewer than 8 units); the autotuner
    returns one of its candidates 8..16 with a positive time for each."""
    import paper_2602_10712_amd as p
    scenes = []
    for k, n in enumerate([3000, 12000, 30000]):
        m = si.meo_variant(n)
        th = si.random_designs(1, seed=300 + k)[0]
        rs, rd = si.materials(m.n_tris, seed=400 + k)
        sc = p.Scene.from_mesh(m)
        sc.set_design(rs, rd, hinge_angles=th[:2])
        scenes.append(sc)
    dev = torch.device("cuda")
    for D in (3, 12):
        sun = torch.as_tensor(si.fibonacci_dirs(D), dtype=torch.float64, device=dev).contiguous()
        out = []
        for tpw in (0, 1, 7, 16):
            prm = p.TraceParams(nu=160, nv=160, bounces=3, seed=9, tiles_per_wave=tpw)
            # design s of a batch draws with design index s: trace design 1 alone with index 1
            F, T = scenes[1].trace(sun.cpu().numpy(), p.TraceParams(nu=160, nv=160, bounces=3, seed=9,
                                                                    design_index=1, tiles_per_wave=tpw))
            Fb = torch.empty((3, D, 3), dtype=torch.float64, device=dev)
            p.srp_batch_trace(scenes, sun, prm, Fb)
            torch.cuda.synchronize()
            out.append((F.cpu().numpy(), Fb.cpu().numpy()))
        for F, Fb in out[1:]:
            assert rel_l2(F, out[0][0]) <= 1e-6
            assert rel_l2(Fb, out[0][1]) <= 1e-6
        assert rel_l2(out[0][1][1], out[0][0]) <= 1e-6  # design 1 of the batch vs its own trace
    with pytest.raises(p.SRPError):
        scenes[0].trace(si.fibonacci_dirs(2), p.TraceParams(nu=16, nv=16, tiles_per_wave=17))
    sun = torch.as_tensor(si.fibonacci_dirs(8), dtype=torch.float64, device=dev).contiguous()
    prm = p.TraceParams(nu=128, nv=128, bounces=3, seed=9)
    for group in (scenes, scenes[:1]):
        best, ms = p.srp_autotune_tiles_per_wave(group, sun, prm)
        assert 8 <= best <= 16 and sorted(ms) == list(range(8, 17))
        assert all(v > 0.0 for v in ms.values()) and ms[best] == min(ms.values())
    for sc in scenes:
        sc.close()
