"""The learned part end to end on the GPU: tracer-generated samples over random designs, training
with the library's BF16-MFMA kernels, accuracy against a high-resolution tracer on held-out
(direction, design) pairs (bar: relative RMS <= 1 % against 1024^2 rays, 3 bounces), tracer
fallback, and the gain over the plain tracer at matched error.

Training set: 2048 random designs x 128 random sun directions = 262,144 samples traced at 128^2 rays
(label noise about 0.5 %); two networks, 30,000 Adam steps of 4096 samples each (cosine decay from
1e-3).  Held out: 128 new designs x 16 new directions at 1024^2."""
import time

import numpy as np
import pytest

import srp_inputs as si

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

PHI, C = 1361.0, 299792458.0


def test_surrogate_trains_and_beats_tracer_at_matched_error():
    import paper_2602_10712_amd as p
    from paper_2602_10712_amd import surrogate as S
    mesh = si.meo_satellite()
    lo, hi = si.DESIGN_LO, si.DESIGN_HI
    f_ref = PHI * 20.0 / C
    rng = np.random.default_rng(4)
    n_d, k = 2048, 128
    designs = si.random_designs(n_d, seed=4)
    sun = si.random_dirs(n_d * k, seed=41).reshape(n_d, k, 3)
    t0 = time.perf_counter()
    F = S.generate_samples(mesh, designs, sun, p.TraceParams(nu=128, nv=128, bounces=3, seed=1))
    gen_s = time.perf_counter() - t0
    x = S.input_features(sun.reshape(-1, 3), np.repeat(designs, k, 0), lo, hi)
    y = (F.reshape(-1, 3) / f_ref).astype(np.float32)
    # held out: new designs and directions, traced at 1024^2 as the reference
    designs_t = si.random_designs(128, seed=5)
    sun_t = si.random_dirs(128 * 16, seed=51).reshape(128, 16, 3)
    F_t = S.generate_samples(mesh, designs_t, sun_t, p.TraceParams(nu=1024, nv=1024, bounces=3, seed=2)).reshape(-1, 3)
    x_t = S.input_features(sun_t.reshape(-1, 3), np.repeat(designs_t, 16, 0), lo, hi)
    nets = []
    t0 = time.perf_counter()
    steps = 30000
    for s in range(2):
        net = p.Surrogate(11, 256, 4, 3, seed=100 + s)
        S.train(net, x, y, steps=steps, batch=4096, lr=1e-3, seed=s)
        nets.append(net)
        print(f"network {s} trained", flush=True)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    sf = S.SurrogateForce(nets, lo, hi, f_ref, threshold=np.inf)
    mean, dis = sf.predict(x_t)
    pred = mean.double().cpu().numpy() * f_ref
    err = S.rel_rms(pred, F_t)
    print(f"samples {len(x)} (generation {gen_s:.1f} s), training 2 x {steps} steps {train_s:.1f} s, "
          f"held-out relative RMS {err:.4f}")
    assert err <= 0.01
    # tracer at decreasing resolution on the same held-out queries: error vs the 512^2 reference
    tracer_err = {}
    for g in (32, 64, 128, 256):
        Fg = S.generate_samples(mesh, designs_t, sun_t, p.TraceParams(nu=g, nv=g, bounces=3, seed=9)).reshape(-1, 3)
        tracer_err[g] = S.rel_rms(Fg, F_t)
    print("tracer relative RMS by grid:", {g: round(e, 4) for g, e in tracer_err.items()})
    g_match = min([g for g, e in tracer_err.items() if e <= err] or [256])
    # throughputs: tracer at that grid (1024 directions of one design), surrogate at 1M queries
    sc = p.Scene.from_mesh(mesh)
    th = designs_t[0]
    sc.set_design(th[2 + 2 * mesh.group].astype(np.float32), th[3 + 2 * mesh.group].astype(np.float32),
                  hinge_angles=th[:2])
    dirs = torch.as_tensor(si.random_dirs(1024, seed=7), device="cuda")
    prm = p.TraceParams(nu=g_match, nv=g_match, bounces=3, seed=3)
    sc.trace(dirs, prm)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(5):
        sc.trace(dirs, prm)
    torch.cuda.synchronize()
    tracer_eps = 5 * 1024 / (time.perf_counter() - t0)
    xq = torch.as_tensor(np.tile(x_t, (1 << 20) // len(x_t) + 1, ).reshape(-1, 11)[: 1 << 20], device="cuda")
    nets[0].forward(xq)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(5):
        nets[0].forward(xq)
    torch.cuda.synchronize()
    surr_eps = 5 * (1 << 20) / (time.perf_counter() - t0)
    print(f"matched error: tracer {g_match}^2 x 3 bounces {tracer_eps / 1e6:.2f} M evals/s vs surrogate "
          f"{surr_eps / 1e6:.1f} M evals/s: gain {surr_eps / tracer_eps:.0f}x")
    assert surr_eps > tracer_eps
    # fallback: a design outside the box and a non-unit direction go to the tracer
    calib_err = ((pred - F_t) ** 2).sum(1) / (F_t ** 2).sum(1).mean()
    thr = S.SurrogateForce.calibrate(dis.cpu().numpy(), calib_err, target=err)
    sf.threshold = thr
    q_theta = np.stack([designs_t[0], designs_t[0] + np.array([0, 0, 0.2, 0, 0, 0, 0, 0])])
    q_theta[1, 2] = 0.55  # rho_s_bus above the box (rho_s + rho_d stays <= 1)
    q_theta[1, 3] = 0.1
    q_sun = sun_t[0, :2]
    Fq, fall = sf.forces(mesh, q_sun, q_theta, p.TraceParams(nu=256, nv=256, bounces=3, seed=2))
    assert fall[1]
    ref = S.generate_samples(mesh, q_theta[1:], q_sun[1:][None], p.TraceParams(nu=256, nv=256, bounces=3, seed=2))
    assert np.allclose(Fq[1], ref[0, 0], rtol=1e-12)
