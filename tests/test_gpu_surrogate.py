"""The learned part end to end on the GPU: tracer-generated samples over random designs, training
with the library's BF16-MFMA kernels, the two-network ensemble with the library's confidence test
(srp_mlp_ensemble) and tracer fallback, its accuracy against a high-resolution tracer, and the gain
over the plain tracer at matched error.

Training set: 4096 random designs x 256 random sun directions = 1,048,576 samples traced at 128^2
rays, 3 bounces (label noise about 0.5 %); two networks, 30,000 Adam steps of 4096 samples each
(cosine decay from 1e-3).  Held out: 16,384 (design, direction) pairs traced at 1024^2 as the
reference, in two splits of 32 new designs x 256 new directions: the calibration split fixes the
disagreement threshold (accepted queries at <= 1 % relative RMS, and the 1 % of queries on which the
two networks disagree most always sent to the tracer),
the evaluation split checks the bar -- relative RMS <= 1 % for the answers the pipeline gives, the
surrogate's where it passes the test and the tracer's (256^2) where it does not."""
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
    n_d, k = 4096, 256
    designs = si.random_designs(n_d, seed=4)
    sun = si.random_dirs(n_d * k, seed=41).reshape(n_d, k, 3)
    t0 = time.perf_counter()
    F = S.generate_samples(mesh, designs, sun, p.TraceParams(nu=128, nv=128, bounces=3, seed=1))
    gen_s = time.perf_counter() - t0
    x = S.input_features(sun.reshape(-1, 3), np.repeat(designs, k, 0), lo, hi)
    y = (F.reshape(-1, 3) / f_ref).astype(np.float32)
    assert len(x) == 1 << 20
    # held out: new designs and directions, traced at 1024^2 as the reference
    held = si.random_designs(64, seed=5)
    sun_h = si.random_dirs(64 * 256, seed=51).reshape(64, 256, 3)
    t0 = time.perf_counter()
    F_h = S.generate_samples(mesh, held, sun_h, p.TraceParams(nu=1024, nv=1024, bounces=3, seed=2))
    ref_s = time.perf_counter() - t0
    split = {}
    for name, sl in (("calib", slice(0, 32)), ("eval", slice(32, 64))):
        th = np.repeat(held[sl], 256, 0)
        sd = sun_h[sl].reshape(-1, 3)
        split[name] = (sd, th, S.input_features(sd, th, lo, hi), F_h[sl].reshape(-1, 3))
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
    # calibration split: the threshold
    _, _, x_c, F_c = split["calib"]
    mean_c, dis_c = sf.predict(x_c)
    pred_c = mean_c.double().cpu().numpy() * f_ref
    err_c = ((pred_c - F_c) ** 2).sum(1) / (F_c ** 2).sum(1).mean()
    thr = S.SurrogateForce.calibrate(dis_c.cpu().numpy(), err_c, target=0.01, max_coverage=0.99)
    sf.threshold = thr
    print(f"samples {len(x)} (generation {gen_s:.1f} s, reference {ref_s:.1f} s), training 2 x {steps} steps "
          f"{train_s:.1f} s; calibration split: ensemble relative RMS {S.rel_rms(pred_c, F_c):.4f}, threshold {thr:.3e}")
    # evaluation split: the pipeline's answers (surrogate where trusted, tracer at 256^2 elsewhere)
    sd_e, th_e, x_e, F_e = split["eval"]
    mean_e, dis_e = sf.predict(x_e)
    pred_e = mean_e.double().cpu().numpy() * f_ref
    fb_params = p.TraceParams(nu=256, nv=256, bounces=3, seed=2)
    Fq, fall = sf.forces(mesh, sd_e, th_e, fb_params)
    Fq = Fq.double().cpu().numpy()
    err_all = S.rel_rms(pred_e, F_e)
    err_pipe = S.rel_rms(Fq, F_e)
    acc = ~fall
    err_acc = S.rel_rms(pred_e[acc], F_e[acc])
    err_rej = S.rel_rms(pred_e[fall], F_e[fall]) if fall.any() else 0.0
    print(f"evaluation split: surrogate alone {err_all:.4f}; {fall.mean():.3%} of queries fail the disagreement "
          f"test (their surrogate error {err_rej:.4f} vs {err_acc:.4f} accepted); pipeline {err_pipe:.4f}")
    assert err_pipe <= 0.01
    assert 0 < fall.sum() <= 0.05 * len(fall)  # the disagreement path fires (every query is in the domain)
    assert err_rej > err_acc  # disagreement singles out the worse answers
    # the accepted queries keep the ensemble's answer
    assert np.allclose(Fq[acc], pred_e[acc], rtol=1e-6, atol=0)

    # tracer at decreasing resolution on the evaluation queries: error vs the 1024^2 reference
    tracer_err = {}
    for g in (32, 64, 128, 256):
        Fg = S.generate_samples(mesh, held[32:64], sun_h[32:64], p.TraceParams(nu=g, nv=g, bounces=3, seed=9))
        tracer_err[g] = S.rel_rms(Fg.reshape(-1, 3), F_e)
    print("tracer relative RMS by grid:", {g: round(e, 4) for g, e in tracer_err.items()})
    g_match = min([g for g, e in tracer_err.items() if e <= err_pipe] or [256])
    # throughputs: tracer at that grid (1024 directions of one design); the ensemble with its
    # confidence test and compaction on 2^20 queries
    sc = p.Scene.from_mesh(mesh)
    th = held[40]
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
    xq = torch.as_tensor(np.tile(x_e, ((1 << 20) // len(x_e) + 1, 1))[: 1 << 20], device="cuda").contiguous()
    sf.evaluate(xq)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(5):
        sf.evaluate(xq)
    torch.cuda.synchronize()
    surr_eps = 5 * (1 << 20) / (time.perf_counter() - t0)
    gain = surr_eps / tracer_eps
    print(f"matched error: tracer {g_match}^2 x 3 bounces {tracer_eps / 1e6:.3f} M evals/s vs ensemble with its "
          f"confidence test {surr_eps / 1e6:.1f} M evals/s: gain {gain:.0f}x")
    assert gain >= 1000.0
    # out of the domain: a design outside the box and a non-unit direction go to the tracer
    q_theta = np.stack([held[40], held[40].copy(), held[41]])
    q_theta[1, 2] = 0.55  # rho_s_bus above the box (rho_s + rho_d stays <= 1)
    q_theta[1, 3] = 0.1
    q_sun = sun_h[40, :3].copy()
    q_sun[2] *= 1.01
    Fo, fall_o = sf.forces(mesh, q_sun, q_theta, fb_params)
    assert fall_o[1] and fall_o[2]
    ref = S.generate_samples(mesh, q_theta[1:2], q_sun[1:2][None], fb_params)
    assert np.allclose(Fo[1].double().cpu().numpy(), ref[0, 0], rtol=1e-6)
    sc.close()

    # the proxy inside the ODE (Alg. 1): one design-gradient iteration of the orbit problem with the
    # ensemble answering the force at every stage time, against the same iteration with the tracer
    scn = si.meo_orbit(n_steps=240, dt=60.0)
    theta_c = held[40].copy()
    delta = np.array([0.0, 0.0, 0.04, -0.04, 0.03, 0.03, -0.03, 0.02])
    tp = p.DesignProblem(mesh, scn, p.TraceParams(nu=256, nv=256, bounces=3, seed=5), lo, hi)
    tp.r_target = tp.final_state(theta_c + delta)[0][:3]
    spb = p.SurrogateDesignProblem(mesh, scn, nets, f_ref, lo, hi, r_target=tp.r_target)
    F_t, F_s = tp.forces(theta_c), spb.forces(theta_c)
    err_f = np.linalg.norm(F_s - F_t) / np.linalg.norm(F_t)
    L_s, g_s = spb.loss_and_grad(theta_c)
    L_t, g_t = tp.loss_and_grad(theta_c)
    # the surrogate's own gradient against central differences of its loss (steps of 4 % of each
    # reflectance range: the BF16 inputs quantise the network below that)
    fd = np.zeros(6)
    for k in range(2, 8):
        hp, hm = theta_c.copy(), theta_c.copy()
        hp[k] += 0.02
        hm[k] -= 0.02
        fd[k - 2] = (spb.loss(hp) - spb.loss(hm)) / 0.04
    err_g = np.abs(g_s[2:] - fd).max() / np.abs(fd).max()
    cos = g_s[2:] @ g_t[2:] / (np.linalg.norm(g_s[2:]) * np.linalg.norm(g_t[2:]))
    times = {}
    for name, prob in (("tracer", tp), ("surrogate", spb)):
        prob.loss_and_grad(theta_c)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(5):
            prob.loss_and_grad(theta_c)
        torch.cuda.synchronize()
        times[name] = (time.perf_counter() - t0) / 5
    print(f"orbit iteration (481 stage times, 256^2 tracer): forces {err_f:.4f} apart; loss tracer {L_t:.4e}, "
          f"surrogate {L_s:.4e}; reflectance gradient vs its central differences {err_g:.4f}, cosine to the "
          f"tracer's {cos:.4f}; {times['tracer'] * 1e3:.2f} ms vs {times['surrogate'] * 1e3:.2f} ms per iteration")
    assert err_f <= 0.02
    assert err_g <= 0.05
    assert cos >= 0.9
    tp.close()


def test_ensemble_confidence_call():
    """srp_mlp_ensemble on hand-made queries: the mean is the average of the two networks, the
    disagreement their distance, and the failing queries (domain or disagreement) come out in
    ascending order; empty input; unequal networks are refused."""
    import paper_2602_10712_amd as p
    a = p.Surrogate(11, 64, 2, 3, seed=1)
    b = p.Surrogate(11, 64, 2, 3, seed=2)
    rng = np.random.default_rng(3)
    n = 5000
    s = rng.standard_normal((n, 3))
    s /= np.linalg.norm(s, axis=1)[:, None]
    d = rng.uniform(-1, 1, (n, 8))
    d[7, 4] = 1.5          # design outside the box
    s[11] *= 1.1           # not a unit vector
    d[4000, 0] = -1.0 - 1e-3
    x = torch.as_tensor(np.concatenate([s, d], 1).astype(np.float32), device="cuda")
    ya = a.forward(x).double().cpu().numpy()
    yb = b.forward(x).double().cpu().numpy()
    dist = np.linalg.norm(ya - yb, axis=1)
    thr = float(np.quantile(dist, 0.9))
    y = torch.empty((n, 3), dtype=torch.float32, device="cuda")
    dis = torch.empty(n, dtype=torch.float32, device="cuda")
    idx = torch.full((n,), -7, dtype=torch.int32, device="cuda")
    cnt = torch.empty(1, dtype=torch.int32, device="cuda")
    p.srp_mlp_ensemble(a.handle, b.handle, x, thr, 2.5, y, idx, cnt, disagree=dis)
    torch.cuda.synchronize()
    assert np.allclose(y.cpu().numpy(), 2.5 * 0.5 * (ya + yb), rtol=1e-6, atol=1e-7)
    assert np.allclose(dis.cpu().numpy(), dist, rtol=1e-5, atol=1e-7)
    expect = np.flatnonzero((dis.cpu().numpy() > thr) | np.isin(np.arange(n), [7, 11, 4000]))
    m = int(cnt.item())
    assert m == len(expect) and np.array_equal(idx.cpu().numpy()[:m], expect)
    # empty input writes a zero count
    p.srp_mlp_ensemble(a.handle, b.handle, x[:0], thr, 1.0, y, idx, cnt)
    torch.cuda.synchronize()
    assert int(cnt.item()) == 0
    c = p.Surrogate(11, 64, 2, 6, seed=3)
    with pytest.raises(p.SRPError):
        p.srp_mlp_ensemble(a.handle, c.handle, x, thr, 1.0, y, idx, cnt)
    for net in (a, b, c):
        net.close()
