"""Surrogate MLP kernels vs the FP64 oracle with BF16 rounding emulation (oracle/mlp.py).

Bars: forward outputs and gradients within 1e-3 relative L2 of
the emulating oracle (FP32 accumulation order and rare single-activation rounding flips); one Adam
step within 1e-3 of the oracle's update; checkpoint/resume reproduces the next step bit for bit.
"""
import numpy as np
import pytest

from oracle import mlp as om

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def rel_l2(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - np.asarray(b, np.float64)) / max(np.linalg.norm(b), 1e-300))


def _lib():
    import paper_2602_10712_amd as p
    return p


@pytest.mark.parametrize("N,width,depth", [(1000, 256, 4), (77, 64, 2), (1, 256, 4), (4099, 32, 1)])
def test_forward_backward_match_oracle(N, width, depth):
    p = _lib()
    n_in, n_out = 11, 3
    s = p.Surrogate(n_in, width, depth, n_out, seed=1)
    flat = om.init_params(n_in, width, depth, n_out, seed=7)
    s.set_params(flat)
    rng = np.random.default_rng(N)
    x = rng.uniform(-1, 1, (N, n_in)).astype(np.float32)
    t = rng.standard_normal((N, n_out)).astype(np.float32)
    layers = om.unpack(flat, n_in, width, depth, n_out)
    y_ref, cache = om.forward(layers, x, emulate=True)
    # inference path and training path
    y_inf = s.forward(x).cpu().numpy()
    assert rel_l2(y_inf, y_ref) <= 1e-3
    y = s.forward(x, keep_activations=True)
    assert rel_l2(y.cpu().numpy(), y_ref) <= 1e-3
    loss_ref, gy_ref = om.mse_grad(y_ref, t)
    g_y = torch.empty_like(y)
    loss = torch.empty(1, dtype=torch.float64, device="cuda")
    p.srp_mlp_mse(s.handle, y, torch.as_tensor(t, device="cuda"), g_y, loss)
    assert abs(loss.item() - loss_ref) <= 1e-3 * loss_ref
    g_x = torch.empty((N, n_in), dtype=torch.float32, device="cuda")
    p.srp_mlp_backward(s.handle, g_y, g_x)
    torch.cuda.synchronize()
    grads_ref, gx_ref = om.backward(layers, cache, gy_ref, emulate=True)
    got = s.get_params()["grads"]
    e = rel_l2(got, om.flatten(grads_ref))
    print(f"N={N} width={width} depth={depth}: grad rel L2 {e:.2e}")
    assert e <= 1e-3
    assert rel_l2(g_x.cpu().numpy(), gx_ref) <= 2e-3


@pytest.mark.parametrize("N,depth,n_in,n_out", [(1, 4, 11, 3), (257, 1, 11, 3), (1000, 2, 16, 32), (1000, 7, 11, 3),
                                               (1 << 20, 4, 11, 3)])
def test_fused_inference_matches_oracle(N, depth, n_in, n_out):
    """The fused width-256 inference kernel (persistent workgroups, streamed half layers) against the
    emulating oracle; for N = 2^20 (the benchmark batch) every workgroup runs 16 tiles, checked on sampled rows
    (queries are independent)."""
    p = _lib()
    s = p.Surrogate(n_in, 256, depth, n_out, seed=1)
    flat = om.init_params(n_in, 256, depth, n_out, seed=11 + depth)
    s.set_params(flat)
    rng = np.random.default_rng(N + depth)
    x = rng.uniform(-1, 1, (N, n_in)).astype(np.float32)
    y = s.forward(x).cpu().numpy()
    rows = np.arange(N) if N <= 4096 else np.sort(rng.choice(N, 3000, replace=False))
    rows = np.union1d(rows, [N - 1])
    layers = om.unpack(flat, n_in, 256, depth, n_out)
    y_ref, _ = om.forward(layers, x[rows], emulate=True)
    e = rel_l2(y[rows], y_ref)
    print(f"fused N={N} depth={depth} n_in={n_in} n_out={n_out}: rel L2 {e:.2e}")
    assert e <= 1e-3
    assert np.isfinite(y).all()


def test_adam_step_and_checkpoint_resume():
    p = _lib()
    n_in, width, depth, n_out = 11, 256, 4, 3
    flat = om.init_params(n_in, width, depth, n_out, seed=3)
    rng = np.random.default_rng(0)
    x = rng.uniform(-1, 1, (512, n_in)).astype(np.float32)
    t = (0.1 * rng.standard_normal((512, n_out))).astype(np.float32)
    s = p.Surrogate(n_in, width, depth, n_out)
    s.set_params(flat)
    # eps = 1 makes the first update proportional to the gradient (not its sign)
    s.train_step(x, torch.as_tensor(t, device="cuda"), lr=1e-2, eps=1.0)
    st = s.get_params()
    layers = om.unpack(flat, n_in, width, depth, n_out)
    y, cache = om.forward(layers, x)
    _, gy = om.mse_grad(y, t)
    grads, _ = om.backward(layers, cache, gy)
    g = om.flatten(grads)
    p1, m1, v1 = om.adam_step(flat, g, np.zeros_like(g), np.zeros_like(g), 1, 1e-2, 0.9, 0.999, 1.0)
    # the first moment is (1 - beta1) g: the gradient itself
    assert rel_l2(st["adam_m"], m1) <= 1e-3
    # the update is ~1e-5 on weights ~0.25: compare it up to the float32 spacing of the weights
    d_gpu = st["params"].astype(np.float64) - flat
    d_ref = p1 - flat
    tol = 1e-2 * np.abs(d_ref) + 4 * np.spacing(np.abs(flat).astype(np.float32)).astype(np.float64)
    assert np.all(np.abs(d_gpu - d_ref) <= tol)
    assert rel_l2(d_gpu, d_ref) <= 3e-3
    assert st["step"] == 1 and not st["grads"].any()
    # checkpoint -> new network -> identical next step
    s2 = p.Surrogate(n_in, width, depth, n_out, seed=99)
    s2.set_params(st["params"], st["adam_m"], st["adam_v"], st["step"])
    tt = torch.as_tensor(t, device="cuda")
    s.train_step(x, tt, lr=1e-3)
    s2.train_step(x, tt, lr=1e-3)
    a, b = s.get_params(), s2.get_params()
    assert np.array_equal(a["params"], b["params"]) and np.array_equal(a["adam_v"], b["adam_v"])


def test_mlp_invalid_arguments():
    p = _lib()
    with pytest.raises(p.SRPError):
        p.srp_mlp_create(11, 250, 4, 3)
    s = p.Surrogate(11, 64, 2, 3)
    with pytest.raises(p.SRPError):  # backward without a kept forward
        p.srp_mlp_backward(s.handle, torch.zeros((4, 3), dtype=torch.float32, device="cuda"))
    with pytest.raises(ValueError):
        s.set_params(np.zeros(5, np.float32))


def test_inference_in_a_captured_graph_replays_like_eager():
    """Fused inference captured into a HIP graph (it allocates and clears nothing): every replay,
    with eager work and synchronisations between replays, equals the eager result bit for bit."""
    import paper_2602_10712_amd as p
    net = p.Surrogate(11, 256, 4, 6, seed=12)
    dev = torch.device("cuda")
    g = torch.Generator(device="cpu").manual_seed(12)
    xs = [(torch.rand((5000 + 700 * i, 11), generator=g) * 2 - 1).to(dev) for i in range(3)]
    ys = [torch.empty((x.shape[0], 6), dtype=torch.float32, device=dev) for x in xs]
    eager = []
    for x in xs:
        y = torch.empty((x.shape[0], 6), dtype=torch.float32, device=dev)
        p.srp_mlp_forward(net.handle, x, y)
        eager.append(y)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        cap = torch.cuda.current_stream()
        for x, y in zip(xs, ys):
            p.srp_mlp_forward(net.handle, x, y, stream=cap.cuda_stream)
    for rep in range(4):
        for y in ys:
            y.fill_(float("nan"))
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        for y, e in zip(ys, eager):
            assert torch.equal(y, e), rep
        # eager work between replays
        scratch = torch.empty((9000, 6), dtype=torch.float32, device=dev)
        p.srp_mlp_forward(net.handle, torch.rand((9000, 11), device=dev), scratch)
        torch.cuda.synchronize()
    del graph
    net.close()
