"""Pins of the MLP oracle (CPU only): torch FP64 autograd, torch bfloat16 rounding, torch Adam."""
import numpy as np
import torch

from oracle import mlp


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(100000) * 10 ** rng.uniform(-30, 30, 100000),
                        [0.0, -0.0, 1.0, 1.00390625, 1.01171875, 65504.0, 3.0e38, -1e-40]]).astype(np.float32)
    ref = torch.tensor(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(mlp.bf16(x), ref)


def torch_net(layers):
    params = []
    for W, b in layers:
        params.append(torch.tensor(W, dtype=torch.float64, requires_grad=True))
        params.append(torch.tensor(b, dtype=torch.float64, requires_grad=True))
    return params


def test_forward_backward_match_torch_fp64():
    n_in, width, depth, n_out = 11, 64, 3, 3
    flat = mlp.init_params(n_in, width, depth, n_out, seed=3)
    layers = mlp.unpack(flat, n_in, width, depth, n_out)
    rng = np.random.default_rng(1)
    x = rng.uniform(-1, 1, (37, n_in))
    t = rng.standard_normal((37, n_out))
    y, cache = mlp.forward(layers, x, emulate=False)
    loss, gy = mlp.mse_grad(y, t)
    grads, gx = mlp.backward(layers, cache, gy, emulate=False)

    params = torch_net(layers)
    xt = torch.tensor(x, requires_grad=True)
    h = xt
    for l in range(depth + 1):
        h = h @ params[2 * l].T + params[2 * l + 1]
        if l < depth:
            h = torch.nn.functional.silu(h)
    lt = ((h - torch.tensor(t)) ** 2).mean()
    lt.backward()
    assert np.allclose(y, h.detach().numpy(), rtol=1e-12, atol=1e-14)
    assert abs(loss - lt.item()) < 1e-12
    ref = np.concatenate([np.concatenate([params[2 * l].grad.numpy().ravel(), params[2 * l + 1].grad.numpy()])
                          for l in range(depth + 1)])
    assert np.allclose(mlp.flatten(grads), ref, rtol=1e-10, atol=1e-14)
    assert np.allclose(gx, xt.grad.numpy(), rtol=1e-10, atol=1e-14)


def test_adam_matches_torch():
    rng = np.random.default_rng(2)
    p0 = rng.standard_normal(50)
    pt = torch.tensor(p0, requires_grad=True)
    opt = torch.optim.Adam([pt], lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    p, m, v = p0.copy(), np.zeros(50), np.zeros(50)
    for step in range(1, 6):
        g = rng.standard_normal(50)
        pt.grad = torch.tensor(g)
        opt.step()
        p, m, v = mlp.adam_step(p, g, m, v, step, 1e-3, 0.9, 0.999, 1e-8)
        assert np.allclose(p, pt.detach().numpy(), rtol=1e-12, atol=1e-15)


def test_emulated_rounding_is_small_perturbation():
    n_in, width, depth, n_out = 11, 256, 4, 3
    flat = mlp.init_params(n_in, width, depth, n_out, seed=4)
    layers = mlp.unpack(flat, n_in, width, depth, n_out)
    x = np.random.default_rng(5).uniform(-1, 1, (64, n_in))
    y_e, _ = mlp.forward(layers, x, emulate=True)
    y_x, _ = mlp.forward(layers, x, emulate=False)
    rel = np.linalg.norm(y_e - y_x) / np.linalg.norm(y_x)
    assert 1e-5 < rel < 3e-2  # bf16 has 8 significant bits
    assert mlp.n_params(11, 256, 4, 3) == 201219
