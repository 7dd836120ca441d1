"""Oracle: the force surrogate network -- TEST INFRASTRUCTURE ONLY.

The paper represents the simulator by a neural proxy (Sec. 3.3, "Representation"): an MLP from
(light direction, design parameters) to force, trained with Adam on simulator samples.  The GPU
network is 11 -> 256 x 4 (SiLU) -> 3 with BF16 operands and FP32 accumulation.  This module is the
plain FP64 reference of that network, its gradients and its Adam update, written out with numpy
matrix products.  With `emulate=True` it rounds to bfloat16 (round-to-nearest-even) at exactly the
points where the GPU kernels round:
  * the network input and every weight matrix before a product,
  * every hidden activation SiLU(z) after it is formed in FP32,
  * every back-propagated gradient dL/dz before it enters a product.
Biases, pre-activations, SiLU and the loss gradient stay FP32 on the GPU (FP64 here).

Pinned by tests/test_oracle_mlp.py: with emulate=False the forward, backward and Adam step match
torch's FP64 autograd and torch.optim.Adam, and bf16() matches torch's bfloat16 conversion.
"""
from __future__ import annotations

import numpy as np


def bf16(x) -> np.ndarray:
    """Round to the nearest bfloat16 (ties to even) after rounding to float32; returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) & 0xFFFF0000).astype(np.uint32)
    out = r.view(np.float32).astype(np.float64)
    nan = np.isnan(f)
    if nan.any():
        out = np.where(nan, np.nan, out)
    return out


def f32(x) -> np.ndarray:
    return np.asarray(x, dtype=np.float32).astype(np.float64)


def sigmoid(z):
    return 1.0 / (1.0 + np.exp(-z))


def silu(z):
    return z * sigmoid(z)


def silu_grad(z):
    s = sigmoid(z)
    return s * (1.0 + z * (1.0 - s))


def unpack(flat, n_in, width, depth, n_out):
    """Flat parameter vector -> [(W [out][in], b [out])] in the library's order
    W0, b0, W1, b1, ..., W_out, b_out."""
    dims = [n_in] + [width] * depth + [n_out]
    out, o = [], 0
    for l in range(depth + 1):
        fi, fo = dims[l], dims[l + 1]
        W = np.asarray(flat[o:o + fo * fi], dtype=np.float64).reshape(fo, fi)
        o += fo * fi
        b = np.asarray(flat[o:o + fo], dtype=np.float64)
        o += fo
        out.append((W, b))
    assert o == len(flat)
    return out


def n_params(n_in, width, depth, n_out):
    dims = [n_in] + [width] * depth + [n_out]
    return sum(dims[l + 1] * dims[l] + dims[l + 1] for l in range(depth + 1))


def init_params(n_in, width, depth, n_out, seed):
    """Seeded initial weights: U(-1/sqrt(fan_in), 1/sqrt(fan_in)) for weights and biases."""
    rng = np.random.default_rng(seed)
    dims = [n_in] + [width] * depth + [n_out]
    flat = []
    for l in range(depth + 1):
        bound = 1.0 / np.sqrt(dims[l])
        flat.append(rng.uniform(-bound, bound, dims[l + 1] * dims[l]))
        flat.append(rng.uniform(-bound, bound, dims[l + 1]))
    return np.concatenate(flat).astype(np.float32)


def forward(layers, x, emulate=True):
    """y [N][n_out] and the cache (inputs of each layer, pre-activations of the hidden layers)."""
    q = bf16 if emulate else (lambda v: np.asarray(v, dtype=np.float64))
    r32 = f32 if emulate else (lambda v: np.asarray(v, dtype=np.float64))
    a = q(x)
    ins, zs = [], []
    for l, (W, b) in enumerate(layers):
        ins.append(a)
        z = r32(a @ q(W).T + r32(b))
        if l < len(layers) - 1:
            zs.append(z)
            a = q(r32(silu(z)))
        else:
            return z, (ins, zs)


def backward(layers, cache, g_y, emulate=True):
    """Gradients (dW, db) per layer and dL/dx for dL/dy = g_y."""
    q = bf16 if emulate else (lambda v: np.asarray(v, dtype=np.float64))
    r32 = f32 if emulate else (lambda v: np.asarray(v, dtype=np.float64))
    ins, zs = cache
    g = r32(g_y)
    grads = [None] * len(layers)
    for l in range(len(layers) - 1, -1, -1):
        W, _ = layers[l]
        gq = q(g)
        grads[l] = (r32(gq.T @ ins[l]), r32(g.sum(0)))
        g_in = gq @ q(W)
        if l > 0:
            g = r32(g_in * r32(silu_grad(zs[l - 1])))
        else:
            g = r32(g_in)
    return grads, g


def flatten(grads):
    return np.concatenate([np.concatenate([dW.ravel(), db.ravel()]) for dW, db in grads])


def mse_grad(y, target):
    """L = mean over all N x n_out entries of (y - t)^2 and dL/dy."""
    d = np.asarray(y, dtype=np.float64) - np.asarray(target, dtype=np.float64)
    return float((d * d).mean()), 2.0 * d / d.size


def adam_step(p, g, m, v, step, lr, b1, b2, eps):
    """Adam (Kingma & Ba 2015) with bias correction; `step` is the 1-based step after this update.
    Returns the new (p, m, v)."""
    p = np.asarray(p, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    m = b1 * np.asarray(m, dtype=np.float64) + (1.0 - b1) * g
    v = b2 * np.asarray(v, dtype=np.float64) + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** step)
    vh = v / (1.0 - b2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
