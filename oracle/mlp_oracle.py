"""FP64 reference of the warm-start network -- TEST INFRASTRUCTURE ONLY.

A fully connected network h_l = act_l(h_{l-1} W_l + b_l), act = ReLU on the
hidden layers and identity on the output, trained with the mean squared error
and Adam.  It predicts the kernel coefficients of the subtraction from the two
PSF stamps and the frame position (the learned warm start of the target
description; the pipeline paper names the spatially varying PSF as the thing
the kernel must follow, "Statement of need").

Parameter packing (shared with the GPU kernels' interface, not their code):
[W_1 (d0 x d1, row-major), b_1 (d1), W_2, b_2, ...] as one flat array.
"""
from __future__ import annotations

import numpy as np

__all__ = ["param_count", "unpack", "init_params", "forward", "backward", "mse", "adam_step"]


def param_count(dims):
    return int(sum(dims[i] * dims[i + 1] + dims[i + 1] for i in range(len(dims) - 1)))


def unpack(params, dims):
    """[(W_l, b_l)] views into the flat parameter vector."""
    out, off = [], 0
    for i in range(len(dims) - 1):
        w = params[off:off + dims[i] * dims[i + 1]].reshape(dims[i], dims[i + 1])
        off += dims[i] * dims[i + 1]
        b = params[off:off + dims[i + 1]]
        off += dims[i + 1]
        out.append((w, b))
    return out


def init_params(dims, seed):
    """He-uniform weights, zero biases (FP64)."""
    rng = np.random.default_rng(seed)
    parts = []
    for i in range(len(dims) - 1):
        lim = np.sqrt(6.0 / dims[i])
        parts.append(rng.uniform(-lim, lim, dims[i] * dims[i + 1]))
        parts.append(np.zeros(dims[i + 1]))
    return np.concatenate(parts)


def forward(params, dims, x):
    """Returns (y, activations) with activations[l] = h_l (h_0 = x)."""
    hs = [np.asarray(x, dtype=np.float64)]
    layers = unpack(np.asarray(params, dtype=np.float64), dims)
    for i, (w, b) in enumerate(layers):
        z = hs[-1] @ w + b
        if i < len(layers) - 1:
            z = np.maximum(z, 0.0)
        hs.append(z)
    return hs[-1], hs


def backward(params, dims, hs, dy):
    """Gradient of sum(dy * y) with respect to the flat parameters, and to the input."""
    layers = unpack(np.asarray(params, dtype=np.float64), dims)
    grads = []
    g = np.asarray(dy, dtype=np.float64)
    for i in range(len(layers) - 1, -1, -1):
        w, _ = layers[i]
        if i < len(layers) - 1:
            g = g * (hs[i + 1] > 0.0)          # ReLU of layer i
        grads.append((hs[i].T @ g, g.sum(axis=0)))
        g = g @ w.T
    grads.reverse()
    flat = np.concatenate([np.concatenate([gw.ravel(), gb]) for gw, gb in grads])
    return flat, g


def mse(y, t):
    """Loss mean((y - t)^2) and its gradient with respect to y."""
    d = np.asarray(y, dtype=np.float64) - np.asarray(t, dtype=np.float64)
    return float(np.mean(d * d)), 2.0 * d / d.size


def adam_step(p, g, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (bias-corrected), returning new (p, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** step)
    vh = v / (1.0 - b2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
