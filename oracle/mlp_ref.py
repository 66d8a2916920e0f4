"""FP64 reference of the learned CTU-time perceptron -- TEST INFRASTRUCTURE ONLY.

Forward and hand-derived backward of y = W3 gelu(W2 gelu(W1 x' + b1) + b2) + b3 with
x' = (x - mean) * inv_std and the exact GELU 0.5 x (1 + erf(x / sqrt(2))), in float64.
Inputs per CTU follow the same definition as the GPU kernel (texture, variance, mean,
four neighbour textures with the own value at the frame edge, previous time, mean of the
four neighbours' previous times, area fraction).
"""
from __future__ import annotations

import numpy as np
from scipy.special import erf

SQRT2 = np.sqrt(2.0)


def gelu(x):
    return 0.5 * x * (1.0 + erf(x / SQRT2))


def gelu_grad(x):
    return 0.5 * (1.0 + erf(x / SQRT2)) + x * np.exp(-0.5 * x * x) / np.sqrt(2.0 * np.pi)


def inputs(w, h, cs, tex, var, mean, prev):
    W, H = (w + cs - 1) // cs, (h + cs - 1) // cs
    tex = np.asarray(tex, np.float64).reshape(H, W)
    var = np.asarray(var, np.float64).reshape(H, W)
    mean = np.asarray(mean, np.float64).reshape(H, W)
    prev = np.asarray(prev, np.float64).reshape(H, W)
    x = np.zeros((H, W, 10))
    for cy in range(H):
        for cx in range(W):
            l = cx - 1 if cx > 0 else cx
            r = cx + 1 if cx + 1 < W else cx
            u = cy - 1 if cy > 0 else cy
            d = cy + 1 if cy + 1 < H else cy
            n = min(cs, w - cx * cs) * min(cs, h - cy * cs)
            x[cy, cx] = [tex[cy, cx], var[cy, cx], mean[cy, cx], tex[cy, l], tex[cy, r],
                         tex[u, cx], tex[d, cx], prev[cy, cx],
                         (prev[cy, l] + prev[cy, r] + prev[u, cx] + prev[d, cx]) / 4.0,
                         n / (cs * cs)]
    return x.reshape(H * W, 10)


def forward(p: dict, x, mean, inv_std):
    xn = (np.asarray(x, np.float64) - mean) * inv_std
    z1 = xn @ p["w1"].T + p["b1"]
    h1 = gelu(z1)
    z2 = h1 @ p["w2"].T + p["b2"]
    h2 = gelu(z2)
    y = h2 @ p["w3"].T + p["b3"]
    return y[:, 0], (xn, z1, h1, z2, h2)


def backward(p: dict, cache, dy):
    """Gradients of sum(dy * y) with respect to every parameter."""
    xn, z1, h1, z2, h2 = cache
    dy = np.asarray(dy, np.float64)[:, None]
    g = {"w3": dy.T @ h2, "b3": dy.sum(axis=0)}
    dz2 = (dy @ p["w3"]) * gelu_grad(z2)
    g["w2"] = dz2.T @ h1
    g["b2"] = dz2.sum(axis=0)
    dz1 = (dz2 @ p["w2"]) * gelu_grad(z1)
    g["w1"] = dz1.T @ xn
    g["b1"] = dz1.sum(axis=0)
    return g
