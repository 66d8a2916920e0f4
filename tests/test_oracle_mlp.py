"""Pins for the FP64 reference of the learned CTU-time perceptron (CPU only): its hand-written
backward against central finite differences and against torch's CPU autograd of the same
network (a library routine with the exact-erf GELU)."""
import numpy as np
import pytest
import torch

from oracle import mlp_ref


def _params(seed):
    rng = np.random.default_rng(seed)
    return {"w1": rng.normal(0, 0.4, (64, 10)), "b1": rng.normal(0, 0.1, 64),
            "w2": rng.normal(0, 0.2, (64, 64)), "b2": rng.normal(0, 0.1, 64),
            "w3": rng.normal(0, 0.2, (1, 64)), "b3": rng.normal(0, 0.1, 1)}


@pytest.mark.parametrize("seed", [0, 1])
def test_backward_matches_finite_differences(seed):
    p = _params(seed)
    rng = np.random.default_rng(seed + 10)
    x = rng.normal(0, 1, (7, 10))
    mean, inv_std = rng.normal(0, 0.1, 10), rng.uniform(0.5, 2.0, 10)
    dy = rng.normal(0, 1, 7)
    y, cache = mlp_ref.forward(p, x, mean, inv_std)
    g = mlp_ref.backward(p, cache, dy)
    h = 1e-6
    for name in p:
        flat = p[name].reshape(-1)
        for idx in rng.choice(flat.size, size=min(12, flat.size), replace=False):
            old = flat[idx]
            flat[idx] = old + h
            yp, _ = mlp_ref.forward(p, x, mean, inv_std)
            flat[idx] = old - h
            ym, _ = mlp_ref.forward(p, x, mean, inv_std)
            flat[idx] = old
            fd = float(np.dot(dy, yp - ym) / (2 * h))
            assert abs(g[name].reshape(-1)[idx] - fd) <= 1e-6 * max(1.0, abs(fd)), (name, idx)


def test_backward_matches_torch_autograd():
    p = _params(3)
    rng = np.random.default_rng(4)
    x = rng.normal(0, 1, (33, 10))
    mean, inv_std = rng.normal(0, 0.1, 10), rng.uniform(0.5, 2.0, 10)
    dy = rng.normal(0, 1, 33)
    y, cache = mlp_ref.forward(p, x, mean, inv_std)
    g = mlp_ref.backward(p, cache, dy)
    tp = {k: torch.tensor(v, dtype=torch.float64, requires_grad=True) for k, v in p.items()}
    xn = (torch.tensor(x) - torch.tensor(mean)) * torch.tensor(inv_std)
    h1 = torch.nn.functional.gelu(xn @ tp["w1"].T + tp["b1"], approximate="none")
    h2 = torch.nn.functional.gelu(h1 @ tp["w2"].T + tp["b2"], approximate="none")
    ty = (h2 @ tp["w3"].T + tp["b3"])[:, 0]
    assert np.allclose(ty.detach().numpy(), y, rtol=1e-12, atol=1e-12)
    (ty * torch.tensor(dy)).sum().backward()
    for k in p:
        assert np.allclose(tp[k].grad.numpy(), g[k], rtol=1e-10, atol=1e-12), k


def test_inputs_definition():
    # 3 x 2 CTU grid of a 300 x 200 frame (CTU 128): partial right and bottom CTUs
    tex = np.arange(6) + 10
    var = np.arange(6) + 20
    mean = np.arange(6) + 30
    prev = np.array([100, 200, 300, 400, 500, 600])
    x = mlp_ref.inputs(300, 200, 128, tex, var, mean, prev)
    # CTU 0 (top-left): left/up neighbours are itself
    assert list(x[0][:7]) == [10, 20, 30, 10, 11, 10, 13]
    assert x[0][7] == 100 and x[0][8] == (100 + 200 + 100 + 400) / 4
    assert x[0][9] == 1.0
    # CTU 5 (bottom-right, 44 x 72 px)
    assert list(x[5][3:7]) == [14, 15, 12, 15]
    assert x[5][9] == 44 * 72 / (128 * 128)
