"""Pins for the network oracle (plain PyTorch CPU): autograd gradients against
finite differences, shapes and parameter count, Adam against its first-step
closed form."""
import math

import pytest
import torch

from oracle import surrogate as S


def _params(seed=0, dtype=torch.float64):
    g = torch.Generator().manual_seed(seed)
    p = {}
    for name, ci, co in S.ENC + [S.BOTTLENECK] + S.DEC:
        p[name] = (torch.randn(co, ci, 3, 3, 3, generator=g, dtype=dtype) * math.sqrt(2 / (27 * ci)),
                   torch.randn(co, generator=g, dtype=dtype) * 0.1)
    name, ci, co = S.HEAD
    p[name] = (torch.randn(co, ci, 1, 1, 1, generator=g, dtype=dtype) * 0.3, torch.zeros(co, dtype=dtype))
    return p


def test_parameter_count_and_shapes():
    p = _params()
    n = sum(w.numel() + b.numel() for w, b in p.values())
    assert n == 872706  # about 0.9 M weights (4 levels, 16..128 channels)
    x = torch.randn(3, 16, 16, 16, dtype=torch.float64)
    pred, act = S.forward(p, x)
    assert pred.shape == (2, 16, 16, 16)
    assert act["b"].shape == (128, 2, 2, 2) and act["d3"].shape == (64, 4, 4, 4) and act["d1"].shape == (16, 16, 16, 16)


def test_gradients_match_finite_differences():
    torch.manual_seed(0)
    p = _params(1)
    x = torch.randn(3, 8, 8, 8, dtype=torch.float64)
    t = torch.randn(8, 8, 8, dtype=torch.complex128)
    L0, grads, _ = S.gradients(p, x, t, 0.7)
    g = torch.Generator().manual_seed(5)
    for name in ("e1a", "b", "d3", "head"):
        w, b = p[name]
        for _ in range(3):
            idx = tuple(int(torch.randint(0, s, (1,), generator=g)) for s in w.shape)
            h = 1e-6
            wp = w.clone(); wp[idx] += h
            wm = w.clone(); wm[idx] -= h
            pp = dict(p); pp[name] = (wp, b)
            pm = dict(p); pm[name] = (wm, b)
            fd = (S.loss(S.forward(pp, x)[0], t, 0.7) - S.loss(S.forward(pm, x)[0], t, 0.7)) / (2 * h)
            assert abs(float(fd) - float(grads[name][0][idx])) < 1e-6 * max(1.0, abs(float(fd)))


def test_adam_first_step_is_sign_step():
    """With zero moments, the first bias-corrected Adam step is lr * g / (|g| + eps)."""
    w = torch.randn(50, dtype=torch.float64)
    g = torch.randn(50, dtype=torch.float64)
    w1, m, v = S.adam(w, g, torch.zeros(50, dtype=torch.float64), torch.zeros(50, dtype=torch.float64), 1, lr=1e-2)
    assert torch.allclose(w - w1, 1e-2 * g / (g.abs() + 1e-8), atol=1e-15)
