"""Pins for the network oracle (plain PyTorch CPU): autograd gradients against
finite differences, shapes and parameter count, Adam against its first-step
closed form."""
import math

import numpy as np
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
    assert n == 873570  # about 0.9 M weights (4 levels, 16..128 channels, 5 inputs)
    x = torch.randn(5, 16, 16, 16, dtype=torch.float64)
    pred, act = S.forward(p, x)
    assert pred.shape == (2, 16, 16, 16)
    assert act["b"].shape == (128, 2, 2, 2) and act["d3"].shape == (64, 4, 4, 4) and act["d1"].shape == (16, 16, 16, 16)


def test_gradients_match_finite_differences():
    torch.manual_seed(0)
    p = _params(1)
    x = torch.randn(5, 8, 8, 8, dtype=torch.float64)
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


def test_features_homogeneous_closed_form():
    """In a homogeneous medium the carried beam is amp(x, y) exp(i k0 h n |z - z0|)
    (attenuated by exp(-k0 h kappa |z - z0|)): the trapezoid sums are exact."""
    D, H, W, plane, w0, k0h = 12, 6, 8, 4, 3.0, 0.7
    n = 1.41 + 0.03j
    f = S.features(np.full((D, H, W), n), plane, w0, k0h)
    yy = np.arange(H)[:, None] - H / 2
    xx = np.arange(W)[None, :] - W / 2
    amp = np.exp(-(xx ** 2 + yy ** 2) / w0 ** 2)
    for z in range(D):
        u = amp * np.exp(1j * k0h * n * abs(z - plane))
        assert np.allclose(f[3, z], u.real, atol=1e-13) and np.allclose(f[4, z], u.imag, atol=1e-13)
    assert np.allclose(f[0], (1.41 - 1.33) / 0.17) and np.allclose(f[1], 0.03 / 0.2)
    assert f[2, plane].min() == 1.0 and f[2].sum() == H * W
    assert abs(f[3, plane, H // 2, W // 2] - 1.0) < 1e-15   # beam centre on the source plane


def test_features_layered_medium_is_optical_path():
    """Two layers along z: the phase at distance d past the interface is the sum of
    the two layers' optical paths (trapezoid puts half a step on each side)."""
    D, H, W, plane, k0h = 10, 2, 2, 0, 0.5
    nid = np.full((D, H, W), 1.0 + 0j)
    nid[5:] = 1.5
    f = S.features(nid, plane, 1e9, k0h)
    u = f[3] + 1j * f[4]
    expect = k0h * (4 * 1.0 + 0.5 * (1.0 + 1.5) + 1.5 * (np.arange(D) - 5))   # z >= 5
    for z in range(5, D):
        assert abs(np.angle(u[z, 0, 0] * np.exp(-1j * expect[z]))) < 1e-12
    for z in range(5):
        assert abs(np.angle(u[z, 0, 0] * np.exp(-1j * k0h * z))) < 1e-12
