"""Reference of the learned-initial-guess network, in plain PyTorch CPU ops.

TEST INFRASTRUCTURE (oracle) -- see ``oracle/__init__.py``.  Written from the
architecture description (not from the HIP code): 4 levels with 16/32/64/128
channels; level l has two 3x3x3 convolutions (zero padding 1) + ReLU on the
encoder side, levels are joined by 2x2x2 average pooling, the bottleneck is
one 64->128 convolution; the decoder upsamples by nearest neighbour,
concatenates the encoder output of that level (skip first) and applies one
3x3x3 convolution + ReLU (192->64, 96->32, 48->16); a 1x1x1 convolution
gives (Re, Im).  Tensors here are channels-first [C, D, H, W] in float64.
The loss is the relative squared L2 error ||s p - x||^2 / ||x||^2.

The 5 input channels (``features``) are functions of the complex index map
n + i kappa and of the fixed source geometry: the scaled index, the scaled
absorption, the source-plane indicator, and the Gaussian beam of the source
carried along the axis of propagation with the phase and attenuation of the
medium it crosses (the optical path k0 h sum (n + i kappa), trapezoidal
between grid planes, from the source plane in both directions).
"""
from __future__ import annotations


import numpy as np

import torch
import torch.nn.functional as F

ENC = [("e1a", 5, 16), ("e1b", 16, 16), ("e2a", 16, 32), ("e2b", 32, 32), ("e3a", 32, 64), ("e3b", 64, 64)]
BOTTLENECK = ("b", 64, 128)
DEC = [("d3", 64 + 128, 64), ("d2", 32 + 64, 32), ("d1", 16 + 32, 16)]
HEAD = ("head", 16, 2)


def features(nidx, plane, w0, k0h, n_bg=1.33, n_span=0.17, kappa_max=0.2):
    """Input channels [5, D, H, W] (float64 numpy) from the complex index nidx [D, H, W]."""
    D, H, W = nidx.shape
    f = np.zeros((5, D, H, W))
    f[0] = (nidx.real - n_bg) / n_span
    f[1] = nidx.imag / kappa_max
    f[2, plane] = 1.0
    yy = np.arange(H)[:, None] - H / 2
    xx = np.arange(W)[None, :] - W / 2
    amp = np.exp(-(xx ** 2 + yy ** 2) / w0 ** 2)
    for z in range(D):
        lo, hi = min(z, plane), max(z, plane)
        path = np.zeros((H, W), dtype=complex)
        for q in range(lo, hi):          # trapezoid between planes q and q + 1
            path += 0.5 * (nidx[q] + nidx[q + 1])
        u = amp * np.exp(1j * k0h * path)
        f[3, z] = u.real
        f[4, z] = u.imag
    return f


def conv(x, w, b, relu=True):
    """3x3x3 (or 1x1x1) convolution, zero padding, optional ReLU; x [C,D,H,W], w [Co,Ci,k,k,k]."""
    y = F.conv3d(x[None], w, b, padding=w.shape[-1] // 2)[0]
    return F.relu(y) if relu else y


def forward(params, feats):
    """params: name -> (w [Co,Ci,k,k,k], b [Co]); feats [3, D, H, W]; returns (pred [2,D,H,W], activations)."""
    act = {}
    h = feats
    skips = []
    for lvl in range(3):
        (na, _, _), (nb, _, _) = ENC[2 * lvl], ENC[2 * lvl + 1]
        h = conv(h, *params[na])
        act[na] = h
        h = conv(h, *params[nb])
        act[nb] = h
        skips.append(h)
        h = F.avg_pool3d(h[None], 2)[0]
    h = conv(h, *params["b"])
    act["b"] = h
    for (nd, _, _), skip in zip(DEC, reversed(skips)):
        up = F.interpolate(h[None], scale_factor=2, mode="nearest")[0]
        h = conv(torch.cat([skip, up], 0), *params[nd])
        act[nd] = h
    pred = conv(h, *params["head"], relu=False)
    return pred, act


def loss(pred, target, scale):
    """||scale * (pred[0] + i pred[1]) - target||^2 / ||target||^2 (target complex [D,H,W])."""
    pr = scale * pred[0] - target.real
    pi = scale * pred[1] - target.imag
    return (pr * pr + pi * pi).sum() / (target.real ** 2 + target.imag ** 2).sum()


def gradients(params, feats, target, scale):
    """Loss and d loss / d (w, b) for every layer, by autograd in float64."""
    p = {k: (w.detach().clone().requires_grad_(True), b.detach().clone().requires_grad_(True))
         for k, (w, b) in params.items()}
    pred, _ = forward(p, feats)
    L = loss(pred, target, scale)
    L.backward()
    return float(L), {k: (w.grad, b.grad) for k, (w, b) in p.items()}, pred.detach()


def adam(w, g, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (Kingma & Ba 2015) with bias correction; returns (w, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return w - lr * mh / (torch.sqrt(vh) + eps), m, v
