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
"""
from __future__ import annotations

import torch
import torch.nn.functional as F

ENC = [("e1a", 3, 16), ("e1b", 16, 16), ("e2a", 16, 32), ("e2b", 32, 32), ("e3a", 32, 64), ("e3b", 64, 64)]
BOTTLENECK = ("b", 64, 128)
DEC = [("d3", 64 + 128, 64), ("d2", 32 + 64, 32), ("d1", 16 + 32, 16)]
HEAD = ("head", 16, 2)


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
