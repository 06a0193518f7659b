"""Learned initial guess: a 3-D convolutional network mapping the refractive
index map to the field, trained on solves of the fixed-point method, used as
x0 for the unchanged iteration (which judges its error and falls back to
x0 = 0 when ||y - A x0|| >= ||y||).

Architecture (4 levels, channels 16/32/64/128, 3x3x3 convolutions, ReLU,
about 0.88 M weights): two convolutions per encoder level with 2x2x2 average
pooling between levels, one 64->128 convolution at the bottleneck, a decoder
of nearest upsampling + concatenation with the skip + one convolution per
level (192->64, 96->32, 48->16), and a 1x1x1 head to (Re, Im).  Every
arithmetic step runs in the library's kernels (usp_nn_*: bf16 matrix-core
convolutions with fp32 accumulation, fp32 Adam master weights); this module
only orders the calls and owns the device buffers (torch tensors).
Activations are bf16 in 16-channel planes ([C/16][V][16], see usp.h), so a
torch tensor of shape (V, C) here is only a buffer of V*C elements.
"""
from __future__ import annotations

import ctypes as ct
import math
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib as L

# (name, cin, cout, taps) -- cin of the first layer is the 16-channel padded input
LAYERS = [
    ("e1a", 16, 16, 27), ("e1b", 16, 16, 27),
    ("e2a", 16, 32, 27), ("e2b", 32, 32, 27),
    ("e3a", 32, 64, 27), ("e3b", 64, 64, 27),
    ("b", 64, 128, 27),
    ("d3", 192, 64, 27), ("d2", 96, 32, 27), ("d1", 48, 16, 27),
    ("head", 16, 16, 1),
]
IN_CH = 5          # real input channels (the rest of the 16 are zero)
OUT_CH = 2         # Re, Im


def _p(t):
    return None if t is None else ct.c_void_p(t.data_ptr())


def _s(dev):
    return ct.c_void_p(torch.cuda.current_stream(dev).cuda_stream)


def effective_parameter_count():
    n = 0
    for name, cin, cout, taps in LAYERS:
        ci = IN_CH if name == "e1a" else cin
        co = OUT_CH if name == "head" else cout
        n += co * taps * ci + co
    return n


class Layer:
    def __init__(self, name, cin, cout, taps, dev, gen):
        self.name, self.cin, self.cout, self.taps = name, cin, cout, taps
        ci = IN_CH if name == "e1a" else cin
        co = OUT_CH if name == "head" else cout
        std = math.sqrt(2.0 / (ci * taps)) if name != "head" else math.sqrt(1.0 / (ci * taps))
        w = torch.zeros(cout, taps, cin)
        w[:co, :, :ci] = torch.randn(co, taps, ci, generator=gen) * std
        self.w = w.to(dev).contiguous()                     # fp32 master
        self.b = torch.zeros(cout, device=dev)
        self.wb = torch.empty(cout, taps, cin, dtype=torch.bfloat16, device=dev)
        npk = (28 if taps == 27 else 1) * cout * cin
        self.wp = torch.empty(npk, dtype=torch.bfloat16, device=dev)   # forward fragments
        self.wt = torch.empty(npk, dtype=torch.bfloat16, device=dev)   # input-gradient fragments
        self.gw = torch.zeros_like(self.w)
        self.gb = torch.zeros_like(self.b)
        self.mw, self.vw = torch.zeros_like(self.w), torch.zeros_like(self.w)
        self.mb, self.vb = torch.zeros_like(self.b), torch.zeros_like(self.b)
        self.sync_bf16()

    def sync_bf16(self):
        lib = L.lib()
        dev = self.w.device
        L.check(lib.usp_nn_to_bf16(_p(self.w), _p(self.wb), self.w.numel(), _s(dev)))
        self.pack()

    def pack(self):
        lib, s = L.lib(), _s(self.w.device)
        L.check(lib.usp_nn_pack_weights(_p(self.wb), _p(self.wp), self.cout, self.taps, self.cin, 0, s))
        L.check(lib.usp_nn_pack_weights(_p(self.wb), _p(self.wt), self.cout, self.taps, self.cin, 1, s))


@dataclass
class Acts:
    x0: torch.Tensor = None
    e1a: torch.Tensor = None
    e1: torch.Tensor = None
    p1: torch.Tensor = None
    e2a: torch.Tensor = None
    e2: torch.Tensor = None
    p2: torch.Tensor = None
    e3a: torch.Tensor = None
    e3: torch.Tensor = None
    p3: torch.Tensor = None
    b: torch.Tensor = None
    c3: torch.Tensor = None
    d3: torch.Tensor = None
    c2: torch.Tensor = None
    d2: torch.Tensor = None
    c1: torch.Tensor = None
    d1: torch.Tensor = None
    pred: torch.Tensor = None


class UNet3D:
    """The network, its parameters and its buffers for one grid shape (D, H, W)."""

    def __init__(self, shape, device="cuda", seed=0, scale=1.0):
        self.shape = tuple(shape)
        D, H, W = self.shape
        if D % 8 or H % 8 or W % 8 or ((D // 8) * (H // 8) * (W // 8)) % 16:
            raise ValueError("sides must be multiples of 8 and the coarsest level a multiple of 16 voxels")
        self.dev = torch.device(device)
        gen = torch.Generator().manual_seed(seed)
        self.layers = {n: Layer(n, ci, co, tp, self.dev, gen) for n, ci, co, tp in LAYERS}
        self.scale = float(scale)   # the network predicts x / scale
        self.step = 0
        self.levels = [(D, H, W), (D // 2, H // 2, W // 2), (D // 4, H // 4, W // 4), (D // 8, H // 8, W // 8)]
        bf = dict(dtype=torch.bfloat16, device=self.dev)
        V = [d * h * w for d, h, w in self.levels]
        self.V = V
        a = Acts()
        a.x0 = torch.empty(V[0], 16, **bf)
        a.c3, a.d3 = torch.empty(V[2], 192, **bf), torch.empty(V[2], 64, **bf)
        a.c2, a.d2 = torch.empty(V[1], 96, **bf), torch.empty(V[1], 32, **bf)
        a.c1, a.d1 = torch.empty(V[0], 48, **bf), torch.empty(V[0], 16, **bf)
        # the skip activations are the leading 16-channel planes of the concat
        # buffers (planes [C/16][V][16]), so the concatenation needs no copy
        lead = lambda buf, v, c: buf.view(-1)[:v * c].view(v, c)
        a.e1a, a.e1 = torch.empty(V[0], 16, **bf), lead(a.c1, V[0], 16)
        a.p1 = torch.empty(V[1], 16, **bf)
        a.e2a, a.e2 = torch.empty(V[1], 32, **bf), lead(a.c2, V[1], 32)
        a.p2 = torch.empty(V[2], 32, **bf)
        a.e3a, a.e3 = torch.empty(V[2], 64, **bf), lead(a.c3, V[2], 64)
        a.p3 = torch.empty(V[3], 64, **bf)
        a.b = torch.empty(V[3], 128, **bf)
        a.pred = torch.empty(V[0], 2, dtype=torch.float32, device=self.dev)
        self.a = a
        # gradient buffers
        def g(v, c):
            return torch.empty(V[v], c, **bf)
        self.gb = {"c1": g(0, 48), "d1": g(0, 16), "t1": g(0, 16),
                   "c2": g(1, 96), "d2": g(1, 32), "t2": g(1, 32), "p1": g(1, 16),
                   "c3": g(2, 192), "d3": g(2, 64), "t3": g(2, 64), "p2": g(2, 32),
                   "b": g(3, 128), "p3": g(3, 64)}
        # likewise the skip part of each concat gradient is the skip gradient
        self.gb["e1"] = lead(self.gb["c1"], V[0], 16)
        self.gb["e2"] = lead(self.gb["c2"], V[1], 32)
        self.gb["e3"] = lead(self.gb["c3"], V[2], 64)
        self.gout = g(0, 16)
        wsz = 0
        for n, ci, co, tp in LAYERS:
            lev = self._level(n)
            d, h, w = self.levels[lev]
            b = ct.c_size_t()
            L.check(L.lib().usp_nn_wgrad_workspace(d, h, w, ci, co, tp, ct.byref(b)))
            wsz = max(wsz, b.value)
        self.wgws = torch.empty(wsz, dtype=torch.uint8, device=self.dev)
        self.lossws = torch.empty(32768, dtype=torch.uint8, device=self.dev)

    @staticmethod
    def _level(name):
        return {"e1a": 0, "e1b": 0, "d1": 0, "head": 0, "e2a": 1, "e2b": 1, "d2": 1, "e3a": 2, "e3b": 2, "d3": 2,
                "b": 3}[name]

    def parameters(self):
        return [(ly.w, ly.b) for ly in self.layers.values()]

    # -- primitive calls ---------------------------------------------------------
    def _conv(self, name, x, out, relu=True, out_f32=False, cstore=None):
        ly = self.layers[name]
        d, h, w = self.levels[self._level(name)]
        L.check(L.lib().usp_nn_conv3d(_p(x), _p(ly.wp), _p(ly.b), _p(out), int(out_f32), cstore or ly.cout, d, h, w,
                                      ly.cin, ly.cout, ly.taps, 1, int(relu), _s(self.dev)))

    def _conv_back(self, name, g, out):
        ly = self.layers[name]
        d, h, w = self.levels[self._level(name)]
        L.check(L.lib().usp_nn_conv3d(_p(g), _p(ly.wt), None, _p(out), 0, ly.cin, d, h, w, ly.cout, ly.cin, ly.taps,
                                      -1, 0, _s(self.dev)))

    def _wgrad(self, name, x, g):
        ly = self.layers[name]
        d, h, w = self.levels[self._level(name)]
        L.check(L.lib().usp_nn_conv3d_wgrad(_p(x), _p(g), _p(ly.gw), _p(ly.gb), _p(self.wgws), self.wgws.numel(), d, h,
                                            w, ly.cin, ly.cout, ly.taps, _s(self.dev)))

    def _pool(self, lev, x, out, backward=False):
        d, h, w = self.levels[lev]
        L.check(L.lib().usp_nn_pool2(_p(x), _p(out), d, h, w, x.shape[1] if not backward else out.shape[1],
                                     int(backward), _s(self.dev)))

    def _up(self, lev, x, out, C, Ctot, c0, backward=False):
        d, h, w = self.levels[lev]
        L.check(L.lib().usp_nn_upsample2(_p(x), _p(out), d, h, w, C, Ctot, c0, int(backward), _s(self.dev)))

    def _copy(self, src, s0, dst, d0, C):
        L.check(L.lib().usp_nn_channel_copy(_p(src), src.shape[1], s0, _p(dst), dst.shape[1], d0, C, src.shape[0],
                                            _s(self.dev)))

    def _relu_back(self, y, g, out, acc=False):
        L.check(L.lib().usp_nn_relu_backward(_p(y), _p(g), _p(out), y.numel(), int(acc), _s(self.dev)))

    # -- network ------------------------------------------------------------------
    def features(self, nidx64, plane=20, w0=16.0, k0h=2 * math.pi * 0.25, n_bg=1.33, n_span=0.17, kappa_max=0.2):
        """Input channels from the complex refractive index (complex64 [D,H,W] device tensor) and the
        source geometry (beam on z = plane with waist w0 voxels; k0h = wavenumber x grid step)."""
        D, H, W = self.shape
        L.check(L.lib().usp_nn_features(_p(nidx64), _p(self.a.x0), D, H, W, n_bg, n_span, kappa_max, plane, k0h,
                                        w0, _s(self.dev)))

    def forward(self):
        a = self.a
        self._conv("e1a", a.x0, a.e1a)
        self._conv("e1b", a.e1a, a.e1)
        self._pool(0, a.e1, a.p1)
        self._conv("e2a", a.p1, a.e2a)
        self._conv("e2b", a.e2a, a.e2)
        self._pool(1, a.e2, a.p2)
        self._conv("e3a", a.p2, a.e3a)
        self._conv("e3b", a.e3a, a.e3)
        self._pool(2, a.e3, a.p3)
        self._conv("b", a.p3, a.b)
        self._up(2, a.b, a.c3, 128, 192, 64)
        self._conv("d3", a.c3, a.d3)
        self._up(1, a.d3, a.c2, 64, 96, 32)
        self._conv("d2", a.c2, a.d2)
        self._up(0, a.d2, a.c1, 32, 48, 16)
        self._conv("d1", a.c1, a.d1)
        self._conv("head", a.d1, a.pred, relu=False, out_f32=True, cstore=2)
        return a.pred

    def loss(self, target64, grad=True, sync=True):
        """Relative squared L2 error of scale * pred against the target field (complex64).
        With sync=False nothing waits for the device: the value stays in the loss
        workspace (``loss_device()``) and None is returned."""
        out = np.zeros(1)
        L.check(L.lib().usp_nn_loss(_p(self.a.pred), _p(target64), self.scale, self.V[0],
                                    _p(self.gout) if grad else None, _p(self.lossws),
                                    out.ctypes.data_as(ct.POINTER(ct.c_double)) if sync else None, _s(self.dev)))
        return float(out[0]) if sync else None

    def loss_device(self):
        """The last loss as a 0-dim float64 device tensor (a view of the loss workspace)."""
        return self.lossws[16384:16392].view(torch.float64)[0]

    def _add(self, dst, src):
        L.check(L.lib().usp_nn_add(_p(dst), _p(src), dst.numel(), _s(self.dev)))

    def backward(self):
        """Gradients of every weight and bias from self.gout (set by loss)."""
        a, g = self.a, self.gb
        # head and decoder level 1
        self._wgrad("head", a.d1, self.gout)
        self._conv_back("head", self.gout, g["d1"])
        self._relu_back(a.d1, g["d1"], g["d1"])
        self._wgrad("d1", a.c1, g["d1"])
        self._conv_back("d1", g["d1"], g["c1"])              # gradient of concat(e1, up(d2))
        self._up(0, g["c1"], g["d2"], 32, 48, 16, backward=True)
        # decoder level 2
        self._relu_back(a.d2, g["d2"], g["d2"])
        self._wgrad("d2", a.c2, g["d2"])
        self._conv_back("d2", g["d2"], g["c2"])
        self._up(1, g["c2"], g["d3"], 64, 96, 32, backward=True)
        # decoder level 3
        self._relu_back(a.d3, g["d3"], g["d3"])
        self._wgrad("d3", a.c3, g["d3"])
        self._conv_back("d3", g["d3"], g["c3"])
        self._up(2, g["c3"], g["b"], 128, 192, 64, backward=True)
        # bottleneck
        self._relu_back(a.b, g["b"], g["b"])
        self._wgrad("b", a.p3, g["b"])
        self._conv_back("b", g["b"], g["p3"])
        # encoder level 3: skip gradient + pooled path
        self._pool(2, g["p3"], g["t3"], backward=True)
        self._add(g["e3"], g["t3"])
        self._relu_back(a.e3, g["e3"], g["e3"])
        self._wgrad("e3b", a.e3a, g["e3"])
        self._conv_back("e3b", g["e3"], g["t3"])
        self._relu_back(a.e3a, g["t3"], g["t3"])
        self._wgrad("e3a", a.p2, g["t3"])
        self._conv_back("e3a", g["t3"], g["p2"])
        # encoder level 2
        self._pool(1, g["p2"], g["t2"], backward=True)
        self._add(g["e2"], g["t2"])
        self._relu_back(a.e2, g["e2"], g["e2"])
        self._wgrad("e2b", a.e2a, g["e2"])
        self._conv_back("e2b", g["e2"], g["t2"])
        self._relu_back(a.e2a, g["t2"], g["t2"])
        self._wgrad("e2a", a.p1, g["t2"])
        self._conv_back("e2a", g["t2"], g["p1"])
        # encoder level 1
        self._pool(0, g["p1"], g["t1"], backward=True)
        self._add(g["e1"], g["t1"])
        self._relu_back(a.e1, g["e1"], g["e1"])
        self._wgrad("e1b", a.e1a, g["e1"])
        self._conv_back("e1b", g["e1"], g["t1"])
        self._relu_back(a.e1a, g["t1"], g["t1"])
        self._wgrad("e1a", a.x0, g["t1"])

    def adam_step(self, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.step += 1
        lib = L.lib()
        for ly in self.layers.values():
            L.check(lib.usp_nn_adam(_p(ly.w), _p(ly.gw), _p(ly.mw), _p(ly.vw), _p(ly.wb), ly.w.numel(), lr, b1, b2,
                                    eps, self.step, _s(self.dev)))
            L.check(lib.usp_nn_adam(_p(ly.b), _p(ly.gb), _p(ly.mb), _p(ly.vb), None, ly.b.numel(), lr, b1, b2, eps,
                                    self.step, _s(self.dev)))
            ly.pack()

    def predict_field(self, out128):
        """x0 = scale * (Re + i Im) of the last forward pass, as complex128 [D,H,W]."""
        L.check(L.lib().usp_nn_pred_to_field(_p(self.a.pred), self.scale, _p(out128), self.V[0], _s(self.dev)))
        return out128
