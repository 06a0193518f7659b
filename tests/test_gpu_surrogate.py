"""GPU parity of the learned-initial-guess network kernels (through the C ABI)
against the plain-PyTorch CPU reference in float64, on bf16-representable
inputs.  Tolerances: single kernels with fp32 accumulation 1e-5 (forward,
input gradient) / 1e-4 (weight gradient, long sums); kernels whose output is
rounded to bf16 2e-2 (relative 2^-8 per element); the whole network
(bf16 activations between layers) 5e-2 on the prediction and 0.99 cosine on
each layer's weight gradient."""
import ctypes as ct
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import surrogate as S

pytestmark = pytest.mark.gpu


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _lib():
    from paper_2207_14222_amd import _lib
    return _lib


def _p(t):
    return None if t is None else ct.c_void_p(t.data_ptr())


def _st():
    return ct.c_void_p(torch.cuda.current_stream().cuda_stream)


def bf(x):
    return x.to(torch.bfloat16)


def to_cf(a, shape):
    """GPU channels-last [V][C] -> channels-first [C, D, H, W] float64 on the CPU."""
    D, H, W = shape
    return a.float().cpu().double().reshape(D, H, W, -1).permute(3, 0, 1, 2).contiguous()


def w_to_torch(w, taps):
    """[Co][taps][Ci] -> [Co][Ci][k][k][k]."""
    co, _, ci = w.shape
    k = 3 if taps == 27 else 1
    return w.float().cpu().double().reshape(co, k, k, k, ci).permute(0, 4, 1, 2, 3).contiguous()


def rel(a, b):
    return float((a - b).norm() / b.norm())


SHAPES = [(16, 16, 27), (16, 32, 27), (64, 128, 27), (192, 64, 27), (48, 16, 27), (16, 16, 1)]


@pytest.mark.parametrize("cin,cout,taps", SHAPES)
def test_conv_forward_input_grad_and_weight_grad(cin, cout, taps):
    _need_gpu()
    L = _lib()
    grid = (8, 16, 16)
    D, H, W = grid
    V = D * H * W
    print(f"[gpu-case] conv {cin}->{cout} taps {taps}", flush=True)
    g = torch.Generator().manual_seed(cin * 1000 + cout)
    x = bf(torch.randn(V, cin, generator=g)).cuda()
    w = bf(torch.randn(cout, taps, cin, generator=g) / math.sqrt(cin * taps)).cuda()
    b = torch.randn(cout, generator=g).cuda()
    out = torch.empty(V, cout, dtype=torch.float32, device="cuda")
    assert L.lib().usp_nn_conv3d(_p(x), _p(w), _p(b), _p(out), 1, cout, D, H, W, cin, cout, taps, 1, 0, _st()) == 0
    xt = to_cf(x, grid).requires_grad_(True)
    wt = w_to_torch(w, taps).requires_grad_(True)
    ref = S.conv(xt, wt, b.cpu().double(), relu=False)
    assert rel(to_cf(out, grid), ref.detach()) < 1e-5
    # input gradient with the transposed weights
    gy = bf(torch.randn(V, cout, generator=g)).cuda()
    wT = torch.empty(cin, taps, cout, dtype=torch.bfloat16, device="cuda")
    assert L.lib().usp_nn_transpose_weights(_p(w), _p(wT), cout, taps, cin, _st()) == 0
    gx = torch.empty(V, cin, dtype=torch.float32, device="cuda")
    assert L.lib().usp_nn_conv3d(_p(gy), _p(wT), None, _p(gx), 1, cin, D, H, W, cout, cin, taps, -1, 0, _st()) == 0
    gyt = to_cf(gy, grid)
    ref_gx, ref_gw = torch.autograd.grad(ref, [xt, wt], gyt)
    assert rel(to_cf(gx, grid), ref_gx) < 1e-5
    # weight and bias gradients
    nb = ct.c_size_t()
    assert L.lib().usp_nn_wgrad_workspace(D, H, W, cin, cout, taps, ct.byref(nb)) == 0
    ws = torch.empty(nb.value, dtype=torch.uint8, device="cuda")
    dw = torch.empty(cout, taps, cin, dtype=torch.float32, device="cuda")
    db = torch.empty(cout, dtype=torch.float32, device="cuda")
    assert L.lib().usp_nn_conv3d_wgrad(_p(x), _p(gy), _p(dw), _p(db), _p(ws), nb.value, D, H, W, cin, cout, taps,
                                       _st()) == 0
    assert rel(w_to_torch(dw, taps), ref_gw) < 1e-4
    assert rel(db.cpu().double(), gyt.sum(dim=(1, 2, 3))) < 1e-4


def test_pool_upsample_and_copies():
    _need_gpu()
    L = _lib()
    D, H, W, C = 8, 16, 32, 16
    V = D * H * W
    g = torch.Generator().manual_seed(3)
    x = bf(torch.randn(V, C, generator=g)).cuda()
    p = torch.empty(V // 8, C, dtype=torch.bfloat16, device="cuda")
    assert L.lib().usp_nn_pool2(_p(x), _p(p), D, H, W, C, 0, _st()) == 0
    ref = torch.nn.functional.avg_pool3d(to_cf(x, (D, H, W))[None], 2)[0]
    assert rel(to_cf(p, (D // 2, H // 2, W // 2)), ref) < 1e-2
    gb = torch.empty(V, C, dtype=torch.bfloat16, device="cuda")
    assert L.lib().usp_nn_pool2(_p(p), _p(gb), D, H, W, C, 1, _st()) == 0
    pc = to_cf(p, (D // 2, H // 2, W // 2))
    assert rel(to_cf(gb, (D, H, W)), torch.nn.functional.interpolate(pc[None], scale_factor=2)[0] / 8) < 1e-2
    # upsample into channels 16..32 of a 48-channel tensor, and its gradient
    cat = torch.zeros(V, 48, dtype=torch.bfloat16, device="cuda")
    assert L.lib().usp_nn_upsample2(_p(p), _p(cat), D, H, W, C, 48, 16, 0, _st()) == 0
    up = to_cf(cat, (D, H, W))[16:32]
    assert rel(up, torch.nn.functional.interpolate(pc[None], scale_factor=2)[0]) < 1e-2
    gc = torch.empty(V // 8, C, dtype=torch.bfloat16, device="cuda")
    assert L.lib().usp_nn_upsample2(_p(cat), _p(gc), D, H, W, C, 48, 16, 1, _st()) == 0
    assert rel(to_cf(gc, (D // 2, H // 2, W // 2)), 8 * pc) < 1e-2


def _oracle_params(net):
    P = {}
    for name, ly in net.layers.items():
        w = w_to_torch(ly.wb, ly.taps)
        ci = 3 if name == "e1a" else ly.cin
        co = 2 if name == "head" else ly.cout
        P[name] = (w[:co, :ci].contiguous(), ly.b.cpu().double()[:co].contiguous())
    return P


def test_network_forward_backward_against_reference():
    _need_gpu()
    from paper_2207_14222_amd import media, surrogate
    print("[gpu-case] unet 32^3", flush=True)
    shape = (32, 32, 32)
    net = surrogate.UNet3D(shape, seed=1, scale=0.5)
    prob = media.helmholtz_spheres(shape=shape, count=30, width=4, w0=4.0, plane=4, seed=9)
    nidx = torch.from_numpy(prob.index.astype(np.complex64)).cuda()
    net.features(nidx, plane=4)
    pred = net.forward().clone()
    feats = to_cf(net.a.x0, shape)[:3]
    P = _oracle_params(net)
    target = torch.from_numpy((prob.source * 0.3 + 0.1j * prob.index.real).astype(np.complex64))
    L_ref, grads, pred_ref = S.gradients(P, feats, target.to(torch.complex128), 0.5)
    pg = pred.cpu().double().reshape(*shape, 2).permute(3, 0, 1, 2)
    assert rel(pg, pred_ref) < 5e-2
    loss = net.loss(target.cuda(), grad=True)
    assert abs(loss - L_ref) < 5e-2 * L_ref
    net.backward()
    torch.cuda.synchronize()
    for name, ly in net.layers.items():
        ci = 3 if name == "e1a" else ly.cin
        co = 2 if name == "head" else ly.cout
        gw = w_to_torch(ly.gw, ly.taps)[:co, :ci].flatten()
        gr = grads[name][0].flatten()
        cos = float(gw @ gr / (gw.norm() * gr.norm()))
        assert cos > 0.99, (name, cos)


def test_training_reduces_loss_on_one_sample():
    _need_gpu()
    from paper_2207_14222_amd import media, surrogate
    print("[gpu-case] unet training 32^3", flush=True)
    shape = (32, 32, 32)
    net = surrogate.UNet3D(shape, seed=2, scale=0.5)
    prob = media.helmholtz_spheres(shape=shape, count=30, width=4, w0=4.0, plane=4, seed=10)
    net.features(torch.from_numpy(prob.index.astype(np.complex64)).cuda(), plane=4)
    target = torch.from_numpy((0.2 * prob.index.real - 0.25 + 0.05j).astype(np.complex64)).cuda()
    losses = []
    for _ in range(60):
        net.forward()
        losses.append(net.loss(target, grad=True))
        net.backward()
        net.adam_step(lr=3e-3)
    assert all(math.isfinite(v) for v in losses)
    assert losses[-1] < 0.5 * losses[0]
