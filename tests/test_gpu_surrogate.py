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
    """16-channel planes [C/16][V][16] (any buffer shape) -> channels-first [C, D, H, W] float64 on the CPU."""
    D, H, W = shape
    t = a.float().cpu().double().reshape(-1, D, H, W, 16)
    return t.permute(0, 4, 1, 2, 3).reshape(-1, D, H, W).contiguous()


def from_cf(x):
    """channels-first [C, D, H, W] -> 16-channel planes [C/16][V][16] (same dtype)."""
    C = x.shape[0]
    return x.reshape(C // 16, 16, -1).permute(0, 2, 1).contiguous()


def rows_to_cf(a, shape):
    """fp32 rows [V][C] -> channels-first [C, D, H, W] float64 on the CPU."""
    D, H, W = shape
    return a.cpu().double().reshape(D, H, W, -1).permute(3, 0, 1, 2).contiguous()


def w_to_torch(w, taps):
    """[Co][taps][Ci] -> [Co][Ci][k][k][k]."""
    co, _, ci = w.shape
    k = 3 if taps == 27 else 1
    return w.float().cpu().double().reshape(co, k, k, k, ci).permute(0, 4, 1, 2, 3).contiguous()


def rel(a, b):
    return float((a - b).norm() / b.norm())


def pack(L, w, transposed):
    cout, taps, cin = w.shape
    pk = torch.empty((28 if taps == 27 else 1) * cout * cin, dtype=torch.bfloat16, device="cuda")
    assert L.lib().usp_nn_pack_weights(_p(w), _p(pk), cout, taps, cin, int(transposed), _st()) == 0
    return pk


SHAPES = [(16, 16, 27), (16, 32, 27), (64, 128, 27), (192, 64, 27), (48, 16, 27), (16, 16, 1)]
# global-load schedules; (32, 7, 32) splits the weight gradient's y sweep into uneven runs (7 = 4 + 3, 2 + 2 + 2 + 1)
GRIDS = [(8, 16, 16), (16, 32, 32), (32, 7, 32)]
WIDE_GRIDS = [(64, 64, 64), (256, 32, 32)]   # the LDS-staged schedules


@pytest.mark.parametrize("grid", GRIDS)
@pytest.mark.parametrize("cin,cout,taps", SHAPES)
def test_conv_forward_input_grad_and_weight_grad(cin, cout, taps, grid):
    _need_gpu()
    L = _lib()
    D, H, W = grid
    V = D * H * W
    print(f"[gpu-case] conv {cin}->{cout} taps {taps} grid {grid}", flush=True)
    g = torch.Generator().manual_seed(cin * 1000 + cout)
    xc = bf(torch.randn(cin, D, H, W, generator=g))
    x = from_cf(xc).cuda()
    w = bf(torch.randn(cout, taps, cin, generator=g) / math.sqrt(cin * taps)).cuda()
    b = torch.randn(cout, generator=g).cuda()
    out = torch.empty(V, cout, dtype=torch.float32, device="cuda")
    wp = pack(L, w, False)
    assert L.lib().usp_nn_conv3d(_p(x), _p(wp), _p(b), _p(out), 1, cout, D, H, W, cin, cout, taps, 1, 0, _st()) == 0
    xt = xc.double().requires_grad_(True)
    wt = w_to_torch(w, taps).requires_grad_(True)
    ref = S.conv(xt, wt, b.cpu().double(), relu=False)
    assert rel(rows_to_cf(out, grid), ref.detach()) < 1e-5
    # bf16 planes output with ReLU
    ob = torch.empty(cout // 16, V, 16, dtype=torch.bfloat16, device="cuda")
    assert L.lib().usp_nn_conv3d(_p(x), _p(wp), _p(b), _p(ob), 0, cout, D, H, W, cin, cout, taps, 1, 1, _st()) == 0
    assert rel(to_cf(ob, grid), torch.relu(ref.detach())) < 1e-2
    # input gradient with the transposed packing
    gyc = bf(torch.randn(cout, D, H, W, generator=g))
    gy = from_cf(gyc).cuda()
    wT = pack(L, w, True)
    gx = torch.empty(V, cin, dtype=torch.float32, device="cuda")
    assert L.lib().usp_nn_conv3d(_p(gy), _p(wT), None, _p(gx), 1, cin, D, H, W, cout, cin, taps, -1, 0, _st()) == 0
    ref_gx, ref_gw = torch.autograd.grad(ref, [xt, wt], gyc.double())
    assert rel(rows_to_cf(gx, grid), ref_gx) < 1e-5
    # weight and bias gradients
    nb = ct.c_size_t()
    assert L.lib().usp_nn_wgrad_workspace(D, H, W, cin, cout, taps, ct.byref(nb)) == 0
    ws = torch.empty(nb.value, dtype=torch.uint8, device="cuda")
    dw = torch.empty(cout, taps, cin, dtype=torch.float32, device="cuda")
    db = torch.empty(cout, dtype=torch.float32, device="cuda")
    assert L.lib().usp_nn_conv3d_wgrad(_p(x), _p(gy), _p(dw), _p(db), _p(ws), nb.value, D, H, W, cin, cout, taps,
                                       _st()) == 0
    assert rel(w_to_torch(dw, taps), ref_gw) < 1e-4
    assert rel(db.cpu().double(), gyc.double().sum(dim=(1, 2, 3))) < 1e-4


def conv_at(xc, w, b, z, y, x, sign):
    """Direct float64 sum at one voxel: sum_tap w[:, tap, :] @ xc[:, (z, y, x) + sign * off(tap)] (+ b)."""
    D, H, W = xc.shape[1:]
    out = np.zeros(w.shape[0]) if b is None else b.copy()
    for tap in range(27):
        dz, dy, dx = tap // 9 - 1, (tap // 3) % 3 - 1, tap % 3 - 1
        zz, yy, xx = z + sign * dz, y + sign * dy, x + sign * dx
        if 0 <= zz < D and 0 <= yy < H and 0 <= xx < W:
            out += w[:, tap, :] @ xc[:, zz, yy, xx]
    return out


@pytest.mark.parametrize("grid", WIDE_GRIDS)
@pytest.mark.parametrize("cin,cout", [(16, 16), (48, 16), (16, 48), (96, 32)])
def test_conv_wide_schedule(cin, cout, grid):
    """Grids of 2^18 voxels (the LDS-staged schedules, 64-wide and 16-wide bricks):
    forward and input gradient against direct float64 sums on sampled voxels
    (faces, corners and brick edges included); the weight gradient in full
    (the voxel-blocked copies and step chunks of a larger grid)."""
    _need_gpu()
    L = _lib()
    D, H, W = grid
    V = D * H * W
    print(f"[gpu-case] conv wide {cin}->{cout} grid {grid}", flush=True)
    g = torch.Generator().manual_seed(7 + cin + cout)
    xc = bf(torch.randn(cin, D, H, W, generator=g))
    x = from_cf(xc).cuda()
    w = bf(torch.randn(cout, 27, cin, generator=g) / math.sqrt(cin * 27)).cuda()
    b = torch.randn(cout, generator=g).cuda()
    out = torch.empty(V, cout, dtype=torch.float32, device="cuda")
    assert L.lib().usp_nn_conv3d(_p(x), _p(pack(L, w, False)), _p(b), _p(out), 1, cout, D, H, W, cin, cout, 27, 1, 0,
                                 _st()) == 0
    gyc = bf(torch.randn(cout, D, H, W, generator=g))
    gy = from_cf(gyc).cuda()
    gx = torch.empty(V, cin, dtype=torch.float32, device="cuda")
    assert L.lib().usp_nn_conv3d(_p(gy), _p(pack(L, w, True)), None, _p(gx), 1, cin, D, H, W, cout, cin, 27, -1, 0,
                                 _st()) == 0
    xn, gyn = xc.double().numpy(), gyc.double().numpy()
    wn = w.float().cpu().double().numpy()
    bn = b.cpu().double().numpy()
    outn = out.cpu().double().numpy().reshape(D, H, W, cout)
    gxn = gx.cpu().double().numpy().reshape(D, H, W, cin)
    rng = np.random.default_rng(0)
    pts = [tuple(int(rng.integers(0, n)) for n in grid) for _ in range(64)]
    pts += [(0, 0, 0), (D - 1, H - 1, W - 1), (0, H - 1, 0), (D - 1, 0, W - 1), (31, 0, 17), (5, H - 1, W - 2),
            (7, 15, 15), (8, 16, 16), (3, 3, 63 % W), (2, 4, 16)]
    for (z, y, x_) in pts:
        r = conv_at(xn, wn, bn, z, y, x_, 1)
        assert np.linalg.norm(outn[z, y, x_] - r) / np.linalg.norm(r) < 1e-5, (z, y, x_)
        r = conv_at(gyn, wn.transpose(2, 1, 0), None, z, y, x_, -1)
        assert np.linalg.norm(gxn[z, y, x_] - r) / np.linalg.norm(r) < 1e-5, (z, y, x_)
    nb = ct.c_size_t()
    assert L.lib().usp_nn_wgrad_workspace(D, H, W, cin, cout, 27, ct.byref(nb)) == 0
    ws = torch.empty(nb.value, dtype=torch.uint8, device="cuda")
    dw = torch.empty(cout, 27, cin, dtype=torch.float32, device="cuda")
    assert L.lib().usp_nn_conv3d_wgrad(_p(x), _p(gy), _p(dw), None, _p(ws), nb.value, D, H, W, cin, cout, 27,
                                       _st()) == 0
    xp = np.pad(xn, ((0, 0), (1, 1), (1, 1), (1, 1)))
    G = gyn.reshape(cout, -1)
    ref = np.empty((cout, 27, cin))
    for tap in range(27):
        kz, ky, kx = tap // 9, (tap // 3) % 3, tap % 3
        ref[:, tap, :] = G @ xp[:, kz:kz + D, ky:ky + H, kx:kx + W].reshape(cin, -1).T
    assert np.linalg.norm(dw.cpu().double().numpy() - ref) / np.linalg.norm(ref) < 1e-4


@pytest.mark.parametrize("cin,cout", [(16, 16), (48, 16), (16, 48)])
def test_conv_two_plane_bricks(cin, cout):
    """128^3 (2^21 voxels; convolutions of 16 input channels run on bricks of
    two output z-planes, 512 threads): forward and input gradient against
    direct float64 sums on sampled voxels, both planes of a brick, brick edges
    and the grid faces included."""
    _need_gpu()
    L = _lib()
    D = H = W = 128
    V = D * H * W
    grid = (D, H, W)
    print(f"[gpu-case] conv two-plane bricks {cin}->{cout} grid {grid}", flush=True)
    g = torch.Generator().manual_seed(11 + cin + cout)
    xc = bf(torch.randn(cin, D, H, W, generator=g))
    x = from_cf(xc).cuda()
    w = bf(torch.randn(cout, 27, cin, generator=g) / math.sqrt(cin * 27)).cuda()
    b = torch.randn(cout, generator=g).cuda()
    out = torch.empty(V, cout, dtype=torch.float32, device="cuda")
    assert L.lib().usp_nn_conv3d(_p(x), _p(pack(L, w, False)), _p(b), _p(out), 1, cout, D, H, W, cin, cout, 27, 1, 0,
                                 _st()) == 0
    gyc = bf(torch.randn(cout, D, H, W, generator=g))
    gy = from_cf(gyc).cuda()
    gx = torch.empty(V, cin, dtype=torch.float32, device="cuda")
    assert L.lib().usp_nn_conv3d(_p(gy), _p(pack(L, w, True)), None, _p(gx), 1, cin, D, H, W, cout, cin, 27, -1, 0,
                                 _st()) == 0
    xn, gyn = xc.double().numpy(), gyc.double().numpy()
    wn = w.float().cpu().double().numpy()
    bn = b.cpu().double().numpy()
    outn = out.cpu().double().numpy().reshape(D, H, W, cout)
    gxn = gx.cpu().double().numpy().reshape(D, H, W, cin)
    rng = np.random.default_rng(1)
    pts = [tuple(int(rng.integers(0, n)) for n in grid) for _ in range(64)]
    pts += [(0, 0, 0), (1, 0, 0), (D - 1, H - 1, W - 1), (D - 2, H - 1, W - 1), (0, H - 1, 0), (1, 3, 63),
            (2, 4, 64), (3, 7, 127), (64, 63, 64), (65, 64, 63), (127, 0, 65), (126, 127, 1)]
    for (z, y, x_) in pts:
        r = conv_at(xn, wn, bn, z, y, x_, 1)
        assert np.linalg.norm(outn[z, y, x_] - r) / np.linalg.norm(r) < 1e-5, (z, y, x_)
        r = conv_at(gyn, wn.transpose(2, 1, 0), None, z, y, x_, -1)
        assert np.linalg.norm(gxn[z, y, x_] - r) / np.linalg.norm(r) < 1e-5, (z, y, x_)


@pytest.mark.parametrize("grid", [(1, 1, 32), (2, 3, 96), (5, 2, 64), (3, 9, 32)])
@pytest.mark.parametrize("cin,cout", [(16, 16), (48, 16), (192, 64)])
def test_weight_gradient_sweep_edge_grids(cin, cout, grid):
    """The y-sweep weight gradient (and its bias) on grids that exercise its edges:
    a single plane and row (every neighbour in the zero padding), a width of three
    32-voxel segments, and few rows split into runs of one and two (the runs that
    stop inside a four-step group are in the first test's (32, 7, 32) grid);
    against float64 sums over the zero-padded grid."""
    _need_gpu()
    L = _lib()
    D, H, W = grid
    print(f"[gpu-case] wgrad sweep {cin}->{cout} grid {grid}", flush=True)
    g = torch.Generator().manual_seed(11 + cin + cout + D + H + W)
    xc = bf(torch.randn(cin, D, H, W, generator=g))
    gyc = bf(torch.randn(cout, D, H, W, generator=g))
    x, gy = from_cf(xc).cuda(), from_cf(gyc).cuda()
    nb = ct.c_size_t()
    assert L.lib().usp_nn_wgrad_workspace(D, H, W, cin, cout, 27, ct.byref(nb)) == 0
    ws = torch.empty(nb.value, dtype=torch.uint8, device="cuda")
    dw = torch.empty(cout, 27, cin, dtype=torch.float32, device="cuda")
    db = torch.empty(cout, dtype=torch.float32, device="cuda")
    assert L.lib().usp_nn_conv3d_wgrad(_p(x), _p(gy), _p(dw), _p(db), _p(ws), nb.value, D, H, W, cin, cout, 27,
                                       _st()) == 0
    xn, gyn = xc.double().numpy(), gyc.double().numpy()
    xp = np.pad(xn, ((0, 0), (1, 1), (1, 1), (1, 1)))
    G = gyn.reshape(cout, -1)
    ref = np.empty((cout, 27, cin))
    for tap in range(27):
        kz, ky, kx = tap // 9, (tap // 3) % 3, tap % 3
        ref[:, tap, :] = G @ xp[:, kz:kz + D, ky:ky + H, kx:kx + W].reshape(cin, -1).T
    assert np.linalg.norm(dw.cpu().double().numpy() - ref) / np.linalg.norm(ref) < 1e-4
    assert rel(db.cpu().double(), gyc.double().sum(dim=(1, 2, 3))) < 1e-4


@pytest.mark.parametrize("n,offset", [(16 * 4096, 0), (16 * 4096 - 8, 8), (1000, 1), (13, 0)])
def test_relu_backward_and_add_match_definition(n, offset):
    """ReLU backward (out = g where y > 0, else 0; plus out when accumulating)
    and the bf16 add, bit for bit against float arithmetic rounded to bf16: the
    16-byte path (aligned, n % 8 == 0) and the element path (an offset of one
    element misaligns the operands; ragged n)."""
    _need_gpu()
    L = _lib()
    print(f"[gpu-case] relu backward / add n {n} offset {offset}", flush=True)
    g = torch.Generator().manual_seed(n + offset)
    def mk():
        return torch.randn(n + offset, generator=g).to(torch.bfloat16).cuda()
    y, gr, out0 = mk(), mk(), mk()
    yv, gv = y[offset:], gr[offset:]
    for acc in (0, 1):
        out = out0.clone()
        ov = out[offset:]
        assert L.lib().usp_nn_relu_backward(_p(yv), _p(gv), _p(ov), n, acc, _st()) == 0
        ref = torch.where(yv.float() > 0, gv.float(), torch.zeros_like(gv.float()))
        if acc:
            ref = ref + out0[offset:].float()
        assert torch.equal(ov.cpu(), ref.to(torch.bfloat16).cpu()), acc
    dst = out0.clone()
    dv = dst[offset:]
    assert L.lib().usp_nn_add(_p(dv), _p(gv), n, _st()) == 0
    assert torch.equal(dv.cpu(), (out0[offset:].float() + gv.float()).to(torch.bfloat16).cpu())


def test_pool_upsample_and_copies():
    _need_gpu()
    L = _lib()
    D, H, W, C = 8, 16, 32, 32
    V = D * H * W
    g = torch.Generator().manual_seed(3)
    xc = bf(torch.randn(C, D, H, W, generator=g))
    x = from_cf(xc).cuda()
    p = torch.empty(C // 16, V // 8, 16, dtype=torch.bfloat16, device="cuda")
    assert L.lib().usp_nn_pool2(_p(x), _p(p), D, H, W, C, 0, _st()) == 0
    ref = torch.nn.functional.avg_pool3d(xc.double()[None], 2)[0]
    assert rel(to_cf(p, (D // 2, H // 2, W // 2)), ref) < 1e-2
    gb = torch.empty(C // 16, V, 16, dtype=torch.bfloat16, device="cuda")
    assert L.lib().usp_nn_pool2(_p(p), _p(gb), D, H, W, C, 1, _st()) == 0
    pc = to_cf(p, (D // 2, H // 2, W // 2))
    assert rel(to_cf(gb, (D, H, W)), torch.nn.functional.interpolate(pc[None], scale_factor=2)[0] / 8) < 1e-2
    # upsample into channels 16..48 of a 64-channel tensor, and its gradient
    cat = torch.zeros(4, V, 16, dtype=torch.bfloat16, device="cuda")
    assert L.lib().usp_nn_upsample2(_p(p), _p(cat), D, H, W, C, 64, 16, 0, _st()) == 0
    cf = to_cf(cat, (D, H, W))
    assert rel(cf[16:48], torch.nn.functional.interpolate(pc[None], scale_factor=2)[0]) < 1e-2
    assert float(cf[:16].abs().max()) == 0.0 and float(cf[48:].abs().max()) == 0.0
    gc = torch.empty(C // 16, V // 8, 16, dtype=torch.bfloat16, device="cuda")
    assert L.lib().usp_nn_upsample2(_p(cat), _p(gc), D, H, W, C, 64, 16, 1, _st()) == 0
    assert rel(to_cf(gc, (D // 2, H // 2, W // 2)), 8 * pc) < 1e-2
    # channel copy of whole planes: channels 16..48 of cat -> 0..32 of a 32-channel tensor
    dst = torch.empty(2, V, 16, dtype=torch.bfloat16, device="cuda")
    assert L.lib().usp_nn_channel_copy(_p(cat), 64, 16, _p(dst), 32, 0, 32, V, _st()) == 0
    assert torch.equal(to_cf(dst, (D, H, W)), cf[16:48])
    # planes must be whole
    assert L.lib().usp_nn_channel_copy(_p(cat), 64, 8, _p(dst), 32, 0, 16, V, _st()) != 0


def test_features_against_oracle():
    """Input channels (incl. the beam carried through the medium) vs the float64 oracle, to bf16 rounding."""
    _need_gpu()
    from paper_2207_14222_amd import media, surrogate
    print("[gpu-case] features 32x16x32", flush=True)
    shape = (32, 16, 32)
    prob = media.helmholtz_spheres(shape=shape, count=20, width=4, w0=5.0, plane=6, seed=11)
    nidx = prob.index.astype(np.complex64)
    net = surrogate.UNet3D(shape, seed=0)
    net.features(torch.from_numpy(nidx).cuda(), plane=6, w0=5.0, k0h=0.5 * math.pi)
    got = to_cf(net.a.x0, shape)
    ref = S.features(nidx.astype(np.complex128), 6, 5.0, 0.5 * math.pi)
    assert float((got[:5] - torch.from_numpy(ref)).abs().max()) < 1e-2
    assert float(got[5:].abs().max()) == 0.0


@pytest.mark.parametrize("D,plane", [(13, 0), (13, 5), (13, 12), (4, 3), (17, 8)])
def test_features_scan_depths_and_source_planes(D, plane):
    """The z scan of the beam channels (segments of z summed, scanned, walked
    again) for depths that do not split evenly into segments and source planes
    at either end, through the C ABI, vs the float64 oracle to bf16 rounding."""
    _need_gpu()
    L = _lib()
    print(f"[gpu-case] features D={D} plane={plane}", flush=True)
    H, W = 6, 40
    rng = np.random.default_rng(D * 31 + plane)
    nidx = (1.33 + 0.17 * rng.random((D, H, W)) + 1j * 0.2 * rng.random((D, H, W))).astype(np.complex64)
    out = torch.zeros(D * H * W * 16, dtype=torch.bfloat16, device="cuda")
    nd = torch.from_numpy(nidx).cuda()
    k0h, w0 = 0.5 * math.pi, 7.0
    L.check(L.lib().usp_nn_features(_p(nd), _p(out), D, H, W, 1.33, 0.17, 0.2, plane, k0h, w0, _st()))
    torch.cuda.synchronize()
    got = to_cf(out, (D, H, W))
    ref = S.features(nidx.astype(np.complex128), plane, w0, k0h)
    assert float((got[:5] - torch.from_numpy(ref)).abs().max()) < 1e-2
    assert float(got[5:].abs().max()) == 0.0


def _oracle_params(net):
    P = {}
    for name, ly in net.layers.items():
        w = w_to_torch(ly.wb, ly.taps)
        ci = 5 if name == "e1a" else ly.cin
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
    net.features(nidx, plane=4, w0=4.0)
    pred = net.forward().clone()
    feats = to_cf(net.a.x0, shape)[:5]
    P = _oracle_params(net)
    target = torch.from_numpy((prob.source * 0.3 + 0.1j * prob.index.real).astype(np.complex64))
    L_ref, grads, pred_ref = S.gradients(P, feats, target.to(torch.complex128), 0.5)
    pg = rows_to_cf(pred, shape)
    assert rel(pg, pred_ref) < 5e-2
    loss = net.loss(target.cuda(), grad=True)
    assert abs(loss - L_ref) < 5e-2 * L_ref
    net.backward()
    torch.cuda.synchronize()
    for name, ly in net.layers.items():
        ci = 5 if name == "e1a" else ly.cin
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
    net.features(torch.from_numpy(prob.index.astype(np.complex64)).cuda(), plane=4, w0=4.0)
    target = torch.from_numpy((0.2 * prob.index.real - 0.25 + 0.05j).astype(np.complex64)).cuda()
    losses = []
    for _ in range(60):
        net.forward()
        losses.append(net.loss(target, grad=True))
        net.backward()
        net.adam_step(lr=3e-3)
    assert all(math.isfinite(v) for v in losses)
    assert losses[-1] < 0.5 * losses[0]
