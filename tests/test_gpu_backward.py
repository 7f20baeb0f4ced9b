"""Backward pass to the input image on the device against the FP64 oracle.

Per-op parity: the backward-data conv (F32 / BF16 gates 1e-5 / 2e-2 relative
L2 on the same inputs); the max-pool gradient and the leaky gradient bit-exact
on inputs whose results are representable (ties included, so the
first-maximum rule is exercised).

Whole-pass parity (dn_input_gradient_arena, dn_nightmare_arena): the pass's
branch decisions (leaky signs, pooling window choices) are read back from the
arena; every decision that differs from the FP64 oracle's own must lie within
the forward's error bound of its threshold (the count per image is printed),
and the gradient must match the oracle's gradient on the device's piece at the
stated gates, FP32 1e-5 and BF16 2e-2 relative L2 per image, at every size
including the full 64 x 416 x 416 batch (tests/branch_check.py)."""
import numpy as np
import pytest

import oracle
import synth
from oracle import backward as ob
from oracle import net as onet
from tests import branch_check as BC
from tests import gpu_util as G

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dn():
    from paper_1811_03882_amd import dn as _dn
    G.torch_cuda()
    return _dn


def _params(cout, cin, k, seed, bn):
    rng = np.random.default_rng([seed, 11])
    p = synth.ConvParams(w=rng.normal(0, np.sqrt(2.0 / (cin * k * k)), (cout, cin, k, k)),
                         bias=rng.normal(0, 0.1, cout))
    if bn:
        p.mean = rng.normal(0, 0.3, cout)
        p.var = rng.uniform(0.5, 1.5, cout)
        p.gamma = rng.uniform(0.9, 1.1, cout)
        p.beta = rng.normal(0, 0.2, cout)
    return p


def _bn_scale(p, eps=1e-5):
    if p.gamma is None:
        return np.ones(p.w.shape[0])
    return p.gamma / np.sqrt(p.var + eps)


def run_conv_backward(dn, dtype, p, n, h, w, st, pad, dy, acc=None):
    torch = G.torch_cuda()
    cout, cin, k, _ = p.w.shape
    d = dn.conv_desc(n, h, w, cin, cout, k, st, pad, dn.LEAKY, 0.1, 0, 0, dtype)
    wb, vb, wsb = dn.conv_backward_sizes(d)
    wbuf, bz, us = G.empty_bytes(wb), G.empty_bytes(vb), G.empty_bytes(vb)
    dn.conv_pack_backward(d, p.w, p.mean, p.var, p.gamma, 1e-5, wbuf, bz, us)
    dyb = G.to_storage(dn, dtype, dy)
    dxb = G.to_storage(dn, dtype, acc) if acc is not None else G.empty_bytes(G.nhwc_bytes(dn, dtype, n, cin, h, w))
    ws = G.empty_bytes(wsb) if wsb else None
    dn.conv_backward_data(d, dyb, wbuf, bz, us, acc is not None, dxb, ws, wsb)
    torch.cuda.synchronize()
    return G.from_storage(dn, dtype, dxb, n, cin, h, w)


# forward convs whose backward-data is checked: batch, H, W, cin, cout, k, stride, pad, bn
BWD_SHAPES = [
    (2, 13, 11, 3, 16, 3, 1, 1, True),      # stem: 3-channel gradient (padded to 4 / 8)
    (1, 16, 16, 32, 64, 3, 1, 1, True),
    (2, 9, 7, 48, 40, 3, 2, 1, True),       # stride 2, ragged: spread gradient
    (1, 16, 18, 64, 128, 3, 2, 1, True),    # stride 2, even
    (3, 9, 11, 32, 125, 1, 1, 0, False),    # 1x1 from 125 channels (padded)
    (1, 8, 8, 256, 96, 3, 1, 1, True),      # long K: channel-block K order, split-K
    (2, 6, 5, 1024, 512, 3, 1, 1, True),    # 9-layer net's 1024-wide layers on a small map
    (1, 1, 1, 16, 32, 3, 1, 1, True),       # 1x1 map: every tap but the centre lies in the padding
    (1, 2, 3, 8, 8, 3, 2, 1, True),         # tiny ragged stride 2 (output 1x2)
]


@pytest.mark.parametrize("dtype", [0, 1], ids=["f32", "bf16"])
@pytest.mark.parametrize("shape", BWD_SHAPES, ids=lambda s: "b%d_%dx%d_c%d_co%d_k%d_s%d_p%d" % s[:8])
def test_conv_backward_data_parity(dn, dtype, shape):
    n, h, w, cin, cout, k, st, pad, bn = shape
    p = _params(cout, cin, k, 300 + cin, bn)
    ho, wo = (h + 2 * pad - k) // st + 1, (w + 2 * pad - k) // st + 1
    dy = synth.make_tensor((n, cout, ho, wo), 17, cout)
    ref = oracle.conv2d_backward_data(dy * _bn_scale(p)[None, :, None, None], p.w, st, pad, h, w)
    got = run_conv_backward(dn, dtype, p, n, h, w, st, pad, dy)
    err = G.rel_l2(got, ref)
    print("conv backward %s %s rel_l2=%.3e" % (G.NAME[dtype], shape, err))
    assert err < G.GATE[dtype]


@pytest.mark.parametrize("dtype", [0, 1], ids=["f32", "bf16"])
def test_conv_backward_data_accumulates(dn, dtype):
    n, h, w, cin, cout, k, st, pad = 2, 10, 9, 16, 32, 3, 2, 1
    p = _params(cout, cin, k, 5, True)
    dy = synth.make_tensor((n, cout, 5, 5), 18, 0)
    acc = synth.make_tensor((n, cin, h, w), 18, 1)
    ref = acc + oracle.conv2d_backward_data(dy * _bn_scale(p)[None, :, None, None], p.w, st, pad, h, w)
    got = run_conv_backward(dn, dtype, p, n, h, w, st, pad, dy, acc=acc)
    assert G.rel_l2(got, ref) < G.GATE[dtype]


def test_backward_rejects_empty_batch(dn):
    d = dn.conv_desc(0, 8, 8, 16, 16, 3, 1, 1, dn.LEAKY, 0.1, 0, 0, dn.F32)
    with pytest.raises(dn.DnError) as e:
        dn.conv_backward_sizes(d)
    assert e.value.status == dn.DN_EINVAL
    torch = G.torch_cuda()
    buf = torch.zeros(64, device="cuda")
    with pytest.raises(dn.DnError) as e:
        dn.maxpool_backward(0, 4, 4, 8, 2, 2, dn.F32, buf, buf, 0, buf)
    assert e.value.status == dn.DN_EINVAL


def test_conv_backward_rejects_fused_and_fp8(dn):
    d = dn.conv_desc(1, 8, 8, 16, 16, 3, 1, 1, dn.LEAKY, 0.1, 2, 0, dn.F32)
    with pytest.raises(dn.DnError) as e:
        dn.conv_backward_sizes(d)
    assert e.value.status == dn.DN_EUNSUPPORTED
    d = dn.conv_desc(1, 8, 8, 16, 16, 3, 1, 1, dn.LEAKY, 0.1, 0, 0, dn.FP8)
    with pytest.raises(dn.DnError) as e:
        dn.conv_backward_sizes(d)
    assert e.value.status == dn.DN_EUNSUPPORTED


# n, h, w, c, size, stride
POOL_BWD = [(2, 8, 10, 16, 2, 2), (1, 7, 9, 24, 2, 2), (2, 13, 13, 32, 2, 1), (1, 9, 8, 8, 3, 2), (1, 5, 6, 3, 3, 1),
            (1, 1, 1, 8, 2, 2), (1, 1, 3, 8, 2, 1)]  # windows that reach past a 1-pixel-high input


@pytest.mark.parametrize("dtype", [0, 1], ids=["f32", "bf16"])
@pytest.mark.parametrize("case", POOL_BWD, ids=lambda c: "b%d_%dx%d_c%d_k%d_s%d" % c)
@pytest.mark.parametrize("accumulate", [0, 1], ids=["write", "acc"])
def test_maxpool_backward_bit_exact(dn, dtype, case, accumulate):
    torch = G.torch_cuda()
    n, h, w, c, size, st = case
    rng = np.random.default_rng(list(case) + [dtype])
    x = rng.integers(-6, 7, (n, c, h, w)) / 4.0     # many ties inside windows
    ho, wo = (h - 1) // st + 1, (w - 1) // st + 1
    dy = rng.integers(-8, 9, (n, c, ho, wo)) / 4.0  # sums of up to 4 stay exact in BF16
    acc = rng.integers(-4, 5, (n, c, h, w)) / 4.0
    ref = oracle.maxpool_backward(x, size, st, dy) + (acc if accumulate else 0.0)
    xb, dyb = G.to_storage(dn, dtype, x), G.to_storage(dn, dtype, dy)
    dxb = G.to_storage(dn, dtype, acc) if accumulate else G.empty_bytes(G.nhwc_bytes(dn, dtype, n, c, h, w))
    dn.maxpool_backward(n, h, w, c, size, st, dtype, xb, dyb, accumulate, dxb)
    torch.cuda.synchronize()
    got = G.from_storage(dn, dtype, dxb, n, c, h, w)
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("dtype", [0, 1], ids=["f32", "bf16"])
def test_leaky_backward_bit_exact(dn, dtype):
    torch = G.torch_cuda()
    n, c, h, w = 2, 24, 7, 9
    rng = np.random.default_rng([dtype, 77])
    a = rng.integers(-3, 4, (n, c, h, w)) / 2.0  # exact zeros take the slope branch
    dy = synth.make_tensor((n, c, h, w), 19, dtype)
    slope = 0.1
    dy_st = dy.astype(np.float32) if dtype == 0 else ob.round_bf16(dy).astype(np.float32)
    ref = np.where(a > 0, dy_st, dy_st * np.float32(slope)).astype(np.float32).astype(np.float64)
    if dtype == 1:
        ref = ob.round_bf16(ref)
    ab, dyb = G.to_storage(dn, dtype, a), G.to_storage(dn, dtype, dy)
    count = n * h * w * dn.channel_pad(dtype, c)
    dn.leaky_backward(dtype, count, ab, dyb, slope, dyb)  # in place
    torch.cuda.synchronize()
    got = G.from_storage(dn, dtype, dyb, n, c, h, w)
    assert np.array_equal(got, ref)


def _small_net():
    return synth.Net("bwd_small", 3, 24, 20, [
        synth.conv(8, 3),
        synth.maxpool(2, 2),
        synth.conv(16, 3, stride=2),
        synth.conv(8, 1),
        synth.conv(16, 3),
        synth.shortcut(2),
        synth.maxpool(2, 1),
        synth.conv(5, 1, bn=False, act=synth.LINEAR),
    ])


def _ingest_net():
    # a 5x5 stem cannot take the first-layer kernel: the image goes through the
    # ingest kernel, and the stem's backward-data conv has pad 4 - 2 = 2
    return synth.Net("bwd_ingest", 3, 18, 22, [
        synth.Layer(synth.CONV, cout=8, ksize=5, stride=1, pad=2, batchnorm=True, activation=synth.LEAKY),
        synth.maxpool(2, 2),
        synth.conv(12, 3),
        synth.maxpool(3, 1),
        synth.conv(6, 1, bn=False, act=synth.LINEAR),
    ])


GRAD_CASES = [  # net builder, batch, h, w, seed, layers
    (_small_net, 2, 24, 20, 31, (0, 2, 5, 7)),
    (_ingest_net, 2, 18, 22, 36, (1, 4)),
    (synth.plain9, 1, 64, 64, 32, (9, 14)),
    (lambda: synth.residual52(units=(1, 2), widths=(64, 128), in_hw=32), 2, 32, 32, 33, (4, 11)),
]


@pytest.mark.parametrize("dtype", [0, 1], ids=["f32", "bf16"])
@pytest.mark.parametrize("case", GRAD_CASES, ids=["small", "ingest_5x5", "plain9_64", "residual_32"])
def test_input_gradient_parity(dn, dtype, case):
    build, n, h, w, seed, layers = case
    net = build()
    params = synth.make_params(net, seed)
    x = synth.make_input(net, n, seed, h=h, w=w)
    for layer in layers:
        print("case %s %s layer %d" % (net.name, G.NAME[dtype], layer), flush=True)
        BC.check_pass(dn, net, dtype, params, x, layer)


@pytest.mark.parametrize("dtype", [0, 1], ids=["f32", "bf16"])
def test_input_gradient_after_backward_autotune(dn, dtype):
    """Tuned tiles (split-K, accumulating epilogues, halo) for every conv of
    the pass, forward and backward, give the same gradient within the gates."""
    net = synth.residual52(units=(1, 2), widths=(64, 128), in_hw=32)
    n, h, w, seed, layer = 2, 32, 32, 37, 11
    params = synth.make_params(net, seed)
    x = synth.make_input(net, n, seed, h=h, w=w)
    BC.check_pass(dn, net, dtype, params, x, layer, tune=True, label="tuned residual_32")


@pytest.mark.parametrize("dtype", [0, 1], ids=["f32", "bf16"])
def test_nightmare_step_parity(dn, dtype):
    torch = G.torch_cuda()
    net = _small_net()
    n, h, w, seed, layer, rate = 2, 24, 20, 34, 5, 0.02
    params = synth.make_params(net, seed)
    x32 = synth.make_input(net, n, seed, h=h, w=w).astype(np.float32).astype(np.float64)
    got, stored, codes = BC.run_device_pass(dn, net, dtype, params, x32, layer, nightmare_rate=rate)
    ref_outs = onet.forward(net, params, x32, upto=layer + 1)
    passes, picks, flips, _ = BC.check_decisions(net, dtype, x32, layer, stored, codes, ref_outs)
    want = ob.ascent_step(x32, ob.input_gradient_on_piece(net, params, x32, layer, passes, picks), rate)
    # the step itself (x' - x) carries the whole error; compare it, clipped as on both sides
    err = G.rel_l2(got - x32, want - x32)
    print("nightmare step %s rel_l2=%.3e, branch flips per image %s" % (G.NAME[dtype], err, list(flips)))
    assert err < G.GATE[dtype]
    assert got.min() >= 0.0 and got.max() <= 1.0
    # further iterations (bound arena) keep the image in range and move it up the energy
    gn = dn.Net(net.layers, net.in_c, h, w, n, dtype=dtype, leaky_slope=net.leaky_slope, bn_eps=net.bn_eps)
    gn.load_params(params)
    gn.bind_arena(G.empty_bytes(gn.input_gradient_arena_bytes(layer, n, h, w)))
    e0 = ob.energy(net, params, got, layer)
    xd = G.dev(got.astype(np.float32))
    gn.nightmare(layer, xd, n, h, w, rate, 3)
    torch.cuda.synchronize()
    x4 = xd.cpu().numpy().astype(np.float64)
    assert x4.min() >= 0.0 and x4.max() <= 1.0
    assert ob.energy(net, params, x4, layer) > e0


@pytest.mark.parametrize("dtype", [0, 1], ids=["f32", "bf16"])
def test_input_gradient_plain9_full_size_all_images(dn, dtype):
    """The 9-layer net at its full size (batch 64, 416x416), gradient of the
    last layer's energy: every image against the oracle on the device's piece,
    with every differing branch decision checked against the forward-error
    bound."""
    net = synth.plain9()
    n, seed, layer = 64, 35, 14
    params = synth.make_params(net, seed)
    x = synth.make_input(net, n, seed)
    errs, got, _, _ = BC.check_pass(dn, net, dtype, params, x, layer, label="plain9 b64 416")
    assert np.all(np.isfinite(got))


def test_input_gradient_errors(dn):
    net = _small_net()
    torch = G.torch_cuda()
    x = torch.zeros((1, 3, 24, 20), device="cuda")
    g = torch.zeros_like(x)
    gn = dn.Net(net.layers, 3, 24, 20, 1, dtype=dn.F32)
    with pytest.raises(dn.DnError) as e:
        gn.input_gradient(7, x, 1, 24, 20, g)
    assert e.value.status == dn.DN_ESTATE  # weights not loaded
    gn.load_params(synth.make_params(net, 0))
    with pytest.raises(dn.DnError) as e:
        gn.input_gradient(8, x, 1, 24, 20, g)
    assert e.value.status == dn.DN_EINVAL  # no such layer
    with pytest.raises(dn.DnError) as e:
        gn.input_gradient(7, x, 1, 24, 20, g)
    assert e.value.status == dn.DN_ESTATE  # no arena bound
    need = gn.input_gradient_arena_bytes(7, 1, 24, 20)
    small = G.empty_bytes(need // 2)
    with pytest.raises(dn.DnError) as e:
        gn.input_gradient_arena(small, need // 2, 7, x, 1, 24, 20, g)
    assert e.value.status == dn.DN_ENOMEM
    f8 = dn.Net(net.layers, 3, 24, 20, 1, dtype=dn.FP8)
    f8.load_params(synth.make_params(net, 0))
    with pytest.raises(dn.DnError) as e:
        f8.input_gradient(7, x, 1, 24, 20, g)
    assert e.value.status == dn.DN_EUNSUPPORTED
