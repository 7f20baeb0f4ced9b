"""GPU parity of the single-layer entry points (C ABI via the binding) against
the FP64 oracle, plus the storage conversions against torch's casts.

Every HIP result is compared element by element with the oracle on the same
seeded FP64 inputs; FP32 within rel-L2 1e-5, BF16 2e-2, FP8 6e-2, and the
exact operations (pooling, conversion) bitwise.
"""
import numpy as np
import pytest

import oracle
import synth
from tests import gpu_util as G

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dn():
    from paper_1811_03882_amd import dn as _dn
    G.torch_cuda()
    return _dn


def _oracle_conv(x, p, k, stride, pad, act, pool=False, res=None, slope=0.1, eps=1e-5):
    y = oracle.conv2d(x, p.w, stride, pad)
    y = oracle.add_bias(y, p.bias)
    if p.mean is not None:
        y = oracle.batchnorm(y, p.mean, p.var, p.gamma, p.beta, eps)
    if act:
        y = oracle.leaky(y, slope)
    if res is not None:
        y = oracle.shortcut(y, res)
    if pool:
        y = oracle.maxpool(y, 2, 2)
    return y


def _params(cout, cin, k, seed, bn=True):
    net = synth.Net("t", cin, 8, 8, [synth.conv(cout, k, bn=bn)])
    return synth.make_params(net, seed)[0]


# ---------------------------------------------------------------- conversions


def test_f32_ingest_egress_roundtrip_exact(dn):
    x = synth.make_tensor((3, 5, 7, 9), 1, 0).astype(np.float32).astype(np.float64)
    buf = G.to_storage(dn, dn.F32, x)
    np.testing.assert_array_equal(G.from_storage(dn, dn.F32, buf, 3, 5, 7, 9), x)


def test_bf16_rounding_matches_torch(dn):
    torch = G.torch_cuda()
    rng = np.random.default_rng(3)
    x = rng.standard_normal((2, 11, 6, 5)).astype(np.float32)
    # include exact ties between two bf16 values (round-half-even cases)
    x.reshape(-1)[:64] = (np.arange(64, dtype=np.float32) + 0.5) * np.float32(2.0 ** -7) + np.float32(1.0)
    buf = G.to_storage(dn, dn.BF16, x.astype(np.float64))
    got = G.from_storage(dn, dn.BF16, buf, *x.shape)
    want = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    np.testing.assert_array_equal(got, want.astype(np.float64))


def test_fp8_codes_and_rounding_match_torch(dn):
    torch = G.torch_cuda()
    codes = torch.arange(256, dtype=torch.uint8).view(torch.float8_e4m3fn).to(torch.float32).numpy()
    finite = codes[np.isfinite(codes)]
    x = finite.reshape(1, 1, 1, -1).astype(np.float64)
    buf = G.to_storage(dn, dn.FP8, x)
    np.testing.assert_array_equal(G.from_storage(dn, dn.FP8, buf, *x.shape), x)  # every code round-trips
    rng = np.random.default_rng(4)
    v = (rng.standard_normal(4096) * rng.choice([1e-3, 0.1, 10.0, 300.0], 4096)).astype(np.float32)
    v[:8] = [500.0, -700.0, 448.0, -448.0, 464.0, 0.0, 2.0 ** -9, -(2.0 ** -10)]
    clamped = np.clip(v, -448.0, 448.0)
    want = torch.from_numpy(clamped).to(torch.float8_e4m3fn).to(torch.float32).numpy()
    x = v.reshape(1, 1, 1, -1).astype(np.float64)
    got = G.from_storage(dn, dn.FP8, G.to_storage(dn, dn.FP8, x), *x.shape)
    np.testing.assert_array_equal(got.reshape(-1), want.astype(np.float64))


# ---------------------------------------------------------------- convolution

# (batch, H, W, Cin, Cout, k, stride, pad, pool, act, bn)
SHAPES = [
    (1, 32, 32, 3, 16, 3, 1, 1, 1, 1, True),     # first layer of the single block
    (2, 24, 20, 16, 32, 3, 1, 1, 1, 1, True),    # pooled, ragged M
    (1, 13, 13, 64, 128, 3, 1, 1, 0, 1, True),   # M = 169 (13x13), ragged tail
    (3, 9, 11, 32, 125, 1, 1, 0, 0, 0, False),   # 1x1 linear, Cout 125 (padded)
    (2, 16, 16, 48, 64, 3, 2, 1, 0, 1, True),    # stride 2
    (1, 8, 8, 256, 96, 3, 1, 1, 0, 1, True),     # long K, channel-block-major K order
    (1, 10, 12, 96, 40, 3, 1, 1, 0, 1, True),    # 3 FP32 channel blocks; BF16 / FP8 tap-major
    (2, 7, 9, 320, 64, 2, 1, 0, 0, 1, True),     # 2x2 filter, 5 BF16 / 10 FP32 channel blocks
]


@pytest.mark.parametrize("dtype", [0, 1, 2], ids=["f32", "bf16", "fp8"])
@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "b%d_%dx%d_c%d_co%d_k%d_s%d_p%d" % s[:8] + ("_pool" if s[8] else ""))
def test_conv_layer_parity(dn, dtype, shape):
    b, h, w, cin, cout, k, st, pad, pool, act, bn = shape
    p = _params(cout, cin, k, 100 + cin, bn)
    x = synth.make_tensor((b, cin, h, w), 7, cin, 0.0, 1.0)
    ref = _oracle_conv(x, p, k, st, pad, act, pool)
    kw = {}
    if dtype == dn.FP8:
        kw = dict(in_scale=G.fp8_scale(x), out_scale=G.fp8_scale(ref))
    got = G.run_conv(dn, dtype, x, p, k, st, pad, act, pool=pool, **kw)
    err = G.rel_l2(got, ref)
    print("conv %s %s rel_l2=%.3e" % (G.NAME[dtype], shape, err))
    assert err < G.GATE[dtype]


# first-layer kernel (fused ingest): (batch, H, W, Cin, Cout, k, stride, pad, pool)
FIRST = [
    (2, 32, 32, 3, 16, 3, 1, 1, 1),     # single block / plain9 stem, pooled
    (1, 40, 72, 3, 32, 3, 1, 1, 0),     # residual stem, ragged tile edges, 2 channel blocks
    (1, 30, 34, 3, 12, 3, 2, 1, 0),     # stride 2, odd channel count
    (2, 18, 20, 4, 48, 3, 1, 1, 1),     # 4 input channels, 3 channel blocks
    (1, 21, 70, 6, 16, 2, 1, 0, 0),     # 6 channels padded to 8, 2x2 filter, ragged columns
    (2, 17, 66, 16, 24, 1, 2, 0, 0),    # 16 channels, 1x1 stride 2
    (1, 33, 40, 1, 64, 4, 2, 1, 0),     # 1 channel, 4x4 stride 2, 4 channel blocks
    (2, 70, 100, 3, 16, 3, 1, 1, 1),    # pooled, 32-row tiles: 3 tile rows (the last 6 rows), ragged columns
]


@pytest.mark.parametrize("dtype", [0, 1, 2], ids=["f32", "bf16", "fp8"])
@pytest.mark.parametrize("shape", FIRST, ids=lambda s: "b%d_%dx%d_c%d_co%d_k%d_s%d_p%d" % s[:8] + ("_pool" if s[8] else ""))
def test_first_layer_kernel_parity(dn, dtype, shape):
    b, h, w, cin, cout, k, st, pad, pool = shape
    p = _params(cout, cin, k, 200 + cout)
    x = synth.make_tensor((b, cin, h, w), 13, cout, 0.0, 1.0)
    ref = _oracle_conv(x, p, k, st, pad, 1, pool)
    kw = dict(in_scale=G.fp8_scale(x), out_scale=G.fp8_scale(ref)) if dtype == dn.FP8 else {}
    got = G.run_conv(dn, dtype, x, p, k, st, pad, 1, pool=pool, input_nchw=1, **kw)
    err = G.rel_l2(got, ref)
    print("first-layer %s %s rel_l2=%.3e" % (G.NAME[dtype], shape, err))
    assert err < G.GATE[dtype]
    if dtype == dn.F32:
        # same layer through the generic implicit-GEMM path: equal within FP32 rounding
        gen = G.run_conv(dn, dtype, x, p, k, st, pad, 1, pool=pool)
        assert G.rel_l2(got, gen) < 1e-6


# halo kernel (small K, <= 64 output channels): (batch, H, W, Cin, Cout, k, stride, pad, pool, residual)
HALO = [
    (2, 24, 20, 16, 32, 3, 1, 1, 1, 0),   # 9-layer c2 shape class, pooled, ragged tile
    (1, 20, 36, 32, 64, 3, 1, 1, 0, 0),   # c3 shape class, two column tiles
    (2, 10, 10, 64, 32, 1, 1, 0, 0, 0),   # 1x1 reduction of a residual unit
    (1, 17, 19, 16, 48, 3, 2, 1, 0, 0),   # stride 2, odd sizes
    (2, 12, 14, 16, 32, 3, 1, 1, 0, 1),   # fused residual add
    (2, 18, 40, 32, 48, 3, 1, 1, 1, 0),   # three 16-channel blocks
]
# full-size 9-layer c2 / c3 classes: more tiles than workgroups, so the
# persistent kernel runs several tiles per workgroup and per XCD run
HALO_BIG = [
    (8, 208, 208, 16, 32, 3, 1, 1, 1, 0),
    (16, 104, 104, 32, 64, 3, 1, 1, 1, 0),
]
HALO_TILE, HALO2_TILE = 100, 101


def halo_cases():
    """(shape, dtype, tile) of HALO + HALO_BIG that the halo kernels take (the
    library's host-side check, no GPU needed); the others are rejected with
    DN_EUNSUPPORTED, which tests/test_abi_cpu.py checks."""
    from paper_1811_03882_amd import dn as _dn
    out = []
    for shape in HALO + HALO_BIG:
        b, h, w, cin, cout, k, st, pad, pool, resid = shape
        for dtype, dname in ((0, "f32"), (1, "bf16"), (2, "fp8")):
            for tile, tname in ((HALO_TILE, "halo"), (HALO2_TILE, "halo2")):
                try:
                    _dn.conv_sizes(_dn.conv_desc(b, h, w, cin, cout, k, st, pad, 1, 0.1, 2 if pool else 0, resid,
                                                 dtype, tile=tile, splits=1))
                except _dn.DnError:
                    continue
                sid = "b%d_%dx%d_c%d_co%d_k%d_s%d_p%d" % shape[:8] + ("_pool" if pool else "") + ("_res" if resid else "")
                out.append(pytest.param(shape, dtype, tile, id="%s-%s-%s" % (sid, dname, tname)))
    return out


@pytest.mark.parametrize("shape,dtype,tile", halo_cases())
def test_halo_kernel_parity(dn, dtype, shape, tile):
    b, h, w, cin, cout, k, st, pad, pool, resid = shape
    p = _params(cout, cin, k, 300 + cout)
    x = synth.make_tensor((b, cin, h, w), 14, cin, 0.0, 1.0)
    ho, wo = (h + 2 * pad - k) // st + 1, (w + 2 * pad - k) // st + 1
    r = synth.make_tensor((b, cout, ho, wo), 14, 99, -1.0, 1.0) if resid else None
    ref = _oracle_conv(x, p, k, st, pad, 1, pool, res=r)
    kw = {}
    if dtype == dn.FP8:
        kw = dict(in_scale=G.fp8_scale(x), out_scale=G.fp8_scale(ref), res_scale=G.fp8_scale(r) if resid else 1.0)
    got = G.run_conv(dn, dtype, x, p, k, st, pad, 1, pool=pool, res=r, tile=tile, splits=1, **kw)
    err = G.rel_l2(got, ref)
    print("halo%s %s %s rel_l2=%.3e" % ("" if tile == HALO_TILE else "2", G.NAME[dtype], shape, err))
    assert err < G.GATE[dtype]
    # same reduction order as the GEMM tiles: identical bits
    gem = G.run_conv(dn, dtype, x, p, k, st, pad, 1, pool=pool, res=r, tile=0, splits=1, **kw)
    np.testing.assert_array_equal(got, gem)


@pytest.mark.parametrize("dtype", [0, 1, 2], ids=["f32", "bf16", "fp8"])
def test_every_tile_config_agrees(dn, dtype):
    b, h, w, cin, cout, k = 2, 12, 14, 40, 72, 3
    p = _params(cout, cin, k, 5)
    x = synth.make_tensor((b, cin, h, w), 8, 0, 0.0, 1.0)
    ref = _oracle_conv(x, p, k, 1, 1, 1)
    kw = dict(in_scale=G.fp8_scale(x), out_scale=G.fp8_scale(ref)) if dtype == dn.FP8 else {}
    outs = []
    for t in range(dn.tile_count()):
        got = G.run_conv(dn, dtype, x, p, k, 1, 1, 1, tile=t, splits=1, **kw)
        err = G.rel_l2(got, ref)
        print("tile %d %s rel_l2=%.3e" % (t, dn.tile_info(t), err))
        assert err < G.GATE[dtype]
        outs.append(got)
    # the K-reduction order does not depend on the tile shape: identical bits
    # among tiles with the same MFMA block (BF16 32x32 blocks sum each 16-wide
    # K step in one instruction, 16x16 blocks each 32-wide step: FP32 rounding
    # differs, so across block sides only the storage rounding may differ)
    side = [dn.tile_info(t)[4] if dtype == dn.BF16 else 16 for t in range(dn.tile_count())]
    for t, o in enumerate(outs):
        first = side.index(side[t])
        np.testing.assert_array_equal(o, outs[first])
        assert G.rel_l2(o, outs[0]) < 1e-3


@pytest.mark.parametrize("dtype", [0, 1], ids=["f32", "bf16"])
def test_split_k_matches_oracle(dn, dtype):
    b, h, w, cin, cout, k = 1, 13, 13, 512, 256, 3
    p = _params(cout, cin, k, 6)
    x = synth.make_tensor((b, cin, h, w), 9, 0, 0.0, 1.0)
    ref = _oracle_conv(x, p, k, 1, 1, 1)
    for sp in (1, 2, 4, 8):
        got = G.run_conv(dn, dtype, x, p, k, 1, 1, 1, tile=0, splits=sp)
        err = G.rel_l2(got, ref)
        print("splits %d rel_l2=%.3e" % (sp, err))
        assert err < G.GATE[dtype]


@pytest.mark.parametrize("dtype", [0, 1, 2], ids=["f32", "bf16", "fp8"])
def test_conv_with_fused_residual(dn, dtype):
    b, h, w, c = 2, 10, 10, 64
    p = _params(c, c // 2, 3, 7)
    x = synth.make_tensor((b, c // 2, h, w), 10, 0, 0.0, 1.0)
    r = synth.make_tensor((b, c, h, w), 10, 1, -1.0, 1.0)
    ref = _oracle_conv(x, p, 3, 1, 1, 1, res=r)
    kw = {}
    if dtype == dn.FP8:
        kw = dict(in_scale=G.fp8_scale(x), res_scale=G.fp8_scale(r), out_scale=G.fp8_scale(ref))
    got = G.run_conv(dn, dtype, x, p, 3, 1, 1, 1, res=r, **kw)
    assert G.rel_l2(got, ref) < G.GATE[dtype]


def test_bf16_32x32_tiles_pool_residual_split(dn):
    """Every BF16 tile with 32x32 MFMA blocks, with the fused pool, the fused
    residual and split-K, against the oracle and against a 16x16 tile."""
    tiles = [t for t in range(dn.tile_count()) if dn.tile_info(t)[4] == 32]
    assert tiles
    b, h, w, cin, cout = 2, 14, 18, 72, 96
    p = _params(cout, cin, 3, 17)
    x = synth.make_tensor((b, cin, h, w), 14, 0, 0.0, 1.0)
    r = synth.make_tensor((b, cout, h, w), 14, 1, -1.0, 1.0)
    ref_pool = _oracle_conv(x, p, 3, 1, 1, 1, pool=True)
    ref_res = _oracle_conv(x, p, 3, 1, 1, 1, res=r)
    base_pool = G.run_conv(dn, dn.BF16, x, p, 3, 1, 1, 1, pool=1, tile=0, splits=1)
    for t in tiles:
        got = G.run_conv(dn, dn.BF16, x, p, 3, 1, 1, 1, pool=1, tile=t, splits=1)
        e1 = G.rel_l2(got, ref_pool)
        got_r = G.run_conv(dn, dn.BF16, x, p, 3, 1, 1, 1, res=r, tile=t, splits=1)
        e2 = G.rel_l2(got_r, ref_res)
        got_s = G.run_conv(dn, dn.BF16, x, p, 3, 1, 1, 1, res=r, tile=t, splits=3)
        e3 = G.rel_l2(got_s, ref_res)
        print("tile %d %s pool %.3e residual %.3e split3 %.3e" % (t, dn.tile_info(t), e1, e2, e3))
        assert max(e1, e2, e3) < G.GATE[dn.BF16]
        assert G.rel_l2(got, base_pool) < 1e-3


# ---------------------------------------------------------------- pool / add


@pytest.mark.parametrize("dtype", [0, 1, 2], ids=["f32", "bf16", "fp8"])
@pytest.mark.parametrize("h,w,size,stride", [(13, 13, 2, 1), (26, 26, 2, 2), (7, 9, 2, 2), (9, 8, 3, 2)])
def test_maxpool_exact(dn, dtype, h, w, size, stride):
    x = synth.make_tensor((2, 20, h, w), 11, h, -2.0, 2.0)
    xs = G.from_storage(dn, dtype, G.to_storage(dn, dtype, x), *x.shape)  # values the storage type holds
    ho, wo = (h - 1) // stride + 1, (w - 1) // stride + 1
    y = G.empty_bytes(G.nhwc_bytes(dn, dtype, 2, 20, ho, wo))
    dn.maxpool(2, h, w, 20, size, stride, dtype, G.to_storage(dn, dtype, xs), y)
    got = G.from_storage(dn, dtype, y, 2, 20, ho, wo)
    np.testing.assert_array_equal(got, oracle.maxpool(xs, size, stride))


def test_shortcut_f32_exact(dn):
    a = synth.make_tensor((2, 8, 5, 5), 12, 0).astype(np.float32).astype(np.float64)
    b = synth.make_tensor((2, 8, 5, 5), 12, 1).astype(np.float32).astype(np.float64)
    y = G.empty_bytes(G.nhwc_bytes(dn, 0, 2, 8, 5, 5))
    cnt = 2 * 5 * 5 * dn.channel_pad(0, 8)
    dn.shortcut(0, cnt, G.to_storage(dn, 0, a), 1.0, G.to_storage(dn, 0, b), 1.0, y, 1.0)
    got = G.from_storage(dn, 0, y, 2, 8, 5, 5)
    np.testing.assert_array_equal(got, (a.astype(np.float32) + b.astype(np.float32)).astype(np.float64))


def test_mfma_peak_probe(dn):
    """The throughput probe runs for every dtype and reports a rate between a
    tenth of and just above the datasheet dense peak."""
    datasheet = {dn.F32: 157.3, dn.BF16: 2516.6, dn.FP8: 5033.2}
    for dt, peak in datasheet.items():
        got = dn.mfma_peak(dt)
        print("MFMA probe dtype %d: %.1f TFLOP/s (datasheet %.1f)" % (dt, got, peak))
        assert 0.1 * peak < got < 1.05 * peak
    with pytest.raises(dn.DnError):
        dn.mfma_peak(9)


def test_bad_arguments_are_rejected(dn):
    d = dn.conv_desc(1, 13, 13, 8, 8, 3, 1, 1, pool=2)  # odd output cannot take the fused pool
    with pytest.raises(dn.DnError) as e:
        dn.conv_sizes(d)
    assert e.value.status == dn.DN_EUNSUPPORTED
    with pytest.raises(dn.DnError) as e:
        dn.conv2d(dn.conv_desc(1, 8, 8, 8, 8, 3, 1, 1), 0, 0, 0, 0, 0, 0)
    assert e.value.status == dn.DN_EINVAL
