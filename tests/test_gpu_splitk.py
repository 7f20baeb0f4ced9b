"""In-kernel split-K finish against the separate finish launch, bitwise.

A net's split convs on small tiles finish in the GEMM kernel itself: the last
of a tile's split workgroups to arrive sums the tile's FP32 partials in split
order and runs the epilogue (larger tiles keep the separate finish launch).
dn_conv2d always finishes with its own launch.  A small net whose convs are
forced through the tune cache to chosen tiles and split counts (a fused 2x2
pool, a fused residual, ragged output channels, split counts that do not
divide the K-tiles, a split with no K-tile at all, one conv on the separate
finish between them) must give the same bits as the same convs run one by one
through dn_conv2d with the same tiles and splits, on every graph replay and
eagerly, and stay within the dtype's gate of the FP64 oracle.
"""
import numpy as np
import pytest

import synth
from oracle import net as onet
from tests import gpu_util as G

pytestmark = pytest.mark.gpu

BATCH, H, W, C = 3, 16, 16, 3
NET = synth.Net("splitk", C, H, W, [
    synth.conv(64, 3),                                  # 0, the first-layer kernel (no split)
    synth.conv(96, 3),                                  # 1, with the pool below fused: pooled split finish
    synth.maxpool(),                                    # 2
    synth.conv(128, 3),                                 # 3
    synth.conv(96, 3),                                  # 4, with the shortcut below fused: residual split finish
    synth.shortcut(2),                                  # 5
    synth.conv(40, 1, bn=False, act=synth.LINEAR),      # 6, 40 output channels
])
# (ci, co, R, pool, res) of each split conv's signature -> (tile, splits)
FORCED = {
    (64, 96, 3, 1, 0): (0, 3),     # 64x64, 9 K-tiles in 3 splits (BF16): in-kernel finish
    (96, 128, 3, 0, 0): (14, 2),   # LDS-DMA 128x128: separate finish
    (128, 96, 3, 0, 1): (9, 8),    # 64x32, 18 K-tiles in 8 splits of 3 (BF16; the last two get none): in-kernel
    (96, 40, 1, 0, 0): (0, 2),     # 64x64, one K-tile per split (BF16): in-kernel
}


@pytest.fixture(scope="module")
def dn():
    from paper_1811_03882_amd import dn as _dn
    G.torch_cuda()
    return _dn


def _sig_key(sig):
    f = dict((t[:2], t[2:]) if t[:2] in ("ci", "co") else (t[:1], t[1:]) for t in sig.split("_") if t)
    return int(f["ci"]), int(f["co"]), int(f["R"]), int(f["p"]), int(f["r"])


def _forced_cache(dn, dtype, params, path, monkeypatch):
    """Tune once to learn the convs' signatures, then rewrite the cache with the forced configurations."""
    monkeypatch.setenv("DN_TUNE_CACHE", str(path))
    n = dn.Net(NET.layers, C, H, W, BATCH, dtype=dtype)
    n.load_params(params)
    arena = G.empty_bytes(2 * n.arena_bytes(BATCH, H, W))
    n.bind_arena(arena)
    n.autotune(BATCH, H, W)
    n.close()
    lines = []
    for line in path.read_text().splitlines():
        name = line.split()[0]
        sig = name.split("/", 1)[1]
        if not sig.startswith("dt%d_" % dtype):
            continue
        ci, co, r, p, res = _sig_key(sig)
        cp = lambda c: dn.channel_pad(dtype, c)
        key = next(k for k in FORCED if (cp(k[0]), cp(k[1]), k[2], k[3], k[4]) == (ci, co, r, p, res))
        t, s = FORCED[key]
        lines.append("%s %d %d\n" % (name, t, s))
    assert len(lines) == len(FORCED)
    path.write_text("".join(lines))


def _separate_chain(dn, dtype, params, x):
    """The same convs through dn_conv2d (separate finish launch), tiles and splits as forced."""
    torch = G.torch_cuda()
    n = x.shape[0]

    def conv(xb, cin, h, w, li, ksize, pool, res, act, first=False):
        p = params[li]
        cout = p.w.shape[0]
        t, s = (-1, 0) if first else FORCED[(cin, cout, ksize, 1 if pool else 0, 1 if res is not None else 0)]
        d = dn.conv_desc(n, h, w, cin, cout, ksize, 1, ksize // 2, act, NET.leaky_slope, 2 if pool else 0,
                         1 if res is not None else 0, dtype, 1.0, 1.0, 1.0, t, s, 1 if first else 0)
        wb, vb, wsb = dn.conv_sizes(d)
        assert first or wsb > 0
        wbuf, bbuf, sbuf = G.empty_bytes(wb), G.empty_bytes(vb), G.empty_bytes(vb)
        dn.conv_pack(d, p.w, p.bias, p.mean, p.var, p.gamma, p.beta, NET.bn_eps, wbuf, bbuf, sbuf)
        ho, wo = (h // 2, w // 2) if pool else (h, w)
        yb = G.empty_bytes(G.nhwc_bytes(dn, dtype, n, cout, ho, wo))
        ws = G.empty_bytes(wsb) if wsb else None
        dn.conv2d(d, xb, wbuf, bbuf, sbuf, res, yb, ws, wsb)
        torch.cuda.synchronize()
        return yb

    y0 = conv(G.dev(x.astype(np.float32)), C, H, W, 0, 3, False, None, dn.LEAKY, first=True)
    y1 = conv(y0, 64, H, W, 1, 3, True, None, dn.LEAKY)
    y3 = conv(y1, 96, H // 2, W // 2, 3, 3, False, None, dn.LEAKY)
    y4 = conv(y3, 128, H // 2, W // 2, 4, 3, False, y1, dn.LEAKY)
    y6 = conv(y4, 96, H // 2, W // 2, 6, 1, False, None, dn.LINEAR)
    return G.from_storage(dn, dtype, y6, n, 40, H // 2, W // 2)


@pytest.mark.parametrize("dtype", [1, 0], ids=["bf16", "f32"])
def test_in_kernel_split_finish_is_bitwise_the_separate_finish(dn, dtype, tmp_path, monkeypatch):
    torch = G.torch_cuda()
    params = synth.make_params(NET, 21)
    x = synth.make_input(NET, BATCH, 21)
    _forced_cache(dn, dtype, params, tmp_path / "tune.txt", monkeypatch)
    ref = _separate_chain(dn, dtype, params, x)
    oracle = onet.forward(NET, params, x)[-1]
    print("separate finish vs oracle rel_l2 %.3e" % G.rel_l2(ref, oracle))
    assert G.rel_l2(ref, oracle) < G.GATE[dtype]
    xd = G.dev(x.astype(np.float32))
    for graph in (True, False):
        n = dn.Net(NET.layers, C, H, W, BATCH, dtype=dtype, use_graph=graph)
        n.load_params(params)
        arena = G.empty_bytes(4 * n.arena_bytes(BATCH, H, W))  # room for the forced splits' partials
        arena.fill_(0xA5)  # the counters start as garbage: each forward zeroes them
        n.bind_arena(arena)
        n.autotune(BATCH, H, W)  # every signature is in the cache: nothing is timed
        assert n.arena_bytes(BATCH, H, W) <= arena.numel()
        for li, layer in enumerate(NET.layers):
            if layer.kind == synth.CONV and li > 0:
                plan = n.layer_plan(li, BATCH, H, W)
                print("layer", li, plan)
                assert plan["splits"] > 1
        y = torch.empty((BATCH, 40, H // 2, W // 2), dtype=torch.float32, device="cuda")
        for rep in range(4):
            y.fill_(float("nan"))
            n.forward(xd, BATCH, H, W, y)
            torch.cuda.synchronize()
            got = y.cpu().numpy().astype(np.float64)
            same = np.array_equal(got, ref)
            print("graph=%s replay %d: bitwise %s, max |diff| %.3e" % (graph, rep, same, np.max(np.abs(got - ref))))
            assert same
        n.close()
