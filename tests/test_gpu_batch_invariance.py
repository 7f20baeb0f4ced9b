"""Batch invariance: with batch_invariant = 1 an image's output has the same
bits whether it runs alone or inside a batch.

Each net is tuned separately at every batch size (tiles may differ with the
batch), but the split-K partition of every conv depends on its K alone and
only tiles of 16x16 MFMA blocks (and the halo kernels, which sum in their
order) run.  Checked bitwise for the 9-layer detection CNN (BF16, 416x416,
images alone against the same images at batch 64 and inside a ragged batch of
5), for the same net in FP32 and FP8 at 160x160 (batch 16; FP8 with one
calibration for every batch size), and for the 52-layer residual CNN (BF16,
256x256, batch 16, whose small-M stages run split-K); the plans are checked
to split the same convs the same way at every batch.  Without the option the same comparison is printed
for reference (the tuner may then pick batch-dependent splits and block
shapes).
"""
import numpy as np
import pytest

import synth
from tests import gpu_util as G

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dn():
    from paper_1811_03882_amd import dn as _dn
    G.torch_cuda()
    return _dn


def _run(dn, net, params, x, h, w, invariant, dtype=1, calib=None):
    """Forward x (N images) through a net tuned at batch N; returns (output, conv plans)."""
    torch = G.torch_cuda()
    b = x.shape[0]
    mb = max(b, calib.shape[0]) if calib is not None else b
    n = dn.Net(net.layers, net.in_c, h, w, mb, dtype=dtype, use_graph=True, batch_invariant=invariant,
               leaky_slope=net.leaky_slope, bn_eps=net.bn_eps)
    n.load_params(params)
    if dtype == dn.FP8:  # one calibration input for every batch size: the same activation scales
        n.calibrate(G.dev(calib.astype(np.float32)), calib.shape[0], h, w)
    arena = G.empty_bytes(2 * n.arena_bytes(b, h, w) + (256 << 20))
    n.bind_arena(arena)
    n.autotune(b, h, w)
    assert n.arena_bytes(b, h, w) <= arena.numel()
    plans = {}
    for li, layer in enumerate(net.layers):
        if layer.kind == synth.CONV and li > 0:
            plans[li] = n.layer_plan(li, b, h, w)
    y = torch.empty((b,) + n.output_shape(h, w), dtype=torch.float32, device="cuda")
    y.fill_(float("nan"))
    n.forward(G.dev(x.astype(np.float32)), b, h, w, y)
    torch.cuda.synchronize()
    out = y.cpu().numpy()
    n.close()
    return out, plans


def _check(dn, net, params, xb, h, w, alone_idx, mixes, tmp_path, monkeypatch, name, dtype=1, calib=None):
    monkeypatch.setenv("DN_TUNE_CACHE", str(tmp_path / ("tune_%s.txt" % name)))
    B = xb.shape[0]
    run = lambda x, inv: _run(dn, net, params, x, h, w, inv, dtype, calib)
    for invariant in (True, False):
        yb, pb = run(xb, invariant)
        assert np.all(np.isfinite(yb))
        results = []
        for i in alone_idx:
            y1, p1 = run(xb[i:i + 1], invariant)
            same = np.array_equal(y1[0], yb[i])
            results.append(same)
            print("%s invariant=%d: image %d alone vs in batch %d: bitwise %s, max |diff| %.3e" %
                  (name, invariant, i, B, same, np.max(np.abs(y1[0] - yb[i]))), flush=True)
            if invariant:
                splits_b = {li: p["splits"] for li, p in pb.items()}
                splits_1 = {li: p["splits"] for li, p in p1.items()}
                assert splits_b == splits_1, (splits_b, splits_1)
        for sel in mixes:
            ym, _ = run(xb[list(sel)], invariant)
            for j, i in enumerate(sel):
                same = np.array_equal(ym[j], yb[i])
                results.append(same)
                print("%s invariant=%d: image %d at %d of a batch of %d vs in batch %d: bitwise %s" %
                      (name, invariant, i, j, len(sel), B, same), flush=True)
        if invariant:
            print("%s splits per conv: %s" % (name, {li: p["splits"] for li, p in pb.items()}))
            assert all(results)


def test_plain9_bf16_alone_equals_in_batch64(dn, tmp_path, monkeypatch):
    net = synth.plain9()
    params = synth.make_params(net, synth.SEED_PLAIN)
    xb = synth.make_input(net, 64, synth.SEED_PLAIN, tag=5)
    _check(dn, net, params, xb, 416, 416, (0, 31, 63), [(63, 7, 12, 0, 40)], tmp_path, monkeypatch, "plain9")


def test_residual52_bf16_alone_equals_in_batch16(dn, tmp_path, monkeypatch):
    net = synth.residual52()
    params = synth.make_params(net, synth.SEED_RESIDUAL)
    xb = synth.make_input(net, 16, synth.SEED_RESIDUAL, tag=5)
    _check(dn, net, params, xb, 256, 256, (0, 9), [(15, 3, 9)], tmp_path, monkeypatch, "residual52")


@pytest.mark.parametrize("dtype", [0, 2], ids=["f32", "fp8"])
def test_plain9_f32_fp8_alone_equals_in_batch16(dn, dtype, tmp_path, monkeypatch):
    net = synth.plain9()
    params = synth.make_params(net, synth.SEED_PLAIN)
    xb = synth.make_input(net, 16, synth.SEED_PLAIN, tag=6, h=160, w=160)
    calib = synth.make_input(net, 4, synth.SEED_CALIB, h=160, w=160)
    _check(dn, net, params, xb, 160, 160, (0, 15), [(15, 2, 9)], tmp_path, monkeypatch, "plain9_%d" % dtype,
           dtype=dtype, calib=calib)
