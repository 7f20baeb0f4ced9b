"""Seeded generator checks: reproducibility, shapes and the moments of each
stated distribution (variance reading of N(a, b))."""
import numpy as np

import synth


def test_reproducible_and_batch_independent_weights():
    net = synth.plain9()
    a = synth.make_params(net, 1)
    b = synth.make_params(net, 1)
    for pa, pb in zip(a, b):
        if pa is not None:
            np.testing.assert_array_equal(pa.w, pb.w)
    x1 = synth.make_input(net, 1, 1, h=32, w=32)
    x4 = synth.make_input(net, 4, 1, h=32, w=32)
    np.testing.assert_array_equal(x1[0], x4[0])
    c = synth.make_params(net, 2)
    assert not np.array_equal(a[0].w, c[0].w)


def test_shapes_and_bn_presence():
    net = synth.plain9()
    p = synth.make_params(net, 1)
    chans = synth.conv_in_channels(net)
    for L, q, cin in zip(net.layers, p, chans):
        if L.kind != synth.CONV:
            assert q is None
            continue
        assert q.w.shape == (L.cout, cin, L.ksize, L.ksize)
        assert (q.mean is not None) == L.batchnorm
    assert p[-1].mean is None and p[-1].w.shape == (125, 1024, 1, 1)


def test_distribution_moments():
    net = synth.residual52()
    p = [q for q in synth.make_params(net, 2) if q is not None]
    big = max(p, key=lambda q: q.w.size)
    fan_in = big.w[0].size
    assert abs(big.w.var() - 2.0 / fan_in) / (2.0 / fan_in) < 0.02
    allb = np.concatenate([q.bias for q in p])
    assert abs(allb.var() - 0.01) < 0.001 and abs(allb.mean()) < 0.01
    mean = np.concatenate([q.mean for q in p])
    assert abs(mean.var() - 0.1) < 0.01
    var = np.concatenate([q.var for q in p])
    assert var.min() >= 0.5 and var.max() < 1.5 and abs(var.mean() - 1.0) < 0.02
    g = np.concatenate([q.gamma for q in p])
    assert g.min() >= 0.9 and g.max() < 1.1
    be = np.concatenate([q.beta for q in p])
    assert abs(be.var() - 0.05) < 0.005
    x = synth.make_input(net, 2, 2)
    assert x.min() >= 0.0 and x.max() < 1.0 and abs(x.mean() - 0.5) < 0.01


def test_serving_trace():
    tr = synth.serving_trace()
    assert len(tr.arrival_s) == 10000
    assert np.all(np.diff(tr.arrival_s) >= 0)
    rate = len(tr.arrival_s) / tr.arrival_s[-1]
    assert 1900 < rate < 2100
    assert set(np.unique(tr.size)) == {160, 224, 320, 416, 608}
