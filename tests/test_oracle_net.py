"""Whole-network oracle checks (CPU): structure, composition and identity units."""
import numpy as np

import oracle
import synth
from oracle import net as onet


def test_layer_counts_and_shapes_small_inputs():
    n9 = synth.plain9()
    assert sum(L.kind == synth.CONV for L in n9.layers) == 9
    r52 = synth.residual52()
    assert sum(L.kind == synth.CONV for L in r52.layers) == 52
    assert sum(L.kind == synth.SHORTCUT for L in r52.layers) == 23
    # 9-layer net on a 64x64 input: 64->32->16->8->4->2, stride-1 pool keeps 2
    p = synth.make_params(n9, 1)
    x = synth.make_input(n9, 1, 1, h=64, w=64)
    outs = onet.forward(n9, p, x)
    assert outs[-1].shape == (1, 125, 2, 2)
    assert outs[10].shape == (1, 512, 2, 2)
    sb = synth.single_block()
    outs = onet.forward(sb, synth.make_params(sb, 0), synth.make_input(sb, 1, 0))
    assert outs[-1].shape == (1, 16, 16, 16)


def test_residual_shapes_small_input():
    net = synth.residual52(in_hw=64)
    p = synth.make_params(net, 2)
    x = synth.make_input(net, 1, 2)
    outs = onet.forward(net, p, x)
    assert outs[0].shape == (1, 32, 64, 64)
    assert outs[-1].shape == (1, 1024, 2, 2)


def test_forward_is_layer_by_layer_composition():
    net = synth.plain9()
    p = synth.make_params(net, 1)
    x = synth.make_input(net, 2, 1, h=32, w=32)
    outs = onet.forward(net, p, x)
    cur = x
    for i, L in enumerate(net.layers):
        if L.kind == synth.CONV:
            y = oracle.conv2d(cur, p[i].w, L.stride, L.pad)
            y = oracle.add_bias(y, p[i].bias)
            if L.batchnorm:
                y = oracle.batchnorm(y, p[i].mean, p[i].var, p[i].gamma, p[i].beta, net.bn_eps)
            if L.activation == synth.LEAKY:
                y = oracle.leaky(y, net.leaky_slope)
        else:
            y = oracle.maxpool(cur, L.ksize, L.stride)
        np.testing.assert_array_equal(outs[i], y)
        cur = y


def test_residual_unit_with_zero_branch_is_identity():
    net = synth.residual52(units=(1, 1, 1, 1, 1), in_hw=32)
    p = synth.make_params(net, 2)
    eps = net.bn_eps
    for i, L in enumerate(net.layers):
        if L.kind == synth.SHORTCUT:
            b = i - 1  # conv3x3 "b" of the unit
            q = p[b]
            q.w = np.zeros_like(q.w)
            q.gamma = np.sqrt(q.var + eps)
            q.beta = q.mean - q.bias
    x = synth.make_input(net, 1, 2)
    outs = onet.forward(net, p, x)
    for i, L in enumerate(net.layers):
        if L.kind == synth.SHORTCUT:
            np.testing.assert_allclose(outs[i], outs[L.src], rtol=0, atol=1e-15)
            np.testing.assert_allclose(outs[i - 1], 0.0, atol=1e-15)


def test_residual_shortcut_adds_the_right_tensor():
    net = synth.residual52(units=(2, 1, 1, 1, 1), in_hw=32)
    p = synth.make_params(net, 2)
    x = synth.make_input(net, 1, 2)
    outs = onet.forward(net, p, x)
    for i, L in enumerate(net.layers):
        if L.kind == synth.SHORTCUT:
            np.testing.assert_array_equal(outs[i], outs[i - 1] + outs[L.src])
            assert net.layers[L.src + 1].ksize == 1  # the unit starts with the 1x1 conv
