"""Pins for the oracle's backward pass to the input (CPU only).

The gradient definitions are pinned to things other than themselves:
* the adjoint identity <conv(x), dy> = <x, conv_backward_data(dy)>, which
  holds exactly for the linear map conv (up to FP64 rounding), for every
  stride, padding and ragged size;
* central finite differences of the forward definitions (conv, maxpool and a
  whole network with BN, leaky, pooling, a strided conv and a shortcut);
* hand-worked cases: a constant input whose pooling windows all tie, an
  identity network whose ascent step has a closed form.
Mutants of the C backward functions must fail at least one of these pins.
"""
import os
import subprocess

import numpy as np
import pytest

import oracle
import synth
from oracle import backward as ob

SRC = os.path.join(os.path.dirname(oracle.__file__), "oracle.c")

CONV_CASES = [  # n, c, h, w, k, r, stride, pad
    (2, 3, 7, 6, 4, 3, 1, 1),
    (1, 2, 9, 8, 3, 3, 2, 1),    # stride 2, odd side (the last row of taps is cut)
    (1, 4, 5, 7, 2, 1, 1, 0),    # 1x1
    (2, 2, 6, 6, 3, 2, 1, 0),    # even filter, no pad
    (1, 3, 10, 9, 2, 3, 2, 0),   # stride 2, no pad, ragged
    (1, 1, 4, 4, 1, 3, 1, 2),    # pad = k - 1 (a "full" convolution)
]


@pytest.mark.parametrize("case", CONV_CASES)
def test_conv_backward_is_the_adjoint(case):
    n, c, h, w, k, r, st, pad = case
    rng = np.random.default_rng(list(case))
    x = rng.normal(size=(n, c, h, w))
    wt = rng.normal(size=(k, c, r, r))
    y = oracle.conv2d(x, wt, st, pad)
    dy = rng.normal(size=y.shape)
    dx = oracle.conv2d_backward_data(dy, wt, st, pad, h, w)
    assert dx.shape == x.shape
    lhs, rhs = float(np.sum(y * dy)), float(np.sum(x * dx))
    assert abs(lhs - rhs) <= 1e-12 * max(1.0, abs(lhs))


@pytest.mark.parametrize("case", CONV_CASES[:3])
def test_conv_backward_finite_differences(case):
    n, c, h, w, k, r, st, pad = case
    rng = np.random.default_rng([9] + list(case))
    x = rng.normal(size=(n, c, h, w))
    wt = rng.normal(size=(k, c, r, r))
    dy = rng.normal(size=oracle.conv2d(x, wt, st, pad).shape)
    dx = oracle.conv2d_backward_data(dy, wt, st, pad, h, w)
    f = lambda z: float(np.sum(oracle.conv2d(z, wt, st, pad) * dy))
    for idx in [tuple(rng.integers(0, s) for s in x.shape) for _ in range(12)] + [(0, 0, 0, 0), (n - 1, c - 1, h - 1, w - 1)]:
        e = np.zeros_like(x)
        e[idx] = 1e-3
        num = (f(x + e) - f(x - e)) / 2e-3  # exact for a linear map up to rounding
        assert abs(num - dx[idx]) <= 1e-8 * max(1.0, abs(num)), idx


def test_conv_backward_hand_case():
    # 3x3 all-ones filter, stride 1, pad 1 on a 2x2 map: every output sees every input
    dx = oracle.conv2d_backward_data(np.ones((1, 1, 2, 2)), np.ones((1, 1, 3, 3)), 1, 1, 2, 2)
    np.testing.assert_array_equal(dx[0, 0], np.full((2, 2), 4.0))
    # single tap at (0, 0) with pad 1: y[i][j] = x[i-1][j-1], so dx[p][q] = dy[p+1][q+1]
    t = np.zeros((1, 1, 3, 3)); t[0, 0, 0, 0] = 1.0
    dy = np.arange(9.0).reshape(1, 1, 3, 3)
    dx = oracle.conv2d_backward_data(dy, t, 1, 1, 3, 3)
    np.testing.assert_array_equal(dx[0, 0], [[4, 5, 0], [7, 8, 0], [0, 0, 0]])


@pytest.mark.parametrize("size,stride,h,w", [(2, 2, 6, 8), (2, 2, 7, 5), (2, 1, 5, 6), (3, 2, 7, 7), (3, 1, 4, 5)])
def test_maxpool_backward_finite_differences(size, stride, h, w):
    rng = np.random.default_rng([size, stride, h, w])
    x = rng.permutation(2 * 3 * h * w).reshape(2, 3, h, w) / 7.0  # distinct values: no ties
    y = oracle.maxpool(x, size, stride)
    dy = rng.normal(size=y.shape)
    dx = oracle.maxpool_backward(x, size, stride, dy)
    f = lambda z: float(np.sum(oracle.maxpool(z, size, stride) * dy))
    num = np.zeros_like(x)
    for idx in np.ndindex(*x.shape):
        e = np.zeros_like(x)
        e[idx] = 1e-4  # far below the 1/7 gap between values: the argmax never moves
        num[idx] = (f(x + e) - f(x - e)) / 2e-4
    np.testing.assert_allclose(dx, num, rtol=1e-9, atol=1e-9)
    # the gradient only moves mass: it sums to the output gradient
    assert abs(dx.sum() - dy.sum()) < 1e-9


def test_maxpool_backward_ties_go_to_the_first_element():
    x = np.ones((1, 1, 4, 4))
    dy = np.arange(1.0, 5.0).reshape(1, 1, 2, 2)
    dx = oracle.maxpool_backward(x, 2, 2, dy)[0, 0]
    want = np.zeros((4, 4)); want[0, 0], want[0, 2], want[2, 0], want[2, 2] = 1, 2, 3, 4
    np.testing.assert_array_equal(dx, want)
    # size 2 stride 1: the window at (i, j) starts at (i, j); the last row/column
    # windows reach past the input, and their first in-bounds element wins
    dy = np.ones((1, 1, 4, 4))
    dx = oracle.maxpool_backward(x, 2, 1, dy)[0, 0]
    np.testing.assert_array_equal(dx, np.ones((4, 4)))


def _small_net():
    return synth.Net("bwd_small", 3, 12, 10, [
        synth.conv(8, 3),                      # 0: BN + leaky
        synth.maxpool(2, 2),                   # 1
        synth.conv(16, 3, stride=2),           # 2: strided
        synth.conv(8, 1),                      # 3
        synth.conv(16, 3),                     # 4
        synth.shortcut(2),                     # 5: 4 + 2
        synth.maxpool(2, 1),                   # 6: size 2 stride 1
        synth.conv(5, 1, bn=False, act=synth.LINEAR),  # 7
    ])


@pytest.mark.parametrize("layer", [0, 2, 5, 7])
def test_input_gradient_finite_differences(layer):
    net = _small_net()
    params = synth.make_params(net, 21)
    x = synth.make_input(net, 2, 21)
    g = ob.input_gradient(net, params, x, layer)
    assert g.shape == x.shape
    rng = np.random.default_rng([layer, 4])
    h = 1e-6
    # directional derivatives along random directions, and a few coordinates
    for _ in range(3):
        v = rng.normal(size=x.shape)
        num = (ob.energy(net, params, x + h * v, layer) - ob.energy(net, params, x - h * v, layer)) / (2 * h)
        assert abs(num - float(np.sum(g * v))) <= 1e-5 * max(1.0, abs(num))
    for _ in range(6):
        idx = tuple(int(rng.integers(0, s)) for s in x.shape)
        e = np.zeros_like(x); e[idx] = h
        num = (ob.energy(net, params, x + e, layer) - ob.energy(net, params, x - e, layer)) / (2 * h)
        assert abs(num - g[idx]) <= 1e-5 * max(1.0, abs(num)), idx


def test_ascent_step_identity_net_closed_form():
    # one linear 1x1 conv with identity weights: a_L = x, E = |x|^2 / 2, g = x
    net = synth.Net("ident", 3, 5, 4, [synth.conv(3, 1, bn=False, act=synth.LINEAR)])
    params = [synth.ConvParams(w=np.eye(3).reshape(3, 3, 1, 1), bias=np.zeros(3))]
    x = synth.make_input(net, 2, 3)
    g = ob.input_gradient(net, params, x, 0)
    np.testing.assert_allclose(g, x, rtol=0, atol=1e-15)
    rate = 0.05
    got = ob.nightmare(net, params, x, 0, rate, 1)
    m = np.abs(x).reshape(2, -1).mean(axis=1)[:, None, None, None]
    np.testing.assert_allclose(got, np.clip(x * (1 + rate / m), 0, 1), rtol=1e-15, atol=1e-15)
    # zero gradient leaves the image as it is
    np.testing.assert_array_equal(ob.ascent_step(x, np.zeros_like(x), rate), x)


BWD_MUTANTS = {
    "bwd_pad_sign": ("const int yy = i * stride - pad + u;", "const int yy = i * stride + pad + u;"),
    "bwd_taps_transposed": ("w[(((size_t)ik * c + ic) * r + u) * s + v]", "w[(((size_t)ik * c + ic) * r + v) * s + u]"),
    "bwd_first_column_dropped": ("if (yy < 0 || yy >= h || xx < 0 || xx >= wd)", "if (yy < 0 || yy >= h || xx < 1 || xx >= wd)"),
    "pool_bwd_last_max": ("if (x[q] > m) {", "if (x[q] >= m) {"),
    "pool_bwd_offset": ("const int off = (size - 1) / 2;\n    for (long t = 0; t < (long)n * c * h * w; ++t)",
                        "const int off = size / 2;\n    for (long t = 0; t < (long)n * c * h * w; ++t)"),
}

BWD_PINS = [
    lambda: [test_conv_backward_is_the_adjoint(c) for c in CONV_CASES],
    test_conv_backward_hand_case,
    lambda: test_maxpool_backward_finite_differences(2, 1, 5, 6),
    lambda: test_maxpool_backward_finite_differences(3, 2, 7, 7),
    test_maxpool_backward_ties_go_to_the_first_element,
]


@pytest.mark.parametrize("name", sorted(BWD_MUTANTS))
def test_backward_mutant_is_caught(name, tmp_path):
    old, new = BWD_MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, "mutation anchor not unique: %s" % name
    cfile = tmp_path / "mut.c"
    cfile.write_text(src.replace(old, new))
    lib = str(tmp_path / ("libmut_%s.so" % name))
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99", "-o", lib, str(cfile), "-lm"])
    caught = False
    with oracle.use_library(lib):
        for pin in BWD_PINS:
            try:
                pin()
            except (AssertionError, ValueError, IndexError):
                caught = True
                break
    assert caught, "mutant %s survived every backward pin" % name


def test_round_bf16_hand_values():
    one = 1.0
    vals = [one + 2.0 ** -8, one + 3 * 2.0 ** -8, one + 2.0 ** -9, -(one + 2.0 ** -7), 3.0e-39, 65504.0, 0.1]
    want = [one, one + 2.0 ** -6, one, -(one + 2.0 ** -7), None, 65536.0, 0.10009765625]
    got = ob.round_bf16(np.array(vals))
    for g, w, v in zip(got, want, vals):
        if w is not None:
            assert g == w, (v, g, w)
    # ties to even: 1 + 2^-8 sits halfway between 1 and 1 + 2^-7 -> 1 (even);
    # 1 + 3*2^-8 sits halfway between 1 + 2^-7 and 1 + 2^-6 -> 1 + 2^-6 (even)
    assert ob.round_bf16(np.array([one + 2.0 ** -7]))[0] == one + 2.0 ** -7  # representable: unchanged


def _first_max_pick(x, size, stride):
    """Window decisions of a max pool by the first-maximum rule (row-major
    window order, taps outside the input never win), by brute force."""
    n, c, h, w = x.shape
    ho, wo, off = (h - 1) // stride + 1, (w - 1) // stride + 1, (size - 1) // 2
    pick = np.empty((n, c, ho, wo), np.int64)
    for a in range(n):
        for k in range(c):
            for i in range(ho):
                for j in range(wo):
                    best, arg = -np.inf, -1
                    for u in range(size):
                        for v in range(size):
                            yy, xx = i * stride - off + u, j * stride - off + v
                            if 0 <= yy < h and 0 <= xx < w and x[a, k, yy, xx] > best:
                                best, arg = x[a, k, yy, xx], u * size + v
                    pick[a, k, i, j] = arg
    return pick


def _own_decisions(net, params, x, layer):
    from oracle import net as onet
    outs = onet.forward(net, params, x, upto=layer + 1)
    ins = [x] + outs[:-1]
    passes, picks = {}, {}
    for i in range(layer + 1):
        L = net.layers[i]
        if L.kind == synth.CONV and L.activation == synth.LEAKY:
            passes[i] = outs[i] > 0.0  # a leaky output has its pre-activation's sign
        elif L.kind == synth.MAXPOOL:
            picks[i] = _first_max_pick(ins[i], L.ksize, L.stride)
    return passes, picks


@pytest.mark.parametrize("layer", [2, 5, 7])
def test_gradient_on_the_oracles_own_piece_is_the_plain_gradient(layer):
    net = _small_net()
    params = synth.make_params(net, 22)
    x = synth.make_input(net, 2, 22)
    plain = ob.input_gradient(net, params, x, layer)
    passes, picks = _own_decisions(net, params, x, layer)
    got = ob.input_gradient_on_piece(net, params, x, layer, passes, picks)
    np.testing.assert_allclose(got, plain, rtol=1e-12, atol=1e-13 * np.abs(plain).max())


def _brute_piece_gradient(x, p1, p2, eps, slope, passes, pick):
    """Pure-Python loops on a 1-image net: conv3x3 pad 1 + bias + BN + leaky
    (decisions `passes`), 2x2 stride-1 max pool (decisions `pick`), conv1x1 +
    bias; gradient of 1/2 * sum(out^2) with respect to x on that piece."""
    _, C, H, W = x.shape
    K = p1.w.shape[0]
    K2 = p2.w.shape[0]
    sc = [p1.gamma[k] / np.sqrt(p1.var[k] + eps) for k in range(K)]
    a1 = [[[0.0] * W for _ in range(H)] for _ in range(K)]
    for k in range(K):
        for i in range(H):
            for j in range(W):
                z = 0.0
                for c in range(C):
                    for r in range(3):
                        for t in range(3):
                            yy, xx = i - 1 + r, j - 1 + t
                            if 0 <= yy < H and 0 <= xx < W:
                                z += p1.w[k, c, r, t] * x[0, c, yy, xx]
                z = (z + p1.bias[k] - p1.mean[k]) * sc[k] + p1.beta[k]
                a1[k][i][j] = z if z > 0 else slope * z
    y = [[[max(a1[k][i + u][j + v] for u in range(2) for v in range(2) if i + u < H and j + v < W)
           for j in range(W)] for i in range(H)] for k in range(K)]
    out = [[[sum(p2.w[m, k, 0, 0] * y[k][i][j] for k in range(K)) + p2.bias[m] for j in range(W)]
            for i in range(H)] for m in range(K2)]
    gy = [[[sum(p2.w[m, k, 0, 0] * out[m][i][j] for m in range(K2)) for j in range(W)] for i in range(H)]
          for k in range(K)]
    ga = [[[0.0] * W for _ in range(H)] for _ in range(K)]
    for k in range(K):
        for i in range(H):
            for j in range(W):
                u, v = divmod(int(pick[0, k, i, j]), 2)
                ga[k][i + u][j + v] += gy[k][i][j]
    gx = np.zeros(x.shape)
    for k in range(K):
        for i in range(H):
            for j in range(W):
                gz = ga[k][i][j] * (1.0 if passes[0, k, i, j] else slope) * sc[k]
                for c in range(C):
                    for r in range(3):
                        for t in range(3):
                            yy, xx = i - 1 + r, j - 1 + t
                            if 0 <= yy < H and 0 <= xx < W:
                                gx[0, c, yy, xx] += gz * p1.w[k, c, r, t]
    return gx


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_gradient_on_a_given_piece_matches_brute_force(seed):
    net = synth.Net("piece", 2, 5, 4, [synth.conv(3, 3), synth.maxpool(2, 1),
                                        synth.conv(2, 1, bn=False, act=synth.LINEAR)])
    params = synth.make_params(net, 60 + seed)
    x = synth.make_input(net, 1, 60 + seed)
    passes, picks = _own_decisions(net, params, x, 2)
    rng = np.random.default_rng([61, seed])
    # flip a third of the leaky decisions and re-pick a third of the windows
    # (any tap inside the input): a piece the oracle would not take itself
    flip = rng.random(passes[0].shape) < 1 / 3
    passes[0] = np.where(flip, ~passes[0], passes[0])
    pick = picks[1].copy()
    H, W = 5, 4
    for idx in zip(*np.nonzero(rng.random(pick.shape) < 1 / 3)):
        _, _, i, j = idx
        valid = [u * 2 + v for u in range(2) for v in range(2) if i + u < H and j + v < W]
        pick[idx] = valid[rng.integers(len(valid))]
    picks[1] = pick
    got = ob.input_gradient_on_piece(net, params, x, 2, passes, picks)
    want = _brute_piece_gradient(x, params[0], params[2], net.bn_eps, net.leaky_slope, passes[0], picks[1])
    np.testing.assert_allclose(got, want, rtol=1e-11, atol=1e-13 * np.abs(want).max())
    # the piece matters: the oracle's own piece gives another gradient
    assert np.abs(ob.input_gradient(net, params, x, 2) - got).max() > 1e-6 * np.abs(got).max()


def test_picked_pool_gradient_rejects_taps_outside_the_input():
    dy = np.ones((1, 1, 2, 2))
    pick = np.zeros((1, 1, 2, 2), np.int64)
    pick[0, 0, 1, 1] = 3  # window at the bottom-right corner of a 2x2 input, stride 1: tap (2, 2) is outside
    with pytest.raises(ValueError):
        ob.maxpool_backward_picked((1, 1, 2, 2), 2, 1, pick, dy)
    pick[0, 0, 1, 1] = 0
    got = ob.maxpool_backward_picked((1, 1, 2, 2), 2, 1, pick, dy)
    np.testing.assert_array_equal(got[0, 0], [[1.0, 1.0], [1.0, 1.0]])
