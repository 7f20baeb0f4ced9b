"""Pins for the FP64 oracle: brute force, closed forms, invariants, library
cross-checks and hand-worked golden fixtures.  CPU only.

Each pin is chosen so that a plausible slip in the oracle (a dropped term, a
wrong sign, a swapped index or operand, an off-by-one in padding or output
size) fails at least one of them; ``test_oracle_mutants.py`` plants such slips
in a copy of the oracle and checks that they are caught.
"""
import os

import numpy as np
import pytest

import oracle
from tests import bruteforce

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden_blocks(name):
    blocks, cur = {}, None
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            if line.startswith("["):
                cur = line.strip("[]")
                blocks[cur] = []
            else:
                blocks[cur].append([float(v) for v in line.split()])
    return {k: np.array(v) for k, v in blocks.items()}


def _x4():
    return (np.arange(16, dtype=np.float64) + 1).reshape(1, 1, 4, 4)


# ---------------------------------------------------------------- golden


def test_golden_conv_and_pool():
    g = _golden_blocks("conv_pool_4x4.txt")
    x = _x4()
    box = np.ones((1, 1, 3, 3))
    np.testing.assert_array_equal(oracle.conv2d(x, box, 1, 1)[0, 0], g["box3x3_s1_p1"])
    np.testing.assert_array_equal(oracle.conv2d(x, box, 2, 1)[0, 0], g["box3x3_s2_p1"])
    t00 = np.zeros((1, 1, 3, 3)); t00[0, 0, 0, 0] = 1
    t12 = np.zeros((1, 1, 3, 3)); t12[0, 0, 1, 2] = 1
    np.testing.assert_array_equal(oracle.conv2d(x, t00, 1, 1)[0, 0], g["tap00_s1_p1"])
    np.testing.assert_array_equal(oracle.conv2d(x, t12, 1, 1)[0, 0], g["tap12_s1_p1"])
    np.testing.assert_array_equal(oracle.maxpool(x, 2, 2)[0, 0], g["maxpool_k2_s2"])
    np.testing.assert_array_equal(oracle.maxpool(x, 2, 1)[0, 0], g["maxpool_k2_s1"])


def test_golden_bn_leaky():
    rows = np.loadtxt(os.path.join(GOLDEN, "bn_leaky.txt"), comments="#")
    for conv_out, b, mu, var, eps, g, be, slope, want in rows:
        y = np.full((1, 1, 1, 1), conv_out)
        y = oracle.add_bias(y, [b])
        y = oracle.batchnorm(y, [mu], [var], [g], [be], eps)
        y = oracle.leaky(y, slope)
        assert y[0, 0, 0, 0] == pytest.approx(want, rel=0, abs=1e-15)


# ---------------------------------------------------------------- conv


@pytest.mark.parametrize("n,c,h,w,k,r,stride,pad", [
    (1, 1, 5, 5, 1, 3, 1, 1), (2, 3, 6, 7, 4, 3, 1, 1), (1, 4, 7, 6, 2, 3, 2, 1),
    (2, 2, 5, 4, 3, 1, 1, 0), (1, 3, 7, 7, 2, 1, 2, 0), (1, 2, 6, 6, 3, 3, 1, 0),
    (2, 3, 4, 5, 2, 3, 2, 0),
])
def test_conv_bruteforce_integer_exact(n, c, h, w, k, r, stride, pad):
    rng = np.random.default_rng([11, n, c, h, w, k, r, stride, pad])
    x = rng.integers(-4, 5, size=(n, c, h, w)).astype(np.float64)
    wt = rng.integers(-3, 4, size=(k, c, r, r)).astype(np.float64)
    got = oracle.conv2d(x, wt, stride, pad)
    want = np.array(bruteforce.conv2d(x.tolist(), wt.tolist(), stride, pad))
    assert got.shape == want.shape
    np.testing.assert_array_equal(got, want)


def test_conv_1x1_identity_exact():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((2, 5, 6, 7))
    w = np.eye(5).reshape(5, 5, 1, 1)
    np.testing.assert_array_equal(oracle.conv2d(x, w, 1, 0), x)


def test_conv_3x3_dirac_identity_and_shift():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((1, 3, 6, 5))
    w = np.zeros((3, 3, 3, 3))
    for c in range(3):
        w[c, c, 1, 1] = 1.0
    np.testing.assert_array_equal(oracle.conv2d(x, w, 1, 1), x)
    # tap (2,0): y[i,j] = x[i+1, j-1], zero fill outside
    w = np.zeros((3, 3, 3, 3))
    for c in range(3):
        w[c, c, 2, 0] = 1.0
    want = np.zeros_like(x)
    want[:, :, :-1, 1:] = x[:, :, 1:, :-1]
    np.testing.assert_array_equal(oracle.conv2d(x, w, 1, 1), want)


def test_conv_channel_permutation_picks_right_input():
    # w[k, c] = 1 iff c == perm[k]  ->  y[k] = x[perm[k]]; catches swapped k/c indexing
    rng = np.random.default_rng(3)
    x = rng.standard_normal((1, 4, 3, 3))
    perm = [2, 0, 3, 1, 1, 2]
    w = np.zeros((6, 4, 1, 1))
    for k, c in enumerate(perm):
        w[k, c, 0, 0] = 1.0
    np.testing.assert_array_equal(oracle.conv2d(x, w, 1, 0), x[:, perm])


def test_conv_1x1_equals_matmul():
    rng = np.random.default_rng(4)
    x = rng.standard_normal((3, 6, 4, 5))
    w = rng.standard_normal((7, 6, 1, 1))
    want = np.einsum("kc,nchw->nkhw", w[:, :, 0, 0], x)
    np.testing.assert_allclose(oracle.conv2d(x, w, 1, 0), want, rtol=1e-13, atol=1e-13)


def test_conv_matches_torch_float64():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(5)
    for (c, h, w, k, r, st, p) in [(3, 17, 13, 8, 3, 1, 1), (8, 16, 16, 5, 3, 2, 1),
                                   (6, 9, 9, 4, 1, 1, 0), (4, 10, 11, 3, 3, 2, 0)]:
        x = rng.standard_normal((2, c, h, w))
        wt = rng.standard_normal((k, c, r, r))
        want = torch.nn.functional.conv2d(torch.from_numpy(x), torch.from_numpy(wt),
                                          stride=st, padding=p).numpy()
        np.testing.assert_allclose(oracle.conv2d(x, wt, st, p), want, rtol=1e-12, atol=1e-12)


def test_conv_linearity():
    rng = np.random.default_rng(6)
    x1, x2 = rng.standard_normal((2, 1, 3, 8, 8))
    w = rng.standard_normal((4, 3, 3, 3))
    a, b = 0.75, -2.5
    lhs = oracle.conv2d(a * x1 + b * x2, w, 1, 1)
    rhs = a * oracle.conv2d(x1, w, 1, 1) + b * oracle.conv2d(x2, w, 1, 1)
    np.testing.assert_allclose(lhs, rhs, rtol=1e-12, atol=1e-12)


def test_conv_output_sizes():
    x = np.zeros((1, 1, 416, 416))
    assert oracle.conv2d(x, np.zeros((1, 1, 3, 3)), 1, 1).shape == (1, 1, 416, 416)
    x = np.zeros((1, 1, 256, 256))
    assert oracle.conv2d(x, np.zeros((1, 1, 3, 3)), 2, 1).shape == (1, 1, 128, 128)
    x = np.zeros((1, 1, 13, 13))
    assert oracle.conv2d(x, np.zeros((1, 1, 1, 1)), 1, 0).shape == (1, 1, 13, 13)


# ---------------------------------------------------------------- bias / BN / leaky


def test_bn_identity_closed_form():
    rng = np.random.default_rng(7)
    y = rng.standard_normal((2, 4, 3, 3))
    mean = rng.standard_normal(4)
    var = rng.uniform(0.5, 1.5, 4)
    eps = 1e-5
    z = oracle.batchnorm(y, mean, var, np.sqrt(var + eps), mean, eps)
    np.testing.assert_allclose(z, y, rtol=1e-14, atol=1e-14)


def test_bias_bn_constant_input_closed_form():
    # x == c everywhere, 3x3 kernel, pad 1: interior conv output = c * sum(w[k]).
    c0, eps = 0.5, 1e-5
    rng = np.random.default_rng(8)
    w = rng.standard_normal((3, 2, 3, 3))
    b, mu = rng.standard_normal(3), rng.standard_normal(3)
    var, g, be = rng.uniform(0.5, 1.5, 3), rng.uniform(0.9, 1.1, 3), rng.standard_normal(3)
    x = np.full((1, 2, 5, 5), c0)
    y = oracle.conv2d(x, w, 1, 1)
    y = oracle.batchnorm(oracle.add_bias(y, b), mu, var, g, be, eps)
    interior = y[0, :, 2, 2]
    want = g * (c0 * w.reshape(3, -1).sum(1) + b - mu) / np.sqrt(var + eps) + be
    np.testing.assert_allclose(interior, want, rtol=1e-13)
    # bias is per output channel, added before the normalisation
    assert not np.allclose(interior, g * (c0 * w.reshape(3, -1).sum(1) - mu) / np.sqrt(var + eps) + be + b)


def test_bn_fold_equivalence():
    # conv(x, w') + b' equals BN(conv(x, w) + b) when w', b' are the fold.
    rng = np.random.default_rng(9)
    x = rng.standard_normal((2, 3, 7, 7))
    w = rng.standard_normal((4, 3, 3, 3))
    b, mu = rng.standard_normal(4), rng.standard_normal(4)
    var, g, be = rng.uniform(0.5, 1.5, 4), rng.uniform(0.9, 1.1, 4), rng.standard_normal(4)
    eps = 1e-5
    ref = oracle.batchnorm(oracle.add_bias(oracle.conv2d(x, w, 1, 1), b), mu, var, g, be, eps)
    sc = g / np.sqrt(var + eps)
    folded = oracle.add_bias(oracle.conv2d(x, w * sc[:, None, None, None], 1, 1), (b - mu) * sc + be)
    np.testing.assert_allclose(folded, ref, rtol=1e-12, atol=1e-12)


def test_leaky_sign_and_homogeneity():
    z = np.array([-3.0, -0.5, 0.0, 0.25, 7.0]).reshape(1, 1, 1, 5)
    np.testing.assert_array_equal(oracle.leaky(z, 0.1), np.where(z > 0, z, 0.1 * z))
    y = oracle.leaky(z, 0.1)
    assert y[0, 0, 0, 0] == pytest.approx(-0.3)
    assert y[0, 0, 0, 2] == 0.0
    a = 3.5
    np.testing.assert_allclose(oracle.leaky(a * z, 0.1), a * oracle.leaky(z, 0.1), rtol=1e-15)


# ---------------------------------------------------------------- maxpool


@pytest.mark.parametrize("h,w,size,stride", [(4, 4, 2, 2), (5, 7, 2, 2), (13, 13, 2, 1),
                                             (6, 5, 2, 1), (7, 7, 3, 2), (5, 6, 3, 1)])
def test_maxpool_bruteforce(h, w, size, stride):
    rng = np.random.default_rng([12, h, w, size, stride])
    x = rng.standard_normal((2, 3, h, w))
    want = np.array(bruteforce.maxpool(x.tolist(), size, stride))
    np.testing.assert_array_equal(oracle.maxpool(x, size, stride), want)


def test_maxpool_invariants():
    rng = np.random.default_rng(13)
    x = rng.standard_normal((2, 3, 8, 8))
    y = oracle.maxpool(x, 2, 2)
    for i in range(4):
        for j in range(4):
            win = x[:, :, 2 * i:2 * i + 2, 2 * j:2 * j + 2].reshape(2, 3, 4)
            assert np.all(y[:, :, i, j] >= win.max(-1))
            assert np.all((win == y[:, :, i, j][..., None]).any(-1))
    np.testing.assert_array_equal(oracle.maxpool(np.full((1, 1, 6, 6), 2.5), 2, 2), np.full((1, 1, 3, 3), 2.5))
    np.testing.assert_array_equal(oracle.maxpool(x + 4.0, 2, 2), y + 4.0)


def test_maxpool_commutes_with_monotone_maps():
    rng = np.random.default_rng(14)
    x = rng.standard_normal((1, 4, 13, 13))
    for s in (1, 2):
        np.testing.assert_array_equal(oracle.maxpool(oracle.leaky(x, 0.1), 2, s),
                                      oracle.leaky(oracle.maxpool(x, 2, s), 0.1))
        np.testing.assert_array_equal(oracle.maxpool(3.0 * x + 1.0, 2, s),
                                      3.0 * oracle.maxpool(x, 2, s) + 1.0)


def test_maxpool_ramp_picks_bottom_right_and_stride1_edges():
    x = np.arange(13 * 13, dtype=np.float64).reshape(1, 1, 13, 13)
    y2 = oracle.maxpool(x[:, :, :12, :12], 2, 2)
    np.testing.assert_array_equal(y2, x[:, :, 1:12:2, 1:12:2])
    y1 = oracle.maxpool(x, 2, 1)
    assert y1.shape == (1, 1, 13, 13)
    np.testing.assert_array_equal(y1[:, :, :12, :12], x[:, :, 1:, 1:])
    np.testing.assert_array_equal(y1[:, :, 12, :12], x[:, :, 12, 1:])
    np.testing.assert_array_equal(y1[:, :, :12, 12], x[:, :, 1:, 12])
    assert y1[0, 0, 12, 12] == x[0, 0, 12, 12]


def test_maxpool_matches_torch_with_neg_inf_pad():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(15)
    x = rng.standard_normal((2, 3, 13, 13))
    for s in (1, 2):
        xp = np.pad(x, ((0, 0), (0, 0), (0, 1), (0, 1)), constant_values=-np.inf)
        want = torch.nn.functional.max_pool2d(torch.from_numpy(xp), 2, s).numpy()
        np.testing.assert_array_equal(oracle.maxpool(x, 2, s), want)


# ---------------------------------------------------------------- shortcut


def test_shortcut_integer_exact_and_shape_check():
    rng = np.random.default_rng(16)
    a = rng.integers(-100, 100, size=(2, 3, 4, 4)).astype(np.float64)
    b = rng.integers(-100, 100, size=(2, 3, 4, 4)).astype(np.float64)
    np.testing.assert_array_equal(oracle.shortcut(a, b), a + b)
    with pytest.raises(ValueError):
        oracle.shortcut(a, b[:, :2])
