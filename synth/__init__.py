"""Seeded synthetic workloads shared by the oracle side and the GPU side.

This module only describes networks and draws random numbers; it holds none
of the forward pass's arithmetic.  Both the FP64 oracle and the HIP library
consume exactly the arrays produced here (the library receives them as FP64
host arrays and does its own folding, rounding and packing).

Networks (the paper's workload is Darknet's detection and image-edit sample
programs, Sec. 5.1.1; their network files are not given, so these synthetic
networks of the same layer vocabulary stand in for them):

* ``single_block``: conv3x3(16)+BN+leaky, maxpool 2/2 on 3x32x32.
* ``plain9``: six conv3x3+BN+leaky blocks of widths 16..512, each followed by a
  2x2 maxpool (stride 2, the last stride 1), conv3x3 to 1024 twice, then a
  linear 1x1 conv to 125 (bias only).  Input 3x416x416.
* ``residual52``: stem conv3x3 to 32, then five stages (C = 64..1024), each a
  stride-2 conv3x3 followed by 1, 2, 8, 8, 4 residual units
  (conv1x1 to C/2, conv3x3 back to C, shortcut add).  52 convolutions.
  Input 3x256x256.

Random draws (readings of the stated distributions; N(a, b) takes b as the
variance, which is what makes N(0, 2/fan_in) the He initialisation):

* weights  N(0, 2/fan_in), fan_in = Cin*R*S
* bias     N(0, 0.01)
* BN mean  N(0, 0.1), var U[0.5, 1.5), gamma U[0.9, 1.1), beta N(0, 0.05)
* input    U[0, 1)

Parameters come from ``numpy.random.default_rng([seed, 0])`` drawn per conv
layer in the order w, bias, mean, var, gamma, beta (the last four only when
the layer has batch normalisation).  Inputs come from a separate stream
``default_rng([seed, 1, tag])`` so that one network can be fed batches of any
size with unchanged weights.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

CONV, MAXPOOL, SHORTCUT = 0, 1, 2
LINEAR, LEAKY = 0, 1


@dataclass(frozen=True)
class Layer:
    kind: int
    cout: int = 0
    ksize: int = 0
    stride: int = 1
    pad: int = 0
    batchnorm: bool = False
    activation: int = LINEAR
    src: int = -1  # shortcut: absolute index of the earlier layer whose output is added


def conv(cout: int, k: int, stride: int = 1, bn: bool = True, act: int = LEAKY) -> Layer:
    return Layer(CONV, cout=cout, ksize=k, stride=stride, pad=k // 2, batchnorm=bn, activation=act)


def maxpool(size: int = 2, stride: int = 2) -> Layer:
    return Layer(MAXPOOL, ksize=size, stride=stride)


def shortcut(src: int) -> Layer:
    return Layer(SHORTCUT, src=src, activation=LINEAR)


@dataclass
class Net:
    name: str
    in_c: int
    in_h: int
    in_w: int
    layers: List[Layer]
    leaky_slope: float = 0.1
    bn_eps: float = 1e-5


def single_block() -> Net:
    return Net("single_block", 3, 32, 32, [conv(16, 3), maxpool(2, 2)])


def plain9() -> Net:
    layers: List[Layer] = []
    widths = (16, 32, 64, 128, 256, 512)
    for i, c in enumerate(widths):
        layers.append(conv(c, 3))
        layers.append(maxpool(2, 1 if i == len(widths) - 1 else 2))
    layers += [conv(1024, 3), conv(1024, 3), conv(125, 1, bn=False, act=LINEAR)]
    return Net("plain9", 3, 416, 416, layers)


def residual52(units=(1, 2, 8, 8, 4), widths=(64, 128, 256, 512, 1024), in_hw: int = 256) -> Net:
    layers: List[Layer] = [conv(32, 3)]
    for c, nu in zip(widths, units):
        layers.append(conv(c, 3, stride=2))
        for _ in range(nu):
            unit_in = len(layers) - 1
            layers.append(conv(c // 2, 1))
            layers.append(conv(c, 3))
            layers.append(shortcut(unit_in))
    return Net("residual52", 3, in_hw, in_hw, layers)


NETS = {"single_block": single_block, "plain9": plain9, "residual52": residual52}


def conv_in_channels(net: Net) -> List[int]:
    """Input channel count seen by each layer (structure only: convs set C,
    pooling and residual adds keep it)."""
    chans, c = [], net.in_c
    for L in net.layers:
        chans.append(c)
        if L.kind == CONV:
            c = L.cout
    return chans


@dataclass
class ConvParams:
    w: np.ndarray                    # [K][C][R][S] float64
    bias: np.ndarray                 # [K]
    mean: Optional[np.ndarray] = None
    var: Optional[np.ndarray] = None
    gamma: Optional[np.ndarray] = None
    beta: Optional[np.ndarray] = None


def make_params(net: Net, seed: int) -> List[Optional[ConvParams]]:
    rng = np.random.default_rng([seed, 0])
    out: List[Optional[ConvParams]] = []
    for L, cin in zip(net.layers, conv_in_channels(net)):
        if L.kind != CONV:
            out.append(None)
            continue
        fan_in = cin * L.ksize * L.ksize
        w = rng.normal(0.0, np.sqrt(2.0 / fan_in), size=(L.cout, cin, L.ksize, L.ksize))
        b = rng.normal(0.0, np.sqrt(0.01), size=L.cout)
        p = ConvParams(w=w, bias=b)
        if L.batchnorm:
            p.mean = rng.normal(0.0, np.sqrt(0.1), size=L.cout)
            p.var = rng.uniform(0.5, 1.5, size=L.cout)
            p.gamma = rng.uniform(0.9, 1.1, size=L.cout)
            p.beta = rng.normal(0.0, np.sqrt(0.05), size=L.cout)
        out.append(p)
    return out


def make_input(net: Net, batch: int, seed: int, tag: int = 0,
               h: Optional[int] = None, w: Optional[int] = None) -> np.ndarray:
    rng = np.random.default_rng([seed, 1, tag])
    return rng.uniform(0.0, 1.0, size=(batch, net.in_c, h or net.in_h, w or net.in_w))


def make_tensor(shape, seed: int, tag: int, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    """Generic seeded uniform tensor for single-layer tests."""
    rng = np.random.default_rng([seed, 2, tag])
    return rng.uniform(lo, hi, size=shape)


# Seeds used throughout (a stated choice; the distributions above fix the rest).
SEED_SINGLE, SEED_PLAIN, SEED_RESIDUAL, SEED_SERVING, SEED_CALIB = 0, 1, 2, 3, 4
SEED_DETECT = 5


@dataclass
class ServingTrace:
    arrival_s: np.ndarray   # [R] seconds since start, nondecreasing
    size: np.ndarray        # [R] square side S of each request
    sizes: tuple = field(default=(160, 224, 320, 416, 608))


def serving_trace(n_requests: int = 10000, rate: float = 2000.0, seed: int = SEED_SERVING,
                  sizes=(160, 224, 320, 416, 608)) -> ServingTrace:
    """Poisson arrivals (exponential gaps of mean 1/rate), side uniform over ``sizes``."""
    rng = np.random.default_rng([seed, 3])
    gaps = rng.exponential(1.0 / rate, size=n_requests)
    side = rng.choice(np.asarray(sizes), size=n_requests)
    return ServingTrace(arrival_s=np.cumsum(gaps), size=side, sizes=tuple(sizes))


def serving_image(i: int, side: int, seed: int = SEED_SERVING, in_c: int = 3) -> np.ndarray:
    rng = np.random.default_rng([seed, 4, i])
    return rng.uniform(0.0, 1.0, size=(1, in_c, side, side))


def region_anchors(anchors: int, seed: int = SEED_DETECT) -> np.ndarray:
    """Anchor (w, h) pairs in grid cells, uniform over [0.5, 12), rng [seed, 6]."""
    return np.random.default_rng([seed, 6]).uniform(0.5, 12.0, 2 * anchors)


def region_output(n: int, anchors: int, classes: int, h: int, w: int, seed: int = SEED_DETECT,
                  tag: int = 0, clusters: int = 0) -> np.ndarray:
    """A synthetic region-head output [n, anchors*(5+classes), h, w] FP32, rng
    [seed, 7, tag]: tx, ty ~ N(0, 1), tw, th ~ N(0, 0.5), to ~ N(-1, 2), class
    logits ~ N(0, 2).  With clusters > 0, that many cells per image get a
    confident object (to = 4, one class logit + 6) in every anchor, and their
    neighbours repeat it, so that many overlapping boxes compete in NMS."""
    rng = np.random.default_rng([seed, 7, tag])
    y = np.empty((n, anchors, 5 + classes, h, w), np.float32)
    y[:, :, 0:2] = rng.normal(0.0, 1.0, (n, anchors, 2, h, w))
    y[:, :, 2:4] = rng.normal(0.0, 0.5, (n, anchors, 2, h, w))
    y[:, :, 4] = rng.normal(-1.0, 2.0, (n, anchors, h, w))
    y[:, :, 5:] = rng.normal(0.0, 2.0, (n, anchors, classes, h, w))
    for i in range(n):
        for _ in range(clusters):
            ci, cj, k = rng.integers(0, h), rng.integers(0, w), rng.integers(0, classes)
            for di in (-1, 0, 1):
                for dj in (-1, 0, 1):
                    ii, jj = ci + di, cj + dj
                    if 0 <= ii < h and 0 <= jj < w:
                        y[i, :, 4, ii, jj] = 4.0 - abs(di) - abs(dj)
                        y[i, :, 5 + k, ii, jj] += 6.0
    return y.reshape(n, anchors * (5 + classes), h, w)
