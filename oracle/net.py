"""Whole-network FP64 forward built from the oracle's per-layer definitions.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Layer semantics follow the Darknet layer vocabulary the paper's workload uses
(Sec. 5.1.1):

* convolution layer: conv2d -> + bias -> [batchnorm] -> activation
  (bias is added before batch normalisation when both are present; this is
  a reading, the paper gives no formula);
* maxpool layer: window ``ksize``, stride ``stride``, -inf outside the input;
* shortcut layer: output of the previous layer + output of layer ``src``,
  then its own activation (linear for every network used here).

``forward`` returns every layer's output so that tests can gate layer by
layer as well as end to end.
"""
from __future__ import annotations

from typing import List, Optional

import numpy as np

from synth import CONV, LEAKY, MAXPOOL, SHORTCUT, ConvParams, Layer, Net

from . import add_bias, batchnorm, conv2d, leaky, maxpool, shortcut


def conv_layer(x: np.ndarray, L: Layer, p: ConvParams, slope: float, eps: float) -> np.ndarray:
    y = conv2d(x, p.w, L.stride, L.pad)
    y = add_bias(y, p.bias)
    if L.batchnorm:
        y = batchnorm(y, p.mean, p.var, p.gamma, p.beta, eps)
    if L.activation == LEAKY:
        y = leaky(y, slope)
    return y


def run_layer(i: int, x: np.ndarray, outs: List[np.ndarray], net: Net,
              params: List[Optional[ConvParams]]) -> np.ndarray:
    L = net.layers[i]
    if L.kind == CONV:
        return conv_layer(x, L, params[i], net.leaky_slope, net.bn_eps)
    if L.kind == MAXPOOL:
        return maxpool(x, L.ksize, L.stride)
    if L.kind == SHORTCUT:
        y = shortcut(x, outs[L.src])
        if L.activation == LEAKY:
            y = leaky(y, net.leaky_slope)
        return y
    raise ValueError("unknown layer kind %r" % (L.kind,))


def forward(net: Net, params: List[Optional[ConvParams]], x: np.ndarray,
            upto: Optional[int] = None) -> List[np.ndarray]:
    """Run layers 0..upto-1 (all by default) on x [N,C,H,W]; return each output."""
    outs: List[np.ndarray] = []
    cur = np.ascontiguousarray(x, dtype=np.float64)
    n = len(net.layers) if upto is None else upto
    for i in range(n):
        cur = run_layer(i, cur, outs, net, params)
        outs.append(cur)
    return outs
