"""Gradient of a layer's activation energy with respect to the input image, and
the image-ascent step built on it, in FP64.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Beside object detection the paper's workload runs Darknet's image
modification program (Sec. 5.1.1), whose mechanism it does not describe.  The
reading used here is the one that program's family follows: pick a layer L,
take the energy of its output

    E(x) = 1/2 * sum over the batch, channels and pixels of a_L(x)^2,

and move the image up its gradient.  dE/da_L = a_L, and the chain rule runs
back through the layers 0..L one at a time:

* conv layer (conv -> + bias -> BN -> leaky): with z the pre-activation,
  dz = da * (1 if z > 0 else slope); BN multiplies channel k by
  gamma_k / sqrt(var_k + eps), so dconv = dz * that factor; then the conv's
  backward-data (``conv2d_backward_data`` in oracle.c);
* maxpool: each window's gradient goes to its first maximal input
  (``maxpool_backward``);
* shortcut (linear): the gradient goes unchanged to both inputs, and a value
  that feeds several layers sums their gradients.

One ascent step: x' = clip(x + rate * g / mean|g|, 0, 1), mean |g| taken per
image (left unchanged where g is zero).

Pins: tests/test_oracle_backward.py checks every piece against central
finite differences of the forward definitions and the adjoint identity of the
convolution, and the step against its closed form on an identity network.
"""
from __future__ import annotations

from typing import List, Optional

import numpy as np

from synth import CONV, LEAKY, MAXPOOL, SHORTCUT, ConvParams, Net

from . import add_bias, batchnorm, conv2d, conv2d_backward_data, maxpool_backward
from .net import forward


def energy(net: Net, params: List[Optional[ConvParams]], x: np.ndarray, layer: int) -> float:
    """E(x) = 1/2 * sum of squares of layer ``layer``'s output."""
    a = forward(net, params, x, upto=layer + 1)[layer]
    return 0.5 * float(np.sum(a * a))


def input_gradient(net: Net, params: List[Optional[ConvParams]], x: np.ndarray, layer: int) -> np.ndarray:
    """dE/dx for E of layer ``layer``; x [N,C,H,W] -> gradient of the same shape."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    outs = forward(net, params, x, upto=layer + 1)
    ins = [x] + outs[:-1]
    grads: List[Optional[np.ndarray]] = [None] * (layer + 2)  # value v: input (0) or output of layer v-1

    def add(v: int, g: np.ndarray) -> None:
        grads[v] = g if grads[v] is None else grads[v] + g

    grads[layer + 1] = outs[layer].copy()
    for i in range(layer, -1, -1):
        L = net.layers[i]
        gy = grads[i + 1]
        xin = ins[i]
        if L.kind == CONV:
            p = params[i]
            z = add_bias(conv2d(xin, p.w, L.stride, L.pad), p.bias)
            if L.batchnorm:
                z = batchnorm(z, p.mean, p.var, p.gamma, p.beta, net.bn_eps)
            if L.activation == LEAKY:
                gy = gy * np.where(z > 0.0, 1.0, net.leaky_slope)
            if L.batchnorm:
                scale = np.asarray(p.gamma, np.float64) / np.sqrt(np.asarray(p.var, np.float64) + net.bn_eps)
                gy = gy * scale[None, :, None, None]
            add(i, conv2d_backward_data(gy, p.w, L.stride, L.pad, xin.shape[2], xin.shape[3]))
        elif L.kind == MAXPOOL:
            add(i, maxpool_backward(xin, L.ksize, L.stride, gy))
        elif L.kind == SHORTCUT:
            if L.activation == LEAKY:
                gy = gy * np.where(outs[i] > 0.0, 1.0, net.leaky_slope)
            add(i, gy)
            add(L.src + 1, gy)
        else:
            raise ValueError("unknown layer kind %r" % (L.kind,))
    return grads[0]


def ascent_step(x: np.ndarray, g: np.ndarray, rate: float) -> np.ndarray:
    """x' = clip(x + rate * g / mean|g|, 0, 1), mean |g| per image."""
    x = np.asarray(x, np.float64)
    g = np.asarray(g, np.float64)
    m = np.mean(np.abs(g).reshape(g.shape[0], -1), axis=1)
    step = np.where(m > 0, rate / np.where(m > 0, m, 1.0), 0.0)
    return np.clip(x + step[:, None, None, None] * g, 0.0, 1.0)


def nightmare(net: Net, params: List[Optional[ConvParams]], x: np.ndarray, layer: int, rate: float,
              iters: int) -> np.ndarray:
    """``iters`` ascent steps on E of layer ``layer``."""
    x = np.asarray(x, np.float64)
    for _ in range(iters):
        x = ascent_step(x, input_gradient(net, params, x, layer), rate)
    return x
