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

``input_gradient_stored`` is the same gradient for the BF16 path's
definition (stored operands rounded to BF16), so that every branch is taken
on the same stored values as on the device.

Pins: tests/test_oracle_backward.py checks every piece against central
finite differences of the forward definitions and the adjoint identity of the
convolution, the step against its closed form on an identity network, the
stored-operand variant against the plain one when nothing is rounded, and the
BF16 rounding against hand-worked values.
"""
from __future__ import annotations

from typing import List, Optional

import numpy as np

from synth import CONV, LEAKY, MAXPOOL, SHORTCUT, ConvParams, Net

from . import add_bias, batchnorm, conv2d, conv2d_backward_data, maxpool, maxpool_backward
from .net import forward


def round_bf16(a) -> np.ndarray:
    """Round to the nearest bfloat16 (ties to even), returned as FP64: the
    8-bit-significand storage format of the BF16 path."""
    f = np.asarray(a, np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16 << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def round_f32(a) -> np.ndarray:
    return np.asarray(a, np.float64).astype(np.float32).astype(np.float64)


def _forward_stored(net: Net, params, x: np.ndarray, layer: int, q, qb):
    """Forward up to ``layer`` with every stored operand in a storage format:
    the input image, the BN-folded weights (fold in FP64, then q) and every
    layer output pass through q; the folded bias through qb; arithmetic is FP64.
    Returns (layer inputs, layer outputs, stored weights)."""
    cur = q(x)
    ins, outs, wq = [], [], {}
    for i in range(layer + 1):
        L = net.layers[i]
        ins.append(cur)
        if L.kind == CONV:
            p = params[i]
            w = np.asarray(p.w, np.float64)
            b = np.asarray(p.bias, np.float64)
            if L.batchnorm:
                sc = np.asarray(p.gamma, np.float64) / np.sqrt(np.asarray(p.var, np.float64) + net.bn_eps)
                w = w * sc[:, None, None, None]
                b = (b - np.asarray(p.mean, np.float64)) * sc + np.asarray(p.beta, np.float64)
            wq[i] = q(w)
            z = add_bias(conv2d(cur, wq[i], L.stride, L.pad), qb(b))
            if L.activation == LEAKY:
                z = np.where(z > 0.0, z, z * net.leaky_slope)
            cur = q(z)
        elif L.kind == MAXPOOL:
            cur = maxpool(cur, L.ksize, L.stride)
        elif L.kind == SHORTCUT:
            cur = q(outs[i - 1] + outs[L.src])
        else:
            raise ValueError("unknown layer kind %r" % (L.kind,))
        outs.append(cur)
    return ins, outs, wq


def input_gradient_stored(net: Net, params, x: np.ndarray, layer: int, q=round_bf16, qb=round_f32) -> np.ndarray:
    """dE/dx of the network whose stored operands are in the format q (the
    BF16 path's definition: BF16 image, folded weights and activations, FP32
    bias).  Every branch (leaky sign, first maximum of a pooling window) is
    taken on the stored activations, as the device takes it; the gradient
    arithmetic is FP64 with the stored weights."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    ins, outs, wq = _forward_stored(net, params, x, layer, q, qb)
    grads: List[Optional[np.ndarray]] = [None] * (layer + 2)

    def add(v: int, g: np.ndarray) -> None:
        grads[v] = g if grads[v] is None else grads[v] + g

    grads[layer + 1] = outs[layer].copy()
    for i in range(layer, -1, -1):
        L = net.layers[i]
        gy = grads[i + 1]
        if L.kind == CONV:
            if L.activation == LEAKY:
                gy = gy * np.where(outs[i] > 0.0, 1.0, net.leaky_slope)
            add(i, conv2d_backward_data(gy, wq[i], L.stride, L.pad, ins[i].shape[2], ins[i].shape[3]))
        elif L.kind == MAXPOOL:
            add(i, maxpool_backward(ins[i], L.ksize, L.stride, gy))
        else:
            add(i, gy)
            add(L.src + 1, gy)
    return grads[0]


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
