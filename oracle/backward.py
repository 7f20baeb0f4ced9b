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

``input_gradient_on_piece`` is the gradient with the branch decisions (leaky
signs, pooling window choices) given by the caller: the gradient of the
piece of the piecewise-linear pass that those decisions select.  The device
comparison takes the decisions the device took, after checking that each one
that differs from this oracle's own lies within the forward error of its
threshold.

Pins: tests/test_oracle_backward.py checks every piece against central
finite differences of the forward definitions and the adjoint identity of the
convolution, the step against its closed form on an identity network, the
BF16 rounding against hand-worked values, and the given-decision gradient
against ``input_gradient`` when the decisions are the oracle's own and
against pure-Python brute force on tiny nets with decisions flipped.
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


def maxpool_backward_picked(shape, size: int, stride: int, pick: np.ndarray, dy: np.ndarray) -> np.ndarray:
    """Max-pool gradient with the window decisions given: the gradient of output
    (n, c, i, j) goes to window element pick[n, c, i, j] = u*size + v, i.e. input
    (i*stride - o + u, j*stride - o + v) with o = (size - 1)//2 (the window of
    ``maxpool``).  A pick outside the input is an error."""
    n, c, h, w = shape
    pick = np.asarray(pick)
    dy = np.asarray(dy, np.float64)
    if pick.shape != dy.shape:
        raise ValueError("pick shape %s != gradient shape %s" % (pick.shape, dy.shape))
    off = (size - 1) // 2
    dx = np.zeros(shape, np.float64)
    for u in range(size):
        for v in range(size):
            nn, cc, i, j = np.nonzero(pick == u * size + v)
            yy = i * stride - off + u
            xx = j * stride - off + v
            if np.any((yy < 0) | (yy >= h) | (xx < 0) | (xx >= w)):
                raise ValueError("a window's gradient was given to a tap outside the input")
            np.add.at(dx, (nn, cc, yy, xx), dy[nn, cc, i, j])
    if np.any((pick < 0) | (pick >= size * size)):
        raise ValueError("pick outside the window")
    return dx


def input_gradient_on_piece(net: Net, params: List[Optional[ConvParams]], x: np.ndarray, layer: int,
                            leaky_pass=None, pool_pick=None) -> np.ndarray:
    """dE/dx with the branch decisions given instead of taken.

    The energy's gradient is piecewise linear in the seed: its pieces are the
    leaky branches (z > 0 or not) and the max-pool window decisions.  This is
    ``input_gradient`` with those decisions supplied by the caller, everything
    else (FP64 forward for the seed, unfolded BN scale, backward-data conv)
    unchanged:

    * ``leaky_pass[i]`` (conv layer i with a leaky activation): bool array of
      layer i's output shape, True where the gradient passes unchanged and
      False where it is scaled by the slope;
    * ``pool_pick[i]`` (maxpool layer i): int array of the pool's output shape,
      the window element u*size + v that receives each window's gradient.

    Layers absent from the dicts decide as ``input_gradient`` does."""
    leaky_pass = leaky_pass or {}
    pool_pick = pool_pick or {}
    x = np.ascontiguousarray(x, dtype=np.float64)
    outs = forward(net, params, x, upto=layer + 1)
    ins = [x] + outs[:-1]
    grads: List[Optional[np.ndarray]] = [None] * (layer + 2)

    def add(v: int, g: np.ndarray) -> None:
        grads[v] = g if grads[v] is None else grads[v] + g

    grads[layer + 1] = outs[layer].copy()
    for i in range(layer, -1, -1):
        L = net.layers[i]
        gy = grads[i + 1]
        xin = ins[i]
        if L.kind == CONV:
            p = params[i]
            if L.activation == LEAKY:
                if i in leaky_pass:
                    passes = np.asarray(leaky_pass[i], bool)
                    if passes.shape != gy.shape:
                        raise ValueError("leaky decisions of layer %d: shape %s != %s" % (i, passes.shape, gy.shape))
                else:
                    z = add_bias(conv2d(xin, p.w, L.stride, L.pad), p.bias)
                    if L.batchnorm:
                        z = batchnorm(z, p.mean, p.var, p.gamma, p.beta, net.bn_eps)
                    passes = z > 0.0
                gy = gy * np.where(passes, 1.0, net.leaky_slope)
            if L.batchnorm:
                scale = np.asarray(p.gamma, np.float64) / np.sqrt(np.asarray(p.var, np.float64) + net.bn_eps)
                gy = gy * scale[None, :, None, None]
            add(i, conv2d_backward_data(gy, p.w, L.stride, L.pad, xin.shape[2], xin.shape[3]))
        elif L.kind == MAXPOOL:
            if i in pool_pick:
                add(i, maxpool_backward_picked(xin.shape, L.ksize, L.stride, pool_pick[i], gy))
            else:
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
