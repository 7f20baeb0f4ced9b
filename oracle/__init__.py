"""FP64 CPU oracle for the Darknet-style CNN forward pass.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  It shares no code
with the HIP library and the library never calls it.

``oracle.c`` holds the per-layer definitions (direct convolution, bias,
unfolded inference batch normalisation, leaky rectifier, max pooling with
-inf padding, residual add), each written as its plain textbook loop nest in
double precision.  ``net.py`` composes them into whole-network forwards.
This module compiles ``oracle.c`` with gcc and exposes numpy-level wrappers.

Parity status per function (the paper prints no tensor, so every pin is a
closed form, an invariant, brute force or a library routine; see the tests
under ``tests/test_oracle_*.py``):
  conv2d, add_bias, batchnorm, leaky, maxpool, shortcut: pinned.
  net forward: composition of the pinned layers; pinned by layer-by-layer
  recomputation and by identity-unit constructions.
  conv2d_backward_data, maxpool_backward (the image-edit gradient): pinned by
  central finite differences of the forward definitions (tests/test_oracle_backward.py).
  detect (``detect.py``, region decode + per-class NMS, FP32 like the device
  kernels): pinned by hand-computed boxes, closed-form IoUs, and brute-force
  checks of the suppression invariants.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None


def build(force: bool = False) -> str:
    """Compile oracle.c into liboracle.so (plain -O2, OpenMP for the outer loops)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load(path: str = None):
    global _lib
    with _lock:
        if _lib is None or path is not None:
            if path is None:
                build()
            lib = ctypes.CDLL(path or _LIB)
            dp = ctypes.POINTER(ctypes.c_double)
            i = ctypes.c_int
            lib.oracle_conv2d.argtypes = [dp, i, i, i, i, dp, i, i, i, i, i, dp]
            lib.oracle_add_bias.argtypes = [dp, i, i, i, dp]
            lib.oracle_batchnorm.argtypes = [dp, i, i, i, dp, dp, dp, dp, ctypes.c_double]
            lib.oracle_leaky.argtypes = [dp, ctypes.c_long, ctypes.c_double]
            lib.oracle_maxpool.argtypes = [dp, i, i, i, i, i, i, dp]
            lib.oracle_shortcut.argtypes = [dp, dp, ctypes.c_long]
            lib.oracle_conv2d_backward_data.argtypes = [dp, i, i, i, i, dp, i, i, i, i, i, i, i, dp]
            lib.oracle_maxpool_backward.argtypes = [dp, i, i, i, i, i, i, dp, dp]
            for f in (lib.oracle_conv2d, lib.oracle_add_bias, lib.oracle_batchnorm,
                      lib.oracle_leaky, lib.oracle_maxpool, lib.oracle_shortcut,
                      lib.oracle_conv2d_backward_data, lib.oracle_maxpool_backward):
                f.restype = None
            _lib = lib
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def conv2d(x, w, stride: int, pad: int) -> np.ndarray:
    """Direct convolution; x [N,C,H,W], w [K,C,R,S] -> [N,K,Ho,Wo]."""
    x, w = _f64(x), _f64(w)
    n, c, h, wd = x.shape
    k, c2, r, s = w.shape
    if c != c2:
        raise ValueError("channel mismatch %d vs %d" % (c, c2))
    ho = (h + 2 * pad - r) // stride + 1
    wo = (wd + 2 * pad - s) // stride + 1
    y = np.empty((n, k, ho, wo), np.float64)
    _load().oracle_conv2d(_p(x), n, c, h, wd, _p(w), k, r, s, stride, pad, _p(y))
    return y


def add_bias(y, b) -> np.ndarray:
    y, b = _f64(y).copy(), _f64(b)
    n, k, h, w = y.shape
    _load().oracle_add_bias(_p(y), n, k, h * w, _p(b))
    return y


def batchnorm(y, mean, var, gamma, beta, eps: float) -> np.ndarray:
    y = _f64(y).copy()
    n, k, h, w = y.shape
    mean, var, gamma, beta = (_f64(a) for a in (mean, var, gamma, beta))
    _load().oracle_batchnorm(_p(y), n, k, h * w, _p(mean), _p(var), _p(gamma), _p(beta), eps)
    return y


def leaky(y, slope: float) -> np.ndarray:
    y = _f64(y).copy()
    _load().oracle_leaky(_p(y), y.size, slope)
    return y


def maxpool(x, size: int, stride: int) -> np.ndarray:
    x = _f64(x)
    n, c, h, w = x.shape
    ho = (h - 1) // stride + 1
    wo = (w - 1) // stride + 1
    y = np.empty((n, c, ho, wo), np.float64)
    _load().oracle_maxpool(_p(x), n, c, h, w, size, stride, _p(y))
    return y


def shortcut(y, x) -> np.ndarray:
    y, x = _f64(y).copy(), _f64(x)
    if y.shape != x.shape:
        raise ValueError("shortcut shape mismatch %s vs %s" % (y.shape, x.shape))
    _load().oracle_shortcut(_p(y), _p(x), y.size)
    return y


def conv2d_backward_data(dy, w, stride: int, pad: int, h: int, wd: int) -> np.ndarray:
    """Gradient of conv2d with respect to its input: dy [N,K,Ho,Wo], w [K,C,R,S] -> [N,C,h,wd]."""
    dy, w = _f64(dy), _f64(w)
    n, k, ho, wo = dy.shape
    k2, c, r, s = w.shape
    if k != k2:
        raise ValueError("channel mismatch %d vs %d" % (k, k2))
    dx = np.empty((n, c, h, wd), np.float64)
    _load().oracle_conv2d_backward_data(_p(dy), n, k, ho, wo, _p(w), c, r, s, stride, pad, h, wd, _p(dx))
    return dx


def maxpool_backward(x, size: int, stride: int, dy) -> np.ndarray:
    """Gradient of maxpool with respect to its input (first maximal element of each window)."""
    x, dy = _f64(x), _f64(dy)
    n, c, h, w = x.shape
    dx = np.empty_like(x)
    _load().oracle_maxpool_backward(_p(x), n, c, h, w, size, stride, _p(dy), _p(dx))
    return dx


class use_library:
    """Context manager: route the wrappers to another build of oracle.c
    (the mutation tests compile deliberately broken copies)."""

    def __init__(self, path: str):
        self.path = path

    def __enter__(self):
        global _lib
        self._saved = _lib
        _load(self.path)
        return self

    def __exit__(self, *exc):
        global _lib
        _lib = self._saved
        return False


def set_threads(n: int) -> None:
    """Set the OpenMP thread count used by the next oracle calls."""
    os.environ["OMP_NUM_THREADS"] = str(n)
    try:
        gomp = ctypes.CDLL("libgomp.so.1")
        gomp.omp_set_num_threads(ctypes.c_int(n))
    except OSError:
        pass


from .net import forward, conv_layer  # noqa: E402  (re-export)
