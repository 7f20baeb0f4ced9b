"""Thin ctypes binding of libdn.so (include/dn.h): argument marshalling only.

Every step of the forward pass runs in the library's HIP kernels.  PyTorch is
used by callers only to own device memory (pass a tensor, its data_ptr() is
taken) and streams (pass a torch stream, its handle is taken).  If libdn.so
is missing this module raises at import time: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence, Tuple

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdn.so")

DN_OK, DN_EINVAL, DN_ENOMEM, DN_EHIP, DN_ESTATE, DN_EUNSUPPORTED, DN_ETIMEDOUT = 0, -1, -2, -3, -4, -5, -6
F32, BF16, FP8 = 0, 1, 2
RESIDENT, PER_LAYER = 0, 1
CONV, MAXPOOL, SHORTCUT = 0, 1, 2
LINEAR, LEAKY = 0, 1
DTYPES = {"f32": F32, "fp32": F32, "bf16": BF16, "fp8": FP8, "fp8_e4m3": FP8}
ESIZE = {F32: 4, BF16: 2, FP8: 1}
FP8_MAX = 448.0


class DnError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("dn error %d: %s" % (status, msg))
        self.status = status


class LayerDesc(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("cout", ctypes.c_int), ("ksize", ctypes.c_int),
                ("stride", ctypes.c_int), ("pad", ctypes.c_int), ("batchnorm", ctypes.c_int),
                ("activation", ctypes.c_int), ("src", ctypes.c_int)]


class NetOpts(ctypes.Structure):
    _fields_ = [("in_c", ctypes.c_int), ("max_h", ctypes.c_int), ("max_w", ctypes.c_int),
                ("max_batch", ctypes.c_int), ("dtype", ctypes.c_int), ("mode", ctypes.c_int),
                ("leaky_slope", ctypes.c_float), ("bn_eps", ctypes.c_double),
                ("use_graph", ctypes.c_int), ("device", ctypes.c_int), ("batch_invariant", ctypes.c_int),
                ("input_u8", ctypes.c_int)]


class ConvDesc(ctypes.Structure):
    _fields_ = [("batch", ctypes.c_int), ("in_h", ctypes.c_int), ("in_w", ctypes.c_int),
                ("in_c", ctypes.c_int), ("cout", ctypes.c_int), ("ksize", ctypes.c_int),
                ("stride", ctypes.c_int), ("pad", ctypes.c_int), ("activation", ctypes.c_int),
                ("leaky_slope", ctypes.c_float), ("pool", ctypes.c_int), ("residual", ctypes.c_int),
                ("dtype", ctypes.c_int), ("in_scale", ctypes.c_float), ("res_scale", ctypes.c_float),
                ("out_scale", ctypes.c_float), ("tile", ctypes.c_int), ("splits", ctypes.c_int),
                ("input_nchw", ctypes.c_int)]


class PoolDesc(ctypes.Structure):
    _fields_ = [("batch", ctypes.c_int), ("h", ctypes.c_int), ("w", ctypes.c_int), ("c", ctypes.c_int),
                ("size", ctypes.c_int), ("stride", ctypes.c_int), ("dtype", ctypes.c_int)]


class GaParams(ctypes.Structure):
    _fields_ = [("population", ctypes.c_int), ("generations", ctypes.c_int), ("crossover", ctypes.c_double),
                ("mutation", ctypes.c_double), ("timeout_s", ctypes.c_double), ("penalty_s", ctypes.c_double),
                ("seed", ctypes.c_ulonglong)]


class GaResult(ctypes.Structure):
    _fields_ = [("best_seconds", ctypes.c_double), ("evaluations", ctypes.c_int), ("memo_hits", ctypes.c_int)]


GA_MEASURE = ctypes.CFUNCTYPE(ctypes.c_double, ctypes.POINTER(ctypes.c_ubyte), ctypes.c_int, ctypes.c_double,
                              ctypes.c_void_p)

_vp, _i, _sz, _f, _d = ctypes.c_void_p, ctypes.c_int, ctypes.c_size_t, ctypes.c_float, ctypes.c_double
_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)

SIGNATURES = {
    "dn_net_create": (_i, [ctypes.POINTER(LayerDesc), _i, ctypes.POINTER(NetOpts), ctypes.POINTER(_vp)]),
    "dn_net_destroy": (None, [_vp]),
    "dn_net_output_shape": (_i, [_vp, _i, _i, _ip, _ip, _ip]),
    "dn_arena_bytes": (_i, [_vp, _i, _i, _i, ctypes.POINTER(_sz)]),
    "dn_bind_arena": (_i, [_vp, _vp, _sz]),
    "dn_load_weights": (_i, [_vp, _i, _dp, _dp, _dp, _dp, _dp, _dp]),
    "dn_calibrate": (_i, [_vp, _vp, _i, _i, _i, _vp]),
    "dn_forward": (_i, [_vp, _vp, _i, _i, _i, _vp, _vp]),
    "dn_forward_arena": (_i, [_vp, _vp, _sz, _vp, _i, _i, _i, _vp, _vp]),
    "dn_autotune": (_i, [_vp, _i, _i, _i, _vp]),
    "dn_time_layer": (_i, [_vp, _i, _i, _i, _i, _i, _vp, ctypes.POINTER(_f)]),
    "dn_layer_plan": (_i, [_vp, _i, _i, _i, _i, _ip, _ip, _ip, _ip]),
    "dn_channel_pad": (_i, [_i, _i]),
    "dn_conv_sizes": (_i, [ctypes.POINTER(ConvDesc), ctypes.POINTER(_sz), ctypes.POINTER(_sz), ctypes.POINTER(_sz)]),
    "dn_conv_pack": (_i, [ctypes.POINTER(ConvDesc), _dp, _dp, _dp, _dp, _dp, _dp, _d, _vp, _vp, _vp, _vp]),
    "dn_conv2d": (_i, [ctypes.POINTER(ConvDesc), _vp, _vp, _vp, _vp, _vp, _vp, _vp, _sz, _vp]),
    "dn_maxpool": (_i, [ctypes.POINTER(PoolDesc), _vp, _vp, _vp]),
    "dn_shortcut": (_i, [_i, _sz, _vp, _f, _vp, _f, _vp, _f, _vp]),
    "dn_ingest": (_i, [_i, _i, _i, _i, _i, _vp, _f, _vp, _vp]),
    "dn_egress": (_i, [_i, _i, _i, _i, _i, _vp, _f, _vp, _vp]),
    "dn_tile_count": (_i, []),
    "dn_tile_info": (_i, [_i, _ip, _ip, _ip, _ip, _ip]),
    "dn_mfma_peak": (_i, [_i, _i, ctypes.POINTER(ctypes.c_double)]),
    "dn_jacobi": (_i, [_vp, _vp, _i, _i, _i, _vp, _vp]),
    "dn_jacobi_per_iteration": (_i, [_vp, _vp, _vp, _i, _i, _i, _dp, _vp]),
    "dn_detect_workspace": (_i, [_i, _i, _i, _i, _i, ctypes.POINTER(_sz)]),
    "dn_detect": (_i, [_vp, _i, _i, _i, _i, _i, ctypes.POINTER(ctypes.c_float), _f, _f, _i, _vp, _sz, _vp, _vp,
                       _vp, _vp]),
    "dn_detect_noalloc": (_i, [_vp, _i, _i, _i, _i, _i, ctypes.POINTER(ctypes.c_float), _f, _f, _i, _vp, _vp, _vp,
                               _vp]),
    "dn_conv_backward_sizes": (_i, [ctypes.POINTER(ConvDesc), ctypes.POINTER(_sz), ctypes.POINTER(_sz),
                                    ctypes.POINTER(_sz)]),
    "dn_conv_pack_backward": (_i, [ctypes.POINTER(ConvDesc), _dp, _dp, _dp, _dp, _d, _vp, _vp, _vp, _vp]),
    "dn_conv_backward_data": (_i, [ctypes.POINTER(ConvDesc), _vp, _vp, _vp, _vp, _i, _vp, _vp, _sz, _vp]),
    "dn_maxpool_backward": (_i, [ctypes.POINTER(PoolDesc), _vp, _vp, _i, _vp, _vp]),
    "dn_leaky_backward": (_i, [_i, _sz, _vp, _vp, _f, _vp, _vp]),
    "dn_input_gradient_arena_bytes": (_i, [_vp, _i, _i, _i, _i, ctypes.POINTER(_sz)]),
    "dn_input_gradient": (_i, [_vp, _i, _vp, _i, _i, _i, _vp, _vp]),
    "dn_input_gradient_arena": (_i, [_vp, _vp, _sz, _i, _vp, _i, _i, _i, _vp, _vp]),
    "dn_input_gradient_readback": (_i, [_vp, _vp, _sz, _i, _i, _i, _i, _i, _i, _vp, _sz, _ip, _vp]),
    "dn_nightmare": (_i, [_vp, _i, _vp, _i, _i, _i, _f, _i, _vp]),
    "dn_nightmare_arena": (_i, [_vp, _vp, _sz, _i, _vp, _i, _i, _i, _f, _i, _vp]),
    "dn_autotune_backward": (_i, [_vp, _i, _i, _i, _i, _vp]),
    "dn_placed_arena_bytes": (_i, [_vp, _i, _i, _i, ctypes.POINTER(_sz)]),
    "dn_placed_transfers": (_i, [_vp, _vp, _i, _i, _i, _i, _ip, _ip, ctypes.POINTER(_sz), ctypes.POINTER(_sz)]),
    "dn_forward_placed": (_i, [_vp, _vp, _i, _vp, _i, _i, _i, _vp, _d, _vp]),
    "dn_cpu_conv2d": (_i, [ctypes.POINTER(ConvDesc), _vp, _vp, _vp, _vp]),
    "dn_cpu_maxpool": (_i, [ctypes.POINTER(PoolDesc), _vp, _vp]),
    "dn_ga_next_generation": (_i, [ctypes.POINTER(GaParams), _i, _vp, _vp, _vp, ctypes.POINTER(ctypes.c_ulonglong)]),
    "dn_ga_search": (_i, [ctypes.POINTER(GaParams), _i, GA_MEASURE, _vp, _vp, _vp, ctypes.POINTER(GaResult)]),
    "dn_ga_place": (_i, [_vp, ctypes.POINTER(GaParams), _vp, _i, _i, _i, _vp, _i, _vp, _vp, _vp,
                         ctypes.POINTER(GaResult)]),
    "dn_last_error": (ctypes.c_char_p, []),
}


def _load():
    # One HIP runtime per process: torch ships its own libamdhip64.so (same
    # SONAME as ROCm's).  Importing torch first makes libdn.so bind to that
    # already-loaded runtime, so that tensors torch allocates and kernels this
    # library launches share one device context.  Loading libdn.so first would
    # pull in a second runtime that cannot open the GPU next to torch's.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(LIB_PATH):
        raise ImportError("libdn.so not built at %s (run python -m paper_1811_03882_amd.build)" % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


LIB = _load()


def last_error() -> str:
    m = LIB.dn_last_error()
    return m.decode() if m else ""


def check(status: int) -> None:
    if status != DN_OK:
        raise DnError(status, last_error())


def ptr(x) -> Optional[int]:
    """Device/host address of a torch tensor, numpy array or int (None stays None)."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    if hasattr(x, "data_ptr"):
        return x.data_ptr()
    if hasattr(x, "ctypes"):
        return x.ctypes.data
    raise TypeError("cannot take the address of %r" % type(x))


def stream_handle(s) -> Optional[int]:
    if s is None:
        return None
    if isinstance(s, int):
        return s
    return s.cuda_stream


def _dptr(a):
    import numpy as np
    if a is None:
        return None, None
    arr = np.ascontiguousarray(a, dtype=np.float64)
    return arr, arr.ctypes.data_as(_dp)


def channel_pad(dtype: int, c: int) -> int:
    return LIB.dn_channel_pad(dtype, c)


def tile_count() -> int:
    return LIB.dn_tile_count()


def jacobi(u, work, n: int, m: int, iters: int, max_change=None, stream=None):
    """Device-resident Jacobi iterations of the Laplace equation (see dn_jacobi)."""
    check(LIB.dn_jacobi(ptr(u), ptr(work), n, m, iters, ptr(max_change), stream_handle(stream)))


def jacobi_per_iteration(u_host: np.ndarray, dev_a, dev_b, iters: int, stream=None) -> float:
    """The per-iteration-transfer variant on a host FP64 grid (updated in place);
    returns the last iteration's max change."""
    assert u_host.dtype == np.float64 and u_host.flags.c_contiguous
    mc = ctypes.c_double()
    check(LIB.dn_jacobi_per_iteration(u_host.ctypes.data, ptr(dev_a), ptr(dev_b), u_host.shape[0], u_host.shape[1],
                                      iters, ctypes.byref(mc), stream_handle(stream)))
    return mc.value


def detect_workspace(batch: int, anchors: int, classes: int, h: int, w: int) -> int:
    v = _sz()
    check(LIB.dn_detect_workspace(batch, anchors, classes, h, w, ctypes.byref(v)))
    return v.value


def detect(y, batch, anchors, classes, h, w, anchor_wh, thresh, nms_thresh, max_det, workspace, ws_bytes,
           dets, det_index, counts, stream=None):
    """Region decode + per-class NMS on the device (see dn_detect)."""
    aw = (ctypes.c_float * len(anchor_wh))(*[float(v) for v in anchor_wh])
    check(LIB.dn_detect(ptr(y), batch, anchors, classes, h, w, aw, float(thresh), float(nms_thresh), max_det,
                        ptr(workspace), ws_bytes, ptr(dets), ptr(det_index), ptr(counts), stream_handle(stream)))


def detect_noalloc(y, batch, anchors, classes, h, w, anchor_wh, thresh, nms_thresh, max_det, dets, det_index, counts,
                   stream=None):
    """dn_detect on the library's fixed per-GPU scratch (no workspace, no allocation)."""
    aw = (ctypes.c_float * len(anchor_wh))(*[float(v) for v in anchor_wh])
    check(LIB.dn_detect_noalloc(ptr(y), batch, anchors, classes, h, w, aw, float(thresh), float(nms_thresh), max_det,
                                ptr(dets), ptr(det_index), ptr(counts), stream_handle(stream)))


def mfma_peak(dtype: int, device: int = 0) -> float:
    """Sustained MFMA throughput (TFLOP/s) of the instruction dtype's convs use."""
    v = ctypes.c_double()
    check(LIB.dn_mfma_peak(dtype, device, ctypes.byref(v)))
    return v.value


def tile_info(t: int) -> Tuple[int, int, int, int, int]:
    """(bm, bn, waves_m, waves_n, BF16 MFMA block side) of tile config t."""
    v = [_i() for _ in range(5)]
    check(LIB.dn_tile_info(t, *[ctypes.byref(x) for x in v]))
    return tuple(x.value for x in v)


def layer_descs(layers) -> "ctypes.Array":
    arr = (LayerDesc * len(layers))()
    for i, L in enumerate(layers):
        arr[i] = LayerDesc(L.kind, L.cout, L.ksize, L.stride, L.pad, int(bool(L.batchnorm)),
                           L.activation, L.src)
    return arr


class Net:
    """A network in the library (dn_net), created from layer objects with the
    fields kind, cout, ksize, stride, pad, batchnorm, activation, src."""

    def __init__(self, layers: Sequence, in_c: int, max_h: int, max_w: int, max_batch: int,
                 dtype: int = F32, mode: int = RESIDENT, leaky_slope: float = 0.1,
                 bn_eps: float = 1e-5, use_graph: bool = False, device: int = 0, batch_invariant: bool = False,
                 input_u8: bool = False):
        self.layers = list(layers)
        self.dtype, self.mode = dtype, mode
        self.in_c = in_c
        opts = NetOpts(in_c, max_h, max_w, max_batch, dtype, mode, leaky_slope, bn_eps,
                       int(bool(use_graph)), device, int(bool(batch_invariant)), int(bool(input_u8)))
        self.input_u8 = bool(input_u8)
        h = _vp()
        descs = layer_descs(self.layers)
        check(LIB.dn_net_create(descs, len(self.layers), ctypes.byref(opts), ctypes.byref(h)))
        self._h = h
        self._arena = None

    @property
    def handle(self):
        return self._h

    def close(self) -> None:
        if self._h:
            LIB.dn_net_destroy(self._h)
            self._h = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def output_shape(self, h: int, w: int) -> Tuple[int, int, int]:
        c, ho, wo = _i(), _i(), _i()
        check(LIB.dn_net_output_shape(self._h, h, w, ctypes.byref(c), ctypes.byref(ho), ctypes.byref(wo)))
        return c.value, ho.value, wo.value

    def arena_bytes(self, batch: int, h: int, w: int) -> int:
        n = _sz()
        check(LIB.dn_arena_bytes(self._h, batch, h, w, ctypes.byref(n)))
        return n.value

    def bind_arena(self, arena, nbytes: Optional[int] = None) -> None:
        if nbytes is None:
            nbytes = arena.numel() * arena.element_size()
        check(LIB.dn_bind_arena(self._h, ptr(arena), nbytes))
        self._arena = arena  # keep the caller's memory alive while bound

    def load_layer(self, layer: int, w, bias, mean=None, var=None, gamma=None, beta=None) -> None:
        keep = [_dptr(a) for a in (w, bias, mean, var, gamma, beta)]
        check(LIB.dn_load_weights(self._h, layer, *[k[1] for k in keep]))

    def load_params(self, params) -> None:
        for i, p in enumerate(params):
            if p is not None:
                self.load_layer(i, p.w, p.bias, p.mean, p.var, p.gamma, p.beta)

    def calibrate(self, x, batch: int, h: int, w: int, stream=None) -> None:
        check(LIB.dn_calibrate(self._h, ptr(x), batch, h, w, stream_handle(stream)))

    def forward(self, x, batch: int, h: int, w: int, y, stream=None) -> None:
        check(LIB.dn_forward(self._h, ptr(x), batch, h, w, ptr(y), stream_handle(stream)))

    def forward_arena(self, arena, nbytes: int, x, batch: int, h: int, w: int, y, stream=None) -> None:
        check(LIB.dn_forward_arena(self._h, ptr(arena), nbytes, ptr(x), batch, h, w, ptr(y),
                                   stream_handle(stream)))

    def autotune(self, batch: int, h: int, w: int, stream=None) -> None:
        check(LIB.dn_autotune(self._h, batch, h, w, stream_handle(stream)))

    def time_layer(self, layer: int, batch: int, h: int, w: int, iters: int, stream=None) -> float:
        ms = _f()
        check(LIB.dn_time_layer(self._h, layer, batch, h, w, iters, stream_handle(stream), ctypes.byref(ms)))
        return ms.value

    def input_gradient_arena_bytes(self, layer: int, batch: int, h: int, w: int) -> int:
        n = _sz()
        check(LIB.dn_input_gradient_arena_bytes(self._h, layer, batch, h, w, ctypes.byref(n)))
        return n.value

    def input_gradient(self, layer: int, x, batch: int, h: int, w: int, grad, stream=None) -> None:
        check(LIB.dn_input_gradient(self._h, layer, ptr(x), batch, h, w, ptr(grad), stream_handle(stream)))

    def input_gradient_arena(self, arena, nbytes: int, layer: int, x, batch: int, h: int, w: int, grad,
                             stream=None) -> None:
        check(LIB.dn_input_gradient_arena(self._h, ptr(arena), nbytes, layer, ptr(x), batch, h, w, ptr(grad),
                                          stream_handle(stream)))

    def autotune_backward(self, layer: int, batch: int, h: int, w: int, stream=None) -> None:
        check(LIB.dn_autotune_backward(self._h, layer, batch, h, w, stream_handle(stream)))

    def input_gradient_readback(self, arena, nbytes: int, layer: int, batch: int, h: int, w: int, of_layer: int,
                                what: int, out=None, out_bytes: int = 0, stream=None) -> bool:
        """Copy a buffer of the last input-gradient pass on `arena` into `out`
        (what: 0 stored output, 1 fused-pool argmax codes, 2 gradient); returns
        whether the pass keeps that buffer."""
        av = _i()
        check(LIB.dn_input_gradient_readback(self._h, ptr(arena), nbytes, layer, batch, h, w, of_layer, what,
                                             ptr(out), out_bytes, ctypes.byref(av), stream_handle(stream)))
        return bool(av.value)

    def nightmare(self, layer: int, x, batch: int, h: int, w: int, rate: float, iters: int, stream=None) -> None:
        check(LIB.dn_nightmare(self._h, layer, ptr(x), batch, h, w, rate, iters, stream_handle(stream)))

    def nightmare_arena(self, arena, nbytes: int, layer: int, x, batch: int, h: int, w: int, rate: float,
                        iters: int, stream=None) -> None:
        check(LIB.dn_nightmare_arena(self._h, ptr(arena), nbytes, layer, ptr(x), batch, h, w, rate, iters,
                                     stream_handle(stream)))

    # ---- layer placement between the host CPU and the GPU (genes: one 0/1 per layer)

    def placed_arena_bytes(self, batch: int, h: int, w: int) -> int:
        n = _sz()
        check(LIB.dn_placed_arena_bytes(self._h, batch, h, w, ctypes.byref(n)))
        return n.value

    def placed_transfers(self, gene, batch: int, h: int, w: int):
        """(h2d copies, d2h copies, h2d bytes, d2h bytes) per placed forward."""
        g = _gene(gene)
        a, b, c, d = _i(), _i(), _sz(), _sz()
        check(LIB.dn_placed_transfers(self._h, g.ctypes.data, len(g), batch, h, w, ctypes.byref(a), ctypes.byref(b),
                                      ctypes.byref(c), ctypes.byref(d)))
        return a.value, b.value, c.value, d.value

    def forward_placed(self, gene, x: np.ndarray, batch: int, h: int, w: int, y: np.ndarray, timeout_s: float = 0.0,
                       stream=None) -> None:
        """Placed forward on host NCHW FP32 arrays x -> y."""
        g = _gene(gene)
        assert x.dtype == np.float32 and x.flags.c_contiguous and y.dtype == np.float32 and y.flags.c_contiguous
        check(LIB.dn_forward_placed(self._h, g.ctypes.data, len(g), x.ctypes.data, batch, h, w, y.ctypes.data,
                                    float(timeout_s), stream_handle(stream)))

    def ga_place(self, params: "GaParams", x: np.ndarray, batch: int, h: int, w: int, y: np.ndarray, reps: int = 3,
                 stream=None):
        """The GA over this net's placements; returns (best gene, per-generation best seconds, GaResult)."""
        L = len(self.layers)
        best = np.zeros(L, dtype=np.uint8)
        gen = np.zeros(params.generations, dtype=np.float64)
        res = GaResult()
        assert x.dtype == np.float32 and y.dtype == np.float32
        check(LIB.dn_ga_place(self._h, ctypes.byref(params), x.ctypes.data, batch, h, w, y.ctypes.data, reps,
                              stream_handle(stream), best.ctypes.data, gen.ctypes.data, ctypes.byref(res)))
        return best, gen, res

    def layer_plan(self, layer: int, batch: int, h: int, w: int):
        v = [_i() for _ in range(4)]
        check(LIB.dn_layer_plan(self._h, layer, batch, h, w, *[ctypes.byref(x) for x in v]))
        return dict(zip(("tile", "splits", "fused_pool", "fused_res"), (x.value for x in v)))


# ------------------------------------------------------------ standalone layers


def conv_desc(batch, in_h, in_w, in_c, cout, ksize, stride, pad, activation=LEAKY, slope=0.1,
              pool=0, residual=0, dtype=F32, in_scale=1.0, res_scale=1.0, out_scale=1.0,
              tile=-1, splits=0, input_nchw=0) -> ConvDesc:
    return ConvDesc(batch, in_h, in_w, in_c, cout, ksize, stride, pad, activation, slope, pool,
                    residual, dtype, in_scale, res_scale, out_scale, tile, splits, input_nchw)


def conv_sizes(d: ConvDesc) -> Tuple[int, int, int]:
    a, b, c = _sz(), _sz(), _sz()
    check(LIB.dn_conv_sizes(ctypes.byref(d), ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
    return a.value, b.value, c.value


def conv_pack(d: ConvDesc, w, bias, mean, var, gamma, beta, eps, w_out, bias_out, wscale_out, stream=None):
    keep = [_dptr(a) for a in (w, bias, mean, var, gamma, beta)]
    check(LIB.dn_conv_pack(ctypes.byref(d), *[k[1] for k in keep], eps, ptr(w_out), ptr(bias_out),
                           ptr(wscale_out), stream_handle(stream)))


def conv2d(d: ConvDesc, x, w_packed, bias, wscale, res, y, workspace=None, ws_bytes=0, stream=None):
    check(LIB.dn_conv2d(ctypes.byref(d), ptr(x), ptr(w_packed), ptr(bias), ptr(wscale), ptr(res), ptr(y),
                        ptr(workspace), ws_bytes, stream_handle(stream)))


def maxpool(batch, h, w, c, size, stride, dtype, x, y, stream=None):
    d = PoolDesc(batch, h, w, c, size, stride, dtype)
    check(LIB.dn_maxpool(ctypes.byref(d), ptr(x), ptr(y), stream_handle(stream)))


def shortcut(dtype, count, a, sa, b, sb, y, sy, stream=None):
    check(LIB.dn_shortcut(dtype, count, ptr(a), sa, ptr(b), sb, ptr(y), sy, stream_handle(stream)))


def ingest(dtype, batch, c, h, w, x, scale, y, stream=None):
    check(LIB.dn_ingest(dtype, batch, c, h, w, ptr(x), scale, ptr(y), stream_handle(stream)))


def egress(dtype, batch, c, h, w, x, scale, y, stream=None):
    check(LIB.dn_egress(dtype, batch, c, h, w, ptr(x), scale, ptr(y), stream_handle(stream)))


def conv_backward_sizes(d: ConvDesc) -> Tuple[int, int, int]:
    a, b, c = _sz(), _sz(), _sz()
    check(LIB.dn_conv_backward_sizes(ctypes.byref(d), ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
    return a.value, b.value, c.value


def conv_pack_backward(d: ConvDesc, w, mean, var, gamma, eps, w_out, zero_bias, unit_scale, stream=None):
    keep = [_dptr(a) for a in (w, mean, var, gamma)]
    check(LIB.dn_conv_pack_backward(ctypes.byref(d), *[k[1] for k in keep], eps, ptr(w_out), ptr(zero_bias),
                                    ptr(unit_scale), stream_handle(stream)))


def conv_backward_data(d: ConvDesc, dy, w_packed, zero_bias, unit_scale, accumulate, dx, workspace=None,
                       ws_bytes=0, stream=None):
    check(LIB.dn_conv_backward_data(ctypes.byref(d), ptr(dy), ptr(w_packed), ptr(zero_bias), ptr(unit_scale),
                                    int(accumulate), ptr(dx), ptr(workspace), ws_bytes, stream_handle(stream)))


def maxpool_backward(batch, h, w, c, size, stride, dtype, x, dy, accumulate, dx, stream=None):
    d = PoolDesc(batch, h, w, c, size, stride, dtype)
    check(LIB.dn_maxpool_backward(ctypes.byref(d), ptr(x), ptr(dy), int(accumulate), ptr(dx), stream_handle(stream)))


def leaky_backward(dtype, count, a, dy, slope, dx, stream=None):
    check(LIB.dn_leaky_backward(dtype, count, ptr(a), ptr(dy), slope, ptr(dx), stream_handle(stream)))


# ------------------------------------------------------------ placement search (host logic)


def _gene(gene) -> np.ndarray:
    g = np.ascontiguousarray(np.asarray(gene, dtype=np.uint8))
    assert g.ndim == 1
    return g


def ga_params(population=30, generations=20, crossover=0.9, mutation=0.05, timeout_s=180.0, penalty_s=1000.0,
              seed=0) -> GaParams:
    """GA parameters; the defaults are the paper's (M 30, T 20, Pc 0.9, Pm 0.05,
    a 3-minute limit scored as 1000 s)."""
    return GaParams(population, generations, crossover, mutation, timeout_s, penalty_s, seed)


def ga_next_generation(params: GaParams, pop: np.ndarray, seconds: np.ndarray, rng_state: int):
    """One generation step; returns (next population, new rng state)."""
    pop = np.ascontiguousarray(pop, dtype=np.uint8)
    sec = np.ascontiguousarray(seconds, dtype=np.float64)
    nxt = np.zeros_like(pop)
    st = ctypes.c_ulonglong(rng_state)
    check(LIB.dn_ga_next_generation(ctypes.byref(params), pop.shape[1], pop.ctypes.data, sec.ctypes.data,
                                    nxt.ctypes.data, ctypes.byref(st)))
    return nxt, st.value


def ga_search(params: GaParams, gene_len: int, measure):
    """GA with a Python measurement measure(gene: np.ndarray, timeout_s) -> seconds;
    returns (best gene, per-generation best seconds, GaResult)."""
    def cb(gp, n, timeout, user):
        return float(measure(np.ctypeslib.as_array(gp, shape=(n,)).copy(), timeout))
    fn = GA_MEASURE(cb)
    best = np.zeros(gene_len, dtype=np.uint8)
    gen = np.zeros(params.generations, dtype=np.float64)
    res = GaResult()
    check(LIB.dn_ga_search(ctypes.byref(params), gene_len, fn, None, best.ctypes.data, gen.ctypes.data,
                           ctypes.byref(res)))
    return best, gen, res


def cpu_conv2d(d: ConvDesc, x: np.ndarray, w: np.ndarray, bias: np.ndarray, y: np.ndarray) -> None:
    """Host FP32 conv of the placement's CPU side on NHWC (padded) arrays."""
    for a in (x, w, bias, y):
        assert a.dtype == np.float32 and a.flags.c_contiguous
    check(LIB.dn_cpu_conv2d(ctypes.byref(d), x.ctypes.data, w.ctypes.data, bias.ctypes.data, y.ctypes.data))


def cpu_maxpool(batch, h, w, c, size, stride, x: np.ndarray, y: np.ndarray) -> None:
    d = PoolDesc(batch, h, w, c, size, stride, F32)
    assert x.dtype == np.float32 and y.dtype == np.float32
    check(LIB.dn_cpu_maxpool(ctypes.byref(d), x.ctypes.data, y.ctypes.data))
