"""Helpers for the GPU parity tests: device staging with torch (memory only),
calls into libdn.so through the binding, and the error metric.

The metric is the relative L2 error over the whole output tensor, computed in
FP64: ||y_gpu - y_ref|| / ||y_ref||.  Gates: FP32 1e-5, BF16 2e-2, FP8 6e-2.
"""
import numpy as np

GATE = {0: 1e-5, 1: 2e-2, 2: 6e-2}
NAME = {0: "f32", 1: "bf16", 2: "fp8"}


def rel_l2(got, ref) -> float:
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    assert got.shape == ref.shape, (got.shape, ref.shape)
    return float(np.linalg.norm(got - ref) / np.linalg.norm(ref))


def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def dev(a, dtype=None):
    torch = torch_cuda()
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def empty_bytes(n):
    torch = torch_cuda()
    return torch.empty(max(int(n), 256), dtype=torch.uint8, device="cuda")


def fp8_scale(x) -> float:
    m = float(np.max(np.abs(x)))
    return m / 448.0 if m > 0 else 1.0


def nhwc_bytes(dn, dtype, n, c, h, w):
    return n * h * w * dn.channel_pad(dtype, c) * dn.ESIZE[dtype]


def to_storage(dn, dtype, x_nchw, scale=1.0, stream=None):
    """FP64 NCHW host array -> FP32 on device -> dn_ingest -> NHWC storage tensor."""
    torch = torch_cuda()
    n, c, h, w = x_nchw.shape
    xf = dev(x_nchw.astype(np.float32))
    buf = empty_bytes(nhwc_bytes(dn, dtype, n, c, h, w))
    dn.ingest(dtype, n, c, h, w, xf, scale, buf, stream)
    torch.cuda.synchronize()
    return buf


def from_storage(dn, dtype, buf, n, c, h, w, scale=1.0, stream=None):
    torch = torch_cuda()
    y = torch.empty((n, c, h, w), dtype=torch.float32, device="cuda")
    dn.egress(dtype, n, c, h, w, buf, scale, y, stream)
    torch.cuda.synchronize()
    return y.cpu().numpy().astype(np.float64)


def run_conv(dn, dtype, x, p, ksize, stride, pad, act, slope=0.1, eps=1e-5, pool=0, res=None,
             in_scale=1.0, res_scale=1.0, out_scale=1.0, tile=-1, splits=0, input_nchw=0):
    """One conv layer through dn_conv_pack + dn_conv2d on FP64 NCHW inputs
    (input_nchw = 1: the first-layer kernel reading the FP32 NCHW image)."""
    torch = torch_cuda()
    n, c, h, w = x.shape
    cout = p.w.shape[0]
    d = dn.conv_desc(n, h, w, c, cout, ksize, stride, pad, act, slope, 2 if pool else 0, 1 if res is not None else 0,
                     dtype, in_scale, res_scale, out_scale, tile, splits, input_nchw)
    wb, vb, wsb = dn.conv_sizes(d)
    wbuf, bbuf, sbuf = empty_bytes(wb), empty_bytes(vb), empty_bytes(vb)
    dn.conv_pack(d, p.w, p.bias, p.mean, p.var, p.gamma, p.beta, eps, wbuf, bbuf, sbuf)
    xb = dev(x.astype(np.float32)) if input_nchw else to_storage(dn, dtype, x, in_scale)
    ho = (h + 2 * pad - ksize) // stride + 1
    wo = (w + 2 * pad - ksize) // stride + 1
    if pool:
        ho //= 2
        wo //= 2
    rb = to_storage(dn, dtype, res, res_scale) if res is not None else None
    yb = empty_bytes(nhwc_bytes(dn, dtype, n, cout, ho, wo))
    ws = empty_bytes(wsb) if wsb else None
    dn.conv2d(d, xb, wbuf, bbuf, sbuf, rb, yb, ws, wsb)
    torch.cuda.synchronize()
    return from_storage(dn, dtype, yb, n, cout, ho, wo, out_scale)
