"""Whole-pass checking of the device's input-gradient pass against the oracle.

The energy's gradient is a piecewise-linear function of the network's
activations: the pieces are chosen by the leaky branches (pre-activation > 0
or not) and by each max-pool window's choice (its first maximum).  Where a
branch variable sits within the forward's rounding error of its threshold,
two correct evaluations may take different pieces, and their gradients then
differ by more than any rounding gate.  So a pass is checked in two steps:

1. Decisions.  Read back every decision the device took (the stored layer
   outputs, whose signs are the leaky branches; the argmax codes of fused
   conv + pool layers; a standalone pool's choice is the first maximum of its
   stored input, which the per-op tests pin bit-exactly).  Compare each with
   the FP64 oracle's own decision.  A decision that differs must lie within a
   forward-error bound of its threshold: |a_ref| <= B(a_ref) for a leaky
   branch, and a_ref[oracle's pick] - a_ref[device's pick] <= B + B for a
   window, with B(a) = K_SIGMA * e_rms + ULP * |a|, e_rms the RMS error of the
   device's stored output of that layer against the oracle's (whose relative
   L2 is itself gated at the forward gate) and ULP the storage format's unit
   in the last place (2^-8 BF16, 2^-23 FP32).
2. Gradient.  Compare the device's gradient with the oracle's gradient on the
   device's piece (``oracle.backward.input_gradient_on_piece``: FP64, the
   oracle's own forward for the seed, the device's decisions) per image, at
   the stated gates (FP32 1e-5, BF16 2e-2 relative L2).
"""
import numpy as np

import synth
from oracle import backward as ob
from oracle import net as onet
from tests import gpu_util as G

K_SIGMA = 8.0
ULP = {0: 2.0 ** -23, 1: 2.0 ** -8}


def first_max_pick(x, size, stride):
    """Window decisions of a max pool by the first-maximum rule (row-major
    window order; taps outside the input never win)."""
    n, c, h, w = x.shape
    ho, wo, off = (h - 1) // stride + 1, (w - 1) // stride + 1, (size - 1) // 2
    taps = np.full((size * size, n, c, ho, wo), -np.inf)
    for u in range(size):
        for v in range(size):
            yy = np.arange(ho) * stride - off + u
            xx = np.arange(wo) * stride - off + v
            iy = np.nonzero((yy >= 0) & (yy < h))[0]
            ix = np.nonzero((xx >= 0) & (xx < w))[0]
            taps[u * size + v][:, :, iy[:, None], ix[None, :]] = x[:, :, yy[iy][:, None], xx[ix][None, :]]
    return np.argmax(taps, axis=0)  # first occurrence of the maximum


def tap_values(x, size, stride, pick):
    """x at the window element `pick` of every pooling window."""
    n, c, h, w = x.shape
    off = (size - 1) // 2
    u, v = pick // size, pick % size
    i = np.arange(pick.shape[2])[None, None, :, None]
    j = np.arange(pick.shape[3])[None, None, None, :]
    yy, xx = i * stride - off + u, j * stride - off + v
    nn = np.arange(n)[:, None, None, None]
    cc = np.arange(c)[None, :, None, None]
    return x[nn, cc, yy, xx]


def run_device_pass(dn, net, dtype, params, x, layer, tune=False, nightmare_rate=None):
    """Run dn_input_gradient_arena (or one dn_nightmare_arena step when
    nightmare_rate is set) on a fresh net; return (gradient or updated image,
    stored outputs {layer: NCHW}, fused-pool codes {pool layer: NCHW})."""
    torch = G.torch_cuda()
    n, _, h, w = x.shape
    gn = dn.Net(net.layers, net.in_c, h, w, n, dtype=dtype, leaky_slope=net.leaky_slope, bn_eps=net.bn_eps)
    gn.load_params(params)
    if tune:
        gn.autotune_backward(layer, n, h, w)
    nb = gn.input_gradient_arena_bytes(layer, n, h, w)
    arena = G.empty_bytes(nb)
    xd = G.dev(x.astype(np.float32))
    if nightmare_rate is None:
        g = torch.empty_like(xd)
        gn.input_gradient_arena(arena, nb, layer, xd, n, h, w, g)
        result = g
    else:
        gn.nightmare_arena(arena, nb, layer, xd, n, h, w, nightmare_rate, 1)
        result = xd
    torch.cuda.synchronize()
    shapes = [o.shape[1:] for o in onet.forward(net, params, x[:1], upto=layer + 1)]
    stored, codes = {}, {}
    for i in range(layer + 1):
        c, ho, wo = shapes[i]
        if gn.input_gradient_readback(arena, nb, layer, n, h, w, i, 0):
            buf = torch.empty((n, c, ho, wo), dtype=torch.float32, device="cuda")
            gn.input_gradient_readback(arena, nb, layer, n, h, w, i, 0, buf, buf.numel() * 4)
            torch.cuda.synchronize()
            stored[i] = buf.cpu().numpy().astype(np.float64)
        if net.layers[i].kind == synth.MAXPOOL and gn.input_gradient_readback(arena, nb, layer, n, h, w, i, 1):
            cp = dn.channel_pad(dtype, c)
            buf = torch.empty(n * ho * wo * cp, dtype=torch.uint8, device="cuda")
            gn.input_gradient_readback(arena, nb, layer, n, h, w, i, 1, buf, buf.numel())
            torch.cuda.synchronize()
            codes[i] = buf.cpu().numpy().reshape(n, ho, wo, cp)[..., :c].transpose(0, 3, 1, 2).astype(np.int64)
    gn.close()
    return result.cpu().numpy().astype(np.float64), stored, codes


def check_decisions(net, dtype, x, layer, stored, codes, ref_outs):
    """Step 1: the device's decisions as oracle inputs (passes, picks), after
    checking every differing decision against the forward-error bound.
    Returns (passes, picks, flips per image, report lines)."""
    n = x.shape[0]
    ins = [x] + ref_outs[:-1]
    e_rms, report = {}, []
    for i, a in sorted(stored.items()):
        ref = ref_outs[i]
        err = G.rel_l2(a, ref)
        assert err < G.GATE[dtype], "stored output of layer %d: rel_l2 %.3e" % (i, err)
        e_rms[i] = float(np.sqrt(np.mean((a - ref) ** 2)))

    def bound(i, a_ref):
        return K_SIGMA * e_rms[i] + ULP[dtype] * np.abs(a_ref)

    passes, picks = {}, {}
    flips = np.zeros(n, np.int64)
    for i in range(layer + 1):
        L = net.layers[i]
        if L.kind == synth.MAXPOOL:
            if i in codes:  # fused with conv i-1: the conv's full output is not stored
                pick = codes[i]
                ei = i  # error scale of the pooled output
            else:
                pick = first_max_pick(stored[i - 1], L.ksize, L.stride)
                ei = i - 1
            own = first_max_pick(ins[i], L.ksize, L.stride)
            diff = pick != own
            if np.any(diff):
                top = tap_values(ins[i], L.ksize, L.stride, own)[diff]
                mine = tap_values(ins[i], L.ksize, L.stride, pick)[diff]
                gap = top - mine
                lim = bound(ei, top) + bound(ei, mine)
                assert np.all(gap <= lim), "pool layer %d: a window choice differs by %.3e > bound %.3e" % (
                    i, float((gap - lim).max() + lim[np.argmax(gap - lim)]), float(lim[np.argmax(gap - lim)]))
                flips += diff.reshape(n, -1).sum(axis=1)
                report.append("pool %d: %d window choices differ (max gap/bound %.2f)"
                              % (i, int(diff.sum()), float((gap / lim).max())))
            picks[i] = pick
        elif L.kind == synth.CONV and L.activation == synth.LEAKY:
            ref = ref_outs[i]
            if i in stored:
                dev = stored[i] > 0.0
                a_sel, ei = ref, i
            else:  # fused with pool i+1: the branch is decided at each window's chosen element, from the pooled sign
                pooled = stored[i + 1]
                dev = np.repeat(np.repeat(pooled > 0.0, 2, axis=2), 2, axis=3)
                # only the chosen element of each window carries gradient: check those
                a_sel = tap_values(ref, 2, 2, codes[i + 1])
                dev_sel = pooled > 0.0
                diff = dev_sel != (a_sel > 0.0)
                ei = i + 1
                if np.any(diff):
                    lim = bound(ei, a_sel[diff])
                    assert np.all(np.abs(a_sel[diff]) <= lim), "leaky layer %d: a branch differs away from 0" % i
                    flips += diff.reshape(n, -1).sum(axis=1)
                    report.append("leaky %d (fused): %d branches differ (max |a|/bound %.2f)"
                                  % (i, int(diff.sum()), float((np.abs(a_sel[diff]) / lim).max())))
                passes[i] = dev
                continue
            diff = dev != (ref > 0.0)
            if np.any(diff):
                lim = bound(ei, a_sel[diff])
                assert np.all(np.abs(a_sel[diff]) <= lim), "leaky layer %d: a branch differs away from 0" % i
                flips += diff.reshape(n, -1).sum(axis=1)
                report.append("leaky %d: %d branches differ (max |a|/bound %.2f)"
                              % (i, int(diff.sum()), float((np.abs(a_sel[diff]) / lim).max())))
            passes[i] = dev
    return passes, picks, flips, report


def check_pass(dn, net, dtype, params, x, layer, tune=False, label=""):
    """Run the device pass and check it (steps 1 and 2); returns the per-image
    gradient errors."""
    x32 = x.astype(np.float32).astype(np.float64)  # the device's input is FP32
    got, stored, codes = run_device_pass(dn, net, dtype, params, x32, layer, tune=tune)
    ref_outs = onet.forward(net, params, x32, upto=layer + 1)
    passes, picks, flips, report = check_decisions(net, dtype, x32, layer, stored, codes, ref_outs)
    ref = ob.input_gradient_on_piece(net, params, x32, layer, passes, picks)
    errs = np.array([G.rel_l2(got[i:i + 1], ref[i:i + 1]) for i in range(x.shape[0])])
    print("input gradient %s %s layer %d: per-image rel_l2 max %.3e, branch flips per image %s%s"
          % (G.NAME[dtype], label or net.name, layer, errs.max(),
             list(flips) if len(flips) <= 8 else "max %d, total %d" % (flips.max(), flips.sum()),
             "".join("\n  " + r for r in report)))
    assert np.all(errs < G.GATE[dtype]), errs
    return errs, got, passes, picks
