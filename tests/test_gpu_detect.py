"""Detection post-processing on the device against the FP32 oracle.

Kept boxes must match the oracle's exactly (same boxes, same order per image
and class; scores and coordinates within FP32 rounding).  The device's expf
and the summation order of the softmax may differ from numpy's by an ulp, so
a threshold or overlap decision that sits within 1e-5 (relative) of its
boundary may legitimately go either way: only then is a difference accepted,
and the device's result is then checked to be a valid greedy suppression."""
import numpy as np
import pytest

import synth
from oracle import detect as od
from tests import gpu_util as G

pytestmark = pytest.mark.gpu

AMB = 1e-5


@pytest.fixture(scope="module")
def dn():
    from paper_1811_03882_amd import dn as _dn
    G.torch_cuda()
    return _dn


def run_detect(dn, y, A, C, thresh, nms, max_det):
    torch = G.torch_cuda()
    n, _, h, w = y.shape
    anchors = synth.region_anchors(A)
    yd = torch.from_numpy(np.ascontiguousarray(y, np.float32)).cuda()
    wsb = dn.detect_workspace(n, A, C, h, w)
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    dets = torch.full((n, C, max_det, 5), -7.0, device="cuda")
    idx = torch.full((n, C, max_det), -7, dtype=torch.int32, device="cuda")
    cnt = torch.full((n, C), -7, dtype=torch.int32, device="cuda")
    dn.detect(yd, n, A, C, h, w, anchors, thresh, nms, max_det, ws, wsb, dets, idx, cnt)
    torch.cuda.synchronize()
    return anchors, dets.cpu().numpy(), idx.cpu().numpy(), cnt.cpu().numpy()


def ambiguous(boxes, scores, thresh, nms):
    """True when some decision of this (image, class) lies within AMB of its boundary."""
    near_t = np.any(np.abs(scores - thresh) <= AMB * max(thresh, 1e-30))
    cand = np.nonzero(scores >= thresh * (1 - AMB))[0]
    for x in range(len(cand)):
        for z in range(x + 1, len(cand)):
            if abs(float(od.iou(boxes[cand[x]], boxes[cand[z]])) - nms) <= AMB:
                return True
    return near_t


def check_valid(boxes, scores, kept, thresh, nms, cap):
    assert len(kept) <= cap
    assert all(scores[b] >= thresh * (1 - AMB) for b in kept)
    for x in range(len(kept)):
        for z in range(x + 1, len(kept)):
            assert od.iou(boxes[kept[x]], boxes[kept[z]]) <= nms + AMB


def compare(dn, y, A, C, thresh, nms, max_det):
    anchors, dets, idx, cnt = run_detect(dn, y, A, C, thresh, nms, max_det)
    ref = od.detect(y, anchors, C, thresh, nms, max_det)
    boxes, scores = od.decode(y, anchors, C)
    n_amb = n_kept = 0
    for n in range(y.shape[0]):
        for k in range(C):
            want = [(b, s, bx) for kk, b, s, bx in ref[n] if kk == k]
            c = int(cnt[n, k])
            got = [int(v) for v in idx[n, k, :c]]
            n_kept += c
            if got == [b for b, _, _ in want]:
                if c:
                    np.testing.assert_allclose(dets[n, k, :c, 0], [s for _, s, _ in want], rtol=2e-6, atol=1e-7)
                    np.testing.assert_allclose(dets[n, k, :c, 1:], np.stack([bx for _, _, bx in want]), rtol=2e-6,
                                               atol=1e-7)
                assert np.all(idx[n, k, c:] == -7)  # nothing written past the count
            else:
                assert ambiguous(boxes[n], scores[n, :, k], thresh, nms), \
                    "image %d class %d: device %s oracle %s" % (n, k, got, [b for b, _, _ in want])
                check_valid(boxes[n], scores[n, :, k], got, thresh, nms, max_det)
                n_amb += 1
    return n_kept, n_amb


@pytest.mark.parametrize("case", [
    dict(n=3, A=5, C=20, h=13, w=13, thresh=0.2, nms=0.45, max_det=50, clusters=0),   # 9-layer head, 416 input
    dict(n=2, A=5, C=20, h=13, w=13, thresh=0.2, nms=0.45, max_det=50, clusters=6),   # crowded: NMS does work
    dict(n=2, A=5, C=20, h=13, w=13, thresh=0.05, nms=0.3, max_det=3, clusters=4),    # the per-class cap binds
    dict(n=1, A=5, C=20, h=19, w=19, thresh=0.2, nms=0.45, max_det=64, clusters=8),   # 608 input, 1805 boxes
    dict(n=1, A=4, C=3, h=32, w=32, thresh=0.3, nms=0.5, max_det=200, clusters=20),   # 4096 boxes: the limit
    dict(n=2, A=1, C=1, h=3, w=5, thresh=0.5, nms=0.45, max_det=4, clusters=1),       # tiny, ragged
], ids=["b3_13x13", "crowded", "cap3", "19x19", "4096_boxes", "tiny"])
def test_detect_matches_oracle(dn, case):
    y = synth.region_output(case["n"], case["A"], case["C"], case["h"], case["w"], tag=case["h"] + case["clusters"],
                            clusters=case["clusters"])
    kept, amb = compare(dn, y, case["A"], case["C"], case["thresh"], case["nms"], case["max_det"])
    print("%s: %d boxes kept, %d ambiguous (image, class) lists" % (case, kept, amb))
    assert kept > 0 and amb <= 2


def test_detect_empty_when_nothing_passes(dn):
    y = synth.region_output(2, 5, 20, 13, 13, tag=99)
    _, dets, idx, cnt = run_detect(dn, y, 5, 20, 1.5, 0.45, 10)  # scores are <= 1
    assert np.all(cnt == 0) and np.all(idx == -7)


def test_detect_batch64_sampled(dn):
    """The bench shape (64 images, 13x13x5 boxes, 20 classes): every image's
    counts, and the full comparison on a sample of images."""
    y = synth.region_output(64, 5, 20, 13, 13, tag=64, clusters=3)
    anchors, dets, idx, cnt = run_detect(dn, y, 5, 20, 0.2, 0.45, 50)
    for n in (0, 17, 63):
        ref = od.detect(y[n:n + 1], anchors, 20, 0.2, 0.45, 50)[0]
        for k in range(20):
            want = [b for kk, b, _, _ in ref if kk == k]
            assert [int(v) for v in idx[n, k, :cnt[n, k]]] == want
    assert cnt.sum() > 0
