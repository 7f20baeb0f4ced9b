"""Pins for the detection post-processing oracle: hand-computed decodes,
closed-form IoUs, and the defining invariants of greedy NMS checked by brute
force on random inputs (so that a wrong sign, index or comparison fails)."""
import numpy as np
import pytest

from oracle import detect as od

F = np.float32


def _region(n, A, C, h, w, fill=-20.0):
    return np.full((n, A * (5 + C), h, w), fill, np.float32)


def _set(y, n, a, C, i, j, tx, ty, tw, th, to, logits):
    base = a * (5 + C)
    for k, v in enumerate((tx, ty, tw, th, to) + tuple(logits)):
        y[n, base + k, i, j] = v


def test_sigmoid_softmax_closed_forms():
    assert od.sigmoid(np.array([0.0]))[0] == F(0.5)
    np.testing.assert_allclose(od.sigmoid(np.array([2.0, -2.0])), [1 / (1 + np.exp(-2)), 1 / (1 + np.exp(2))], rtol=1e-6)
    p = od.softmax(np.array([[1.0, 1.0, 1.0, 1.0]]))
    np.testing.assert_allclose(p, 0.25, rtol=1e-7)
    p = od.softmax(np.array([[np.log(3.0), 0.0]]))  # 3 : 1
    np.testing.assert_allclose(p, [[0.75, 0.25]], rtol=1e-6)


def test_decode_hand_computed_box():
    A, C, h, w = 2, 3, 2, 4
    anchors = [1.0, 2.0, 3.0, 0.5]
    y = _region(1, A, C, h, w)
    # cell (i=1, j=2), anchor 1: centre offsets 0.5, sizes exp(ln 2) * anchor
    _set(y, 0, 1, C, 1, 2, 0.0, 0.0, np.log(2.0), 0.0, 0.0, (np.log(3.0), 0.0, -np.inf))
    boxes, scores = od.decode(y, anchors, C)
    b = (1 * w + 2) * A + 1
    np.testing.assert_allclose(boxes[0, b], [(2 + 0.5) / 4, (1 + 0.5) / 2, 3.0 * 2 / 4, 0.5 * 1 / 2], rtol=1e-6)
    # objectness 0.5, probabilities 3/4, 1/4, 0
    np.testing.assert_allclose(scores[0, b], [0.375, 0.125, 0.0], rtol=1e-6, atol=1e-12)


def test_iou_closed_forms():
    a = np.array([0.5, 0.5, 0.2, 0.2], F)
    np.testing.assert_allclose(od.iou(a, a), 1.0, rtol=1e-6)  # edges vs area: FP32 rounding
    b = np.array([0.6, 0.5, 0.2, 0.2], F)          # shifted by half a width: 1/3
    np.testing.assert_allclose(od.iou(a, b), 1.0 / 3.0, rtol=1e-6)
    c = np.array([0.5, 0.5, 0.1, 0.1], F)          # nested: area ratio 1/4
    np.testing.assert_allclose(od.iou(a, c), 0.25, rtol=1e-6)
    d = np.array([0.9, 0.9, 0.1, 0.1], F)          # disjoint
    assert od.iou(a, d) == F(0)
    np.testing.assert_allclose(od.iou(a, b), od.iou(b, a), rtol=0)


def test_nms_suppresses_overlap_and_keeps_order():
    A, C, h, w = 1, 2, 1, 2
    anchors = [1.0, 1.0]
    y = _region(1, A, C, h, w)
    # two boxes of class 0 in neighbouring cells, width 1 cell -> wide boxes overlap
    _set(y, 0, 0, C, 0, 0, 0.0, 0.0, np.log(1.5), 0.0, 4.0, (5.0, -5.0))
    _set(y, 0, 0, C, 0, 1, -4.0, 0.0, np.log(1.5), 0.0, 3.0, (5.0, -5.0))
    boxes, scores = od.decode(y, anchors, C)
    ov = od.iou(boxes[0, 0], boxes[0, 1])
    assert ov > 0.45
    s4 = 1 / (1 + np.exp(4.0))
    inter = 0.625 - ((1 + s4) / 2 - 0.375)          # right edge of box 0 - left edge of box 1; heights equal
    np.testing.assert_allclose(ov, inter / (1.5 - inter), rtol=1e-5)
    dets = od.detect(y, anchors, C, 0.2, 0.45, 10)[0]
    assert [(k, b) for k, b, _, _ in dets] == [(0, 0)]      # box 1 suppressed by the higher box 0
    dets = od.detect(y, anchors, C, 0.2, float(ov), 10)[0]  # IoU equal to the threshold is kept
    assert [(k, b) for k, b, _, _ in dets] == [(0, 0), (0, 1)]
    dets = od.detect(y, anchors, C, 0.99, 0.45, 10)[0]      # threshold above both scores
    assert dets == []


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_nms_invariants_brute_force(seed):
    rng = np.random.default_rng([seed, 9])
    A, C, h, w = 3, 4, 5, 6
    anchors = rng.uniform(0.5, 3.0, 2 * A)
    y = rng.normal(0.0, 2.0, (2, A * (5 + C), h, w)).astype(np.float32)
    thresh, nt, cap = 0.2, 0.4, 7
    boxes, scores = od.decode(y, anchors, C)
    out = od.detect(y, anchors, C, thresh, nt, cap)
    for n in range(2):
        for k in range(C):
            kept = [(b, s) for kk, b, s, _ in out[n] if kk == k]
            s = scores[n, :, k]
            cand = sorted([b for b in range(h * w * A) if s[b] >= F(thresh)], key=lambda b: (-float(s[b]), b))
            # order, cap, threshold
            assert [b for b, _ in kept] == [b for b in cand if b in {q for q, _ in kept}]
            assert len(kept) <= cap
            assert all(sc >= thresh for _, sc in kept)
            # no two kept boxes overlap beyond the threshold
            for x in range(len(kept)):
                for z in range(x + 1, len(kept)):
                    assert od.iou(boxes[n, kept[x][0]], boxes[n, kept[z][0]]) <= F(nt)
            # every candidate ranked before the last kept one and not kept overlaps an
            # earlier kept box beyond the threshold
            if kept:
                last = cand.index(kept[-1][0])
                keptset = {b for b, _ in kept}
                for pos, b in enumerate(cand[:last]):
                    if b not in keptset:
                        assert any(od.iou(boxes[n, b], boxes[n, q]) > F(nt) for q in cand[:pos] if q in keptset)
