"""Detection post-processing of a region-layer output, written out plainly.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The paper evaluates Darknet's object-detection sample program (Sec. 5.1.1)
but states no decoding rule, so the rule here is a reading (Darknet's
region-layer convention): the output of the 9-layer network's last 1x1 conv has
``A * (5 + C)`` channels per grid cell; for anchor ``a`` its channels
``a*(5+C) + (0..4)`` are the box and objectness terms ``tx, ty, tw, th, to``
and the next ``C`` channels are class logits.  For cell (row i, column j) of
an H x W grid:

* box centre ``x = (j + sigmoid(tx)) / W``, ``y = (i + sigmoid(ty)) / H``;
* box size ``w = anchor_w[a] * exp(tw) / W``, ``h = anchor_h[a] * exp(th) / H``;
* class probabilities ``p = softmax(logits)`` (max-shifted);
* score of class k ``= sigmoid(to) * p[k]``; a (box, class) pair is a
  candidate when its score is at least ``thresh``.

Per image and class, candidates are ordered by score (descending), ties by
the box index ``(i*W + j)*A + a`` (ascending), and kept greedily: a candidate
survives unless an already kept box of the same class overlaps it with
IoU > ``nms_thresh``; at most ``max_det`` boxes are kept per class.

Every decision (threshold, IoU comparison) is taken in FP32, the precision
of the device kernels, on values computed step by step in FP32.
"""
from __future__ import annotations

from typing import List, Tuple

import numpy as np

F = np.float32


def sigmoid(x: np.ndarray) -> np.ndarray:
    x = x.astype(F)
    return (F(1) / (F(1) + np.exp(-x))).astype(F)


def softmax(z: np.ndarray) -> np.ndarray:
    """Softmax over the last axis, shifted by the maximum, FP32."""
    z = z.astype(F)
    e = np.exp(z - z.max(axis=-1, keepdims=True)).astype(F)
    return (e / e.sum(axis=-1, keepdims=True, dtype=F)).astype(F)


def decode(y: np.ndarray, anchors: np.ndarray, num_classes: int) -> Tuple[np.ndarray, np.ndarray]:
    """y: [N, A*(5+C), H, W] region output.  Returns boxes [N, H*W*A, 4]
    (x, y, w, h) and scores [N, H*W*A, C], box index (i*W + j)*A + a."""
    n, ch, h, w = y.shape
    A = len(anchors) // 2
    C = num_classes
    assert ch == A * (5 + C)
    t = y.astype(F).reshape(n, A, 5 + C, h, w).transpose(0, 3, 4, 1, 2)  # [N, H, W, A, 5+C]
    jj = np.arange(w, dtype=F).reshape(1, 1, w, 1)
    ii = np.arange(h, dtype=F).reshape(1, h, 1, 1)
    aw = np.asarray(anchors[0::2], dtype=F).reshape(1, 1, 1, A)
    ah = np.asarray(anchors[1::2], dtype=F).reshape(1, 1, 1, A)
    bx = ((jj + sigmoid(t[..., 0])) / F(w)).astype(F)
    by = ((ii + sigmoid(t[..., 1])) / F(h)).astype(F)
    bw = ((aw * np.exp(t[..., 2])) / F(w)).astype(F)
    bh = ((ah * np.exp(t[..., 3])) / F(h)).astype(F)
    obj = sigmoid(t[..., 4])
    p = softmax(t[..., 5:])
    scores = (obj[..., None] * p).astype(F)
    boxes = np.stack([bx, by, bw, bh], axis=-1)
    return boxes.reshape(n, h * w * A, 4), scores.reshape(n, h * w * A, C)


def iou(b1: np.ndarray, b2: np.ndarray) -> F:
    """Intersection over union of two (x, y, w, h) centre boxes, FP32."""
    l1, r1 = F(b1[0] - b1[2] / F(2)), F(b1[0] + b1[2] / F(2))
    t1, d1 = F(b1[1] - b1[3] / F(2)), F(b1[1] + b1[3] / F(2))
    l2, r2 = F(b2[0] - b2[2] / F(2)), F(b2[0] + b2[2] / F(2))
    t2, d2 = F(b2[1] - b2[3] / F(2)), F(b2[1] + b2[3] / F(2))
    iw = F(max(F(0), F(min(r1, r2) - max(l1, l2))))
    ih = F(max(F(0), F(min(d1, d2) - max(t1, t2))))
    inter = F(iw * ih)
    union = F(F(b1[2] * b1[3]) + F(b2[2] * b2[3]) - inter)
    return F(inter / union) if union > 0 else F(0)


def detect(y: np.ndarray, anchors, num_classes: int, thresh: float, nms_thresh: float,
           max_det: int) -> List[List[Tuple[int, int, float, np.ndarray]]]:
    """Per image, the kept detections as (class, box index, score, box),
    ordered by class, then score descending, then box index."""
    boxes, scores = decode(y, np.asarray(anchors, dtype=F), num_classes)
    out = []
    for n in range(y.shape[0]):
        dets = []
        for k in range(num_classes):
            s = scores[n, :, k]
            cand = [int(b) for b in np.nonzero(s >= F(thresh))[0]]
            cand.sort(key=lambda b: (-float(s[b]), b))
            kept: List[int] = []
            for b in cand:
                if len(kept) == max_det:
                    break
                if all(iou(boxes[n, b], boxes[n, q]) <= F(nms_thresh) for q in kept):
                    kept.append(b)
            dets += [(k, b, float(s[b]), boxes[n, b].copy()) for b in kept]
        out.append(dets)
    return out
