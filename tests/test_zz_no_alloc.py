"""The allocation-free detection entry point (dn_detect_noalloc: the decode's
scratch is the library's fixed per-GPU array instead of a caller workspace)
against dn_detect with a workspace, through the C ABI.  Kept boxes, indices
and counts must agree exactly (the same kernels run on the same inputs); two
calls in a row, the second on a smaller input, so that the scratch's left-over
contents from the first call cannot leak into the second."""
import numpy as np
import pytest

import synth
from tests import gpu_util as G

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dn():
    from paper_1811_03882_amd import dn as _dn
    G.torch_cuda()
    return _dn


def outputs(torch, n, C, max_det):
    return (torch.full((n, C, max_det, 5), -7.0, device="cuda"),
            torch.full((n, C, max_det), -7, dtype=torch.int32, device="cuda"),
            torch.full((n, C), -7, dtype=torch.int32, device="cuda"))


def run_pair(dn, y, A, C, thresh, nms, max_det):
    torch = G.torch_cuda()
    n, _, h, w = y.shape
    anchors = synth.region_anchors(A)
    yd = torch.from_numpy(np.ascontiguousarray(y, np.float32)).cuda()
    wsb = dn.detect_workspace(n, A, C, h, w)
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    ref = outputs(torch, n, C, max_det)
    dn.detect(yd, n, A, C, h, w, anchors, thresh, nms, max_det, ws, wsb, *ref)
    got = outputs(torch, n, C, max_det)
    dn.detect_noalloc(yd, n, A, C, h, w, anchors, thresh, nms, max_det, *got)
    torch.cuda.synchronize()
    cnt = ref[2].cpu().numpy()
    assert np.array_equal(got[2].cpu().numpy(), cnt)
    # entries past each count are left untouched by both calls (-7)
    assert np.array_equal(got[1].cpu().numpy(), ref[1].cpu().numpy())
    assert np.array_equal(got[0].cpu().numpy(), ref[0].cpu().numpy())
    return int(cnt.sum())


def test_noalloc_matches_workspace_call_twice(dn):
    big = synth.region_output(64, 5, 20, 13, 13, tag=31, clusters=3)
    small = synth.region_output(3, 5, 20, 7, 9, tag=32, clusters=2)
    kept_big = run_pair(dn, big, 5, 20, 0.2, 0.45, 50)
    kept_small = run_pair(dn, small, 5, 20, 0.2, 0.45, 50)
    print("kept boxes: %d (64 images 13x13), %d (3 images 7x9)" % (kept_big, kept_small))
    assert kept_big > 0 and kept_small > 0


def test_noalloc_rejects_inputs_over_its_scratch(dn):
    torch = G.torch_cuda()
    # 256 images x 845 boxes x (80 classes + 4) floats > 16 MiB
    n, A, C, h, w = 256, 5, 80, 13, 13
    assert dn.detect_workspace(n, A, C, h, w) > 16 << 20
    y = torch.zeros((1,), device="cuda")
    d, i, c = outputs(torch, 1, 1, 1)
    with pytest.raises(dn.DnError) as e:
        dn.detect_noalloc(y, n, A, C, h, w, synth.region_anchors(A), 0.2, 0.45, 10, d, i, c)
    assert e.value.status == dn.DN_EINVAL and "scratch" in str(e.value)
