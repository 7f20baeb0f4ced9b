"""GPU serving loop: continuous batching over resolution buckets on the real
library.  Checks that every request completes, that batches overlap on the
device, that each result is the same alone and in the mix (BF16 tolerance),
and that sampled results match the FP64 oracle."""
import numpy as np
import pytest

import synth
from oracle import net as onet
from tests import gpu_util as G

pytestmark = pytest.mark.gpu

SIZES = (160, 224, 320, 416, 608)


@pytest.fixture(scope="module")
def env():
    torch = G.torch_cuda()
    from paper_1811_03882_amd import dn, serve
    net = synth.plain9()
    params = synth.make_params(net, synth.SEED_PLAIN)
    n = dn.Net(net.layers, net.in_c, 608, 608, 64, dtype=dn.BF16, use_graph=False)
    n.load_params(params)
    images = {}

    def image_of(r):
        if r.rid not in images:
            images[r.rid] = synth.serving_image(r.rid, r.size).astype(np.float32)[0]
        return images[r.rid]

    return torch, dn, serve, net, params, n, image_of


def test_mixed_trace_completes_overlaps_and_matches_alone(env):
    torch, dn, serve, net, params, n, image_of = env
    trace = synth.serving_trace(400, 2000.0, synth.SEED_SERVING)
    reqs = serve.make_requests(trace)
    ex = serve.DnExecutor(n, torch, budget_bytes=4 << 30, n_slots=4, image_of=image_of, max_batch=64,
                          max_size=608)
    sch = serve.Scheduler(ex, budget_bytes=4 << 30, sizes=SIZES, max_batch=64)
    st = sch.run(reqs)
    print("serving 400 req: %s" % st.as_dict())
    assert st.completed == 400 and st.failed == 0 and st.rejected == 0
    assert sch.max_inflight >= 2, "no two batches were ever in flight together"
    # the same request alone (batch 1, nothing else on the device) == in the mix
    picks = []
    for s in SIZES:
        picks += [r for r in reqs if r.size == s][:2]
    for r in picks:
        alone = serve.Request(r.rid, r.size, 0.0)
        ex1 = serve.DnExecutor(n, torch, budget_bytes=1 << 30, n_slots=1, image_of=image_of, max_batch=1,
                               max_size=r.size)
        serve.Scheduler(ex1, budget_bytes=1 << 30, sizes=SIZES, max_batch=1).run([alone])
        err = G.rel_l2(r.output, alone.output)
        print("request %d S=%d alone vs mix rel diff %.3e" % (r.rid, r.size, err))
        assert err < 2e-2
        del ex1
    # sampled results against the FP64 oracle
    for r in (picks[0], picks[-1]):
        ref = onet.forward(net, params, image_of(r)[None].astype(np.float64))[-1][0]
        err = G.rel_l2(r.output, ref)
        print("request %d S=%d vs oracle rel_l2 %.3e" % (r.rid, r.size, err))
        assert err < 2e-2


def test_fixed_slots_replay_graphs_overlap_on_device_and_match_alone_bitwise(env):
    """Fixed per-slot regions with captured graphs, on a batch-invariant net
    whose frames arrive in pinned host buffers: once every (slot, batch, size)
    graph is captured, a burst keeps several batches on the GPU at once (their
    event intervals intersect), and each sampled request's output has the same
    bits alone as in the mix."""
    torch, dn, serve, net, params, _, image_of = env
    pinned = {}

    def frame(r):
        key = (r.rid, r.size)
        if key not in pinned:
            pinned[key] = torch.from_numpy(synth.serving_image(r.rid, r.size).astype(np.float32)[0]).pin_memory()
        return pinned[key]
    mb = 16
    n = dn.Net(net.layers, net.in_c, 608, 608, mb, dtype=dn.BF16, use_graph=True, batch_invariant=True)
    n.load_params(params)
    ex = serve.DnExecutor(n, torch, budget_bytes=0, n_slots=4, image_of=frame, max_batch=mb, max_size=608,
                          fixed_slots=True, sizes=SIZES)
    assert ex.pool.numel() == 4 * ex.region
    for slot in range(4):
        for size in SIZES:
            for b in (1, 2, 4, 8, 16):
                ex.launch(slot, [serve.Request(10 ** 6 + size, size, 0.0)], b, size, 0)[0].synchronize()
    reqs = serve.make_requests(synth.serving_trace(300, 20000.0, synth.SEED_SERVING))
    for r in reqs:  # the frames are in their pinned buffers before they arrive
        frame(r)
    ex.intervals.clear()
    ref = torch.cuda.Event(enable_timing=True)
    ref.record()
    sch = serve.Scheduler(ex, ex.pool.numel(), SIZES, max_batch=mb)
    st = sch.run(reqs)
    torch.cuda.synchronize()
    ov = serve.device_overlap(ex.intervals, ref)
    print("fixed-slot serving 300 req: %s\ndevice: %s" % (st.as_dict(), ov))
    errors = [r.error for r in reqs if r.error]
    assert st.completed == 300 and st.failed == 0, errors[:3]
    assert ov["max_in_flight"] >= 2 and ov["overlap_frac"] > 0.0, "batches never overlapped on the device"
    picks = []
    for s in SIZES:
        picks += [r for r in reqs if r.size == s][:2]
    for r in picks:
        alone = serve.Request(r.rid, r.size, 0.0)
        serve.Scheduler(ex, ex.pool.numel(), SIZES, max_batch=1).run([alone])
        same = np.array_equal(r.output, alone.output)
        print("request %d S=%d alone vs in the mix: bitwise %s" % (r.rid, r.size, same))
        assert same
    del ex
    n.close()
