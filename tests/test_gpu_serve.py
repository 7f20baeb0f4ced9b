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
