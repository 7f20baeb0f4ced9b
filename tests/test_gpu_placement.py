"""GPU tests of the layer placement (the paper's offload search applied to the
net's layers, Sec. 3.2-3.3, Sec. 4, Sec. 5.1.2): placed forwards against the
FP64 oracle for several genes (FP32 gate 1e-5 end to end), the all-GPU gene
against the resident forward (bitwise), the copies each gene implies under the
transfer rule, the time limit, and the GA over a small net's placements.
"""
import numpy as np
import pytest

import synth
from oracle import net as onet
from tests import gpu_util as G

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dn():
    from paper_1811_03882_amd import dn as _dn
    G.torch_cuda()
    return _dn


def placed_net(dn, net, seed, batch, h, w):
    torch = G.torch_cuda()
    n = dn.Net(net.layers, net.in_c, h, w, batch, dtype=dn.F32, leaky_slope=net.leaky_slope, bn_eps=net.bn_eps)
    params = synth.make_params(net, seed)
    n.load_params(params)
    arena = G.empty_bytes(max(n.placed_arena_bytes(batch, h, w), n.arena_bytes(batch, h, w)))
    n.bind_arena(arena)
    torch.cuda.synchronize()
    return n, params


def genes_for(L, seed):
    rng = np.random.default_rng(seed)
    gs = [np.ones(L, np.uint8), np.zeros(L, np.uint8), np.arange(L, dtype=np.uint8) % 2,
          1 - (np.arange(L, dtype=np.uint8) % 2)]
    gs += [rng.integers(0, 2, L).astype(np.uint8) for _ in range(4)]
    return gs


@pytest.mark.parametrize("which", ["plain9", "residual"])
def test_placed_forward_matches_oracle(dn, which):
    if which == "plain9":
        net, seed, batch, h, w = synth.plain9(), synth.SEED_PLAIN, 2, 64, 96
    else:
        net, seed, batch, h, w = synth.residual52(units=(1, 2), widths=(32, 64), in_hw=32), synth.SEED_RESIDUAL, 2, 32, 32
    n, params = placed_net(dn, net, seed, batch, h, w)
    x = synth.make_input(net, batch, seed, h=h, w=w)
    ref = onet.forward(net, params, x)[-1]
    xh = np.ascontiguousarray(x.astype(np.float32))
    y = np.empty((batch,) + n.output_shape(h, w), np.float32)
    L = len(net.layers)
    for gene in genes_for(L, 7):
        print("gene", "".join(map(str, gene)), flush=True)
        y.fill(np.nan)
        n.forward_placed(gene, xh, batch, h, w, y)
        err = G.rel_l2(y, ref)
        print("  rel_l2 %.3e" % err)
        assert err < 1e-5, ("".join(map(str, gene)), err)
    n.close()


def test_all_gpu_gene_is_the_resident_forward(dn):
    torch = G.torch_cuda()
    net, seed, batch, h, w = synth.plain9(), synth.SEED_PLAIN, 2, 96, 64
    n, _ = placed_net(dn, net, seed, batch, h, w)
    x = synth.make_input(net, batch, seed, h=h, w=w).astype(np.float32)
    y = np.empty((batch,) + n.output_shape(h, w), np.float32)
    n.forward_placed(np.ones(len(net.layers), np.uint8), x, batch, h, w, y)
    yd = torch.empty(y.shape, dtype=torch.float32, device="cuda")
    n.forward(G.dev(x), batch, h, w, yd)
    torch.cuda.synchronize()
    assert np.array_equal(yd.cpu().numpy(), y)
    n.close()


def test_transfers_follow_the_rule(dn):
    net, batch, h, w = synth.plain9(), 1, 64, 64
    n, _ = placed_net(dn, net, synth.SEED_PLAIN, batch, h, w)
    L = len(net.layers)
    c, ho, wo = n.output_shape(h, w)
    xb, yb = batch * 3 * h * w * 4, batch * c * ho * wo * 4
    # all on the GPU: the image in, the result out, nothing else
    assert n.placed_transfers(np.ones(L, np.uint8), batch, h, w) == (1, 1, xb, yb)
    # all on the host: nothing crosses
    assert n.placed_transfers(np.zeros(L, np.uint8), batch, h, w) == (0, 0, 0, 0)
    # one host layer in the middle (the 2x2/2 pool after conv 2): its input
    # comes back once and its output goes over once
    g = np.ones(L, np.uint8)
    g[3] = 0
    conv2_out = batch * (h // 2) * (w // 2) * dn.channel_pad(dn.F32, 32) * 4
    pool_out = batch * (h // 4) * (w // 4) * dn.channel_pad(dn.F32, 32) * 4
    assert n.placed_transfers(g, batch, h, w) == (2, 2, xb + pool_out, yb + conv2_out)
    # host first half, GPU second half: one crossing in the middle and the result out
    g = np.zeros(L, np.uint8)
    g[8:] = 1
    h2d, d2h, _, b = n.placed_transfers(g, batch, h, w)
    assert (h2d, d2h, b) == (1, 1, yb)
    with pytest.raises(dn.DnError):
        n.placed_transfers(np.ones(L - 1, np.uint8), batch, h, w)
    with pytest.raises(dn.DnError):
        n.placed_transfers(np.full(L, 2, np.uint8), batch, h, w)
    n.close()


def test_timeout_and_errors(dn):
    net, batch, h, w = synth.plain9(), 1, 64, 64
    n, params = placed_net(dn, net, synth.SEED_PLAIN, batch, h, w)
    L = len(net.layers)
    x = synth.make_input(net, batch, synth.SEED_PLAIN, h=h, w=w).astype(np.float32)
    y = np.empty((batch,) + n.output_shape(h, w), np.float32)
    with pytest.raises(dn.DnError) as e:
        n.forward_placed(np.zeros(L, np.uint8), x, batch, h, w, y, timeout_s=1e-9)
    assert e.value.status == dn.DN_ETIMEDOUT
    n.forward_placed(np.zeros(L, np.uint8), x, batch, h, w, y)  # still usable
    ref = onet.forward(net, params, x.astype(np.float64))[-1]
    assert G.rel_l2(y, ref) < 1e-5
    bf = dn.Net(net.layers, 3, h, w, 1, dtype=dn.BF16)
    with pytest.raises(dn.DnError) as e:
        bf.placed_arena_bytes(1, h, w)
    assert e.value.status == dn.DN_EUNSUPPORTED
    bf.close()
    with pytest.raises(dn.DnError) as e:
        n.forward_placed(np.ones(L + 1, np.uint8), x, batch, h, w, y)
    assert e.value.status == dn.DN_EINVAL
    n.close()


def test_ga_place_small(dn):
    net, batch, h, w = synth.plain9(), 1, 64, 64
    n, params = placed_net(dn, net, synth.SEED_PLAIN, batch, h, w)
    L = len(net.layers)
    x = synth.make_input(net, batch, synth.SEED_PLAIN, h=h, w=w).astype(np.float32)
    y = np.empty((batch,) + n.output_shape(h, w), np.float32)
    p = dn.ga_params(population=8, generations=4, timeout_s=30.0, seed=3)
    best, gen, res = n.ga_place(p, x, batch, h, w, y, reps=1)
    print("best gene", "".join(map(str, best)), "%.3f ms" % (res.best_seconds * 1e3), "evaluations", res.evaluations,
          "memo hits", res.memo_hits, "per generation", gen.tolist())
    assert res.evaluations + res.memo_hits == 8 * 4
    assert all(b >= a for a, b in zip(gen[1:], gen[:-1]))
    assert res.best_seconds == gen.min() and 0 < res.best_seconds < 30.0
    n.forward_placed(best, x, batch, h, w, y)
    ref = onet.forward(net, params, x.astype(np.float64))[-1]
    assert G.rel_l2(y, ref) < 1e-5
    n.close()
