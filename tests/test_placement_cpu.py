"""Host logic of the layer placement, CPU only: the library's genetic search
(dn_ga_next_generation, dn_ga_search) against the oracle's (oracle/ga.py) on
the same seeds and the same fake measurements, which must give the same genes
bit for bit, and the host FP32 layer code (dn_cpu_conv2d, dn_cpu_maxpool)
against the FP64 oracle.  Nothing here touches a GPU."""
import random

import numpy as np
import pytest

import oracle
import oracle.ga as oga
from paper_1811_03882_amd import dn


def _fake(L, seed, timeout_every=0, fail_every=0):
    rnd = random.Random(seed)
    table = {}

    def t(gene, timeout):
        key = tuple(int(v) for v in gene)
        if key not in table:
            v = rnd.uniform(0.001, 0.2)
            h = hash(key)
            if timeout_every and h % timeout_every == 0:
                v = timeout * 1.5
            if fail_every and h % fail_every == 1:
                v = -1.0
            table[key] = v
        return table[key]
    return t


@pytest.mark.parametrize("L,M,T,Pc,Pm,seed", [
    (15, 30, 20, 0.9, 0.05, 0),     # the 9-layer net's 15 layers, the paper's parameters
    (75, 30, 20, 0.9, 0.05, 1),     # the residual net's 75 layers (paper: 75 loops)
    (1, 5, 4, 0.9, 0.5, 2),         # one gene value: no crossover point
    (6, 1, 5, 0.9, 0.05, 3),        # population of one: elite only
    (9, 7, 6, 0.0, 1.0, 4),         # mutation only, every value flips
    (9, 8, 6, 1.0, 0.0, 5),         # crossover only
    (12, 11, 9, 0.9, 0.05, 2 ** 63 + 12345),
])
def test_library_search_equals_oracle(L, M, T, Pc, Pm, seed):
    t_lib = _fake(L, seed, timeout_every=7, fail_every=11)
    t_ora = _fake(L, seed, timeout_every=7, fail_every=11)
    calls_lib = []

    def m_lib(g, to):
        calls_lib.append(tuple(int(v) for v in g))
        return t_lib(g, to)
    p = dn.ga_params(M, T, Pc, Pm, timeout_s=0.15, penalty_s=1000.0, seed=seed)
    best, gen, res = dn.ga_search(p, L, m_lib)
    obest, obest_t, ogen, oeval, ohits = oga.search(L, t_ora, M=M, T=T, Pc=Pc, Pm=Pm, timeout_s=0.15,
                                                    penalty_s=1000.0, seed=seed)
    assert tuple(int(v) for v in best) == obest
    assert res.best_seconds == obest_t
    assert list(gen) == ogen
    assert (res.evaluations, res.memo_hits) == (oeval, ohits)
    assert len(calls_lib) == len(set(calls_lib)) == res.evaluations


@pytest.mark.parametrize("seed", range(5))
def test_library_generation_step_equals_oracle(seed):
    rnd = random.Random(seed)
    L = rnd.randint(2, 40)
    M = rnd.randint(1, 33)
    pop = [[rnd.randint(0, 1) for _ in range(L)] for _ in range(M)]
    secs = [rnd.choice([rnd.uniform(1e-3, 2.0), 1000.0]) for _ in range(M)]
    Pc, Pm = rnd.random(), rnd.random() * 0.3
    state = rnd.getrandbits(64)
    p = dn.ga_params(M, 1, Pc, Pm, seed=0)
    nxt, st = dn.ga_next_generation(p, np.array(pop, dtype=np.uint8), np.array(secs), state)
    rng = oga.SplitMix64(state)
    onxt = oga.next_generation([list(g) for g in pop], secs, Pc, Pm, rng)
    assert nxt.tolist() == onxt
    assert st == rng.state


def test_search_rejects_bad_parameters():
    with pytest.raises(dn.DnError) as e:
        dn.ga_search(dn.ga_params(population=0), 5, lambda g, t: 1.0)
    assert e.value.status == dn.DN_EINVAL
    with pytest.raises(dn.DnError):
        dn.ga_search(dn.ga_params(crossover=1.5), 5, lambda g, t: 1.0)
    with pytest.raises(dn.DnError):
        dn.ga_search(dn.ga_params(timeout_s=0.0), 5, lambda g, t: 1.0)
    with pytest.raises(dn.DnError):
        dn.ga_next_generation(dn.ga_params(population=2), np.zeros((2, 3), np.uint8), np.array([1.0, -1.0]), 0)


def test_search_abort_from_measurement():
    with pytest.raises(dn.DnError) as e:
        dn.ga_search(dn.ga_params(population=4, generations=2), 5, lambda g, t: float("nan"))
    assert e.value.status == dn.DN_ESTATE


# ------------------------------------------------------------ host layer code


def _pad_nhwc(x, cp):
    n, c, h, w = x.shape
    out = np.zeros((n, h, w, cp), dtype=np.float32)
    out[..., :c] = np.transpose(x, (0, 2, 3, 1))
    return out


@pytest.mark.parametrize("n,c,h,w,k,cout,stride,pad,act", [
    (1, 3, 13, 11, 3, 16, 1, 1, dn.LEAKY),
    (2, 5, 9, 7, 3, 19, 2, 1, dn.LEAKY),      # channel tails on both sides, stride 2
    (1, 16, 8, 8, 1, 37, 1, 0, dn.LINEAR),    # 1x1, linear, cout % 16 != 0
    (3, 8, 6, 10, 3, 32, 1, 0, dn.LEAKY),     # no padding
    (1, 4, 1, 1, 3, 4, 1, 1, dn.LEAKY),       # one pixel: every tap but the centre is padding
])
def test_cpu_conv_matches_oracle(n, c, h, w, k, cout, stride, pad, act):
    rng = np.random.default_rng(c * 100 + cout)
    x = rng.uniform(-1, 1, (n, c, h, w))
    wt = rng.normal(0, np.sqrt(2.0 / (c * k * k)), (cout, c, k, k))
    b = rng.normal(0, 0.1, cout)
    ref = oracle.add_bias(oracle.conv2d(x, wt, stride, pad), b)
    if act == dn.LEAKY:
        ref = oracle.leaky(ref, 0.1)
    cp, cop = dn.channel_pad(dn.F32, c), dn.channel_pad(dn.F32, cout)
    ho, wo = (h + 2 * pad - k) // stride + 1, (w + 2 * pad - k) // stride + 1
    y = np.full((n, ho, wo, cop), np.nan, dtype=np.float32)
    d = dn.conv_desc(n, h, w, c, cout, k, stride, pad, activation=act, slope=0.1, dtype=dn.F32)
    dn.cpu_conv2d(d, _pad_nhwc(x.astype(np.float32), cp), wt.astype(np.float32), b.astype(np.float32), y)
    assert np.all(y[..., cout:] == 0.0)
    got = np.transpose(y[..., :cout], (0, 3, 1, 2)).astype(np.float64)
    # the oracle takes FP32-rounded x and w so the gate measures accumulation only
    ref32 = oracle.add_bias(oracle.conv2d(x.astype(np.float32), wt.astype(np.float32), stride, pad),
                            b.astype(np.float32))
    if act == dn.LEAKY:
        ref32 = oracle.leaky(ref32, 0.1)
    err = np.linalg.norm(got - ref32) / np.linalg.norm(ref32)
    assert err < 1e-6, err
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < 1e-5


@pytest.mark.parametrize("h,w,size,stride", [(13, 13, 2, 1), (8, 6, 2, 2), (7, 9, 3, 2), (5, 5, 3, 1)])
def test_cpu_maxpool_exact(h, w, size, stride):
    rng = np.random.default_rng(h * w)
    c = 6
    x = rng.integers(-50, 50, (2, c, h, w)).astype(np.float64) / 4.0
    ref = oracle.maxpool(x, size, stride)
    cp = dn.channel_pad(dn.F32, c)
    ho, wo = (h - 1) // stride + 1, (w - 1) // stride + 1
    y = np.zeros((2, ho, wo, cp), dtype=np.float32)
    dn.cpu_maxpool(2, h, w, c, size, stride, _pad_nhwc(x.astype(np.float32), cp), y)
    assert np.array_equal(np.transpose(y[..., :c], (0, 3, 1, 2)).astype(np.float64), ref)
