"""Pins of the oracle's genetic placement search (oracle/ga.py), CPU only.

The paper prints no run of its GA, so each pin checks a property its
description fixes (Sec. 3.3, Sec. 4, Sec. 5.1.2): the generator against its
published outputs, fitness = time^(-1/2) through the selection frequencies
it must produce, the elite carried over unchanged, one-point crossover,
value-wise mutation at rate Pm, the memo, the timeout penalty, and on short
genes the search's answer against brute force.  Every pin takes the module
under test as an argument so that the planted mutants at the bottom (copies
of oracle/ga.py with one slip each) can be run through the same pins.
"""
import math
import os
import random
import types

import pytest

import oracle.ga as ga_mod

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "splitmix64.txt")


def golden_vectors():
    out = []
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        v = [int(t) for t in line.split()]
        out.append((v[0], v[1:]))
    return out


# ------------------------------------------------------------------ pins


def pin_generator(ga):
    for seed, outs in golden_vectors():
        r = ga.SplitMix64(seed)
        assert [r.next() for _ in outs] == outs
    r = ga.SplitMix64(7)
    u = [r.uniform() for _ in range(40000)]
    assert min(u) >= 0.0 and max(u) < 1.0
    assert abs(sum(u) / len(u) - 0.5) < 0.01
    bits = [r.bit() for _ in range(40000)]
    assert abs(sum(bits) / len(bits) - 0.5) < 0.01


def pin_fitness(ga):
    assert ga.fitness(4.0) == 0.5
    assert ga.fitness(0.01) == 10.0
    assert ga.fitness(1000.0) == 1.0 / math.sqrt(1000.0)


def _pop(L, genes):
    return [list(g) for g in genes]


def pin_selection_follows_fitness(ga):
    # two genes with times 1 and 4: fitness 1 and 1/2, so parents come from
    # gene 0 twice as often (time^-1 would give 4:1, a uniform pick 1:1)
    L = 6
    pop = _pop(L, [[0] * L, [1] * L])
    rng = ga.SplitMix64(11)
    counts = [0, 0]
    for _ in range(3000):
        nxt = ga.next_generation(pop, [1.0, 4.0], 0.0, 0.0, rng)
        for g in nxt[1:]:
            counts[g[0]] += 1
    frac = counts[0] / sum(counts)
    assert abs(frac - 2.0 / 3.0) < 0.02, frac


def pin_roulette_proportions(ga):
    fit = [1.0, 2.0, 3.0, 4.0]
    rng = ga.SplitMix64(3)
    n = 40000
    c = [0] * 4
    for _ in range(n):
        c[ga.roulette(fit, rng)] += 1
    for i in range(4):
        assert abs(c[i] / n - fit[i] / 10.0) < 0.01, c


def pin_elite(ga):
    L = 8
    rnd = random.Random(5)
    genes = [[rnd.randint(0, 1) for _ in range(L)] for _ in range(10)]
    secs = [rnd.uniform(1.0, 2.0) for _ in range(10)]
    secs[7] = 0.5
    rng = ga.SplitMix64(1)
    for Pc, Pm in ((0.9, 0.05), (1.0, 1.0), (0.0, 0.0)):
        nxt = ga.next_generation(_pop(L, genes), secs, Pc, Pm, rng)
        assert len(nxt) == 10
        assert nxt[0] == genes[7]


def pin_copies_without_operators(ga):
    L = 7
    rnd = random.Random(9)
    genes = [[rnd.randint(0, 1) for _ in range(L)] for _ in range(9)]
    secs = [rnd.uniform(0.1, 3.0) for _ in range(9)]
    rng = ga.SplitMix64(2)
    for _ in range(50):
        nxt = ga.next_generation(_pop(L, genes), secs, 0.0, 0.0, rng)
        assert all(g in genes for g in nxt)


def pin_one_point_crossover(ga):
    # parents all-0 and all-1: a crossed child is 0^k 1^(L-k) or 1^k 0^(L-k)
    # with 1 <= k <= L-1, and the two children of a pair complement each other
    L = 9
    pop = _pop(L, [[0] * L, [1] * L, [1] * L])
    rng = ga.SplitMix64(4)
    cuts = set()
    for _ in range(400):
        nxt = ga.next_generation(pop, [1.0, 1.0, 1.0], 1.0, 0.0, rng)
        c1, c2 = nxt[1], nxt[2]
        for c in (c1, c2):
            k = next((j for j in range(1, L) if c[j] != c[0]), L)
            assert all(c[j] == c[0] for j in range(k)) and all(c[j] != c[0] for j in range(k, L))
            if c1 != c2:
                assert 1 <= k <= L - 1
                cuts.add(k)
        assert c1 == c2 or all(a != b for a, b in zip(c1, c2))
    assert cuts == set(range(1, L))


def pin_mutation(ga):
    L = 10
    M = 21
    pop = _pop(L, [[0] * L for _ in range(M)])
    rng = ga.SplitMix64(6)
    ones = total = full = 0
    for _ in range(300):
        nxt = ga.next_generation(pop, [1.0] * M, 0.0, 0.25, rng)
        for g in nxt[1:]:
            ones += sum(g)
            total += L
            full += sum(g) == L
    assert abs(ones / total - 0.25) < 0.01
    assert full < 5  # values flip one by one, not whole genes
    nxt = ga.next_generation(_pop(L, [[0, 1] * 5, [1, 0] * 5]), [1.0, 2.0], 0.0, 1.0, rng)
    for g in nxt[1:]:
        assert g in ([1, 0] * 5, [0, 1] * 5)


def _landscape(L, seed):
    rnd = random.Random(seed)
    table = {}

    def t(gene):
        key = tuple(gene)
        if key not in table:
            table[key] = rnd.uniform(0.01, 1.0)
        return table[key]
    return t


def pin_memo_and_monotone(ga):
    L = 12
    t = _landscape(L, 3)
    calls = []

    def measure(gene, timeout):
        calls.append(tuple(gene))
        return t(gene)
    best, best_t, gen_best, n_eval, hits = ga.search(L, measure, M=30, T=20, seed=8)
    assert len(calls) == len(set(calls)) == n_eval
    assert n_eval + hits == 30 * 20
    assert best_t == min(t(g) for g in calls) and t(best) == best_t
    assert all(b >= a for a, b in zip(gen_best[1:], gen_best[:-1]))  # elite: never worse


def pin_timeout_penalty(ga):
    # the fastest genes take longer than the limit: they score 1000 s
    L = 6

    def measure(gene, timeout):
        s = sum(gene)
        if s >= 5:
            return timeout * 2.0
        if s == 0:
            return -1.0  # a failed run
        return 10.0 - s
    best, best_t, gen_best, n_eval, hits = ga.search(L, measure, M=16, T=12, timeout_s=9.5, seed=2)
    assert sum(best) == 4 and best_t == 6.0
    # every run over the limit (or failing): every score is the penalty
    best, best_t, gen_best, _, _ = ga.search(L, lambda g, to: 2.0 * to if sum(g) % 2 else -1.0, M=8, T=3,
                                             timeout_s=9.5, seed=5)
    assert best_t == 1000.0 and gen_best == [1000.0] * 3


def pin_brute_force_small(ga):
    # L = 4: 16 genes; the search's answer is the best of all of them
    for seed in range(4):
        t = _landscape(4, 100 + seed)
        allt = {}
        for k in range(16):
            g = tuple((k >> j) & 1 for j in range(4))
            allt[g] = t(g)
        best, best_t, _, _, _ = ga.search(4, lambda g, to: t(g), M=16, T=20, seed=seed)
        assert best_t == min(allt.values()) and allt[best] == best_t


PINS = [pin_generator, pin_fitness, pin_selection_follows_fitness, pin_roulette_proportions, pin_elite,
        pin_copies_without_operators, pin_one_point_crossover, pin_mutation, pin_memo_and_monotone,
        pin_timeout_penalty, pin_brute_force_small]


@pytest.mark.parametrize("pin", PINS, ids=[p.__name__ for p in PINS])
def test_oracle_ga_pin(pin):
    pin(ga_mod)


# ------------------------------------------------------------------ planted mutants

MUTANTS = {
    "fitness_inverse_time": ("return 1.0 / math.sqrt(seconds)", "return 1.0 / seconds"),
    "no_elite": ("nxt = [list(pop[elite])]", "nxt = []"),
    "elite_is_slowest": ("if seconds[i] < seconds[elite]:", "if seconds[i] > seconds[elite]:"),
    "roulette_uniform": ("    target = rng.uniform() * total\n", "    return int(rng.uniform() * len(fit))\n"),
    "cut_may_be_zero": ("cut = 1 + rng.next() % (L - 1)", "cut = rng.next() % L"),
    "crossover_rate_inverted": ("if rng.uniform() < Pc and L >= 2:", "if rng.uniform() >= Pc and L >= 2:"),
    "mutation_per_gene": ("            for j in range(L):\n                if rng.uniform() < Pm:\n"
                          "                    child[j] = 1 - child[j]",
                          "            if rng.uniform() < Pm:\n                for j in range(L):\n"
                          "                    child[j] = 1 - child[j]"),
    "no_memo": ("            if key in memo:", "            if False:"),
    "timeout_ignored": ("if t < 0 or t > timeout_s:", "if t < 0:"),
    "generator_shift": ("z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64",
                        "z = ((z ^ (z >> 29)) * 0x94D049BB133111EB) & MASK64"),
    "best_is_last": ("if best_t is None or t < best_t:", "if best_t is None or t <= best_t + 1e9:"),
}


def _mutant_module(name):
    old, new = MUTANTS[name]
    src = open(ga_mod.__file__).read()
    assert src.count(old) == 1, "mutation anchor not found: %s" % name
    mod = types.ModuleType("ga_mutant_" + name)
    exec(compile(src.replace(old, new), "<mutant %s>" % name, "exec"), mod.__dict__)
    return mod


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_ga_mutant_is_caught(name):
    mod = _mutant_module(name)
    caught = []
    for pin in PINS:
        try:
            pin(mod)
        except (AssertionError, ZeroDivisionError, IndexError, TypeError, StopIteration):
            caught.append(pin.__name__)
    assert caught, "mutant %s survived every pin" % name
