"""The paper's genetic offload search, written out plainly.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Sec. 3.3 and Sec. 4 describe the search; Sec. 5.1.2 gives its parameters.
A gene has one value per candidate (here: per layer; 1 = run on the GPU,
0 = leave on the CPU).  The steps, in the paper's order:

1. initialisation: M genes whose values are drawn at random as 0 or 1;
2. evaluation: each gene's program is run and timed; its fitness is
   (time)^(-1/2), so shorter is fitter without one fast gene taking over the
   selection; a run over the time limit counts as a fixed long time
   (1000 s for the paper's 3-minute limit); a gene seen before is not run
   again, its earlier time is reused;
3. selection: roulette selection on the fitness, plus the fittest gene of
   the generation carried over unchanged (elite);
4. crossover: with rate Pc, two selected genes swap the values after one
   point;
5. mutation: each value flips 0 <-> 1 with rate Pm;
6. steps 2-5 repeat for T generations; the answer is the fittest gene.

The paper gives no random generator and no draw order, so these are this
reading's choices, fixed so that a run is a pure function of the seed and the
measured times (the library's search follows the same order and must give
the same genes):
  * random numbers come from SplitMix64 (Steele, Lea and Flood, OOPSLA
    2014): state += 0x9E3779B97F4A7C15, then z ^= z >> 30, z *= 0xBF58476D1CE4E5B9,
    z ^= z >> 27, z *= 0x94D049BB133111EB, z ^= z >> 31 (64-bit arithmetic);
    a uniform number in [0, 1) is (draw >> 11) * 2^-53, a random bit the top
    bit of a draw;
  * initial values are drawn gene by gene, value by value;
  * a generation's next population starts with the elite (the first gene of
    least time); the rest are pairs: parent a, parent b (each one roulette
    draw: the first index whose running fitness sum exceeds u * total), the
    crossover draw (cross when u < Pc), the cut point 1 + draw mod (L - 1)
    when crossing (values from the cut on are swapped), then one mutation
    draw per value of the first child and one per value of the second; when
    only one place is left, the second child is dropped;
  * fitness is 1 / sqrt(time) and the running sums add fitness in index
    order, both in double precision;
  * the answer is the first-measured gene of least time.

Parity: pinned by tests/test_oracle_ga.py (SplitMix64's published outputs,
uniformity, exhaustive search on short genes, the elite invariant, the memo,
the selection frequencies against the fitness proportions, the crossover and
mutation structure), and planted mutants must fail those pins.
"""
from __future__ import annotations

import math
from typing import Callable, Dict, List, Sequence, Tuple

MASK64 = (1 << 64) - 1


class SplitMix64:
    """The SplitMix64 generator from its published definition."""

    def __init__(self, state: int):
        self.state = state & MASK64

    def next(self) -> int:
        self.state = (self.state + 0x9E3779B97F4A7C15) & MASK64
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
        return z ^ (z >> 31)

    def uniform(self) -> float:
        return (self.next() >> 11) * 2.0 ** -53

    def bit(self) -> int:
        return self.next() >> 63


def fitness(seconds: float) -> float:
    """(time)^(-1/2) (Sec. 5.1.2)."""
    return 1.0 / math.sqrt(seconds)


def initial_population(M: int, L: int, rng: SplitMix64) -> List[List[int]]:
    """Step 1: M genes of L random 0/1 values."""
    pop = []
    for _ in range(M):
        pop.append([rng.bit() for _ in range(L)])
    return pop


def roulette(fit: Sequence[float], rng: SplitMix64) -> int:
    """Roulette selection: index i with probability fit[i] / sum(fit)."""
    total = 0.0
    for f in fit:
        total += f
    target = rng.uniform() * total
    acc = 0.0
    for i, f in enumerate(fit):
        acc += f
        if target < acc:
            return i
    return len(fit) - 1


def next_generation(pop: List[List[int]], seconds: Sequence[float], Pc: float, Pm: float,
                    rng: SplitMix64) -> List[List[int]]:
    """Steps 3-5: elite, then roulette pairs, one-point crossover, mutation."""
    M, L = len(pop), len(pop[0])
    fit = [fitness(t) for t in seconds]
    elite = 0
    for i in range(M):
        if seconds[i] < seconds[elite]:
            elite = i
    nxt = [list(pop[elite])]
    while len(nxt) < M:
        a = roulette(fit, rng)
        b = roulette(fit, rng)
        c1, c2 = list(pop[a]), list(pop[b])
        if rng.uniform() < Pc and L >= 2:
            cut = 1 + rng.next() % (L - 1)
            c1[cut:], c2[cut:] = c2[cut:], c1[cut:]
        for child in (c1, c2):
            for j in range(L):
                if rng.uniform() < Pm:
                    child[j] = 1 - child[j]
        nxt.append(c1)
        if len(nxt) < M:
            nxt.append(c2)
    return nxt


def search(L: int, measure: Callable[[Tuple[int, ...], float], float], M: int = 30, T: int = 20,
           Pc: float = 0.9, Pm: float = 0.05, timeout_s: float = 180.0, penalty_s: float = 1000.0,
           seed: int = 0):
    """The whole search.  measure(gene, timeout_s) -> seconds (< 0: the run
    failed).  Returns (best gene, best time, per-generation best times,
    number of distinct genes measured, number of memo hits)."""
    rng = SplitMix64(seed)
    pop = initial_population(M, L, rng)
    memo: Dict[Tuple[int, ...], float] = {}
    best, best_t = None, None
    gen_best = []
    hits = 0
    for g in range(T):
        secs = []
        for gene in pop:
            key = tuple(gene)
            if key in memo:
                t = memo[key]
                hits += 1
            else:
                t = measure(key, timeout_s)
                if t < 0 or t > timeout_s:
                    t = penalty_s
                memo[key] = t
                if best_t is None or t < best_t:
                    best, best_t = key, t
            secs.append(t)
        gen_best.append(min(secs))
        if g + 1 < T:
            pop = next_generation(pop, secs, Pc, Pm, rng)
    return best, best_t, gen_best, len(memo), hits
