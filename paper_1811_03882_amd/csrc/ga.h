// Genetic search over per-layer CPU/GPU placements: the paper's offload
// search (Sec. 3.3 and Sec. 4; parameters and fitness in Sec. 5.1.2).  A gene
// holds one bit per layer, 1 = the layer runs on the GPU.  Host code only.
#pragma once

#include <cstdint>
#include <functional>

namespace dnga {

struct Params {
    int population;     // M
    int generations;    // T
    double crossover;   // Pc: probability that a selected pair is crossed at one point
    double mutation;    // Pm: probability that one gene value flips
    double timeout_s;   // a measurement over this (or a failed one) scores as penalty_s
    double penalty_s;
    uint64_t seed;
};

// SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom number
// generators", OOPSLA 2014): the state advances by the golden-ratio increment
// and the output is the state passed through the variant-13 finalizer.
uint64_t splitmix64(uint64_t *state);
// Uniform double in [0, 1) from the top 53 bits of one draw.
double uniform(uint64_t *state);
// Fitness of a measured time: (time)^(-1/2), as 1 / sqrt(time).
double fitness(double seconds);

// Draw the initial population: M genes of L values, each value the top bit
// of one draw, gene by gene.
void initial_population(const Params &p, int L, uint8_t *pop, uint64_t *state);

// The next generation from a measured one (pop[M][L], seconds[M]):
//   next[0] = the fittest gene (elite; the first one on ties), unchanged;
//   then pairs of children until M genes: two parents by roulette on the
//   fitness (each pick one draw), a crossover draw, and with probability Pc a
//   cut point 1 + draw % (L - 1) (one draw; L >= 2) after which the two
//   children swap tails; then every value of the first child and then of the
//   second flips with probability Pm (one draw per value); the second child
//   of the last pair is dropped when M - 1 is odd.
void next_generation(const Params &p, int L, const uint8_t *pop, const double *seconds, uint8_t *next,
                     uint64_t *state);

struct Result {
    double best_seconds = 0;
    int evaluations = 0;  // distinct genes measured
    int memo_hits = 0;    // genes scored from an earlier measurement
};

// Run T generations.  measure(gene, timeout_s) returns seconds; a negative
// value is a failed run (scored as penalty_s), NaN aborts the search (returns
// false).  Each distinct gene is measured once (memo).  best receives the
// fittest gene seen (first measured among ties), gen_best[g] (may be null)
// the best score of generation g.
bool search(const Params &p, int L, const std::function<double(const uint8_t *, double)> &measure, uint8_t *best,
            double *gen_best, Result *res);

}  // namespace dnga
