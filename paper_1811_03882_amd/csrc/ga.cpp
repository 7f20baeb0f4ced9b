// Genetic placement search (see ga.h).  Selection, crossover and mutation
// follow the paper's description of its GA (Sec. 3.3, Sec. 4): roulette
// selection on the fitness plus an elite kept unchanged, one-point crossover
// at rate Pc, value-by-value mutation at rate Pm, a memo so that a gene seen
// before is not measured again, and a timeout scored as a fixed long time
// (Sec. 5.1.2).  The order of random draws is fixed so that a run is a pure
// function of the seed and the measurements.
#include "ga.h"

#include <cmath>
#include <cstring>
#include <map>
#include <string>
#include <vector>

namespace dnga {

uint64_t splitmix64(uint64_t *state)
{
    uint64_t z = (*state += 0x9e3779b97f4a7c15ULL);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

double uniform(uint64_t *state) { return (double)(splitmix64(state) >> 11) * 0x1.0p-53; }

double fitness(double seconds) { return 1.0 / std::sqrt(seconds); }

void initial_population(const Params &p, int L, uint8_t *pop, uint64_t *state)
{
    for (int i = 0; i < p.population; ++i)
        for (int j = 0; j < L; ++j) pop[(size_t)i * L + j] = (uint8_t)(splitmix64(state) >> 63);
}

static int roulette(const std::vector<double> &fit, double total, uint64_t *state)
{
    const double target = uniform(state) * total;
    double acc = 0.0;
    for (size_t i = 0; i < fit.size(); ++i) {
        acc += fit[i];
        if (target < acc) return (int)i;
    }
    return (int)fit.size() - 1;
}

void next_generation(const Params &p, int L, const uint8_t *pop, const double *seconds, uint8_t *next,
                     uint64_t *state)
{
    const int M = p.population;
    std::vector<double> fit(M);
    double total = 0.0;
    int elite = 0;
    for (int i = 0; i < M; ++i) {
        fit[i] = fitness(seconds[i]);
        total += fit[i];
        if (seconds[i] < seconds[elite]) elite = i;
    }
    std::memcpy(next, pop + (size_t)elite * L, L);
    std::vector<uint8_t> c1(L), c2(L);
    for (int k = 1; k < M;) {
        const int a = roulette(fit, total, state);
        const int b = roulette(fit, total, state);
        std::memcpy(c1.data(), pop + (size_t)a * L, L);
        std::memcpy(c2.data(), pop + (size_t)b * L, L);
        if (uniform(state) < p.crossover && L >= 2) {
            const int cut = 1 + (int)(splitmix64(state) % (uint64_t)(L - 1));
            for (int j = cut; j < L; ++j) std::swap(c1[j], c2[j]);
        }
        for (int j = 0; j < L; ++j)
            if (uniform(state) < p.mutation) c1[j] ^= 1;
        for (int j = 0; j < L; ++j)
            if (uniform(state) < p.mutation) c2[j] ^= 1;
        std::memcpy(next + (size_t)k++ * L, c1.data(), L);
        if (k < M) std::memcpy(next + (size_t)k++ * L, c2.data(), L);
    }
}

bool search(const Params &p, int L, const std::function<double(const uint8_t *, double)> &measure, uint8_t *best,
            double *gen_best, Result *res)
{
    const int M = p.population;
    uint64_t state = p.seed;
    std::vector<uint8_t> pop((size_t)M * L), next((size_t)M * L);
    std::vector<double> sec(M);
    std::map<std::string, double> memo;
    Result r;
    bool have_best = false;
    initial_population(p, L, pop.data(), &state);
    for (int g = 0; g < p.generations; ++g) {
        double gb = 0.0;
        for (int i = 0; i < M; ++i) {
            const uint8_t *gene = pop.data() + (size_t)i * L;
            const std::string key((const char *)gene, (size_t)L);
            auto it = memo.find(key);
            double t;
            if (it != memo.end()) {
                t = it->second;
                ++r.memo_hits;
            } else {
                t = measure(gene, p.timeout_s);
                if (std::isnan(t)) return false;
                if (t < 0.0 || t > p.timeout_s) t = p.penalty_s;
                memo.emplace(key, t);
                ++r.evaluations;
                if (!have_best || t < r.best_seconds) {
                    r.best_seconds = t;
                    std::memcpy(best, gene, L);
                    have_best = true;
                }
            }
            sec[i] = t;
            if (i == 0 || t < gb) gb = t;
        }
        if (gen_best) gen_best[g] = gb;
        if (g + 1 < p.generations) {
            next_generation(p, L, pop.data(), sec.data(), next.data(), &state);
            pop.swap(next);
        }
    }
    if (res) *res = r;
    return true;
}

}  // namespace dnga
