// Sanitizer run of the library's host-only code (built with
// -fsanitize=address,undefined by tests/test_sanitizers.py): the host FP32
// layer code of the placement (conv against a plain loop nest on ragged
// shapes, pool, add, layout changes) and the genetic search (edge-case
// parameters, a fake timer).  Exits non-zero on a mismatch; the sanitizers
// abort on any memory or undefined-behaviour error.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "cpu_layers.h"
#include "ga.h"

static int failures = 0;
#define CHECK(c)                                                   \
    do {                                                           \
        if (!(c)) {                                                \
            std::fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
            ++failures;                                            \
        }                                                          \
    } while (0)

static void conv_case(int n, int H, int W, int cin_p, int cout_p, int R, int stride, int pad, int act, unsigned seed)
{
    std::mt19937 g(seed);
    std::uniform_real_distribution<float> u(-1.f, 1.f);
    const int Ho = (H + 2 * pad - R) / stride + 1, Wo = (W + 2 * pad - R) / stride + 1;
    std::vector<float> x((size_t)n * H * W * cin_p), w((size_t)cout_p * R * R * cin_p), b(cout_p);
    for (auto &v : x) v = u(g);
    for (auto &v : w) v = u(g);
    for (auto &v : b) v = u(g);
    // w as [co][r][s][c]
    auto wval = [&](int co, int r, int s, int c) { return w[(((size_t)co * R + r) * R + s) * cin_p + c]; };
    std::vector<float> packed(w.size()), y((size_t)n * Ho * Wo * cout_p, NAN);
    dncpu::pack_weights(wval, cout_p, R, R, cin_p, packed.data());
    dncpu::conv(x.data(), n, H, W, cin_p, packed.data(), b.data(), cout_p, R, R, stride, pad, act, 0.1f, y.data(), Ho,
                Wo);
    double err = 0, ref2 = 0;
    for (int in = 0; in < n; ++in)
        for (int i = 0; i < Ho; ++i)
            for (int j = 0; j < Wo; ++j)
                for (int co = 0; co < cout_p; ++co) {
                    double acc = b[co];
                    for (int r = 0; r < R; ++r)
                        for (int s = 0; s < R; ++s) {
                            const int ii = i * stride - pad + r, jj = j * stride - pad + s;
                            if (ii < 0 || ii >= H || jj < 0 || jj >= W) continue;
                            for (int c = 0; c < cin_p; ++c)
                                acc += (double)x[(((size_t)in * H + ii) * W + jj) * cin_p + c] * wval(co, r, s, c);
                        }
                    if (act && !(acc > 0)) acc *= 0.1;
                    const double got = y[(((size_t)in * Ho + i) * Wo + j) * cout_p + co];
                    err += (got - acc) * (got - acc);
                    ref2 += acc * acc;
                }
    CHECK(std::sqrt(err / ref2) < 1e-5);
}

int main()
{
    conv_case(1, 7, 5, 4, 16, 3, 1, 1, 1, 1);
    conv_case(2, 9, 11, 12, 20, 3, 2, 1, 1, 2);   // cout tail of 4
    conv_case(1, 4, 4, 8, 4, 1, 1, 0, 0, 3);      // tail only
    conv_case(3, 1, 1, 4, 33, 3, 1, 1, 1, 4);     // one pixel, tail of 1
    conv_case(1, 13, 13, 32, 48, 3, 1, 0, 1, 5);  // no padding
    // pool / add / layout
    {
        std::vector<float> x(2 * 5 * 7 * 4), y(2 * 5 * 7 * 4);
        for (size_t i = 0; i < x.size(); ++i) x[i] = (float)((i * 7919) % 23) - 11.f;
        dncpu::maxpool(x.data(), 2, 5, 7, 4, 2, 1, y.data(), 5, 7);
        for (int c = 0; c < 4; ++c) CHECK(y[(4 * 7 + 6) * 4 + c] == x[(4 * 7 + 6) * 4 + c]);  // corner window
        std::vector<float> z(x.size());
        dncpu::add(x.data(), y.data(), z.data(), x.size());
        for (size_t i = 0; i < x.size(); ++i) CHECK(z[i] == x[i] + y[i]);
        std::vector<float> nchw(2 * 3 * 5 * 7), back(nchw.size());
        for (size_t i = 0; i < nchw.size(); ++i) nchw[i] = (float)i;
        dncpu::ingest(nchw.data(), 2, 3, 5, 7, 4, x.data());
        dncpu::egress(x.data(), 2, 3, 5, 7, 4, back.data());
        for (size_t i = 0; i < nchw.size(); ++i) CHECK(back[i] == nchw[i]);
    }
    // genetic search: edge parameters and a fake timer
    for (int L : {1, 2, 15, 75}) {
        for (int M : {1, 2, 7, 30}) {
            dnga::Params p{M, 5, 0.9, 0.05, 0.5, 1000.0, (uint64_t)(L * 131 + M)};
            std::vector<uint8_t> best(L);
            std::vector<double> gen(p.generations);
            dnga::Result r;
            auto fake = [&](const uint8_t *g, double) {
                int ones = 0;
                for (int j = 0; j < L; ++j) ones += g[j];
                return ones == L ? 2.0 : 0.01 + 0.001 * (L - ones) + (g[0] ? -1.0 : 0.0) * 0.0;
            };
            CHECK(dnga::search(p, L, fake, best.data(), gen.data(), &r));
            CHECK(r.evaluations + r.memo_hits == M * p.generations);
            for (int g = 1; g < p.generations; ++g) CHECK(gen[g] <= gen[g - 1]);
        }
    }
    if (failures) std::fprintf(stderr, "%d checks failed\n", failures);
    else std::printf("host code checks passed\n");
    return failures ? 1 : 0;
}
