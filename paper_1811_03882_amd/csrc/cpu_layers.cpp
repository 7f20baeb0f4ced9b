// Host FP32 layer kernels for the CPU side of the layer placement (see
// cpu_layers.h).  A direct convolution over NHWC: each task owns one block of
// 16 output channels and a run of output pixels; the block's weights
// ([R][S][cin_p][16], contiguous) stay in the core's cache while the run's
// pixels stream past, six pixels at a time held in registers (6 x 16 FP32
// accumulators), one broadcast input value times one 16-wide weight row per
// step.  Vector code is written with the compiler's vector extensions.
#include "cpu_layers.h"

#include <algorithm>
#include <atomic>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <mutex>
#include <thread>
#include <vector>

namespace dncpu {

// ---------------------------------------------------------------- worker pool

namespace {

class Pool {
public:
    explicit Pool(int n) : n_(n)
    {
        for (int i = 1; i < n; ++i) workers_.emplace_back([this] { loop(); });
    }
    int size() const { return n_; }

    void run(int tasks, const std::function<void(int)> &body)
    {
        if (tasks <= 0) return;
        std::lock_guard<std::mutex> one(call_mu_);  // one parallel region at a time
        if (workers_.empty() || tasks == 1) {
            for (int t = 0; t < tasks; ++t) body(t);
            return;
        }
        {
            std::lock_guard<std::mutex> g(mu_);
            body_ = &body;
            tasks_ = tasks;
            next_.store(0);
            active_ = (int)workers_.size();
            ++gen_;
        }
        cv_.notify_all();
        work();
        std::unique_lock<std::mutex> g(mu_);
        done_.wait(g, [&] { return active_ == 0; });
        body_ = nullptr;
    }

private:
    void work()
    {
        for (;;) {
            const int t = next_.fetch_add(1);
            if (t >= tasks_) break;
            (*body_)(t);
        }
    }
    void loop()
    {
        unsigned seen = 0;
        for (;;) {
            {
                std::unique_lock<std::mutex> g(mu_);
                cv_.wait(g, [&] { return gen_ != seen; });
                seen = gen_;
            }
            work();
            std::lock_guard<std::mutex> g(mu_);
            if (--active_ == 0) done_.notify_all();
        }
    }

    int n_;
    std::vector<std::thread> workers_;
    std::mutex call_mu_, mu_;
    std::condition_variable cv_, done_;
    const std::function<void(int)> *body_ = nullptr;
    int tasks_ = 0, active_ = 0;
    unsigned gen_ = 0;
    std::atomic<int> next_{0};
};

int env_threads()
{
    for (const char *name : {"DN_CPU_THREADS", "OMP_NUM_THREADS"}) {
        const char *v = getenv(name);
        if (v && atoi(v) > 0) return std::min(atoi(v), 256);
    }
    const unsigned hw = std::thread::hardware_concurrency();
    return (int)std::max(1u, std::min(hw, 16u));
}

Pool &pool()
{
    // Workers wait on a condition variable for the life of the process; the
    // pool is never destroyed, so no join runs during static destruction.
    static Pool *p = new Pool(env_threads());
    return *p;
}

}  // namespace

int threads() { return pool().size(); }

void parallel_for(int tasks, const std::function<void(int)> &body) { pool().run(tasks, body); }

// ---------------------------------------------------------------- conv

typedef float v8 __attribute__((vector_size(32)));
typedef float v8u __attribute__((vector_size(32), aligned(4)));

static inline v8 ld8(const float *p) { return *(const v8u *)p; }
static inline void st8(float *p, v8 v) { *(v8u *)p = v; }

namespace {

constexpr int CB = 16;  // output channels per block
constexpr int PB = 6;   // output pixels per register block

struct ConvCtx {
    const float *x, *w, *bias, *zeros;
    float *y;
    int n, H, W, cin_p, cout_p, R, S, stride, pad, act, Ho, Wo;
    float slope;
    int M, nfull, rem;
};

// Input row pointers of the PB pixels m0.. for tap (r, s): a pixel outside the
// output range, or a tap in the zero padding, reads the zero row.
struct PixBase { int n, bi, bj; bool valid; };

inline void pix_bases(const ConvCtx &c, int m0, PixBase *pb)
{
    for (int q = 0; q < PB; ++q) {
        const int m = m0 + q;
        pb[q].valid = m < c.M;
        if (!pb[q].valid) { pb[q].n = pb[q].bi = pb[q].bj = 0; continue; }
        const int j = m % c.Wo, t = m / c.Wo, i = t % c.Ho;
        pb[q].n = t / c.Ho;
        pb[q].bi = i * c.stride - c.pad;
        pb[q].bj = j * c.stride - c.pad;
    }
}

inline const float *tap_ptr(const ConvCtx &c, const PixBase &p, int r, int s)
{
    const int ii = p.bi + r, jj = p.bj + s;
    if (!p.valid || ii < 0 || ii >= c.H || jj < 0 || jj >= c.W) return c.zeros;
    return c.x + (((size_t)p.n * c.H + ii) * c.W + jj) * c.cin_p;
}

inline v8 epilogue(const ConvCtx &c, v8 v)
{
    if (c.act) {
        const v8 neg = v * c.slope;
        v = v > 0.0f ? v : neg;
    }
    return v;
}

// One full 16-channel block over pixels [m_begin, m_end).
void conv_block16(const ConvCtx &c, int blk, int m_begin, int m_end)
{
    const size_t bstride = (size_t)c.R * c.S * c.cin_p * CB;
    const float *wb = c.w + blk * bstride;
    const int co = blk * CB;
    const v8 b0 = ld8(c.bias + co), b1 = ld8(c.bias + co + 8);
    PixBase pb[PB];
    for (int m0 = m_begin; m0 < m_end; m0 += PB) {
        pix_bases(c, m0, pb);
        for (int q = 0; q < PB; ++q)
            if (m0 + q >= m_end) pb[q].valid = false;
        v8 acc[PB][2];
        for (int q = 0; q < PB; ++q) acc[q][0] = acc[q][1] = (v8){0, 0, 0, 0, 0, 0, 0, 0};
        for (int r = 0; r < c.R; ++r) {
            for (int s = 0; s < c.S; ++s) {
                const float *xp[PB];
                for (int q = 0; q < PB; ++q) xp[q] = tap_ptr(c, pb[q], r, s);
                const float *wt = wb + (size_t)(r * c.S + s) * c.cin_p * CB;
                for (int ci = 0; ci < c.cin_p; ++ci) {
                    const v8 w0 = ld8(wt + ci * CB), w1 = ld8(wt + ci * CB + 8);
                    for (int q = 0; q < PB; ++q) {
                        const float xv = xp[q][ci];
                        acc[q][0] += w0 * xv;
                        acc[q][1] += w1 * xv;
                    }
                }
            }
        }
        for (int q = 0; q < PB; ++q) {
            if (!pb[q].valid) continue;
            float *yp = c.y + (size_t)(m0 + q) * c.cout_p + co;
            st8(yp, epilogue(c, acc[q][0] + b0));
            st8(yp + 8, epilogue(c, acc[q][1] + b1));
        }
    }
}

// The remaining cout_p % 16 channels (scalar), weights [R][S][cin_p][rem].
void conv_tail(const ConvCtx &c, int m_begin, int m_end)
{
    const float *wt0 = c.w + (size_t)c.nfull * c.R * c.S * c.cin_p * CB;
    const int co0 = c.nfull * CB;
    PixBase pb[PB];
    for (int m0 = m_begin; m0 < m_end; m0 += PB) {
        pix_bases(c, m0, pb);
        for (int q = 0; q < PB; ++q) {
            if (!pb[q].valid || m0 + q >= m_end) continue;
            float acc[CB] = {0};
            for (int r = 0; r < c.R; ++r)
                for (int s = 0; s < c.S; ++s) {
                    const float *xp = tap_ptr(c, pb[q], r, s);
                    const float *wt = wt0 + (size_t)(r * c.S + s) * c.cin_p * c.rem;
                    for (int ci = 0; ci < c.cin_p; ++ci)
                        for (int k = 0; k < c.rem; ++k) acc[k] += wt[ci * c.rem + k] * xp[ci];
                }
            float *yp = c.y + (size_t)(m0 + q) * c.cout_p + co0;
            for (int k = 0; k < c.rem; ++k) {
                float v = acc[k] + c.bias[co0 + k];
                if (c.act && !(v > 0.0f)) v *= c.slope;
                yp[k] = v;
            }
        }
    }
}

}  // namespace

void pack_weights(const std::function<float(int, int, int, int)> &wval, int cout_p, int R, int S, int cin_p,
                  float *out)
{
    const int nfull = cout_p / CB, rem = cout_p % CB;
    size_t o = 0;
    for (int b = 0; b < nfull; ++b)
        for (int r = 0; r < R; ++r)
            for (int s = 0; s < S; ++s)
                for (int ci = 0; ci < cin_p; ++ci)
                    for (int k = 0; k < CB; ++k) out[o++] = wval(b * CB + k, r, s, ci);
    for (int r = 0; r < R; ++r)
        for (int s = 0; s < S; ++s)
            for (int ci = 0; ci < cin_p; ++ci)
                for (int k = 0; k < rem; ++k) out[o++] = wval(nfull * CB + k, r, s, ci);
}

void conv(const float *x, int n, int H, int W, int cin_p, const float *w, const float *bias, int cout_p, int R,
          int S, int stride, int pad, int act, float slope, float *y, int Ho, int Wo)
{
    std::vector<float> zeros((size_t)cin_p, 0.0f);
    ConvCtx c{x, w, bias, zeros.data(), y, n, H, W, cin_p, cout_p, R, S, stride, pad, act, Ho, Wo, slope,
              n * Ho * Wo, cout_p / CB, cout_p % CB};
    const int blocks = c.nfull + (c.rem ? 1 : 0);
    if (blocks == 0 || c.M == 0) return;
    const int pix_blocks = (c.M + PB - 1) / PB;
    const int want = std::max(1, (4 * threads() + blocks - 1) / blocks);
    const int groups = std::min(pix_blocks, want);
    const int per = (pix_blocks + groups - 1) / groups * PB;  // pixels per task, a multiple of PB
    parallel_for(blocks * groups, [&](int t) {
        const int blk = t / groups, g = t % groups;
        const int m_begin = g * per, m_end = std::min(c.M, m_begin + per);
        if (m_begin >= m_end) return;
        if (blk < c.nfull) conv_block16(c, blk, m_begin, m_end);
        else conv_tail(c, m_begin, m_end);
    });
}

// ---------------------------------------------------------------- pool, add, layout

void maxpool(const float *x, int n, int H, int W, int cp, int k, int stride, float *y, int Ho, int Wo)
{
    const int off = (k - 1) / 2;
    parallel_for(n * Ho, [&](int t) {
        const int b = t / Ho, i = t % Ho;
        std::vector<float> acc((size_t)cp);
        for (int j = 0; j < Wo; ++j) {
            std::fill(acc.begin(), acc.end(), -std::numeric_limits<float>::infinity());
            for (int u = 0; u < k; ++u) {
                const int ii = i * stride - off + u;
                if (ii < 0 || ii >= H) continue;
                for (int v = 0; v < k; ++v) {
                    const int jj = j * stride - off + v;
                    if (jj < 0 || jj >= W) continue;
                    const float *xp = x + (((size_t)b * H + ii) * W + jj) * cp;
                    for (int ch = 0; ch < cp; ++ch) acc[ch] = xp[ch] > acc[ch] ? xp[ch] : acc[ch];
                }
            }
            std::memcpy(y + (((size_t)b * Ho + i) * Wo + j) * cp, acc.data(), (size_t)cp * sizeof(float));
        }
    });
}

void add(const float *a, const float *b, float *y, size_t count)
{
    const size_t chunk = 1 << 16;
    const int tasks = (int)((count + chunk - 1) / chunk);
    parallel_for(tasks, [&](int t) {
        const size_t e = std::min(count, (size_t)(t + 1) * chunk);
        for (size_t i = (size_t)t * chunk; i < e; ++i) y[i] = a[i] + b[i];
    });
}

void ingest(const float *x, int n, int c, int h, int w, int cp, float *y)
{
    parallel_for(n * h, [&](int t) {
        const int b = t / h, i = t % h;
        for (int j = 0; j < w; ++j) {
            float *yp = y + (((size_t)b * h + i) * w + j) * cp;
            for (int ch = 0; ch < cp; ++ch) yp[ch] = ch < c ? x[(((size_t)b * c + ch) * h + i) * w + j] : 0.0f;
        }
    });
}

void egress(const float *x, int n, int c, int h, int w, int cp, float *y)
{
    parallel_for(n * h, [&](int t) {
        const int b = t / h, i = t % h;
        for (int j = 0; j < w; ++j) {
            const float *xp = x + (((size_t)b * h + i) * w + j) * cp;
            for (int ch = 0; ch < c; ++ch) y[(((size_t)b * c + ch) * h + i) * w + j] = xp[ch];
        }
    });
}

}  // namespace dncpu
