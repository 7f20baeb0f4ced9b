// Host runtime and C ABI (include/dn.h) of the Darknet-style CNN forward
// library: layer-list validation, the execution plan with its fusions, the
// liveness-packed activation arena, weight upload / FP64 fold, the resident
// and per-layer-transfer forwards, hipGraph capture/replay, FP8 calibration
// and the tile autotuner; the backward pass to the input image and the image
// ascent (with their own plan and autotuner), the standalone layer and
// backward ops, detection post-processing and the Jacobi/Laplace iteration.
//
// Transfer placement follows the rule of Sec. 3.2 of the paper: a copy is
// placed outside the outermost loop that does not define (host->device) or
// use (device->host) the data.  Weights are defined once per load, so they
// cross once in dn_load_weights; the input is defined once per frame, so it
// crosses once per forward; intermediate activations are produced and
// consumed on the device only, so they never cross.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdarg>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/dn.h"
#include "cpu_layers.h"
#include "dn_kernels.h"
#include "ga.h"

using namespace dnk;

// ---------------------------------------------------------------- errors

static thread_local std::string g_err;

static dn_status fail(dn_status st, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
static dn_status fail(dn_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

#define HIPCHK(expr)                                                                              \
    do {                                                                                          \
        hipError_t e_ = (expr);                                                                   \
        if (e_ != hipSuccess) return fail(DN_EHIP, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

#define STCHK(expr)                     \
    do {                                \
        dn_status s_ = (expr);          \
        if (s_ != DN_OK) return s_;     \
    } while (0)

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// ---------------------------------------------------------------- net objects

struct ConvWeights {
    int cin = 0, cin_p = 0, cout = 0, cout_p = 0, k_pad = 0;
    int k_pad32 = 0;          // k_pad of the FP32 calibration copy
    void *w = nullptr;        // packed, net dtype
    float *bias = nullptr;    // [cout_p]
    float *wscale = nullptr;  // [cout_p]
    void *w32 = nullptr;      // FP8 nets: FP32 packed copy for calibration
    float *bias32 = nullptr, *wscale32 = nullptr;
    std::vector<unsigned char> host_w;  // per-layer mode: host copy of the packed weights
    std::vector<float> host_bias, host_wscale;
    void *pinned = nullptr;   // pinned staging of host_w|bias|wscale (per-layer mode)
    // backward-data conv (F32 / BF16 nets): transposed, flipped, BN-scaled
    // weights [cin_p][kb_pad], a zero bias and unit scales of cin_p entries
    void *wb = nullptr;
    float *bzero = nullptr, *bscale = nullptr;
    int kb_pad = 0;
    size_t wbytes = 0;
    bool loaded = false;
    // placed forward: host copy of the folded FP32 weights in the host conv's
    // blocked layout (read back from the device on first use)
    std::vector<float> cpu_w, cpu_b;
};

enum OpKind { OP_CONV = 0, OP_POOL = 1, OP_ADD = 2 };

struct Op {
    int kind = OP_CONV;
    int layer = 0;       // layer index whose output this op produces
    int conv = -1;       // conv layer index (OP_CONV)
    int in = 0, in2 = -1, out = 0;  // value ids: value v = output of layer v-1, value 0 = net input
    bool pool = false, res = false;
    bool first = false;  // first-layer kernel reading the NCHW FP32 input directly
    int H = 0, W = 0, Ho = 0, Wo = 0, cin_p = 0, cout = 0, cout_p = 0;  // op geometry
    int c_log = 0;       // logical channels of the output
    int tile = -1, splits = 1;
    size_t ws_bytes = 0;
    bool argmax = false;  // fused pool: also store each window's argmax (input-gradient pass)
    size_t argmax_off = 0;
};

struct Value { int c = 0, cp = 0, h = 0, w = 0; size_t bytes = 0, off = 0; int first = 0, last = 0; };

struct Plan {
    int dtype = 0, mode = 0, batch = 0, h = 0, w = 0;
    std::vector<Op> ops;
    std::vector<Value> vals;   // index = value id
    size_t ws_off = 0, ws_bytes = 0;
    // split-K tile counters (in-kernel finish), zeroed at the start of every
    // forward that has a conv finishing in-kernel; 0 bytes = every split conv
    // finishes with a separate launch
    size_t cnt_off = 0, cnt_bytes = 0;
    bool any_fused = false;
    size_t xin_off = 0, yout_off = 0;  // per-layer mode FP32 staging of x / y
    size_t total = 0;
    int out_val = 0;
};

struct GraphKey {
    int batch, h, w;
    const void *x, *y, *arena;
    bool operator<(const GraphKey &o) const
    {
        return std::tie(batch, h, w, x, y, arena) < std::tie(o.batch, o.h, o.w, o.x, o.y, o.arena);
    }
};

struct dn_net {
    std::vector<dn_layer_desc> L;
    dn_net_opts o{};
    std::vector<ConvWeights> cw;            // per layer (only convs used)
    std::vector<int> in_c;                  // logical input channels per layer
    std::vector<float> scale;               // FP8: per value (index = value id) activation scale
    bool calibrated = false;
    void *arena = nullptr;
    size_t arena_bytes = 0;
    hipStream_t cap_stream = nullptr;       // capture stream (never the legacy null stream)
    // Two instances of each captured forward, launched alternately: a launch
    // then never has to wait for the previous replay of the same instance to
    // retire, so the host can queue the next forward while one runs.
    struct GraphPair { hipGraphExec_t exec[2] = {nullptr, nullptr}; unsigned next = 0; size_t total = 0; };
    std::map<GraphKey, GraphPair> graphs;
    // resident-forward plans per (batch, h, w); like the graphs, dropped
    // whenever weights, scales or tuned tiles change
    std::map<std::tuple<int, int, int>, std::shared_ptr<const Plan>> plans;
    std::map<std::string, std::pair<int, int>> tuned;  // conv signature -> (tile, splits)
    std::string tune_key;                   // device arch, HIP runtime version, tile table (tune-cache file key)
    std::map<std::tuple<int, int, int>, std::vector<unsigned char *>> host_vals;  // per-layer mode
    std::map<std::tuple<int, int, int>, std::vector<unsigned char *>> host_place;  // placed forward
    std::mutex mu;
};

static void drop_graphs(dn_net *net)
{
    for (auto &kv : net->graphs)
        for (hipGraphExec_t e : kv.second.exec)
            if (e) (void)hipGraphExecDestroy(e);
    net->graphs.clear();
    net->plans.clear();
}

// ---------------------------------------------------------------- helpers


static int out_side_conv(int x, int k, int st, int pad) { return (x + 2 * pad - k) / st + 1; }

// The network's first conv takes the fused-ingest kernel when one filter row
// of every input channel fits a 16-element run of the staged window and its
// output channels fit in registers.
static bool first_ok(int in_c, const dn_layer_desc &d, int dt)
{
    (void)dt;
    return d.kind == DN_CONV && in_c <= 16 && first_cp(in_c) * d.ksize <= 16 && d.ksize <= FIRST_MAX_R &&
           d.cout <= FIRST_MAX_COUT && d.stride <= 2;
}
static bool first_eligible(const dn_net *net, int dt)
{
    return !net->L.empty() && first_ok(net->o.in_c, net->L[0], dt);
}
static int out_side_pool(int x, int st) { return (x - 1) / st + 1; }

extern "C" int dn_channel_pad(int dtype, int c)
{
    if (dtype < 0 || dtype > 2 || c < 0) return -1;
    return cpad(dtype, c);
}

static dn_status check_dtype(int dt)
{
    if (dt != DN_F32 && dt != DN_BF16 && dt != DN_FP8_E4M3) return fail(DN_EINVAL, "unknown dtype %d", dt);
    return DN_OK;
}

// Heuristic tile when the autotuner has not run: the 176x128 LDS-DMA tile
// (two workgroups per CU) when it yields about one round of work, else the
// largest tile that still gives >= 1 workgroup per CU, small-N tiles for
// narrow layers, split-K when the grid stays small.
static void heuristic_tile(int M, int N, int K, int *tile, int *splits)
{
    const int CUS = 256;
    static const int TILE_176x128 = [] {
        for (int t = 0; t < tile_count(); ++t) {
            const TileCfg c = tile_cfg(t);
            if (c.bm == 176 && c.bn == 128 && c.wm == 1 && c.wn == 8) return t;
        }
        return 2;
    }();
    int best = 2;
    if (N <= 16) best = 6;
    else if (N <= 32) best = 7;
    else if (N <= 64) best = (M >= 256 * 64) ? 1 : 0;
    else if ((long)((M + 175) / 176) * ((N + 127) / 128) >= CUS - 16) best = TILE_176x128;
    else {
        const int cands[] = {4, 3, 2, 8, 0};
        best = 0;
        for (int c : cands) {
            const TileCfg t = tile_cfg(c);
            const long tiles = (long)((M + t.bm - 1) / t.bm) * ((N + t.bn - 1) / t.bn);
            if (tiles >= CUS) { best = c; break; }
        }
    }
    const TileCfg t = tile_cfg(best);
    const long tiles = (long)((M + t.bm - 1) / t.bm) * ((N + t.bn - 1) / t.bn);
    int s = 1;
    const int ktiles = K;  // caller passes K in k-tiles
    while (tiles * s * 2 <= 2 * CUS && ktiles / (s * 2) >= 4) s *= 2;
    *tile = best;
    *splits = s;
}

// Tune-cache signature of a forward conv; batch-invariant nets keep their
// own entries (their candidates are restricted, see below).
static std::string conv_sig(int dt, const Op &op, int batch, int R, int stride, bool inv)
{
    char b[256];
    snprintf(b, sizeof b, "dt%d_b%d_H%d_W%d_ci%d_co%d_R%d_s%d_p%d_r%d%s", dt, batch, op.H, op.W, op.cin_p,
             op.cout_p, R, stride, (int)op.pool, (int)op.res, inv ? "_bi" : "");
    return b;
}

static bool is_halo(int t) { return t == HALO_TILE || t == HALO2_TILE; }

// Batch-invariant nets.  An output's sum runs over K in the same order at
// every batch size when (1) its split-K partition depends on K alone and
// (2) every tile forms its K-steps from the same MFMA instruction.  (1): one
// split per 64 K-tiles, at most 4, a power of two (a batch-1 forward of the
// widest convs still spreads over more workgroups).  (2): tiles of 16x16
// blocks only; BF16's 32x32 blocks take their products in other groups.  The
// halo kernels sum in the order of the 16x16 GEMM tiles and run unsplit.
static int invariant_splits(int nkt)
{
    int s = 1;
    while (s < 4 && nkt >= 64 * s) s *= 2;
    return s;
}

static bool invariant_tile_ok(int dt, int tile, int splits)
{
    if (is_halo(tile)) return splits == 1;
    return tile >= 0 && tile < tile_count() && (dt != BF16 || tile_cfg(tile).mf != 32);
}

// Which split convs finish in the GEMM launch itself.  That finish runs on
// the one workgroup per output tile that arrives last, which reads
// splits x BM x BN partial sums.  Measured on the residual net's small-M
// layers (batch 16) it beats the separate finish launch while that share is
// at most 16K values (64x64 and 64x32 tiles up to 4 and 8 splits: by up to a
// third of the layer's time) and loses to it beyond, by up to 20% (a few
// large tiles leave the whole reduction to a few workgroups).
static bool finish_in_kernel(int tile, int splits)
{
    if (splits < 2 || splits > SPLITK_FUSED_MAX || is_halo(tile) || tile < 0 || tile >= tile_count()) return false;
    const TileCfg t = tile_cfg(tile);
    return (long)splits * t.bm * t.bn <= 16384;
}

// Fill ConvArgs for an op of plan p, reading from base (arena).
static ConvArgs conv_args(const dn_net *net, const Plan &p, const Op &op, char *base, bool use32)
{
    const dn_layer_desc &d = net->L[op.conv];
    const ConvWeights &cw = net->cw[op.conv];
    ConvArgs a{};
    a.x = base + p.vals[op.in].off;
    a.w = use32 ? cw.w32 : cw.w;
    a.bias = use32 ? cw.bias32 : cw.bias;
    a.wscale = use32 ? cw.wscale32 : cw.wscale;
    a.res = op.res ? base + p.vals[op.in2].off : nullptr;
    a.y = base + p.vals[op.out].off;
    a.partial = (float *)(base + p.ws_off);
    a.argmax = op.argmax ? (unsigned char *)(base + op.argmax_off) : nullptr;
    a.batch = p.batch;
    a.H = op.H; a.W = op.W; a.cin_p = op.cin_p;
    a.Ho = op.pool ? op.Ho * 2 : op.Ho;
    a.Wo = op.pool ? op.Wo * 2 : op.Wo;
    a.cout_p = op.cout_p;
    a.R = d.ksize; a.S = d.ksize; a.stride = d.stride; a.pad = d.pad;
    a.k_pad = use32 ? cw.k_pad32 : cw.k_pad;
    a.M = p.batch * a.Ho * a.Wo;
    a.pool = op.pool ? 1 : 0;
    a.act = d.activation;
    a.slope = net->o.leaky_slope;
    a.in_scale = a.res_scale = a.out_inv_scale = 1.0f;
    if (p.dtype == FP8) {
        a.in_scale = net->scale[op.in];
        a.res_scale = op.res ? net->scale[op.in2] : 1.0f;
        a.out_inv_scale = 1.0f / net->scale[op.out];
    }
    a.splits = op.splits;
    const int nkt = a.k_pad / bk_el(use32 ? (int)F32 : p.dtype);
    a.ktiles_per_split = (nkt + op.splits - 1) / op.splits;
    a.tile_count = nullptr;
    if (p.cnt_bytes && finish_in_kernel(op.tile, op.splits) &&
        (size_t)op.splits * a.M * a.cout_p * sizeof(float) <= 0x7fffffffu)
        a.tile_count = (unsigned *)(base + p.cnt_off);
    return a;
}

// ---------------------------------------------------------------- planning

// Can this conv op run the halo kernel (small K, <= 64 output channels)?
static bool op_halo_ok(const dn_net *net, int dtype, const Op &op, int k_pad)
{
    if (op.kind != OP_CONV || op.first) return false;
    const dn_layer_desc &d = net->L[op.conv];
    ConvArgs a{};
    a.R = a.S = d.ksize; a.stride = d.stride; a.pad = d.pad;
    a.cin_p = op.cin_p; a.cout_p = op.cout_p; a.k_pad = k_pad;
    return halo_ok(dtype, a);
}

// Can this conv op run the persistent halo kernel?
static bool op_halo2_ok(const dn_net *net, int dtype, const Op &op, int k_pad)
{
    if (op.kind != OP_CONV || op.first) return false;
    const dn_layer_desc &d = net->L[op.conv];
    ConvArgs a{};
    a.R = a.S = d.ksize; a.stride = d.stride; a.pad = d.pad;
    a.cin_p = op.cin_p; a.cout_p = op.cout_p; a.k_pad = k_pad;
    a.H = op.H; a.W = op.W; a.Ho = op.pool ? op.Ho * 2 : op.Ho; a.Wo = op.pool ? op.Wo * 2 : op.Wo;
    return halo2_ok(dtype, a);
}

// pool_fuse_upto >= 0 (input-gradient pass, per-layer mode otherwise): fuse a
// conv with the 2x2/2 pool after it when that pool's layer index is at most
// pool_fuse_upto; no residual fusion.
// gene != nullptr (placed forward): layer i runs on the GPU iff gene[i]; a
// conv fuses with the layer after it only when both are on the GPU, the
// first-layer kernel is used only when layer 0 is on the GPU, every value
// keeps its own buffer (no reuse), and the image / result get FP32 staging.
static dn_status make_plan(const dn_net *net, int dtype, int mode, int batch, int h, int w, Plan *out,
                           int pool_fuse_upto = -1, const unsigned char *gene = nullptr)
{
    const int n = (int)net->L.size();
    if (batch <= 0 || h <= 0 || w <= 0) return fail(DN_EINVAL, "batch/h/w must be positive (%d, %d, %d)", batch, h, w);
    Plan p;
    p.dtype = dtype; p.mode = mode; p.batch = batch; p.h = h; p.w = w;
    const int es = esize(dtype);
    // value geometry
    p.vals.resize(n + 1);
    p.vals[0].c = net->o.in_c; p.vals[0].h = h; p.vals[0].w = w;
    for (int i = 0; i < n; ++i) {
        const dn_layer_desc &d = net->L[i];
        const Value &in = p.vals[i];
        Value &v = p.vals[i + 1];
        if (d.kind == DN_CONV) {
            v.c = d.cout;
            v.h = out_side_conv(in.h, d.ksize, d.stride, d.pad);
            v.w = out_side_conv(in.w, d.ksize, d.stride, d.pad);
        } else if (d.kind == DN_MAXPOOL) {
            v.c = in.c; v.h = out_side_pool(in.h, d.stride); v.w = out_side_pool(in.w, d.stride);
        } else {
            const Value &s = p.vals[d.src + 1];
            if (s.c != in.c || s.h != in.h || s.w != in.w)
                return fail(DN_EINVAL, "shortcut layer %d: shape of layer %d (%dx%dx%d) != previous (%dx%dx%d)", i, d.src, s.c, s.h, s.w, in.c, in.h, in.w);
            v = in;
        }
        if (v.h <= 0 || v.w <= 0) return fail(DN_EINVAL, "input %dx%d too small for layer %d", h, w, i);
    }
    for (auto &v : p.vals) {
        v.cp = cpad(dtype, v.c);
        v.bytes = align256((size_t)batch * v.h * v.w * v.cp * es);
        v.first = -2; v.last = -2;
    }
    // consumers count (to know whether a conv output may be fused away)
    std::vector<int> uses(n + 1, 0);
    for (int i = 0; i < n; ++i) {
        uses[i]++;  // layer i reads value i (its input)
        if (net->L[i].kind == DN_SHORTCUT) uses[net->L[i].src + 1]++;
    }
    uses[n]++;  // net output
    // ops
    for (int i = 0; i < n; ++i) {
        const dn_layer_desc &d = net->L[i];
        Op op;
        op.layer = i;
        op.in = i;
        op.out = i + 1;
        op.c_log = p.vals[i + 1].c;
        if (d.kind == DN_CONV) {
            op.kind = OP_CONV;
            op.conv = i;
            op.first = (i == 0) && first_eligible(net, dtype) && (!gene || gene[0]);
            op.H = p.vals[i].h; op.W = p.vals[i].w; op.cin_p = p.vals[i].cp;
            op.Ho = p.vals[i + 1].h; op.Wo = p.vals[i + 1].w;
            op.cout = d.cout; op.cout_p = p.vals[i + 1].cp;
            bool fuse = mode == DN_MODE_RESIDENT || (pool_fuse_upto >= 0 && i + 1 <= pool_fuse_upto);
            if (gene && (i + 1 >= n || !gene[i] || !gene[i + 1])) fuse = false;
            if (fuse && i + 1 < n && uses[i + 1] == 1) {
                const dn_layer_desc &nx = net->L[i + 1];
                if (nx.kind == DN_MAXPOOL && nx.ksize == 2 && nx.stride == 2 && op.Ho % 2 == 0 && op.Wo % 2 == 0) {
                    op.pool = true;
                    op.layer = i + 1; op.out = i + 2;
                    op.Ho /= 2; op.Wo /= 2;
                    ++i;
                } else if (mode == DN_MODE_RESIDENT && nx.kind == DN_SHORTCUT && nx.src != i &&
                           nx.activation == DN_ACT_LINEAR) {
                    op.res = true;
                    op.in2 = nx.src + 1;
                    op.layer = i + 1; op.out = i + 2;
                    ++i;
                }
            }
        } else if (d.kind == DN_MAXPOOL) {
            op.kind = OP_POOL;
            op.H = p.vals[i].h; op.W = p.vals[i].w; op.Ho = p.vals[i + 1].h; op.Wo = p.vals[i + 1].w;
            op.cout_p = p.vals[i + 1].cp;
        } else {
            op.kind = OP_ADD;
            op.in2 = d.src + 1;
            op.cout_p = p.vals[i + 1].cp;
        }
        p.ops.push_back(op);
    }
    // the first-layer kernel reads the caller's input itself: value 0 needs no buffer
    if (!p.ops.empty() && p.ops[0].first) p.vals[0].bytes = 0;
    // liveness: value produced at op index (value 0 at -1), last use = max consumer op index
    p.vals[0].first = -1;
    for (int k = 0; k < (int)p.ops.size(); ++k) {
        Op &op = p.ops[k];
        p.vals[op.out].first = k;
        p.vals[op.in].last = std::max(p.vals[op.in].last, k);
        if (op.in2 >= 0) p.vals[op.in2].last = std::max(p.vals[op.in2].last, k);
    }
    p.out_val = p.ops.back().out;
    p.vals[p.out_val].last = (int)p.ops.size();  // egress
    // greedy first-fit placement in production order
    std::vector<std::pair<size_t, size_t>> live;  // (off, size) of live blocks with their value id below
    std::vector<int> live_id;
    size_t top = 0;
    auto place = [&](int vid) {
        std::vector<std::pair<size_t, size_t>> blocks = live;
        std::sort(blocks.begin(), blocks.end());
        size_t cur = 0;
        for (auto &b : blocks) {
            if (b.first >= cur + p.vals[vid].bytes) break;
            cur = std::max(cur, b.first + b.second);
        }
        p.vals[vid].off = cur;
        top = std::max(top, cur + p.vals[vid].bytes);
        live.push_back({cur, p.vals[vid].bytes});
        live_id.push_back(vid);
    };
    auto release = [&](int k) {
        for (size_t j = 0; j < live.size();) {
            if (p.vals[live_id[j]].last == k) {
                live.erase(live.begin() + j);
                live_id.erase(live_id.begin() + j);
            } else {
                ++j;
            }
        }
    };
    if (gene) {  // every value its own buffer
        size_t off = 0;
        p.vals[0].off = 0;
        off = p.vals[0].bytes;
        for (const Op &op : p.ops) {
            p.vals[op.out].off = off;
            off += p.vals[op.out].bytes;
        }
        top = off;
    } else {
        place(0);
        for (int k = 0; k < (int)p.ops.size(); ++k) {
            place(p.ops[k].out);
            release(k);
        }
    }
    // split-K scratch and tile choice
    size_t ws = 0, counters = 0;
    for (Op &op : p.ops) {
        if (op.kind != OP_CONV || op.first) continue;
        const dn_layer_desc &d = net->L[op.conv];
        const int K = d.ksize * d.ksize * op.cin_p;
        const int k_pad = (K + bk_el(dtype) - 1) / bk_el(dtype) * bk_el(dtype);
        const int M = op.pool ? batch * (2 * op.Ho) * (2 * op.Wo) : batch * op.Ho * op.Wo;
        const bool inv = net->o.batch_invariant != 0;
        const std::string sig = conv_sig(dtype, op, batch, d.ksize, d.stride, inv);
        auto it = net->tuned.find(sig);
        if (it != net->tuned.end()) {
            op.tile = it->second.first;
            op.splits = it->second.second;
        } else if (op_halo2_ok(net, dtype, op, k_pad)) {
            op.tile = HALO2_TILE;
            op.splits = 1;
        } else if (op_halo_ok(net, dtype, op, k_pad)) {
            op.tile = HALO_TILE;
            op.splits = 1;
        } else {
            heuristic_tile(M, op.cout_p, k_pad / bk_el(dtype), &op.tile, &op.splits);
        }
        if (inv) {
            op.splits = invariant_splits(k_pad / bk_el(dtype));
            if (!invariant_tile_ok(dtype, op.tile, op.splits)) {
                int unused;
                heuristic_tile(M, op.cout_p, k_pad / bk_el(dtype), &op.tile, &unused);  // 16x16-block tiles
            }
        }
        op.ws_bytes = op.splits > 1 ? align256((size_t)op.splits * M * op.cout_p * 4) : 0;
        ws = std::max(ws, op.ws_bytes);
        counters = std::max(counters, splitk_counters(M, op.cout_p));  // the autotuner may split any of them
        p.any_fused = p.any_fused || finish_in_kernel(op.tile, op.splits);
    }
    p.cnt_off = align256(top);
    p.cnt_bytes = align256(counters * sizeof(unsigned));
    p.ws_off = align256(p.cnt_off + p.cnt_bytes);
    p.ws_bytes = ws;
    size_t end = p.ws_off + ws;
    if (mode == DN_MODE_PER_LAYER || gene) {
        p.xin_off = align256(end);
        end = p.xin_off + align256((size_t)batch * net->o.in_c * h * w * 4);
        p.yout_off = align256(end);
        const Value &ov = p.vals[p.out_val];
        end = p.yout_off + align256((size_t)batch * ov.c * ov.h * ov.w * 4);
    }
    p.total = align256(end);
    *out = std::move(p);
    return DN_OK;
}

// ---------------------------------------------------------------- enqueue

// x8 set: the image is 8-bit pixels (value q / 255) instead of FP32 x.
static dn_status enqueue_first(const dn_net *net, const Plan &p, const Op &op, const float *x, char *base,
                               hipStream_t s, bool use32, const unsigned char *x8 = nullptr)
{
    const dn_layer_desc &d = net->L[op.conv];
    const ConvWeights &cw = net->cw[op.conv];
    FirstArgs a{};
    a.x = x8 ? nullptr : x;
    a.x8 = x8;
    a.w = use32 ? cw.w32 : cw.w;
    a.bias = use32 ? cw.bias32 : cw.bias;
    a.wscale = use32 ? cw.wscale32 : cw.wscale;
    a.y = base + p.vals[op.out].off;
    a.batch = p.batch; a.C = p.vals[0].c; a.H = p.h; a.W = p.w;
    a.Ho = op.pool ? op.Ho * 2 : op.Ho;
    a.Wo = op.pool ? op.Wo * 2 : op.Wo;
    a.cout_p = op.cout_p;
    a.k_pad = first_kpad(use32 ? (int)F32 : p.dtype, d.ksize);
    a.R = a.S = d.ksize; a.stride = d.stride; a.pad = d.pad;
    a.pool = op.pool ? 1 : 0;
    a.argmax = op.argmax ? (unsigned char *)(base + op.argmax_off) : nullptr;
    a.act = d.activation;
    a.slope = net->o.leaky_slope;
    a.in_inv_scale = a.in_scale = a.out_inv_scale = 1.0f;
    if (!use32 && p.dtype == FP8) {
        a.in_inv_scale = 1.0f / net->scale[0];
        a.in_scale = net->scale[0];
        a.out_inv_scale = 1.0f / net->scale[op.out];
    }
    HIPCHK(launch_conv_first(use32 ? (int)F32 : p.dtype, a, s));
    return DN_OK;
}

static dn_status enqueue_op(const dn_net *net, const Plan &p, const Op &op, char *base, hipStream_t s, bool use32,
                            int tile_override = -1, int splits_override = 0, const float *xin = nullptr,
                            const unsigned char *xin8 = nullptr)
{
    if (op.kind == OP_CONV && op.first) {
        if (!xin && !xin8) return fail(DN_EINVAL, "first-layer kernel needs the input image");
        return enqueue_first(net, p, op, xin, base, s, use32, xin8);
    }
    if (op.kind == OP_CONV) {
        Op o2 = op;
        if (tile_override >= 0) o2.tile = tile_override;
        if (splits_override > 0) o2.splits = splits_override;
        ConvArgs a = conv_args(net, p, o2, base, use32);
        const int dt = use32 ? F32 : p.dtype;
        HIPCHK(launch_conv(dt, o2.tile, a, s));
        if (o2.splits > 1 && !a.tile_count) HIPCHK(launch_splitk_reduce(dt, a, s));
    } else if (op.kind == OP_POOL) {
        const dn_layer_desc &d = net->L[op.layer];
        const Value &vi = p.vals[op.in];
        HIPCHK(launch_maxpool(use32 ? F32 : p.dtype, base + vi.off, base + p.vals[op.out].off, p.batch, vi.h, vi.w,
                              vi.cp, d.ksize, d.stride, op.Ho, op.Wo, s));
    } else {
        const Value &vo = p.vals[op.out];
        float sa = 1.f, sb = 1.f, isy = 1.f;
        if (!use32 && p.dtype == FP8) {
            sa = net->scale[op.in]; sb = net->scale[op.in2]; isy = 1.0f / net->scale[op.out];
        }
        HIPCHK(launch_add(use32 ? F32 : p.dtype, base + p.vals[op.in].off, sa, base + p.vals[op.in2].off, sb,
                          base + vo.off, isy, (size_t)p.batch * vo.h * vo.w * vo.cp, s));
    }
    return DN_OK;
}

// Zero the split-K tile counters of plan p (a fill kernel, so that it can be
// captured in a graph).  Every launch leaves them zero again, so one fill per
// forward covers all of its split convs.
static dn_status zero_counters(const Plan &p, char *base, hipStream_t s)
{
    if (p.cnt_bytes) HIPCHK(launch_zero_f32((float *)(base + p.cnt_off), p.cnt_bytes / sizeof(float), s));
    return DN_OK;
}

static dn_status enqueue_resident(const dn_net *net, const Plan &p, char *base, const float *x, float *y, hipStream_t s)
{
    if (p.any_fused) STCHK(zero_counters(p, base, s));
    const Value &v0 = p.vals[0];
    const float in_inv = p.dtype == FP8 ? 1.0f / net->scale[0] : 1.0f;
    // 8-bit input nets: x holds the NCHW frames as bytes, converted on the device
    const unsigned char *x8 = net->o.input_u8 ? (const unsigned char *)x : nullptr;
    const float *xf = x8 ? nullptr : x;
    if (!p.ops[0].first)
        HIPCHK(launch_ingest(p.dtype, xf, p.batch, v0.c, v0.h, v0.w, v0.cp, in_inv, base + v0.off, s, x8));
    for (const Op &op : p.ops) STCHK(enqueue_op(net, p, op, base, s, false, -1, 0, xf, x8));
    const Value &vo = p.vals[p.out_val];
    const float osc = p.dtype == FP8 ? net->scale[p.out_val] : 1.0f;
    HIPCHK(launch_egress(p.dtype, base + vo.off, p.batch, vo.c, vo.h, vo.w, vo.cp, osc, y, s));
    return DN_OK;
}

static dn_status check_ready(const dn_net *net, bool need_calib)
{
    for (size_t i = 0; i < net->L.size(); ++i)
        if (net->L[i].kind == DN_CONV && !net->cw[i].loaded)
            return fail(DN_ESTATE, "weights of conv layer %zu not loaded", i);
    if (need_calib && net->o.dtype == DN_FP8_E4M3 && !net->calibrated)
        return fail(DN_ESTATE, "FP8 net used before dn_calibrate");
    return DN_OK;
}

static dn_status check_dims(const dn_net *net, int batch, int h, int w)
{
    if (batch <= 0 || batch > net->o.max_batch) return fail(DN_EINVAL, "batch %d outside 1..%d", batch, net->o.max_batch);
    if (h <= 0 || w <= 0 || h > net->o.max_h || w > net->o.max_w)
        return fail(DN_EINVAL, "input %dx%d outside 1..%dx%d", h, w, net->o.max_h, net->o.max_w);
    return DN_OK;
}

static bool is_device_ptr(const void *p)
{
    hipPointerAttribute_t at;
    if (hipPointerGetAttributes(&at, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return at.type == hipMemoryTypeDevice || at.type == hipMemoryTypeManaged;
}

// ---------------------------------------------------------------- C ABI

extern "C" const char *dn_last_error(void) { return g_err.c_str(); }

extern "C" dn_status dn_net_create(const dn_layer_desc *layers, int n, const dn_net_opts *o, dn_net **out)
{
    if (!out) return fail(DN_EINVAL, "out is NULL");
    *out = nullptr;
    if (!layers || n <= 0 || !o) return fail(DN_EINVAL, "need a non-empty layer list and options");
    STCHK(check_dtype(o->dtype));
    if (o->mode != DN_MODE_RESIDENT && o->mode != DN_MODE_PER_LAYER) return fail(DN_EINVAL, "unknown mode %d", o->mode);
    if (o->input_u8 && o->mode != DN_MODE_RESIDENT) return fail(DN_EUNSUPPORTED, "8-bit input needs a resident-mode net");
    if (o->in_c <= 0 || o->in_c > 16) return fail(DN_EINVAL, "in_c %d outside 1..16", o->in_c);
    if (o->max_h <= 0 || o->max_w <= 0 || o->max_batch <= 0) return fail(DN_EINVAL, "max_h/max_w/max_batch must be positive");
    if (!(o->bn_eps > 0.0)) return fail(DN_EINVAL, "bn_eps must be > 0");
    int c = o->in_c;
    std::vector<int> chans;
    for (int i = 0; i < n; ++i) {
        const dn_layer_desc &d = layers[i];
        chans.push_back(c);
        if (d.kind == DN_CONV) {
            if (d.cout <= 0 || d.ksize <= 0 || d.stride <= 0 || d.pad < 0)
                return fail(DN_EINVAL, "conv layer %d: bad cout/ksize/stride/pad", i);
            if (d.activation != DN_ACT_LINEAR && d.activation != DN_ACT_LEAKY)
                return fail(DN_EINVAL, "conv layer %d: unknown activation %d", i, d.activation);
            c = d.cout;
        } else if (d.kind == DN_MAXPOOL) {
            if (d.ksize <= 0 || d.stride <= 0) return fail(DN_EINVAL, "maxpool layer %d: bad size/stride", i);
        } else if (d.kind == DN_SHORTCUT) {
            if (d.src < 0 || d.src >= i)
                return fail(DN_EINVAL, "shortcut layer %d: src %d must name an earlier layer", i, d.src);
            if (d.activation != DN_ACT_LINEAR)
                return fail(DN_EUNSUPPORTED, "shortcut layer %d: only a linear shortcut is supported", i);
        } else {
            return fail(DN_EINVAL, "layer %d: unknown kind %d", i, d.kind);
        }
    }
    int ndev = 0;
    HIPCHK(hipGetDeviceCount(&ndev));
    if (o->device < 0 || o->device >= ndev) return fail(DN_EINVAL, "device %d not present (%d devices)", o->device, ndev);
    HIPCHK(hipSetDevice(o->device));
    dn_net *net = new (std::nothrow) dn_net();
    if (!net) return fail(DN_ENOMEM, "out of host memory");
    net->L.assign(layers, layers + n);
    net->o = *o;
    net->cw.resize(n);
    net->in_c = chans;
    net->scale.assign(n + 1, 1.0f);
    {
        hipDeviceProp_t prop;
        int rt = 0;
        char key[320];
        if (hipGetDeviceProperties(&prop, o->device) != hipSuccess || hipRuntimeGetVersion(&rt) != hipSuccess) {
            delete net;
            return fail(DN_EHIP, "device properties");
        }
        snprintf(key, sizeof key, "%s|hip%d|tiles%d", prop.gcnArchName, rt, tile_count());
        net->tune_key = key;
        for (char &ch : net->tune_key)
            if (ch == ' ' || ch == '/') ch = '_';
    }
    if (hipStreamCreateWithFlags(&net->cap_stream, hipStreamNonBlocking) != hipSuccess) {
        delete net;
        return fail(DN_EHIP, "hipStreamCreate failed");
    }
    // shape check against the largest input
    Plan p;
    dn_status st = make_plan(net, o->dtype, o->mode, 1, o->max_h, o->max_w, &p);
    if (st != DN_OK) {
        dn_net_destroy(net);
        return st;
    }
    *out = net;
    return DN_OK;
}

static void free_weights(ConvWeights &cw)
{
    if (cw.w) (void)hipFree(cw.w);
    if (cw.bias) (void)hipFree(cw.bias);
    if (cw.wscale) (void)hipFree(cw.wscale);
    if (cw.w32) (void)hipFree(cw.w32);
    if (cw.bias32) (void)hipFree(cw.bias32);
    if (cw.wscale32) (void)hipFree(cw.wscale32);
    if (cw.pinned) (void)hipHostFree(cw.pinned);
    if (cw.wb) (void)hipFree(cw.wb);
    if (cw.bzero) (void)hipFree(cw.bzero);
    if (cw.bscale) (void)hipFree(cw.bscale);
    cw = ConvWeights();
}

extern "C" void dn_net_destroy(dn_net *net)
{
    if (!net) return;
    (void)hipSetDevice(net->o.device);
    (void)hipDeviceSynchronize();
    drop_graphs(net);
    for (auto &cw : net->cw) free_weights(cw);
    for (auto *m : {&net->host_vals, &net->host_place})
        for (auto &kv : *m)
            for (unsigned char *b : kv.second)
                if (b) (void)hipHostFree(b);
    if (net->cap_stream) (void)hipStreamDestroy(net->cap_stream);
    delete net;
}

extern "C" dn_status dn_net_output_shape(const dn_net *net, int h, int w, int *c, int *ho, int *wo)
{
    if (!net || !c || !ho || !wo) return fail(DN_EINVAL, "NULL argument");
    Plan p;
    STCHK(make_plan(net, net->o.dtype, net->o.mode, 1, h, w, &p));
    const Value &v = p.vals[p.out_val];
    *c = v.c; *ho = v.h; *wo = v.w;
    return DN_OK;
}

extern "C" dn_status dn_arena_bytes(const dn_net *net, int batch, int h, int w, size_t *bytes)
{
    if (!net || !bytes) return fail(DN_EINVAL, "NULL argument");
    Plan p;
    STCHK(make_plan(net, net->o.dtype, net->o.mode, batch, h, w, &p));
    *bytes = p.total;
    return DN_OK;
}

extern "C" dn_status dn_bind_arena(dn_net *net, void *dev_ptr, size_t bytes)
{
    if (!net) return fail(DN_EINVAL, "net is NULL");
    if (!dev_ptr || bytes == 0) return fail(DN_EINVAL, "arena pointer/size missing");
    if (((uintptr_t)dev_ptr & 255) != 0) return fail(DN_EINVAL, "arena must be 256-byte aligned");
    if (!is_device_ptr(dev_ptr)) return fail(DN_EINVAL, "arena is not device memory");
    std::lock_guard<std::mutex> g(net->mu);
    net->arena = dev_ptr;
    net->arena_bytes = bytes;
    return DN_OK;
}

static dn_status pack_to(dn_net *net, int layer, int dt, const double *dw, const double *db, const double *dm,
                         const double *dv, const double *dg, const double *dbe, int has_bn, void **w, float **b,
                         float **s, hipStream_t st)
{
    ConvWeights &cw = net->cw[layer];
    const dn_layer_desc &d = net->L[layer];
    const int cin_p = cpad(dt, cw.cin);
    const bool compact = layer == 0 && first_eligible(net, dt);
    const int K = d.ksize * d.ksize * cin_p;
    const int k_pad = compact ? first_kpad(dt, d.ksize) : (K + bk_el(dt) - 1) / bk_el(dt) * bk_el(dt);
    const int cout_p = cpad(dt, d.cout);
    const size_t wb = (size_t)cout_p * k_pad * esize(dt);
    HIPCHK(hipMalloc(w, wb));
    HIPCHK(hipMalloc((void **)b, cout_p * sizeof(float)));
    HIPCHK(hipMalloc((void **)s, cout_p * sizeof(float)));
    HIPCHK(launch_fold_pack(dt, compact ? 1 : 0, dw, db, dm, dv, dg, dbe, net->o.bn_eps, has_bn, d.cout, cw.cin,
                            d.ksize, d.ksize, cin_p, k_pad, cout_p, *w, *b, *s, st));
    if (w == &cw.w) {
        cw.cin_p = cin_p; cw.cout = d.cout; cw.cout_p = cout_p; cw.k_pad = k_pad; cw.wbytes = wb;
    } else {
        cw.k_pad32 = k_pad;
    }
    return DN_OK;
}

// Backward-data weights of conv layer `layer`: the conv with the forward's
// input and output channels swapped, filter flipped, BN scale folded in.
static dn_status pack_backward(dn_net *net, int layer, const double *dw, const double *db, const double *dm,
                               const double *dv, const double *dg, const double *dbe, int has_bn, hipStream_t st)
{
    ConvWeights &cw = net->cw[layer];
    const dn_layer_desc &d = net->L[layer];
    const int dt = net->o.dtype;
    const int cin_p = cpad(dt, d.cout), cout_p = cpad(dt, cw.cin);
    const int K = d.ksize * d.ksize * cin_p;
    const int k_pad = (K + bk_el(dt) - 1) / bk_el(dt) * bk_el(dt);
    HIPCHK(hipMalloc(&cw.wb, (size_t)cout_p * k_pad * esize(dt)));
    HIPCHK(hipMalloc((void **)&cw.bzero, cout_p * sizeof(float)));
    HIPCHK(hipMalloc((void **)&cw.bscale, cout_p * sizeof(float)));
    HIPCHK(launch_fold_pack(dt, 2, dw, db, dm, dv, dg, dbe, net->o.bn_eps, has_bn, cw.cin, d.cout, d.ksize, d.ksize,
                            cin_p, k_pad, cout_p, cw.wb, cw.bzero, cw.bscale, st));
    cw.kb_pad = k_pad;
    return DN_OK;
}

extern "C" dn_status dn_load_weights(dn_net *net, int layer, const double *w, const double *bias, const double *mean,
                                     const double *var, const double *gamma, const double *beta)
{
    if (!net) return fail(DN_EINVAL, "net is NULL");
    if (layer < 0 || layer >= (int)net->L.size() || net->L[layer].kind != DN_CONV)
        return fail(DN_EINVAL, "layer %d is not a conv layer", layer);
    const dn_layer_desc &d = net->L[layer];
    if (!w || !bias) return fail(DN_EINVAL, "conv layer %d: w and bias are required", layer);
    const bool any_bn = mean || var || gamma || beta;
    const bool all_bn = mean && var && gamma && beta;
    if (d.batchnorm ? !all_bn : any_bn)
        return fail(DN_EINVAL, "conv layer %d: BN arrays must be all present iff the layer has batchnorm", layer);
    std::lock_guard<std::mutex> g(net->mu);
    HIPCHK(hipSetDevice(net->o.device));
    ConvWeights &cw = net->cw[layer];
    free_weights(cw);
    cw.cin = net->in_c[layer];
    const size_t nw = (size_t)d.cout * cw.cin * d.ksize * d.ksize;
    const size_t nvec = d.cout;
    double *dbuf = nullptr;
    const size_t tot = nw + 5 * nvec;
    HIPCHK(hipMalloc(&dbuf, tot * sizeof(double)));
    double *dw = dbuf, *db = dbuf + nw, *dm = db + nvec, *dv = dm + nvec, *dg = dv + nvec, *dbe = dg + nvec;
    hipStream_t st = net->cap_stream;
    dn_status rc = DN_OK;
    auto cp = [&](double *dst, const double *src, size_t n) -> bool {
        return hipMemcpyAsync(dst, src, n * sizeof(double), hipMemcpyHostToDevice, st) == hipSuccess;
    };
    bool ok = cp(dw, w, nw) && cp(db, bias, nvec);
    if (ok && d.batchnorm) ok = cp(dm, mean, nvec) && cp(dv, var, nvec) && cp(dg, gamma, nvec) && cp(dbe, beta, nvec);
    if (!ok) rc = fail(DN_EHIP, "weight upload failed: %s", hipGetErrorString(hipGetLastError()));
    if (rc == DN_OK)
        rc = pack_to(net, layer, net->o.dtype, dw, db, dm, dv, dg, dbe, d.batchnorm, &cw.w, &cw.bias, &cw.wscale, st);
    if (rc == DN_OK && net->o.dtype == DN_FP8_E4M3)
        rc = pack_to(net, layer, F32, dw, db, dm, dv, dg, dbe, d.batchnorm, &cw.w32, &cw.bias32, &cw.wscale32, st);
    if (rc == DN_OK && net->o.dtype != DN_FP8_E4M3) rc = pack_backward(net, layer, dw, db, dm, dv, dg, dbe, d.batchnorm, st);
    if (rc == DN_OK && hipStreamSynchronize(st) != hipSuccess) rc = fail(DN_EHIP, "weight fold/pack failed");
    (void)hipFree(dbuf);
    if (rc != DN_OK) {
        free_weights(cw);
        return rc;
    }
    if (net->o.mode == DN_MODE_PER_LAYER) {
        // host copy of the packed weights: the per-layer mode re-uploads them around every layer
        const size_t vb = (size_t)cw.cout_p * sizeof(float);
        if (hipHostMalloc(&cw.pinned, cw.wbytes + 2 * vb, hipHostMallocDefault) != hipSuccess) {
            free_weights(cw);
            return fail(DN_ENOMEM, "pinned host weights");
        }
        char *hp = (char *)cw.pinned;
        if (hipMemcpy(hp, cw.w, cw.wbytes, hipMemcpyDeviceToHost) != hipSuccess ||
            hipMemcpy(hp + cw.wbytes, cw.bias, vb, hipMemcpyDeviceToHost) != hipSuccess ||
            hipMemcpy(hp + cw.wbytes + vb, cw.wscale, vb, hipMemcpyDeviceToHost) != hipSuccess) {
            free_weights(cw);
            return fail(DN_EHIP, "weight readback failed");
        }
    }
    cw.loaded = true;
    net->calibrated = false;
    drop_graphs(net);
    return DN_OK;
}

// The resident plan of (batch, h, w), built once and shared until the next
// change of weights, scales or tuned tiles.
static dn_status resident_plan(dn_net *net, int batch, int h, int w, std::shared_ptr<const Plan> *out)
{
    const auto key = std::make_tuple(batch, h, w);
    {
        std::lock_guard<std::mutex> g(net->mu);
        auto it = net->plans.find(key);
        if (it != net->plans.end()) {
            *out = it->second;
            return DN_OK;
        }
    }
    auto p = std::make_shared<Plan>();
    STCHK(make_plan(net, net->o.dtype, DN_MODE_RESIDENT, batch, h, w, p.get()));
    std::lock_guard<std::mutex> g(net->mu);
    net->plans[key] = p;
    *out = p;
    return DN_OK;
}

// Captured forwards kept per net (two executable instances each).  Callers
// whose buffers repeat (fixed serving slots) stay far below it; buffers that
// never repeat would otherwise grow the cache without bound.
constexpr size_t MAX_GRAPHS = 4096;

static dn_status forward_resident(dn_net *net, void *arena, size_t arena_bytes, const void *x, int batch, int h,
                                  int w, void *y, hipStream_t s)
{
    const GraphKey key{batch, h, w, x, y, arena};
    if (net->o.use_graph) {
        // a forward captured for these buffers: its plan, weights and scales
        // are unchanged (any change drops the graphs), so replay it directly
        hipGraphExec_t exec = nullptr;
        size_t need = 0;
        {
            std::lock_guard<std::mutex> g(net->mu);
            auto it = net->graphs.find(key);
            if (it != net->graphs.end()) {
                exec = it->second.exec[it->second.next++ & 1];
                need = it->second.total;
            }
        }
        if (exec) {
            if (arena_bytes < need) return fail(DN_ENOMEM, "arena has %zu bytes, plan needs %zu", arena_bytes, need);
            HIPCHK(hipGraphLaunch(exec, s));
            return DN_OK;
        }
    }
    STCHK(check_ready(net, true));
    STCHK(check_dims(net, batch, h, w));
    if (!x || !y) return fail(DN_EINVAL, "x/y are NULL");
    if (!arena) return fail(DN_ESTATE, "no arena bound");
    std::shared_ptr<const Plan> pp;
    STCHK(resident_plan(net, batch, h, w, &pp));
    const Plan &p = *pp;
    if (arena_bytes < p.total) return fail(DN_ENOMEM, "arena has %zu bytes, plan needs %zu", arena_bytes, p.total);
    bool full;
    {
        std::lock_guard<std::mutex> g(net->mu);
        full = net->graphs.size() >= MAX_GRAPHS;
    }
    // without graphs, or with the cache full (buffers that never repeat), launch eagerly
    if (!net->o.use_graph || full) return enqueue_resident(net, p, (char *)arena, (const float *)x, (float *)y, s);
    hipGraph_t graph = nullptr;
    HIPCHK(hipStreamBeginCapture(net->cap_stream, hipStreamCaptureModeThreadLocal));
    dn_status rc = enqueue_resident(net, p, (char *)arena, (const float *)x, (float *)y, net->cap_stream);
    hipError_t e = hipStreamEndCapture(net->cap_stream, &graph);
    if (rc != DN_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc;
    }
    if (e != hipSuccess) return fail(DN_EHIP, "graph capture failed: %s", hipGetErrorString(e));
    dn_net::GraphPair gp;
    for (int i = 0; i < 2 && e == hipSuccess; ++i) e = hipGraphInstantiate(&gp.exec[i], graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
        for (hipGraphExec_t x2 : gp.exec)
            if (x2) (void)hipGraphExecDestroy(x2);
        return fail(DN_EHIP, "graph instantiate failed: %s", hipGetErrorString(e));
    }
    hipGraphExec_t exec = gp.exec[0];
    gp.next = 1;
    gp.total = p.total;
    {
        std::lock_guard<std::mutex> g(net->mu);
        net->graphs[key] = gp;
    }
    HIPCHK(hipGraphLaunch(exec, s));
    return DN_OK;
}

// Naive offload baseline: every layer's input, weights and output cross PCIe
// around its own kernel, with a full synchronisation per layer.
static dn_status forward_per_layer(dn_net *net, const void *x, int batch, int h, int w, void *y, hipStream_t s)
{
    STCHK(check_ready(net, true));
    STCHK(check_dims(net, batch, h, w));
    if (!x || !y) return fail(DN_EINVAL, "x/y are NULL");
    if (!net->arena) return fail(DN_ESTATE, "no arena bound");
    if (is_device_ptr(x) || is_device_ptr(y)) return fail(DN_EINVAL, "per-layer mode takes host x/y");
    Plan p;
    STCHK(make_plan(net, net->o.dtype, DN_MODE_PER_LAYER, batch, h, w, &p));
    if (net->arena_bytes < p.total) return fail(DN_ENOMEM, "arena has %zu bytes, plan needs %zu", net->arena_bytes, p.total);
    char *base = (char *)net->arena;
    // host-side copy of every activation (the CPU-resident data of a naive offload)
    std::vector<unsigned char *> *hv;
    {
        std::lock_guard<std::mutex> g(net->mu);
        auto key = std::make_tuple(batch, h, w);
        hv = &net->host_vals[key];
        if (hv->empty()) {
            for (const Value &v : p.vals) {
                unsigned char *b = nullptr;
                if (hipHostMalloc((void **)&b, v.bytes, hipHostMallocDefault) != hipSuccess) {
                    for (unsigned char *q : *hv) (void)hipHostFree(q);
                    hv->clear();
                    return fail(DN_ENOMEM, "pinned host activations");
                }
                hv->push_back(b);
            }
        }
    }
    const Value &v0 = p.vals[0];
    const size_t xbytes = (size_t)batch * v0.c * h * w * 4;
    // input: host -> device, ingest, device -> host
    const float *xdev = (const float *)(base + p.xin_off);
    if (!p.ops[0].first) {
        HIPCHK(hipMemcpyAsync(base + p.xin_off, x, xbytes, hipMemcpyHostToDevice, s));
        const float in_inv = p.dtype == FP8 ? 1.0f / net->scale[0] : 1.0f;
        HIPCHK(launch_ingest(p.dtype, xdev, batch, v0.c, h, w, v0.cp, in_inv, base + v0.off, s));
        HIPCHK(hipMemcpyAsync((*hv)[0], base + v0.off, v0.bytes, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
    }
    if (p.any_fused) STCHK(zero_counters(p, base, s));
    for (const Op &op : p.ops) {
        if (op.first)
            HIPCHK(hipMemcpyAsync(base + p.xin_off, x, xbytes, hipMemcpyHostToDevice, s));
        else
            HIPCHK(hipMemcpyAsync(base + p.vals[op.in].off, (*hv)[op.in], p.vals[op.in].bytes, hipMemcpyHostToDevice, s));
        if (op.in2 >= 0)
            HIPCHK(hipMemcpyAsync(base + p.vals[op.in2].off, (*hv)[op.in2], p.vals[op.in2].bytes, hipMemcpyHostToDevice, s));
        if (op.kind == OP_CONV) {
            ConvWeights &cw = net->cw[op.conv];
            const size_t vb = (size_t)cw.cout_p * sizeof(float);
            const char *hp = (const char *)cw.pinned;
            HIPCHK(hipMemcpyAsync(cw.w, hp, cw.wbytes, hipMemcpyHostToDevice, s));
            HIPCHK(hipMemcpyAsync(cw.bias, hp + cw.wbytes, vb, hipMemcpyHostToDevice, s));
            HIPCHK(hipMemcpyAsync(cw.wscale, hp + cw.wbytes + vb, vb, hipMemcpyHostToDevice, s));
        }
        STCHK(enqueue_op(net, p, op, base, s, false, -1, 0, xdev));
        HIPCHK(hipMemcpyAsync((*hv)[op.out], base + p.vals[op.out].off, p.vals[op.out].bytes, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
    }
    const Value &vo = p.vals[p.out_val];
    HIPCHK(hipMemcpyAsync(base + vo.off, (*hv)[p.out_val], vo.bytes, hipMemcpyHostToDevice, s));
    const float osc = p.dtype == FP8 ? net->scale[p.out_val] : 1.0f;
    HIPCHK(launch_egress(p.dtype, base + vo.off, batch, vo.c, vo.h, vo.w, vo.cp, osc, (float *)(base + p.yout_off), s));
    HIPCHK(hipMemcpyAsync(y, base + p.yout_off, (size_t)batch * vo.c * vo.h * vo.w * 4, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return DN_OK;
}

extern "C" dn_status dn_forward(dn_net *net, const void *x, int batch, int h, int w, void *y, void *stream)
{
    if (!net) return fail(DN_EINVAL, "net is NULL");
    if (hipSetDevice(net->o.device) != hipSuccess) return fail(DN_EHIP, "hipSetDevice");
    if (net->o.mode == DN_MODE_PER_LAYER) return forward_per_layer(net, x, batch, h, w, y, (hipStream_t)stream);
    return forward_resident(net, net->arena, net->arena_bytes, x, batch, h, w, y, (hipStream_t)stream);
}

extern "C" dn_status dn_forward_arena(dn_net *net, void *arena, size_t arena_bytes, const void *x, int batch, int h,
                                      int w, void *y, void *stream)
{
    if (!net) return fail(DN_EINVAL, "net is NULL");
    if (net->o.mode != DN_MODE_RESIDENT) return fail(DN_EUNSUPPORTED, "dn_forward_arena needs a resident-mode net");
    if (!arena || ((uintptr_t)arena & 255)) return fail(DN_EINVAL, "arena missing or not 256-byte aligned");
    if (hipSetDevice(net->o.device) != hipSuccess) return fail(DN_EHIP, "hipSetDevice");
    return forward_resident(net, arena, arena_bytes, x, batch, h, w, y, (hipStream_t)stream);
}

extern "C" dn_status dn_calibrate(dn_net *net, const float *x, int batch, int h, int w, void *stream)
{
    if (!net) return fail(DN_EINVAL, "net is NULL");
    if (net->o.dtype != DN_FP8_E4M3) return fail(DN_EINVAL, "dn_calibrate is for FP8 nets");
    STCHK(check_ready(net, false));
    STCHK(check_dims(net, batch, h, w));
    if (!x || !is_device_ptr(x)) return fail(DN_EINVAL, "calibration input must be device memory");
    HIPCHK(hipSetDevice(net->o.device));
    hipStream_t s = (hipStream_t)stream;
    // FP32 forward over the unfused layer list (each layer's own tensor gets a scale)
    Plan p;
    STCHK(make_plan(net, F32, DN_MODE_PER_LAYER, batch, h, w, &p));
    char *base = nullptr;
    const size_t nv = p.vals.size();
    HIPCHK(hipMalloc(&base, p.total + align256(nv * sizeof(float))));
    float *amax = (float *)(base + p.total);
    dn_status rc = DN_OK;
    auto run = [&]() -> dn_status {
        HIPCHK(launch_zero_f32(amax, nv, s));
        if (p.any_fused) STCHK(zero_counters(p, base, s));
        const Value &v0 = p.vals[0];
        if (!p.ops[0].first) HIPCHK(launch_ingest(F32, x, batch, v0.c, h, w, v0.cp, 1.0f, base + v0.off, s));
        HIPCHK(launch_amax(x, (size_t)batch * v0.c * h * w, amax, s));
        for (const Op &op : p.ops) {
            STCHK(enqueue_op(net, p, op, base, s, true, -1, 0, x));
            const Value &vo = p.vals[op.out];
            HIPCHK(launch_amax((const float *)(base + vo.off), (size_t)batch * vo.h * vo.w * vo.cp, amax + op.out, s));
        }
        std::vector<float> hm(nv);
        HIPCHK(hipMemcpyAsync(hm.data(), amax, nv * sizeof(float), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        for (size_t v = 0; v < nv; ++v) net->scale[v] = hm[v] > 0.f ? hm[v] / 448.0f : 1.0f;
        // a max pool only selects values: its output keeps its input's scale
        for (size_t i = 0; i < net->L.size(); ++i)
            if (net->L[i].kind == DN_MAXPOOL) net->scale[i + 1] = net->scale[i];
        return DN_OK;
    };
    rc = run();
    (void)hipStreamSynchronize(s);
    (void)hipFree(base);
    if (rc == DN_OK) {
        std::lock_guard<std::mutex> g(net->mu);
        net->calibrated = true;
        drop_graphs(net);
    }
    return rc;
}

// ---------------------------------------------------------------- placement (layer on CPU or GPU)
//
// The paper's offload search (Sec. 3.3, Sec. 4) decides loop by loop whether
// a loop runs on the GPU and inserts the copies its transfer rule (Sec. 3.2)
// implies.  Here the unit is one layer: a gene byte per layer picks the GPU
// kernels or the host FP32 layer code (cpu_layers.cpp), and each layer output
// crosses at most once, right after the layer that produces it, when a layer
// on the other side reads it.

static bool op_on_gpu(const Op &op, const unsigned char *gene)
{
    return gene[op.kind == OP_CONV ? op.conv : op.layer] != 0;
}

struct Crossings {
    std::vector<char> on_gpu;   // per value: produced by a GPU layer (value 0 is the host image)
    std::vector<char> to_dev;   // host-produced value that a GPU layer reads
    std::vector<char> to_host;  // GPU-produced value that a host layer reads
    bool x_to_dev = false;      // a GPU layer reads the image
    bool y_from_dev = false;    // a GPU layer produces the result
};

static Crossings crossings(const Plan &p, const unsigned char *gene)
{
    Crossings c;
    const size_t nv = p.vals.size();
    c.on_gpu.assign(nv, 0);
    c.to_dev.assign(nv, 0);
    c.to_host.assign(nv, 0);
    for (const Op &op : p.ops) c.on_gpu[op.out] = op_on_gpu(op, gene);
    for (const Op &op : p.ops) {
        const bool g = op_on_gpu(op, gene);
        for (int v : {op.in, op.in2}) {
            if (v < 0) continue;
            if (v == 0) {
                if (g) c.x_to_dev = true;
            } else if (g && !c.on_gpu[v]) {
                c.to_dev[v] = 1;
            } else if (!g && c.on_gpu[v]) {
                c.to_host[v] = 1;
            }
        }
    }
    c.y_from_dev = c.on_gpu[p.out_val] != 0;
    return c;
}

static size_t tensor_bytes(const Plan &p, int v)
{
    const Value &x = p.vals[v];
    return (size_t)p.batch * x.h * x.w * x.cp * sizeof(float);
}

static dn_status placed_check(const dn_net *net, const unsigned char *gene, int gene_len)
{
    if (net->o.dtype != DN_F32) return fail(DN_EUNSUPPORTED, "layer placement needs an FP32 net");
    if (net->o.mode != DN_MODE_RESIDENT) return fail(DN_EUNSUPPORTED, "layer placement needs a resident-mode net");
    if (net->o.input_u8) return fail(DN_EUNSUPPORTED, "layer placement takes an FP32 image");
    if (!gene) return DN_OK;
    if (gene_len != (int)net->L.size())
        return fail(DN_EINVAL, "gene has %d values, the net has %zu layers", gene_len, net->L.size());
    for (int i = 0; i < gene_len; ++i)
        if (gene[i] > 1) return fail(DN_EINVAL, "gene value %d at layer %d is not 0 or 1", (int)gene[i], i);
    return DN_OK;
}

// Arena bound for every gene: all values (the all-host plan has every one),
// the larger split-K scratch of the unfused and fully fused plans (a conv is
// either), and the image / result staging.
static dn_status placed_bytes(const dn_net *net, int batch, int h, int w, size_t *bytes)
{
    std::vector<unsigned char> g0(net->L.size(), 0), g1(net->L.size(), 1);
    Plan p0, p1;
    STCHK(make_plan(net, F32, DN_MODE_RESIDENT, batch, h, w, &p0, -1, g0.data()));
    STCHK(make_plan(net, F32, DN_MODE_RESIDENT, batch, h, w, &p1, -1, g1.data()));
    const size_t staging = p0.total - (p0.ws_off + p0.ws_bytes);
    *bytes = p0.ws_off + std::max(p0.ws_bytes, p1.ws_bytes) + staging;
    return DN_OK;
}

// Host copy of every conv's folded FP32 weights, read back from the device
// once (weights are defined once per load, Sec. 3.2) and reordered from the
// packed GEMM layout into the host conv's blocked layout.
static dn_status ensure_cpu_weights(dn_net *net)
{
    std::lock_guard<std::mutex> g(net->mu);
    for (size_t i = 0; i < net->L.size(); ++i) {
        if (net->L[i].kind != DN_CONV) continue;
        ConvWeights &cw = net->cw[i];
        if (!cw.cpu_w.empty()) continue;
        const dn_layer_desc &d = net->L[i];
        const int R = d.ksize, S = d.ksize, cin_p = cw.cin_p, cout_p = cw.cout_p, k_pad = cw.k_pad;
        std::vector<float> packed((size_t)cout_p * k_pad), bias(cout_p);
        HIPCHK(hipMemcpy(packed.data(), cw.w, packed.size() * sizeof(float), hipMemcpyDeviceToHost));
        HIPCHK(hipMemcpy(bias.data(), cw.bias, bias.size() * sizeof(float), hipMemcpyDeviceToHost));
        const bool compact = i == 0 && first_eligible(net, F32);
        const int CP = first_cp(cw.cin), CB = kblock_ch(F32, cin_p, R * S);
        auto wval = [&](int co, int r, int s, int c) -> float {
            size_t k;
            if (compact) {
                if (c >= CP) return 0.0f;
                k = (size_t)r * 16 + s * CP + c;
            } else {
                const int cb = c / CB;
                k = (size_t)(cb * R * S + r * S + s) * CB + (c - cb * CB);
            }
            return packed[(size_t)co * k_pad + k];
        };
        std::vector<float> blocked((size_t)cout_p * R * S * cin_p);
        dncpu::pack_weights(wval, cout_p, R, S, cin_p, blocked.data());
        cw.cpu_w.swap(blocked);
        cw.cpu_b.swap(bias);
    }
    return DN_OK;
}

static void cpu_op(const dn_net *net, const Plan &p, const Op &op, const std::vector<unsigned char *> &hv)
{
    float *out = (float *)hv[op.out];
    const float *in = (const float *)hv[op.in];
    if (op.kind == OP_CONV) {  // never fused: fusion needs both layers on the GPU
        const dn_layer_desc &d = net->L[op.conv];
        const ConvWeights &cw = net->cw[op.conv];
        dncpu::conv(in, p.batch, op.H, op.W, op.cin_p, cw.cpu_w.data(), cw.cpu_b.data(), op.cout_p, d.ksize, d.ksize,
                    d.stride, d.pad, d.activation, net->o.leaky_slope, out, op.Ho, op.Wo);
    } else if (op.kind == OP_POOL) {
        const dn_layer_desc &d = net->L[op.layer];
        const Value &vi = p.vals[op.in];
        dncpu::maxpool(in, p.batch, vi.h, vi.w, vi.cp, d.ksize, d.stride, out, op.Ho, op.Wo);
    } else {
        dncpu::add(in, (const float *)hv[op.in2], out, tensor_bytes(p, op.out) / sizeof(float));
    }
}

static dn_status forward_placed(dn_net *net, const unsigned char *gene, const float *x, int batch, int h, int w,
                                float *y, double timeout_s, hipStream_t s)
{
    const auto t0 = std::chrono::steady_clock::now();
    STCHK(check_ready(net, true));
    STCHK(check_dims(net, batch, h, w));
    if (!x || !y) return fail(DN_EINVAL, "x/y are NULL");
    if (is_device_ptr(x) || is_device_ptr(y)) return fail(DN_EINVAL, "the placed forward takes host x/y");
    if (!net->arena) return fail(DN_ESTATE, "no arena bound");
    size_t need = 0;
    STCHK(placed_bytes(net, batch, h, w, &need));
    if (net->arena_bytes < need) return fail(DN_ENOMEM, "arena has %zu bytes, placement needs %zu", net->arena_bytes, need);
    STCHK(ensure_cpu_weights(net));
    Plan p;
    STCHK(make_plan(net, F32, DN_MODE_RESIDENT, batch, h, w, &p, -1, gene));
    const Crossings c = crossings(p, gene);
    std::vector<unsigned char *> *hv;
    {
        std::lock_guard<std::mutex> g(net->mu);
        hv = &net->host_place[std::make_tuple(batch, h, w)];
        if (hv->empty()) {
            for (size_t v = 0; v < p.vals.size(); ++v) {
                unsigned char *b = nullptr;
                if (hipHostMalloc((void **)&b, std::max<size_t>(tensor_bytes(p, (int)v), 16), hipHostMallocDefault) !=
                    hipSuccess) {
                    for (unsigned char *q : *hv) (void)hipHostFree(q);
                    hv->clear();
                    return fail(DN_ENOMEM, "pinned host activations");
                }
                hv->push_back(b);
            }
        }
    }
    char *base = (char *)net->arena;
    const Value &v0 = p.vals[0];
    const float *xdev = (const float *)(base + p.xin_off);
    if (c.x_to_dev) {
        HIPCHK(hipMemcpyAsync(base + p.xin_off, x, (size_t)batch * v0.c * h * w * sizeof(float),
                              hipMemcpyHostToDevice, s));
        if (!p.ops[0].first) HIPCHK(launch_ingest(F32, xdev, batch, v0.c, h, w, v0.cp, 1.0f, base + v0.off, s));
    } else {
        dncpu::ingest(x, batch, v0.c, h, w, v0.cp, (float *)(*hv)[0]);
    }
    if (p.any_fused) STCHK(zero_counters(p, base, s));
    bool pending = false;  // device->host copies not waited for yet
    for (const Op &op : p.ops) {
        if (op_on_gpu(op, gene)) {
            STCHK(enqueue_op(net, p, op, base, s, false, -1, 0, xdev));
            if (c.to_host[op.out]) {
                HIPCHK(hipMemcpyAsync((*hv)[op.out], base + p.vals[op.out].off, tensor_bytes(p, op.out),
                                      hipMemcpyDeviceToHost, s));
                pending = true;
            }
        } else {
            if (pending) {
                HIPCHK(hipStreamSynchronize(s));
                pending = false;
            }
            cpu_op(net, p, op, *hv);
            if (c.to_dev[op.out])
                HIPCHK(hipMemcpyAsync(base + p.vals[op.out].off, (*hv)[op.out], tensor_bytes(p, op.out),
                                      hipMemcpyHostToDevice, s));
        }
        if (timeout_s > 0.0 &&
            std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count() > timeout_s) {
            (void)hipStreamSynchronize(s);
            return fail(DN_ETIMEDOUT, "placed forward passed its %.3f s limit after layer %d", timeout_s, op.layer);
        }
    }
    const Value &vo = p.vals[p.out_val];
    if (c.y_from_dev) {
        HIPCHK(launch_egress(F32, base + vo.off, batch, vo.c, vo.h, vo.w, vo.cp, 1.0f, (float *)(base + p.yout_off), s));
        HIPCHK(hipMemcpyAsync(y, base + p.yout_off, (size_t)batch * vo.c * vo.h * vo.w * sizeof(float),
                              hipMemcpyDeviceToHost, s));
    } else {
        if (pending) HIPCHK(hipStreamSynchronize(s));
        dncpu::egress((const float *)(*hv)[p.out_val], batch, vo.c, vo.h, vo.w, vo.cp, y);
    }
    // also waits for host->device copies still reading the pinned host buffers
    HIPCHK(hipStreamSynchronize(s));
    return DN_OK;
}

extern "C" dn_status dn_placed_arena_bytes(const dn_net *net, int batch, int h, int w, size_t *bytes)
{
    if (!net || !bytes) return fail(DN_EINVAL, "NULL argument");
    STCHK(placed_check(net, nullptr, 0));
    return placed_bytes(net, batch, h, w, bytes);
}

extern "C" dn_status dn_placed_transfers(const dn_net *net, const unsigned char *gene, int gene_len, int batch, int h,
                                         int w, int *h2d, int *d2h, size_t *h2d_bytes, size_t *d2h_bytes)
{
    if (!net || !gene) return fail(DN_EINVAL, "NULL argument");
    STCHK(placed_check(net, gene, gene_len));
    Plan p;
    STCHK(make_plan(net, F32, DN_MODE_RESIDENT, batch, h, w, &p, -1, gene));
    const Crossings c = crossings(p, gene);
    int nh = 0, nd = 0;
    size_t bh = 0, bd = 0;
    if (c.x_to_dev) {
        ++nh;
        bh += (size_t)batch * p.vals[0].c * h * w * sizeof(float);
    }
    if (c.y_from_dev) {
        const Value &vo = p.vals[p.out_val];
        ++nd;
        bd += (size_t)batch * vo.c * vo.h * vo.w * sizeof(float);
    }
    for (size_t v = 0; v < p.vals.size(); ++v) {
        if (c.to_dev[v]) { ++nh; bh += tensor_bytes(p, (int)v); }
        if (c.to_host[v]) { ++nd; bd += tensor_bytes(p, (int)v); }
    }
    if (h2d) *h2d = nh;
    if (d2h) *d2h = nd;
    if (h2d_bytes) *h2d_bytes = bh;
    if (d2h_bytes) *d2h_bytes = bd;
    return DN_OK;
}

extern "C" dn_status dn_forward_placed(dn_net *net, const unsigned char *gene, int gene_len, const float *x, int batch,
                                       int h, int w, float *y, double timeout_s, void *stream)
{
    if (!net || !gene) return fail(DN_EINVAL, "NULL argument");
    STCHK(placed_check(net, gene, gene_len));
    if (hipSetDevice(net->o.device) != hipSuccess) return fail(DN_EHIP, "hipSetDevice");
    return forward_placed(net, gene, x, batch, h, w, y, timeout_s, (hipStream_t)stream);
}

extern "C" dn_status dn_cpu_conv2d(const dn_conv_desc *d, const float *x, const float *w, const float *bias, float *y)
{
    if (!d || !x || !w || !bias || !y) return fail(DN_EINVAL, "NULL argument");
    if (d->dtype != DN_F32 || d->pool || d->residual || d->input_nchw)
        return fail(DN_EUNSUPPORTED, "host conv: FP32, no fused pool / residual, NHWC input only");
    if (d->batch <= 0 || d->in_h <= 0 || d->in_w <= 0 || d->in_c <= 0 || d->cout <= 0 || d->ksize <= 0 ||
        d->stride <= 0 || d->pad < 0)
        return fail(DN_EINVAL, "bad conv geometry");
    if (d->activation != DN_ACT_LINEAR && d->activation != DN_ACT_LEAKY) return fail(DN_EINVAL, "unknown activation");
    const int Ho = out_side_conv(d->in_h, d->ksize, d->stride, d->pad);
    const int Wo = out_side_conv(d->in_w, d->ksize, d->stride, d->pad);
    if (Ho <= 0 || Wo <= 0) return fail(DN_EINVAL, "input too small for the filter");
    const int cin_p = cpad(F32, d->in_c), cout_p = cpad(F32, d->cout), k = d->ksize;
    auto wval = [&](int co, int r, int s, int c) -> float {
        if (co >= d->cout || c >= d->in_c) return 0.0f;
        return w[(((size_t)co * d->in_c + c) * k + r) * k + s];
    };
    std::vector<float> blocked((size_t)cout_p * k * k * cin_p), b(cout_p, 0.0f);
    dncpu::pack_weights(wval, cout_p, k, k, cin_p, blocked.data());
    std::copy(bias, bias + d->cout, b.begin());
    dncpu::conv(x, d->batch, d->in_h, d->in_w, cin_p, blocked.data(), b.data(), cout_p, k, k, d->stride, d->pad,
                d->activation, d->leaky_slope, y, Ho, Wo);
    return DN_OK;
}

extern "C" dn_status dn_cpu_maxpool(const dn_pool_desc *d, const float *x, float *y)
{
    if (!d || !x || !y) return fail(DN_EINVAL, "NULL argument");
    if (d->dtype != DN_F32) return fail(DN_EUNSUPPORTED, "host max pool: FP32 only");
    if (d->batch <= 0 || d->h <= 0 || d->w <= 0 || d->c <= 0 || d->size <= 0 || d->stride <= 0)
        return fail(DN_EINVAL, "bad pool geometry");
    dncpu::maxpool(x, d->batch, d->h, d->w, cpad(F32, d->c), d->size, d->stride, y, out_side_pool(d->h, d->stride),
                   out_side_pool(d->w, d->stride));
    return DN_OK;
}

// ---------------------------------------------------------------- GA placement search

static dn_status ga_params(const dn_ga_params *p, int L, dnga::Params *out)
{
    if (!p) return fail(DN_EINVAL, "GA parameters are NULL");
    if (L < 1) return fail(DN_EINVAL, "gene length %d < 1", L);
    if (p->population < 1 || p->generations < 1)
        return fail(DN_EINVAL, "population %d / generations %d must be >= 1", p->population, p->generations);
    if (!(p->crossover >= 0.0 && p->crossover <= 1.0) || !(p->mutation >= 0.0 && p->mutation <= 1.0))
        return fail(DN_EINVAL, "crossover / mutation rates must lie in [0, 1]");
    if (!(p->timeout_s > 0.0) || !(p->penalty_s > 0.0)) return fail(DN_EINVAL, "timeout and penalty must be > 0");
    *out = dnga::Params{p->population, p->generations, p->crossover, p->mutation, p->timeout_s, p->penalty_s,
                        (uint64_t)p->seed};
    return DN_OK;
}

extern "C" dn_status dn_ga_next_generation(const dn_ga_params *p, int gene_len, const unsigned char *pop,
                                           const double *seconds, unsigned char *next, unsigned long long *rng_state)
{
    dnga::Params gp;
    STCHK(ga_params(p, gene_len, &gp));
    if (!pop || !seconds || !next || !rng_state) return fail(DN_EINVAL, "NULL argument");
    for (int i = 0; i < gp.population; ++i)
        if (!(seconds[i] > 0.0) || std::isinf(seconds[i])) return fail(DN_EINVAL, "time %d is not positive and finite", i);
    uint64_t st = *rng_state;
    dnga::next_generation(gp, gene_len, pop, seconds, next, &st);
    *rng_state = st;
    return DN_OK;
}

extern "C" dn_status dn_ga_search(const dn_ga_params *p, int gene_len, dn_ga_measure_fn measure, void *user,
                                  unsigned char *best_gene, double *gen_best, dn_ga_result *res)
{
    dnga::Params gp;
    STCHK(ga_params(p, gene_len, &gp));
    if (!measure || !best_gene) return fail(DN_EINVAL, "NULL argument");
    dnga::Result r;
    auto fn = [&](const uint8_t *g, double timeout) { return measure(g, gene_len, timeout, user); };
    if (!dnga::search(gp, gene_len, fn, best_gene, gen_best, &r)) return fail(DN_ESTATE, "the measurement aborted the search");
    if (res) *res = dn_ga_result{r.best_seconds, r.evaluations, r.memo_hits};
    return DN_OK;
}

extern "C" dn_status dn_ga_place(dn_net *net, const dn_ga_params *p, const float *x, int batch, int h, int w, float *y,
                                 int reps, void *stream, unsigned char *best_gene, double *gen_best, dn_ga_result *res)
{
    if (!net || !best_gene) return fail(DN_EINVAL, "NULL argument");
    const int L = (int)net->L.size();
    dnga::Params gp;
    STCHK(ga_params(p, L, &gp));
    STCHK(placed_check(net, nullptr, 0));
    if (reps < 1) return fail(DN_EINVAL, "reps %d < 1", reps);
    HIPCHK(hipSetDevice(net->o.device));
    hipStream_t s = (hipStream_t)stream;
    for (unsigned char v : {1, 0}) {  // warm-up: host buffers, host weights, kernels
        std::vector<unsigned char> g(L, v);
        STCHK(forward_placed(net, g.data(), x, batch, h, w, y, 0.0, s));
    }
    dn_status err = DN_OK;
    auto fn = [&](const uint8_t *g, double timeout) -> double {
        std::vector<double> t;
        for (int r = 0; r < reps; ++r) {
            const auto a = std::chrono::steady_clock::now();
            const dn_status st = forward_placed(net, g, x, batch, h, w, y, timeout, s);
            const double dt = std::chrono::duration<double>(std::chrono::steady_clock::now() - a).count();
            if (st == DN_ETIMEDOUT) return -1.0;
            if (st != DN_OK) {
                err = st;
                return std::nan("");
            }
            t.push_back(dt);
        }
        std::sort(t.begin(), t.end());
        return t[t.size() / 2];
    };
    dnga::Result r;
    if (!dnga::search(gp, L, fn, best_gene, gen_best, &r)) return err;  // dn_last_error holds the forward's message
    if (res) *res = dn_ga_result{r.best_seconds, r.evaluations, r.memo_hits};
    return DN_OK;
}

// ---------------------------------------------------------------- autotuner

// $DN_TUNE_CACHE holds lines "<device key>/<conv signature> <tile> <splits>";
// only lines whose device key is this net's (same GPU architecture, HIP
// runtime version and tile table) are used, so a cache written elsewhere
// never selects tiles here.  Lines of other keys are kept when saving.
static void read_tune_file(const char *path, std::vector<std::pair<std::string, std::pair<int, int>>> *out)
{
    FILE *f = fopen(path, "r");
    if (!f) return;
    char key[512];
    int t, s;
    while (fscanf(f, "%511s %d %d", key, &t, &s) == 3) out->push_back({key, {t, s}});
    fclose(f);
}

static void load_tune_cache(dn_net *net)
{
    const char *path = getenv("DN_TUNE_CACHE");
    if (!path) return;
    std::vector<std::pair<std::string, std::pair<int, int>>> lines;
    read_tune_file(path, &lines);
    const std::string pre = net->tune_key + "/";
    for (auto &l : lines) {
        if (l.first.compare(0, pre.size(), pre) != 0) continue;
        const int t = l.second.first, s = l.second.second;
        if (((t >= 0 && t < tile_count()) || is_halo(t)) && s >= 1)
            net->tuned[l.first.substr(pre.size())] = {t, s};
    }
}

static void save_tune_cache(const dn_net *net)
{
    const char *path = getenv("DN_TUNE_CACHE");
    if (!path) return;
    std::vector<std::pair<std::string, std::pair<int, int>>> lines;
    read_tune_file(path, &lines);
    const std::string pre = net->tune_key + "/";
    FILE *f = fopen(path, "w");
    if (!f) return;
    for (auto &l : lines)
        if (l.first.compare(0, pre.size(), pre) != 0)
            fprintf(f, "%s %d %d\n", l.first.c_str(), l.second.first, l.second.second);
    for (auto &kv : net->tuned) fprintf(f, "%s%s %d %d\n", pre.c_str(), kv.first.c_str(), kv.second.first, kv.second.second);
    fclose(f);
}

// The tuned choice: the fastest candidate, except that candidates within
// `tie` of it count as tied and the tie goes to the first in a fixed order
// (fewest splits, then lowest config index), so that two configurations whose
// timings differ by run-to-run noise do not trade places between runs.  The
// candidates within TUNE_TIE of the fastest in the first, short timing are
// timed again, longer and interleaved, and the pick among them uses the
// narrower TUNE_TIE_FINE.
constexpr float TUNE_TIE = 0.03f, TUNE_TIE_FINE = 0.01f;
static void pick_tuned(const std::vector<std::tuple<float, int, int>> &timed, int *tile, int *splits,
                       float tie = TUNE_TIE)
{
    if (timed.empty()) return;
    float best = 1e30f;
    for (const auto &c : timed) best = std::min(best, std::get<0>(c));
    bool have = false;
    for (const auto &c : timed) {
        if (std::get<0>(c) > best * (1.0f + tie)) continue;
        const int t = std::get<1>(c), sp = std::get<2>(c);
        if (!have || sp < *splits || (sp == *splits && t < *tile)) {
            *tile = t;
            *splits = sp;
            have = true;
        }
    }
}

static bool tile_fits(int tile, int cout_p)
{
    const TileCfg t = tile_cfg(tile);
    // avoid tiles whose N extent is more than 4x the layer width (pure waste)
    return t.bn <= std::max(16, cout_p) * 4 && t.bn <= std::max(cout_p, 16) * 2;
}

extern "C" dn_status dn_autotune(dn_net *net, int batch, int h, int w, void *stream)
{
    if (!net) return fail(DN_EINVAL, "net is NULL");
    if (net->o.mode != DN_MODE_RESIDENT) return fail(DN_EUNSUPPORTED, "autotune runs on resident-mode nets");
    STCHK(check_ready(net, true));
    STCHK(check_dims(net, batch, h, w));
    if (!net->arena) return fail(DN_ESTATE, "no arena bound");
    HIPCHK(hipSetDevice(net->o.device));
    hipStream_t s = (hipStream_t)stream;
    load_tune_cache(net);
    // plan with the largest split-K candidate so the scratch region is big enough
    Plan p;
    STCHK(make_plan(net, net->o.dtype, DN_MODE_RESIDENT, batch, h, w, &p));
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    char *base = (char *)net->arena;
    dn_status rc = zero_counters(p, base, s);
    for (const Op &op : p.ops) {
        if (rc != DN_OK) break;
        if (op.kind != OP_CONV || op.first) continue;
        const dn_layer_desc &d = net->L[op.conv];
        const bool inv = net->o.batch_invariant != 0;
        const std::string sig = conv_sig(p.dtype, op, batch, d.ksize, d.stride, inv);
        if (net->tuned.count(sig)) continue;
        const int M = batch * (op.pool ? op.Ho * 2 : op.Ho) * (op.pool ? op.Wo * 2 : op.Wo);
        const int nkt = net->cw[op.conv].k_pad / bk_el(p.dtype);
        std::vector<std::tuple<float, int, int>> timed;  // (ms, tile, splits)
        // mean time of `iters` back-to-back launches of one configuration
        auto time_cfg = [&](int t, int sp, int iters) -> float {
            float ms = 0.f;
            if (hipEventRecord(e0, s) != hipSuccess) rc = fail(DN_EHIP, "event");
            for (int it = 0; it < iters && rc == DN_OK; ++it) rc = enqueue_op(net, p, op, base, s, false, t, sp);
            if (rc == DN_OK && (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess))
                rc = fail(DN_EHIP, "tuning launch failed: %s", hipGetErrorString(hipGetLastError()));
            if (rc == DN_OK) (void)hipEventElapsedTime(&ms, e0, e1);
            return ms / iters;
        };
        std::vector<int> cands;
        if (op_halo_ok(net, p.dtype, op, net->cw[op.conv].k_pad)) cands.push_back(HALO_TILE);
        if (op_halo2_ok(net, p.dtype, op, net->cw[op.conv].k_pad)) cands.push_back(HALO2_TILE);
        for (int t = 0; t < tile_count(); ++t)
            if (tile_fits(t, op.cout_p)) cands.push_back(t);
        for (int t : cands) {
            if (rc != DN_OK) break;
            const TileCfg tc = is_halo(t) ? TileCfg{1 << 30, 1 << 30, 1, 1} : tile_cfg(t);
            const long tiles = (long)((M + tc.bm - 1) / tc.bm) * ((op.cout_p + tc.bn - 1) / tc.bn);
            const int sp_lo = inv ? invariant_splits(nkt) : 1, sp_hi = inv ? sp_lo : 16;
            for (int sp = sp_lo; sp <= sp_hi && rc == DN_OK; sp *= 2) {
                if (inv && !invariant_tile_ok(p.dtype, t, sp)) break;
                if (is_halo(t) && sp > 1) break;
                if (!inv && sp > 1 && (tiles * sp > 4 * 256 || nkt / sp < 2)) break;
                const size_t need = sp > 1 ? (size_t)sp * M * op.cout_p * 4 : 0;
                if (p.ws_off + need > net->arena_bytes) continue;
                float ms = 0.f;
                for (int rep = 0; rep < 2 && rc == DN_OK; ++rep)  // rep 0 = warm-up
                    ms = time_cfg(t, sp, rep ? 5 : 1);
                if (rc == DN_OK) timed.emplace_back(ms, t, sp);
            }
        }
        if (rc != DN_OK) break;
        // the near-ties again: three rounds of 20 launches each, round-robin
        // over the candidates so that a clock change affects them alike; each
        // keeps the median of its rounds
        float best = 1e30f;
        for (const auto &c : timed) best = std::min(best, std::get<0>(c));
        std::vector<size_t> near;
        for (size_t i = 0; i < timed.size(); ++i)
            if (std::get<0>(timed[i]) <= best * (1.0f + TUNE_TIE)) near.push_back(i);
        if (near.size() > 1) {
            std::vector<std::vector<float>> rounds(near.size());
            for (int r = 0; r < 3 && rc == DN_OK; ++r)
                for (size_t k = 0; k < near.size() && rc == DN_OK; ++k) {
                    const auto &c = timed[near[k]];
                    rounds[k].push_back(time_cfg(std::get<1>(c), std::get<2>(c), 20));
                }
            if (rc != DN_OK) break;
            std::vector<std::tuple<float, int, int>> fine;
            for (size_t k = 0; k < near.size(); ++k) {
                std::sort(rounds[k].begin(), rounds[k].end());
                fine.emplace_back(rounds[k][1], std::get<1>(timed[near[k]]), std::get<2>(timed[near[k]]));
            }
            timed.swap(fine);
        }
        int bt = op.tile, bs = op.splits;
        pick_tuned(timed, &bt, &bs, near.size() > 1 ? TUNE_TIE_FINE : TUNE_TIE);
        std::lock_guard<std::mutex> g(net->mu);
        net->tuned[sig] = {bt, bs};
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc == DN_OK) {
        std::lock_guard<std::mutex> g(net->mu);
        save_tune_cache(net);
        drop_graphs(net);
    }
    return rc;
}

extern "C" dn_status dn_layer_plan(const dn_net *net, int layer, int batch, int h, int w, int *tile, int *splits,
                                   int *fused_pool, int *fused_res)
{
    if (!net) return fail(DN_EINVAL, "net is NULL");
    Plan p;
    STCHK(make_plan(net, net->o.dtype, DN_MODE_RESIDENT, batch, h, w, &p));
    for (const Op &op : p.ops) {
        if (op.kind == OP_CONV && op.conv == layer) {
            if (tile) *tile = op.first ? -2 : op.tile;
            if (splits) *splits = op.splits;
            if (fused_pool) *fused_pool = op.pool;
            if (fused_res) *fused_res = op.res;
            return DN_OK;
        }
    }
    return fail(DN_EINVAL, "layer %d is not a conv layer", layer);
}

// ---------------------------------------------------------------- Jacobi / Laplace

static dn_status jacobi_check(int n, int m, int iters)
{
    if (n <= 0 || m <= 0 || iters < 0) return fail(DN_EINVAL, "jacobi: non-positive size or negative iterations");
    if ((size_t)n * m >= ((size_t)1 << 40)) return fail(DN_EINVAL, "jacobi: grid too large");
    return DN_OK;
}

// Device-resident: the grid and its partner buffer stay in HBM for all the
// iterations; no host round-trip.  u holds the result.
extern "C" dn_status dn_jacobi(double *u, double *work, int n, int m, int iters, double *max_change, void *stream)
{
    STCHK(jacobi_check(n, m, iters));
    if (!u || !work) return fail(DN_EINVAL, "jacobi: NULL grid");
    hipStream_t s = (hipStream_t)stream;
    const size_t bytes = (size_t)n * m * sizeof(double);
    if (iters == 0) {
        if (max_change) HIPCHK(launch_zero_f32((float *)max_change, 2, s));  // a fill kernel, not a memset node
        return DN_OK;
    }
    HIPCHK(hipMemcpyAsync(work, u, bytes, hipMemcpyDeviceToDevice, s));  // boundary values in both buffers
    double *a = u, *b = work;
    for (int it = 0; it < iters; ++it) {
        const bool last = it + 1 == iters;
        HIPCHK(launch_jacobi_step(a, b, n, m, last ? (unsigned long long *)max_change : nullptr, s));
        std::swap(a, b);
    }
    if (a != u) HIPCHK(hipMemcpyAsync(u, a, bytes, hipMemcpyDeviceToDevice, s));
    return DN_OK;
}

// The naive offload the paper's rule removes: the grid lives on the host and
// crosses PCIe in both directions around every iteration, with a full
// synchronisation each time.  Synchronous.
extern "C" dn_status dn_jacobi_per_iteration(double *u_host, double *dev_a, double *dev_b, int n, int m, int iters,
                                             double *max_change_host, void *stream)
{
    STCHK(jacobi_check(n, m, iters));
    if (!u_host || !dev_a || !dev_b) return fail(DN_EINVAL, "jacobi: NULL buffer");
    if (is_device_ptr(u_host)) return fail(DN_EINVAL, "jacobi per-iteration mode takes a host grid");
    hipStream_t s = (hipStream_t)stream;
    const size_t bytes = (size_t)n * m * sizeof(double);
    unsigned long long *dmax = nullptr;
    HIPCHK(hipMalloc(&dmax, sizeof(unsigned long long)));
    dn_status rc = DN_OK;
    unsigned long long hmax = 0;
    for (int it = 0; it < iters && rc == DN_OK; ++it) {
        if (hipMemcpyAsync(dev_a, u_host, bytes, hipMemcpyHostToDevice, s) != hipSuccess ||
            hipMemcpyAsync(dev_b, dev_a, bytes, hipMemcpyDeviceToDevice, s) != hipSuccess ||
            launch_jacobi_step(dev_a, dev_b, n, m, dmax, s) != hipSuccess ||
            hipMemcpyAsync(u_host, dev_b, bytes, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipMemcpyAsync(&hmax, dmax, sizeof hmax, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            rc = fail(DN_EHIP, "jacobi iteration %d failed", it);
    }
    (void)hipFree(dmax);
    if (rc == DN_OK && max_change_host) {
        double d;
        memcpy(&d, &hmax, sizeof d);
        *max_change_host = iters > 0 ? d : 0.0;
    }
    return rc;
}

// ---------------------------------------------------------------- detection

static dn_status detect_check(int batch, int anchors, int classes, int h, int w)
{
    if (batch <= 0 || anchors <= 0 || classes <= 0 || h <= 0 || w <= 0)
        return fail(DN_EINVAL, "detect: non-positive size");
    if (anchors > DETECT_MAX_ANCHORS) return fail(DN_EUNSUPPORTED, "detect: at most %d anchors", DETECT_MAX_ANCHORS);
    if ((long)h * w * anchors > DETECT_MAX_BOXES)
        return fail(DN_EUNSUPPORTED, "detect: h*w*anchors must be <= %d", DETECT_MAX_BOXES);
    return DN_OK;
}

extern "C" dn_status dn_detect_workspace(int batch, int anchors, int classes, int h, int w, size_t *bytes)
{
    if (!bytes) return fail(DN_EINVAL, "bytes is NULL");
    STCHK(detect_check(batch, anchors, classes, h, w));
    const size_t B = (size_t)h * w * anchors;
    *bytes = align256((size_t)batch * classes * B * 4) + (size_t)batch * B * 16;
    return DN_OK;
}

extern "C" dn_status dn_detect(const float *y, int batch, int anchors, int classes, int h, int w,
                               const float *anchor_wh, float thresh, float nms_thresh, int max_det,
                               void *workspace, size_t ws_bytes, float *dets, int *det_index, int *counts,
                               void *stream)
{
    STCHK(detect_check(batch, anchors, classes, h, w));
    if (!y || !anchor_wh || !workspace || !dets || !det_index || !counts) return fail(DN_EINVAL, "detect: NULL pointer");
    if (max_det <= 0) return fail(DN_EINVAL, "detect: max_det must be positive");
    if (!(thresh == thresh) || !(nms_thresh == nms_thresh)) return fail(DN_EINVAL, "detect: NaN threshold");
    size_t need = 0;
    STCHK(dn_detect_workspace(batch, anchors, classes, h, w, &need));
    if (ws_bytes < need) return fail(DN_EINVAL, "detect: workspace has %zu bytes, needs %zu", ws_bytes, need);
    DetectArgs a{};
    a.y = y;
    for (int i = 0; i < 2 * anchors; ++i) a.anchors[i] = anchor_wh[i];
    a.N = batch; a.A = anchors; a.C = classes; a.H = h; a.W = w;
    a.thresh = thresh; a.nms_thresh = nms_thresh; a.max_det = max_det;
    const size_t B = (size_t)h * w * anchors;
    a.score = (float *)workspace;
    a.box = (float *)((char *)workspace + align256((size_t)batch * classes * B * 4));
    a.dets = dets; a.det_index = det_index; a.counts = counts;
    HIPCHK(launch_detect(a, (hipStream_t)stream));
    return DN_OK;
}

extern "C" dn_status dn_detect_noalloc(const float *y, int batch, int anchors, int classes, int h, int w,
                                       const float *anchor_wh, float thresh, float nms_thresh, int max_det,
                                       float *dets, int *det_index, int *counts, void *stream)
{
    STCHK(detect_check(batch, anchors, classes, h, w));
    size_t need = 0;
    STCHK(dn_detect_workspace(batch, anchors, classes, h, w, &need));
    if (need > DETECT_NOALLOC_BYTES)
        return fail(DN_EINVAL, "detect (no allocation): the decode needs %zu bytes, the fixed scratch holds %zu; "
                    "use dn_detect with a workspace", need, DETECT_NOALLOC_BYTES);
    void *ws = nullptr;
    HIPCHK(detect_scratch(&ws));
    return dn_detect(y, batch, anchors, classes, h, w, anchor_wh, thresh, nms_thresh, max_det, ws, need, dets,
                     det_index, counts, stream);
}

extern "C" dn_status dn_mfma_peak(int dtype, int device, double *tflops)
{
    if (!tflops) return fail(DN_EINVAL, "tflops is NULL");
    STCHK(check_dtype(dtype));
    HIPCHK(hipSetDevice(device));
    int cus = 0;
    HIPCHK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device));
    const int blocks = cus * 8, iters = dtype == FP8 ? 2000 : 4000;  // 8 waves per SIMD
    float *out = nullptr;
    HIPCHK(hipMalloc(&out, (size_t)blocks * 256 * sizeof(float)));
    hipStream_t s = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    dn_status rc = DN_OK;
    float best = 0.f;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
        hipEventCreate(&e1) != hipSuccess)
        rc = fail(DN_EHIP, "stream / event creation failed");
    if (rc == DN_OK && (launch_mfma_peak(dtype, out, blocks, 200, s) != hipSuccess || hipStreamSynchronize(s) != hipSuccess))
        rc = fail(DN_EHIP, "probe warm-up failed");
    for (int rep = 0; rep < 3 && rc == DN_OK; ++rep) {
        float ms = 0.f;
        if (hipEventRecord(e0, s) != hipSuccess || launch_mfma_peak(dtype, out, blocks, iters, s) != hipSuccess ||
            hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
            rc = fail(DN_EHIP, "probe launch failed");
            break;
        }
        if (best == 0.f || ms < best) best = ms;
    }
    if (rc == DN_OK) *tflops = mfma_peak_flops_per_launch(dtype, blocks, iters) / (best * 1e-3) / 1e12;
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (s) (void)hipStreamDestroy(s);
    (void)hipFree(out);
    return rc;
}

extern "C" dn_status dn_time_layer(dn_net *net, int layer, int batch, int h, int w, int iters, void *stream, float *avg_ms)
{
    if (!net || !avg_ms || iters <= 0) return fail(DN_EINVAL, "bad argument");
    STCHK(check_ready(net, true));
    STCHK(check_dims(net, batch, h, w));
    if (!net->arena) return fail(DN_ESTATE, "no arena bound");
    HIPCHK(hipSetDevice(net->o.device));
    Plan p;
    STCHK(make_plan(net, net->o.dtype, DN_MODE_RESIDENT, batch, h, w, &p));
    if (net->arena_bytes < p.total) return fail(DN_ENOMEM, "arena too small");
    const Op *found = nullptr;
    for (const Op &op : p.ops)
        if (op.layer == layer || op.conv == layer) found = &op;
    if (!found) return fail(DN_EINVAL, "no op computes layer %d", layer);
    hipStream_t s = (hipStream_t)stream;
    float *xin = nullptr;
    if (found->first) {  // the first-layer kernel reads an NCHW image: time it on zeros
        const size_t xb = (size_t)batch * net->o.in_c * h * w * sizeof(float);
        HIPCHK(hipMalloc(&xin, xb));
        if (hipMemsetAsync(xin, 0, xb, s) != hipSuccess) {
            (void)hipFree(xin);
            return fail(DN_EHIP, "memset");
        }
    }
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    dn_status rc = finish_in_kernel(found->tile, found->splits) ? zero_counters(p, (char *)net->arena, s) : DN_OK;
    if (rc == DN_OK && hipEventRecord(e0, s) != hipSuccess) rc = fail(DN_EHIP, "event record");
    for (int i = 0; i < iters && rc == DN_OK; ++i) rc = enqueue_op(net, p, *found, (char *)net->arena, s, false, -1, 0, xin);
    if (rc == DN_OK && (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess))
        rc = fail(DN_EHIP, "timed launches failed");
    float ms = 0.f;
    if (rc == DN_OK) (void)hipEventElapsedTime(&ms, e0, e1);
    *avg_ms = ms / iters;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (xin) {
        (void)hipStreamSynchronize(s);
        (void)hipFree(xin);
    }
    return rc;
}

// ---------------------------------------------------------------- standalone layers

static dn_status conv_geometry(const dn_conv_desc *d, ConvArgs *a, int *tile, int *splits, size_t *wbytes,
                               size_t *vbytes, size_t *wsbytes)
{
    if (!d) return fail(DN_EINVAL, "desc is NULL");
    STCHK(check_dtype(d->dtype));
    if (d->batch <= 0 || d->in_h <= 0 || d->in_w <= 0 || d->in_c <= 0 || d->cout <= 0 || d->ksize <= 0 ||
        d->stride <= 0 || d->pad < 0)
        return fail(DN_EINVAL, "conv desc: non-positive size");
    if (d->activation != DN_ACT_LINEAR && d->activation != DN_ACT_LEAKY) return fail(DN_EINVAL, "conv desc: activation");
    if (d->pool != 0 && d->pool != 2) return fail(DN_EUNSUPPORTED, "conv desc: only a fused 2x2 stride-2 pool is supported");
    if (d->pool && d->residual) return fail(DN_EUNSUPPORTED, "conv desc: pool and residual together");
    const int dt = d->dtype;
    const int cin_p = cpad(dt, d->in_c), cout_p = cpad(dt, d->cout);
    if (d->input_nchw) {
        dn_layer_desc ld{DN_CONV, d->cout, d->ksize, d->stride, d->pad, 0, d->activation, 0};
        if (!first_ok(d->in_c, ld, dt))
            return fail(DN_EUNSUPPORTED, "conv desc: input_nchw needs in_c <= 16, (in_c rounded up to 4, 8 or 16) * k <= 16, k <= %d, cout <= %d, stride <= 2",
                        FIRST_MAX_R, FIRST_MAX_COUT);
        if (d->residual) return fail(DN_EUNSUPPORTED, "conv desc: input_nchw with residual");
    }
    const int Ho = out_side_conv(d->in_h, d->ksize, d->stride, d->pad);
    const int Wo = out_side_conv(d->in_w, d->ksize, d->stride, d->pad);
    if (Ho <= 0 || Wo <= 0) return fail(DN_EINVAL, "conv desc: output is empty");
    if (d->pool && (Ho % 2 || Wo % 2)) return fail(DN_EUNSUPPORTED, "conv desc: fused pool needs an even output (%dx%d)", Ho, Wo);
    const int K = d->ksize * d->ksize * cin_p;
    const int k_pad = d->input_nchw ? first_kpad(dt, d->ksize) : (K + bk_el(dt) - 1) / bk_el(dt) * bk_el(dt);
    const long Ml = (long)d->batch * Ho * Wo;
    if (Ml > (1L << 30)) return fail(DN_EUNSUPPORTED, "conv desc: too many output pixels");
    const int M = (int)Ml;
    int t = d->tile, sp = d->splits;
    int ht, hs;
    heuristic_tile(M, cout_p, k_pad / bk_el(dt), &ht, &hs);
    if (t < 0) t = ht;
    if (sp <= 0) sp = (d->tile < 0) ? hs : 1;
    if (t >= tile_count() && !is_halo(t)) return fail(DN_EINVAL, "tile %d out of range", t);
    const int nkt = std::max(1, k_pad / bk_el(dt));
    if (sp > nkt) sp = nkt;
    if (d->input_nchw || is_halo(t)) sp = 1;
    if (is_halo(t)) {
        ConvArgs h{};
        h.R = h.S = d->ksize; h.stride = d->stride; h.pad = d->pad; h.cin_p = cin_p; h.cout_p = cout_p; h.k_pad = k_pad;
        h.H = d->in_h; h.W = d->in_w; h.Ho = Ho; h.Wo = Wo;
        if (t == HALO_TILE ? !halo_ok(dt, h) : !halo2_ok(dt, h))
            return fail(DN_EUNSUPPORTED, "conv desc: this shape cannot use the halo kernel %d", t);
    }
    if (a) {
        memset(a, 0, sizeof *a);
        a->batch = d->batch; a->H = d->in_h; a->W = d->in_w; a->cin_p = cin_p;
        a->Ho = Ho; a->Wo = Wo; a->cout_p = cout_p;
        a->R = a->S = d->ksize; a->stride = d->stride; a->pad = d->pad;
        a->k_pad = k_pad; a->M = M; a->pool = d->pool ? 1 : 0;
        a->act = d->activation; a->slope = d->leaky_slope;
        a->in_scale = dt == FP8 ? d->in_scale : 1.0f;
        a->res_scale = dt == FP8 ? d->res_scale : 1.0f;
        a->out_inv_scale = dt == FP8 ? 1.0f / d->out_scale : 1.0f;
        a->splits = sp;
        a->ktiles_per_split = (nkt + sp - 1) / sp;
        if (dt == FP8 && !(d->in_scale > 0 && d->out_scale > 0 && (!d->residual || d->res_scale > 0)))
            return fail(DN_EINVAL, "conv desc: FP8 scales must be positive");
    }
    if (tile) *tile = t;
    if (splits) *splits = sp;
    if (wbytes) *wbytes = (size_t)cout_p * k_pad * esize(dt);
    if (vbytes) *vbytes = (size_t)cout_p * sizeof(float);
    if (wsbytes) *wsbytes = sp > 1 ? (size_t)sp * M * cout_p * sizeof(float) : 0;
    return DN_OK;
}

extern "C" dn_status dn_conv_sizes(const dn_conv_desc *d, size_t *w_bytes, size_t *vec_bytes, size_t *ws_bytes)
{
    return conv_geometry(d, nullptr, nullptr, nullptr, w_bytes, vec_bytes, ws_bytes);
}

extern "C" dn_status dn_conv_pack(const dn_conv_desc *d, const double *w, const double *bias, const double *mean,
                                  const double *var, const double *gamma, const double *beta, double eps,
                                  void *w_packed, float *bias_out, float *wscale_out, void *stream)
{
    size_t wb = 0, vb = 0;
    STCHK(conv_geometry(d, nullptr, nullptr, nullptr, &wb, &vb, nullptr));
    if (!w || !bias || !w_packed || !bias_out || !wscale_out) return fail(DN_EINVAL, "conv pack: NULL pointer");
    const bool any_bn = mean || var || gamma || beta, all_bn = mean && var && gamma && beta;
    if (any_bn && !all_bn) return fail(DN_EINVAL, "conv pack: BN arrays must be all present or all NULL");
    if (all_bn && !(eps > 0)) return fail(DN_EINVAL, "conv pack: eps must be > 0");
    const int dt = d->dtype;
    const int cin_p = cpad(dt, d->in_c), cout_p = cpad(dt, d->cout);
    const int k_pad = (int)(wb / esize(dt) / cout_p);
    const size_t nw = (size_t)d->cout * d->in_c * d->ksize * d->ksize, nv = d->cout;
    hipStream_t s = (hipStream_t)stream;
    double *buf = nullptr;
    HIPCHK(hipMalloc(&buf, (nw + 6 * nv) * sizeof(double)));
    double *dw = buf, *db = buf + nw, *dm = db + nv, *dv = dm + nv, *dg = dv + nv, *dbe = dg + nv;
    dn_status rc = DN_OK;
    auto cp = [&](double *dst, const double *src, size_t n) {
        return hipMemcpyAsync(dst, src, n * sizeof(double), hipMemcpyHostToDevice, s) == hipSuccess;
    };
    bool ok = cp(dw, w, nw) && cp(db, bias, nv);
    if (ok && all_bn) ok = cp(dm, mean, nv) && cp(dv, var, nv) && cp(dg, gamma, nv) && cp(dbe, beta, nv);
    if (!ok) rc = fail(DN_EHIP, "conv pack upload failed");
    if (rc == DN_OK && launch_fold_pack(dt, d->input_nchw ? 1 : 0, dw, db, dm, dv, dg, dbe, eps, all_bn ? 1 : 0, d->cout, d->in_c, d->ksize,
                                        d->ksize, cin_p, k_pad, cout_p, w_packed, bias_out, wscale_out, s) != hipSuccess)
        rc = fail(DN_EHIP, "fold/pack launch failed");
    if (hipStreamSynchronize(s) != hipSuccess && rc == DN_OK) rc = fail(DN_EHIP, "fold/pack failed");
    (void)hipFree(buf);
    return rc;
}

extern "C" dn_status dn_conv2d(const dn_conv_desc *d, const void *x, const void *w_packed, const float *bias,
                               const float *wscale, const void *res, void *y, void *workspace, size_t ws_bytes,
                               void *stream)
{
    ConvArgs a;
    int tile = 0, splits = 1;
    size_t need = 0;
    STCHK(conv_geometry(d, &a, &tile, &splits, nullptr, nullptr, &need));
    if (!x || !w_packed || !bias || !y) return fail(DN_EINVAL, "conv2d: NULL pointer");
    if (d->dtype == DN_FP8_E4M3 && !wscale) return fail(DN_EINVAL, "conv2d: FP8 needs wscale");
    if (d->residual && !res) return fail(DN_EINVAL, "conv2d: residual requested without res");
    if (need > 0 && (!workspace || ws_bytes < need))
        return fail(DN_EINVAL, "conv2d: split-K %d needs %zu workspace bytes (%zu given)", splits, need, ws_bytes);
    if (d->input_nchw) {
        FirstArgs f{};
        f.x = (const float *)x; f.w = w_packed; f.bias = bias; f.wscale = wscale; f.y = y;
        f.batch = a.batch; f.C = d->in_c; f.H = a.H; f.W = a.W; f.Ho = a.Ho; f.Wo = a.Wo;
        f.cout_p = a.cout_p; f.k_pad = a.k_pad; f.R = f.S = d->ksize; f.stride = d->stride; f.pad = d->pad;
        f.pool = a.pool; f.act = a.act; f.slope = a.slope;
        f.in_inv_scale = d->dtype == DN_FP8_E4M3 ? 1.0f / d->in_scale : 1.0f;
        f.in_scale = a.in_scale;
        f.out_inv_scale = a.out_inv_scale;
        HIPCHK(launch_conv_first(d->dtype, f, (hipStream_t)stream));
        return DN_OK;
    }
    a.x = x; a.w = w_packed; a.bias = bias; a.wscale = wscale;
    a.res = d->residual ? res : nullptr;
    a.y = y;
    a.partial = (float *)workspace;
    HIPCHK(launch_conv(d->dtype, tile, a, (hipStream_t)stream));
    if (splits > 1) HIPCHK(launch_splitk_reduce(d->dtype, a, (hipStream_t)stream));
    return DN_OK;
}

extern "C" dn_status dn_maxpool(const dn_pool_desc *d, const void *x, void *y, void *stream)
{
    if (!d || !x || !y) return fail(DN_EINVAL, "maxpool: NULL argument");
    STCHK(check_dtype(d->dtype));
    if (d->batch <= 0 || d->h <= 0 || d->w <= 0 || d->c <= 0 || d->size <= 0 || d->stride <= 0)
        return fail(DN_EINVAL, "maxpool: non-positive size");
    const int cp = cpad(d->dtype, d->c);
    HIPCHK(launch_maxpool(d->dtype, x, y, d->batch, d->h, d->w, cp, d->size, d->stride, out_side_pool(d->h, d->stride),
                          out_side_pool(d->w, d->stride), (hipStream_t)stream));
    return DN_OK;
}

extern "C" dn_status dn_shortcut(int dtype, size_t count, const void *a, float sa, const void *b, float sb, void *y,
                                 float sy, void *stream)
{
    STCHK(check_dtype(dtype));
    if (!a || !b || !y) return fail(DN_EINVAL, "shortcut: NULL argument");
    if (count % seg_el(dtype)) return fail(DN_EINVAL, "shortcut: count must be a multiple of %d", seg_el(dtype));
    if (dtype == DN_FP8_E4M3 && !(sa > 0 && sb > 0 && sy > 0)) return fail(DN_EINVAL, "shortcut: FP8 scales must be positive");
    const bool f8 = dtype == DN_FP8_E4M3;
    HIPCHK(launch_add(dtype, a, f8 ? sa : 1.f, b, f8 ? sb : 1.f, y, f8 ? 1.0f / sy : 1.f, count, (hipStream_t)stream));
    return DN_OK;
}

extern "C" dn_status dn_ingest(int dtype, int batch, int c, int h, int w, const float *x, float scale, void *y,
                               void *stream)
{
    STCHK(check_dtype(dtype));
    if (!x || !y || batch <= 0 || c <= 0 || h <= 0 || w <= 0) return fail(DN_EINVAL, "ingest: bad argument");
    if (dtype == DN_FP8_E4M3 && !(scale > 0)) return fail(DN_EINVAL, "ingest: FP8 scale must be positive");
    HIPCHK(launch_ingest(dtype, x, batch, c, h, w, cpad(dtype, c), dtype == DN_FP8_E4M3 ? 1.0f / scale : 1.0f, y,
                         (hipStream_t)stream));
    return DN_OK;
}

extern "C" dn_status dn_egress(int dtype, int batch, int c, int h, int w, const void *x, float scale, float *y,
                               void *stream)
{
    STCHK(check_dtype(dtype));
    if (!x || !y || batch <= 0 || c <= 0 || h <= 0 || w <= 0) return fail(DN_EINVAL, "egress: bad argument");
    HIPCHK(launch_egress(dtype, x, batch, c, h, w, cpad(dtype, c), dtype == DN_FP8_E4M3 ? scale : 1.0f, y,
                         (hipStream_t)stream));
    return DN_OK;
}

// ---------------------------------------------------------------- backward to the input

// The backward-data conv of forward conv `f`, as a forward conv over the
// (spread, when f is strided) output gradient: in_c = f.cout, cout = f.in_c,
// stride 1, pad k-1-pad, linear, bias 0.  hz x wz is its input size.
static dn_status bwd_desc(const dn_conv_desc *f, int accumulate, dn_conv_desc *b, int *ho, int *wo, int *hz, int *wz,
                          int tile = -1, int splits = 0)
{
    if (!f) return fail(DN_EINVAL, "conv desc is NULL");
    if (f->dtype != DN_F32 && f->dtype != DN_BF16) return fail(DN_EUNSUPPORTED, "backward: F32 and BF16 only");
    if (f->pool || f->residual || f->input_nchw)
        return fail(DN_EUNSUPPORTED, "backward: the forward conv must be unfused (no pool, residual or NCHW input)");
    if (f->batch <= 0 || f->in_h <= 0 || f->in_w <= 0 || f->in_c <= 0 || f->cout <= 0 || f->ksize <= 0 ||
        f->stride <= 0 || f->pad < 0)
        return fail(DN_EINVAL, "conv desc: non-positive size");
    if (f->pad > f->ksize - 1) return fail(DN_EUNSUPPORTED, "backward: pad %d > ksize - 1", f->pad);
    *ho = out_side_conv(f->in_h, f->ksize, f->stride, f->pad);
    *wo = out_side_conv(f->in_w, f->ksize, f->stride, f->pad);
    if (*ho <= 0 || *wo <= 0) return fail(DN_EINVAL, "conv desc: output is empty");
    *hz = f->in_h + 2 * f->pad - f->ksize + 1;
    *wz = f->in_w + 2 * f->pad - f->ksize + 1;
    memset(b, 0, sizeof *b);
    b->batch = f->batch; b->in_h = *hz; b->in_w = *wz; b->in_c = f->cout;
    b->cout = f->in_c; b->ksize = f->ksize; b->stride = 1; b->pad = f->ksize - 1 - f->pad;
    b->activation = DN_ACT_LINEAR; b->dtype = f->dtype; b->residual = accumulate ? 1 : 0;
    b->in_scale = b->res_scale = b->out_scale = 1.0f;
    b->tile = -1; b->splits = 0;
    ConvArgs a;
    STCHK(conv_geometry(b, &a, nullptr, nullptr, nullptr, nullptr, nullptr));
    if (tile >= 0) {  // an explicit (tuned) choice
        if (tile == HALO_TILE && !halo_ok(f->dtype, a)) return fail(DN_EUNSUPPORTED, "backward: halo tile does not fit");
        if (tile == HALO2_TILE && !halo2_ok(f->dtype, a)) return fail(DN_EUNSUPPORTED, "backward: halo tile does not fit");
        b->tile = tile;
        b->splits = is_halo(tile) ? 1 : std::max(1, splits);
    } else if (halo2_ok(f->dtype, a)) {
        b->tile = HALO2_TILE;
    } else if (halo_ok(f->dtype, a)) {
        b->tile = HALO_TILE;
    }
    return DN_OK;
}

// Tune-cache key of the backward-data conv of forward conv f.
static std::string bwd_sig(const dn_conv_desc *f, int accumulate)
{
    char k[256];
    snprintf(k, sizeof k, "bwd_dt%d_b%d_H%d_W%d_ci%d_co%d_R%d_s%d_p%d_a%d", f->dtype, f->batch, f->in_h, f->in_w, f->in_c,
             f->cout, f->ksize, f->stride, f->pad, accumulate);
    return k;
}

// Scratch of a backward-data conv: split-K partials, then the spread gradient.
static dn_status bwd_scratch(const dn_conv_desc *f, const dn_conv_desc *b, int hz, int wz, size_t *ws, size_t *z)
{
    size_t need = 0;
    STCHK(conv_geometry(b, nullptr, nullptr, nullptr, nullptr, nullptr, &need));
    *ws = align256(need);
    *z = f->stride > 1 ? align256((size_t)f->batch * hz * wz * cpad(f->dtype, f->cout) * esize(f->dtype)) : 0;
    return DN_OK;
}

extern "C" dn_status dn_conv_backward_sizes(const dn_conv_desc *d, size_t *w_bytes, size_t *vec_bytes, size_t *ws_bytes)
{
    dn_conv_desc b;
    int ho, wo, hz, wz;
    STCHK(bwd_desc(d, 0, &b, &ho, &wo, &hz, &wz));
    size_t ws = 0, z = 0;
    STCHK(bwd_scratch(d, &b, hz, wz, &ws, &z));
    if (w_bytes || vec_bytes) STCHK(conv_geometry(&b, nullptr, nullptr, nullptr, w_bytes, vec_bytes, nullptr));
    if (ws_bytes) *ws_bytes = ws + z;
    return DN_OK;
}

extern "C" dn_status dn_conv_pack_backward(const dn_conv_desc *d, const double *w, const double *mean,
                                           const double *var, const double *gamma, double eps, void *w_packed,
                                           float *zero_bias, float *unit_scale, void *stream)
{
    dn_conv_desc b;
    int ho, wo, hz, wz;
    STCHK(bwd_desc(d, 0, &b, &ho, &wo, &hz, &wz));
    size_t wb = 0;
    STCHK(conv_geometry(&b, nullptr, nullptr, nullptr, &wb, nullptr, nullptr));
    if (!w || !w_packed || !zero_bias || !unit_scale) return fail(DN_EINVAL, "backward pack: NULL pointer");
    const bool any_bn = mean || var || gamma, all_bn = mean && var && gamma;
    if (any_bn && !all_bn) return fail(DN_EINVAL, "backward pack: BN arrays must be all present or all NULL");
    if (all_bn && !(eps > 0)) return fail(DN_EINVAL, "backward pack: eps must be > 0");
    const int dt = d->dtype;
    const int cin_p = cpad(dt, d->cout), cout_p = cpad(dt, d->in_c);
    const int k_pad = (int)(wb / esize(dt) / cout_p);
    const size_t nw = (size_t)d->cout * d->in_c * d->ksize * d->ksize, nv = d->cout;
    hipStream_t s = (hipStream_t)stream;
    double *buf = nullptr;
    HIPCHK(hipMalloc(&buf, (nw + 3 * nv) * sizeof(double)));
    double *dw = buf, *dm = buf + nw, *dv = dm + nv, *dg = dv + nv;
    dn_status rc = DN_OK;
    auto cp = [&](double *dst, const double *src, size_t n) {
        return hipMemcpyAsync(dst, src, n * sizeof(double), hipMemcpyHostToDevice, s) == hipSuccess;
    };
    bool ok = cp(dw, w, nw);
    if (ok && all_bn) ok = cp(dm, mean, nv) && cp(dv, var, nv) && cp(dg, gamma, nv);
    if (!ok) rc = fail(DN_EHIP, "backward pack upload failed");
    if (rc == DN_OK && launch_fold_pack(dt, 2, dw, nullptr, dm, dv, dg, nullptr, eps, all_bn ? 1 : 0, d->in_c, d->cout,
                                        d->ksize, d->ksize, cin_p, k_pad, cout_p, w_packed, zero_bias, unit_scale,
                                        s) != hipSuccess)
        rc = fail(DN_EHIP, "backward fold/pack launch failed");
    if (hipStreamSynchronize(s) != hipSuccess && rc == DN_OK) rc = fail(DN_EHIP, "backward fold/pack failed");
    (void)hipFree(buf);
    return rc;
}

// Enqueue dx (+)= backward-data conv of dy, scratch = [split-K | spread gradient].
static dn_status enqueue_conv_backward(const dn_conv_desc *f, const void *dy, const void *w_packed,
                                       const float *zero_bias, const float *unit_scale, int accumulate, void *dx,
                                       void *scratch, size_t scratch_bytes, hipStream_t s, int tile = -1,
                                       int splits = 0)
{
    dn_conv_desc b;
    int ho, wo, hz, wz;
    STCHK(bwd_desc(f, accumulate, &b, &ho, &wo, &hz, &wz, tile, splits));
    size_t ws = 0, z = 0;
    STCHK(bwd_scratch(f, &b, hz, wz, &ws, &z));
    if (ws + z > 0 && (!scratch || scratch_bytes < ws + z))
        return fail(DN_EINVAL, "conv backward: needs %zu workspace bytes (%zu given)", ws + z, scratch_bytes);
    const void *src = dy;
    if (f->stride > 1) {
        void *zb = (char *)scratch + ws;
        HIPCHK(launch_dilate(f->dtype, dy, zb, f->batch, ho, wo, cpad(f->dtype, f->cout), hz, wz, f->stride, s));
        src = zb;
    }
    ConvArgs a;
    int use_tile = 0, use_splits = 1;
    STCHK(conv_geometry(&b, &a, &use_tile, &use_splits, nullptr, nullptr, nullptr));
    a.x = src; a.w = w_packed; a.bias = zero_bias; a.wscale = unit_scale;
    a.res = accumulate ? dx : nullptr;
    a.y = dx;
    a.partial = (float *)scratch;
    HIPCHK(launch_conv(f->dtype, use_tile, a, s));
    if (use_splits > 1) HIPCHK(launch_splitk_reduce(f->dtype, a, s));
    return DN_OK;
}

extern "C" dn_status dn_conv_backward_data(const dn_conv_desc *d, const void *dy, const void *w_packed,
                                           const float *zero_bias, const float *unit_scale, int accumulate, void *dx,
                                           void *workspace, size_t ws_bytes, void *stream)
{
    if (!dy || !w_packed || !zero_bias || !unit_scale || !dx) return fail(DN_EINVAL, "conv backward: NULL pointer");
    return enqueue_conv_backward(d, dy, w_packed, zero_bias, unit_scale, accumulate, dx, workspace, ws_bytes,
                                 (hipStream_t)stream);
}

extern "C" dn_status dn_maxpool_backward(const dn_pool_desc *d, const void *x, const void *dy, int accumulate,
                                         void *dx, void *stream)
{
    if (!d || !x || !dy || !dx) return fail(DN_EINVAL, "maxpool backward: NULL argument");
    if (d->dtype != DN_F32 && d->dtype != DN_BF16) return fail(DN_EUNSUPPORTED, "backward: F32 and BF16 only");
    if (d->batch <= 0 || d->h <= 0 || d->w <= 0 || d->c <= 0 || d->size <= 0 || d->stride <= 0)
        return fail(DN_EINVAL, "maxpool backward: non-positive size");
    HIPCHK(launch_maxpool_bwd(d->dtype, x, dy, dx, d->batch, d->h, d->w, cpad(d->dtype, d->c), d->size, d->stride,
                              out_side_pool(d->h, d->stride), out_side_pool(d->w, d->stride), accumulate ? 1 : 0,
                              -1.0f, (hipStream_t)stream));
    return DN_OK;
}

extern "C" dn_status dn_leaky_backward(int dtype, size_t count, const void *a, const void *dy, float slope, void *dx,
                                       void *stream)
{
    if (dtype != DN_F32 && dtype != DN_BF16) return fail(DN_EUNSUPPORTED, "backward: F32 and BF16 only");
    if (!a || !dy || !dx) return fail(DN_EINVAL, "leaky backward: NULL argument");
    if (count % seg_el(dtype)) return fail(DN_EINVAL, "leaky backward: count must be a multiple of %d", seg_el(dtype));
    if (!(slope >= 0.0f && slope <= 1.0f)) return fail(DN_EINVAL, "leaky backward: slope must lie in [0, 1]");
    HIPCHK(launch_leaky_bwd(dtype, a, dy, dx, slope, count, (hipStream_t)stream));
    return DN_OK;
}

// The input-gradient pass of a net: the unfused forward up to layer `target`
// keeping every layer output, then the layers' backward in reverse order.
struct BwdPlan {
    Plan p;                          // unfused forward plan; vals[].off = forward outputs
    int nops = 0, seed = 0;          // ops 0..nops-1 run; seed = value whose gradient starts the pass
    std::vector<size_t> goff, gbytes;  // gradient of each value 0..seed
    std::vector<dn_conv_desc> fwd;   // per op: the forward conv as a standalone desc (convs only)
    std::vector<char> pool_leaky;    // per op: this pool applies the leaky gradient of its input's producer
    std::vector<char> acc;           // per op: its input's gradient already holds a contribution (add, not write)
    std::vector<std::pair<int, int>> btile;  // per conv op: backward (tile, splits); (-1, 0) = heuristic
    size_t bws_off = 0, bws_bytes = 0;  // backward conv scratch
    size_t gin_off = 0, mabs_off = 0;   // NCHW FP32 input gradient, per-image mean |g|
    size_t total = 0;
};

static dn_status make_bwd_plan(const dn_net *net, int target, int batch, int h, int w, BwdPlan *out)
{
    const int dt = net->o.dtype;
    if (dt != DN_F32 && dt != DN_BF16) return fail(DN_EUNSUPPORTED, "input gradient: F32 and BF16 nets only");
    if (target < 0 || target >= (int)net->L.size()) return fail(DN_EINVAL, "layer %d out of range", target);
    BwdPlan b;
    STCHK(make_plan(net, dt, DN_MODE_PER_LAYER, batch, h, w, &b.p, target));
    Plan &p = b.p;
    p.cnt_bytes = 0;  // regions laid out below; split convs finish with a separate launch
    p.any_fused = false;
    b.nops = 0;  // ops computing layers 0..target (a conv with its fused pool is one op)
    while (b.nops < (int)p.ops.size() && p.ops[b.nops].layer <= target) ++b.nops;
    b.seed = target + 1;
    if (b.nops == 0 || p.ops[b.nops - 1].out != b.seed) return fail(DN_EINVAL, "layer %d: no op ends there", target);
    // every produced value keeps its own buffer (the full-size output of a conv
    // with a fused pool is never stored: its windows' argmax codes are)
    std::vector<char> produced(b.seed + 1, 0);
    produced[0] = 1;
    for (int k = 0; k < b.nops; ++k) produced[p.ops[k].out] = 1;
    size_t off = 0;
    for (int v = 0; v <= b.seed; ++v) {
        p.vals[v].off = off;
        if (produced[v]) off += p.vals[v].bytes;
    }
    for (int k = 0; k < b.nops; ++k) {
        Op &op = p.ops[k];
        if (op.kind != OP_CONV || !op.pool) continue;
        op.argmax = true;
        op.argmax_off = off;
        off += align256((size_t)batch * op.Ho * op.Wo * op.cout_p);
    }
    p.ws_off = align256(off);
    off = p.ws_off + align256(p.ws_bytes);
    b.goff.resize(b.seed + 1);
    b.gbytes.resize(b.seed + 1);
    for (int v = 0; v <= b.seed; ++v) {
        const Value &vv = p.vals[v];
        b.gbytes[v] = align256((size_t)batch * vv.h * vv.w * vv.cp * esize(dt));
        b.goff[v] = off;
        off += b.gbytes[v];
    }
    b.fwd.resize(b.nops);
    // a pool whose input is a leaky conv's output read by nothing else applies
    // that conv's leaky gradient itself (the conv op then skips its pass)
    std::vector<int> readers(b.seed + 1, 0);
    for (int k = 0; k < b.nops; ++k) {
        readers[p.ops[k].in]++;
        if (p.ops[k].in2 >= 0) readers[p.ops[k].in2]++;
    }
    b.pool_leaky.assign(b.nops, 0);
    for (int k = 1; k < b.nops; ++k) {
        const Op &op = p.ops[k], &prev = p.ops[k - 1];
        if (op.kind == OP_POOL && prev.kind == OP_CONV && prev.out == op.in && readers[op.in] == 1 &&
            net->L[prev.conv].activation == DN_ACT_LEAKY)
            b.pool_leaky[k] = 1;
    }
    // which gradient writes add to an earlier contribution (the reverse walk's order)
    b.acc.assign(b.nops, 0);
    {
        std::vector<char> have(b.seed + 1, 0);
        have[b.seed] = 1;
        for (int k = b.nops - 1; k >= 0; --k) {
            const Op &op = p.ops[k];
            b.acc[k] = have[op.in];
            have[op.in] = 1;
            if (op.kind == OP_ADD) have[op.in2] = 1;
        }
    }
    b.btile.assign(b.nops, {-1, 0});
    size_t bws = 0;
    for (int k = 0; k < b.nops; ++k) {
        const Op &op = p.ops[k];
        if (op.kind != OP_CONV) continue;
        const dn_layer_desc &d = net->L[op.conv];
        dn_conv_desc &f = b.fwd[k];
        memset(&f, 0, sizeof f);
        f.batch = batch; f.in_h = p.vals[op.in].h; f.in_w = p.vals[op.in].w; f.in_c = p.vals[op.in].c;
        f.cout = d.cout; f.ksize = d.ksize; f.stride = d.stride; f.pad = d.pad;
        f.activation = d.activation; f.leaky_slope = net->o.leaky_slope; f.dtype = dt;
        f.in_scale = f.res_scale = f.out_scale = 1.0f; f.tile = -1;
        auto it = net->tuned.find(bwd_sig(&f, b.acc[k]));
        if (it != net->tuned.end()) b.btile[k] = it->second;
        dn_conv_desc bd;
        int ho, wo, hz, wz;
        STCHK(bwd_desc(&f, b.acc[k], &bd, &ho, &wo, &hz, &wz, b.btile[k].first, b.btile[k].second));
        size_t ws = 0, z = 0;
        STCHK(bwd_scratch(&f, &bd, hz, wz, &ws, &z));
        bws = std::max(bws, ws + z);
    }
    b.bws_off = off;
    b.bws_bytes = bws;
    off += bws;
    b.gin_off = off;
    off += align256((size_t)batch * net->o.in_c * h * w * sizeof(float));
    b.mabs_off = off;
    off += align256(ascend_scratch_bytes(batch));
    b.total = off;
    *out = std::move(b);
    return DN_OK;
}

static dn_status enqueue_input_gradient(const dn_net *net, const BwdPlan &b, char *base, const float *x, hipStream_t s)
{
    const Plan &p = b.p;
    const int dt = p.dtype;
    const Value &v0 = p.vals[0];
    if (!p.ops[0].first) HIPCHK(launch_ingest(dt, x, p.batch, v0.c, v0.h, v0.w, v0.cp, 1.0f, base + v0.off, s));
    for (int k = 0; k < b.nops; ++k) STCHK(enqueue_op(net, p, p.ops[k], base, s, false, -1, 0, x));
    // objective: half the sum of squares of the seed layer's output -> its gradient is the output itself
    HIPCHK(hipMemcpyAsync(base + b.goff[b.seed], base + p.vals[b.seed].off, b.gbytes[b.seed], hipMemcpyDeviceToDevice, s));
    std::vector<char> have(b.seed + 1, 0);  // shortcut inputs: copy first, add after
    have[b.seed] = 1;
    for (int k = b.nops - 1; k >= 0; --k) {
        const Op &op = p.ops[k];
        char *gout = base + b.goff[op.out];
        const Value &vo = p.vals[op.out];
        const size_t count = (size_t)p.batch * vo.h * vo.w * vo.cp;
        if (op.kind == OP_CONV && op.pool) {
            // fused 2x2/2 pool: each window's gradient goes to its argmax element,
            // times the leaky gradient there (the pooled output has its sign)
            const dn_layer_desc &d = net->L[op.conv];
            const ConvWeights &cw = net->cw[op.conv];
            char *gfull = base + b.goff[op.conv + 1];
            HIPCHK(launch_unpool_bwd(dt, (const unsigned char *)(base + op.argmax_off), base + vo.off, gout, gfull,
                                     p.batch, op.Ho, op.Wo, op.cout_p,
                                     d.activation == DN_ACT_LEAKY ? net->o.leaky_slope : -1.0f, s));
            STCHK(enqueue_conv_backward(&b.fwd[k], gfull, cw.wb, cw.bzero, cw.bscale, b.acc[k], base + b.goff[op.in],
                                        base + b.bws_off, b.bws_bytes, s, b.btile[k].first, b.btile[k].second));
            have[op.in] = 1;
        } else if (op.kind == OP_CONV) {
            const dn_layer_desc &d = net->L[op.conv];
            const ConvWeights &cw = net->cw[op.conv];
            const bool masked = k + 1 < b.nops && b.pool_leaky[k + 1];  // the pool after it applied the leaky gradient
            if (d.activation == DN_ACT_LEAKY && !masked)
                HIPCHK(launch_leaky_bwd(dt, base + vo.off, gout, gout, net->o.leaky_slope, count, s));
            STCHK(enqueue_conv_backward(&b.fwd[k], gout, cw.wb, cw.bzero, cw.bscale, b.acc[k], base + b.goff[op.in],
                                        base + b.bws_off, b.bws_bytes, s, b.btile[k].first, b.btile[k].second));
            have[op.in] = 1;
        } else if (op.kind == OP_POOL) {
            const dn_layer_desc &d = net->L[op.layer];
            const Value &vi = p.vals[op.in];
            HIPCHK(launch_maxpool_bwd(dt, base + vi.off, gout, base + b.goff[op.in], p.batch, vi.h, vi.w, vi.cp, d.ksize,
                                      d.stride, vo.h, vo.w, b.acc[k], b.pool_leaky[k] ? net->o.leaky_slope : -1.0f, s));
            have[op.in] = 1;
        } else {
            for (int src : {op.in, op.in2}) {
                char *g = base + b.goff[src];
                if (have[src]) HIPCHK(launch_add(dt, g, 1.f, gout, 1.f, g, 1.f, count, s));
                else HIPCHK(hipMemcpyAsync(g, gout, count * esize(dt), hipMemcpyDeviceToDevice, s));
                have[src] = 1;
            }
        }
    }
    HIPCHK(launch_egress(dt, base + b.goff[0], p.batch, v0.c, v0.h, v0.w, v0.cp, 1.0f, (float *)(base + b.gin_off), s));
    return DN_OK;
}

static dn_status bwd_prepare(const dn_net *net, int layer, int batch, int h, int w, BwdPlan *b)
{
    if (net->o.dtype != DN_F32 && net->o.dtype != DN_BF16)
        return fail(DN_EUNSUPPORTED, "input gradient: F32 and BF16 nets only");
    STCHK(check_ready(net, false));
    STCHK(check_dims(net, batch, h, w));
    for (size_t i = 0; i < net->L.size(); ++i)
        if (net->L[i].kind == DN_CONV && !net->cw[i].wb) return fail(DN_ESTATE, "conv layer %zu has no backward weights", i);
    return make_bwd_plan(net, layer, batch, h, w, b);
}

extern "C" dn_status dn_input_gradient_arena_bytes(const dn_net *net, int layer, int batch, int h, int w, size_t *bytes)
{
    if (!net || !bytes) return fail(DN_EINVAL, "NULL argument");
    BwdPlan b;
    STCHK(bwd_prepare(net, layer, batch, h, w, &b));
    *bytes = b.total;
    return DN_OK;
}

static dn_status bwd_arena_check(const BwdPlan &b, const void *arena, size_t arena_bytes)
{
    if (!arena) return fail(DN_ESTATE, "input gradient: no arena (bind one or pass one)");
    if ((uintptr_t)arena & 255) return fail(DN_EINVAL, "input gradient: arena must be 256-byte aligned");
    if (arena_bytes < b.total)
        return fail(DN_ENOMEM, "input gradient: arena has %zu bytes, the pass needs %zu (dn_input_gradient_arena_bytes)",
                    arena_bytes, b.total);
    return DN_OK;
}

static dn_status input_gradient_on(dn_net *net, void *arena, size_t arena_bytes, int layer, const float *x, int batch,
                                   int h, int w, float *grad, hipStream_t s)
{
    if (!net) return fail(DN_EINVAL, "net is NULL");
    if (!grad) return fail(DN_EINVAL, "grad is NULL");
    if (!x) return fail(DN_EINVAL, "x is NULL");
    HIPCHK(hipSetDevice(net->o.device));
    BwdPlan b;
    STCHK(bwd_prepare(net, layer, batch, h, w, &b));
    STCHK(bwd_arena_check(b, arena, arena_bytes));
    char *base = (char *)arena;
    STCHK(enqueue_input_gradient(net, b, base, x, s));
    HIPCHK(hipMemcpyAsync(grad, base + b.gin_off, (size_t)batch * net->o.in_c * h * w * sizeof(float),
                          hipMemcpyDeviceToDevice, s));
    return DN_OK;
}

extern "C" dn_status dn_input_gradient(dn_net *net, int layer, const float *x, int batch, int h, int w, float *grad,
                                       void *stream)
{
    if (!net) return fail(DN_EINVAL, "net is NULL");
    return input_gradient_on(net, net->arena, net->arena_bytes, layer, x, batch, h, w, grad, (hipStream_t)stream);
}

extern "C" dn_status dn_input_gradient_arena(dn_net *net, void *arena, size_t arena_bytes, int layer, const float *x,
                                             int batch, int h, int w, float *grad, void *stream)
{
    return input_gradient_on(net, arena, arena_bytes, layer, x, batch, h, w, grad, (hipStream_t)stream);
}

extern "C" dn_status dn_input_gradient_readback(const dn_net *net, void *arena, size_t arena_bytes, int layer,
                                                int batch, int h, int w, int of_layer, int what, void *out,
                                                size_t out_bytes, int *available, void *stream)
{
    if (!net) return fail(DN_EINVAL, "net is NULL");
    if (what < 0 || what > 2) return fail(DN_EINVAL, "readback: unknown kind %d", what);
    HIPCHK(hipSetDevice(net->o.device));
    BwdPlan b;
    STCHK(bwd_prepare(net, layer, batch, h, w, &b));
    STCHK(bwd_arena_check(b, arena, arena_bytes));
    if (of_layer < 0 || of_layer > layer) return fail(DN_EINVAL, "readback: layer %d outside 0..%d", of_layer, layer);
    const Plan &p = b.p;
    const int v = of_layer + 1;
    const Value &vv = p.vals[v];
    bool have = false;
    size_t need = 0;
    const Op *fused = nullptr;  // the conv op whose fused pool is layer of_layer
    for (int k = 0; k < b.nops; ++k) {
        if (p.ops[k].out == v) have = true;
        if (p.ops[k].kind == OP_CONV && p.ops[k].pool && p.ops[k].layer == of_layer) fused = &p.ops[k];
    }
    if (what == 1) {
        have = fused != nullptr;
        need = fused ? (size_t)batch * fused->Ho * fused->Wo * fused->cout_p : 0;
    } else if (what == 2) {
        have = true;  // every value 0..seed has a gradient buffer
        need = (size_t)batch * vv.c * vv.h * vv.w * sizeof(float);
    } else {
        need = (size_t)batch * vv.c * vv.h * vv.w * sizeof(float);
    }
    if (available) *available = have ? 1 : 0;
    if (!out) return DN_OK;
    if (!have) return fail(DN_EINVAL, "readback: the pass stores no %s for layer %d",
                           what == 1 ? "argmax codes" : "output", of_layer);
    if (out_bytes < need) return fail(DN_EINVAL, "readback: output buffer has %zu bytes, needs %zu", out_bytes, need);
    hipStream_t s = (hipStream_t)stream;
    char *base = (char *)arena;
    if (what == 1)
        HIPCHK(hipMemcpyAsync(out, base + fused->argmax_off, need, hipMemcpyDeviceToDevice, s));
    else
        HIPCHK(launch_egress(p.dtype, base + (what == 0 ? vv.off : b.goff[v]), batch, vv.c, vv.h, vv.w, vv.cp, 1.0f,
                             (float *)out, s));
    return DN_OK;
}

static dn_status nightmare_on(dn_net *net, void *arena, size_t arena_bytes, int layer, float *x, int batch, int h,
                              int w, float rate, int iters, hipStream_t s)
{
    if (!net) return fail(DN_EINVAL, "net is NULL");
    if (iters < 0) return fail(DN_EINVAL, "iters must be >= 0");
    if (!std::isfinite(rate)) return fail(DN_EINVAL, "rate must be finite");
    if (!x) return fail(DN_EINVAL, "x is NULL");
    HIPCHK(hipSetDevice(net->o.device));
    BwdPlan b;
    STCHK(bwd_prepare(net, layer, batch, h, w, &b));
    STCHK(bwd_arena_check(b, arena, arena_bytes));
    char *base = (char *)arena;
    for (int it = 0; it < iters; ++it) {
        STCHK(enqueue_input_gradient(net, b, base, x, s));
        HIPCHK(launch_ascend(x, (const float *)(base + b.gin_off), (double *)(base + b.mabs_off), batch,
                             (size_t)net->o.in_c * h * w, rate, s));
    }
    return DN_OK;
}

extern "C" dn_status dn_nightmare(dn_net *net, int layer, float *x, int batch, int h, int w, float rate, int iters,
                                  void *stream)
{
    if (!net) return fail(DN_EINVAL, "net is NULL");
    return nightmare_on(net, net->arena, net->arena_bytes, layer, x, batch, h, w, rate, iters, (hipStream_t)stream);
}

extern "C" dn_status dn_nightmare_arena(dn_net *net, void *arena, size_t arena_bytes, int layer, float *x, int batch,
                                        int h, int w, float rate, int iters, void *stream)
{
    return nightmare_on(net, arena, arena_bytes, layer, x, batch, h, w, rate, iters, (hipStream_t)stream);
}

// Time `launch` (which enqueues one candidate) 1 + 5 times; the mean of the last 5 in ms, or a status.
template <typename F> static dn_status time_candidate(F launch, hipEvent_t e0, hipEvent_t e1, hipStream_t s, float *ms)
{
    for (int rep = 0; rep < 2; ++rep) {  // rep 0 = warm-up
        const int iters = rep ? 5 : 1;
        HIPCHK(hipEventRecord(e0, s));
        for (int it = 0; it < iters; ++it) STCHK(launch());
        HIPCHK(hipEventRecord(e1, s));
        HIPCHK(hipEventSynchronize(e1));
        if (rep) {
            HIPCHK(hipEventElapsedTime(ms, e0, e1));
            *ms /= iters;
        }
    }
    return DN_OK;
}

constexpr size_t BWD_TUNE_SCRATCH = (size_t)512 << 20;

static dn_status autotune_backward(dn_net *net, int layer, int batch, int h, int w, hipStream_t s, hipEvent_t e0,
                                   hipEvent_t e1, char *base)
{
    BwdPlan b;
    STCHK(bwd_prepare(net, layer, batch, h, w, &b));
    char *scratch = base + b.total;  // candidate split-K partials (and spread gradients) go here
    Plan p = b.p;
    p.ws_off = b.total;
    const int dt = p.dtype;
    // the unfused forward convs (first-layer kernel excepted): same candidates as dn_autotune
    for (int k = 0; k < b.nops; ++k) {
        const Op &op = p.ops[k];
        if (op.kind != OP_CONV || op.first) continue;
        const dn_layer_desc &d = net->L[op.conv];
        const bool inv = net->o.batch_invariant != 0;
        const std::string sig = conv_sig(dt, op, batch, d.ksize, d.stride, inv);
        if (net->tuned.count(sig)) continue;
        const int M = batch * (op.pool ? op.Ho * 2 : op.Ho) * (op.pool ? op.Wo * 2 : op.Wo);
        const int nkt = net->cw[op.conv].k_pad / bk_el(dt);
        std::vector<int> cands;
        if (op_halo_ok(net, dt, op, net->cw[op.conv].k_pad)) cands.push_back(HALO_TILE);
        if (op_halo2_ok(net, dt, op, net->cw[op.conv].k_pad)) cands.push_back(HALO2_TILE);
        for (int t = 0; t < tile_count(); ++t)
            if (tile_fits(t, op.cout_p)) cands.push_back(t);
        std::vector<std::tuple<float, int, int>> timed;
        for (int t : cands) {
            const TileCfg tc = is_halo(t) ? TileCfg{1 << 30, 1 << 30, 1, 1} : tile_cfg(t);
            const long tiles = (long)((M + tc.bm - 1) / tc.bm) * ((op.cout_p + tc.bn - 1) / tc.bn);
            const int sp_lo = inv ? invariant_splits(nkt) : 1, sp_hi = inv ? sp_lo : 16;
            for (int sp = sp_lo; sp <= sp_hi; sp *= 2) {
                if (inv && !invariant_tile_ok(dt, t, sp)) break;
                if (is_halo(t) && sp > 1) break;
                if (!inv && sp > 1 && (tiles * sp > 4 * 256 || nkt / sp < 2)) break;
                if (sp > 1 && (size_t)sp * M * op.cout_p * 4 > BWD_TUNE_SCRATCH) continue;
                float ms = 0.f;
                STCHK(time_candidate([&] { return enqueue_op(net, p, op, base, s, false, t, sp); }, e0, e1, s, &ms));
                timed.emplace_back(ms, t, sp);
            }
        }
        int bt = op.tile, bs = op.splits;
        pick_tuned(timed, &bt, &bs);
        std::lock_guard<std::mutex> g(net->mu);
        net->tuned[sig] = {bt, bs};
    }
    // the backward-data convs
    for (int k = 0; k < b.nops; ++k) {
        const Op &op = p.ops[k];
        if (op.kind != OP_CONV) continue;
        const dn_conv_desc &f = b.fwd[k];
        const std::string sig = bwd_sig(&f, b.acc[k]);
        if (net->tuned.count(sig)) continue;
        const ConvWeights &cw = net->cw[op.conv];
        dn_conv_desc bd;
        int ho, wo, hz, wz;
        STCHK(bwd_desc(&f, b.acc[k], &bd, &ho, &wo, &hz, &wz));
        ConvArgs a;
        STCHK(conv_geometry(&bd, &a, nullptr, nullptr, nullptr, nullptr, nullptr));
        const int nkt = a.k_pad / bk_el(dt);
        std::vector<int> cands;
        if (halo_ok(dt, a)) cands.push_back(HALO_TILE);
        if (halo2_ok(dt, a)) cands.push_back(HALO2_TILE);
        for (int t = 0; t < tile_count(); ++t)
            if (tile_fits(t, a.cout_p)) cands.push_back(t);
        std::vector<std::tuple<float, int, int>> timed;
        for (int t : cands) {
            const TileCfg tc = is_halo(t) ? TileCfg{1 << 30, 1 << 30, 1, 1} : tile_cfg(t);
            const long tiles = (long)((a.M + tc.bm - 1) / tc.bm) * ((a.cout_p + tc.bn - 1) / tc.bn);
            for (int sp = 1; sp <= 16; sp *= 2) {
                if (is_halo(t) && sp > 1) break;
                if (sp > 1 && (tiles * sp > 4 * 256 || nkt / sp < 2)) break;
                dn_conv_desc cd;
                int h2, w2, hz2, wz2;
                STCHK(bwd_desc(&f, b.acc[k], &cd, &h2, &w2, &hz2, &wz2, t, sp));
                size_t ws = 0, z = 0;
                STCHK(bwd_scratch(&f, &cd, hz2, wz2, &ws, &z));
                if (ws + z > BWD_TUNE_SCRATCH) continue;
                float ms = 0.f;
                // the gradient of the full-size conv output (for a fused pool: the unpooled one)
                char *gy = base + b.goff[op.pool ? op.conv + 1 : op.out];
                STCHK(time_candidate([&] {
                    return enqueue_conv_backward(&f, gy, cw.wb, cw.bzero, cw.bscale, b.acc[k], base + b.goff[op.in],
                                                 scratch, BWD_TUNE_SCRATCH, s, t, sp);
                }, e0, e1, s, &ms));
                timed.emplace_back(ms, t, sp);
            }
        }
        std::pair<int, int> bt{-1, 0};
        pick_tuned(timed, &bt.first, &bt.second);
        std::lock_guard<std::mutex> g(net->mu);
        net->tuned[sig] = bt;
    }
    return DN_OK;
}

extern "C" dn_status dn_autotune_backward(dn_net *net, int layer, int batch, int h, int w, void *stream)
{
    if (!net) return fail(DN_EINVAL, "net is NULL");
    HIPCHK(hipSetDevice(net->o.device));
    load_tune_cache(net);
    BwdPlan b;
    STCHK(bwd_prepare(net, layer, batch, h, w, &b));
    // a synchronous tuning call: the pass's buffers and the candidates'
    // scratch live in a temporary allocation freed before returning
    char *base = nullptr;
    HIPCHK(hipMalloc(&base, b.total + BWD_TUNE_SCRATCH));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    dn_status rc = DN_OK;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) rc = fail(DN_EHIP, "hipEventCreate");
    if (rc == DN_OK) rc = autotune_backward(net, layer, batch, h, w, (hipStream_t)stream, e0, e1, base);
    (void)hipStreamSynchronize((hipStream_t)stream);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(base);
    if (rc == DN_OK) {
        std::lock_guard<std::mutex> g(net->mu);
        save_tune_cache(net);
        drop_graphs(net);
    }
    return rc;
}

extern "C" int dn_tile_count(void) { return tile_count(); }

extern "C" dn_status dn_tile_info(int tile, int *bm, int *bn, int *waves_m, int *waves_n, int *mfma_bf16)
{
    if (tile < 0 || tile >= tile_count()) return fail(DN_EINVAL, "tile %d out of range", tile);
    const TileCfg t = tile_cfg(tile);
    if (bm) *bm = t.bm;
    if (bn) *bn = t.bn;
    if (waves_m) *waves_m = t.wm;
    if (waves_n) *waves_n = t.wn;
    if (mfma_bf16) *mfma_bf16 = t.mf ? t.mf : 16;
    return DN_OK;
}
