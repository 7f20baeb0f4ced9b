// Implicit-GEMM convolution for gfx950 (CDNA4) with a fused epilogue.
//
// GEMM view (M = batch*Ho*Wo output pixels, N = output channels,
// K = R*S*Cin_pad):  Y[m][j] = sum_k A[m][k] * B[k][j].
// A is never materialised: each 128-byte K-slice of an A row is gathered from
// the NHWC input as eight 16-byte segments, each lying inside one filter tap
// (r, s) because channels are padded to 16 bytes, and staged in LDS.  The K
// order is k = (cb*R*S + r*S + s)*CB + ci (c = cb*CB + ci, CB = kblock_ch()):
// tap-major for narrow layers, channel-block-major for wide ones.  B is the
// packed weight matrix [cout_p][k_pad] (K contiguous).  Products run on MFMA
// with FP32 accumulation:
//   FP32  v_mfma_f32_16x16x4_f32        (4 issues per 16-wide K step)
//   BF16  v_mfma_f32_16x16x32_bf16
//   FP8   v_mfma_f32_16x16x128_f8f6f4   (OCP e4m3 operands)
// Every lane supplies its row (A) / column (B) of a 16x16 block with the same
// K subset for both operands, so each dot product covers every k once.
//
// Epilogue (per output element, FP32): acc * (FP8 weight scale * input scale)
// + folded bias -> leaky or linear -> [+ residual] -> [max over the four rows
// of a 2x2 pooling window] -> round to the storage type -> NHWC store.
// Pooling after the activation and after rounding are both exact because the
// activation and the rounding are monotone non-decreasing.
#include <algorithm>
#include <type_traits>

#include "dn_kernels.h"

namespace dnk {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef float f16v __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef int i32x8 __attribute__((ext_vector_type(8)));

// ---------------------------------------------------------------- conversions

__device__ __forceinline__ uint16_t f2bf(float f)
{
    return __builtin_bit_cast(uint16_t, (__bf16)f);  // v_cvt_pk_bf16_f32: round to nearest even
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
__device__ __forceinline__ uint8_t f2e4m3(float f)
{
    f = fminf(fmaxf(f, -448.0f), 448.0f);  // saturate
    return (uint8_t)(__builtin_amdgcn_cvt_pk_fp8_f32(f, f, 0, false) & 0xFF);
}
__device__ __forceinline__ float e4m32f(uint32_t b) { return __builtin_amdgcn_cvt_f32_fp8((int)b, 0); }

template <int DT> __device__ __forceinline__ float load_el(const void *p, size_t i)
{
    if constexpr (DT == F32) return ((const float *)p)[i];
    else if constexpr (DT == BF16) return bf2f(((const uint16_t *)p)[i]);
    else return e4m32f(((const uint8_t *)p)[i]);
}
template <int DT> __device__ __forceinline__ void store_el(void *p, size_t i, float v)
{
    if constexpr (DT == F32) ((float *)p)[i] = v;
    else if constexpr (DT == BF16) ((uint16_t *)p)[i] = f2bf(v);
    else ((uint8_t *)p)[i] = f2e4m3(v);
}
// four consecutive elements (i a multiple of 4), storage type -> FP32, one load
template <int DT> __device__ __forceinline__ void load4(const void *p, size_t i, float *v)
{
    if constexpr (DT == F32) {
        const float4 t = *reinterpret_cast<const float4 *>((const float *)p + i);
        v[0] = t.x; v[1] = t.y; v[2] = t.z; v[3] = t.w;
    } else if constexpr (DT == BF16) {
        const uint2 t = *reinterpret_cast<const uint2 *>((const uint16_t *)p + i);
        v[0] = bf2f((uint16_t)(t.x & 0xFFFFu)); v[1] = bf2f((uint16_t)(t.x >> 16));
        v[2] = bf2f((uint16_t)(t.y & 0xFFFFu)); v[3] = bf2f((uint16_t)(t.y >> 16));
    } else {
        const unsigned t = *reinterpret_cast<const unsigned *>((const uint8_t *)p + i);
#pragma unroll
        for (int j = 0; j < 4; ++j) v[j] = e4m32f((t >> (8 * j)) & 0xFFu);
    }
}
// four consecutive channels, FP32 values -> storage type, one store
template <int DT> __device__ __forceinline__ void store4(void *y, size_t idx, const float *v)
{
    if constexpr (DT == F32) {
        *reinterpret_cast<float4 *>((float *)y + idx) = make_float4(v[0], v[1], v[2], v[3]);
    } else if constexpr (DT == BF16) {
        *reinterpret_cast<uint2 *>((uint16_t *)y + idx) =
            make_uint2((unsigned)f2bf(v[0]) | ((unsigned)f2bf(v[1]) << 16), (unsigned)f2bf(v[2]) | ((unsigned)f2bf(v[3]) << 16));
    } else {
        *reinterpret_cast<unsigned *>((uint8_t *)y + idx) = (unsigned)f2e4m3(v[0]) | ((unsigned)f2e4m3(v[1]) << 8) |
                                                            ((unsigned)f2e4m3(v[2]) << 16) | ((unsigned)f2e4m3(v[3]) << 24);
    }
}

// ---------------------------------------------------------------- MFMA step

template <int DT> struct Tr;
// SPL: 16-byte segments per lane per MFMA K-step; KSPT: K-steps per 128-byte K-tile.
template <> struct Tr<F32> { static constexpr int SPL = 1, KSPT = 2; };
template <> struct Tr<BF16> { static constexpr int SPL = 1, KSPT = 2; };
template <> struct Tr<FP8> { static constexpr int SPL = 2, KSPT = 1; };

typedef unsigned int u32x4_t __attribute__((ext_vector_type(4)));

template <int DT> __device__ __forceinline__ void mma(f4 &acc, const u32x4_t *a, const u32x4_t *b)
{
    if constexpr (DT == F32) {
        const float af[4] = {__uint_as_float(a[0].x), __uint_as_float(a[0].y), __uint_as_float(a[0].z), __uint_as_float(a[0].w)};
        const float bf[4] = {__uint_as_float(b[0].x), __uint_as_float(b[0].y), __uint_as_float(b[0].z), __uint_as_float(b[0].w)};
#pragma unroll
        for (int j = 0; j < 4; ++j) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(af[j], bf[j], acc, 0, 0, 0);
    } else if constexpr (DT == BF16) {
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a[0]), __builtin_bit_cast(bf16x8, b[0]), acc, 0, 0, 0);
    } else {
        const i32x8 av = {(int)a[0].x, (int)a[0].y, (int)a[0].z, (int)a[0].w, (int)a[1].x, (int)a[1].y, (int)a[1].z, (int)a[1].w};
        const i32x8 bv = {(int)b[0].x, (int)b[0].y, (int)b[0].z, (int)b[0].w, (int)b[1].x, (int)b[1].y, (int)b[1].z, (int)b[1].w};
        // format 0 = e4m3 for both operands, no block scaling
        acc = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(av, bv, acc, 0, 0, 0, 0, 0, 0);
    }
}

// Blocks are dealt to the 8 XCDs round-robin; renumber them so that each XCD
// receives a contiguous run of tiles (neighbouring tiles share A rows / B
// columns in that XCD's L2).
__device__ __forceinline__ int xcd_remap(int bid, int G)
{
    const int per = (G + 7) >> 3;
    const int xcd = bid & 7, loc = bid >> 3;
    const int tall = G - (per - 1) * 8;
    return xcd < tall ? xcd * per + loc : tall * per + (xcd - tall) * (per - 1) + loc;
}

// Logical tile id -> (M tile, N tile).  N tiles are taken in groups of four;
// within a group the id runs over (M tile, N tile in group), N fastest.  The
// run of ids one XCD receives is then a block of about 8 M tiles x 4 N tiles
// rather than 4 x 8 when N has 8 tiles, which balances the input rows and
// weight columns its L2 has to hold.
__device__ __forceinline__ void tile_mn(int logical, int mt, int ntn, int &mi, int &ni)
{
    constexpr int GN = 4;
    const int ngf = ntn / GN;            // complete groups
    const int gtiles = mt * GN;
    if (logical < ngf * gtiles) {
        const int g = logical / gtiles, r = logical - g * gtiles;
        mi = r / GN;
        ni = g * GN + (r - (r / GN) * GN);
    } else {
        const int w = ntn - ngf * GN, r = logical - ngf * gtiles;
        mi = r / w;
        ni = ngf * GN + (r - (r / w) * w);
    }
}

// Leaky: v for v > 0, else v * slope.  For 0 <= slope <= 1 that is exactly
// max(v, v * slope) (signed zeros and NaN included), two instructions.
__device__ __forceinline__ float activate(float v, int act, float slope)
{
    if (act != 1) return v;
    if (slope >= 0.0f && slope <= 1.0f) return fmaxf(v, v * slope);
    return v > 0.0f ? v : v * slope;
}

// The same function as one select: with lin_slope = slope for leaky and 1 for
// linear, v > 0 ? v : v * lin_slope equals activate(v, act, slope) bit for bit
// (for any slope; signed zeros and NaN included), without a branch on act.
__device__ __forceinline__ float act_slope(int act, float slope) { return act == 1 ? slope : 1.0f; }
__device__ __forceinline__ float activate_sel(float v, float lin_slope) { return v > 0.0f ? v : v * lin_slope; }

// The value an output takes once stored (rounded to the storage type).
template <int DT> __device__ __forceinline__ float stored_value(float v)
{
    if constexpr (DT == F32) return v;
    else if constexpr (DT == BF16) return bf2f(f2bf(v));
    else return e4m32f(f2e4m3(v));
}

// Index (2*dy + dx) of the first maximal stored output of a 2x2 window whose
// accumulators are acc[0..3] in row-major window order: the branch the
// max-pool gradient follows.
// The output is activate(acc * scl + bias) * post, as in the caller's epilogue.
template <int DT> __device__ __forceinline__ unsigned char window_argmax(const float *acc, float scl, float bias,
                                                                        int act, float slope, float post)
{
    int k = 0;
    float m = stored_value<DT>(activate(acc[0] * scl + bias, act, slope) * post);
#pragma unroll
    for (int q = 1; q < 4; ++q) {
        const float o = stored_value<DT>(activate(acc[q] * scl + bias, act, slope) * post);
        if (o > m) { m = o; k = q; }
    }
    return (unsigned char)k;
}

// ---------------------------------------------------------------- the kernel

// Global-memory accesses go through explicit address-space-1 pointers so that
// the compiler emits global (not flat) loads: their completion is tracked by
// vmcnt alone and the LDS traffic of the current K-tile is not serialised
// behind the prefetch of the next one.
#define GLOBAL __attribute__((address_space(1)))
typedef u32x4_t u32x4;

__device__ __forceinline__ u32x4 gload16(const void *base, size_t byte_off)
{
    return *(const GLOBAL u32x4 *)((const GLOBAL char *)base + byte_off);
}

// Epilogue shared by the implicit-GEMM kernels.  MFMA 16x16 output layout:
// lane holds column (lane & 15) and rows 4*(lane >> 4) + i, i = 0..3; rowb /
// colb are this lane's first row / column.  With split-K the raw FP32
// partial sums go to the scratch plane of this split instead; when the last
// split finishes the tile in the same launch (a.tile_count set) they are
// device-scope stores, written through to where every XCD reads them.
// acc[g][f] holds rows rowb + g*RSTR + (0..3) of column colb + f*CSTR (16x16
// blocks: RSTR = CSTR = 16; 32x32 blocks split into four row quads: RSTR = 8,
// CSTR = 32).  Every quad starts at a multiple of 4, so with a fused pool it is
// one 2x2 window.
template <int DT, int FM, int FN, int RSTR = 16, int CSTR = 16>
__device__ __forceinline__ void conv_epilogue(const ConvArgs &a, f4 (&acc)[FM][FN], int rowb, int colb)
{
    if (a.splits > 1) {
        float *P = a.partial + (size_t)blockIdx.z * a.M * a.cout_p;
#pragma unroll
        for (int fn = 0; fn < FN; ++fn) {
            const int col = colb + fn * CSTR;
            if (col >= a.cout_p) continue;
#pragma unroll
            for (int fm = 0; fm < FM; ++fm)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int m = rowb + fm * RSTR + i;
                    if (m >= a.M) continue;
                    float *q = P + (size_t)m * a.cout_p + col;
                    if (a.tile_count) __hip_atomic_store(q, acc[fm][fn][i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    else *q = acc[fm][fn][i];
                }
        }
        return;
    }
#pragma unroll
    for (int fn = 0; fn < FN; ++fn) {
        const int col = colb + fn * CSTR;
        if (col >= a.cout_p) continue;
        const float bias = a.bias[col];
        const float scl = (DT == FP8) ? a.wscale[col] * a.in_scale : 1.0f;
#pragma unroll
        for (int fm = 0; fm < FM; ++fm) {
            const int mb = rowb + fm * RSTR;
            if (mb >= a.M) continue;
            if (a.pool) {
                // rows mb..mb+3 are one 2x2 window (M is a multiple of 4 here); pooling
                // the accumulators is exact: scale > 0, and bias, activation and
                // rounding are monotone
                const float mx = fmaxf(fmaxf(acc[fm][fn][0], acc[fm][fn][1]), fmaxf(acc[fm][fn][2], acc[fm][fn][3]));
                store_el<DT>(a.y, (size_t)(mb >> 2) * a.cout_p + col, activate(mx * scl + bias, a.act, a.slope) * a.out_inv_scale);
                if (a.argmax) {
                    const float w4[4] = {acc[fm][fn][0], acc[fm][fn][1], acc[fm][fn][2], acc[fm][fn][3]};
                    a.argmax[(size_t)(mb >> 2) * a.cout_p + col] = window_argmax<DT>(w4, scl, bias, a.act, a.slope, a.out_inv_scale);
                }
            } else {
                float v[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) v[i] = activate(acc[fm][fn][i] * scl + bias, a.act, a.slope);
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int m = mb + i;
                    if (m >= a.M) break;
                    float o = v[i];
                    if (a.res) o += load_el<DT>(a.res, (size_t)m * a.cout_p + col) * a.res_scale;
                    store_el<DT>(a.y, (size_t)m * a.cout_p + col, o * a.out_inv_scale);
                }
            }
        }
    }
}

// 16-byte device-scope load (the buffer instruction's SC1 bit): it misses in
// the caches that other XCDs' stores do not reach.  off: bytes from base.
__device__ __forceinline__ f4 load16_dev(const float *base, unsigned off)
{
    const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc((void *)base, (short)0, 0x7fffffff, 0x00020000);
    return __builtin_bit_cast(f4, __builtin_amdgcn_raw_buffer_load_b128(r, (int)off, 0, 16));
}

// Split-K finish of one output group: rows (2x2 windows when pooled) `ro`,
// channels col..col+3 (cout_p is a multiple of 4): the partial sums added in
// split order, then the same epilogue as the unsplit path, one vector store.
// Both finishes below call it, so they round alike.  The separate finish
// reads each split's partials with one 16-byte load as it adds them; the
// in-kernel finish (DEV) issues the device-scope loads of all splits first,
// so that they are in flight together, then adds them in the same order.
template <int DT, bool DEV = false> __device__ __forceinline__ void splitk_finish4(const ConvArgs &a, size_t ro, int col)
{
    float bias[4], scl[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        bias[j] = a.bias[col + j];
        scl[j] = (DT == FP8) ? a.wscale[col + j] * a.in_scale : 1.0f;
    }
    const size_t plane = (size_t)a.M * a.cout_p;
    auto total = [&](size_t m, float *t) {
        t[0] = t[1] = t[2] = t[3] = 0.0f;
        if constexpr (DEV) {
            f4 v[SPLITK_FUSED_MAX];
#pragma unroll
            for (int z = 0; z < SPLITK_FUSED_MAX; ++z)
                if (z < a.splits) v[z] = load16_dev(a.partial, (unsigned)((z * plane + m * a.cout_p + col) * sizeof(float)));
#pragma unroll
            for (int z = 0; z < SPLITK_FUSED_MAX; ++z)
                if (z < a.splits) { t[0] += v[z][0]; t[1] += v[z][1]; t[2] += v[z][2]; t[3] += v[z][3]; }
        } else {
            for (int z = 0; z < a.splits; ++z) {
                const float4 p = *reinterpret_cast<const float4 *>(a.partial + z * plane + m * a.cout_p + col);
                t[0] += p.x; t[1] += p.y; t[2] += p.z; t[3] += p.w;
            }
        }
    };
    float o[4], t[4];
    if (a.pool) {
        float w4[4][4];  // [column][window element]
#pragma unroll
        for (int j = 0; j < 4; ++j) o[j] = -INFINITY;
        for (int q = 0; q < 4; ++q) {
            total(ro * 4 + q, t);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                w4[j][q] = t[j];
                o[j] = fmaxf(o[j], activate(t[j] * scl[j] + bias[j], a.act, a.slope));
            }
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) o[j] *= a.out_inv_scale;
        if (a.argmax) {
#pragma unroll
            for (int j = 0; j < 4; ++j) a.argmax[ro * a.cout_p + col + j] = window_argmax<DT>(w4[j], scl[j], bias[j], a.act, a.slope, a.out_inv_scale);
        }
    } else {
        total(ro, t);
#pragma unroll
        for (int j = 0; j < 4; ++j) o[j] = activate(t[j] * scl[j] + bias[j], a.act, a.slope);
        if (a.res) {
            float r[4];
            load4<DT>(a.res, ro * a.cout_p + col, r);
#pragma unroll
            for (int j = 0; j < 4; ++j) o[j] += r[j] * a.res_scale;
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) o[j] *= a.out_inv_scale;
    }
    store4<DT>(a.y, ro * a.cout_p + col, o);
}

// Separate split-K finish: one thread per output group.
template <int DT>
__global__ void __launch_bounds__(256) splitk_reduce(ConvArgs a)
{
    const size_t rows = a.pool ? (size_t)(a.M >> 2) : (size_t)a.M;
    const int cq = a.cout_p >> 2;
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= rows * cq) return;
    splitk_finish4<DT>(a, idx / cq, (int)(idx % cq) * 4);
}

// In-kernel split-K finish (a.tile_count set).  Each split's workgroup of an
// output tile, once its partial plane is written, counts itself in the tile's
// counter; the last of the a.splits workgroups to arrive sums the tile's
// partials in split order and runs the epilogue, then sets the counter back
// to zero for the next launch that uses it.  The L2 caches of the XCDs are
// not coherent with each other: the partials travel by device-scope stores,
// all complete (vmcnt 0) before the workgroup counts itself, and device-scope
// loads issued after the count is seen, so no cache-wide write-back or
// invalidate is needed.
template <int DT, int BM, int BN, int NT>
__device__ __forceinline__ void splitk_tail(const ConvArgs &a, int m0, int n0)
{
    __shared__ int s_last;
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned *cnt = a.tile_count + blockIdx.x;
        const int last = __hip_atomic_fetch_add(cnt, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == (unsigned)(a.splits - 1);
        if (last) __hip_atomic_store(cnt, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        s_last = last;
    }
    __syncthreads();
    if (!s_last) return;
    const int rows = a.pool ? BM / 4 : BM;
    const int r0 = a.pool ? m0 / 4 : m0;
    const int rend = a.pool ? a.M / 4 : a.M;
    constexpr int CQ = BN / 4;
    for (int i = threadIdx.x; i < rows * CQ; i += NT) {
        const int r = r0 + i / CQ, col = n0 + (i % CQ) * 4;
        if (r < rend && col < a.cout_p) splitk_finish4<DT, true>(a, (size_t)r, col);
    }
}

// Position of one lane's 16-byte K segment in the packed K order, advanced
// K-tile by K-tile (a workgroup loads its K-tiles in increasing order): the
// filter tap (r, s) and input channel c0 of k = kt*BKE + sc*SEG, with the
// divisions done once at the first K-tile instead of at every one.
// Tap-major order: k = tap*cin_p + c.  Channel-block-major (cbsh >= 0):
// blocks of CB = 2^cbsh channels, every tap of a block before the next block;
// a K-tile lies inside one block (BKE divides CB).  The segment is inside K
// when r < R and c0 < cin_p.
struct KPos {
    int r, s, c0, off, cbase;  // off, cbase: offset in and start of the channel block
    __device__ __forceinline__ void init(int k0, int cin_p, int RS, int S, int cbsh)
    {
        int tap;
        if (cbsh < 0) {
            tap = k0 / cin_p;
            c0 = k0 - tap * cin_p;
            off = cbase = 0;
        } else {
            const int blk = k0 >> cbsh, cb = blk / RS;
            tap = blk - cb * RS;
            cbase = cb << cbsh;
            off = k0 & ((1 << cbsh) - 1);
            c0 = cbase + off;
        }
        r = tap / S;
        s = tap - r * S;
    }
    __device__ __forceinline__ void next(int bke, int cin_p, int R, int S, int cbsh)
    {
        if (cbsh < 0) {
            c0 += bke;
            while (c0 >= cin_p) {
                c0 -= cin_p;
                if (++s == S) { s = 0; ++r; }
            }
        } else {
            off += bke;
            if (off >= (1 << cbsh)) {
                off -= 1 << cbsh;
                if (++s == S) {
                    s = 0;
                    if (++r == R) { r = 0; cbase += 1 << cbsh; }
                }
            }
            c0 = cbase + off;
        }
    }
};

template <int DT, int BM, int BN, int WM, int WN>
__global__ void __launch_bounds__(64 * WM * WN) conv_igemm(ConvArgs a)
{
    constexpr int NT = 64 * WM * WN;
    constexpr int ES = esize(DT), SEG = seg_el(DT), BKE = bk_el(DT);
    constexpr int RSTEP = NT / 8;                       // rows covered per load pass
    constexpr int AR = BM / RSTEP;                      // A rows per thread
    constexpr int BR = (BN + RSTEP - 1) / RSTEP;        // B rows per thread
    constexpr int WTM = BM / WM, WTN = BN / WN, FM = WTM / 16, FN = WTN / 16;
    constexpr int SPL = Tr<DT>::SPL, KSPT = Tr<DT>::KSPT;
    static_assert(BM % RSTEP == 0 && WTM % 16 == 0 && WTN % 16 == 0, "tile shape");

    __shared__ u32x4 sA[2][BM * 8];
    __shared__ u32x4 sB[2][BN * 8];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave % WM, wn = wave / WM;

    const int ntn = (a.cout_p + BN - 1) / BN;
    const int logical = xcd_remap(blockIdx.x, gridDim.x);
    int mi, ni;
    tile_mn(logical, gridDim.x / ntn, ntn, mi, ni);
    const int m0 = mi * BM, n0 = ni * BN;

    // ---- per-row gather state for A (fixed for the whole K loop)
    const int sc = tid & 7;
    const int rbase = tid >> 3;
    int a_pix[AR], a_hi[AR], a_wi[AR];
#pragma unroll
    for (int i = 0; i < AR; ++i) {
        const int m = m0 + rbase + i * RSTEP;
        a_pix[i] = 0; a_hi[i] = -(1 << 28); a_wi[i] = 0;
        if (m < a.M) {
            int n, ho, wo;
            if (a.pool) {
                const int q = m & 3, win = m >> 2, wp2 = a.Wo >> 1, hp2 = a.Ho >> 1;
                const int wp = win % wp2, t = win / wp2;
                ho = 2 * (t % hp2) + (q >> 1); wo = 2 * wp + (q & 1); n = t / hp2;
            } else {
                wo = m % a.Wo; const int t = m / a.Wo; ho = t % a.Ho; n = t / a.Ho;
            }
            a_pix[i] = n * a.H * a.W;
            a_hi[i] = ho * a.stride - a.pad;
            a_wi[i] = wo * a.stride - a.pad;
        }
    }
    bool b_ok[BR];
    size_t b_off[BR];
#pragma unroll
    for (int i = 0; i < BR; ++i) {
        const int row = rbase + i * RSTEP, n = n0 + row;
        b_ok[i] = row < BN && n < a.cout_p;
        b_off[i] = ((size_t)(b_ok[i] ? n : 0) * a.k_pad + sc * SEG) * ES;
    }

    const int nkt = a.k_pad / BKE;
    const int kt0 = blockIdx.z * a.ktiles_per_split;
    const int kt1 = min(nkt, kt0 + a.ktiles_per_split);
    const int RS = a.R * a.S;
    const int cbsh = kblock_ch(DT, a.cin_p, RS) == a.cin_p ? -1 : 7 - (ES >> 1);  // log2 of a 128-byte block
    const u32x4 zero4 = {0u, 0u, 0u, 0u};
    KPos kp;
    kp.init(kt0 * BKE + sc * SEG, a.cin_p, RS, a.S, cbsh);
    long long a_base[AR];  // element offset of each row's tap (0, 0), channel 0 (meaningful where in range)
#pragma unroll
    for (int i = 0; i < AR; ++i) a_base[i] = ((long long)a_pix[i] + (long long)a_hi[i] * a.W + a_wi[i]) * a.cin_p;

    u32x4 ra[AR], rb[BR];
    f4 acc[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};

    const int lrow = lane & 15, lgrp = lane >> 4;

// Issue the global loads of K-tile KT into ra / rb (no wait).  KT must be the
// K-tile after the previous call's (kp advances one K-tile per call).
#define DN_GLOAD(KT)                                                                           \
    do {                                                                                       \
        const int r_ = kp.r, s_ = kp.s;                                                        \
        const bool kv_ = r_ < a.R && kp.c0 < a.cin_p;                                          \
        const long long toff_ = ((long long)r_ * a.W + s_) * a.cin_p + kp.c0;                  \
        _Pragma("unroll") for (int i = 0; i < AR; ++i) {                                       \
            const int hi_ = a_hi[i] + r_, wi_ = a_wi[i] + s_;                                  \
            const bool ok_ = kv_ && (unsigned)hi_ < (unsigned)a.H && (unsigned)wi_ < (unsigned)a.W; \
            const size_t off_ = ok_ ? (size_t)(a_base[i] + toff_) * ES : 0;                    \
            ra[i] = ok_ ? gload16(a.x, off_) : zero4;                                          \
        }                                                                                      \
        const size_t kb_ = (size_t)(KT) * BKE * ES;                                            \
        _Pragma("unroll") for (int i = 0; i < BR; ++i)                                         \
            rb[i] = b_ok[i] ? gload16(a.w, b_off[i] + kb_) : zero4;                            \
        kp.next(BKE, a.cin_p, a.R, a.S, cbsh);                                                 \
    } while (0)

// Write ra / rb into LDS stage BUF (rows swizzled: segment s of row r sits at s ^ (r & 7)).
#define DN_SSTORE(BUF)                                                                         \
    do {                                                                                       \
        _Pragma("unroll") for (int i = 0; i < AR; ++i) {                                       \
            const int row_ = rbase + i * RSTEP;                                                \
            sA[BUF][row_ * 8 + (sc ^ (row_ & 7))] = ra[i];                                     \
        }                                                                                      \
        _Pragma("unroll") for (int i = 0; i < BR; ++i) {                                       \
            const int row_ = rbase + i * RSTEP;                                                \
            if (row_ < BN) sB[BUF][row_ * 8 + (sc ^ (row_ & 7))] = rb[i];                      \
        }                                                                                      \
    } while (0)

    if (kt0 < kt1) {
        DN_GLOAD(kt0);
        DN_SSTORE(0);
    }
    __syncthreads();
    for (int kt = kt0; kt < kt1; ++kt) {
        const int buf = (kt - kt0) & 1;
        const bool more = kt + 1 < kt1;
        if (more) DN_GLOAD(kt + 1);
#pragma unroll
        for (int ks = 0; ks < KSPT; ++ks) {
            u32x4 af[FM][SPL], bfr[FN][SPL];
#pragma unroll
            for (int fm = 0; fm < FM; ++fm) {
                const int row = wm * WTM + fm * 16 + lrow;
#pragma unroll
                for (int j = 0; j < SPL; ++j) {
                    const int seg = ks * 4 * SPL + lgrp * SPL + j;
                    af[fm][j] = sA[buf][row * 8 + (seg ^ (row & 7))];
                }
            }
#pragma unroll
            for (int fn = 0; fn < FN; ++fn) {
                const int row = wn * WTN + fn * 16 + lrow;
#pragma unroll
                for (int j = 0; j < SPL; ++j) {
                    const int seg = ks * 4 * SPL + lgrp * SPL + j;
                    bfr[fn][j] = sB[buf][row * 8 + (seg ^ (row & 7))];
                }
            }
#pragma unroll
            for (int fm = 0; fm < FM; ++fm)
#pragma unroll
                for (int fn = 0; fn < FN; ++fn) mma<DT>(acc[fm][fn], af[fm], bfr[fn]);
        }
        // keep the LDS stores of the next tile behind this tile's MFMAs, so the
        // wait for its global loads overlaps the matrix work
        __builtin_amdgcn_sched_barrier(0);
        if (more) DN_SSTORE(buf ^ 1);
        __syncthreads();
    }
#undef DN_GLOAD
#undef DN_SSTORE

    conv_epilogue<DT, FM, FN>(a, acc, m0 + wm * WTM + 4 * lgrp, n0 + wn * WTN + lrow);
    if (a.splits > 1 && a.tile_count) splitk_tail<DT, BM, BN, NT>(a, m0, n0);
}

// ---------------------------------------------------------------- LDS-DMA variant
// Same GEMM, but the K-tiles travel global -> LDS directly
// (buffer_load_dwordx4 ... lds: lane L of a wave instruction writes bytes
// [16L, 16L + 16) of a 1 KB LDS block, i.e. row L/8, physical segment L%8 of
// an 8-row group).  No VGPR staging, so NS-1 K-tiles can be in flight while
// one is multiplied.  Out-of-range taps and rows use an offset past the
// buffer's size, for which the buffer load returns zeros.
#define DN_OOB 0x80000000u

__device__ __forceinline__ void lds_barrier() { asm volatile("s_barrier" ::: "memory"); }

template <int N> __device__ __forceinline__ void wait_vm()
{
    // s_waitcnt vmcnt(N) with expcnt / lgkmcnt left at their maxima (no wait)
    static_assert(N >= 0 && N < 64, "vmcnt range");
    __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (7 << 4) | (15 << 8));
}

typedef int i32x4 __attribute__((ext_vector_type(4)));

// Buffer resource (V#) for raw 32-bit-offset loads: base, stride 0,
// num_records = size in bytes (loads at or past it return zeros).
__device__ __forceinline__ i32x4 make_rsrc(const void *base, unsigned bytes)
{
    const unsigned long long b = (unsigned long long)base;
    return i32x4{(int)(unsigned)b, (int)(unsigned)(b >> 32), (int)bytes, 0x00020000};
}

// One 16-byte-per-lane global -> LDS transfer.  Issued as inline assembly so
// that the compiler does not see an LDS write in flight: it would otherwise
// drain every outstanding transfer (vmcnt(0)) before each LDS read, and the
// pipeline below could not keep K-tiles in flight.  Completion is tracked by
// the explicit vmcnt waits + barrier of the main loop.
// m0 is reserved for the compiler's own LDS-DMA / message use, none of which
// this file emits; listing it as clobbered keeps any such use correct.
#pragma clang diagnostic push
#pragma clang diagnostic ignored "-Winline-asm"
__device__ __forceinline__ void dma16(const i32x4 &rsrc, unsigned voff, const void *lds_dst)
{
    // the destination is wave-uniform by construction; say so to the compiler
    const unsigned m0v = __builtin_amdgcn_readfirstlane(
        (unsigned)(size_t)(const __attribute__((address_space(3))) void *)lds_dst);
    asm volatile("s_mov_b32 m0, %0\n\ts_nop 0\n\tbuffer_load_dwordx4 %1, %2, 0 offen lds"
                 :
                 : "s"(m0v), "v"(voff), "s"(rsrc)
                 : "memory", "m0");
}
#pragma clang diagnostic pop

// SPR = 16-byte segments per LDS row (8: 128-byte K-tile, 4: 64-byte K-tile,
// which halves a stage so that four stages of a 256x256 tile fit in LDS).
// Row r stores logical segment s at physical segment s ^ swz(r); swz makes
// the 16 lanes of an MFMA fragment read hit distinct banks.
template <int SPR> __device__ __forceinline__ int seg_swz(int row)
{
    return SPR == 8 ? (row & 7) : ((row >> 2) & 3);
}

// MF = 16: 16x16 MFMA blocks (every dtype); MF = 32: 32x32x16 BF16 blocks,
// which take twice the passes of a 16x16x32 block for twice the products
// (the same rate) but read each 1 KB operand fragment for twice the work, so
// a tile needs half the LDS reads per product.  A 32x32 fragment: lane l holds row l%32 and K
// elements [8*(l/32), 8*(l/32) + 8) of the 16-element step, i.e. one 16-byte
// segment; the result quad q of a lane covers rows 8q + 4*(l/32) + (0..3).
template <int DT, int BM, int BN, int WM, int WN, int NS, int SPR, int MF = 16>
__global__ void __launch_bounds__(64 * WM * WN) conv_igemm_dl(ConvArgs a)
{
    constexpr int NW = WM * WN;
    constexpr int ES = esize(DT), SEG = seg_el(DT);
    constexpr int BKE = SPR * SEG;                      // K elements per tile
    constexpr int RPI = 64 / SPR;                       // rows filled by one wave-wide transfer
    constexpr int RSTEP = RPI * NW;
    constexpr int AGRP = BM / RPI, BGRP = BN / RPI;     // row groups (one transfer each) per tile
    constexpr int AR = (AGRP + NW - 1) / NW, BR = (BGRP + NW - 1) / NW;  // transfers per wave (max)
    constexpr int LPT = AR + BR;
    constexpr int WTM = BM / WM, WTN = BN / WN, FM = WTM / MF, FN = WTN / MF;
    constexpr int SPL = Tr<DT>::SPL;
    constexpr int KSPT = MF == 16 ? SPR / (4 * SPL) : SPR / 2;  // MFMA K-steps per tile
    static_assert(MF == 16 || (MF == 32 && DT == BF16), "32x32 blocks are BF16 only");
    static_assert(KSPT >= 1 && (MF == 32 || KSPT * 4 * SPL == SPR), "K-tile / MFMA step mismatch");
    static_assert(BM % RPI == 0 && BN % RPI == 0 && WTM % MF == 0 && WTN % MF == 0, "tile shape");
    typedef std::conditional_t<MF == 16, f4, f16v> accT;
    static_assert(NS >= 2 && NS <= 4 && LPT * (NS - 2) < 64, "pipeline depth");

    __shared__ u32x4 sA[NS][BM * SPR];
    __shared__ u32x4 sB[NS][BN * SPR];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave % WM, wn = wave / WM;
    const int ntn = (a.cout_p + BN - 1) / BN;
    const int logical = xcd_remap(blockIdx.x, gridDim.x);
    int mi, ni;
    tile_mn(logical, gridDim.x / ntn, ntn, mi, ni);
    const int m0 = mi * BM, n0 = ni * BN;
    // transfers this wave issues per K-tile (waves share the row groups round-robin)
    const int my_a = (AGRP - wave + NW - 1) / NW, my_b = (BGRP - wave + NW - 1) / NW;
    const int my_lpt = my_a + my_b;

    // lane L of a transfer fills row L/SPR, physical segment L%SPR of its row
    // group; with the swizzle that is the logical segment below
    const int rbase = wave * RPI + lane / SPR;          // this lane's row in the wave's first group
    const int sc = (lane % SPR) ^ seg_swz<SPR>(rbase);
    int a_pix[AR], a_hi[AR], a_wi[AR];
#pragma unroll
    for (int i = 0; i < AR; ++i) {
        const int m = m0 + rbase + i * RSTEP;
        a_pix[i] = 0; a_hi[i] = -(1 << 28); a_wi[i] = 0;
        if (m < a.M) {
            int n, ho, wo;
            if (a.pool) {
                const int q = m & 3, win = m >> 2, wp2 = a.Wo >> 1, hp2 = a.Ho >> 1;
                const int wp = win % wp2, t = win / wp2;
                ho = 2 * (t % hp2) + (q >> 1); wo = 2 * wp + (q & 1); n = t / hp2;
            } else {
                wo = m % a.Wo; const int t = m / a.Wo; ho = t % a.Ho; n = t / a.Ho;
            }
            a_pix[i] = n * a.H * a.W;
            a_hi[i] = ho * a.stride - a.pad;
            a_wi[i] = wo * a.stride - a.pad;
        }
    }
    unsigned b_off[BR];
#pragma unroll
    for (int i = 0; i < BR; ++i) {
        const int n = n0 + rbase + i * RSTEP;
        b_off[i] = n < a.cout_p ? (unsigned)(((size_t)n * a.k_pad + sc * SEG) * ES) : DN_OOB;
    }
    const i32x4 rx = make_rsrc(a.x, a.x_bytes);
    const i32x4 rw = make_rsrc(a.w, a.w_bytes);

    const int nkt = a.k_pad / BKE;
    const int tpk = bk_el(DT) / BKE;                    // tiles per 128-byte split-K unit
    const int kt0 = blockIdx.z * a.ktiles_per_split * tpk;
    const int kt1 = min(nkt, kt0 + a.ktiles_per_split * tpk);
    const int RS = a.R * a.S;
    // channel-block-major K order uses a power-of-two block (32 / 64 / 128 channels)
    const int cbsh = kblock_ch(DT, a.cin_p, RS) == a.cin_p ? -1 : 7 - (ES >> 1);
    KPos kp;  // this lane's K segment of the next K-tile to issue (issued in increasing order)
    kp.init(kt0 * BKE + sc * SEG, a.cin_p, RS, a.S, cbsh);
    long long a_base[AR];  // element offset of each row's tap (0, 0), channel 0 (meaningful where in range)
#pragma unroll
    for (int i = 0; i < AR; ++i) a_base[i] = ((long long)a_pix[i] + (long long)a_hi[i] * a.W + a_wi[i]) * a.cin_p;

    auto issue = [&](int kt, int st) {
        const int r = kp.r, s = kp.s;
        const bool kv = r < a.R && kp.c0 < a.cin_p;
        const long long toff = ((long long)r * a.W + s) * a.cin_p + kp.c0;
#pragma unroll
        for (int i = 0; i < AR; ++i) {
            if (AGRP % NW != 0 && i == AR - 1 && i >= my_a) break;  // wave-uniform
            const int hi = a_hi[i] + r, wi = a_wi[i] + s;
            const bool ok = kv && (unsigned)hi < (unsigned)a.H && (unsigned)wi < (unsigned)a.W;
            const unsigned off = ok ? (unsigned)((a_base[i] + toff) * ES) : DN_OOB;
            dma16(rx, off, &sA[st][(wave + i * NW) * 64]);
        }
        const unsigned kb = (unsigned)(kt * BKE * ES);
#pragma unroll
        for (int i = 0; i < BR; ++i) {
            if (BGRP % NW != 0 && i == BR - 1 && i >= my_b) break;  // wave-uniform
            const unsigned off = b_off[i] == DN_OOB ? DN_OOB : b_off[i] + kb;
            dma16(rw, off, &sB[st][(wave + i * NW) * 64]);
        }
        kp.next(BKE, a.cin_p, a.R, a.S, cbsh);
    };

    accT acc[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) acc[i][j] = accT{};
    const int lrow = lane & 15, lgrp = lane >> 4;

#pragma unroll
    for (int st = 0; st < NS - 1; ++st)
        if (kt0 + st < kt1) issue(kt0 + st, st);

    int cs = 0;  // stage holding tile kt
    for (int kt = kt0; kt < kt1; ++kt) {
        // this wave's transfers of tile kt landed; later tiles may stay in flight
        const int after = min(NS - 2, kt1 - 1 - kt);  // tiles issued after kt so far
        if (after == 0) wait_vm<0>();
        else if (my_lpt == LPT) { if (after >= 2) wait_vm<LPT * 2>(); else wait_vm<LPT>(); }
        else if (my_lpt == LPT - 1) { if (after >= 2) wait_vm<(LPT - 1) * 2>(); else wait_vm<LPT - 1>(); }
        else { if (after >= 2) wait_vm<(LPT > 1 ? LPT - 2 : 0) * 2>(); else wait_vm<(LPT > 1 ? LPT - 2 : 0)>(); }
        lds_barrier();  // every wave's transfers landed; every wave is done with tile kt-1
        if (kt + NS - 1 < kt1) issue(kt + NS - 1, cs == 0 ? NS - 1 : cs - 1);
        if constexpr (MF == 32) {
            const int r32 = lane & 31, h = lane >> 5;
#pragma unroll
            for (int ks = 0; ks < KSPT; ++ks) {
                const int seg = ks * 2 + h;
                u32x4 af[FM], bfr[FN];
#pragma unroll
                for (int fm = 0; fm < FM; ++fm) {
                    const int row = wm * WTM + fm * 32 + r32;
                    af[fm] = sA[cs][row * SPR + (seg ^ seg_swz<SPR>(row))];
                }
#pragma unroll
                for (int fn = 0; fn < FN; ++fn) {
                    const int row = wn * WTN + fn * 32 + r32;
                    bfr[fn] = sB[cs][row * SPR + (seg ^ seg_swz<SPR>(row))];
                }
#pragma unroll
                for (int fm = 0; fm < FM; ++fm)
#pragma unroll
                    for (int fn = 0; fn < FN; ++fn)
                        acc[fm][fn] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, af[fm]),
                                                                             __builtin_bit_cast(bf16x8, bfr[fn]),
                                                                             acc[fm][fn], 0, 0, 0);
            }
        } else {
#pragma unroll
        for (int ks = 0; ks < KSPT; ++ks) {
            u32x4 af[FM][SPL], bfr[FN][SPL];
#pragma unroll
            for (int fm = 0; fm < FM; ++fm) {
                const int row = wm * WTM + fm * 16 + lrow;
#pragma unroll
                for (int j = 0; j < SPL; ++j) {
                    const int seg = ks * 4 * SPL + lgrp * SPL + j;
                    af[fm][j] = sA[cs][row * SPR + (seg ^ seg_swz<SPR>(row))];
                }
            }
#pragma unroll
            for (int fn = 0; fn < FN; ++fn) {
                const int row = wn * WTN + fn * 16 + lrow;
#pragma unroll
                for (int j = 0; j < SPL; ++j) {
                    const int seg = ks * 4 * SPL + lgrp * SPL + j;
                    bfr[fn][j] = sB[cs][row * SPR + (seg ^ seg_swz<SPR>(row))];
                }
            }
#pragma unroll
            for (int fm = 0; fm < FM; ++fm)
#pragma unroll
                for (int fn = 0; fn < FN; ++fn) mma<DT>(acc[fm][fn], af[fm], bfr[fn]);
        }
        }
        cs = cs + 1 == NS ? 0 : cs + 1;
    }
    if constexpr (MF == 32) {
        f4 q4[FM * 4][FN];
#pragma unroll
        for (int fm = 0; fm < FM; ++fm)
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int fn = 0; fn < FN; ++fn)
                    q4[fm * 4 + q][fn] = f4{acc[fm][fn][4 * q], acc[fm][fn][4 * q + 1], acc[fm][fn][4 * q + 2], acc[fm][fn][4 * q + 3]};
        conv_epilogue<DT, FM * 4, FN, 8, 32>(a, q4, m0 + wm * WTM + 4 * (lane >> 5), n0 + wn * WTN + (lane & 31));
    } else {
        conv_epilogue<DT, FM, FN>(a, acc, m0 + wm * WTM + 4 * lgrp, n0 + wn * WTN + lrow);
    }
    if (a.splits > 1 && a.tile_count) splitk_tail<DT, BM, BN, 64 * NW>(a, m0, n0);
}

// Dynamic LDS above the default per-kernel limit must be enabled per kernel.
template <typename K> static void allow_lds(K kernel, size_t bytes)
{
    if (bytes > 64 * 1024) (void)hipFuncSetAttribute((const void *)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

// ---------------------------------------------------------------- first layer
// The network's first convolution reads the caller's NCHW FP32 image itself
// (the ingest is fused).  A th x 64 output tile (th = 16, or 8 when the window
// of 16 rows would not fit in LDS) stages its input window in LDS as NHWC in
// the storage type, channels padded to CP = 4, 8 or 16 with zeros.  The packed
// weights use the K order k = r*16 + s*CP + c (CP*S <= 16), so the 16 K
// elements of filter row r for output pixel (ho, wo) are the window pixels
// (ho*stride + r, wo*stride + s), s < S: a contiguous span of the window, read
// straight into the MFMA operand (read units past S are zero, matching zero
// weights).  The weights are operand A and stay in registers for the tile;
// pixels are operand B, so a lane's accumulator holds four consecutive output
// channels of one pixel and leaves with one vector store.  With POOL a
// 16-pixel block is four 2x2 windows on lanes 4w..4w+3, reduced by two quad
// shuffles.

constexpr int FT_W = 64;   // conv output columns per workgroup tile

__host__ __device__ constexpr int first_kstep(int dt) { return dt == FP8 ? 128 : (dt == BF16 ? 32 : 16); }
int first_kpad(int dt, int R) { return (R * 16 + first_kstep(dt) - 1) / first_kstep(dt) * first_kstep(dt); }

// CP floats -> one window pixel in the storage type (CP*esize bytes at dst)
// (sc is 1 except for FP8, so only FP8 multiplies)
template <int DT, int CP> __device__ __forceinline__ void put_pixel(unsigned char *dst, const float *v, float sc)
{
    constexpr int NW = CP * esize(DT) / 4;  // 32-bit words
    unsigned w[NW];
#pragma unroll
    for (int i = 0; i < NW; ++i) {
        if constexpr (DT == F32) {
            w[i] = __float_as_uint(v[i]);
        } else if constexpr (DT == BF16) {
            w[i] = (unsigned)f2bf(v[2 * i]) | ((unsigned)f2bf(v[2 * i + 1]) << 16);
        } else {
            w[i] = (unsigned)f2e4m3(v[4 * i] * sc) | ((unsigned)f2e4m3(v[4 * i + 1] * sc) << 8) |
                   ((unsigned)f2e4m3(v[4 * i + 2] * sc) << 16) | ((unsigned)f2e4m3(v[4 * i + 3] * sc) << 24);
        }
    }
    if constexpr (NW == 1) {
        *reinterpret_cast<unsigned *>(dst) = w[0];
    } else if constexpr (NW == 2) {
        *reinterpret_cast<uint2 *>(dst) = make_uint2(w[0], w[1]);
    } else {
#pragma unroll
        for (int q = 0; q < NW / 4; ++q)
            reinterpret_cast<u32x4 *>(dst)[q] = u32x4{w[4 * q], w[4 * q + 1], w[4 * q + 2], w[4 * q + 3]};
    }
}


// s * v + c for a wave-uniform s (24-bit operands) as one v_mad_u32_u24.
// Written out because, for v in {0, 1}, the compiler turns the multiply into
// a select plus an add (two instructions).
__device__ __forceinline__ unsigned mad_u24(int s, int v, int c)
{
    unsigned r;
    asm("v_mad_u32_u24 %0, %1, %2, %3" : "=v"(r) : "s"(s), "v"(v), "v"(c));
    return r;
}
typedef unsigned u32x2 __attribute__((ext_vector_type(2)));

// AM (with POOL): also store each window's argmax code (a.argmax); a template
// flag so that the forward's own instantiations carry none of that code.
template <int DT, bool POOL, int CP, bool AM = false, int NBM = FIRST_MAX_COUT / 16>
__global__ void __launch_bounds__(256) conv_first(FirstArgs a)
{
    constexpr int ES = esize(DT), SEG = seg_el(DT);
    constexpr int SPL = Tr<DT>::SPL, KSTEP = first_kstep(DT);
    constexpr int KPL = KSTEP / 4;                               // K elements per lane per step
    constexpr int PIXB = CP * ES;                                // bytes per window pixel
    constexpr int UB = PIXB < 16 ? PIXB : 16;                    // LDS read unit
    constexpr int UPS = 16 / UB;                                 // read units per 16-byte segment
    constexpr int MAXKS = DT == FP8 ? 1 : (DT == BF16 ? 2 : 4);  // K-steps for R <= FIRST_MAX_R
    constexpr int MAXNB = NBM;  // 16-channel output blocks this instance handles at most
    extern __shared__ __align__(16) unsigned char lds_raw[];
    const int LH = (a.th - 1) * a.stride + a.R, LW = (FT_W - 1) * a.stride + a.S;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lrow = lane & 15, lgrp = lane >> 4;
    // tiles in (image, row band, column) order, dealt to the XCDs in
    // contiguous runs: the halo rows a tile shares with the band above were
    // read through the same L2 shortly before
    const int ntx = (a.Wo + FT_W - 1) / FT_W, nty = (a.Ho + a.th - 1) / a.th;
    const int logical = xcd_remap(blockIdx.x, gridDim.x);
    const int n = logical / (ntx * nty), trem = logical - n * (ntx * nty);
    const int th0 = (trem / ntx) * a.th, tw0 = (trem % ntx) * FT_W;
    const int hi0 = th0 * a.stride - a.pad, wi0 = tw0 * a.stride - a.pad;
    const int KS = a.k_pad / KSTEP;

    // ---- stage the window: thread per pixel, PB pixels (all their channel
    // loads) in flight per thread, (row, col) advanced incrementally.  The
    // image's C planes are one buffer resource: a pixel outside the image
    // gets an offset past its size and the channels C..CP-1 lie past it too,
    // so both read as zero without a branch.
    {
        constexpr int PB = CP == 4 ? 5 : (CP == 8 ? 3 : 2);
        const int npix = LH * LW;
        const unsigned plane = (unsigned)a.H * (unsigned)a.W;
        auto stage = [&](auto u8tag) {
            constexpr bool U8 = decltype(u8tag)::value;
            constexpr unsigned EB = U8 ? 1 : 4;  // bytes per input element
            const void *img = U8 ? (const void *)(a.x8 + (size_t)n * a.C * plane) : (const void *)(a.x + (size_t)n * a.C * plane);
            const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc((void *)img, (short)0, (int)(a.C * plane * EB), 0x00020000);
            int lr = tid / LW, lc = tid % LW;
            const int dlr = 256 / LW, dlc = 256 % LW;
            for (int base = 0; base < npix; base += 256 * PB) {
                float v[PB][CP];
#pragma unroll
                for (int j = 0; j < PB; ++j) {
                    const int hi = hi0 + lr, wi = wi0 + lc;
                    const bool ok = base + j * 256 + tid < npix && (unsigned)hi < (unsigned)a.H && (unsigned)wi < (unsigned)a.W;
                    const unsigned off = ok ? (unsigned)(hi * a.W + wi) * EB : 0x80000000u;
#pragma unroll
                    for (int c = 0; c < CP; ++c) {
                        if constexpr (U8)
                            v[j][c] = __fdiv_rn((float)__builtin_amdgcn_raw_buffer_load_b8(rs, (int)off, (int)(c * plane), 0), 255.0f);
                        else
                            v[j][c] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, (int)off, (int)(c * plane * 4), 0));
                    }
                    lc += dlc; lr += dlr;
                    if (lc >= LW) { lc -= LW; ++lr; }
                }
#pragma unroll
                for (int j = 0; j < PB; ++j) {
                    const int p = base + j * 256 + tid;
                    if (p < npix) put_pixel<DT, CP>(lds_raw + (size_t)p * PIXB, v[j], a.in_inv_scale);
                }
            }
        };
        if (a.x8) stage(std::true_type{});
        else stage(std::false_type{});
    }

    // 16 zero bytes after the window: read units past row R or tap S read here
    const int zaddr = (LH * LW * PIXB + 15) & ~15;
    if (tid == 0) *reinterpret_cast<u32x4 *>(lds_raw + zaddr) = u32x4{0u, 0u, 0u, 0u};

    const int nb_count = (a.cout_p + 15) / 16;
    // ---- A fragments (weights) for every 16-channel block, kept in registers
    u32x4 aw[MAXNB][MAXKS][SPL];
#pragma unroll
    for (int nb = 0; nb < MAXNB; ++nb)
#pragma unroll
        for (int ks = 0; ks < MAXKS; ++ks)
#pragma unroll
            for (int j = 0; j < SPL; ++j) {
                aw[nb][ks][j] = u32x4{0u, 0u, 0u, 0u};
                if (nb < nb_count && nb * 16 + lrow < a.cout_p && ks < KS) {
                    const size_t off = ((size_t)(nb * 16 + lrow) * a.k_pad + ks * KSTEP + lgrp * KPL) * ES + j * 16;
                    aw[nb][ks][j] = gload16(a.w, off);
                }
            }
    __syncthreads();

    // per-lane epilogue constants, loaded once.  POOL: pixels are MFMA operand A,
    // so a lane holds one channel (nb*16 + lrow) of the four pixels of one 2x2
    // window and pools in registers.  Otherwise: weights are operand A and a
    // lane holds channels nb*16 + 4*lgrp + (0..3) of one pixel.  The output
    // scale (1 except FP8) folds into scale and bias for BF16 / FP32.
    const float ofold = DT == FP8 ? 1.0f : a.out_inv_scale;
    float bias4[MAXNB][4], scl4[MAXNB][4];
#pragma unroll
    for (int nb = 0; nb < MAXNB; ++nb)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int ch = POOL ? nb * 16 + lrow : nb * 16 + 4 * lgrp + i;
            const bool live = nb < nb_count && ch < a.cout_p;
            bias4[nb][i] = live ? a.bias[ch] * ofold : 0.0f;
            scl4[nb][i] = (DT == FP8 && live) ? a.wscale[ch] * a.in_scale : ofold;
        }
    const float opost = DT == FP8 ? a.out_inv_scale : 1.0f;
    const float lsl = act_slope(a.act, a.slope);
    // this image's output; offsets inside one image fit in 31 bits (checked at launch)
    const int Hy = POOL ? a.Ho >> 1 : a.Ho, Wy = POOL ? a.Wo >> 1 : a.Wo;
    unsigned char *yimg = reinterpret_cast<unsigned char *>(a.y) + (size_t)n * Hy * Wy * a.cout_p * ES;
    // the lane's part of its pixel position; the block's part is wave-uniform
    int lho, lwo;
    if (POOL) {
        lho = (lrow & 3) >> 1;
        lwo = 2 * (lrow >> 2) + (lrow & 1);
    } else {
        lho = 0;
        lwo = lrow;
    }
    const int lpx = (lho * LW + lwo) * a.stride * PIXB;
    // ---- the read units of this lane's K segments: a unit is live inside
    // filter row R and tap S.  Its LDS address for the block at byte offset
    // bpx is bpx * live + ua (one 24-bit multiply-add; LDS addresses are below
    // 2^24): the block's pixel plus the lane's pixel and unit offset where
    // live, the zero area where not.
    // the window's LDS address, so that a unit's address needs no further add
    const int lds_base = (int)(unsigned)(size_t)(const __attribute__((address_space(3))) unsigned char *)lds_raw;
    int ua[MAXKS][SPL][UPS], ulive[MAXKS][SPL][UPS];
#pragma unroll
    for (int ks = 0; ks < MAXKS; ++ks)
#pragma unroll
        for (int j = 0; j < SPL; ++j)
#pragma unroll
            for (int u = 0; u < UPS; ++u) {
                const int k0 = ks * KSTEP + lgrp * KPL + j * SEG;
                const int r = k0 / 16, rb = (k0 % 16) * ES + u * UB;  // byte within the run
                const int s = rb / PIXB;
                const bool live = ks < KS && r < a.R && s < a.S;
                ulive[ks][j][u] = live ? 1 : 0;
                ua[ks][j][u] = lds_base + (live ? lpx + (r * LW + s) * PIXB + rb % PIXB : zaddr);
            }
    auto read_b = [&](int bpx, u32x4 (&bf)[MAXKS][SPL]) {
#pragma unroll
        for (int ks = 0; ks < MAXKS; ++ks)
#pragma unroll
            for (int j = 0; j < SPL; ++j) {
                unsigned wv[4];
#pragma unroll
                for (int u = 0; u < UPS; ++u) {
                    const unsigned addr = mad_u24(bpx, ulive[ks][j][u], ua[ks][j][u]);
                    if constexpr (UB == 16) {
                        const u32x4 t = *(const __attribute__((address_space(3))) u32x4 *)(size_t)addr;
                        wv[0] = t.x; wv[1] = t.y; wv[2] = t.z; wv[3] = t.w;
                    } else if constexpr (UB == 8) {
                        const u32x2 t = *(const __attribute__((address_space(3))) u32x2 *)(size_t)addr;
                        wv[2 * u] = t.x; wv[2 * u + 1] = t.y;
                    } else {
                        wv[u] = *(const __attribute__((address_space(3))) unsigned *)(size_t)addr;
                    }
                }
                bf[ks][j] = u32x4{wv[0], wv[1], wv[2], wv[3]};
            }
    };

    if constexpr (POOL) {
        // Wave w takes, in every band of two output rows, the 16-pixel blocks
        // at columns 8w and 8w + 32 (four 2x2 windows each).  Lane (lgrp,
        // lrow) stores channel nb*16 + lrow of window lgrp: a wave-uniform
        // offset plus a lane constant, through a buffer resource the size of
        // the image's output, so that a window past the right edge (offset
        // moved past the size) is dropped without a branch.
        const __amdgpu_buffer_rsrc_t ry =
            __builtin_amdgcn_make_buffer_rsrc((void *)yimg, (short)0, (int)((size_t)Hy * Wy * a.cout_p * ES), 0x00020000);
        const unsigned lane_off = (unsigned)((lgrp * a.cout_p + lrow) * ES);
        const int bands = min(a.th >> 1, Hy - (th0 >> 1));
        for (int band = 0; band < bands; ++band) {
            const int hp = (th0 >> 1) + band;
#pragma unroll
            for (int hf = 0; hf < 2; ++hf) {
                const int bwo = 8 * (wave + 4 * hf);
                const int bpx = (2 * band * LW + bwo) * a.stride * PIXB;
                u32x4 bf[MAXKS][SPL];
                read_b(bpx, bf);
                const int wpb = (tw0 >> 1) + (bwo >> 1);
                const bool wok = wpb + lgrp < Wy;
#pragma unroll
                for (int nb = 0; nb < MAXNB; ++nb) {
                    if (nb >= nb_count) break;
                    // acc[i]: channel nb*16 + lrow of pixel 4*lgrp + i = quadrant i of window lgrp.
                    // The max is taken on the accumulators: scale > 0, bias, activation
                    // and rounding are monotone, so this equals pooling the outputs.
                    f4 acc = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                    for (int ks = 0; ks < MAXKS; ++ks) mma<DT>(acc, bf[ks], aw[nb][ks]);
                    const int col = nb * 16 + lrow;
                    const float mx = fmaxf(fmaxf(acc[0], acc[1]), fmaxf(acc[2], acc[3]));
                    const float o = activate_sel(mx * scl4[nb][0] + bias4[nb][0], lsl) * opost;
                    const bool ok = wok && col < a.cout_p;
                    const int soff = ((hp * Wy + wpb) * a.cout_p + nb * 16) * ES;
                    const int voff = ok ? (int)lane_off : (int)0x80000000u;
                    if constexpr (DT == F32) __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(o), ry, voff, soff, 0);
                    else if constexpr (DT == BF16) __builtin_amdgcn_raw_buffer_store_b16(f2bf(o), ry, voff, soff, 0);
                    else __builtin_amdgcn_raw_buffer_store_b8(f2e4m3(o), ry, voff, soff, 0);
                    if constexpr (AM) {
                        if (ok) {
                            const float w4[4] = {acc[0], acc[1], acc[2], acc[3]};
                            a.argmax[(size_t)n * Hy * Wy * a.cout_p + (hp * Wy + wpb + lgrp) * a.cout_p + col] =
                                window_argmax<DT>(w4, scl4[nb][0], bias4[nb][0], a.act, a.slope, opost);
                        }
                    }
                }
            }
        }
    } else {
        const int blocks = a.th * FT_W / 16;  // 16-pixel MFMA blocks per tile
        for (int b = wave; b < blocks; b += 4) {
            const int bho = b / (FT_W / 16), bwo = (b % (FT_W / 16)) * 16;
            const int bpx = (bho * LW + bwo) * a.stride * PIXB;
            u32x4 bf[MAXKS][SPL];
            read_b(bpx, bf);
            // K steps past k_pad multiply zero weights by zero data: no branches
#pragma unroll
            for (int nb = 0; nb < MAXNB; ++nb) {
                if (nb >= nb_count) break;
                // acc[i]: channel ch0 + i of this lane's pixel
                f4 acc = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int ks = 0; ks < MAXKS; ++ks) mma<DT>(acc, aw[nb][ks], bf[ks]);
                const int ch0 = nb * 16 + 4 * lgrp;
                float v[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) v[i] = activate_sel(acc[i] * scl4[nb][i] + bias4[nb][i], lsl) * opost;
                const int ho = th0 + bho, wo = tw0 + bwo + lrow;
                if (ho < a.Ho && ch0 < a.cout_p && wo < a.Wo) store4<DT>(yimg, (ho * a.Wo + wo) * a.cout_p + ch0, v);
            }
        }
    }
}

static size_t first_lds_for(int C, int R, int S, int stride, int th, int dt)
{
    const int LH = (th - 1) * stride + R, LW = (FT_W - 1) * stride + S;
    return (((size_t)LH * LW * first_cp(C) * esize(dt) + 15) & ~(size_t)15) + 16;  // window + 16 zero bytes
}
// 32 output rows per tile where that window stays small enough for the
// workgroups per CU the registers allow (fewer halo rows and per-tile set-up
// per output), else 16, else 8.
static int first_tile_h(int dt, int C, int R, int S, int stride)
{
    if (first_lds_for(C, R, S, stride, 32, dt) <= 20 * 1024) return 32;
    return first_lds_for(C, R, S, stride, 16, dt) <= FIRST_LDS_MAX ? 16 : 8;
}
size_t first_lds_bytes(int dt, int C, int R, int S, int stride)
{
    return first_lds_for(C, R, S, stride, first_tile_h(dt, C, R, S, stride), dt);
}

hipError_t launch_conv_first(int dt, const FirstArgs &a, hipStream_t s)
{
    FirstArgs b = a;
    b.th = first_tile_h(dt, a.C, a.R, a.S, a.stride);
    const size_t lds = first_lds_for(a.C, a.R, a.S, a.stride, b.th, dt);
    // one image's input planes (up to the padded channel count) and output
    // are addressed through buffer resources with 31-bit offsets
    if (lds > FIRST_LDS_MAX || a.R > FIRST_MAX_R || a.C > 16 || first_cp(a.C) * a.S > 16 || a.cout_p > FIRST_MAX_COUT ||
        a.stride > 2 || (a.cout_p & 3) || (size_t)a.Ho * a.Wo * a.cout_p * esize(dt) >= (1u << 31) ||
        (size_t)first_cp(a.C) * a.H * a.W * 4 >= (1u << 31))
        return hipErrorInvalidValue;
    const long nblk = (long)((a.Wo + FT_W - 1) / FT_W) * ((a.Ho + b.th - 1) / b.th) * a.batch;
    if (nblk >= (1L << 31)) return hipErrorInvalidValue;
    dim3 grid((unsigned)nblk);
#define DN_FIRST_CP(D, P, C, M)                                                                      \
    do {                                                                                             \
        if (b.cout_p <= 16) {                                                                        \
            allow_lds(conv_first<D, P, C, M, 1>, lds);                                               \
            hipLaunchKernelGGL((conv_first<D, P, C, M, 1>), grid, dim3(256), lds, s, b);             \
        } else {                                                                                     \
            allow_lds(conv_first<D, P, C, M>, lds);                                                  \
            hipLaunchKernelGGL((conv_first<D, P, C, M>), grid, dim3(256), lds, s, b);                \
        }                                                                                            \
    } while (0)
#define DN_FIRST_P(D, P, M)                                                                          \
    do {                                                                                             \
        const int cp = first_cp(a.C);                                                                \
        if (cp == 4) DN_FIRST_CP(D, P, 4, M);                                                        \
        else if (cp == 8) DN_FIRST_CP(D, P, 8, M);                                                   \
        else DN_FIRST_CP(D, P, 16, M);                                                               \
    } while (0)
#define DN_FIRST(D)                                                                                  \
    do {                                                                                             \
        if (b.pool) DN_FIRST_P(D, true, false);                                                      \
        else DN_FIRST_P(D, false, false);                                                            \
    } while (0)
    if (b.argmax && (!b.pool || dt == FP8)) return hipErrorInvalidValue;
    if (b.argmax) {  // the input-gradient pass (F32 / BF16)
        if (dt == F32) DN_FIRST_P(F32, true, true);
        else DN_FIRST_P(BF16, true, true);
        return hipGetLastError();
    }
    switch (dt) {
    case F32: DN_FIRST(F32); break;
    case BF16: DN_FIRST(BF16); break;
    case FP8: DN_FIRST(FP8); break;
    default: return hipErrorInvalidValue;
    }
#undef DN_FIRST
#undef DN_FIRST_P
#undef DN_FIRST_CP
    return hipGetLastError();
}

// Division by a runtime divisor d >= 1 without the integer-divide sequence:
// q = umulhi(n, ceil(2^32 / d)) is exact whenever n * d < 2^32 (true for
// every LDS index here).
struct FastDiv {
    unsigned m, d;
    __device__ explicit FastDiv(unsigned d_) : m(d_ > 1 ? 0xFFFFFFFFu / d_ + 1u : 0u), d(d_) {}
    __device__ __forceinline__ unsigned div(unsigned n) const { return d > 1 ? __umulhi(n, m) : n; }
};

// ---------------------------------------------------------------- halo kernel
// Small convolutions (K = R*S*Cin_p up to HALO_KMAX elements, Cout <= 64):
// one workgroup owns a TH x 32 output tile and every output channel.  Its
// input window (tile + filter halo) is read from HBM once into LDS, NHWC,
// each pixel padded to an odd number of 16-byte chunks so that the 16 lanes
// of a fragment read hit distinct banks; the weights [cout_p][K] sit in LDS
// as well (rows padded the same way).  The whole K loop then runs out of
// LDS: a lane's A-fragment segment is the 16-byte channel chunk (tap, c0) of
// its pixel, read directly from the window, so no input element is fetched
// once per filter tap as in the gathered implicit GEMM.

constexpr int HT_W = 32;
constexpr int HALO_KMAX_BYTES = 1280;  // K * element size (the offset table holds 20 MFMA K-steps)

int halo_lds_bytes(int dt, const ConvArgs &a, int th)
{
    const int ES = esize(dt), SEG = seg_el(dt);
    const int kstep = 4 * (dt == FP8 ? 32 : (dt == BF16 ? 8 : 4));
    const int K = a.R * a.S * a.cin_p;
    const int ku = (K + kstep - 1) / kstep * kstep;
    const int cps = a.cin_p / SEG, pst = cps | 1;
    const int wch = ku * ES / 16, wst = wch | 1;
    const int lh = (th - 1) * a.stride + a.R, lw = (HT_W - 1) * a.stride + a.S;
    const int coutp = (a.cout_p + 15) / 16 * 16;
    return (lh * lw * pst + coutp * wst + 1) * 16;  // window, weights, one zero chunk
}

constexpr int HALO_LDS_MAX = 96 * 1024;

bool halo_ok(int dt, const ConvArgs &a)
{
    return kblock_ch(dt, a.cin_p, a.R * a.S) == a.cin_p && a.R * a.S * a.cin_p * esize(dt) <= HALO_KMAX_BYTES &&
           a.cout_p <= 64 && a.stride <= 2 && (size_t)a.Ho * a.Wo * a.cout_p < (1u << 31) &&
           (size_t)a.H * a.W * a.cin_p * esize(dt) < (1u << 31) &&
           halo_lds_bytes(dt, a, 8) <= HALO_LDS_MAX;
}


// AM (with POOL): also store each window's argmax code (a.argmax).
template <int DT, bool POOL, int TH, int NB, bool AM = false>
__global__ void __launch_bounds__(256) conv_halo(ConvArgs a)
{
    constexpr int ES = esize(DT), SEG = seg_el(DT);
    constexpr int SPL = Tr<DT>::SPL;
    constexpr int KPL = 4 * SPL * SEG / 4;                 // K elements per lane per MFMA step
    constexpr int KSTEP = 4 * KPL;
    constexpr int BLOCKS = TH * HT_W / 16, NBW = BLOCKS / 4;  // MFMA blocks per tile / per wave
    constexpr int MAXNB = NB;                                 // 16-channel output blocks
    static_assert(KPL == SPL * SEG, "lane K chunk");
    extern __shared__ __align__(16) unsigned char halo_raw[];
    u32x4 *win = reinterpret_cast<u32x4 *>(halo_raw);

    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lrow = lane & 15, lgrp = lane >> 4;
    const int n = blockIdx.z, th0 = blockIdx.y * TH, tw0 = blockIdx.x * HT_W;
    const int K = a.R * a.S * a.cin_p;
    const int KS = (K + KSTEP - 1) / KSTEP;
    const int cps = a.cin_p / SEG, pst = cps | 1;
    const int wch = KS * KSTEP * ES / 16, wst = wch | 1;
    const int LH = (TH - 1) * a.stride + a.R, LW = (HT_W - 1) * a.stride + a.S;
    u32x4 *wlds = win + LH * LW * pst;
    constexpr int nb_count = NB;
    const u32x4 z4 = {0u, 0u, 0u, 0u};
    const int zchunk = LH * LW * pst + NB * 16 * wst;  // reads past K land on this zero chunk
    if (tid == 0) win[zchunk] = z4;

    // ---- input window -> LDS (8 loads in flight per thread)
    {
        const int hi0 = th0 * a.stride - a.pad, wi0 = tw0 * a.stride - a.pad;
        const int tot = LH * LW * cps;
        const FastDiv by_cps(cps), by_lw(LW);
        const unsigned char *ximg = reinterpret_cast<const unsigned char *>(a.x) + (size_t)n * a.H * a.W * a.cin_p * ES;
        for (int base = 0; base < tot; base += 256 * 8) {
            u32x4 v[8];
            int dst[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int e = base + j * 256 + tid;
                const int px = by_cps.div(e), ch = e - px * cps;
                const int lr = by_lw.div(px), lc = px - lr * LW;
                const int hi = hi0 + lr, wi = wi0 + lc;
                const bool ok = e < tot && (unsigned)hi < (unsigned)a.H && (unsigned)wi < (unsigned)a.W;
                const unsigned off = ok ? (unsigned)(((hi * a.W + wi) * a.cin_p + ch * SEG) * ES) : 0u;
                v[j] = ok ? gload16(ximg, off) : z4;
                dst[j] = e < tot ? px * pst + ch : -1;
            }
#pragma unroll
            for (int j = 0; j < 8; ++j)
                if (dst[j] >= 0) win[dst[j]] = v[j];
        }
        // weights: rows [cout_p][KS*KSTEP] (K beyond k_pad reads as zero)
        const int wtot = nb_count * 16 * wch;
        const FastDiv by_wch(wch);
        for (int e = tid; e < wtot; e += 256) {
            const int row = by_wch.div(e), ch = e - row * wch;
            const bool ok = row < a.cout_p && (ch + 1) * 16 <= a.k_pad * ES;
            wlds[row * wst + ch] = ok ? gload16(a.w, (size_t)row * a.k_pad * ES + ch * 16) : z4;
        }
    }
    __syncthreads();

    // ---- window offsets (in chunks) of every 16-byte K segment, -1 beyond K:
    // table[(ks*4 + lane group)*SPL + j], one division per entry per workgroup
    __shared__ int toff_tab[20 * 4 * 2];
    for (int e = tid; e < KS * 4 * SPL; e += 256) {
        const int j = e % SPL, g = (e / SPL) % 4, ks = e / (4 * SPL);
        const int k = ks * KSTEP + g * KPL + j * SEG;
        int o = -1;
        if (k < K) {
            const int tap = k / a.cin_p, c0 = k - tap * a.cin_p;
            const int r = tap / a.S, sx = tap - r * a.S;
            o = (r * LW + sx) * pst + c0 / SEG;
        }
        toff_tab[e] = o;
    }
    __syncthreads();

    // ---- this wave's blocks: pixel of lane (A row) per block
    int pbase[NBW];
#pragma unroll
    for (int i = 0; i < NBW; ++i) {
        const int b = wave + 4 * i;
        int hl, wl;
        if (POOL) {
            const int rp = b / (HT_W / 8), wg = b % (HT_W / 8);
            hl = 2 * rp + ((lrow >> 1) & 1);
            wl = 2 * (wg * 4 + (lrow >> 2)) + (lrow & 1);
        } else {
            hl = b / (HT_W / 16);
            wl = (b % (HT_W / 16)) * 16 + lrow;
        }
        pbase[i] = (hl * a.stride * LW + wl * a.stride) * pst;
    }

    f4 acc[NBW][MAXNB];
#pragma unroll
    for (int i = 0; i < NBW; ++i)
#pragma unroll
        for (int j = 0; j < MAXNB; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};

    for (int ks = 0; ks < KS; ++ks) {
        int toff[SPL];
#pragma unroll
        for (int j = 0; j < SPL; ++j) toff[j] = toff_tab[(ks * 4 + lgrp) * SPL + j];
        u32x4 bfr[MAXNB][SPL];
#pragma unroll
        for (int nb = 0; nb < MAXNB; ++nb)
#pragma unroll
            for (int j = 0; j < SPL; ++j)
                bfr[nb][j] = nb < nb_count ? wlds[(nb * 16 + lrow) * wst + (ks * KSTEP + lgrp * KPL + j * SEG) / SEG] : z4;
#pragma unroll
        for (int i = 0; i < NBW; ++i) {
            u32x4 af[SPL];
#pragma unroll
            for (int j = 0; j < SPL; ++j) af[j] = win[toff[j] >= 0 ? pbase[i] + toff[j] : zchunk];
#pragma unroll
            for (int nb = 0; nb < MAXNB; ++nb)
                if (nb < nb_count) mma<DT>(acc[i][nb], af, bfr[nb]);
        }
    }

    // ---- epilogue: bias, activation, [residual], [2x2 max], round, NHWC store
    // (offsets inside one image fit in 32 bits: checked by halo_ok)
    const int Hp = a.Ho >> 1, Wp = a.Wo >> 1;
    const size_t img = POOL ? (size_t)Hp * Wp * a.cout_p : (size_t)a.Ho * a.Wo * a.cout_p;
    unsigned char *yimg = reinterpret_cast<unsigned char *>(a.y) + (size_t)n * img * ES;
    const unsigned char *rimg = a.res ? reinterpret_cast<const unsigned char *>(a.res) + (size_t)n * img * ES : nullptr;
#pragma unroll
    for (int nb = 0; nb < MAXNB; ++nb) {
        if (nb >= nb_count) break;
        const int col = nb * 16 + lrow;
        if (col >= a.cout_p) continue;
        const float bias = a.bias[col];
        const float scl = (DT == FP8) ? a.wscale[col] * a.in_scale : 1.0f;
#pragma unroll
        for (int i = 0; i < NBW; ++i) {
            const int b = wave + 4 * i;
            if (POOL) {
                // a lane's four rows are one 2x2 window: pool the accumulators
                // (scale > 0; bias, activation and rounding are monotone)
                const float mx = fmaxf(fmaxf(acc[i][nb][0], acc[i][nb][1]), fmaxf(acc[i][nb][2], acc[i][nb][3]));
                const float o = activate(mx * scl + bias, a.act, a.slope) * a.out_inv_scale;
                const int rp = b / (HT_W / 8), wg = b % (HT_W / 8);
                const int hp = (th0 >> 1) + rp, wp = (tw0 >> 1) + wg * 4 + lgrp;
                if (hp < Hp && wp < Wp) {
                    store_el<DT>(yimg, (hp * Wp + wp) * a.cout_p + col, o);
                    if constexpr (AM) {
                        const float w4[4] = {acc[i][nb][0], acc[i][nb][1], acc[i][nb][2], acc[i][nb][3]};
                        a.argmax[(size_t)n * img + (hp * Wp + wp) * a.cout_p + col] = window_argmax<DT>(w4, scl, bias, a.act, a.slope, a.out_inv_scale);
                    }
                }
            } else {
                float v[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) v[q] = activate(acc[i][nb][q] * scl + bias, a.act, a.slope);
                const int ho = th0 + b / (HT_W / 16);
                if (ho < a.Ho) {
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int wo = tw0 + (b % (HT_W / 16)) * 16 + 4 * lgrp + q;
                        if (wo >= a.Wo) continue;
                        const int o = (ho * a.Wo + wo) * a.cout_p + col;
                        float r = v[q];
                        if (rimg) r += load_el<DT>(rimg, o) * a.res_scale;
                        store_el<DT>(yimg, o, r * a.out_inv_scale);
                    }
                }
            }
        }
    }
}

template <int DT, bool POOL, int TH, bool AM = false>
static hipError_t go_halo(const ConvArgs &a, dim3 grid, size_t lds, hipStream_t s)
{
    switch ((a.cout_p + 15) / 16) {
    case 1: allow_lds(conv_halo<DT, POOL, TH, 1, AM>, lds); hipLaunchKernelGGL((conv_halo<DT, POOL, TH, 1, AM>), grid, dim3(256), lds, s, a); break;
    case 2: allow_lds(conv_halo<DT, POOL, TH, 2, AM>, lds); hipLaunchKernelGGL((conv_halo<DT, POOL, TH, 2, AM>), grid, dim3(256), lds, s, a); break;
    case 3: allow_lds(conv_halo<DT, POOL, TH, 3, AM>, lds); hipLaunchKernelGGL((conv_halo<DT, POOL, TH, 3, AM>), grid, dim3(256), lds, s, a); break;
    case 4: allow_lds(conv_halo<DT, POOL, TH, 4, AM>, lds); hipLaunchKernelGGL((conv_halo<DT, POOL, TH, 4, AM>), grid, dim3(256), lds, s, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int DT>
static hipError_t go_halo_dt(const ConvArgs &a, int th, dim3 grid, size_t lds, hipStream_t s)
{
    if constexpr (DT != FP8) {
        if (a.pool && a.argmax)  // the input-gradient pass
            return th == 16 ? go_halo<DT, true, 16, true>(a, grid, lds, s) : go_halo<DT, true, 8, true>(a, grid, lds, s);
    }
    if (th == 16) return a.pool ? go_halo<DT, true, 16>(a, grid, lds, s) : go_halo<DT, false, 16>(a, grid, lds, s);
    return a.pool ? go_halo<DT, true, 8>(a, grid, lds, s) : go_halo<DT, false, 8>(a, grid, lds, s);
}

hipError_t launch_conv_halo(int dt, const ConvArgs &a, hipStream_t s)
{
    if (!halo_ok(dt, a)) return hipErrorInvalidValue;
    // 16-row tiles when two workgroups still fit in a CU's LDS, else 8 rows
    const int th = halo_lds_bytes(dt, a, 16) <= 80 * 1024 ? 16 : 8;
    dim3 grid((a.Wo + HT_W - 1) / HT_W, (a.Ho + th - 1) / th, a.batch);
    const size_t lds = halo_lds_bytes(dt, a, th);
    switch (dt) {
    case F32: return go_halo_dt<F32>(a, th, grid, lds, s);
    case BF16: return go_halo_dt<BF16>(a, th, grid, lds, s);
    case FP8: return go_halo_dt<FP8>(a, th, grid, lds, s);
    default: return hipErrorInvalidValue;
    }
}

// ---------------------------------------------------------------- persistent halo kernel
// The halo kernel's operation and reduction order (every output element is one
// 16x16 MFMA chain over the same K steps, in order, with the same K subset per
// lane as the GEMM tiles), restructured so that loads overlap the products:
//   * two workgroups per CU each loop over TH x 32 output tiles (every
//     output channel);
//   * each wave keeps the weights of its output channels (NBP 16-channel
//     blocks of NG groups) in registers for the whole run (no per-tile weight
//     staging) and owns a part of each tile's 16-pixel MFMA blocks (NQ parts,
//     NG * NQ = 4 waves); one fragment read from LDS feeds one MFMA per
//     channel block;
//   * a block is 16 consecutive pixels of one output row, so the 16 lanes of
//     a fragment read hit 16 distinct LDS banks (odd chunk pitch per pixel);
//     a wave owns blocks in vertical pairs, so with a fused 2x2 pool each
//     window's four outputs sit in one lane's accumulators (rows r and r+1,
//     two neighbouring columns);
//   * input windows travel global -> LDS directly (buffer_load ... lds) into
//     NBUF buffers, so the windows of the next NBUF-1 tiles are in flight
//     while one is multiplied (one barrier per tile);
//   * tiles are dealt out in runs of consecutive tiles per XCD, so the halo
//     rows and columns that neighbouring tiles share are read through the
//     same L2.

// Output rows per tile: 16, or 8 for four 16-channel blocks (whose
// accumulators and weights would not leave room for 16 rows).
__host__ __device__ constexpr int h2_th(int nb) { return nb >= 4 ? 8 : 16; }
// K steps whose weights a wave keeps in registers (BF16 / FP32: 10, FP8: 5).
__host__ __device__ constexpr int h2_ksmax(int dt) { return dt == FP8 ? 5 : 10; }
constexpr int H2_MAXBLK = 16;  // 1 KB window blocks one wave transfers per tile (at most)

// Chunk pitch of a window pixel: odd (the 16 lanes of a fragment read, 16
// consecutive pixels, hit distinct banks) and at least one chunk longer than
// the pixel's channels (the padding chunk, loaded as zeros, is what K
// segments past K read).
__host__ __device__ constexpr int h2_pitch(int cps) { return (cps & 1) ? cps + 2 : cps + 1; }
// 16-channel blocks per wave: every block up to 3, two of four.
__host__ __device__ constexpr int h2_nbp(int nb) { return nb == 4 ? 2 : nb; }
// Tile row of block i of pixel part q (of nq): blocks come as (row pair, row
// in pair, column half), column half fastest; row pairs are dealt to the
// parts in turn.
__device__ __forceinline__ int h2_row(int q, int nq, int i) { return 2 * (q + nq * (i >> 2)) + ((i >> 1) & 1); }

// s_waitcnt vmcnt(n) for a run-time n in [0, 40] (larger n waits for 0).
template <int N> __device__ __forceinline__ void wait_vm_upto(int n)
{
    if constexpr (N > 0) {
        if (n == N) { wait_vm<N>(); return; }
        wait_vm_upto<N - 1>(n);
    } else {
        wait_vm<0>();
    }
}

template <int DT, bool POOL, int NB, bool AM = false>
__global__ void __launch_bounds__(256, 2) conv_halo2(ConvArgs a, int nbuf)
{
    constexpr int ES = esize(DT), SEG = seg_el(DT);
    constexpr int SPL = Tr<DT>::SPL;
    constexpr int KPL = SPL * SEG, KSTEP = 4 * KPL;
    constexpr int KSM = h2_ksmax(DT);
    constexpr int NBP = h2_nbp(NB), NG = NB / NBP, NQ = 4 / NG;
    constexpr int TH = h2_th(NB), BLOCKS = TH * HT_W / 16, BPW = BLOCKS / NQ;
    static_assert(NG * NBP == NB && (TH / 2) % NQ == 0, "wave split");
    extern __shared__ __align__(16) unsigned char halo_raw[];
    u32x4 *lds = reinterpret_cast<u32x4 *>(halo_raw);

    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wg = wave % NG, wq = wave / NG;  // channel group, pixel part
    const int lrow = lane & 15, lgrp = lane >> 4;
    const int K = a.R * a.S * a.cin_p;
    const int KS = (K + KSTEP - 1) / KSTEP;
    const int cps = a.cin_p / SEG, pst = h2_pitch(cps);
    const int LH = (TH - 1) * a.stride + a.R, LW = (HT_W - 1) * a.stride + a.S;
    const int npx = LH * LW;
    const int wslots = (npx * pst + 63) / 64 * 64, nblk = wslots / 64;  // 16-byte slots per buffer
    const int ntw = (a.Wo + HT_W - 1) / HT_W, nth = (a.Ho + TH - 1) / TH;
    const int per_img = ntw * nth, total = a.batch * per_img;
    const unsigned img_bytes = (unsigned)((size_t)a.H * a.W * a.cin_p * ES);
    const u32x4 z4 = {0u, 0u, 0u, 0u};

    // this workgroup's tiles: XCD (blockIdx % 8) owns a run of consecutive tiles
    const int xcd = blockIdx.x & 7, li = blockIdx.x >> 3, per_xcd = gridDim.x >> 3;
    const int run = (total + 7) / 8;
    const int t_end = min(total, (xcd + 1) * run);
    const int t0 = xcd * run + li;
    if (t0 >= t_end) return;  // whole workgroup
    const int my_tiles = (t_end - t0 + per_xcd - 1) / per_xcd;

    // window slots this wave transfers: blocks wave, wave + 4, ...; lane L
    // of a block fills slot 64*block + L = pixel * pst + chunk (chunks past
    // the pixel's channels are padding and load zeros)
    const int dw = nblk > wave ? (nblk - wave + 3) / 4 : 0;
    const FastDiv by_pst(pst), by_lw(LW);
    int s_lr[H2_MAXBLK], s_lc[H2_MAXBLK], s_off[H2_MAXBLK];
#pragma unroll
    for (int q = 0; q < H2_MAXBLK; ++q) {
        const int sl = (wave + 4 * q) * 64 + lane;
        const int px = by_pst.div(sl), ch = sl - px * pst;
        const int lr = by_lw.div(px), lc = px - lr * LW;
        const bool live = q < dw && ch < cps && px < npx;
        s_lr[q] = live ? lr : -(1 << 20);
        s_lc[q] = lc;
        s_off[q] = (lc * a.cin_p + ch * SEG) * ES;
    }
    auto issue = [&](int k) {  // the window of this workgroup's k-th tile into buffer k % nbuf
        const int tt = t0 + k * per_xcd;
        const int n = tt / per_img, rem = tt - n * per_img;
        const int hi0 = (rem / ntw) * TH * a.stride - a.pad, wi0 = (rem % ntw) * HT_W * a.stride - a.pad;
        i32x4 rs = make_rsrc(reinterpret_cast<const unsigned char *>(a.x) + (size_t)n * img_bytes, img_bytes);
        // wave-uniform by construction; keep it in scalar registers
        rs.x = __builtin_amdgcn_readfirstlane(rs.x);
        rs.y = __builtin_amdgcn_readfirstlane(rs.y);
        rs.z = __builtin_amdgcn_readfirstlane(rs.z);
        rs.w = __builtin_amdgcn_readfirstlane(rs.w);
        u32x4 *dst = lds + (k % nbuf) * wslots;
#pragma unroll
        for (int q = 0; q < H2_MAXBLK; ++q) {
            if (q >= dw) break;  // wave-uniform
            const int hi = hi0 + s_lr[q], wi = wi0 + s_lc[q];
            const bool ok = (unsigned)hi < (unsigned)a.H && (unsigned)wi < (unsigned)a.W;
            const unsigned off = ok ? (unsigned)((hi * a.W + wi0) * a.cin_p * ES + s_off[q]) : DN_OOB;
            dma16(rs, off, dst + (wave + 4 * q) * 64);
        }
    };
    // the first nbuf - 1 windows go out before anything else
    for (int k = 0; k < nbuf - 1 && k < my_tiles; ++k) issue(k);

    // weights of this wave's output channels, all K steps, in registers
    u32x4 wr[NBP][KSM][SPL];
#pragma unroll
    for (int nb = 0; nb < NBP; ++nb)
#pragma unroll
        for (int ks = 0; ks < KSM; ++ks)
#pragma unroll
            for (int j = 0; j < SPL; ++j) {
                const int ch = (wg * NBP + nb) * 16 + lrow;
                const int k = ks * KSTEP + lgrp * KPL + j * SEG;
                wr[nb][ks][j] = (ks < KS && ch < a.cout_p) ? gload16(a.w, ((size_t)ch * a.k_pad + k) * ES) : z4;
            }
    // byte offset, relative to the lane's pixel, of the 16-byte chunk that
    // holds this lane's K segment j of step ks; segments past K read the
    // pixel's own padding chunk (always zero)
    int toffb[KSM][SPL];
#pragma unroll
    for (int ks = 0; ks < KSM; ++ks)
#pragma unroll
        for (int j = 0; j < SPL; ++j) {
            const int k = ks * KSTEP + lgrp * KPL + j * SEG;
            int o = cps;
            if (k < K) {
                const int tap = k / a.cin_p, c0 = k - tap * a.cin_p;
                const int r = tap / a.S, sx = tap - r * a.S;
                o = (r * LW + sx) * pst + c0 / SEG;
            }
            toffb[ks][j] = o * 16;
        }
    // this wave's blocks: block i is tile row h2_row(wq, NQ, i), columns
    // 16 * (i & 1) + (0..15); lane lrow reads the A row of pixel lrow
    int pbb[BPW];
#pragma unroll
    for (int i = 0; i < BPW; ++i)
        pbb[i] = (h2_row(wq, NQ, i) * a.stride * LW + (16 * (i & 1) + lrow) * a.stride) * pst * 16;
    float bias[NBP], scl[NBP];
#pragma unroll
    for (int nb = 0; nb < NBP; ++nb) {
        const int col = (wg * NBP + nb) * 16 + lrow;
        bias[nb] = col < a.cout_p ? a.bias[col] : 0.0f;
        scl[nb] = (DT == FP8 && col < a.cout_p) ? a.wscale[col] * a.in_scale : 1.0f;
    }
    const int Hp = a.Ho >> 1, Wp = a.Wo >> 1;
    const size_t img = POOL ? (size_t)Hp * Wp * a.cout_p : (size_t)a.Ho * a.Wo * a.cout_p;
    const float lsl = act_slope(a.act, a.slope);

    for (int k = 0; k < my_tiles; ++k) {
        // this wave's transfers of tile k landed (loads complete in order; the
        // ones still allowed in flight are those of the tiles issued after it)
        wait_vm_upto<40>(min(nbuf - 2, my_tiles - 1 - k) * dw);
        // the barrier: every wave's transfers landed and every wave is done
        // with tile k - 1's buffer
        lds_barrier();
        if (k + nbuf - 1 < my_tiles) issue(k + nbuf - 1);
        const int t = t0 + k * per_xcd;
        const int n = t / per_img, rem = t - n * per_img;
        const int th0 = (rem / ntw) * TH, tw0 = (rem % ntw) * HT_W;

        f4 acc[BPW][NBP];
#pragma unroll
        for (int i = 0; i < BPW; ++i)
#pragma unroll
            for (int nb = 0; nb < NBP; ++nb) acc[i][nb] = f4{0.f, 0.f, 0.f, 0.f};
        const unsigned char *wbuf = halo_raw + (size_t)(k % nbuf) * wslots * 16;
        const unsigned char *blk[BPW];
#pragma unroll
        for (int i = 0; i < BPW; ++i) blk[i] = wbuf + pbb[i];
#pragma unroll
        for (int ks = 0; ks < KSM; ++ks) {
            if (ks < KS) {
                u32x4 af[BPW][SPL];
#pragma unroll
                for (int i = 0; i < BPW; ++i)
#pragma unroll
                    for (int j = 0; j < SPL; ++j) af[i][j] = *reinterpret_cast<const u32x4 *>(blk[i] + toffb[ks][j]);
#pragma unroll
                for (int i = 0; i < BPW; ++i)
#pragma unroll
                    for (int nb = 0; nb < NBP; ++nb) mma<DT>(acc[i][nb], af[i], wr[nb][ks]);
            }
        }

        // epilogue: bias, activation, [residual], [2x2 max], round, NHWC store
        unsigned char *yimg = reinterpret_cast<unsigned char *>(a.y) + (size_t)n * img * ES;
        const unsigned char *rimg = a.res ? reinterpret_cast<const unsigned char *>(a.res) + (size_t)n * img * ES : nullptr;
        const __amdgpu_buffer_rsrc_t ry = __builtin_amdgcn_make_buffer_rsrc((void *)yimg, (short)0, (int)(img * ES), 0x00020000);
#pragma unroll
        for (int nb = 0; nb < NBP; ++nb) {
            const int col = (wg * NBP + nb) * 16 + lrow;
            if (col >= a.cout_p) continue;
            if constexpr (POOL) {
                // blocks i (row 2k) and i + 2 (row 2k + 1) of the same column
                // half: lane column pairs (4*lgrp + 2j, + 1) are the windows
                // The store offset is a wave-uniform part (window row, the
                // block's first window) plus a lane part; a window past the
                // right edge gets an offset past the image's output, which
                // the buffer store drops.
#pragma unroll
                for (int i = 0; i < BPW; ++i) {
                    if (i & 2) continue;
                    const int hp = (th0 + h2_row(wq, NQ, i)) >> 1;
                    if (hp >= Hp) continue;
                    const int wpb = (tw0 + 16 * (i & 1)) >> 1;
                    const int soff = (hp * Wp + wpb) * a.cout_p * ES;
#pragma unroll
                    for (int j = 0; j < 2; ++j) {
                        const float w4[4] = {acc[i][nb][2 * j], acc[i][nb][2 * j + 1], acc[i + 2][nb][2 * j],
                                             acc[i + 2][nb][2 * j + 1]};
                        const float mx = fmaxf(fmaxf(w4[0], w4[1]), fmaxf(w4[2], w4[3]));
                        const float o = activate_sel(mx * scl[nb] + bias[nb], lsl) * a.out_inv_scale;
                        const int wp = wpb + 2 * lgrp + j;
                        const int voff = wp < Wp ? ((2 * lgrp + j) * a.cout_p + col) * ES : (int)DN_OOB;
                        if constexpr (DT == F32) __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(o), ry, voff, soff, 0);
                        else if constexpr (DT == BF16) __builtin_amdgcn_raw_buffer_store_b16(f2bf(o), ry, voff, soff, 0);
                        else __builtin_amdgcn_raw_buffer_store_b8(f2e4m3(o), ry, voff, soff, 0);
                        if constexpr (AM) {
                            if (wp < Wp)
                                a.argmax[(size_t)n * img + (hp * Wp + wp) * a.cout_p + col] =
                                    window_argmax<DT>(w4, scl[nb], bias[nb], a.act, a.slope, a.out_inv_scale);
                        }
                    }
                }
            } else {
#pragma unroll
                for (int i = 0; i < BPW; ++i) {
                    const int ho = th0 + h2_row(wq, NQ, i);
                    if (ho >= a.Ho) continue;
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int wo = tw0 + 16 * (i & 1) + 4 * lgrp + q;
                        if (wo >= a.Wo) continue;
                        const int o = (ho * a.Wo + wo) * a.cout_p + col;
                        float r = activate_sel(acc[i][nb][q] * scl[nb] + bias[nb], lsl);
                        if (rimg) r += load_el<DT>(rimg, o) * a.res_scale;
                        store_el<DT>(yimg, o, r * a.out_inv_scale);
                    }
                }
            }
        }
    }
}

// Window slots (16 bytes) of one LDS buffer of the persistent halo kernel.
static int halo2_wslots(int dt, const ConvArgs &a)
{
    const int cps = a.cin_p / seg_el(dt);
    const int th = h2_th((a.cout_p + 15) / 16);
    const int lh = (th - 1) * a.stride + a.R, lw = (HT_W - 1) * a.stride + a.S;
    return (lh * lw * h2_pitch(cps) + 63) / 64 * 64;
}

constexpr size_t H2_LDS_MAX = 76 * 1024;  // two workgroups per CU

// Window buffers: as many as fit (up to 4), at least 2.
static int halo2_nbuf(int dt, const ConvArgs &a)
{
    const size_t per = (size_t)halo2_wslots(dt, a) * 16;
    int nb = 4;
    while (nb > 2 && nb * per > H2_LDS_MAX) --nb;
    return nb;
}

bool halo2_ok(int dt, const ConvArgs &a)
{
    const int kstep = dt == FP8 ? 128 : (dt == BF16 ? 32 : 16);
    const int K = a.R * a.S * a.cin_p;
    const int ws = halo2_wslots(dt, a);
    const int nb = (a.cout_p + 15) / 16;
    return kblock_ch(dt, a.cin_p, a.R * a.S) == a.cin_p && nb <= 4 && nb != 3 && (K + kstep - 1) / kstep <= h2_ksmax(dt) &&
           a.stride <= 2 && (size_t)a.Ho * a.Wo * a.cout_p * esize(dt) < (1u << 31) &&
           (size_t)a.H * a.W * a.cin_p * esize(dt) < (1u << 31) && ws / 64 <= 4 * H2_MAXBLK &&
           2 * (size_t)ws * 16 <= H2_LDS_MAX;
}

template <int DT, bool POOL, bool AM>
static hipError_t go_halo2(const ConvArgs &a, int grid, int nbuf, size_t lds, hipStream_t s)
{
    switch ((a.cout_p + 15) / 16) {
    case 1: allow_lds(conv_halo2<DT, POOL, 1, AM>, lds); hipLaunchKernelGGL((conv_halo2<DT, POOL, 1, AM>), dim3(grid), dim3(256), lds, s, a, nbuf); break;
    case 2: allow_lds(conv_halo2<DT, POOL, 2, AM>, lds); hipLaunchKernelGGL((conv_halo2<DT, POOL, 2, AM>), dim3(grid), dim3(256), lds, s, a, nbuf); break;
    case 4: allow_lds(conv_halo2<DT, POOL, 4, AM>, lds); hipLaunchKernelGGL((conv_halo2<DT, POOL, 4, AM>), dim3(grid), dim3(256), lds, s, a, nbuf); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int DT>
static hipError_t go_halo2_dt(const ConvArgs &a, int grid, int nbuf, size_t lds, hipStream_t s)
{
    if constexpr (DT != FP8) {
        if (a.pool && a.argmax) return go_halo2<DT, true, true>(a, grid, nbuf, lds, s);
    }
    return a.pool ? go_halo2<DT, true, false>(a, grid, nbuf, lds, s) : go_halo2<DT, false, false>(a, grid, nbuf, lds, s);
}

hipError_t launch_conv_halo2(int dt, const ConvArgs &a, hipStream_t s)
{
    if (!halo2_ok(dt, a)) return hipErrorInvalidValue;
    const int th = h2_th((a.cout_p + 15) / 16);
    const long tiles = (long)a.batch * ((a.Ho + th - 1) / th) * ((a.Wo + HT_W - 1) / HT_W);
    const int nbuf = halo2_nbuf(dt, a);
    const size_t lds = (size_t)nbuf * halo2_wslots(dt, a) * 16;
    // two workgroups per CU, a multiple of 8 (the tile runs are per XCD)
    const long want = std::min<long>(tiles, 512L);
    const int grid = (int)std::max<long>(8, (want + 7) / 8 * 8);
    switch (dt) {
    case F32: return go_halo2_dt<F32>(a, grid, nbuf, lds, s);
    case BF16: return go_halo2_dt<BF16>(a, grid, nbuf, lds, s);
    case FP8: return go_halo2_dt<FP8>(a, grid, nbuf, lds, s);
    default: return hipErrorInvalidValue;
    }
}

// ---------------------------------------------------------------- dispatch

static const TileCfg kTiles[] = {
    {64, 64, 2, 2},    // 0
    {128, 64, 2, 2},   // 1
    {128, 128, 2, 2},  // 2
    {256, 128, 2, 2},  // 3
    {256, 256, 2, 4},  // 4
    {128, 256, 2, 4},  // 5
    {256, 16, 4, 1},   // 6
    {256, 32, 4, 1},   // 7
    {64, 128, 1, 4},   // 8
    {64, 32, 2, 2},    // 9
    {256, 256, 2, 2},  // 10: 4 waves of 128x128
    {192, 256, 1, 4},  // 11: 57 M-tiles x 4 for M = 64*169
    {128, 256, 1, 4},  // 12
    // LDS-DMA pipeline variants (bm, bn, waves_m, waves_n; stages in dispatch)
    {256, 128, 2, 2},  // 13: 3 stages
    {128, 128, 2, 2},  // 14: 4 stages
    {256, 256, 2, 4},  // 15: 2 stages
    {192, 256, 1, 4},  // 16: 2 stages
    {128, 256, 2, 4},  // 17: 3 stages
    {256, 128, 2, 4},  // 18: 3 stages, 8 waves
    // 64-byte K-tiles (FP32 / BF16; FP8 falls back to 128-byte tiles)
    {256, 256, 2, 4},  // 19: 4 stages, 8 waves
    {192, 256, 1, 4},  // 20: 4 stages
    {128, 256, 2, 4},  // 21: 4 stages, 8 waves
    {256, 128, 2, 2},  // 22: 4 stages
    // 31 x 8 = 248 tiles for M = 64*169, N = 1024 (one round on 256 CUs)
    {352, 128, 2, 4},  // 23: 2 stages, 8 waves
    {352, 128, 2, 2},  // 24: 2 stages, 4 waves
    {352, 128, 2, 8},  // 25: 2 stages, 16 waves (4 per SIMD)
    {256, 256, 2, 8},  // 26: 2 stages, 16 waves
    // 32x32x16 BF16 blocks (other dtypes run the same tile with 16x16 blocks)
    {384, 128, 4, 2, 32},  // 27: 29 x 8 = 232 tiles for M = 64*169; 2 stages, 8 waves of 96x64
    {384, 128, 4, 4, 32},  // 28: 2 stages, 16 waves of 96x32
    {256, 256, 2, 4, 32},  // 29: 2 stages, 8 waves of 128x64
    {256, 256, 4, 4, 32},  // 30: 2 stages, 16 waves of 64x64
    {256, 128, 4, 2, 32},  // 31: 3 stages, 8 waves of 64x64
    {128, 128, 2, 2, 32},  // 32: 4 stages, 4 waves of 64x64
    {352, 128, 11, 1, 32}, // 33: 2 stages, 11 waves of 32x128
    // 64-byte K-tiles, 4 stages (three K-tiles in flight)
    {352, 128, 2, 8},      // 34: 16 waves
    {384, 128, 4, 2, 32},  // 35: 8 waves of 96x64
    {384, 128, 4, 4, 32},  // 36: 16 waves of 96x32
    {256, 256, 4, 4, 32},  // 37: 16 waves of 64x64
    {352, 128, 11, 1, 32}, // 38: 11 waves of 32x128
    // half-height tiles sized so that two workgroups share a CU (LDS <= 80 KB):
    // the second workgroup computes while the first waits for its K-tile
    {176, 128, 1, 8},      // 39: 2 stages, 8 waves of 176x16
    {176, 128, 1, 4},      // 40: 2 stages, 4 waves of 176x32
    {192, 128, 2, 2, 32},  // 41: 2 stages, 4 waves of 96x64
    {192, 128, 2, 4, 32},  // 42: 2 stages, 8 waves of 96x32
    // small LDS-DMA tiles for small-M layers: deep pipelines in 48-64 KB, so
    // two or three workgroups share a CU and keep more K-tiles in flight
    {64, 64, 2, 2},        // 43: 4 stages, 4 waves of 32x32
    {64, 64, 2, 2},        // 44: 3 stages
    {128, 64, 2, 2},       // 45: 4 stages, 4 waves of 64x32
    {64, 128, 2, 2},       // 46: 4 stages, 4 waves of 32x64
    {64, 32, 2, 2},        // 47: 4 stages, 4 waves of 32x16
};

int tile_count() { return (int)(sizeof(kTiles) / sizeof(kTiles[0])); }
TileCfg tile_cfg(int i) { return kTiles[i]; }

size_t splitk_counters(int M, int cout_p)
{
    size_t most = 0;
    for (int i = 0; i < tile_count(); ++i) {
        const TileCfg t = kTiles[i];
        most = std::max(most, (size_t)((M + t.bm - 1) / t.bm) * ((cout_p + t.bn - 1) / t.bn));
    }
    return most;
}

template <int DT, int BM, int BN, int WM, int WN>
static hipError_t go(const ConvArgs &a, hipStream_t s)
{
    const int mt = (a.M + BM - 1) / BM, nt = (a.cout_p + BN - 1) / BN;
    dim3 grid(mt * nt, 1, a.splits);
    hipLaunchKernelGGL((conv_igemm<DT, BM, BN, WM, WN>), grid, dim3(64 * WM * WN), 0, s, a);
    return hipGetLastError();
}

template <int DT, int BM, int BN, int WM, int WN, int NS, int SPR = 8, int MF = 16>
static hipError_t go_dl(ConvArgs a, hipStream_t s)
{
    if constexpr (MF == 32 && DT != BF16) {
        return go_dl<DT, BM, BN, WM, WN, NS, SPR, 16>(a, s);  // 32x32 blocks: BF16 only
    } else {
        // buffer offsets are 32-bit: the LDS-DMA kernels need tensors below 2 GiB
        const size_t xb = (size_t)a.batch * a.H * a.W * a.cin_p * esize(DT);
        const size_t wb = (size_t)a.cout_p * a.k_pad * esize(DT);
        if (xb >= DN_OOB || wb >= DN_OOB) return go<DT, 128, 128, 2, 2>(a, s);  // register-staged path
        a.x_bytes = (unsigned)xb;
        a.w_bytes = (unsigned)wb;
        const int mt = (a.M + BM - 1) / BM, nt = (a.cout_p + BN - 1) / BN;
        dim3 grid(mt * nt, 1, a.splits);
        if constexpr (DT == FP8 && SPR == 4) {
            return go_dl<DT, BM, BN, WM, WN, NS == 4 ? 2 : NS, 8, MF>(a, s);  // FP8 K-steps need 128-byte tiles
        } else {
            hipLaunchKernelGGL((conv_igemm_dl<DT, BM, BN, WM, WN, NS, SPR, MF>), grid, dim3(64 * WM * WN), 0, s, a);
        }
        return hipGetLastError();
    }
}

template <int DT>
static hipError_t dispatch(int tile, const ConvArgs &a, hipStream_t s)
{
    switch (tile) {
    case 0: return go<DT, 64, 64, 2, 2>(a, s);
    case 1: return go<DT, 128, 64, 2, 2>(a, s);
    case 2: return go<DT, 128, 128, 2, 2>(a, s);
    case 3: return go<DT, 256, 128, 2, 2>(a, s);
    case 4: return go<DT, 256, 256, 2, 4>(a, s);
    case 5: return go<DT, 128, 256, 2, 4>(a, s);
    case 6: return go<DT, 256, 16, 4, 1>(a, s);
    case 7: return go<DT, 256, 32, 4, 1>(a, s);
    case 8: return go<DT, 64, 128, 1, 4>(a, s);
    case 9: return go<DT, 64, 32, 2, 2>(a, s);
    case 10: return go<DT, 256, 256, 2, 2>(a, s);
    case 11: return go<DT, 192, 256, 1, 4>(a, s);
    case 12: return go<DT, 128, 256, 1, 4>(a, s);
    case 13: return go_dl<DT, 256, 128, 2, 2, 3>(a, s);
    case 14: return go_dl<DT, 128, 128, 2, 2, 4>(a, s);
    case 15: return go_dl<DT, 256, 256, 2, 4, 2>(a, s);
    case 16: return go_dl<DT, 192, 256, 1, 4, 2>(a, s);
    case 17: return go_dl<DT, 128, 256, 2, 4, 3>(a, s);
    case 18: return go_dl<DT, 256, 128, 2, 4, 3>(a, s);
    case 19: return go_dl<DT, 256, 256, 2, 4, 4, 4>(a, s);
    case 20: return go_dl<DT, 192, 256, 1, 4, 4, 4>(a, s);
    case 21: return go_dl<DT, 128, 256, 2, 4, 4, 4>(a, s);
    case 22: return go_dl<DT, 256, 128, 2, 2, 4, 4>(a, s);
    case 23: return go_dl<DT, 352, 128, 2, 4, 2>(a, s);
    case 24: return go_dl<DT, 352, 128, 2, 2, 2>(a, s);
    case 25: return go_dl<DT, 352, 128, 2, 8, 2>(a, s);
    case 26: return go_dl<DT, 256, 256, 2, 8, 2>(a, s);
    case 27: return go_dl<DT, 384, 128, 4, 2, 2, 8, 32>(a, s);
    case 28: return go_dl<DT, 384, 128, 4, 4, 2, 8, 32>(a, s);
    case 29: return go_dl<DT, 256, 256, 2, 4, 2, 8, 32>(a, s);
    case 30: return go_dl<DT, 256, 256, 4, 4, 2, 8, 32>(a, s);
    case 31: return go_dl<DT, 256, 128, 4, 2, 3, 8, 32>(a, s);
    case 32: return go_dl<DT, 128, 128, 2, 2, 4, 8, 32>(a, s);
    case 33: return go_dl<DT, 352, 128, 11, 1, 2, 8, 32>(a, s);
    case 34: return go_dl<DT, 352, 128, 2, 8, 4, 4>(a, s);
    case 35: return go_dl<DT, 384, 128, 4, 2, 4, 4, 32>(a, s);
    case 36: return go_dl<DT, 384, 128, 4, 4, 4, 4, 32>(a, s);
    case 37: return go_dl<DT, 256, 256, 4, 4, 4, 4, 32>(a, s);
    case 38: return go_dl<DT, 352, 128, 11, 1, 4, 4, 32>(a, s);
    case 39: return go_dl<DT, 176, 128, 1, 8, 2>(a, s);
    case 40: return go_dl<DT, 176, 128, 1, 4, 2>(a, s);
    case 41: return go_dl<DT, 192, 128, 2, 2, 2, 8, 32>(a, s);
    case 42: return go_dl<DT, 192, 128, 2, 4, 2, 8, 32>(a, s);
    case 43: return go_dl<DT, 64, 64, 2, 2, 4>(a, s);
    case 44: return go_dl<DT, 64, 64, 2, 2, 3>(a, s);
    case 45: return go_dl<DT, 128, 64, 2, 2, 4>(a, s);
    case 46: return go_dl<DT, 64, 128, 2, 2, 4>(a, s);
    case 47: return go_dl<DT, 64, 32, 2, 2, 4>(a, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_conv(int dt, int tile, const ConvArgs &a, hipStream_t s)
{
    if (a.tile_count && (a.splits > SPLITK_FUSED_MAX ||
                         (size_t)a.splits * a.M * a.cout_p * sizeof(float) > 0x7fffffffu))
        return hipErrorInvalidValue;  // beyond the in-kernel finish's loads
    if (tile == HALO_TILE) return a.splits > 1 ? hipErrorInvalidValue : launch_conv_halo(dt, a, s);
    if (tile == HALO2_TILE) return a.splits > 1 ? hipErrorInvalidValue : launch_conv_halo2(dt, a, s);
    switch (dt) {
    case F32: return dispatch<F32>(tile, a, s);
    case BF16: return dispatch<BF16>(tile, a, s);
    case FP8: return dispatch<FP8>(tile, a, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_splitk_reduce(int dt, const ConvArgs &a, hipStream_t s)
{
    if (a.cout_p & 3) return hipErrorInvalidValue;  // channel padding keeps cout_p a multiple of 4
    const size_t rows = a.pool ? (size_t)(a.M >> 2) : (size_t)a.M;
    const size_t n = rows * (size_t)(a.cout_p >> 2);
    const unsigned blocks = (unsigned)((n + 255) / 256);
    switch (dt) {
    case F32: hipLaunchKernelGGL(splitk_reduce<F32>, dim3(blocks), dim3(256), 0, s, a); break;
    case BF16: hipLaunchKernelGGL(splitk_reduce<BF16>, dim3(blocks), dim3(256), 0, s, a); break;
    case FP8: hipLaunchKernelGGL(splitk_reduce<FP8>, dim3(blocks), dim3(256), 0, s, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace dnk
