// Implicit-GEMM convolution for gfx950 (CDNA4) with a fused epilogue.
//
// GEMM view (M = batch*Ho*Wo output pixels, N = output channels,
// K = R*S*Cin_pad):  Y[m][j] = sum_k A[m][k] * B[k][j].
// A is never materialised: each 128-byte K-slice of an A row is gathered from
// the NHWC input as eight 16-byte segments, each lying inside one filter tap
// (r, s) because channels are padded to 16 bytes, and staged in LDS.  B is the
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
#include "dn_kernels.h"

namespace dnk {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef int i32x8 __attribute__((ext_vector_type(8)));

// ---------------------------------------------------------------- conversions

__device__ __forceinline__ uint16_t f2bf(float f)
{
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest even
    return (uint16_t)(u >> 16);
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

// ---------------------------------------------------------------- MFMA step

template <int DT> struct Tr;
// SPL: 16-byte segments per lane per MFMA K-step; KSPT: K-steps per 128-byte K-tile.
template <> struct Tr<F32> { static constexpr int SPL = 1, KSPT = 2; };
template <> struct Tr<BF16> { static constexpr int SPL = 1, KSPT = 2; };
template <> struct Tr<FP8> { static constexpr int SPL = 2, KSPT = 1; };

template <int DT> __device__ __forceinline__ void mma(f4 &acc, const uint4 *a, const uint4 *b)
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

__device__ __forceinline__ float activate(float v, int act, float slope)
{
    return (act == 1 && !(v > 0.0f)) ? v * slope : v;
}

// ---------------------------------------------------------------- the kernel

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

    __shared__ uint4 sA[2][BM * 8];
    __shared__ uint4 sB[2][BN * 8];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave % WM, wn = wave / WM;

    const int ntn = (a.cout_p + BN - 1) / BN;
    const int logical = xcd_remap(blockIdx.x, gridDim.x);
    const int m0 = (logical / ntn) * BM, n0 = (logical % ntn) * BN;

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

    const int nkt = a.k_pad / BKE;
    const int kt0 = blockIdx.z * a.ktiles_per_split;
    const int kt1 = min(nkt, kt0 + a.ktiles_per_split);
    const int RS = a.R * a.S;

    uint4 ra[AR], rb[BR];
    const uint4 zero4 = make_uint4(0, 0, 0, 0);

    auto gload = [&](int kt) {
        const int k0 = kt * BKE + sc * SEG;
        const int tap = k0 / a.cin_p;
        const int c0 = k0 - tap * a.cin_p;
        const int r = tap / a.S, s = tap - (tap / a.S) * a.S;
        const bool kv = tap < RS;
#pragma unroll
        for (int i = 0; i < AR; ++i) {
            const int hi = a_hi[i] + r, wi = a_wi[i] + s;
            const bool ok = kv && (unsigned)hi < (unsigned)a.H && (unsigned)wi < (unsigned)a.W;
            const int hh = ok ? hi : 0, ww = ok ? wi : 0;  // no address arithmetic on rejected taps
            const size_t off = ((size_t)(a_pix[i] + hh * a.W + ww) * a.cin_p + c0) * ES;
            ra[i] = ok ? *(const uint4 *)((const char *)a.x + off) : zero4;
        }
#pragma unroll
        for (int i = 0; i < BR; ++i) {
            const int row = rbase + i * RSTEP, n = n0 + row;
            const bool ok = row < BN && n < a.cout_p;
            const size_t off = ((size_t)n * a.k_pad + (size_t)kt * BKE + sc * SEG) * ES;
            rb[i] = ok ? *(const uint4 *)((const char *)a.w + off) : zero4;
        }
    };
    auto sstore = [&](int buf) {
#pragma unroll
        for (int i = 0; i < AR; ++i) {
            const int row = rbase + i * RSTEP;
            sA[buf][row * 8 + (sc ^ (row & 7))] = ra[i];
        }
#pragma unroll
        for (int i = 0; i < BR; ++i) {
            const int row = rbase + i * RSTEP;
            if (row < BN) sB[buf][row * 8 + (sc ^ (row & 7))] = rb[i];
        }
    };

    f4 acc[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};

    const int lrow = lane & 15, lgrp = lane >> 4;
    if (kt0 < kt1) {
        gload(kt0);
        sstore(0);
    }
    __syncthreads();
    for (int kt = kt0; kt < kt1; ++kt) {
        const int buf = (kt - kt0) & 1;
        if (kt + 1 < kt1) gload(kt + 1);
#pragma unroll
        for (int ks = 0; ks < KSPT; ++ks) {
            uint4 af[FM][SPL], bfr[FN][SPL];
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
        if (kt + 1 < kt1) sstore(buf ^ 1);
        __syncthreads();
    }

    // ---- epilogue.  MFMA 16x16 output layout: lane holds column (lane & 15)
    // and rows 4*(lane >> 4) + i, i = 0..3.
    const int colb = n0 + wn * WTN + lrow;
    const int rowb = m0 + wm * WTM + 4 * lgrp;
    if (a.splits > 1) {
        float *P = a.partial + (size_t)blockIdx.z * a.M * a.cout_p;
#pragma unroll
        for (int fn = 0; fn < FN; ++fn) {
            const int col = colb + fn * 16;
            if (col >= a.cout_p) continue;
#pragma unroll
            for (int fm = 0; fm < FM; ++fm)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int m = rowb + fm * 16 + i;
                    if (m < a.M) P[(size_t)m * a.cout_p + col] = acc[fm][fn][i];
                }
        }
        return;
    }
#pragma unroll
    for (int fn = 0; fn < FN; ++fn) {
        const int col = colb + fn * 16;
        if (col >= a.cout_p) continue;
        const float bias = a.bias[col];
        const float scl = (DT == FP8) ? a.wscale[col] * a.in_scale : 1.0f;
#pragma unroll
        for (int fm = 0; fm < FM; ++fm) {
            const int mb = rowb + fm * 16;
            if (mb >= a.M) continue;
            float v[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) v[i] = activate(acc[fm][fn][i] * scl + bias, a.act, a.slope);
            if (a.pool) {
                // rows mb..mb+3 are one 2x2 window (M is a multiple of 4 here)
                const float mx = fmaxf(fmaxf(v[0], v[1]), fmaxf(v[2], v[3]));
                store_el<DT>(a.y, (size_t)(mb >> 2) * a.cout_p + col, mx * a.out_inv_scale);
            } else {
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

// Split-K finish: sum the partials in split order, then the same epilogue.
template <int DT>
__global__ void __launch_bounds__(256) splitk_reduce(ConvArgs a)
{
    const size_t rows = a.pool ? (size_t)(a.M >> 2) : (size_t)a.M;
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= rows * a.cout_p) return;
    const int col = (int)(idx % a.cout_p);
    const size_t ro = idx / a.cout_p;
    const float bias = a.bias[col];
    const float scl = (DT == FP8) ? a.wscale[col] * a.in_scale : 1.0f;
    const size_t plane = (size_t)a.M * a.cout_p;
    auto total = [&](size_t m) {
        float s = 0.0f;
        for (int z = 0; z < a.splits; ++z) s += a.partial[z * plane + m * a.cout_p + col];
        return s;
    };
    if (a.pool) {
        float mx = -INFINITY;
        for (int q = 0; q < 4; ++q) mx = fmaxf(mx, activate(total(ro * 4 + q) * scl + bias, a.act, a.slope));
        store_el<DT>(a.y, ro * a.cout_p + col, mx * a.out_inv_scale);
    } else {
        float o = activate(total(ro) * scl + bias, a.act, a.slope);
        if (a.res) o += load_el<DT>(a.res, ro * a.cout_p + col) * a.res_scale;
        store_el<DT>(a.y, ro * a.cout_p + col, o * a.out_inv_scale);
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
};

int tile_count() { return (int)(sizeof(kTiles) / sizeof(kTiles[0])); }
TileCfg tile_cfg(int i) { return kTiles[i]; }

template <int DT, int BM, int BN, int WM, int WN>
static hipError_t go(const ConvArgs &a, hipStream_t s)
{
    const int mt = (a.M + BM - 1) / BM, nt = (a.cout_p + BN - 1) / BN;
    dim3 grid(mt * nt, 1, a.splits);
    hipLaunchKernelGGL((conv_igemm<DT, BM, BN, WM, WN>), grid, dim3(64 * WM * WN), 0, s, a);
    return hipGetLastError();
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
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_conv(int dt, int tile, const ConvArgs &a, hipStream_t s)
{
    switch (dt) {
    case F32: return dispatch<F32>(tile, a, s);
    case BF16: return dispatch<BF16>(tile, a, s);
    case FP8: return dispatch<FP8>(tile, a, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_splitk_reduce(int dt, const ConvArgs &a, hipStream_t s)
{
    const size_t rows = a.pool ? (size_t)(a.M >> 2) : (size_t)a.M;
    const size_t n = rows * a.cout_p;
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
