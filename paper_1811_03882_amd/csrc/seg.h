// Element conversions and 16-byte segment codecs shared by the memory-bound
// kernels (aux.hip, backward.hip).  Internal to the library.
#pragma once

#include "dn_kernels.h"

namespace dnk {

// ---------------------------------------------------------------- conversions
// (same rounding as the conv epilogue: nearest even; FP8 saturates at +-448)

__device__ __forceinline__ uint16_t f2bf(float f)
{
    return __builtin_bit_cast(uint16_t, (__bf16)f);  // v_cvt_pk_bf16_f32: round to nearest even
}
__device__ __forceinline__ float bf2f(uint32_t h) { return __uint_as_float(h << 16); }
__device__ __forceinline__ uint32_t f2e4m3(float f)
{
    f = fminf(fmaxf(f, -448.0f), 448.0f);
    return (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(f, f, 0, false) & 0xFFu;
}
__device__ __forceinline__ float e4m32f(uint32_t b) { return __builtin_amdgcn_cvt_f32_fp8((int)b, 0); }

// Decode / encode one 16-byte segment (4, 8 or 16 elements) to/from floats.
template <int DT> struct Seg;
template <> struct Seg<F32> {
    static constexpr int N = 4;
    __device__ static void dec(uint4 u, float *f) { f[0] = __uint_as_float(u.x); f[1] = __uint_as_float(u.y); f[2] = __uint_as_float(u.z); f[3] = __uint_as_float(u.w); }
    __device__ static uint4 enc(const float *f) { return make_uint4(__float_as_uint(f[0]), __float_as_uint(f[1]), __float_as_uint(f[2]), __float_as_uint(f[3])); }
};
template <> struct Seg<BF16> {
    static constexpr int N = 8;
    __device__ static void dec(uint4 u, float *f)
    {
        const uint32_t w[4] = {u.x, u.y, u.z, u.w};
        for (int i = 0; i < 4; ++i) { f[2 * i] = bf2f(w[i] & 0xFFFFu); f[2 * i + 1] = bf2f(w[i] >> 16); }
    }
    __device__ static uint4 enc(const float *f)
    {
        uint32_t w[4];
        for (int i = 0; i < 4; ++i) w[i] = (uint32_t)f2bf(f[2 * i]) | ((uint32_t)f2bf(f[2 * i + 1]) << 16);
        return make_uint4(w[0], w[1], w[2], w[3]);
    }
};
template <> struct Seg<FP8> {
    static constexpr int N = 16;
    __device__ static void dec(uint4 u, float *f)
    {
        const uint32_t w[4] = {u.x, u.y, u.z, u.w};
        for (int i = 0; i < 4; ++i)
            for (int j = 0; j < 4; ++j) f[4 * i + j] = e4m32f((w[i] >> (8 * j)) & 0xFFu);
    }
    __device__ static uint4 enc(const float *f)
    {
        uint32_t w[4];
        for (int i = 0; i < 4; ++i)
            w[i] = f2e4m3(f[4 * i]) | (f2e4m3(f[4 * i + 1]) << 8) | (f2e4m3(f[4 * i + 2]) << 16) | (f2e4m3(f[4 * i + 3]) << 24);
        return make_uint4(w[0], w[1], w[2], w[3]);
    }
};

}  // namespace dnk
