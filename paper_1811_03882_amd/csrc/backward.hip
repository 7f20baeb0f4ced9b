// Backward pass to the input image (the image-modification workload the
// paper ran beside detection, Sec. 5.1.1): the memory-bound pieces around the
// backward-data convolutions, which themselves run on the forward conv
// kernels with transposed, flipped weights (fold_pack mode 2).
//
//   leaky_bwd     dz = dy * (a > 0 ? 1 : slope), a = the layer's forward output
//                 (for 0 <= slope the sign of the output is the sign of the
//                 pre-activation, so the forward output decides the branch)
//   maxpool_bwd   each window hands its gradient to the first maximal input of
//                 the window in row-major order (the forward's strict compare);
//                 gather form: one thread per input segment walks the windows
//                 that contain it, so there are no atomics and the sum order
//                 is the window order; non-overlapping windows take the tiled
//                 form (one thread per window).  Either form can apply the
//                 leaky gradient of the layer that produced the pool's input
//                 (that layer's output is the pool's input, so its sign is at
//                 hand), saving a pass over the largest tensors
//   unpool_bwd    the gradient through a pool fused into its conv: the conv's
//                 epilogue stored each window's argmax code, so the full-size
//                 conv output never has to be kept
//   dilate        spreads a stride-s output gradient onto the stride-1 grid
//                 (zeros between), so a strided conv's backward-data is a
//                 stride-1 conv over the spread gradient
//   absmean       per-image mean of |g| (FP64 chunk sums in a fixed order)
//   ascend        x = clamp(x + rate * g / mean|g|, 0, 1), per image
//
// NHWC activations with 16-byte padded channels; one thread per 16-byte
// segment wherever the layout allows.
#include "dn_kernels.h"
#include "seg.h"

namespace dnk {

template <int DT>
__global__ void __launch_bounds__(256) leaky_bwd(const uint4 *a, const uint4 *dy, uint4 *dx, float slope, size_t nseg)
{
    constexpr int E = Seg<DT>::N;
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nseg) return;
    float fa[E], fg[E];
    Seg<DT>::dec(a[t], fa);
    Seg<DT>::dec(dy[t], fg);
#pragma unroll
    for (int e = 0; e < E; ++e) fg[e] = fa[e] > 0.0f ? fg[e] : fg[e] * slope;
    dx[t] = Seg<DT>::enc(fg);
}

// Leaky gradient factor of an element whose forward output is a (mask < 0: none).
__device__ __forceinline__ float leaky_factor(float a, float mask) { return (mask < 0.0f || a > 0.0f) ? 1.0f : mask; }

// Non-overlapping windows with no offset (stride == size <= 2): every input
// element lies in exactly one window, so one thread per (window, segment) finds the first
// maximum and writes the whole window's gradient: each element of x, dy and dx
// moves once.
template <int DT>
__global__ void __launch_bounds__(256) maxpool_bwd_tiled(const void *x, const void *dy, void *dx, int n, int h, int w,
                                                         int cp, int size, int ho, int wo, int accumulate, float mask)
{
    constexpr int E = Seg<DT>::N;
    const int nseg = cp / E;
    const size_t total = (size_t)n * ho * wo * nseg;
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= total) return;
    const int sg = (int)(t % nseg);
    const size_t p = t / nseg;
    const int oj = (int)(p % wo);
    const size_t q = p / wo;
    const int oi = (int)(q % ho);
    const int img = (int)(q / ho);
    const uint4 *X = (const uint4 *)x;
    // the window (size <= 2, no offset) stays in registers: x is read once
    float f[4][E], m[E];
    size_t o[4];
    bool in[4];
    int at[E];
#pragma unroll
    for (int e = 0; e < E; ++e) { m[e] = -INFINITY; at[e] = -1; }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int u = k >> 1, v = k & 1;
        const int yy = oi * size + u, xx = oj * size + v;
        in[k] = u < size && v < size && yy < h && xx < w;
        o[k] = (((size_t)img * h + yy) * w + xx) * nseg + sg;
        if (in[k]) {
            Seg<DT>::dec(X[o[k]], f[k]);
#pragma unroll
            for (int e = 0; e < E; ++e)
                if (f[k][e] > m[e]) { m[e] = f[k][e]; at[e] = k; }
        }
    }
    float d[E];
    Seg<DT>::dec(((const uint4 *)dy)[t], d);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (!in[k]) continue;
        float g[E];
#pragma unroll
        for (int e = 0; e < E; ++e) g[e] = at[e] == k ? d[e] * leaky_factor(f[k][e], mask) : 0.0f;
        if (accumulate) {
            float o2[E];
            Seg<DT>::dec(((const uint4 *)dx)[o[k]], o2);
#pragma unroll
            for (int e = 0; e < E; ++e) g[e] = o2[e] + g[e];
        }
        ((uint4 *)dx)[o[k]] = Seg<DT>::enc(g);
    }
}

template <int DT>
__global__ void __launch_bounds__(256) maxpool_bwd(const void *x, const void *dy, void *dx, int n, int h, int w,
                                                   int cp, int size, int stride, int ho, int wo, int accumulate,
                                                   float mask)
{
    constexpr int E = Seg<DT>::N;
    const int nseg = cp / E;
    const size_t total = (size_t)n * h * w * nseg;
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= total) return;
    const int sg = (int)(t % nseg);
    const size_t p = t / nseg;
    const int j = (int)(p % w);
    const size_t q = p / w;
    const int i = (int)(q % h);
    const int img = (int)(q / h);
    const int off = (size - 1) / 2;
    // windows (oi, oj) whose rows oi*stride-off .. +size-1 contain i (same for j)
    const int li = i + off - size + 1, lj = j + off - size + 1;
    const int oi0 = li <= 0 ? 0 : (li + stride - 1) / stride, oi1 = min(ho - 1, (i + off) / stride);
    const int oj0 = lj <= 0 ? 0 : (lj + stride - 1) / stride, oj1 = min(wo - 1, (j + off) / stride);
    const uint4 *X = (const uint4 *)x;
    float g[E];
#pragma unroll
    for (int e = 0; e < E; ++e) g[e] = 0.0f;
    for (int oi = oi0; oi <= oi1; ++oi) {
        for (int oj = oj0; oj <= oj1; ++oj) {
            float m[E];
            int at[E];
#pragma unroll
            for (int e = 0; e < E; ++e) { m[e] = -INFINITY; at[e] = -1; }
            for (int u = 0; u < size; ++u) {
                const int yy = oi * stride - off + u;
                if (yy < 0 || yy >= h) continue;
                for (int v = 0; v < size; ++v) {
                    const int xx = oj * stride - off + v;
                    if (xx < 0 || xx >= w) continue;
                    float f[E];
                    Seg<DT>::dec(X[(((size_t)img * h + yy) * w + xx) * nseg + sg], f);
#pragma unroll
                    for (int e = 0; e < E; ++e)
                        if (f[e] > m[e]) { m[e] = f[e]; at[e] = u * size + v; }
                }
            }
            const int mine = (i - (oi * stride - off)) * size + (j - (oj * stride - off));
            float d[E];
            Seg<DT>::dec(((const uint4 *)dy)[(((size_t)img * ho + oi) * wo + oj) * nseg + sg], d);
#pragma unroll
            for (int e = 0; e < E; ++e)
                if (at[e] == mine) g[e] += d[e];
        }
    }
    if (mask >= 0.0f) {
        float f[E];
        Seg<DT>::dec(X[t], f);
#pragma unroll
        for (int e = 0; e < E; ++e) g[e] *= leaky_factor(f[e], mask);
    }
    if (accumulate) {
        float o[E];
        Seg<DT>::dec(((const uint4 *)dx)[t], o);
#pragma unroll
        for (int e = 0; e < E; ++e) g[e] = o[e] + g[e];
    }
    ((uint4 *)dx)[t] = Seg<DT>::enc(g);
}

// One thread per pooled (pixel, 16-byte segment): E argmax codes, the pooled
// values (their sign is the sign of the window's maximal conv output) and the
// output gradient in, the four segments of the 2x2 window out.
template <int DT>
__global__ void __launch_bounds__(256) unpool_bwd(const unsigned char *argmax, const void *pooled, const void *dy,
                                                  void *dz, int n, int hp, int wp, int cp, float mask)
{
    constexpr int E = Seg<DT>::N;
    const int nseg = cp / E;
    const size_t total = (size_t)n * hp * wp * nseg;
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= total) return;
    const int sg = (int)(t % nseg);
    const size_t p = t / nseg;
    const int j = (int)(p % wp);
    const size_t q = p / wp;
    const int i = (int)(q % hp);
    const int img = (int)(q / hp);
    float a[E], d[E];
    Seg<DT>::dec(((const uint4 *)pooled)[t], a);
    Seg<DT>::dec(((const uint4 *)dy)[t], d);
    unsigned char am[E];
    if constexpr (E == 4) {
        const unsigned v = reinterpret_cast<const unsigned *>(argmax)[t];
#pragma unroll
        for (int e = 0; e < 4; ++e) am[e] = (unsigned char)(v >> (8 * e));
    } else {
        const uint2 v = reinterpret_cast<const uint2 *>(argmax)[t];
#pragma unroll
        for (int e = 0; e < 4; ++e) { am[e] = (unsigned char)(v.x >> (8 * e)); am[e + 4] = (unsigned char)(v.y >> (8 * e)); }
    }
#pragma unroll
    for (int e = 0; e < E; ++e) d[e] *= leaky_factor(a[e], mask);
    const int w = 2 * wp, h = 2 * hp;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        float g[E];
#pragma unroll
        for (int e = 0; e < E; ++e) g[e] = am[e] == k ? d[e] : 0.0f;
        const size_t o = (((size_t)img * h + 2 * i + (k >> 1)) * w + 2 * j + (k & 1)) * nseg + sg;
        ((uint4 *)dz)[o] = Seg<DT>::enc(g);
    }
}

__global__ void __launch_bounds__(256) dilate(const uint4 *dy, uint4 *z, int n, int ho, int wo, int nseg, int hz, int wz,
                                              int stride)
{
    const size_t total = (size_t)n * hz * wz * nseg;
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= total) return;
    const int sg = (int)(t % nseg);
    const size_t p = t / nseg;
    const int j = (int)(p % wz);
    const size_t q = p / wz;
    const int i = (int)(q % hz);
    const int img = (int)(q / hz);
    uint4 v = make_uint4(0u, 0u, 0u, 0u);
    if (i % stride == 0 && j % stride == 0 && i / stride < ho && j / stride < wo)
        v = dy[(((size_t)img * ho + i / stride) * wo + j / stride) * nseg + sg];
    z[t] = v;
}

// Per-image sum of |g| in two fixed-order stages: ABS_CHUNKS workgroups per
// image each reduce one contiguous chunk (FP64), then one wave per image adds
// the chunk sums in chunk order.
constexpr int ABS_CHUNKS = 64, ABS_THREADS = 256;

__global__ void __launch_bounds__(ABS_THREADS) absmean_chunks(const float *g, size_t per_image, double *part)
{
    __shared__ double red[ABS_THREADS];
    const float *gi = g + (size_t)blockIdx.y * per_image;
    double s = 0.0;
    if (per_image % 4 == 0) {  // 16-byte loads: chunks of whole float4s
        const size_t q = per_image / 4, chunk = (q + ABS_CHUNKS - 1) / ABS_CHUNKS;
        const size_t b = blockIdx.x * chunk, e = min(q, b + chunk);
        const float4 *g4 = reinterpret_cast<const float4 *>(gi);
        for (size_t k = b + threadIdx.x; k < e; k += ABS_THREADS) {
            const float4 v = g4[k];
            s += fabs((double)v.x);
            s += fabs((double)v.y);
            s += fabs((double)v.z);
            s += fabs((double)v.w);
        }
    } else {
        const size_t chunk = (per_image + ABS_CHUNKS - 1) / ABS_CHUNKS;
        const size_t b = blockIdx.x * chunk, e = min(per_image, b + chunk);
        for (size_t k = b + threadIdx.x; k < e; k += ABS_THREADS) s += fabs((double)gi[k]);
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int off = ABS_THREADS / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[(size_t)blockIdx.y * ABS_CHUNKS + blockIdx.x] = red[0];
}

__global__ void absmean_final(const double *part, size_t per_image, double *out)
{
    if (threadIdx.x != 0) return;
    double s = 0.0;
    for (int c = 0; c < ABS_CHUNKS; ++c) s += part[(size_t)blockIdx.x * ABS_CHUNKS + c];
    out[blockIdx.x] = s / (double)per_image;
}

__device__ __forceinline__ float ascend1(float x, float g, float step) { return fminf(fmaxf(x + step * g, 0.0f), 1.0f); }

// per_image % 4 == 0: one thread per float4 (a float4 never straddles two images)
__global__ void __launch_bounds__(256) ascend4(float4 *x, const float4 *g, const double *mean_abs, size_t per_image4,
                                               size_t total4, float rate)
{
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= total4) return;
    const double m = mean_abs[t / per_image4];
    const float step = m > 0.0 ? (float)((double)rate / m) : 0.0f;
    float4 v = x[t];
    const float4 d = g[t];
    v.x = ascend1(v.x, d.x, step);
    v.y = ascend1(v.y, d.y, step);
    v.z = ascend1(v.z, d.z, step);
    v.w = ascend1(v.w, d.w, step);
    x[t] = v;
}

__global__ void __launch_bounds__(256) ascend(float *x, const float *g, const double *mean_abs, size_t per_image,
                                              size_t total, float rate)
{
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= total) return;
    const double m = mean_abs[t / per_image];
    const float step = m > 0.0 ? (float)((double)rate / m) : 0.0f;
    x[t] = ascend1(x[t], g[t], step);
}

hipError_t launch_leaky_bwd(int dt, const void *a, const void *dy, void *dx, float slope, size_t count, hipStream_t s)
{
    const size_t nseg = count / seg_el(dt);
    if (nseg == 0) return hipSuccess;
    dim3 g((unsigned)((nseg + 255) / 256)), b(256);
    const uint4 *A = (const uint4 *)a, *D = (const uint4 *)dy;
    uint4 *X = (uint4 *)dx;
    switch (dt) {
    case F32: hipLaunchKernelGGL(leaky_bwd<F32>, g, b, 0, s, A, D, X, slope, nseg); break;
    case BF16: hipLaunchKernelGGL(leaky_bwd<BF16>, g, b, 0, s, A, D, X, slope, nseg); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_maxpool_bwd(int dt, const void *x, const void *dy, void *dx, int n, int h, int w, int cp, int size,
                              int stride, int ho, int wo, int accumulate, float mask, hipStream_t s)
{
    dim3 b(256);
    if (stride == size && (size - 1) / 2 == 0) {  // windows tile the input exactly (no offset)
        const size_t total = (size_t)n * ho * wo * (cp / seg_el(dt));
        if (total == 0) return hipSuccess;
        dim3 g((unsigned)((total + 255) / 256));
        switch (dt) {
        case F32: hipLaunchKernelGGL(maxpool_bwd_tiled<F32>, g, b, 0, s, x, dy, dx, n, h, w, cp, size, ho, wo, accumulate, mask); break;
        case BF16: hipLaunchKernelGGL(maxpool_bwd_tiled<BF16>, g, b, 0, s, x, dy, dx, n, h, w, cp, size, ho, wo, accumulate, mask); break;
        default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    const size_t total = (size_t)n * h * w * (cp / seg_el(dt));
    if (total == 0) return hipSuccess;
    dim3 g((unsigned)((total + 255) / 256));
    switch (dt) {
    case F32: hipLaunchKernelGGL(maxpool_bwd<F32>, g, b, 0, s, x, dy, dx, n, h, w, cp, size, stride, ho, wo, accumulate, mask); break;
    case BF16: hipLaunchKernelGGL(maxpool_bwd<BF16>, g, b, 0, s, x, dy, dx, n, h, w, cp, size, stride, ho, wo, accumulate, mask); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_unpool_bwd(int dt, const unsigned char *argmax, const void *pooled, const void *dy, void *dz, int n,
                             int hp, int wp, int cp, float mask, hipStream_t s)
{
    const size_t total = (size_t)n * hp * wp * (cp / seg_el(dt));
    if (total == 0) return hipSuccess;
    dim3 g((unsigned)((total + 255) / 256)), b(256);
    switch (dt) {
    case F32: hipLaunchKernelGGL(unpool_bwd<F32>, g, b, 0, s, argmax, pooled, dy, dz, n, hp, wp, cp, mask); break;
    case BF16: hipLaunchKernelGGL(unpool_bwd<BF16>, g, b, 0, s, argmax, pooled, dy, dz, n, hp, wp, cp, mask); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_dilate(int dt, const void *dy, void *z, int n, int ho, int wo, int cp, int hz, int wz, int stride,
                         hipStream_t s)
{
    const int nseg = cp / seg_el(dt);
    const size_t total = (size_t)n * hz * wz * nseg;
    if (total == 0) return hipSuccess;
    hipLaunchKernelGGL(dilate, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, (const uint4 *)dy, (uint4 *)z,
                       n, ho, wo, nseg, hz, wz, stride);
    return hipGetLastError();
}

size_t ascend_scratch_bytes(int n) { return (size_t)n * (ABS_CHUNKS + 1) * sizeof(double); }

hipError_t launch_ascend(float *x, const float *g, double *scratch, int n, size_t per_image, float rate, hipStream_t s)
{
    if (n <= 0 || per_image == 0) return hipSuccess;
    double *mean_abs = scratch, *part = scratch + n;
    hipLaunchKernelGGL(absmean_chunks, dim3(ABS_CHUNKS, n), dim3(ABS_THREADS), 0, s, g, per_image, part);
    hipLaunchKernelGGL(absmean_final, dim3(n), dim3(64), 0, s, part, per_image, mean_abs);
    const size_t total = (size_t)n * per_image;
    if (per_image % 4 == 0 && ((uintptr_t)x & 15) == 0 && ((uintptr_t)g & 15) == 0) {
        const size_t total4 = total / 4;
        hipLaunchKernelGGL(ascend4, dim3((unsigned)((total4 + 255) / 256)), dim3(256), 0, s, (float4 *)x,
                           (const float4 *)g, mean_abs, per_image / 4, total4, rate);
    } else {
        hipLaunchKernelGGL(ascend, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, x, g, mean_abs, per_image,
                           total, rate);
    }
    return hipGetLastError();
}

}  // namespace dnk
