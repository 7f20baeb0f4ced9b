// Detection post-processing of a region-layer output, on the device.
//
// The workload's detection program turns the last layer's output into boxes
// (Sec. 5.1.1).  The rule (a reading; the paper gives none): each grid cell
// holds A anchors x (5 + C) channels: tx, ty, tw, th, to, then C class
// logits.  Box centre ((j + sigmoid(tx)) / W, (i + sigmoid(ty)) / H), size
// (anchor_w * exp(tw) / W, anchor_h * exp(th) / H), class scores
// sigmoid(to) * softmax(logits).  Per image and class, candidates with
// score >= thresh are ranked by score (descending, ties by box index
// (i*W + j)*A + a) and kept greedily unless a kept box overlaps them with
// IoU > nms_thresh, at most max_det per class.
//
// Two kernels: decode (one thread per box, coalesced over the grid cells of
// one channel plane) writes every box and every class score to the
// workspace; nms (one workgroup per image and class) sorts the class's boxes
// in LDS with a bitonic network and runs the greedy suppression, one kept box
// per step, the whole workgroup testing the remaining candidates.
// Arithmetic is FP32 with contraction off, in the order the definition
// states, so threshold and overlap decisions are reproducible.
#include "dn_kernels.h"

#include <mutex>

#pragma clang fp contract(off)

namespace dnk {

__device__ __forceinline__ float sigm(float x) { return 1.0f / (1.0f + expf(-x)); }

__global__ void __launch_bounds__(256) detect_decode(DetectArgs a)
{
    const int HW = a.H * a.W, B = HW * a.A;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;  // (n, anchor, cell), cell fastest
    if (t >= a.N * B) return;
    const int n = t / B, r = t - n * B, anc = r / HW, cell = r - anc * HW;
    const int i = cell / a.W, j = cell - i * a.W;
    const int b = cell * a.A + anc;  // box index
    const float *p = a.y + ((size_t)n * a.A * (5 + a.C) + (size_t)anc * (5 + a.C)) * HW + cell;
    const float bx = ((float)j + sigm(p[0])) / (float)a.W;
    const float by = ((float)i + sigm(p[(size_t)HW])) / (float)a.H;
    const float bw = (a.anchors[2 * anc] * expf(p[2 * (size_t)HW])) / (float)a.W;
    const float bh = (a.anchors[2 * anc + 1] * expf(p[3 * (size_t)HW])) / (float)a.H;
    const float obj = sigm(p[4 * (size_t)HW]);
    float mx = -INFINITY;
    for (int k = 0; k < a.C; ++k) mx = fmaxf(mx, p[(size_t)(5 + k) * HW]);
    float sum = 0.0f;
    for (int k = 0; k < a.C; ++k) sum += expf(p[(size_t)(5 + k) * HW] - mx);
    float *sc = a.score + (size_t)n * a.C * B + b;
    for (int k = 0; k < a.C; ++k) sc[(size_t)k * B] = obj * (expf(p[(size_t)(5 + k) * HW] - mx) / sum);
    reinterpret_cast<float4 *>(a.box)[(size_t)n * B + b] = make_float4(bx, by, bw, bh);
}

__device__ __forceinline__ float box_iou(float4 p, float4 q)
{
    const float l1 = p.x - p.z / 2.0f, r1 = p.x + p.z / 2.0f, t1 = p.y - p.w / 2.0f, d1 = p.y + p.w / 2.0f;
    const float l2 = q.x - q.z / 2.0f, r2 = q.x + q.z / 2.0f, t2 = q.y - q.w / 2.0f, d2 = q.y + q.w / 2.0f;
    const float iw = fmaxf(0.0f, fminf(r1, r2) - fmaxf(l1, l2));
    const float ih = fmaxf(0.0f, fminf(d1, d2) - fmaxf(t1, t2));
    const float inter = iw * ih;
    const float uni = p.z * p.w + q.z * q.w - inter;
    return uni > 0.0f ? inter / uni : 0.0f;
}

// Sort key: score bits (scores are >= 0, so their bits order like the
// values) above the complemented box index, descending = score desc, index asc.
__global__ void __launch_bounds__(256) detect_nms(DetectArgs a)
{
    extern __shared__ __align__(16) unsigned char nms_raw[];
    const int B = a.H * a.W * a.A;
    int P = 1;
    while (P < B) P <<= 1;
    unsigned long long *key = reinterpret_cast<unsigned long long *>(nms_raw);   // [P]
    float4 *cbox = reinterpret_cast<float4 *>(nms_raw + (size_t)P * 8);         // [P]
    unsigned char *keep = nms_raw + (size_t)P * 24;                               // [P]
    __shared__ int ncand;
    const int n = blockIdx.x / a.C, k = blockIdx.x - (blockIdx.x / a.C) * a.C;
    const int tid = threadIdx.x;
    const float *sc = a.score + ((size_t)n * a.C + k) * B;
    if (tid == 0) ncand = 0;
    __syncthreads();
    int mine = 0;
    for (int e = tid; e < P; e += 256) {
        unsigned long long kv = 0ull;
        if (e < B) {
            const float s = sc[e];
            if (s >= a.thresh) {
                kv = ((unsigned long long)__float_as_uint(s) << 32) | (unsigned)(~(unsigned)e);
                ++mine;
            }
        }
        key[e] = kv;
    }
    atomicAdd(&ncand, mine);
    // bitonic sort, descending
    for (int size = 2; size <= P; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            __syncthreads();
            for (int e = tid; e < P / 2; e += 256) {
                const int lo = 2 * e - (e & (stride - 1));
                const int hi = lo + stride;
                const bool desc = (lo & size) == 0;
                const unsigned long long x = key[lo], y = key[hi];
                if ((x < y) == desc) {
                    key[lo] = y;
                    key[hi] = x;
                }
            }
        }
    }
    __syncthreads();
    const int m = ncand;
    const float4 *bx = reinterpret_cast<const float4 *>(a.box) + (size_t)n * B;
    for (int e = tid; e < m; e += 256) {
        cbox[e] = bx[~(unsigned)(key[e] & 0xFFFFFFFFull)];
        keep[e] = 1;
    }
    __syncthreads();
    const size_t obase = ((size_t)n * a.C + k) * a.max_det;
    int kept = 0;
    for (int i = 0; i < m && kept < a.max_det; ++i) {
        if (!keep[i]) continue;  // uniform: keep[] is only written before the barrier below
        const float4 bi = cbox[i];
        if (tid == 0) {
            const unsigned bidx = ~(unsigned)(key[i] & 0xFFFFFFFFull);
            float *d = a.dets + (obase + kept) * 5;
            d[0] = __uint_as_float((unsigned)(key[i] >> 32));
            d[1] = bi.x; d[2] = bi.y; d[3] = bi.z; d[4] = bi.w;
            a.det_index[obase + kept] = (int)bidx;
        }
        ++kept;
        for (int j = i + 1 + tid; j < m; j += 256)
            if (keep[j] && box_iou(bi, cbox[j]) > a.nms_thresh) keep[j] = 0;
        __syncthreads();
    }
    if (tid == 0) a.counts[(size_t)n * a.C + k] = kept;
}

size_t detect_nms_lds(int boxes)
{
    int P = 1;
    while (P < boxes) P <<= 1;
    return (size_t)P * 25;
}

// ---------------------------------------------------------------- fixed scratch
// The decoded scores and boxes of dn_detect_noalloc live here instead of in a
// caller workspace.  Each GPU the library runs on holds its own copy for the
// life of the process; calls on one GPU share it.  In host code the array's
// name is not a device address: its address is taken once per device with
// hipGetSymbolAddress (that device current) and only that address is used.
static __device__ __align__(256) unsigned char scratch[DETECT_NOALLOC_BYTES];

hipError_t detect_scratch(void **ptr)
{
    constexpr int MAX_DEVICES = 64;
    static std::mutex mu;
    static void *addr[MAX_DEVICES] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> g(mu);
    if (!addr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        addr[dev] = p;
    }
    *ptr = addr[dev];
    return hipSuccess;
}

hipError_t launch_detect(const DetectArgs &a, hipStream_t s)
{
    const int B = a.H * a.W * a.A;
    const long total = (long)a.N * B;
    hipLaunchKernelGGL(detect_decode, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, a);
    const size_t lds = detect_nms_lds(B);
    if (lds > 64 * 1024)
        (void)hipFuncSetAttribute((const void *)detect_nms, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(detect_nms, dim3((unsigned)(a.N * a.C)), dim3(256), lds, s, a);
    return hipGetLastError();
}

}  // namespace dnk
