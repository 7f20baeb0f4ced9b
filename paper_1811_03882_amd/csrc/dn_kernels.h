// Internal interface between the runtime (runtime.cpp) and the HIP kernels
// (conv.hip, aux.hip) of the Darknet-style CNN forward library.  Not part of
// the public C ABI (include/dn.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace dnk {

enum { F32 = 0, BF16 = 1, FP8 = 2 };

__host__ __device__ constexpr int esize(int dt) { return dt == F32 ? 4 : dt == BF16 ? 2 : 1; }
// Elements per 16-byte segment: the unit of every global load and of the
// channel padding of NHWC activations.
__host__ __device__ constexpr int seg_el(int dt) { return 16 / esize(dt); }
__host__ __device__ constexpr int cpad(int dt, int c) { return (c + seg_el(dt) - 1) / seg_el(dt) * seg_el(dt); }
// K-tile of the implicit GEMM: 128 bytes of one A/B row (8 segments).
__host__ __device__ constexpr int bk_el(int dt) { return 128 / esize(dt); }
// Channels per K block of a packed weight row: k = (cb*R*S + r*S + s)*CB + ci
// with input channel c = cb*CB + ci.  When a layer's padded channels span
// more than one 128-byte K-tile and it has more than one tap, CB is one
// 128-byte block: every tap of one channel block comes before the next block,
// so the taps' re-reads of the same input pixels follow each other closely
// (L2 hits).  Otherwise CB = cin_p, the tap-major order k = (r*S + s)*cin_p + c.
__host__ __device__ constexpr int kblock_ch(int dt, int cin_p, int RS)
{
    return (RS > 1 && cin_p * esize(dt) > 128 && (cin_p * esize(dt)) % 128 == 0) ? 128 / esize(dt) : cin_p;
}

// Arguments of one implicit-GEMM convolution launch.
//   A[m][k] = x[n][ho*st - pad + r][wo*st - pad + s][c],  k = (r*S + s)*cin_p + c
//   B[k][j] = w_packed[j][k]   (packed [cout_p][k_pad], K contiguous)
//   m runs over (n, ho, wo), or over (n, ho/2, wo/2, dy, dx) when pool = 1 so
//   that each 2x2 pooling window is four consecutive rows.
struct ConvArgs {
    const void *x;
    const void *w;
    const float *bias;     // [cout_p] folded bias
    const float *wscale;   // [cout_p] FP8 per-channel weight scale (else unused)
    const void *res;       // residual, output-shaped NHWC, or nullptr
    void *y;               // NHWC output with cout_p channels
    float *partial;        // split-K scratch [splits][M][cout_p] FP32
    int batch, H, W, cin_p;
    int Ho, Wo, cout_p;
    int R, S, stride, pad;
    int k_pad;             // multiple of bk_el(dtype); K = R*S*cin_p <= k_pad
    int M;                 // batch*Ho*Wo
    int pool;              // fused 2x2 stride-2 max pool
    int act;               // 0 linear, 1 leaky
    float slope;
    float in_scale, res_scale, out_inv_scale;  // FP8 scales (1 otherwise)
    int splits, ktiles_per_split;
    unsigned x_bytes, w_bytes;  // buffer sizes (set by the launcher)
    // fused pool only, may be nullptr: per pooled output element, the index
    // 2*dy + dx of the first maximal stored value of its 2x2 window
    unsigned char *argmax;
    // split-K only, may be nullptr: one zeroed counter per output tile
    // (splitk_counters()); set, the last split to finish a tile runs the
    // split-K finish itself, else launch_splitk_reduce must follow
    unsigned *tile_count;
};

// First convolution of a network, reading the NCHW FP32 input directly.
// Weights packed in the order k = r*16 + s*CP + c, CP = first_cp(C), k_pad = first_kpad().
struct FirstArgs {
    const float *x;        // NCHW FP32 image batch
    const unsigned char *x8;  // or, when set, NCHW 8-bit pixels with value q / 255
    const void *w;
    const float *bias, *wscale;
    void *y;               // NHWC output (pooled when pool = 1)
    int batch, C, H, W, Ho, Wo, cout_p, k_pad;
    int R, S, stride, pad;
    int pool, act;
    float slope;
    float in_inv_scale;    // FP8: 1 / input scale (else 1)
    float in_scale, out_inv_scale;
    int th;                // output rows per tile (set by launch_conv_first)
    unsigned char *argmax; // pool = 1 only, may be nullptr: as ConvArgs::argmax
};
// Channels of one staged window pixel: C rounded up to 4, 8 or 16.
__host__ __device__ constexpr int first_cp(int C) { return C <= 4 ? 4 : (C <= 8 ? 8 : 16); }
// A conv qualifies for the first-layer kernel when C <= 16, first_cp(C)*S <= 16,
// R <= FIRST_MAX_R, cout <= FIRST_MAX_COUT and stride <= 2.
constexpr int FIRST_MAX_R = 4;
constexpr int FIRST_MAX_COUT = 64;
constexpr size_t FIRST_LDS_MAX = 160 * 1024;
int first_kpad(int dt, int R);
hipError_t launch_conv_first(int dt, const FirstArgs &a, hipStream_t s);
size_t first_lds_bytes(int dt, int C, int R, int S, int stride);

// Small-K convolutions can run the halo kernel instead of a GEMM tile:
// launch_conv(dt, HALO_TILE, ...) when halo_ok() (no split-K).
constexpr int HALO_TILE = 100;
bool halo_ok(int dt, const ConvArgs &a);
hipError_t launch_conv_halo(int dt, const ConvArgs &a, hipStream_t s);
// The persistent halo kernel (weights in registers, double-buffered windows,
// same reduction order): launch_conv(dt, HALO2_TILE, ...) when halo2_ok().
constexpr int HALO2_TILE = 101;
bool halo2_ok(int dt, const ConvArgs &a);
hipError_t launch_conv_halo2(int dt, const ConvArgs &a, hipStream_t s);

struct TileCfg { int bm, bn, wm, wn, mf; };  // mf: MFMA block side for BF16 (0 = 16)

int tile_count();
TileCfg tile_cfg(int i);
// Launch the conv (one GEMM launch; for splits > 1 it writes partials, and
// either the last split of each tile (tile_count set) or launch_splitk_reduce
// finishes the epilogue).
hipError_t launch_conv(int dt, int tile, const ConvArgs &a, hipStream_t s);
hipError_t launch_splitk_reduce(int dt, const ConvArgs &a, hipStream_t s);
// Most splits, and most partial bytes (offsets of its 16-byte loads), of a
// conv finishing in-kernel (ConvArgs::tile_count set).
constexpr int SPLITK_FUSED_MAX = 8;
// Counters ConvArgs::tile_count needs for an M x cout_p GEMM under any tile
// configuration (the most output tiles any of them makes).
size_t splitk_counters(int M, int cout_p);

// mode 0 packs k = (cb*R*S + r*S + s)*CB + ci; mode 1 packs k = r*16 + s*first_cp(cin) + c
// (first-layer kernel; cin_p unused); mode 2 packs the transposed, flipped
// weights of a forward conv's backward-data conv (cout, cin are the forward cin, cout).
hipError_t launch_fold_pack(int dt, int mode, const double *w, const double *bias, const double *mean,
                            const double *var, const double *gamma, const double *beta,
                            double eps, int has_bn, int cout, int cin, int R, int S, int cin_p,
                            int k_pad, int cout_p, void *wout, float *bout, float *sout,
                            hipStream_t s);
// x8 set: the source is NCHW 8-bit pixels with value q / 255 (x unused).
hipError_t launch_ingest(int dt, const float *x, int n, int c, int h, int w, int cp,
                         float inv_scale, void *y, hipStream_t s, const unsigned char *x8 = nullptr);
hipError_t launch_egress(int dt, const void *x, int n, int c, int h, int w, int cp, float scale,
                         float *y, hipStream_t s);
hipError_t launch_maxpool(int dt, const void *x, void *y, int n, int h, int w, int cp, int size,
                          int stride, int ho, int wo, hipStream_t s);
hipError_t launch_add(int dt, const void *a, float sa, const void *b, float sb, void *y,
                      float inv_sy, size_t count, hipStream_t s);
// amax of |x| over `count` FP32 values, max-combined into *out (caller zeroes *out).
hipError_t launch_amax(const float *x, size_t count, float *out, hipStream_t s);
hipError_t launch_zero_f32(float *p, size_t count, hipStream_t s);
// Backward pass to the input (backward.hip; F32 and BF16).
// dx = dy * (a > 0 ? 1 : slope) over `count` padded elements (dx may be dy).
hipError_t launch_leaky_bwd(int dt, const void *a, const void *dy, void *dx, float slope, size_t count, hipStream_t s);
// Max-pool gradient (first maximal element of each window); accumulate = 1 adds to dx.
// mask >= 0 also multiplies by the leaky gradient of x (1 where x > 0, else mask).
hipError_t launch_maxpool_bwd(int dt, const void *x, const void *dy, void *dx, int n, int h, int w, int cp, int size,
                              int stride, int ho, int wo, int accumulate, float mask, hipStream_t s);
// Gradient of a conv output through its fused 2x2/2 pool: dz[n][2i+dy][2j+dx][c] =
// dy[n][i][j][c] * (leaky gradient from the pooled output's sign, mask >= 0) where
// argmax[n][i][j][c] == 2*dy + dx, else 0; every element of dz is written.
hipError_t launch_unpool_bwd(int dt, const unsigned char *argmax, const void *pooled, const void *dy, void *dz, int n,
                             int hp, int wp, int cp, float mask, hipStream_t s);
// z[n][hz][wz][cp] = dy[n][i/stride][j/stride] where stride divides i and j, else 0.
hipError_t launch_dilate(int dt, const void *dy, void *z, int n, int ho, int wo, int cp, int hz, int wz, int stride,
                         hipStream_t s);
// Per image: m = mean |g|, then x = clamp(x + rate * g / m, 0, 1) (FP32 NCHW);
// scratch: ascend_scratch_bytes(n) bytes (m first, n doubles).
size_t ascend_scratch_bytes(int n);
hipError_t launch_ascend(float *x, const float *g, double *scratch, int n, size_t per_image, float rate, hipStream_t s);
// Region decode + per-class NMS (detect.hip).
constexpr int DETECT_MAX_ANCHORS = 16;
constexpr int DETECT_MAX_BOXES = 4096;  // H * W * A per image (sorted in LDS)
struct DetectArgs {
    const float *y;                       // [N][A*(5+C)][H][W] FP32
    float anchors[2 * DETECT_MAX_ANCHORS]; // (w, h) per anchor, in grid cells
    int N, A, C, H, W;
    float thresh, nms_thresh;
    int max_det;                          // kept boxes per image and class (capacity)
    float *score;                         // workspace [N][C][H*W*A]
    float *box;                           // workspace [N][H*W*A][4]
    float *dets;                          // [N][C][max_det][5]: score, x, y, w, h
    int *det_index;                       // [N][C][max_det]: box index (i*W + j)*A + a
    int *counts;                          // [N][C]
};
hipError_t launch_detect(const DetectArgs &a, hipStream_t s);
size_t detect_nms_lds(int boxes);
// Fixed device scratch of the allocation-free detection entry point: one
// file-scope array per GPU (detect.hip), DETECT_NOALLOC_BYTES long.
// detect_scratch() returns its device address on the current device (looked
// up once per device, then cached).
constexpr size_t DETECT_NOALLOC_BYTES = (size_t)16 << 20;
hipError_t detect_scratch(void **ptr);

// One Jacobi iteration of the Laplace equation on an [n][m] FP64 grid
// (jacobi.hip); max_change (device, may be NULL) receives the bits of the
// largest interior change.
hipError_t launch_jacobi_step(const double *u, double *v, int n, int m, unsigned long long *max_change, hipStream_t s);

// MFMA-only throughput probe (measurement): blocks x 256 threads, out holds
// blocks * 256 floats.
hipError_t launch_mfma_peak(int dt, float *out, int blocks, int iters, hipStream_t s);
double mfma_peak_flops_per_launch(int dt, int blocks, int iters);

}  // namespace dnk
