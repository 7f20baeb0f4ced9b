/*
 * dn.h — C ABI of the MI355X (gfx950) Darknet-style CNN forward library.
 *
 * The operation is the forward pass of the convolutional network that the
 * paper offloads to the GPU (Darknet's detection and image-edit sample
 * programs, Sec. 5.1.1): convolution + bias + inference batch normalisation
 * + leaky rectifier, max pooling and residual (shortcut) layers.  The
 * paper's contribution, hoisting CPU<->GPU copies out of every loop that does
 * not define or use the data (Sec. 3.2), becomes the library's resident mode:
 * weights are uploaded once at load time, the input crosses once per forward,
 * every intermediate activation stays in a device arena, and the output
 * crosses once.  The per-layer mode copies each layer's input, weights and
 * output around its kernel, the naive per-loop offload that Sec. 3.2 removes.
 * Beside the forward: the backward pass to the input image and the image
 * ascent of the image-edit program (dn_input_gradient, dn_nightmare), the
 * detection post-processing (dn_detect) and the paper's second sample program,
 * Jacobi iteration for the Laplace equation (dn_jacobi).
 *
 * Conventions for every function:
 *   - returns dn_status (0 = DN_OK, negative = error); never throws or aborts;
 *     on failure dn_last_error() holds a message (thread-local).
 *   - "device pointer" = memory on the net's / the call's GPU (hipMalloc or a
 *     torch CUDA tensor); "host pointer" = CPU memory.  The caller owns every
 *     pointer it passes; the library keeps none of them beyond the call except
 *     the arena bound with dn_bind_arena (kept until rebind or destroy).
 *   - stream arguments are hipStream_t passed as void* (NULL = null stream).
 *     Enqueueing calls return without waiting; kernel faults surface at the
 *     caller's next synchronisation.
 *   - Activations on the device are NHWC with the channel count padded to
 *     dn_channel_pad(dtype, C) (16-byte multiples); padded channels hold 0.
 *   - Reduced precisions: BF16 (round to nearest even) and FP8 OCP e4m3
 *     (round to nearest even, saturating at +-448, per-output-channel weight
 *     scales, one per-tensor activation scale); every product accumulates in
 *     FP32.  Batch-norm folding into the weights runs in FP64 on the GPU.
 */
#ifndef DN_H
#define DN_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum dn_status {
    DN_OK = 0,
    DN_EINVAL = -1,        /* bad argument, shape or pointer kind */
    DN_ENOMEM = -2,        /* allocation failed or arena too small */
    DN_EHIP = -3,          /* a HIP runtime call failed */
    DN_ESTATE = -4,        /* call out of order (e.g. forward before load/bind) */
    DN_EUNSUPPORTED = -5,  /* valid request the library does not implement */
    DN_ETIMEDOUT = -6      /* a placed forward ran past its time limit */
} dn_status;

typedef enum dn_dtype { DN_F32 = 0, DN_BF16 = 1, DN_FP8_E4M3 = 2 } dn_dtype;
typedef enum dn_mode { DN_MODE_RESIDENT = 0, DN_MODE_PER_LAYER = 1 } dn_mode;
typedef enum dn_kind { DN_CONV = 0, DN_MAXPOOL = 1, DN_SHORTCUT = 2 } dn_kind;
typedef enum dn_act { DN_ACT_LINEAR = 0, DN_ACT_LEAKY = 1 } dn_act;

/* One layer of the network, in Darknet's layer vocabulary (Sec. 5.1.1).
 *   DN_CONV:     cout, ksize (square R = S), stride, pad (zero padding),
 *                batchnorm (1 = bias then inference BN), activation.
 *                y = act(BN(conv(x) + bias)).
 *   DN_MAXPOOL:  ksize = window, stride; -inf outside the input; output side
 *                (H - 1) / stride + 1; window starts at i*stride - (ksize-1)/2.
 *   DN_SHORTCUT: src = absolute index of an earlier layer; output =
 *                previous layer's output + layer src's output, shapes equal;
 *                activation must be DN_ACT_LINEAR (else DN_EUNSUPPORTED). */
typedef struct dn_layer_desc {
    int kind;
    int cout, ksize, stride, pad;
    int batchnorm;
    int activation;
    int src;
} dn_layer_desc;

typedef struct dn_net_opts {
    int in_c;            /* input channels (<= 16) */
    int max_h, max_w;    /* largest input size the net will see */
    int max_batch;
    int dtype;           /* dn_dtype of activations and weights */
    int mode;            /* dn_mode */
    float leaky_slope;   /* 0.1 for the Darknet leaky rectifier */
    double bn_eps;       /* batch-norm epsilon (1e-5) */
    int use_graph;       /* 1: resident forwards are captured once per
                            (batch, h, w, x, y, arena) into a hipGraph and replayed;
                            at most 4096 are kept per net, later new buffers
                            run without capture */
    int device;          /* HIP device ordinal */
    int batch_invariant; /* 1: every output element is reduced in an order that
                            does not depend on the batch size, so an image gives
                            the same bits alone and inside any batch: the
                            split-K partition of each conv is a function of its
                            K alone (dn_layer_plan reports it) and only tiles of
                            16x16 MFMA blocks run; tiles may still differ with
                            the batch.  0: tiles and splits tuned per batch. */
    int input_u8;        /* 1 (resident mode only): the x of dn_forward and
                            dn_forward_arena is NCHW 8-bit pixels, value q / 255
                            (a camera frame), converted on the device; the
                            image crosses PCIe at a quarter of the FP32 bytes.
                            0: NCHW FP32. */
} dn_net_opts;

typedef struct dn_net dn_net;

/* ---- network object ---------------------------------------------------- */

/* Validate the layer list and build the execution plan.  `layers` is copied. */
dn_status dn_net_create(const dn_layer_desc *layers, int n, const dn_net_opts *opts, dn_net **out);

/* Free everything the library allocated for the net (NULL-safe, idempotent
 * for distinct handles; the bound arena is the caller's and is not freed). */
void dn_net_destroy(dn_net *net);

/* Output shape (logical channels) for an input of h x w. */
dn_status dn_net_output_shape(const dn_net *net, int h, int w, int *c, int *ho, int *wo);

/* Device bytes the resident plan needs for (batch, h, w): every live
 * activation buffer (liveness-packed, 256-byte aligned) plus split-K scratch.
 * The per-layer mode uses the same arena as its device staging area. */
dn_status dn_arena_bytes(const dn_net *net, int batch, int h, int w, size_t *bytes);

/* Bind caller-owned device memory as the activation arena (kept until
 * rebind/destroy; must outlive every forward enqueued with it). */
dn_status dn_bind_arena(dn_net *net, void *dev_ptr, size_t bytes);

/* Upload one conv layer's FP64 host parameters: w [cout][cin][k][k], bias
 * [cout]; mean/var/gamma/beta [cout] or all NULL when the layer has no BN.
 * The library copies them, folds BN in FP64 on the GPU
 * (w' = w*g/sqrt(v+eps), b' = (b-m)*g/sqrt(v+eps) + beta), rounds to the net
 * dtype and packs; host arrays may be freed on return.  Synchronous. */
dn_status dn_load_weights(dn_net *net, int layer, const double *w, const double *bias,
                          const double *mean, const double *var,
                          const double *gamma, const double *beta);

/* FP8 nets only: set the static per-tensor activation scales from a
 * calibration input (device NCHW FP32, batch x in_c x h x w).  Runs an FP32
 * forward on the GPU with the same folded weights, takes amax of every
 * activation tensor, scale = amax / 448.  Synchronous. */
dn_status dn_calibrate(dn_net *net, const float *x, int batch, int h, int w, void *stream);

/* Forward.  Resident mode: x and y are device pointers (x NCHW FP32, or
 * NCHW uint8 for an input_u8 net; y NCHW FP32 of dn_net_output_shape); one ingest, the conv/pool/shortcut kernels and one
 * egress are enqueued on `stream` with no host synchronisation and no
 * allocation (or one hipGraphLaunch when use_graph is set).
 * Per-layer mode: x and y are host pointers; every layer's input and weights
 * are copied host->device, its kernel runs, its output is copied back and
 * the stream is synchronised before the next layer.
 * Requires all conv weights loaded (DN_ESTATE), an arena of at least
 * dn_arena_bytes (DN_ENOMEM) and, for FP8, calibration (DN_ESTATE). */
dn_status dn_forward(dn_net *net, const void *x, int batch, int h, int w, void *y, void *stream);

/* Same as dn_forward in resident mode with an explicit arena instead of the
 * bound one, so that several forwards may be in flight on disjoint arenas
 * (the serving loop gives each in-flight slot its own arena). */
dn_status dn_forward_arena(dn_net *net, void *arena, size_t arena_bytes, const void *x,
                           int batch, int h, int w, void *y, void *stream);

/* Pick a tile shape (and split-K factor) for every conv of the plan for
 * (batch, h, w) by timing the candidates on the bound arena; results are
 * cached in the net (and in the file named by $DN_TUNE_CACHE, if set).
 * Synchronous; overwrites arena contents. */
dn_status dn_autotune(dn_net *net, int batch, int h, int w, void *stream);

/* Average duration in ms of one launch of the kernel(s) that compute
 * `layer` in the resident plan for (batch, h, w), timed with hipEvents over
 * `iters` back-to-back launches on `stream` (arena contents are used as
 * they are).  Synchronous. */
dn_status dn_time_layer(dn_net *net, int layer, int batch, int h, int w, int iters,
                        void *stream, float *avg_ms);

/* Description of the resident plan's kernel for conv `layer` (tile config
 * index, split-K factor, fused pool / residual flags). */
dn_status dn_layer_plan(const dn_net *net, int layer, int batch, int h, int w,
                        int *tile, int *splits, int *fused_pool, int *fused_res);

/* ---- standalone layer kernels on device memory ------------------------- */

int dn_channel_pad(int dtype, int c);

typedef struct dn_conv_desc {
    int batch, in_h, in_w, in_c;   /* logical input (NHWC storage, channels padded) */
    int cout, ksize, stride, pad;
    int activation;
    float leaky_slope;
    int pool;        /* 0, or 2 = fused 2x2 stride-2 max pool (output side / 2) */
    int residual;    /* 1 = add `res` (output-shaped NHWC tensor) after the activation */
    int dtype;
    float in_scale;  /* FP8: x = q * in_scale (else ignored) */
    float res_scale; /* FP8: res = q * res_scale */
    float out_scale; /* FP8: y_q = y / out_scale */
    int tile;        /* -1 = library heuristic, else a tile config index */
    int splits;      /* 0 = library heuristic, else split-K factor */
    int input_nchw;  /* 1: x is the NCHW FP32 network input (ingest fused into the
                        conv; needs CP*ksize <= 16 where CP = in_c rounded
                        up to 4, 8 or 16 (in_c <= 16), ksize <= 4, cout <= 64,
                        stride <= 2, else DN_EUNSUPPORTED; weights packed in
                        the order k = r*16 + s*CP + c) */
} dn_conv_desc;

/* Bytes of the packed weight buffer, the FP32 bias / weight-scale buffers
 * and the split-K scratch the conv needs. */
dn_status dn_conv_sizes(const dn_conv_desc *d, size_t *w_bytes, size_t *vec_bytes, size_t *ws_bytes);

/* FP64 BN fold + round + pack of host parameters (same meaning as
 * dn_load_weights) into caller device buffers w_packed, bias (FP32),
 * wscale (FP32; all ones unless FP8).  Synchronous on `stream`. */
dn_status dn_conv_pack(const dn_conv_desc *d, const double *w, const double *bias,
                       const double *mean, const double *var, const double *gamma,
                       const double *beta, double eps, void *w_packed, float *bias_out,
                       float *wscale_out, void *stream);

/* Implicit-GEMM convolution (M = batch*Ho*Wo, N = cout, K = k*k*Cin_pad)
 * with the fused epilogue: +bias', activation, [+res], [2x2 max], round.
 * x, y, res, workspace: device.  Enqueue only.  With input_nchw = 1 the
 * first-layer kernel runs instead (x = NCHW FP32, no split-K, no residual). */
dn_status dn_conv2d(const dn_conv_desc *d, const void *x, const void *w_packed,
                    const float *bias, const float *wscale, const void *res, void *y,
                    void *workspace, size_t ws_bytes, void *stream);

typedef struct dn_pool_desc {
    int batch, h, w, c, size, stride, dtype;
} dn_pool_desc;

/* Max pool over NHWC device tensors (FP8: input and output share one scale). */
dn_status dn_maxpool(const dn_pool_desc *d, const void *x, void *y, void *stream);

/* y = a + b over NHWC device tensors of `count` padded elements
 * (FP8: values scaled by sa, sb, result divided by sy). */
dn_status dn_shortcut(int dtype, size_t count, const void *a, float sa, const void *b, float sb,
                      void *y, float sy, void *stream);

/* NCHW FP32 (device) -> NHWC storage dtype with padded channels. */
dn_status dn_ingest(int dtype, int batch, int c, int h, int w, const float *x, float scale,
                    void *y, void *stream);

/* NHWC storage dtype (padded channels) -> NCHW FP32 (device). */
dn_status dn_egress(int dtype, int batch, int c, int h, int w, const void *x, float scale,
                    float *y, void *stream);

/* ---- backward pass to the input image: the image-modification program the
 * paper ran beside detection (Sec. 5.1.1), which ascends the gradient of a
 * layer's activation energy with respect to the input image.  The paper does
 * not describe it; the definitions here are the plain derivatives of the
 * forward layers above.  F32 and BF16 only (else DN_EUNSUPPORTED); the
 * gradients have the storage dtype and the NHWC padded layout of the
 * activations they belong to, with FP32 accumulation.
 *
 * Backward-data conv of a forward conv `d` (unfused: pool = residual =
 * input_nchw = 0, pad <= ksize - 1):
 *   dx[n,c,p,q] = sum over k,r,s with p = i*stride - pad + r, q = j*stride - pad + s
 *                 of dy[n,k,i,j] * w'[k,c,r,s],  w' = w * gamma[k] / sqrt(var[k] + eps)
 * (w' = w without BN).  It runs as a stride-1 forward conv over dy (spread
 * onto the stride-1 grid with zeros when stride > 1) with channels swapped,
 * the filter flipped and pad ksize - 1 - pad.  dy: NHWC [batch][Ho][Wo][cout
 * padded]; dx: NHWC [batch][in_h][in_w][in_c padded]; accumulate = 1 adds
 * the result to dx (dx then also is read).  The workspace (device, caller
 * owned) holds split-K partials and the spread gradient. */
dn_status dn_conv_backward_sizes(const dn_conv_desc *d, size_t *w_bytes, size_t *vec_bytes, size_t *ws_bytes);
/* FP64 BN scale fold, flip, transpose, round and pack of the host weights w
 * [cout][in_c][k][k] (BN arrays all present or all NULL) into caller device
 * buffers: w_packed (w_bytes), zero_bias and unit_scale (vec_bytes each).
 * Synchronous on `stream`. */
dn_status dn_conv_pack_backward(const dn_conv_desc *d, const double *w, const double *mean,
                                const double *var, const double *gamma, double eps, void *w_packed,
                                float *zero_bias, float *unit_scale, void *stream);
dn_status dn_conv_backward_data(const dn_conv_desc *d, const void *dy, const void *w_packed,
                                const float *zero_bias, const float *unit_scale, int accumulate, void *dx,
                                void *workspace, size_t ws_bytes, void *stream);

/* Max-pool gradient: every window hands its gradient to its first maximal
 * element in row-major window order (the forward's comparison), elements
 * outside the input never win.  x: the pool's forward input; dy: gradient of
 * its output; dx (+)= result (accumulate = 1 adds).  NHWC device tensors. */
dn_status dn_maxpool_backward(const dn_pool_desc *d, const void *x, const void *dy, int accumulate,
                              void *dx, void *stream);

/* Leaky-rectifier gradient over `count` padded elements: dx = dy where the
 * layer's forward output a > 0, else dy * slope (0 <= slope <= 1, so a has the
 * sign of the pre-activation).  dx may be dy. */
dn_status dn_leaky_backward(int dtype, size_t count, const void *a, const void *dy, float slope, void *dx,
                            void *stream);

/* Gradient with respect to the input image of E = 1/2 * sum of squares of
 * layer `layer`'s output over the batch.  x, grad: device NCHW FP32
 * [batch][in_c][h][w].  Runs the forward up to `layer` keeping every layer
 * output (a conv and the 2x2/2 pool after it run fused and keep the pooled
 * output plus each window's argmax code instead of the full-size conv
 * output), then each layer's backward in reverse order (gradients of a
 * shortcut's two inputs add up).  Needs every conv's weights loaded
 * (DN_ESTATE).  Every buffer of the pass (stored layer outputs, argmax codes,
 * gradients, scratch) lives in the caller's arena: the one bound with
 * dn_bind_arena, which must hold at least dn_input_gradient_arena_bytes
 * (else DN_ENOMEM; none bound: DN_ESTATE).  No allocation, no host
 * synchronisation: enqueue only.  Calls that share an arena must not overlap
 * (same stream, or ordered by the caller); dn_input_gradient_arena takes an
 * explicit arena (256-byte aligned device memory) so that passes on disjoint
 * arenas may run concurrently. */
dn_status dn_input_gradient_arena_bytes(const dn_net *net, int layer, int batch, int h, int w, size_t *bytes);
dn_status dn_input_gradient(dn_net *net, int layer, const float *x, int batch, int h, int w, float *grad,
                            void *stream);
dn_status dn_input_gradient_arena(dn_net *net, void *arena, size_t arena_bytes, int layer, const float *x,
                                  int batch, int h, int w, float *grad, void *stream);

/* Read back what the last input-gradient pass on `arena` (same net, layer,
 * batch, h, w) left there, into caller device memory `out` (out_bytes), on
 * `stream`; for inspecting the branches the pass took (tests):
 *   what = 0: the stored output of layer of_layer (0 <= of_layer <= layer),
 *             NCHW FP32 [batch][c][ho][wo]; not stored for a conv whose
 *             2x2/2 pool ran fused (*available = 0);
 *   what = 1: the argmax codes of pool layer of_layer when it ran fused with
 *             the conv before it: uint8 NHWC [batch][ho][wo][c padded], code
 *             2*dy + dx of the window element that received the gradient;
 *   what = 2: the gradient of E with respect to layer of_layer's output
 *             (for a conv with a fused pool: its full-size output), NCHW FP32.
 * *available (may be NULL) tells whether the pass keeps that buffer; with
 * out = NULL only *available is set.  Enqueue only. */
dn_status dn_input_gradient_readback(const dn_net *net, void *arena, size_t arena_bytes, int layer, int batch,
                                     int h, int w, int of_layer, int what, void *out, size_t out_bytes,
                                     int *available, void *stream);

/* Tile autotuner of the input-gradient pass for (layer, batch, h, w): times
 * every candidate tile configuration x split-K of each unfused forward conv
 * and each backward-data conv of the pass (hipEvents, synchronous on
 * `stream`) and keeps the fastest, like dn_autotune (same $DN_TUNE_CACHE).
 * A tuning call: it allocates a temporary device buffer (the pass's arena
 * plus 512 MB of candidate scratch) and frees it before returning.
 * Optional: untuned convs use the library's heuristic. */
dn_status dn_autotune_backward(dn_net *net, int layer, int batch, int h, int w, void *stream);

/* `iters` steps of gradient ascent on E with respect to the image, in place:
 * x = clamp(x + rate * g / mean|g|, 0, 1), mean |g| per image (a step of
 * `rate` in the mean absolute sense).  Same buffers and rules as
 * dn_input_gradient (bound arena, or the explicit one of dn_nightmare_arena,
 * of at least dn_input_gradient_arena_bytes); no host round-trip between
 * iterations, no allocation. */
dn_status dn_nightmare(dn_net *net, int layer, float *x, int batch, int h, int w, float rate, int iters,
                       void *stream);
dn_status dn_nightmare_arena(dn_net *net, void *arena, size_t arena_bytes, int layer, float *x, int batch, int h,
                             int w, float rate, int iters, void *stream);

/* ---- Jacobi iteration for the Laplace equation: the second program the
 * paper's transfer rule sped up (Sec. 4, the paragraph before Sec. 5).
 * u: [n][m] FP64 row-major grid whose first/last rows and columns are fixed
 * (Dirichlet) values.  One iteration replaces every interior point by
 * 0.25 * (up + down + left + right), summed in that order (FP64, no fused
 * multiply-add), from the previous iterate.
 *
 * dn_jacobi: device-resident.  u and work are device buffers of n*m doubles
 * (caller-owned; work is scratch).  Runs `iters` iterations with no host
 * round-trip; u holds the result.  max_change (device, one double, may be
 * NULL) receives the largest |change| of the last iteration (0 for
 * iters = 0).  Enqueue only.
 *
 * dn_jacobi_per_iteration: the naive offload, for comparison.  u_host is a
 * host grid; every iteration copies it to dev_a, runs one step into dev_b,
 * copies dev_b back to u_host and synchronises.  dev_a, dev_b: device, n*m
 * doubles each.  max_change_host (may be NULL) as above.  Synchronous.
 *
 * Non-positive sizes, negative iterations, NULL grids, or a device pointer
 * passed as u_host: DN_EINVAL. */
dn_status dn_jacobi(double *u, double *work, int n, int m, int iters, double *max_change, void *stream);
dn_status dn_jacobi_per_iteration(double *u_host, double *dev_a, double *dev_b, int n, int m, int iters,
                                  double *max_change_host, void *stream);

/* ---- detection post-processing (the workload's detection program, Sec.
 * 5.1.1; the paper gives no decoding rule, so this one is a stated reading).
 * y: device, [batch][anchors*(5+classes)][h][w] FP32, the dn_forward output of
 * a region head: per anchor a, channels a*(5+classes) + (0..4) are
 * tx, ty, tw, th, to and the next `classes` channels are class logits.
 * Box index b = (i*w + j)*anchors + a for grid cell (row i, column j).
 * Box (centre x, centre y, width, height) in image fractions:
 *   ((j + sigmoid(tx)) / w, (i + sigmoid(ty)) / h,
 *    anchor_w * exp(tw) / w, anchor_h * exp(th) / h);
 * score of class k = sigmoid(to) * softmax(logits)[k].
 * Per image and class: candidates with score >= thresh, ranked by score
 * (descending; ties by box index ascending), are kept greedily unless a kept
 * box overlaps them with IoU > nms_thresh; at most max_det are kept.
 * Outputs (device, caller-owned): dets [batch][classes][max_det][5] = score,
 * x, y, w, h; det_index [batch][classes][max_det]; counts [batch][classes]
 * (entries past counts are left untouched).  anchor_wh: host, 2*anchors
 * floats (w, h per anchor, in grid cells), copied at the call.
 * workspace: device, at least dn_detect_workspace() bytes.  Enqueue only.
 * Limits: anchors <= 16, h*w*anchors <= 4096, else DN_EUNSUPPORTED;
 * non-positive sizes, NULL pointers, NaN thresholds or a short workspace are
 * DN_EINVAL.  Decisions are taken in FP32. */
dn_status dn_detect_workspace(int batch, int anchors, int classes, int h, int w, size_t *bytes);
dn_status dn_detect(const float *y, int batch, int anchors, int classes, int h, int w,
                    const float *anchor_wh, float thresh, float nms_thresh, int max_det,
                    void *workspace, size_t ws_bytes, float *dets, int *det_index, int *counts,
                    void *stream);

/* ---- placement of layers between the host CPU and the GPU: the paper's
 * offload search (Sec. 3.3 and Sec. 4) with its transfer rule (Sec. 3.2)
 * and GA parameters (Sec. 5.1.2), applied to this library's layers.  A gene
 * holds one byte per layer of the net (gene_len = number of layers):
 * 1 = the layer runs on the GPU (the library's kernels), 0 = on the host CPU
 * (the library's host FP32 layer code, worker threads: $DN_CPU_THREADS, else
 * $OMP_NUM_THREADS, else up to 16).  The host side runs only where a gene
 * puts it; dn_forward never uses it.  FP32 resident-mode nets only (else
 * DN_EUNSUPPORTED).
 *
 * Transfers follow Sec. 3.2 at layer granularity: weights stay where they
 * were defined (device weights for GPU layers; a host copy of the same folded
 * FP32 weights, read back once on the first placed call, for host layers); a
 * layer output crosses once, right after the layer that produces it, when a
 * layer on the other side reads it; the image crosses once when a GPU layer
 * reads it; the result crosses once when a GPU layer produces it.  A conv and
 * the 2x2/2 pool (or linear shortcut) after it run fused when both are on
 * the GPU, as in the resident forward, so the all-GPU gene runs the resident
 * plan with one input and one output crossing. */

/* Device bytes a placed forward of (batch, h, w) needs in the bound arena,
 * for any gene (every layer output keeps its own buffer, plus split-K
 * scratch and FP32 staging of the image and the result). */
dn_status dn_placed_arena_bytes(const dn_net *net, int batch, int h, int w, size_t *bytes);

/* The crossings a gene implies (host logic, nothing runs): h2d / d2h counts
 * and bytes of copies per forward, image and result included.  Any output
 * pointer may be NULL.  gene_len must equal the number of layers and every
 * gene value be 0 or 1 (else DN_EINVAL). */
dn_status dn_placed_transfers(const dn_net *net, const unsigned char *gene, int gene_len, int batch, int h, int w,
                              int *h2d, int *d2h, size_t *h2d_bytes, size_t *d2h_bytes);

/* Forward with each layer on the side its gene value names.  x, y: host
 * NCHW FP32 (x [batch][in_c][h][w], y of dn_net_output_shape).  Uses the
 * bound arena (at least dn_placed_arena_bytes, else DN_ENOMEM) and, per
 * (batch, h, w), pinned host buffers the library allocates on first use and
 * keeps until destroy.  Synchronous: returns after y is written.  With
 * timeout_s > 0 a forward still running after timeout_s seconds stops
 * between two layers and returns DN_ETIMEDOUT (y is then undefined). */
dn_status dn_forward_placed(dn_net *net, const unsigned char *gene, int gene_len, const float *x, int batch, int h,
                            int w, float *y, double timeout_s, void *stream);

/* Host FP32 layer code of the placement on host buffers (checked on their
 * own by the tests): dn_cpu_conv2d runs the conv of d (dtype DN_F32, no
 * fused pool or residual, input_nchw = 0, else DN_EUNSUPPORTED) with
 * already folded host weights w [cout][in_c][k][k] and bias [cout]: y =
 * act(conv(x, w) + bias), x / y NHWC with padded channels
 * (dn_channel_pad(DN_F32, .)); dn_cpu_maxpool pools NHWC x into y like
 * dn_maxpool (dtype DN_F32). */
dn_status dn_cpu_conv2d(const dn_conv_desc *d, const float *x, const float *w, const float *bias, float *y);
dn_status dn_cpu_maxpool(const dn_pool_desc *d, const float *x, float *y);

typedef struct dn_ga_params {
    int population;          /* M, >= 1 (paper: 30) */
    int generations;         /* T, >= 1 (paper: 20) */
    double crossover;        /* Pc in [0, 1] (paper: 0.9), one-point */
    double mutation;         /* Pm in [0, 1] (paper: 0.05), per gene value */
    double timeout_s;        /* > 0: a slower (or failed) measurement scores penalty_s */
    double penalty_s;        /* > 0 (paper: 1000 s for its 3-minute limit) */
    unsigned long long seed; /* SplitMix64 state the search starts from */
} dn_ga_params;

typedef struct dn_ga_result {
    double best_seconds;     /* score of best_gene */
    int evaluations;         /* distinct genes measured */
    int memo_hits;           /* genes scored from an earlier measurement */
} dn_ga_result;

/* Measurement callback: seconds taken by the program with this gene; < 0 =
 * the run failed (scored as penalty_s); NaN aborts the search. */
typedef double (*dn_ga_measure_fn)(const unsigned char *gene, int gene_len, double timeout_s, void *user);

/* One GA generation step (host logic): from the measured population pop
 * [M][L] with times seconds [M] to next [M][L], drawing from the SplitMix64
 * state *rng_state (updated).  Fitness = time^(-1/2); next[0] is the fittest
 * gene (first on ties) unchanged (elite); the rest are children of pairs
 * picked by roulette on the fitness, crossed at one random point with
 * probability Pc, then flipped value by value with probability Pm.  The
 * draw order per pair is: parent a, parent b, the crossover draw, the cut
 * point (only when crossing, L >= 2), then one mutation draw per value of
 * the first child and one per value of the second; the second child of the
 * last pair is dropped when M - 1 is odd.  seconds must be positive. */
dn_status dn_ga_next_generation(const dn_ga_params *p, int gene_len, const unsigned char *pop, const double *seconds,
                                unsigned char *next, unsigned long long *rng_state);

/* T generations of the GA (host logic): initial genes drawn value by value
 * (top bit of one draw each), each generation measured (a gene seen before
 * reuses its score), then dn_ga_next_generation.  best_gene [L] receives the
 * fittest gene measured; gen_best [T] (may be NULL) the best score of each
 * generation; *res the counts.  DN_EINVAL on bad parameters, DN_ESTATE when
 * the callback aborted. */
dn_status dn_ga_search(const dn_ga_params *p, int gene_len, dn_ga_measure_fn measure, void *user,
                       unsigned char *best_gene, double *gen_best, dn_ga_result *res);

/* The GA over this net's layer placements: each gene is measured as the
 * median wall time of `reps` dn_forward_placed runs on the host buffers x / y
 * (after one untimed run of the all-GPU and of the all-CPU gene, which also
 * allocates the host buffers); timeout_s of p bounds each run.  Same outputs
 * as dn_ga_search; y holds the last run's result. */
dn_status dn_ga_place(dn_net *net, const dn_ga_params *p, const float *x, int batch, int h, int w, float *y,
                      int reps, void *stream, unsigned char *best_gene, double *gen_best, dn_ga_result *res);

/* dn_detect without a workspace argument, for callers that cannot allocate
 * device memory (code under hipGraph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  The decode's scratch is a fixed array of 16 MiB
 * inside the library, one per GPU, held until the process ends; the call
 * allocates nothing (no hipMalloc / hipFree / allocating library routine)
 * and runs on the current device.  Inputs needing more than 16 MiB of
 * scratch (batch*classes*h*w*anchors*4 rounded up to 256 bytes, plus
 * batch*h*w*anchors*16) are rejected with DN_EINVAL.  Every call on one GPU
 * shares that GPU's scratch: calls that overlap on one GPU (different
 * streams, or host threads) race and must be ordered by the caller.  Other
 * arguments, outputs and errors as dn_detect. */
dn_status dn_detect_noalloc(const float *y, int batch, int anchors, int classes, int h, int w,
                            const float *anchor_wh, float thresh, float nms_thresh, int max_det,
                            float *dets, int *det_index, int *counts, void *stream);

/* Measurement helper: the matrix-core throughput the device sustains for the
 * MFMA instruction the convolutions of `dtype` use (16x16x4 FP32, 16x16x32
 * BF16, 16x16x128 FP8), from a kernel that only multiplies (8 waves per SIMD,
 * 8 independent accumulators per wave, no memory traffic); best of three
 * timed launches, in TFLOP/s.  Synchronous; allocates and frees a small
 * device buffer.  DN_EINVAL for a NULL pointer or unknown dtype, DN_EHIP on
 * a HIP failure. */
dn_status dn_mfma_peak(int dtype, int device, double *tflops);

/* Number of compiled conv tile configurations and their shapes: output tile
 * bm x bn, waves_m x waves_n waves, and the side of the MFMA blocks a BF16
 * conv uses with it (16 or 32; other dtypes always use 16x16 blocks).  Tiles
 * with the same block side give bitwise-identical results; 16 and 32 differ
 * by FP32 summation order only.  Any out-pointer may be NULL; a tile outside
 * [0, dn_tile_count()) is DN_EINVAL. */
int dn_tile_count(void);
dn_status dn_tile_info(int tile, int *bm, int *bn, int *waves_m, int *waves_n, int *mfma_bf16);

const char *dn_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* DN_H */
