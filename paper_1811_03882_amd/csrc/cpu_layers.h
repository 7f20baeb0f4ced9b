// Host (CPU) FP32 layer kernels: the "CPU" side of the paper's per-loop
// CPU/GPU placement (Sec. 3.3, Sec. 4).  A layer the placement gene leaves on
// the CPU runs here, on the same NHWC layout with 16-byte padded channels as
// the device activations of an FP32 net, so that a value crossing between the
// host and the device is a plain copy of its buffer.  Only the placed forward
// (dn_forward_placed) calls these; the forward passes never do.
//
// Compiled by the host compiler alone (no HIP): nothing here touches a GPU.
#pragma once

#include <cstddef>
#include <functional>

namespace dncpu {

// Threads of the process-wide worker pool: $DN_CPU_THREADS, else
// $OMP_NUM_THREADS, else the hardware concurrency capped at 16.
int threads();

// Run body(t) for t in [0, tasks) on the pool and wait for all of them.
void parallel_for(int tasks, const std::function<void(int)> &body);

// y = act(conv(x, w) + bias) over NHWC tensors.
//   x [n][H][W][cin_p], y [n][Ho][Wo][cout_p]
//   w [cout_p/16 blocks][R][S][cin_p][16] for the first cout_p/16*16 output
//     channels, then [R][S][cin_p][cout_p % 16] for the rest (see pack_weights)
//   act 0 linear, 1 leaky with slope (0 <= slope <= 1).
// Zero padding outside the input; padded output channels get act(0 + bias) =
// 0 because their weights and bias are zero.
void conv(const float *x, int n, int H, int W, int cin_p, const float *w, const float *bias, int cout_p, int R,
          int S, int stride, int pad, int act, float slope, float *y, int Ho, int Wo);

// Reorder weights given as wval(co, r, s, c) (co < cout_p, c < cin_p) into the
// blocked layout conv() reads; out holds cout_p*R*S*cin_p floats.
void pack_weights(const std::function<float(int, int, int, int)> &wval, int cout_p, int R, int S, int cin_p,
                  float *out);

// Max pool, window k x k, stride s, window of output (i, j) starting at
// (i*s - (k-1)/2, j*s - (k-1)/2); taps outside the input never win.
void maxpool(const float *x, int n, int H, int W, int cp, int k, int stride, float *y, int Ho, int Wo);

// y = a + b over count floats.
void add(const float *a, const float *b, float *y, size_t count);

// NCHW [n][c][h][w] -> NHWC [n][h][w][cp] (padded channels 0), and back.
void ingest(const float *x, int n, int c, int h, int w, int cp, float *y);
void egress(const float *x, int n, int c, int h, int w, int cp, float *y);

}  // namespace dncpu
