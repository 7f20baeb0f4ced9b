/*
 * FP64 CPU oracle for the Darknet-style CNN forward pass.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the parity reference for the HIP
 * library; only the test-suite, the smoke check and the CPU-baseline leg of
 * the benchmark may load it.  It shares no code, header, table or helper with
 * the GPU path (paper_1811_03882_amd/csrc), and the GPU path never calls it.
 *
 * What it computes.  The paper offloads the loops of Darknet, a C neural
 * network framework, and evaluates its object-detection and image-edit
 * sample programs (Sec. 5.1.1).  The loops it moves to the GPU are those of a
 * CNN forward pass; the paper states no layer formula, so each function below
 * is the plain textbook definition of one layer, written in the most direct
 * loop form, in double precision, NCHW layout:
 *
 *   conv2d     y[n,k,i,j] = sum_{c,r,s} w[k,c,r,s] * x[n,c,i*st-p+r,j*st-p+s]
 *              (taps outside the image read 0)
 *   bias       y += b[k]
 *   batchnorm  y = gamma[k] * (y - mean[k]) / sqrt(var[k] + eps) + beta[k]
 *              (inference form, statistics given, not folded)
 *   leaky      y = y if y > 0 else slope * y
 *   maxpool    y[n,c,i,j] = max over the size x size window starting at
 *              (i*st - o, j*st - o), o = (size-1)/2; taps outside are -inf
 *              output side = (H - 1)/st + 1
 *   shortcut   y += x  (elementwise residual add)
 *
 * The whole-network composition (which layer feeds which) lives in
 * oracle/net.py.  OpenMP only splits the outermost independent loops
 * (image, output channel); every output element is one sequential sum in
 * ascending (c, r, s) order.
 */
#include <math.h>
#include <stddef.h>

/* Direct convolution, zero padding. x: [n][c][h][w], wt: [k][c][r][s],
 * y: [n][k][ho][wo] with ho = (h + 2*pad - r)/stride + 1 (same for wo). */
void oracle_conv2d(const double *x, int n, int c, int h, int w,
                   const double *wt, int k, int r, int s,
                   int stride, int pad, double *y)
{
    const int ho = (h + 2 * pad - r) / stride + 1;
    const int wo = (w + 2 * pad - s) / stride + 1;
#pragma omp parallel for collapse(2) schedule(static)
    for (int in = 0; in < n; ++in)
        for (int ik = 0; ik < k; ++ik)
            for (int i = 0; i < ho; ++i)
                for (int j = 0; j < wo; ++j) {
                    double acc = 0.0;
                    for (int ic = 0; ic < c; ++ic)
                        for (int ir = 0; ir < r; ++ir)
                            for (int is = 0; is < s; ++is) {
                                const int yy = i * stride - pad + ir;
                                const int xx = j * stride - pad + is;
                                if (yy < 0 || yy >= h || xx < 0 || xx >= w)
                                    continue;
                                acc += wt[((size_t)(ik * c + ic) * r + ir) * s + is] *
                                       x[((size_t)(in * c + ic) * h + yy) * w + xx];
                            }
                    y[((size_t)(in * k + ik) * ho + i) * wo + j] = acc;
                }
}

/* Per-channel bias: y[n][k][hw] += b[k]. */
void oracle_add_bias(double *y, int n, int k, int hw, const double *b)
{
    for (int in = 0; in < n; ++in)
        for (int ik = 0; ik < k; ++ik)
            for (int p = 0; p < hw; ++p)
                y[((size_t)in * k + ik) * hw + p] += b[ik];
}

/* Inference batch normalisation with given statistics, unfolded. */
void oracle_batchnorm(double *y, int n, int k, int hw,
                      const double *mean, const double *var,
                      const double *gamma, const double *beta, double eps)
{
    for (int in = 0; in < n; ++in)
        for (int ik = 0; ik < k; ++ik) {
            const double sd = sqrt(var[ik] + eps);
            for (int p = 0; p < hw; ++p) {
                double *v = &y[((size_t)in * k + ik) * hw + p];
                *v = gamma[ik] * (*v - mean[ik]) / sd + beta[ik];
            }
        }
}

/* Leaky rectifier. */
void oracle_leaky(double *y, long count, double slope)
{
    for (long i = 0; i < count; ++i)
        if (!(y[i] > 0.0))
            y[i] = slope * y[i];
}

/* Max pooling with -inf outside the input.  x: [n][c][h][w]. */
void oracle_maxpool(const double *x, int n, int c, int h, int w,
                    int size, int stride, double *y)
{
    const int ho = (h - 1) / stride + 1;
    const int wo = (w - 1) / stride + 1;
    const int off = (size - 1) / 2;
    for (int in = 0; in < n; ++in)
        for (int ic = 0; ic < c; ++ic)
            for (int i = 0; i < ho; ++i)
                for (int j = 0; j < wo; ++j) {
                    double m = -INFINITY;
                    for (int u = 0; u < size; ++u)
                        for (int v = 0; v < size; ++v) {
                            const int yy = i * stride - off + u;
                            const int xx = j * stride - off + v;
                            if (yy < 0 || yy >= h || xx < 0 || xx >= w)
                                continue;
                            const double t = x[((size_t)(in * c + ic) * h + yy) * w + xx];
                            if (t > m)
                                m = t;
                        }
                    y[((size_t)(in * c + ic) * ho + i) * wo + j] = m;
                }
}

/* Residual add: y += x elementwise. */
void oracle_shortcut(double *y, const double *x, long count)
{
    for (long i = 0; i < count; ++i)
        y[i] += x[i];
}

/* Backward of the convolution with respect to its input (the gradient the
   image-edit program propagates to the image): for every output position and
   tap, dx[n,c,i*stride-pad+r, j*stride-pad+s] += dy[n,k,i,j] * w[k,c,r,s];
   taps outside the input contribute nothing.  dx is [n,c,h,wd], zeroed here. */
void oracle_conv2d_backward_data(const double *dy, int n, int k, int ho, int wo,
                                 const double *w, int c, int r, int s, int stride, int pad,
                                 int h, int wd, double *dx)
{
    for (long t = 0; t < (long)n * c * h * wd; ++t)
        dx[t] = 0.0;
    /* each (image, input channel) plane is written by one thread only */
#pragma omp parallel for collapse(2) schedule(static)
    for (int in = 0; in < n; ++in)
        for (int ic = 0; ic < c; ++ic)
            for (int ik = 0; ik < k; ++ik)
                for (int i = 0; i < ho; ++i)
                    for (int j = 0; j < wo; ++j) {
                        const double g = dy[((size_t)(in * k + ik) * ho + i) * wo + j];
                        for (int u = 0; u < r; ++u)
                            for (int v = 0; v < s; ++v) {
                                const int yy = i * stride - pad + u;
                                const int xx = j * stride - pad + v;
                                if (yy < 0 || yy >= h || xx < 0 || xx >= wd)
                                    continue;
                                dx[((size_t)(in * c + ic) * h + yy) * wd + xx] +=
                                    g * w[(((size_t)ik * c + ic) * r + u) * s + v];
                            }
                    }
}

/* Backward of max pooling: every output window hands its gradient to the
   first maximal input of the window (row-major order inside the window, the
   same strict comparison as the forward); dx is [n,c,h,w], zeroed here. */
void oracle_maxpool_backward(const double *x, int n, int c, int h, int w,
                             int size, int stride, const double *dy, double *dx)
{
    const int ho = (h - 1) / stride + 1;
    const int wo = (w - 1) / stride + 1;
    const int off = (size - 1) / 2;
    for (long t = 0; t < (long)n * c * h * w; ++t)
        dx[t] = 0.0;
    for (int in = 0; in < n; ++in)
        for (int ic = 0; ic < c; ++ic)
            for (int i = 0; i < ho; ++i)
                for (int j = 0; j < wo; ++j) {
                    double m = -INFINITY;
                    long arg = -1;
                    for (int u = 0; u < size; ++u)
                        for (int v = 0; v < size; ++v) {
                            const int yy = i * stride - off + u;
                            const int xx = j * stride - off + v;
                            if (yy < 0 || yy >= h || xx < 0 || xx >= w)
                                continue;
                            const long q = ((long)(in * c + ic) * h + yy) * w + xx;
                            if (x[q] > m) {
                                m = x[q];
                                arg = q;
                            }
                        }
                    if (arg >= 0)
                        dx[arg] += dy[((size_t)(in * c + ic) * ho + i) * wo + j];
                }
}
