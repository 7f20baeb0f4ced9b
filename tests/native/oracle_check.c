/* Sanitizer run of the oracle's C layer definitions (built with
 * -fsanitize=address,undefined by tests/test_sanitizers.py): every function
 * on ragged shapes, strides and paddings, including windows and taps that
 * fall off every edge.  Values are checked by the Python pins; this run is
 * about memory and undefined behaviour. */
#include <stdio.h>
#include <stdlib.h>

void oracle_conv2d(const double *x, int n, int c, int h, int w, const double *wt, int k, int r, int s, int stride,
                   int pad, double *y);
void oracle_add_bias(double *y, int n, int k, int hw, const double *b);
void oracle_batchnorm(double *y, int n, int k, int hw, const double *mean, const double *var, const double *gamma,
                      const double *beta, double eps);
void oracle_leaky(double *y, long count, double slope);
void oracle_maxpool(const double *x, int n, int c, int h, int w, int size, int stride, double *y);
void oracle_shortcut(double *y, const double *x, long count);
void oracle_conv2d_backward_data(const double *dy, int n, int k, int ho, int wo, const double *w, int c, int r, int s,
                                 int stride, int pad, int h, int wd, double *dx);
void oracle_maxpool_backward(const double *x, int n, int c, int h, int w, int size, int stride, const double *dy,
                             double *dx);

static double *fill(long count, unsigned seed)
{
    double *p = malloc(sizeof(double) * (count > 0 ? count : 1));
    for (long i = 0; i < count; ++i) p[i] = (double)((i * 2654435761u + seed) % 1000) / 500.0 - 1.0;
    return p;
}

int main(void)
{
    const int shapes[][8] = {/* n c h w k r stride pad */
                             {1, 3, 7, 5, 4, 3, 1, 1}, {2, 4, 6, 9, 3, 3, 2, 1}, {1, 2, 1, 1, 2, 3, 1, 1},
                             {2, 5, 8, 8, 6, 1, 1, 0}, {1, 1, 5, 4, 1, 3, 2, 0}, {1, 2, 13, 13, 2, 3, 1, 1}};
    for (size_t t = 0; t < sizeof shapes / sizeof shapes[0]; ++t) {
        const int n = shapes[t][0], c = shapes[t][1], h = shapes[t][2], w = shapes[t][3], k = shapes[t][4];
        const int r = shapes[t][5], st = shapes[t][6], pad = shapes[t][7];
        const int ho = (h + 2 * pad - r) / st + 1, wo = (w + 2 * pad - r) / st + 1;
        if (ho <= 0 || wo <= 0) continue;
        double *x = fill((long)n * c * h * w, 1), *wt = fill((long)k * c * r * r, 2), *b = fill(k, 3);
        double *m = fill(k, 4), *v = fill(k, 5), *g = fill(k, 6), *be = fill(k, 7);
        for (int i = 0; i < k; ++i) v[i] = v[i] * v[i] + 0.5;
        double *y = fill((long)n * k * ho * wo, 8);
        oracle_conv2d(x, n, c, h, w, wt, k, r, r, st, pad, y);
        oracle_add_bias(y, n, k, ho * wo, b);
        oracle_batchnorm(y, n, k, ho * wo, m, v, g, be, 1e-5);
        oracle_leaky(y, (long)n * k * ho * wo, 0.1);
        double *dx = fill((long)n * c * h * w, 9);
        oracle_conv2d_backward_data(y, n, k, ho, wo, wt, c, r, r, st, pad, h, w, dx);
        for (int size = 1; size <= 3; ++size)
            for (int ps = 1; ps <= 2; ++ps) {
                const int po = (h - 1) / ps + 1, qo = (w - 1) / ps + 1;
                double *py = fill((long)n * c * po * qo, 10), *pdy = fill((long)n * c * po * qo, 11);
                oracle_maxpool(x, n, c, h, w, size, ps, py);
                oracle_maxpool_backward(x, n, c, h, w, size, ps, pdy, dx);
                free(py);
                free(pdy);
            }
        oracle_shortcut(x, dx, (long)n * c * h * w);
        free(x); free(wt); free(b); free(m); free(v); free(g); free(be); free(y); free(dx);
    }
    printf("oracle checks ran\n");
    return 0;
}
