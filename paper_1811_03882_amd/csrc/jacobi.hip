// Jacobi iteration for the Laplace equation (second workload of the paper's
// transfer rule: the sample program solved with Jacobi's method, Sec. 4).
//
// One iteration: every interior point of the [n][m] FP64 grid becomes the
// average of its four neighbours from the previous iterate, summed in the
// order up + down + left + right (contraction off, so the result is the
// same in every rounding as the plain definition); the boundary stays fixed.
// HBM-bound: each iteration reads one grid and writes one.  A thread owns a
// column segment of STRIP rows, keeps the vertical neighbours in registers
// and reads the horizontal ones through the L1, so every element leaves HBM
// about once per iteration.  The largest change of the iteration is reduced
// per wave and folded into one global maximum (non-negative doubles order
// like their bit patterns).
#include "dn_kernels.h"

#pragma clang fp contract(off)

namespace dnk {

constexpr int JAC_BX = 64, JAC_BY = 4, JAC_STRIP = 8;

__global__ void __launch_bounds__(JAC_BX * JAC_BY) jacobi_step(const double *__restrict__ u, double *__restrict__ v,
                                                              int n, int m, unsigned long long *max_change)
{
    const int j = blockIdx.x * JAC_BX + (threadIdx.x % JAC_BX);
    const int i0 = (blockIdx.y * JAC_BY + threadIdx.x / JAC_BX) * JAC_STRIP;
    double ch = 0.0;
    if (j < m && i0 < n) {
        const bool edge_col = j == 0 || j == m - 1;
        double up = i0 > 0 ? u[(size_t)(i0 - 1) * m + j] : 0.0;
        double mid = u[(size_t)i0 * m + j];
        for (int r = 0; r < JAC_STRIP; ++r) {
            const int i = i0 + r;
            if (i >= n) break;
            const double down = i + 1 < n ? u[(size_t)(i + 1) * m + j] : 0.0;
            double out = mid;
            if (!edge_col && i > 0 && i < n - 1) {
                const double left = u[(size_t)i * m + j - 1], right = u[(size_t)i * m + j + 1];
                double s = up + down;
                s = s + left;
                s = s + right;
                out = 0.25 * s;
                ch = fmax(ch, fabs(out - mid));
            }
            v[(size_t)i * m + j] = out;
            up = mid;
            mid = down;
        }
    }
    if (max_change) {
        // wave maximum, then one atomic per wave
        for (int off = 32; off > 0; off >>= 1) ch = fmax(ch, __shfl_xor(ch, off));
        if ((threadIdx.x & 63) == 0) atomicMax(max_change, (unsigned long long)__double_as_longlong(ch));
    }
}

__global__ void jacobi_zero(unsigned long long *p) { *p = 0ull; }

hipError_t launch_jacobi_step(const double *u, double *v, int n, int m, unsigned long long *max_change, hipStream_t s)
{
    if (max_change) hipLaunchKernelGGL(jacobi_zero, dim3(1), dim3(1), 0, s, max_change);
    dim3 grid((m + JAC_BX - 1) / JAC_BX, (n + JAC_BY * JAC_STRIP - 1) / (JAC_BY * JAC_STRIP));
    hipLaunchKernelGGL(jacobi_step, grid, dim3(JAC_BX * JAC_BY), 0, s, u, v, n, m, max_change);
    return hipGetLastError();
}

}  // namespace dnk
