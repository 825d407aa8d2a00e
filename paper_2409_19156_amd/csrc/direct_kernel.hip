// Direct evaluation of the radial polynomials from their closed form (paper
// Sec. 2, Eq. radial-part-eq): R = sum_s c_s r^(n-2s), each term formed on its
// own and the terms summed in order of s, in FP64.  This is the comparator the
// paper contrasts the Jacobi recurrence with (its accuracy figure): the
// alternating terms of very different size lose digits as n - m grows.  It is
// provided for accuracy comparisons only; zp_radial is the accurate path.
#include <hip/hip_runtime.h>

#include "zp_internal.hpp"

namespace zp {
namespace {

__device__ __forceinline__ double ipow_d(double x, int e)
{
    double acc = 1.0;
    while (e) {
        if (e & 1) acc *= x;
        x *= x;
        e >>= 1;
    }
    return acc;
}

// grid: (point tiles of 256, modes)
__global__ __launch_bounds__(256) void direct_kernel(const int32_t *__restrict__ nn, const int32_t *__restrict__ mm,
                                                     const int64_t *__restrict__ off, const double *__restrict__ coef,
                                                     const double *__restrict__ r, int64_t P, int64_t M, int J,
                                                     double *__restrict__ out)
{
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t i = blockIdx.y;
    if (p >= P) return;
    const int n = nn[i];
    const int a = mm[i] < 0 ? -mm[i] : mm[i];
    const int K = (n - a) / 2;
    const double x = r[p];
    const double *c = coef + off[i];
    for (int j = 0; j <= J; ++j) {
        double sum = 0.0;
        for (int s = 0; s <= K; ++s) {
            const int e = n - 2 * s - j;
            if (e < 0) continue;
            sum += c[j * (K + 1) + s] * ipow_d(x, e);
        }
        out[((int64_t)j * M + i) * P + p] = sum;
    }
}

} // namespace

zp_status launch_direct_kernel(const Plan &plan, const double *d_r, int64_t P, int J, double *out, hipStream_t s)
{
    const int64_t M = (int64_t)plan.n.size();
    if (M > 65535) return set_error(ZP_ERR_ARG, "direct evaluation takes at most 65535 modes per call");
    const dim3 grid((unsigned)((P + 255) / 256), (unsigned)M);
    hipLaunchKernelGGL(direct_kernel, grid, dim3(256), 0, s, plan.d_direct_n, plan.d_direct_m, plan.d_direct_off,
                       plan.d_direct_coef, d_r, P, M, J, out);
    return hip_check(hipGetLastError(), "direct kernel launch");
}

} // namespace zp
