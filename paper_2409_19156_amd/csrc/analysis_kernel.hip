// Elementwise steps of the analysis transform (coefficients from samples by
// quadrature): the weighting of the samples before the contraction over
// points, and the division by each mode's norm after it.
#include <hip/hip_runtime.h>

#include "series.hpp"

namespace zp {
namespace {

constexpr int kThreads = 256;

// wf[p][b] = w[p] f[p][b]
__global__ __launch_bounds__(kThreads) void weight_kernel(const double *__restrict__ w, const double *__restrict__ f,
                                                          int64_t P, int64_t B, double *__restrict__ wf)
{
    const int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (t >= P * B) return;
    wf[t] = w[t / B] * f[t];
}

// c[col][b] *= 2(n+1) / (eps_m pi) for every emission of the chain in
// blockIdx.x (n = 2K + alpha; eps = 2 for m = 0, else 1): the inverse of
// the integral of Z^2 over the unit disc.  Every column belongs to exactly
// one emission, so no two threads touch one element.
__global__ __launch_bounds__(kThreads) void norm_kernel(const Chain *__restrict__ chains,
                                                        const Emit *__restrict__ emits, int64_t B,
                                                        double *__restrict__ c)
{
    const int64_t b = (int64_t)blockIdx.y * kThreads + threadIdx.x;
    if (b >= B) return;
    const Chain ch = chains[blockIdx.x];
    const double inv_pi = 0.318309886183790671537767526745028724; // 1/pi
    for (int e = ch.emit_off; e < ch.emit_off + ch.emit_cnt; ++e) {
        const Emit em = emits[e];
        const double n1 = (double)(2 * em.K + ch.alpha + 1);
        const double s = (ch.alpha == 0 ? 1.0 : 2.0) * n1 * inv_pi;
        c[(int64_t)em.col * B + b] *= s;
    }
}

} // namespace

zp_status launch_weight(const double *w, const double *f, int64_t P, int64_t B, double *wf, hipStream_t s)
{
    const int64_t n = P * B;
    if (n == 0) return ZP_OK;
    const int64_t blocks = (n + kThreads - 1) / kThreads;
    if (blocks > INT32_MAX) return set_error(ZP_ERR_ARG, "P * B too large for one launch");
    hipLaunchKernelGGL(weight_kernel, dim3((unsigned)blocks), dim3(kThreads), 0, s, w, f, P, B, wf);
    return hip_check(hipGetLastError(), "weight kernel launch");
}

zp_status launch_mode_norm(const Plan &plan, int64_t B, double *c, hipStream_t s)
{
    if (plan.chains.empty() || B == 0) return ZP_OK;
    const int64_t by = (B + kThreads - 1) / kThreads;
    if (by > 65535) return set_error(ZP_ERR_ARG, "B too large for one launch");
    const dim3 grid((unsigned)plan.chains.size(), (unsigned)by);
    hipLaunchKernelGGL(norm_kernel, grid, dim3(kThreads), 0, s, plan.d_chains, plan.d_emits, B, c);
    return hip_check(hipGetLastError(), "mode norm kernel launch");
}

} // namespace zp
