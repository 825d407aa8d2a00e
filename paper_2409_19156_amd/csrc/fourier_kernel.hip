// Fourier factors of the three-dimensional spectral series (the paper's
// duplicated-mode use, Sec. 3 footnote) and the mixing of coefficients
// between the full mode list (n, m, l) and its distinct (n, m) pairs.
//
// F_l(phi) = cos(l phi) for l >= 0 and sin(|l| phi) for l < 0, the same
// convention as the angular factor of Eq. zernike-poly.  These kernels touch
// O(J (Q + B) + U Q B) values, small next to the basis and the contraction
// over points, so they are plain FP64 kernels.
#include <hip/hip_runtime.h>

#include "series3d.hpp"

namespace zp {
namespace {

constexpr int kThreads = 256;

// F_l(phi), or dF_l/dphi.  |l| * phi is split exactly into ph + pe (|l| is
// at most 2^20, so the FMA residual is exact); sincos(ph) then takes a
// first-order correction for pe.
__device__ __forceinline__ double fourier(int l, double phi, bool deriv)
{
    const double fa = (double)(l < 0 ? -l : l);
    const double ph = fa * phi;
    const double pe = __builtin_fma(fa, phi, -ph);
    double s0, c0;
    sincos(ph, &s0, &c0);
    const double sn = __builtin_fma(pe, c0, s0);
    const double cs = __builtin_fma(-pe, s0, c0);
    if (!deriv) return l >= 0 ? cs : sn;
    return l >= 0 ? -fa * sn : fa * cs;
}

// grid: (ceil(Q*B / 256), min(U, 65535)); threads stride over pairs in y.
__global__ __launch_bounds__(kThreads) void mix_kernel(const int32_t *__restrict__ uptr,
                                                       const int32_t *__restrict__ jl, const int32_t *__restrict__ l,
                                                       const double *__restrict__ c, int64_t B,
                                                       const double *__restrict__ phi, int64_t QB, int64_t U,
                                                       bool deriv, double *__restrict__ T)
{
    const int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (e >= QB) return;
    const int64_t q = e / B, b = e - q * B;
    const double ph = phi[q];
    for (int64_t u = blockIdx.y; u < U; u += gridDim.y) {
        double acc = 0.0;
        for (int t = uptr[u]; t < uptr[u + 1]; ++t) {
            const int j = jl[t];
            acc = __builtin_fma(c[(int64_t)j * B + b], fourier(l[j], ph, deriv), acc);
        }
        T[u * QB + e] = acc;
    }
}

// One thread per (j, b).
__global__ __launch_bounds__(kThreads) void unmix_kernel(const int32_t *__restrict__ owner,
                                                         const int32_t *__restrict__ l,
                                                         const double *__restrict__ gT, int64_t B,
                                                         const double *__restrict__ phi, int64_t Q, int64_t J,
                                                         double *__restrict__ grad_c)
{
    const int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (t >= J * B) return;
    const int64_t j = t / B, b = t - j * B;
    const int lj = l[j];
    const double *row = gT + (int64_t)owner[j] * Q * B + b;
    double acc = 0.0;
    for (int64_t q = 0; q < Q; ++q) acc = __builtin_fma(fourier(lj, phi[q], false), row[q * B], acc);
    grad_c[t] = acc;
}

// One workgroup per q; lanes stride over modes j, then a fixed-order tree
// reduction in LDS.
__global__ __launch_bounds__(kThreads) void phi_grad_kernel(const int32_t *__restrict__ owner,
                                                            const int32_t *__restrict__ l,
                                                            const double *__restrict__ gT,
                                                            const double *__restrict__ c, int64_t B,
                                                            const double *__restrict__ phi, int64_t Q, int64_t J,
                                                            double *__restrict__ grad_phi)
{
    __shared__ double red[kThreads];
    const int64_t q = blockIdx.x;
    const double ph = phi[q];
    double acc = 0.0;
    for (int64_t j = threadIdx.x; j < J; j += kThreads) {
        const double *g = gT + ((int64_t)owner[j] * Q + q) * B;
        const double *cj = c + j * B;
        double s = 0.0;
        for (int64_t b = 0; b < B; ++b) s = __builtin_fma(cj[b], g[b], s);
        acc = __builtin_fma(fourier(l[j], ph, true), s, acc);
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = kThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) grad_phi[q] = red[0];
}

} // namespace

zp_status launch_fourier_mix(const Plan3 &p, const double *c, int64_t B, const double *phi, int64_t Q, bool deriv,
                             double *T, hipStream_t s)
{
    const int64_t U = (int64_t)p.un.size(), QB = Q * B;
    if (U == 0 || QB == 0) return ZP_OK;
    const int64_t bx = (QB + kThreads - 1) / kThreads;
    if (bx > INT32_MAX) return set_error(ZP_ERR_ARG, "Q * B too large for one launch");
    const dim3 grid((unsigned)bx, (unsigned)std::min<int64_t>(U, 65535));
    hipLaunchKernelGGL(mix_kernel, grid, dim3(kThreads), 0, s, p.d_uptr, p.d_jl, p.d_l, c, B, phi, QB, U, deriv, T);
    return hip_check(hipGetLastError(), "fourier mix launch");
}

zp_status launch_fourier_unmix(const Plan3 &p, const double *gT, int64_t B, const double *phi, int64_t Q,
                               double *grad_c, hipStream_t s)
{
    const int64_t J = (int64_t)p.n.size();
    if (J == 0 || B == 0) return ZP_OK;
    const int64_t bx = (J * B + kThreads - 1) / kThreads;
    if (bx > INT32_MAX) return set_error(ZP_ERR_ARG, "J * B too large for one launch");
    hipLaunchKernelGGL(unmix_kernel, dim3((unsigned)bx), dim3(kThreads), 0, s, p.d_owner, p.d_l, gT, B, phi, Q, J,
                       grad_c);
    return hip_check(hipGetLastError(), "fourier unmix launch");
}

zp_status launch_fourier_phi_grad(const Plan3 &p, const double *gT, const double *c, int64_t B, const double *phi,
                                  int64_t Q, double *grad_phi, hipStream_t s)
{
    const int64_t J = (int64_t)p.n.size();
    if (Q == 0) return ZP_OK;
    if (Q > INT32_MAX) return set_error(ZP_ERR_ARG, "Q too large for one launch");
    hipLaunchKernelGGL(phi_grad_kernel, dim3((unsigned)Q), dim3(kThreads), 0, s, p.d_owner, p.d_l, gT, c, B, phi, Q,
                       J, grad_phi);
    return hip_check(hipGetLastError(), "fourier phi-gradient launch");
}

} // namespace zp
