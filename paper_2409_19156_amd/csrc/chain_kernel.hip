// Radial Zernike polynomials, their r-derivatives and the full Zernike basis
// on gfx950 (MI355X).
//
// Work decomposition: one lane per point, one workgroup per (256-point tile,
// recurrence chain).  A chain is one alpha = |m| (Algorithm 1 of the paper:
// the chain P_k^{(alpha,0)}, k = 0..Kmax, serves every requested n of that
// alpha).  Every lane of a workgroup walks the same chain in lock step, so
// the per-step coefficients are wave-uniform; they are staged in LDS and read
// as broadcasts.  Each requested (n, m) on the chain is emitted when the walk
// reaches its degree K = (n - alpha)/2: the lane assembles R and its
// r-derivatives, applies the angular factor, and stores.  For a fixed column
// the 64 lanes of a wave store 64 consecutive points: 512 contiguous bytes
// per FP64 store instruction, marked non-temporal because outputs are not
// re-read by this kernel.
//
// Arithmetic: the endpoint-anchored difference form of the beta = 0 Jacobi
// recurrence (see zp_internal.hpp) with the derivatives with respect to
// s carried alongside:
//   d_k^(i) = cc_k d_{k-1}^(i) - bs_k (i v_{k-1}^(i-1) + s v_{k-1}^(i)),
//   v_k^(i) = v_{k-1}^(i) + d_k^(i).
// A lane takes the low anchor (s = 2r^2) when r^2 < 1/2 and the high anchor
// (s = 2(1 - r^2), formed by one fused multiply-add) otherwise, so s <= 1.
// Assembly at degree K (Eq. jacobi-relation, chain rule through s(r), and
// Leibniz on r^alpha):
//   g = v(s(r)):  g' = s' v',  g'' = s'^2 v'' + s'' v',  g''' = s'^3 v''' + 3 s' s'' v''
//   with s' = +-4r, s'' = +-4 (low/high),
//   d^j R / dr^j = A * sum_i C(j,i) [alpha!/(alpha-i)! r^(alpha-i)] g^(j-i),
//   A = (-1)^K C(K+alpha, K) (low) or 1 (high).
#include <hip/hip_runtime.h>

#include <climits>

#include "zp_internal.hpp"

namespace zp {
namespace {

constexpr int kBlock = 256;     // points per workgroup (4 waves)
constexpr int kTabChunk = 256;  // recurrence steps staged in LDS at a time

__device__ __forceinline__ uint16_t bf16_rne(float f)
{
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ double bf16_to_double(uint16_t h)
{
    return (double)__uint_as_float((uint32_t)h << 16);
}

__device__ __forceinline__ void store_plane(const Planes &o, int q, int64_t idx, double v)
{
    switch (o.fmt[q]) {
    case F64:
        __builtin_nontemporal_store(v, (double *)o.plane[q] + idx);
        break;
    case F32:
        __builtin_nontemporal_store((float)v, (float *)o.plane[q] + idx);
        break;
    default: { // B16X3: v ~ hi + mid + lo, residuals exact in FP64
        uint16_t *b = (uint16_t *)o.plane[q] + idx;
        const uint16_t h = bf16_rne((float)v);
        const double r1 = v - bf16_to_double(h);
        const uint16_t md = bf16_rne((float)r1);
        const double r2 = r1 - bf16_to_double(md);
        const uint16_t l = bf16_rne((float)r2);
        __builtin_nontemporal_store(h, b);
        __builtin_nontemporal_store(md, b + o.sub);
        __builtin_nontemporal_store(l, b + 2 * o.sub);
        break;
    }
    }
}

// x^e for e >= 0 by binary powering (about 2 log2(e) roundings).
__device__ __forceinline__ double ipow(double x, int e)
{
    double acc = 1.0;
    while (e) {
        if (e & 1) acc *= x;
        x *= x;
        e >>= 1;
    }
    return acc;
}

template <int J, bool ANG>
__global__ __launch_bounds__(kBlock) void chain_kernel(const Chain *__restrict__ chains,
                                                       const Coef *__restrict__ coefs,
                                                       const Emit *__restrict__ emits,
                                                       const double *__restrict__ r,
                                                       const double *__restrict__ theta, int64_t P,
                                                       Planes out)
{
    __shared__ Coef tab[kTabChunk];

    const Chain ch = chains[blockIdx.y];
    const int alpha = ch.alpha;
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const bool live = p < P;
    const double x = live ? r[p] : 0.0;

    // Anchor and s(r).
    const double x2 = x * x;
    const bool high = !(x2 < 0.5);
    const double s = high ? __builtin_fma(-2.0 * x, x, 2.0) : 2.0 * x2;
    const double s1 = high ? -4.0 * x : 4.0 * x; // ds/dr
    const double s2 = high ? -4.0 : 4.0;         // d2s/dr2

    // w[i] = d^i/dr^i r^alpha = alpha!/(alpha-i)! r^(alpha-i), 0 for i > alpha.
    // Each w[i] is formed the same way whatever J is, so every output
    // selection gives bitwise identical values.
    double w[J + 1];
#pragma unroll
    for (int i = 0; i <= J; ++i) {
        if (i > alpha) {
            w[i] = 0.0;
            continue;
        }
        double f = 1.0;
        for (int t = 0; t < i; ++t) f *= (double)(alpha - t);
        w[i] = f * ipow(x, alpha - i);
    }

    double cs = 0.0, sn = 0.0;
    if (ANG) {
        const double th = live ? theta[p] : 0.0;
        // alpha * theta split exactly into ph + pe; then one first-order
        // correction of sincos(ph) for the tail pe.
        const double fa = (double)alpha;
        const double ph = fa * th;
        const double pe = __builtin_fma(fa, th, -ph);
        double s0, c0;
        sincos(ph, &s0, &c0);
        sn = __builtin_fma(pe, c0, s0);
        cs = __builtin_fma(-pe, s0, c0);
    }

    double v[J + 1], d[J + 1];
#pragma unroll
    for (int i = 0; i <= J; ++i) {
        v[i] = i == 0 ? 1.0 : 0.0;
        d[i] = 0.0;
    }

    const int e_end = ch.emit_off + ch.emit_cnt;
    int e = ch.emit_off;
    int nextK = e < e_end ? emits[e].K : INT_MAX;

    auto emit_all = [&](int k) {
        while (nextK == k) {
            const Emit em = emits[e];
            ++e;
            nextK = e < e_end ? emits[e].K : INT_MAX;
            // g^(j) = d^j/dr^j v(s(r))
            double g[J + 1];
            g[0] = v[0];
            if (J >= 1) g[1] = s1 * v[1];
            if (J >= 2) g[2] = __builtin_fma(s1 * s1, v[2], s2 * v[1]);
            if (J >= 3) g[3] = __builtin_fma(s1 * s1 * s1, v[3], 3.0 * s1 * s2 * v[2]);
            const double A = high ? 1.0 : em.a_lo;
            double R[J + 1];
            R[0] = A * (w[0] * g[0]);
            if (J >= 1) R[1] = A * __builtin_fma(w[0], g[1], w[1] * g[0]);
            if (J >= 2) R[2] = A * (__builtin_fma(w[0], g[2], 2.0 * w[1] * g[1]) + w[2] * g[0]);
            if (J >= 3)
                R[3] = A * (__builtin_fma(w[0], g[3], 3.0 * w[1] * g[2]) + __builtin_fma(3.0 * w[2], g[1], w[3] * g[0]));
            if (!live) continue;
            const int64_t idx = (int64_t)em.col * out.ld + p;
            const bool is_sin = em.flags & 1;
            const double fac = ANG ? (is_sin ? sn : cs) : 1.0;
#pragma unroll
            for (int q = 0; q <= J; ++q)
                if (out.plane[q]) store_plane(out, q, idx, ANG ? R[q] * fac : R[q]);
            if (ANG && out.plane[4]) {
                // d/dtheta of R cos(m theta) = -m R sin(m theta) (m >= 0);
                // of R sin(|m| theta) = |m| R cos(|m| theta) (m < 0).
                const double fa = (double)alpha;
                store_plane(out, 4, idx, is_sin ? fa * R[0] * cs : -fa * R[0] * sn);
            }
        }
    };

    emit_all(0);
    for (int k0 = 1; k0 <= ch.kmax; k0 += kTabChunk) {
        const int cnt = min(kTabChunk, ch.kmax - k0 + 1);
        __syncthreads();
        for (int t = threadIdx.x; t < cnt; t += kBlock) tab[t] = coefs[ch.coef_off + (k0 - 1) + t];
        __syncthreads();
        for (int kk = 0; kk < cnt; ++kk) {
            const Coef cf = tab[kk];
            const double cc = high ? cf.cc_hi : cf.cc_lo;
            const double bs = high ? cf.bs_hi : cf.bs_lo;
            // All d use the step k-1 values of v; then v advances.
#pragma unroll
            for (int i = J; i >= 1; --i) {
                const double t = __builtin_fma(s, v[i], (double)i * v[i - 1]);
                d[i] = __builtin_fma(cc, d[i], -bs * t);
            }
            d[0] = __builtin_fma(cc, d[0], -bs * (s * v[0]));
#pragma unroll
            for (int i = 0; i <= J; ++i) v[i] += d[i];
            emit_all(k0 + kk);
        }
    }
}

template <int J, bool ANG>
hipError_t launch(const Plan &plan, const double *r, const double *th, int64_t P, const Planes &o, hipStream_t s)
{
    const dim3 grid((unsigned)((P + kBlock - 1) / kBlock), (unsigned)plan.chains.size());
    hipLaunchKernelGGL((chain_kernel<J, ANG>), grid, dim3(kBlock), 0, s, plan.d_chains, plan.d_coefs,
                       plan.d_emits, r, th, P, o);
    return hipGetLastError();
}

} // namespace

zp_status launch_chain_kernel(const Plan &plan, const double *d_r, const double *d_theta, int64_t P, int J,
                              bool angular, const Planes &out, hipStream_t s)
{
    if (P <= 0 || plan.chains.empty()) return ZP_OK;
    if ((P + kBlock - 1) / kBlock > (int64_t)INT_MAX) return set_error(ZP_ERR_ARG, "too many points for one launch");
    hipError_t e;
    if (angular) {
        switch (J) {
        case 0: e = launch<0, true>(plan, d_r, d_theta, P, out, s); break;
        case 1: e = launch<1, true>(plan, d_r, d_theta, P, out, s); break;
        case 2: e = launch<2, true>(plan, d_r, d_theta, P, out, s); break;
        default: e = launch<3, true>(plan, d_r, d_theta, P, out, s); break;
        }
    } else {
        switch (J) {
        case 0: e = launch<0, false>(plan, d_r, nullptr, P, out, s); break;
        case 1: e = launch<1, false>(plan, d_r, nullptr, P, out, s); break;
        case 2: e = launch<2, false>(plan, d_r, nullptr, P, out, s); break;
        default: e = launch<3, false>(plan, d_r, nullptr, P, out, s); break;
        }
    }
    return hip_check(e, "chain_kernel launch");
}

} // namespace zp
