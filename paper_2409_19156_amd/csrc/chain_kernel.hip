// Radial Zernike polynomials, their r-derivatives and the full Zernike basis
// on gfx950 (MI355X).
//
// Work decomposition: one lane per point (two adjacent points per lane when
// every output plane is FP64), one workgroup (256 lanes) per (point tile,
// recurrence chain).  A chain is one alpha = |m| (Algorithm 1 of the paper:
// the chain P_k^{(alpha,0)}, k = 0..Kmax, serves every requested n of that
// alpha).  Every lane of a workgroup walks the same chain in lock step, so
// the per-step coefficients are wave-uniform; they are staged in LDS and read
// as broadcasts.  Each requested (n, m) on the chain is emitted when the walk
// reaches its degree K = (n - alpha)/2: the lane assembles R and its
// r-derivatives, applies the angular factor, and stores.  For a fixed column
// the 64 lanes of a wave store 128 consecutive points: 1 KB contiguous per
// store instruction (16 bytes per lane), marked non-temporal because outputs
// are not re-read by this kernel.
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

typedef uint32_t u4 __attribute__((ext_vector_type(4)));

// v ~ hi + mid + lo as three bf16 values; the residuals are exact in FP64.
__device__ __forceinline__ void split3(double v, uint16_t &h, uint16_t &m, uint16_t &l)
{
    h = bf16_rne((float)v);
    const double r1 = v - bf16_to_double(h);
    m = bf16_rne((float)r1);
    const double r2 = r1 - bf16_to_double(m);
    l = bf16_rne((float)r2);
}

__device__ __forceinline__ void store_fmt(void *base, int fmt, int64_t sub, int64_t idx, double v)
{
    switch (fmt) {
    case F64:
        __builtin_nontemporal_store(v, (double *)base + idx);
        break;
    case F32:
        __builtin_nontemporal_store((float)v, (float *)base + idx);
        break;
    default: { // B16X3
        uint16_t *b = (uint16_t *)base + idx;
        uint16_t h, md, l;
        split3(v, h, md, l);
        __builtin_nontemporal_store(h, b);
        __builtin_nontemporal_store(md, b + sub);
        __builtin_nontemporal_store(l, b + 2 * sub);
        break;
    }
    }
}

__device__ __forceinline__ void store_plane(const Planes &o, int q, int64_t idx, double v)
{
    store_fmt(o.plane[q], o.fmt[q], o.sub, idx, v);
}

// One k-blocked bf16 group register (8 emissions x 16 bits per plane); see
// the kernel for how groups are formed.
template <int NW>
__device__ __forceinline__ void kb_push(uint32_t (&w)[NW][4], double val, uint16_t *kb, int64_t kb_sub, int eidx,
                                        bool full_group)
{
    uint16_t hv[3];
    split3(val, hv[0], hv[1], hv[2]);
    if (full_group) {
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            uint32_t *x4 = w[q < NW ? q : 0];
            x4[0] = __builtin_amdgcn_alignbit(x4[1], x4[0], 16);
            x4[1] = __builtin_amdgcn_alignbit(x4[2], x4[1], 16);
            x4[2] = __builtin_amdgcn_alignbit(x4[3], x4[2], 16);
            x4[3] = (x4[3] >> 16) | ((uint32_t)hv[q] << 16);
        }
        if ((eidx & 7) == 7) {
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                const uint32_t *x4 = w[q < NW ? q : 0];
                const u4 vv = {x4[0], x4[1], x4[2], x4[3]};
                __builtin_nontemporal_store(vv, (u4 *)(kb + q * kb_sub));
            }
        }
    } else {
        // groups shared with another chain piece: the two workgroups write
        // different bytes of the same 16-byte blocks; plain stores let L2
        // merge them before the lines go to memory
#pragma unroll
        for (int q = 0; q < 3; ++q) kb[q * kb_sub + (eidx & 7)] = hv[q];
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

typedef double d2 __attribute__((ext_vector_type(2)));

// NPL points per lane (1, or 2 for FP64-only outputs: each store then writes
// 16 bytes per lane, 1 KB per wave).  POLAR: the points are a tensor grid,
// point p = i * nt + j at radius r[i] and angle theta[j]; with two points per
// lane (nt even) both lie on one radius, and the lane's radial recurrence
// (the state sized RS below) runs once for both.  Every value is formed
// exactly as for the same point given as (r_p, theta_p).
template <int J, bool ANG, bool KB, int NPL, bool DIR, bool SEC, bool POLAR>
__global__ __launch_bounds__(kBlock) void chain_kernel(const Chain *__restrict__ chains,
                                                       const Coef *__restrict__ coefs,
                                                       const Emit *__restrict__ emits,
                                                       const double *__restrict__ r,
                                                       const double *__restrict__ theta, int64_t P,
                                                       Planes out, int64_t nt)
{
    static_assert(NPL == 1 || (NPL == 2 && !KB), "two points per lane only for plain FP64 planes");
    static_assert(!DIR || (ANG && J >= 1), "the directional derivative needs the basis and dZ/dr");
    static_assert(!SEC || (DIR && J >= 2 && NPL == 1 && !KB), "second-order planes need d2Z/dr2, one point per lane");
    static_assert(!POLAR || (ANG && !KB && !DIR), "polar grids: plain basis planes");
    constexpr int RS = POLAR ? 1 : NPL; // radial states per lane
    __shared__ Coef tab[kTabChunk];

    const Chain ch = chains[blockIdx.y];
    const int alpha = ch.alpha;
    const int64_t p0 = ((int64_t)blockIdx.x * kBlock + threadIdx.x) * NPL;
    // polar: radius row and first angle of the lane's points (nt even, p0 even)
    const int64_t prow = POLAR ? p0 / nt : 0, pcol = POLAR ? p0 - prow * nt : 0;

    bool live[NPL], high[RS];
    double x[RS], s[RS], s1[RS], s2[RS], cs[NPL], sn[NPL], tr[NPL], tt[NPL];
    double w[RS][J + 1], v[RS][J + 1], d[RS][J + 1];
#pragma unroll
    for (int u = 0; u < NPL; ++u) {
        live[u] = p0 + u < P;
        tr[u] = (DIR && live[u] && out.dir_r) ? out.dir_r[p0 + u] : 0.0;  // tangent of r
        tt[u] = (DIR && live[u] && out.dir_th) ? out.dir_th[p0 + u] : 0.0; // tangent of theta
    }
#pragma unroll
    for (int u = 0; u < RS; ++u) {
        x[u] = !live[u] ? 0.0 : POLAR ? r[prow] : r[p0 + u];
        // Anchor and s(r), ds/dr, d2s/dr2.
        const double x2 = x[u] * x[u];
        high[u] = !(x2 < 0.5);
        s[u] = high[u] ? __builtin_fma(-2.0 * x[u], x[u], 2.0) : 2.0 * x2;
        s1[u] = high[u] ? -4.0 * x[u] : 4.0 * x[u];
        s2[u] = high[u] ? -4.0 : 4.0;
        // w[i] = d^i/dr^i r^alpha = alpha!/(alpha-i)! r^(alpha-i), 0 for
        // i > alpha.  Each w[i] is formed the same way whatever J is, so
        // every output selection gives bitwise identical values.
#pragma unroll
        for (int i = 0; i <= J; ++i) {
            if (i > alpha) {
                w[u][i] = 0.0;
                continue;
            }
            double f = 1.0;
            for (int t = 0; t < i; ++t) f *= (double)(alpha - t);
            w[u][i] = f * ipow(x[u], alpha - i);
        }
#pragma unroll
        for (int i = 0; i <= J; ++i) {
            v[u][i] = i == 0 ? 1.0 : 0.0;
            d[u][i] = 0.0;
        }
    }
#pragma unroll
    for (int u = 0; u < NPL; ++u) {
        cs[u] = 0.0;
        sn[u] = 0.0;
        if (ANG) {
            const double th = live[u] ? (POLAR ? theta[pcol + u] : theta[p0 + u]) : 0.0;
            // alpha * theta split exactly into ph + pe; then one first-order
            // correction of sincos(ph) for the tail pe.
            const double fa = (double)alpha;
            const double ph = fa * th;
            const double pe = __builtin_fma(fa, th, -ph);
            double s0, c0;
            sincos(ph, &s0, &c0);
            sn[u] = __builtin_fma(pe, c0, s0);
            cs[u] = __builtin_fma(-pe, s0, c0);
        }
    }

    const int e_end = ch.emit_off + ch.emit_cnt;
    int e = ch.emit_off;
    int nextK = e < e_end ? emits[e].K : INT_MAX;

    // Staging for the k-blocked bf16 copy of Z: a 128-bit shift register per
    // plane collects the eight emissions of a group that lies wholly on this
    // chain piece; groups that straddle a boundary are stored element-wise.
    uint32_t kbw[3][4] = {};
    uint32_t kbd[DIR ? 3 : 1][4] = {};

    auto emit_all = [&](int k) {
        while (nextK == k) {
            const int eidx = e;
            const Emit em = emits[e];
            ++e;
            nextK = e < e_end ? emits[e].K : INT_MAX;
            const bool is_sin = em.flags & 1;
            double val[5][NPL], vdir[NPL], vsr[NPL], vst[NPL];
            // d^j R / dr^j of each radial state
            double Rs[RS][J + 1];
#pragma unroll
            for (int u = 0; u < RS; ++u) {
                // g^(j) = d^j/dr^j v(s(r))
                double g[J + 1];
                g[0] = v[u][0];
                if (J >= 1) g[1] = s1[u] * v[u][1];
                if (J >= 2) g[2] = __builtin_fma(s1[u] * s1[u], v[u][2], s2[u] * v[u][1]);
                if (J >= 3) g[3] = __builtin_fma(s1[u] * s1[u] * s1[u], v[u][3], 3.0 * s1[u] * s2[u] * v[u][2]);
                const double A = high[u] ? 1.0 : em.a_lo;
                const double *wu = w[u];
                double *R = Rs[u];
                R[0] = A * (wu[0] * g[0]);
                if (J >= 1) R[1] = A * __builtin_fma(wu[0], g[1], wu[1] * g[0]);
                if (J >= 2) R[2] = A * (__builtin_fma(wu[0], g[2], 2.0 * wu[1] * g[1]) + wu[2] * g[0]);
                if (J >= 3)
                    R[3] = A * (__builtin_fma(wu[0], g[3], 3.0 * wu[1] * g[2]) +
                                __builtin_fma(3.0 * wu[2], g[1], wu[3] * g[0]));
            }
#pragma unroll
            for (int u = 0; u < NPL; ++u) {
                const double *R = Rs[POLAR ? 0 : u];
                const double fac = ANG ? (is_sin ? sn[u] : cs[u]) : 1.0;
#pragma unroll
                for (int q = 0; q <= J; ++q) val[q][u] = ANG ? R[q] * fac : R[q];
                // d/dtheta of R cos(m theta) = -m R sin(m theta) (m >= 0);
                // of R sin(|m| theta) = |m| R cos(|m| theta) (m < 0).
                const double fa = (double)alpha;
                val[4][u] = ANG ? (is_sin ? fa * R[0] * cs[u] : -fa * R[0] * sn[u]) : 0.0;
                vdir[u] = DIR ? __builtin_fma(tr[u], val[J >= 1 ? 1 : 0][u], tt[u] * val[4][u]) : 0.0;
                if (SEC) {
                    // d2Z/(dr dtheta) = d/dtheta of R' cos|sin; d2Z/dtheta2 = -m^2 Z
                    const double zrt = is_sin ? fa * R[J >= 1 ? 1 : 0] * cs[u] : -fa * R[J >= 1 ? 1 : 0] * sn[u];
                    const double ztt = -fa * fa * val[0][u];
                    vsr[u] = __builtin_fma(tr[u], val[J >= 2 ? 2 : 0][u], tt[u] * zrt);
                    vst[u] = __builtin_fma(tr[u], zrt, tt[u] * ztt);
                } else {
                    vsr[u] = vst[u] = 0.0;
                }
            }
            const int64_t idx = (int64_t)em.col * out.ld + p0;
            if (NPL == 2) {
                // planes are FP64 here; a pair of points is 16 bytes, aligned
                // because ld and p0 are even
#pragma unroll
                for (int q = 0; q < 6; ++q) {
                    void *base = q < 5 ? out.plane[q] : out.dir;
                    if ((q > J && q < 4) || (q == 4 && !ANG) || (q == 5 && !DIR) || !base) continue;
                    const double *vq = q < 5 ? val[q] : vdir;
                    double *dst = (double *)base + idx;
                    if (live[NPL - 1]) {
                        const d2 pair = {vq[0], vq[NPL - 1]};
                        __builtin_nontemporal_store(pair, (d2 *)dst);
                    } else if (live[0]) {
                        __builtin_nontemporal_store(vq[0], dst);
                    }
                }
                continue;
            }
            if (!live[0]) continue;
#pragma unroll
            for (int q = 0; q <= J; ++q)
                if (out.plane[q]) store_plane(out, q, idx, val[q][0]);
            if (ANG && out.plane[4]) store_plane(out, 4, idx, val[4][0]);
            // the series' bf16 path keeps only the k-blocked copy (out.dir null)
            if (DIR && out.dir) store_fmt(out.dir, out.dir_fmt, out.sub, idx, vdir[0]);
            if (SEC && out.sec_r) store_fmt(out.sec_r, out.sec_fmt, out.sub, idx, vsr[0]);
            if (SEC && out.sec_t) store_fmt(out.sec_t, out.sec_fmt, out.sub, idx, vst[0]);
            if (KB) {
                const int g8 = eidx & ~7;
                const bool full = g8 >= ch.emit_off && g8 + 8 <= e_end;
                const int64_t off = ((int64_t)(eidx >> 3) * out.kb_ld + p0) * 8;
                if (out.kb) kb_push(kbw, val[0][0], (uint16_t *)out.kb + off, out.kb_sub, eidx, full);
                if (DIR && out.kb_dir) kb_push(kbd, vdir[0], (uint16_t *)out.kb_dir + off, out.kb_sub, eidx, full);
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
#pragma unroll
            for (int u = 0; u < RS; ++u) {
                const double cc = high[u] ? cf.cc_hi : cf.cc_lo;
                const double bs = high[u] ? cf.bs_hi : cf.bs_lo;
                // All d use the step k-1 values of v; then v advances.
#pragma unroll
                for (int i = J; i >= 1; --i) {
                    const double t = __builtin_fma(s[u], v[u][i], (double)i * v[u][i - 1]);
                    d[u][i] = __builtin_fma(cc, d[u][i], -bs * t);
                }
                d[u][0] = __builtin_fma(cc, d[u][0], -bs * (s[u] * v[u][0]));
#pragma unroll
                for (int i = 0; i <= J; ++i) v[u][i] += d[u][i];
            }
            emit_all(k0 + kk);
        }
    }
}

// Workgroups wanted before whole chains are cut into pieces: a few per
// resident slot on 256 CUs, so the heaviest chains do not form a tail.
constexpr int64_t kMinWorkgroups = 8192;

template <int J, bool ANG, bool KB, int NPL, bool DIR = false, bool SEC = false, bool POLAR = false>
hipError_t launch(const Plan &plan, const double *r, const double *th, int64_t P, const Planes &o, hipStream_t s,
                  int64_t nt = 0)
{
    const int64_t tiles = (P + (int64_t)kBlock * NPL - 1) / ((int64_t)kBlock * NPL);
    // pieces when whole chains give too few workgroups, and while their count
    // fits the grid's second dimension (chains: at most ZP_N_MAX + 1)
    const bool use_pieces = tiles * (int64_t)plan.chains.size() < kMinWorkgroups && plan.pieces.size() <= 65535;
    const Chain *list = use_pieces ? plan.d_pieces : plan.d_chains;
    const size_t count = use_pieces ? plan.pieces.size() : plan.chains.size();
    const dim3 grid((unsigned)tiles, (unsigned)count);
    hipLaunchKernelGGL((chain_kernel<J, ANG, KB, NPL, DIR, SEC, POLAR>), grid, dim3(kBlock), 0, s, list, plan.d_coefs,
                       plan.d_emits, r, th, P, o, nt);
    return hipGetLastError();
}

template <int J, bool ANG, bool DIR = false>
hipError_t launch_npl(const Plan &plan, const double *r, const double *th, int64_t P, const Planes &o, hipStream_t s)
{
    bool all_f64 = !DIR || o.dir_fmt == F64;
    for (int q = 0; q < 5; ++q)
        if (o.plane[q] && o.fmt[q] != F64) all_f64 = false;
    if (all_f64 && (o.ld % 2) == 0) return launch<J, ANG, false, 2, DIR>(plan, r, th, P, o, s);
    return launch<J, ANG, false, 1, DIR>(plan, r, th, P, o, s);
}

} // namespace

zp_status launch_chain_kernel_polar(const Plan &plan, const double *d_r, int64_t nr, const double *d_theta, int64_t nt,
                                    int J, const Planes &out, hipStream_t s)
{
    const int64_t P = nr * nt;
    if (P <= 0 || plan.chains.empty()) return ZP_OK;
    if ((P + kBlock - 1) / kBlock > (int64_t)INT_MAX) return set_error(ZP_ERR_ARG, "too many points for one launch");
    bool all_f64 = true;
    for (int q = 0; q < 5; ++q)
        if (out.plane[q] && out.fmt[q] != F64) all_f64 = false;
    if (out.kb || out.dir || out.kb_dir || out.sec_r || out.sec_t || J < 0 || J > 3)
        return set_error(ZP_ERR_ARG, "internal: polar grids take plain basis planes");
    const bool two = all_f64 && (nt % 2) == 0; // a lane's two points then share their radius
    hipError_t e;
    switch (J) {
    case 0:
        e = two ? launch<0, true, false, 2, false, false, true>(plan, d_r, d_theta, P, out, s, nt)
                : launch<0, true, false, 1, false, false, true>(plan, d_r, d_theta, P, out, s, nt);
        break;
    case 1:
        e = two ? launch<1, true, false, 2, false, false, true>(plan, d_r, d_theta, P, out, s, nt)
                : launch<1, true, false, 1, false, false, true>(plan, d_r, d_theta, P, out, s, nt);
        break;
    case 2:
        e = two ? launch<2, true, false, 2, false, false, true>(plan, d_r, d_theta, P, out, s, nt)
                : launch<2, true, false, 1, false, false, true>(plan, d_r, d_theta, P, out, s, nt);
        break;
    default:
        e = two ? launch<3, true, false, 2, false, false, true>(plan, d_r, d_theta, P, out, s, nt)
                : launch<3, true, false, 1, false, false, true>(plan, d_r, d_theta, P, out, s, nt);
        break;
    }
    return hip_check(e, "chain_kernel launch");
}

zp_status launch_chain_kernel(const Plan &plan, const double *d_r, const double *d_theta, int64_t P, int J,
                              bool angular, const Planes &out, hipStream_t s)
{
    if (P <= 0 || plan.chains.empty()) return ZP_OK;
    if ((P + kBlock - 1) / kBlock > (int64_t)INT_MAX) return set_error(ZP_ERR_ARG, "too many points for one launch");
    hipError_t e;
    const bool dir = out.dir || out.kb_dir;
    const bool sec = out.sec_r || out.sec_t;
    if (sec) { // second-order planes (with the plain planes and dir): J = 2, one point per lane
        if (!angular || J != 2 || out.kb || out.kb_dir)
            return set_error(ZP_ERR_ARG, "internal: second-order output needs the basis, J = 2, no k-blocked copy");
        e = launch<2, true, false, 1, true, true>(plan, d_r, d_theta, P, out, s);
        return hip_check(e, "chain_kernel launch");
    }
    if (dir && (!angular || J != 1)) return set_error(ZP_ERR_ARG, "internal: directional output needs the basis, J = 1");
    if (out.kb || out.kb_dir) { // series: k-blocked copies of Z and / or its directional derivative
        if (!angular || J > 1) return set_error(ZP_ERR_ARG, "internal: k-blocked output needs the basis, J <= 1");
        if (dir)
            e = launch<1, true, true, 1, true>(plan, d_r, d_theta, P, out, s);
        else
            e = J == 0 ? launch<0, true, true, 1>(plan, d_r, d_theta, P, out, s)
                       : launch<1, true, true, 1>(plan, d_r, d_theta, P, out, s);
    } else if (dir) {
        e = launch_npl<1, true, true>(plan, d_r, d_theta, P, out, s);
    } else if (angular) {
        switch (J) {
        case 0: e = launch_npl<0, true>(plan, d_r, d_theta, P, out, s); break;
        case 1: e = launch_npl<1, true>(plan, d_r, d_theta, P, out, s); break;
        case 2: e = launch_npl<2, true>(plan, d_r, d_theta, P, out, s); break;
        default: e = launch_npl<3, true>(plan, d_r, d_theta, P, out, s); break;
        }
    } else {
        switch (J) {
        case 0: e = launch_npl<0, false>(plan, d_r, nullptr, P, out, s); break;
        case 1: e = launch_npl<1, false>(plan, d_r, nullptr, P, out, s); break;
        case 2: e = launch_npl<2, false>(plan, d_r, nullptr, P, out, s); break;
        default: e = launch_npl<3, false>(plan, d_r, nullptr, P, out, s); break;
        }
    }
    return hip_check(e, "chain_kernel launch");
}

} // namespace zp
