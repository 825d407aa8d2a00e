// Analysis transform: Zernike coefficients from samples of a function on the
// unit disc by quadrature, the inverse of the series for band-limited data
// (the spectral-method use of the basis, Sec. 1).
//
// The basis is orthogonal over the disc with
//   integral of Z_k Z_k' dA = delta_kk' N_k,  N_k = eps_m pi / (2 (n + 1)),
// eps_m = 2 for m = 0 and 1 otherwise (the radial orthogonality integral
// 1 / (2(n+1)) times the angular one, 2 pi or pi).  With a quadrature rule
// (r_p, theta_p, w_p) that integrates every product Z_k f exactly,
//   c_k = (1 / N_k) sum_p w_p Z_k(p) f(p).
// On the device this is the series' adjoint contraction dL/dc = Z g with
// g = w * f, followed by the division by N_k.
//
// zp_analysis_grid builds such a rule for modes with n <= L: Gauss-Legendre
// in t = r^2 (R_n^m R_n'^m r dr is a polynomial of degree (n + n')/2 <= L in
// t times dt/2, so ceil((L+1)/2) nodes are exact) times the trapezoidal rule
// with at least 2L+1 equispaced angles (exact for cos(k theta), |k| <= 2L).
#include <cmath>

#include "series.hpp"

namespace zp {
zp_status check_modes_arg(const int32_t *n, const int32_t *m, int64_t M);
zp_status launch_weight(const double *w, const double *f, int64_t P, int64_t B, double *wf, hipStream_t s);
zp_status launch_mode_norm(const Plan &plan, int64_t B, double *c, hipStream_t s);
} // namespace zp

using namespace zp;

namespace {

// Gauss-Legendre rule on [-1, 1] with N nodes x_i = cos(phi_i), returned as
// r_i = sqrt((1 + x_i)/2) (ascending) and the weights w_i.  Newton's method
// runs on the angle phi (P_N(cos phi) = 0), started from the asymptotic
// estimate phi = pi (i + 3/4) / (N + 1/2), with the Legendre three-term
// recurrence in long double.  Working with the angle keeps the nodes next
// to x = -1 accurate: (1 + x)/2 = cos^2(phi/2) and (1 - x)/2 = sin^2(phi/2)
// need no cancelling subtraction.  w_i = 2 / (sin^2 phi_i P_N'(x_i)^2).
void gauss_legendre_r(int64_t N, std::vector<long double> &r, std::vector<long double> &w)
{
    r.assign((size_t)N, 0.0L);
    w.assign((size_t)N, 0.0L);
    const long double pi = 3.141592653589793238462643383279502884L;
    // returns P_N(z); dp = P_N'(z) = N (z P_N - P_{N-1}) / (z^2 - 1), z^2 - 1 = -sin^2
    auto legendre = [N](long double z, long double s2, long double &dp) {
        long double p0 = 1.0L, p1 = z;
        for (int64_t k = 2; k <= N; ++k) {
            const long double p2 = ((long double)(2 * k - 1) * z * p1 - (long double)(k - 1) * p0) / (long double)k;
            p0 = p1;
            p1 = p2;
        }
        dp = -(long double)N * (z * p1 - p0) / s2;
        return p1;
    };
    for (int64_t i = 0; i < (N + 1) / 2; ++i) {
        long double ph = pi * ((long double)i + 0.75L) / ((long double)N + 0.5L); // node cos(ph) > 0 side
        long double dp = 0.0L;
        for (int it = 0; it < 100; ++it) {
            const long double sn = std::sin(ph);
            const long double p = legendre(std::cos(ph), sn * sn, dp);
            const long double dph = p / (-sn * dp); // d/dphi P_N(cos phi) = -sin(phi) P_N'
            ph -= dph;
            if (std::fabs(dph) <= 1e-19L * ph) break;
        }
        const long double sn = std::sin(ph);
        legendre(std::cos(ph), sn * sn, dp);
        const long double wi = 2.0L / (sn * sn * dp * dp);
        r[(size_t)i] = std::sin(ph / 2.0L);         // x = -cos(ph): (1 + x)/2 = sin^2(ph/2)
        r[(size_t)(N - 1 - i)] = std::cos(ph / 2.0L); // x = +cos(ph): (1 + x)/2 = cos^2(ph/2)
        w[(size_t)i] = wi;
        w[(size_t)(N - 1 - i)] = wi;
    }
}

size_t al(size_t x) { return (x + 255) / 256 * 256; }

constexpr int64_t kMaxGridRadii = 4096;

} // namespace

extern "C" {

zp_status zp_analysis_grid(int64_t nr, int64_t nt, double *h_r, double *h_theta, double *h_w)
{
    if (nr < 1 || nt < 1) return set_error(ZP_ERR_ARG, "nr and nt must be positive");
    if (!h_r || !h_theta || !h_w) return set_error(ZP_ERR_ARG, "null pointer");
    // Newton's method with the O(nr) recurrence is O(nr^2) in all: nr <= 4096 keeps the rule below
    // ~0.1 s of host time and is exact up to n = 8191, beyond the largest degree the library accepts.
    if (nr > kMaxGridRadii || nt > (1 << 24)) return set_error(ZP_ERR_ARG, "grid too large");
    std::vector<long double> rr, w;
    gauss_legendre_r(nr, rr, w);
    const long double two_pi = 6.283185307179586476925286766559005768L;
    for (int64_t i = 0; i < nr; ++i) {
        // t = r^2 = (1 + x)/2: r dr = dt / 2 and dt = dx / 2; theta: 2 pi / nt
        const long double wr = w[(size_t)i] / 4.0L * (two_pi / (long double)nt);
        const double r = (double)rr[(size_t)i];
        for (int64_t j = 0; j < nt; ++j) {
            const int64_t p = i * nt + j;
            h_r[p] = r;
            h_theta[p] = (double)(two_pi * (long double)j / (long double)nt);
            h_w[p] = (double)wr;
        }
    }
    return ZP_OK;
}

zp_status zp_series_analysis_workspace(int64_t M, int64_t P, int64_t B, int32_t prec, size_t *full_bytes,
                                       size_t *min_bytes)
{
    if (M < 0 || P < 0 || B < 0) return set_error(ZP_ERR_ARG, "negative M, P or B");
    if (!full_bytes) return set_error(ZP_ERR_ARG, "null full_bytes");
    size_t f = 0, mn = 0;
    zp_status st = zp_series_workspace(M, P, B, prec, &f, &mn);
    if (st != ZP_OK) return st;
    const size_t head = al(8 * (size_t)P * (size_t)B);
    *full_bytes = head + f;
    if (min_bytes) *min_bytes = head + mn;
    return ZP_OK;
}

zp_status zp_series_analysis(const int32_t *h_n, const int32_t *h_m, int64_t M, const double *d_r,
                             const double *d_theta, const double *d_w, int64_t P, const double *d_f, int64_t B,
                             int32_t prec, double *d_c, void *d_ws, size_t ws_bytes, void *stream)
{
    zp_status st = check_modes_arg(h_n, h_m, M);
    if (st != ZP_OK) return st;
    if (P < 0 || B < 0) return set_error(ZP_ERR_ARG, "negative P or B");
    if (prec < ZP_FP64 || prec > ZP_BF16X3) return set_error(ZP_ERR_PREC, "prec must be ZP_FP64, ZP_FP32 or ZP_BF16X3");
    if (M == 0 || B == 0) return ZP_OK;
    if (!d_c) return set_error(ZP_ERR_ARG, "null pointer");
    hipStream_t s = (hipStream_t)stream;
    if (P == 0) // an empty quadrature: every coefficient is zero
        return launch_zero_pad(d_c, CT_F64, 0, 0, M, B, 0, s);
    if (!d_r || !d_theta || !d_w || !d_f) return set_error(ZP_ERR_ARG, "null pointer");
    if (!d_ws || ((uintptr_t)d_ws & 255)) return set_error(ZP_ERR_ARG, "workspace must be non-null and 256-byte aligned");
    size_t f = 0, mn = 0;
    st = zp_series_workspace(M, P, B, prec, &f, &mn);
    if (st != ZP_OK) return st;
    const size_t head = al(8 * (size_t)P * (size_t)B);
    if (ws_bytes < head + mn)
        return set_error(ZP_ERR_WORKSPACE, "workspace smaller than the minimum (zp_series_analysis_workspace)");
    std::shared_ptr<Plan> plan;
    st = get_plan(h_n, h_m, M, &plan);
    if (st != ZP_OK) return st;
    double *wf = (double *)d_ws;
    st = launch_weight(d_w, d_f, P, B, wf, s);
    if (st != ZP_OK) return st;
    st = zp_series_bwd(h_n, h_m, M, d_r, d_theta, P, nullptr, B, prec, wf, nullptr, d_c, nullptr, nullptr,
                       (char *)d_ws + head, ws_bytes - head, stream);
    if (st != ZP_OK) return st;
    return launch_mode_norm(*plan, B, d_c, s);
}

} // extern "C"
