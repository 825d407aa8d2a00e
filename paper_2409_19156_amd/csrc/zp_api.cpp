// C ABI entry points of libzp (declared in include/zp.h): host-side argument
// validation, plan lookup and kernel dispatch.  All validation precedes any
// HIP call, so error paths run without a GPU.
#include <cstdio>
#include <cstdint>
#include <cstring>
#include <string>

#include "zp_internal.hpp"

namespace zp {

namespace {
thread_local std::string t_last_error;
}

zp_status set_error(zp_status s, const std::string &msg)
{
    t_last_error = msg;
    return s;
}

zp_status hip_check(hipError_t e, const char *what)
{
    if (e == hipSuccess) return ZP_OK;
    return set_error(ZP_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

zp_status check_modes_arg(const int32_t *n, const int32_t *m, int64_t M)
{
    if (M < 0) return set_error(ZP_ERR_ARG, "M < 0");
    if (M > 0 && (!n || !m)) return set_error(ZP_ERR_ARG, "null mode array");
    if (M > INT32_MAX) return set_error(ZP_ERR_ARG, "M exceeds 2^31 - 1");
    int64_t bad = -1;
    if (validate_modes(n, m, M, &bad) != ZP_OK) {
        char buf[160];
        std::snprintf(buf, sizeof buf,
                      "mode %lld: (n, m) = (%d, %d) violates n >= 0, |m| <= n, n - |m| even, n <= %d",
                      (long long)bad, n[bad], m[bad], ZP_N_MAX);
        return set_error(ZP_ERR_MODE, buf);
    }
    return ZP_OK;
}

} // namespace zp

using namespace zp;

extern "C" {

zp_status zp_radial(const int32_t *h_n, const int32_t *h_m, int64_t M, const double *d_r, int64_t P,
                    int32_t max_dr, double *d_out, void *stream)
{
    zp_status st = check_modes_arg(h_n, h_m, M);
    if (st != ZP_OK) return st;
    if (max_dr < 0 || max_dr > 3) return set_error(ZP_ERR_ORDER, "max_dr must be 0..3");
    if (P < 0) return set_error(ZP_ERR_ARG, "P < 0");
    if (M == 0 || P == 0) return ZP_OK;
    if (!d_r || !d_out) return set_error(ZP_ERR_ARG, "null point or output pointer");
    std::shared_ptr<Plan> plan;
    st = get_plan(h_n, h_m, M, &plan);
    if (st != ZP_OK) return st;
    Planes o{};
    o.ld = P;
    for (int q = 0; q <= max_dr; ++q) {
        o.plane[q] = d_out + (size_t)q * (size_t)M * (size_t)P;
        o.fmt[q] = F64;
    }
    return launch_chain_kernel(*plan, d_r, nullptr, P, max_dr, false, o, (hipStream_t)stream);
}

zp_status zp_basis(const int32_t *h_n, const int32_t *h_m, int64_t M, const double *d_r, const double *d_theta,
                   int64_t P, uint32_t mask, double *d_out, void *stream)
{
    zp_status st = check_modes_arg(h_n, h_m, M);
    if (st != ZP_OK) return st;
    if (mask == 0 || (mask & ~31u)) return set_error(ZP_ERR_ARG, "mask must be a nonzero subset of bits 0..4");
    if (P < 0) return set_error(ZP_ERR_ARG, "P < 0");
    if (M == 0 || P == 0) return ZP_OK;
    if (!d_r || !d_theta || !d_out) return set_error(ZP_ERR_ARG, "null point or output pointer");
    std::shared_ptr<Plan> plan;
    st = get_plan(h_n, h_m, M, &plan);
    if (st != ZP_OK) return st;
    Planes o{};
    o.ld = P;
    int np = 0, J = 0;
    for (int q = 0; q < 5; ++q) {
        if (!((mask >> q) & 1u)) continue;
        o.plane[q] = d_out + (size_t)np * (size_t)M * (size_t)P;
        o.fmt[q] = F64;
        ++np;
        if (q >= 1 && q <= 3) J = q;
    }
    return launch_chain_kernel(*plan, d_r, d_theta, P, J, true, o, (hipStream_t)stream);
}

zp_status zp_basis_polar(const int32_t *h_n, const int32_t *h_m, int64_t M, const double *d_r, int64_t NR,
                         const double *d_theta, int64_t NT, uint32_t mask, double *d_out, void *stream)
{
    zp_status st = check_modes_arg(h_n, h_m, M);
    if (st != ZP_OK) return st;
    if (mask == 0 || (mask & ~31u)) return set_error(ZP_ERR_ARG, "mask must be a nonzero subset of bits 0..4");
    if (NR < 0 || NT < 0) return set_error(ZP_ERR_ARG, "NR < 0 or NT < 0");
    if (NR > 0 && NT > INT64_MAX / NR) return set_error(ZP_ERR_ARG, "NR * NT overflows");
    const int64_t P = NR * NT;
    if (M == 0 || P == 0) return ZP_OK;
    if (!d_r || !d_theta || !d_out) return set_error(ZP_ERR_ARG, "null point or output pointer");
    std::shared_ptr<Plan> plan;
    st = get_plan(h_n, h_m, M, &plan);
    if (st != ZP_OK) return st;
    Planes o{};
    o.ld = P;
    int np = 0, J = 0;
    for (int q = 0; q < 5; ++q) {
        if (!((mask >> q) & 1u)) continue;
        o.plane[q] = d_out + (size_t)np * (size_t)M * (size_t)P;
        o.fmt[q] = F64;
        ++np;
        if (q >= 1 && q <= 3) J = q;
    }
    return launch_chain_kernel_polar(*plan, d_r, NR, d_theta, NT, J, o, (hipStream_t)stream);
}

zp_status zp_radial_direct(const int32_t *h_n, const int32_t *h_m, int64_t M, const double *d_r, int64_t P,
                           int32_t max_dr, double *d_out, void *stream)
{
    zp_status st = check_modes_arg(h_n, h_m, M);
    if (st != ZP_OK) return st;
    if (max_dr < 0 || max_dr > 3) return set_error(ZP_ERR_ORDER, "max_dr must be 0..3");
    if (P < 0) return set_error(ZP_ERR_ARG, "P < 0");
    if (M == 0 || P == 0) return ZP_OK;
    if (!d_r || !d_out) return set_error(ZP_ERR_ARG, "null point or output pointer");
    if (M > 65535) return set_error(ZP_ERR_ARG, "direct evaluation takes at most 65535 modes per call");
    std::shared_ptr<Plan> plan;
    st = get_plan(h_n, h_m, M, &plan);
    if (st != ZP_OK) return st;
    st = get_direct_table(*plan);
    if (st != ZP_OK) return st;
    return launch_direct_kernel(*plan, d_r, P, max_dr, d_out, (hipStream_t)stream);
}

zp_status zp_radial_zernike_recursion(const int32_t *h_n, const int32_t *h_m, int64_t M, const double *d_r, int64_t P,
                                      int32_t max_dr, double *d_out, void *stream)
{
    zp_status st = check_modes_arg(h_n, h_m, M);
    if (st != ZP_OK) return st;
    if (max_dr < 0 || max_dr > 3) return set_error(ZP_ERR_ORDER, "max_dr must be 0..3");
    if (P < 0) return set_error(ZP_ERR_ARG, "P < 0");
    for (int64_t i = 0; i < M; ++i)
        if (h_n[i] > kZrecNmax) return set_error(ZP_ERR_ARG, "the Zernike-recursion comparator takes n <= 60");
    if (M == 0 || P == 0) return ZP_OK;
    if (!d_r || !d_out) return set_error(ZP_ERR_ARG, "null point or output pointer");
    std::shared_ptr<Plan> plan;
    st = get_plan(h_n, h_m, M, &plan);
    if (st != ZP_OK) return st;
    st = get_zrec_table(*plan);
    if (st != ZP_OK) return st;
    return launch_zrec_kernel(*plan, d_r, P, max_dr, d_out, (hipStream_t)stream);
}

const char *zp_status_string(zp_status s)
{
    switch (s) {
    case ZP_OK: return "ok";
    case ZP_ERR_MODE: return "invalid mode: need n >= 0, |m| <= n, n - |m| even, n <= ZP_N_MAX";
    case ZP_ERR_ARG: return "invalid argument";
    case ZP_ERR_ORDER: return "derivative order must be 0..3";
    case ZP_ERR_WORKSPACE: return "workspace too small";
    case ZP_ERR_HIP: return "HIP runtime error";
    case ZP_ERR_PREC: return "unknown precision";
    }
    return "unknown status";
}

const char *zp_last_error(void) { return t_last_error.c_str(); }

void zp_cache_clear(void)
{
    clear_plans();
    clear_plans3();
}

int32_t zp_abi_version(void) { return 1; }

} // extern "C"
