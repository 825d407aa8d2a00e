// Three-dimensional spectral series (the paper's duplicated-mode use, Sec. 3
// footnote): f(r, theta, phi) = sum_j c_j R_{n_j}^{|m_j|}(r) F_{m_j}(theta)
// F_{l_j}(phi) on a tensor grid of P polar points times Q toroidal angles.
//
// Modes with the same (n, m) and different l are "duplicated": their Zernike
// factor is the same.  The library therefore
//   1. finds the U distinct (n, m) pairs of the J modes (host, cached);
//   2. folds the Fourier factor into the coefficients:
//        T[u][q][b] = sum over modes j of pair u of c[j][b] F_{l_j}(phi_q);
//   3. runs the planar series over the U pairs with Q*B coefficient sets:
//        f[p][q][b] = sum_u Z_u(r_p, theta_p) T[u][q][b].
// The contraction then has U instead of J terms; with every (n, m) paired
// with 2L+1 values of l that is a factor 2L+1 less work than the planar
// series over the duplicated list.
//
// Adjoint, for an upstream gradient g [P][Q][B]: the planar backward with
// c = T gives dL/dT, dL/dr and dL/dtheta; then
//   dL/dc[j][b] = sum_q F_{l_j}(phi_q) dL/dT[u_j][q][b]
//   dL/dphi[q]  = sum_j sum_b dF_{l_j}/dphi(phi_q) c[j][b] dL/dT[u_j][q][b].
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <iterator>
#include <list>
#include <mutex>
#include <unordered_map>

#include "series3d.hpp"

namespace zp {
zp_status check_modes_arg(const int32_t *n, const int32_t *m, int64_t M);

void dedup_modes(const int32_t *n, const int32_t *m, int64_t J, std::vector<int32_t> &un, std::vector<int32_t> &um,
                 std::vector<int32_t> &owner)
{
    un.clear();
    um.clear();
    owner.resize((size_t)J);
    std::unordered_map<int64_t, int32_t> seen;
    seen.reserve((size_t)J * 2);
    for (int64_t j = 0; j < J; ++j) {
        const int64_t key = ((int64_t)n[j] << 32) ^ (int64_t)(uint32_t)m[j];
        auto it = seen.find(key);
        if (it == seen.end()) {
            it = seen.emplace(key, (int32_t)un.size()).first;
            un.push_back(n[j]);
            um.push_back(m[j]);
        }
        owner[(size_t)j] = it->second;
    }
}

Plan3::~Plan3()
{
    if (dmem) {
        int cur = -1;
        (void)hipGetDevice(&cur);
        (void)hipSetDevice(device);
        (void)hipDeviceSynchronize(); // kernels may still read the tables
        (void)hipFree(dmem);
        if (cur >= 0) (void)hipSetDevice(cur);
    }
}

namespace {

std::mutex g_mu3;
// Most recently used first; never destroyed (no HIP call at static destruction).
std::list<std::shared_ptr<Plan3>> &g_cache3 = *new std::list<std::shared_ptr<Plan3>>();

size_t capacity3()
{
    static size_t cap = [] {
        const char *e = std::getenv("ZP_PLAN_CACHE");
        long v = e ? std::strtol(e, nullptr, 10) : 16;
        return (size_t)std::max(1L, v);
    }();
    return cap;
}

zp_status upload3(Plan3 &p)
{
    const size_t J = p.n.size(), U = p.un.size();
    std::vector<int32_t> uptr(U + 1, 0), jl(J);
    for (size_t j = 0; j < J; ++j) ++uptr[(size_t)p.owner[j] + 1];
    for (size_t u = 0; u < U; ++u) uptr[u + 1] += uptr[u];
    std::vector<int32_t> fill(uptr.begin(), uptr.end() - 1);
    for (size_t j = 0; j < J; ++j) jl[(size_t)fill[(size_t)p.owner[j]]++] = (int32_t)j; // ascending j per pair
    // layout: uptr [U+1] | jl [J] | owner [J] | l [J], each 256-byte aligned
    auto al = [](size_t x) { return (x + 255) / 256 * 256; };
    const size_t o1 = al((U + 1) * 4), o2 = o1 + al(J * 4), o3 = o2 + al(J * 4), total = o3 + al(J * 4);
    std::vector<unsigned char> host(total, 0);
    std::copy_n((const unsigned char *)uptr.data(), (U + 1) * 4, host.data());
    std::copy_n((const unsigned char *)jl.data(), J * 4, host.data() + o1);
    std::copy_n((const unsigned char *)p.owner.data(), J * 4, host.data() + o2);
    std::copy_n((const unsigned char *)p.l.data(), J * 4, host.data() + o3);
    zp_status st = hip_check(hipMalloc(&p.dmem, total), "hipMalloc(3-D plan)");
    if (st != ZP_OK) return st;
    st = hip_check(hipMemcpy(p.dmem, host.data(), total, hipMemcpyHostToDevice), "hipMemcpy(3-D plan)");
    if (st != ZP_OK) return st;
    const unsigned char *b = (const unsigned char *)p.dmem;
    p.d_uptr = (const int32_t *)b;
    p.d_jl = (const int32_t *)(b + o1);
    p.d_owner = (const int32_t *)(b + o2);
    p.d_l = (const int32_t *)(b + o3);
    return ZP_OK;
}

} // namespace

// As get_plan: the lookup under the lock, a missing plan built without it,
// and plans pushed out of the cache released after the lock is dropped.
zp_status get_plan3(const int32_t *n, const int32_t *m, const int32_t *l, int64_t J, std::shared_ptr<Plan3> *out)
{
    int dev = 0;
    zp_status st = hip_check(hipGetDevice(&dev), "hipGetDevice");
    if (st != ZP_OK) return st;
    auto lookup = [&]() -> bool { // under the lock
        for (auto it = g_cache3.begin(); it != g_cache3.end(); ++it) {
            Plan3 &p = **it;
            if (p.device == dev && (int64_t)p.n.size() == J && std::equal(p.n.begin(), p.n.end(), n) &&
                std::equal(p.m.begin(), p.m.end(), m) && std::equal(p.l.begin(), p.l.end(), l)) {
                g_cache3.splice(g_cache3.begin(), g_cache3, it);
                *out = g_cache3.front();
                return true;
            }
        }
        return false;
    };
    {
        std::lock_guard<std::mutex> lock(g_mu3);
        if (lookup()) return ZP_OK;
    }
    auto p = std::make_shared<Plan3>();
    p->n.assign(n, n + J);
    p->m.assign(m, m + J);
    p->l.assign(l, l + J);
    dedup_modes(n, m, J, p->un, p->um, p->owner);
    p->device = dev;
    st = upload3(*p);
    if (st != ZP_OK) return st;
    std::list<std::shared_ptr<Plan3>> released; // destroyed after the lock below
    {
        std::lock_guard<std::mutex> lock(g_mu3);
        if (lookup()) {
            released.push_back(std::move(p));
        } else {
            g_cache3.push_front(p);
            *out = p;
            while (g_cache3.size() > capacity3()) released.splice(released.end(), g_cache3, std::prev(g_cache3.end()));
        }
    }
    return ZP_OK;
}

void clear_plans3()
{
    std::list<std::shared_ptr<Plan3>> drop;
    {
        std::lock_guard<std::mutex> lock(g_mu3);
        drop.swap(g_cache3);
    }
    drop.clear();
}

} // namespace zp

using namespace zp;

namespace {

size_t al(size_t x) { return (x + 255) / 256 * 256; }

zp_status checks3(const int32_t *n, const int32_t *m, const int32_t *l, int64_t J, int64_t P, int64_t Q, int64_t B,
                  int32_t prec)
{
    zp_status st = check_modes_arg(n, m, J);
    if (st != ZP_OK) return st;
    if (J > 0 && !l) return set_error(ZP_ERR_ARG, "null l array");
    for (int64_t j = 0; j < J; ++j)
        if (l[j] < -ZP_L_MAX || l[j] > ZP_L_MAX) {
            char buf[96];
            snprintf(buf, sizeof buf, "mode %lld: |l| = %d exceeds ZP_L_MAX", (long long)j, l[j]);
            return set_error(ZP_ERR_MODE, buf);
        }
    if (P < 0 || Q < 0 || B < 0) return set_error(ZP_ERR_ARG, "negative P, Q or B");
    if (prec < ZP_FP64 || prec > ZP_BF16X3) return set_error(ZP_ERR_PREC, "prec must be ZP_FP64, ZP_FP32 or ZP_BF16X3");
    return ZP_OK;
}

int64_t distinct_pairs(const int32_t *n, const int32_t *m, int64_t J)
{
    std::vector<int32_t> un, um, owner;
    dedup_modes(n, m, J, un, um, owner);
    return (int64_t)un.size();
}

// Workspace: T [U][Q*B] | dL/dT [U][Q*B] | the planar series' workspace.
size_t head_bytes(int64_t U, int64_t Q, int64_t B) { return 2 * al(8 * (size_t)U * (size_t)Q * (size_t)B); }

// Host-side check that ws_bytes covers the head and the planar series'
// minimum, before any device work.
zp_status check_ws3(const int32_t *n, const int32_t *m, int64_t J, int64_t P, int64_t Q, int64_t B, int32_t prec,
                    size_t ws_bytes)
{
    const int64_t U = distinct_pairs(n, m, J);
    size_t f = 0, mn = 0;
    zp_status st = zp_series_workspace(U, P, Q * B, prec, &f, &mn);
    if (st != ZP_OK) return st;
    if (ws_bytes < head_bytes(U, Q, B) + mn)
        return set_error(ZP_ERR_WORKSPACE, "workspace smaller than the minimum (zp_series3d_workspace)");
    return ZP_OK;
}

} // namespace

extern "C" {

zp_status zp_series3d_workspace(const int32_t *h_n, const int32_t *h_m, const int32_t *h_l, int64_t J, int64_t P,
                                int64_t Q, int64_t B, int32_t prec, size_t *full_bytes, size_t *min_bytes)
{
    zp_status st = checks3(h_n, h_m, h_l, J, P, Q, B, prec);
    if (st != ZP_OK) return st;
    if (!full_bytes) return set_error(ZP_ERR_ARG, "null full_bytes");
    const int64_t U = distinct_pairs(h_n, h_m, J);
    size_t f = 0, mn = 0;
    st = zp_series_workspace(U, P, Q * B, prec, &f, &mn);
    if (st != ZP_OK) return st;
    *full_bytes = head_bytes(U, Q, B) + f;
    if (min_bytes) *min_bytes = head_bytes(U, Q, B) + mn;
    return ZP_OK;
}

zp_status zp_series3d_cache_bytes(const int32_t *h_n, const int32_t *h_m, const int32_t *h_l, int64_t J, int64_t P,
                                  int32_t prec, size_t *bytes)
{
    zp_status st = checks3(h_n, h_m, h_l, J, P, 0, 0, prec);
    if (st != ZP_OK) return st;
    return zp_series_cache_bytes(distinct_pairs(h_n, h_m, J), P, prec, bytes);
}

zp_status zp_series3d_fwd(const int32_t *h_n, const int32_t *h_m, const int32_t *h_l, int64_t J, const double *d_r,
                          const double *d_theta, int64_t P, const double *d_phi, int64_t Q, const double *d_c,
                          int64_t B, int32_t prec, double *d_f, void *d_cache, void *d_ws, size_t ws_bytes,
                          void *stream)
{
    zp_status st = checks3(h_n, h_m, h_l, J, P, Q, B, prec);
    if (st != ZP_OK) return st;
    if (J == 0 || P == 0 || Q == 0 || B == 0) return ZP_OK;
    if (!d_r || !d_theta || !d_phi || !d_c || !d_f) return set_error(ZP_ERR_ARG, "null pointer");
    if (!d_ws || ((uintptr_t)d_ws & 255)) return set_error(ZP_ERR_ARG, "workspace must be non-null and 256-byte aligned");
    if ((uintptr_t)d_cache & 255) return set_error(ZP_ERR_ARG, "cache must be 256-byte aligned");
    st = check_ws3(h_n, h_m, J, P, Q, B, prec, ws_bytes);
    if (st != ZP_OK) return st;
    std::shared_ptr<Plan3> p;
    st = get_plan3(h_n, h_m, h_l, J, &p);
    if (st != ZP_OK) return st;
    const int64_t U = (int64_t)p->un.size();
    const size_t head = head_bytes(U, Q, B);
    hipStream_t s = (hipStream_t)stream;
    double *T = (double *)d_ws;
    st = launch_fourier_mix(*p, d_c, B, d_phi, Q, false, T, s);
    if (st != ZP_OK) return st;
    return zp_series_fwd(p->un.data(), p->um.data(), U, d_r, d_theta, P, T, Q * B, prec, d_f, d_cache,
                         (char *)d_ws + head, ws_bytes - head, stream);
}

zp_status zp_series3d_bwd(const int32_t *h_n, const int32_t *h_m, const int32_t *h_l, int64_t J, const double *d_r,
                          const double *d_theta, int64_t P, const double *d_phi, int64_t Q, const double *d_c,
                          int64_t B, int32_t prec, const double *d_g, const void *d_cache, double *d_grad_c,
                          double *d_grad_r, double *d_grad_theta, double *d_grad_phi, void *d_ws, size_t ws_bytes,
                          void *stream)
{
    zp_status st = checks3(h_n, h_m, h_l, J, P, Q, B, prec);
    if (st != ZP_OK) return st;
    if (J == 0 || P == 0 || Q == 0 || B == 0) return ZP_OK;
    if (!d_r || !d_theta || !d_phi || !d_c || !d_g) return set_error(ZP_ERR_ARG, "null pointer");
    if (!d_grad_c && !d_grad_r && !d_grad_theta && !d_grad_phi) return ZP_OK;
    if (!d_ws || ((uintptr_t)d_ws & 255)) return set_error(ZP_ERR_ARG, "workspace must be non-null and 256-byte aligned");
    if ((uintptr_t)d_cache & 255) return set_error(ZP_ERR_ARG, "cache must be 256-byte aligned");
    st = check_ws3(h_n, h_m, J, P, Q, B, prec, ws_bytes);
    if (st != ZP_OK) return st;
    std::shared_ptr<Plan3> p;
    st = get_plan3(h_n, h_m, h_l, J, &p);
    if (st != ZP_OK) return st;
    const int64_t U = (int64_t)p->un.size();
    const size_t head = head_bytes(U, Q, B);
    hipStream_t s = (hipStream_t)stream;
    double *T = (double *)d_ws;
    double *gT = (double *)((char *)d_ws + head / 2);
    st = launch_fourier_mix(*p, d_c, B, d_phi, Q, false, T, s);
    if (st != ZP_OK) return st;
    const bool need_gT = d_grad_c || d_grad_phi;
    st = zp_series_bwd(p->un.data(), p->um.data(), U, d_r, d_theta, P, T, Q * B, prec, d_g, d_cache,
                       need_gT ? gT : nullptr, d_grad_r, d_grad_theta, (char *)d_ws + head, ws_bytes - head, stream);
    if (st != ZP_OK) return st;
    if (d_grad_c) {
        st = launch_fourier_unmix(*p, gT, B, d_phi, Q, d_grad_c, s);
        if (st != ZP_OK) return st;
    }
    if (d_grad_phi) {
        st = launch_fourier_phi_grad(*p, gT, d_c, B, d_phi, Q, d_grad_phi, s);
        if (st != ZP_OK) return st;
    }
    return ZP_OK;
}

} // extern "C"
