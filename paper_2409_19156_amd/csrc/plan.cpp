// Host-side plans: mode validation, grouping of modes into one recurrence
// chain per alpha = |m| (Algorithm 1 of the paper: a chain serves every n of
// its alpha), per-step coefficients, and a small device-side cache.
#include <algorithm>
#include <cstdlib>
#include <iterator>
#include <list>
#include <mutex>

#include "zp_internal.hpp"

namespace zp {

zp_status validate_modes(const int32_t *n, const int32_t *m, int64_t M, int64_t *bad)
{
    for (int64_t i = 0; i < M; ++i) {
        const int64_t a = m[i] < 0 ? -(int64_t)m[i] : (int64_t)m[i];
        // Sec. 2: n >= 0, |m| <= n, n - |m| even.
        if (n[i] < 0 || a > n[i] || ((n[i] - a) & 1) || n[i] > ZP_N_MAX) {
            *bad = i;
            return ZP_ERR_MODE;
        }
    }
    return ZP_OK;
}

// Ratio of two exactly representable integers: correctly rounded.
static double ratio(int64_t num, int64_t den) { return (double)num / (double)den; }

// (-1)^K C(K + alpha, K), rounded to double from 64-bit-significand
// arithmetic (at most ~2K roundings of 2^-64 each before the final one).
static double signed_binom(int K, int alpha)
{
    long double v = 1.0L;
    for (int i = 1; i <= K; ++i) v = v * (long double)(alpha + i) / (long double)i;
    return (double)((K & 1) ? -v : v);
}

std::shared_ptr<Plan> build_plan_host(const int32_t *n, const int32_t *m, int64_t M)
{
    auto plan = std::make_shared<Plan>();
    plan->n.assign(n, n + M);
    plan->m.assign(m, m + M);
    int amax = -1;
    for (int64_t i = 0; i < M; ++i) {
        amax = std::max(amax, std::abs(m[i]));
        plan->nmax = std::max(plan->nmax, n[i]);
    }
    // Emits grouped by alpha; within a chain sorted by K (stable, so
    // duplicates keep the caller's column order).
    std::vector<std::vector<Emit>> by_alpha(amax + 1);
    for (int64_t i = 0; i < M; ++i) {
        const int a = std::abs(m[i]);
        Emit e{};
        e.K = (n[i] - a) / 2;
        e.col = (int32_t)i;
        e.flags = m[i] < 0 ? 1 : 0;
        e.a_lo = signed_binom(e.K, a);
        by_alpha[a].push_back(e);
    }
    struct Tmp {
        Chain c;
        double cost;
    };
    std::vector<Tmp> tmp;
    for (int a = 0; a <= amax; ++a) {
        auto &v = by_alpha[a];
        if (v.empty()) continue;
        std::stable_sort(v.begin(), v.end(), [](const Emit &x, const Emit &y) { return x.K < y.K; });
        Chain c{};
        c.alpha = a;
        c.kmax = v.back().K;
        c.coef_off = (int32_t)plan->coefs.size();
        c.emit_off = (int32_t)plan->emits.size();
        c.emit_cnt = (int32_t)v.size();
        for (int k = 1; k <= c.kmax; ++k) {
            const int64_t K = k, A = a;
            Coef cf{};
            if (k == 1) {
                cf.cc_lo = 0.0;
                cf.cc_hi = 0.0;
            } else {
                cf.cc_lo = ratio((K - 1) * (K - 1) * (2 * K + A), (K + A) * (K + A) * (2 * K + A - 2));
                cf.cc_hi = ratio((K + A - 1) * (K - 1) * (2 * K + A), K * (K + A) * (2 * K + A - 2));
            }
            cf.bs_lo = ratio((2 * K + A - 1) * (2 * K + A), 2 * (K + A) * (K + A));
            cf.bs_hi = ratio((2 * K + A - 1) * (2 * K + A), 2 * K * (K + A));
            plan->coefs.push_back(cf);
        }
        plan->emits.insert(plan->emits.end(), v.begin(), v.end());
        // Work estimate: stores dominate; the recurrence costs about one
        // store-equivalent per few steps.
        tmp.push_back({c, 4.0 * c.emit_cnt + 0.5 * c.kmax});
    }
    std::stable_sort(tmp.begin(), tmp.end(), [](const Tmp &x, const Tmp &y) { return x.cost > y.cost; });
    for (auto &t : tmp) plan->chains.push_back(t.c);

    // Pieces of at most kSegEmits emissions, cut on multiples of 8.
    std::vector<Tmp> pieces;
    for (const Chain &c : plan->chains) {
        int e0 = c.emit_off;
        const int end = c.emit_off + c.emit_cnt;
        while (e0 < end) {
            int e1 = std::min(end, (e0 / 8) * 8 + kSegEmits);
            if (e1 <= e0) e1 = std::min(end, e0 + kSegEmits);
            Chain p = c;
            p.emit_off = e0;
            p.emit_cnt = e1 - e0;
            p.kmax = plan->emits[e1 - 1].K;
            pieces.push_back({p, 4.0 * p.emit_cnt + 0.5 * p.kmax});
            e0 = e1;
        }
    }
    std::stable_sort(pieces.begin(), pieces.end(), [](const Tmp &x, const Tmp &y) { return x.cost > y.cost; });
    for (auto &t : pieces) plan->pieces.push_back(t.c);
    return plan;
}

// c_s = (-1)^s C(n-s, s) C(n-2s, (n-m)/2 - s) (Eq. radial-part-eq-binom), in
// 64-bit-significand arithmetic, times (n-2s)!/(n-2s-j)!.
static double direct_coef(int n, int m, int s, int j)
{
    const int e = n - 2 * s;
    if (e < j) return 0.0;
    auto binom = [](int top, int k) {
        long double v = 1.0L;
        for (int i = 1; i <= k; ++i) v = v * (long double)(top - k + i) / (long double)i;
        return v;
    };
    long double c = binom(n - s, s) * binom(n - 2 * s, (n - m) / 2 - s);
    for (int t = 0; t < j; ++t) c *= (long double)(e - t);
    return (double)((s & 1) ? -c : c);
}

zp_status get_direct_table(Plan &plan)
{
    std::call_once(plan.direct_once, [&plan] {
        const size_t M = plan.n.size();
        std::vector<int64_t> off(M + 1, 0);
        for (size_t i = 0; i < M; ++i) {
            const int K = (plan.n[i] - std::abs(plan.m[i])) / 2;
            off[i + 1] = off[i] + 4 * (K + 1);
        }
        std::vector<double> coef((size_t)off[M]);
        for (size_t i = 0; i < M; ++i) {
            const int n = plan.n[i], m = std::abs(plan.m[i]), K = (n - m) / 2;
            for (int j = 0; j < 4; ++j)
                for (int s = 0; s <= K; ++s) coef[(size_t)off[i] + (size_t)j * (K + 1) + s] = direct_coef(n, m, s, j);
        }
        // layout: offsets int64[M+1] | n int32[M] | m int32[M] | coefficients
        const size_t a = (M + 1) * sizeof(int64_t), a_al = (a + 255) / 256 * 256;
        const size_t b = M * sizeof(int32_t), b_al = (b + 255) / 256 * 256;
        const size_t total = a_al + 2 * b_al + coef.size() * sizeof(double);
        std::vector<unsigned char> host(total, 0);
        std::copy_n((const unsigned char *)off.data(), a, host.data());
        std::copy_n((const unsigned char *)plan.n.data(), b, host.data() + a_al);
        std::copy_n((const unsigned char *)plan.m.data(), b, host.data() + a_al + b_al);
        std::copy_n((const unsigned char *)coef.data(), coef.size() * sizeof(double), host.data() + a_al + 2 * b_al);
        void *d = nullptr;
        zp_status st = hip_check(hipMalloc(&d, total), "hipMalloc(direct table)");
        if (st == ZP_OK) st = hip_check(hipMemcpy(d, host.data(), total, hipMemcpyHostToDevice), "hipMemcpy(direct table)");
        plan.direct_status = st;
        if (st == ZP_OK) {
            plan.d_direct = d;
            plan.d_direct_off = (const int64_t *)d;
            plan.d_direct_n = (const int32_t *)((unsigned char *)d + a_al);
            plan.d_direct_m = (const int32_t *)((unsigned char *)d + a_al + b_al);
            plan.d_direct_coef = (const double *)((unsigned char *)d + a_al + 2 * b_al);
        }
    });
    return plan.direct_status == ZP_OK ? ZP_OK : set_error(plan.direct_status, "direct table upload failed");
}

zp_status get_zrec_table(Plan &plan)
{
    std::call_once(plan.zrec_once, [&plan] {
        const int nmax = plan.nmax;
        // triangle entry of (n, alpha): rows k < n hold k/2 + 1 entries each
        auto entry = [](int n, int a) {
            int t = 0;
            for (int k = 0; k < n; ++k) t += k / 2 + 1;
            return t + (a - (n & 1)) / 2;
        };
        const int T = entry(nmax + 1, (nmax + 1) & 1);
        std::vector<int32_t> cnt((size_t)T + 1, 0), cols(plan.n.size());
        for (size_t i = 0; i < plan.n.size(); ++i) ++cnt[(size_t)entry(plan.n[i], std::abs(plan.m[i])) + 1];
        for (int t = 0; t < T; ++t) cnt[(size_t)t + 1] += cnt[(size_t)t];
        std::vector<int32_t> fill(cnt.begin(), cnt.end() - 1);
        for (size_t i = 0; i < plan.n.size(); ++i) // caller's order within an entry
            cols[(size_t)fill[(size_t)entry(plan.n[i], std::abs(plan.m[i]))]++] = (int32_t)i;
        const size_t a = cnt.size() * sizeof(int32_t), a_al = (a + 255) / 256 * 256;
        const size_t total = a_al + cols.size() * sizeof(int32_t);
        std::vector<unsigned char> host(total, 0);
        std::copy_n((const unsigned char *)cnt.data(), a, host.data());
        std::copy_n((const unsigned char *)cols.data(), cols.size() * sizeof(int32_t), host.data() + a_al);
        void *d = nullptr;
        zp_status st = hip_check(hipMalloc(&d, total), "hipMalloc(recursion table)");
        if (st == ZP_OK) st = hip_check(hipMemcpy(d, host.data(), total, hipMemcpyHostToDevice), "hipMemcpy(recursion table)");
        plan.zrec_status = st;
        if (st == ZP_OK) {
            plan.d_zrec = d;
            plan.d_zrec_off = (const int32_t *)d;
            plan.d_zrec_cols = (const int32_t *)((unsigned char *)d + a_al);
        }
    });
    return plan.zrec_status == ZP_OK ? ZP_OK : set_error(plan.zrec_status, "recursion table upload failed");
}

Plan::~Plan()
{
    if (!dmem && !d_direct && !d_zrec) return;
    int cur = -1;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(device);
    (void)hipDeviceSynchronize(); // kernels may still read the tables
    if (d_zrec) (void)hipFree(d_zrec);
    if (d_direct) (void)hipFree(d_direct);
    if (dmem) (void)hipFree(dmem);
    if (cur >= 0) (void)hipSetDevice(cur);
}

// Device image of a plan's tables: chains and pieces side by side, then the
// coefficients, the emissions and the permutation, each 256-byte aligned.
size_t plan_image(const Plan &p, std::vector<unsigned char> *host, PlanOffsets *o)
{
    const size_t a = (p.chains.size() + p.pieces.size()) * sizeof(Chain);
    const size_t b = std::max<size_t>(p.coefs.size(), 1) * sizeof(Coef);
    const size_t c = p.emits.size() * sizeof(Emit);
    const size_t d = p.emits.size() * sizeof(int32_t);
    o->coefs = (a + 255) / 256 * 256;
    o->emits = o->coefs + (b + 255) / 256 * 256;
    o->perm = o->emits + (c + 255) / 256 * 256;
    o->total = o->perm + d;
    if (!host) return o->total;
    host->assign(o->total, 0);
    unsigned char *h = host->data();
    std::copy_n((const unsigned char *)p.chains.data(), p.chains.size() * sizeof(Chain), h);
    std::copy_n((const unsigned char *)p.pieces.data(), p.pieces.size() * sizeof(Chain),
                h + p.chains.size() * sizeof(Chain));
    if (!p.coefs.empty()) std::copy_n((const unsigned char *)p.coefs.data(), p.coefs.size() * sizeof(Coef), h + o->coefs);
    std::copy_n((const unsigned char *)p.emits.data(), c, h + o->emits);
    for (size_t e = 0; e < p.emits.size(); ++e) {
        const int32_t col = p.emits[e].col;
        std::copy_n((const unsigned char *)&col, sizeof col, h + o->perm + e * sizeof(int32_t));
    }
    return o->total;
}

void plan_bind(Plan &p, const void *base, const PlanOffsets &o)
{
    const unsigned char *b = (const unsigned char *)base;
    p.d_chains = (const Chain *)b;
    p.d_pieces = p.d_chains + p.chains.size();
    p.d_coefs = (const Coef *)(b + o.coefs);
    p.d_emits = (const Emit *)(b + o.emits);
    p.d_perm = (const int32_t *)(b + o.perm);
}

static zp_status upload(Plan &p)
{
    std::vector<unsigned char> host;
    PlanOffsets o;
    plan_image(p, &host, &o);
    zp_status st = hip_check(hipMalloc(&p.dmem, o.total), "hipMalloc(plan)");
    if (st != ZP_OK) return st;
    st = hip_check(hipMemcpy(p.dmem, host.data(), o.total, hipMemcpyHostToDevice), "hipMemcpy(plan)");
    if (st != ZP_OK) return st;
    plan_bind(p, p.dmem, o);
    return ZP_OK;
}

namespace {
std::mutex g_mu;
// Most recently used first.  Heap-allocated and never destroyed, so no HIP
// call runs during static destruction at process exit.
std::list<std::shared_ptr<Plan>> &g_cache = *new std::list<std::shared_ptr<Plan>>();

size_t cache_capacity()
{
    static size_t cap = [] {
        const char *e = std::getenv("ZP_PLAN_CACHE");
        long v = e ? std::strtol(e, nullptr, 10) : 16;
        return (size_t)std::max(1L, v);
    }();
    return cap;
}
} // namespace

// Looks the mode list up under the cache lock.  A missing plan is built and
// uploaded without the lock (a plan of the same list built meanwhile by another
// thread wins), and plans pushed out of the cache are released after the lock
// is dropped: releasing one synchronizes its device, since kernels may still
// read its tables.
zp_status get_plan(const int32_t *n, const int32_t *m, int64_t M, std::shared_ptr<Plan> *out)
{
    int dev = 0;
    zp_status st = hip_check(hipGetDevice(&dev), "hipGetDevice");
    if (st != ZP_OK) return st;
    auto same = [&](const Plan &p) {
        return p.device == dev && (int64_t)p.n.size() == M && std::equal(p.n.begin(), p.n.end(), n) &&
               std::equal(p.m.begin(), p.m.end(), m);
    };
    auto lookup = [&]() -> bool { // under the lock
        for (auto it = g_cache.begin(); it != g_cache.end(); ++it) {
            if (same(**it)) {
                g_cache.splice(g_cache.begin(), g_cache, it);
                *out = g_cache.front();
                return true;
            }
        }
        return false;
    };
    {
        std::lock_guard<std::mutex> lock(g_mu);
        if (lookup()) return ZP_OK;
    }
    std::shared_ptr<Plan> plan = build_plan_host(n, m, M);
    plan->device = dev;
    st = upload(*plan);
    if (st != ZP_OK) return st;
    std::list<std::shared_ptr<Plan>> released; // destroyed after the lock below
    {
        std::lock_guard<std::mutex> lock(g_mu);
        if (lookup()) {
            released.push_back(std::move(plan));
        } else {
            g_cache.push_front(plan);
            *out = plan;
            while (g_cache.size() > cache_capacity()) released.splice(released.end(), g_cache, std::prev(g_cache.end()));
        }
    }
    return ZP_OK;
}

void clear_plans()
{
    std::list<std::shared_ptr<Plan>> drop;
    {
        std::lock_guard<std::mutex> lock(g_mu);
        drop.swap(g_cache);
    }
    drop.clear();
}

} // namespace zp
