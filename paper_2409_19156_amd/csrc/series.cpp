// Zernike series f = Z^T c and its adjoint: host orchestration of the basis
// kernel, the conversion kernels and the MFMA contractions.
//
// Forward, per chunk of points [p0, p0+Pc):
//   1. basis Z of the chunk in the contraction type (zero padded) -> cache or ws
//      (with a cache, also dZ/dr and dZ/dtheta for the backward)
//   2. f[p0.., :] = Z^T c                     (GEMM, K = modes)
// Backward, per chunk:
//   1. Z, dZ/dr, dZ/dtheta from the cache, or recomputed into ws
//   2. g of the chunk converted to the contraction type
//   3. grad_c (+)= Z g                         (split-K GEMM, K = points, then a
//                                               fixed-order reduction; chunks add
//                                               in order)
//   4. H^T = c g^T tile by tile (K = coefficient sets) with the epilogue
//      grad_r[p] = sum_k H^T[k][p] dZ_k/dr(p), grad_theta likewise; H is never
//      stored.  Per-tile partial sums are reduced in a fixed order.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "series.hpp"

namespace zp {

int device_cus()
{
    static std::mutex mu;
    static int cus[64] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 0;
    std::lock_guard<std::mutex> lock(mu);
    if (!cus[dev] && hipDeviceGetAttribute(&cus[dev], hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        cus[dev] = 0;
    return cus[dev];
}

zp_status check_modes_arg(const int32_t *n, const int32_t *m, int64_t M);
}

using namespace zp;

namespace {

int ct_of(int32_t prec) { return prec == ZP_FP64 ? CT_F64 : prec == ZP_FP32 ? CT_F32 : CT_BF3; }
size_t dsize_of(int ct) { return ct == CT_F64 ? 8 : 4; } // dZ/dr, dZ/dtheta planes
// Z as the backward's split-K contraction reads it: FP64, or FP32 (the bf16
// contraction splits FP32 values into its three planes while loading them)
int zct_of(int ct) { return ct == CT_F64 ? CT_F64 : CT_F32; }
size_t zsize_of(int ct) { return ct == CT_F64 ? 8 : 4; }
int zlay_of(int ct) { return ct == CT_BF3 ? LAY_KC32 : LAY_KC; }
size_t al(size_t x) { return (x + 255) / 256 * 256; }

// Cache: Z [Mp][Pp] (FP64; FP32 for the FP32 and bf16 contractions), then
// dZ/dr and dZ/dtheta [M][Pp].
struct CacheLayout {
    int64_t Mp, Pp;
    size_t z_off, zr_off, zt_off, total;
    CacheLayout(int64_t M, int64_t P, int ct)
    {
        Mp = pad_up(M);
        Pp = pad_up(P);
        z_off = 0;
        zr_off = al(zsize_of(ct) * (size_t)Mp * (size_t)Pp);
        zt_off = zr_off + al(dsize_of(ct) * (size_t)M * (size_t)Pp);
        total = zt_off + al(dsize_of(ct) * (size_t)M * (size_t)Pp);
    }
};

// Split-K count for grad_c: enough workgroups to fill the chip several times,
// preferring a count that is a whole number of waves over the 256 CUs (one
// workgroup per CU at a time), each split a whole number of pads and at least
// kMinSplitPads of them: shorter splits spend more on writing and reducing
// their partial sums than they gain in parallelism (n <= 64 on 8192 points:
// 32 -> 8 splits made forward + backward 3-12% faster; n <= 40 on 16384
// points: 64 -> 16 splits, 2%).
constexpr int64_t kMinSplitPads = 8;

int splits_for(int64_t M, int64_t B, int64_t Kp, int ct)
{
    (void)ct;
    const int64_t tiles = ((M + 127) / 128) * ((B + 127) / 128);
    const int64_t units = Kp / kPad;
    int best = 1;
    double best_eff = 0.0;
    for (int64_t s = 1; s <= units && s <= 64; ++s) {
        if (units % s) continue;
        if (s > 1 && units / s < kMinSplitPads) break;
        const int64_t wgs = tiles * s;
        const double waves = (double)wgs / 256.0;
        const double eff = waves / std::ceil(waves);   // occupancy of the last wave
        const double score = eff * std::min(1.0, waves / 4.0); // and enough waves
        if (score > best_eff + 1e-9) {
            best_eff = score;
            best = (int)s;
        }
    }
    return best;
}

// Workspace for one chunk of Pc points.
//   c      : coefficients in the contraction type, [Mp][Bp]; for the bf16
//            forward transposed and in chain-major mode order, [Bp][Mp]
//   z      : the chunk's basis in the contraction type (forward: k-blocked for
//            bf16, [Mp][Pcp] otherwise; backward without a cache: [Mp][Pcp])
//   zr, zt : dZ/dr, dZ/dtheta of the chunk (backward without a cache)
//   g, gt  : the chunk's upstream gradient [Pcp][Bp] (and [Bp][Pcp] for bf16)
//   pc, pr : split-K partials of dL/dc and column-dot partials of dL/dr, dL/dtheta
struct WsLayout {
    int64_t Mp, Bp, Pcp;
    int S, T;
    size_t c_off, z_off, zr_off, zt_off, g_off, gt_off, pc_off, pr_off, total;
    WsLayout(int64_t M, int64_t Pc, int64_t B, int ct, bool fwd, bool bwd, bool have_cache)
    {
        Mp = pad_up(M);
        Bp = pad_up(B);
        Pcp = pad_up(Pc);
        const size_t e = ct_bytes(ct);
        S = splits_for(M, B, Pcp, ct);
        T = (int)((M + coldot_bm(ct) - 1) / coldot_bm(ct));
        size_t o = 0;
        c_off = o;
        o += al(e * (size_t)Mp * (size_t)Bp);
        z_off = o;
        const bool need_z = (fwd && ct == CT_BF3) || !have_cache;
        if (need_z) o += al(e * (size_t)Mp * (size_t)Pcp);
        zr_off = o;
        if (bwd && !have_cache) o += al(dsize_of(ct) * (size_t)M * (size_t)Pcp);
        zt_off = o;
        if (bwd && !have_cache) o += al(dsize_of(ct) * (size_t)M * (size_t)Pcp);
        g_off = gt_off = pc_off = pr_off = o;
        if (bwd) {
            o += al(e * (size_t)Pcp * (size_t)Bp);
            gt_off = o;
            if (ct == CT_BF3) o += al(e * (size_t)Bp * (size_t)Pcp);
            pc_off = o;
            o += al(8 * (size_t)S * (size_t)M * (size_t)B);
            pr_off = o;
            o += al(8 * (size_t)T * 2 * (size_t)Pc);
        }
        total = o;
    }
};

// Workspace of the forward-mode derivative for one chunk: the stacked
// coefficients [nblk * Mp][Bp] (transposed for bf16) and the stacked basis
// [nblk * Mp][Pcp] (k-blocked for bf16), nblk = 2 (Z with the coefficient
// tangent, and the directional derivative of Z with c).
struct JvpLayout {
    size_t c_off, z_off, total;
    JvpLayout(int64_t M, int64_t Pc, int64_t B, int ct)
    {
        const int64_t K2 = 2 * pad_up(M);
        const size_t e = ct_bytes(ct);
        c_off = 0;
        z_off = al(e * (size_t)K2 * (size_t)pad_up(B));
        total = z_off + al(e * (size_t)K2 * (size_t)pad_up(Pc));
    }
};

int64_t jvp_chunk_for(int64_t M, int64_t P, int64_t B, int ct, size_t ws_bytes)
{
    if (JvpLayout(M, P, B, ct).total <= ws_bytes) return P;
    int64_t lo = 0, hi = pad_up(P) / kPad;
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) / 2;
        if (JvpLayout(M, mid * kPad, B, ct).total <= ws_bytes)
            lo = mid;
        else
            hi = mid - 1;
    }
    return std::min<int64_t>(lo * kPad, P);
}

// Largest chunk (multiple of kPad, <= P) whose workspace fits ws_bytes; 0 if none.
int64_t chunk_for(int64_t M, int64_t P, int64_t B, int ct, bool fwd, bool bwd, bool have_cache, size_t ws_bytes)
{
    if (WsLayout(M, P, B, ct, fwd, bwd, have_cache).total <= ws_bytes) return P;
    int64_t lo = 0, hi = pad_up(P) / kPad; // in units of kPad
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) / 2;
        if (WsLayout(M, mid * kPad, B, ct, fwd, bwd, have_cache).total <= ws_bytes)
            lo = mid;
        else
            hi = mid - 1;
    }
    return std::min<int64_t>(lo * kPad, P);
}

zp_status common_checks(const int32_t *n, const int32_t *m, int64_t M, int64_t P, int64_t B, int32_t prec)
{
    zp_status st = check_modes_arg(n, m, M);
    if (st != ZP_OK) return st;
    if (P < 0 || B < 0) return set_error(ZP_ERR_ARG, "negative P or B");
    if (prec < ZP_FP64 || prec > ZP_BF16X3) return set_error(ZP_ERR_PREC, "prec must be ZP_FP64, ZP_FP32 or ZP_BF16X3");
    return ZP_OK;
}

// A second stream per device for the forward's pipeline (created once, at the
// default priority, never destroyed: no HIP call at static destruction).
hipStream_t helper_stream()
{
    static std::mutex mu;
    static hipStream_t streams[64] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
    std::lock_guard<std::mutex> lock(mu);
    if (!streams[dev] && hipStreamCreateWithFlags(&streams[dev], hipStreamNonBlocking) != hipSuccess)
        streams[dev] = nullptr;
    return streams[dev];
}

// Forward pipeline: chunks of points alternate between the caller's stream
// and the helper stream; chunk i+1's basis starts when chunk i's basis has
// finished, so it runs under chunk i's contraction.  A chunk's contraction
// has one 128 x 128 output tile per compute unit (two for bf16, whose tiles
// take a whole unit each), which leaves room beside it for the next basis:
// with 65536 points x 1024 sets that is 16 chunks for FP64 and FP32, the
// fastest of 1 to 32 chunks on the series of n <= 64, and 8 for bf16, whose
// forward took within 3% of the same time for every count from 1 to 8.
// Returns the chunk length, or 0 for no pipeline.
int64_t pipe_chunk(int64_t P, int64_t B, int ct)
{
    constexpr int64_t kMinChunk = 2048, kMinPoints = 8192, kTile = 128;
    const int cus = device_cus();
    if (cus <= 0 || P < kMinPoints) return 0;
    const int64_t col_tiles = (B + kTile - 1) / kTile;
    const int64_t tiles = (ct == CT_BF3 ? 2 : 1) * (int64_t)cus;
    const int64_t len = std::max(kMinChunk, (tiles + col_tiles - 1) / col_tiles * kTile);
    return 2 * len <= P ? len : 0;
}

// Chunks of a basis-then-contraction loop on two streams: chunk i runs on
// the caller's stream (even i) or the helper stream (odd i), and its basis
// waits for chunk i-1's basis, so that it runs under chunk i-1's contraction.
// Chunk i+2 may reuse chunk i's workspace buffer: they share a stream.  The
// helper stream forks from the caller's stream at start() and joins it at
// finish().  Switched off, every chunk runs on the caller's stream.
class ChunkPipe {
public:
    ChunkPipe(hipStream_t s, bool on) : s_(s), h_(on ? helper_stream() : nullptr) {}
    ~ChunkPipe()
    {
        if (open_) (void)finish(); // an early return still joins the helper stream
        for (hipEvent_t e : ev_) (void)hipEventDestroy(e); // released once completed
    }
    ChunkPipe(const ChunkPipe &) = delete;
    ChunkPipe &operator=(const ChunkPipe &) = delete;

    bool on() const { return h_ != nullptr; }
    hipStream_t stream(int chunk) const { return on() && (chunk & 1) ? h_ : s_; }
    zp_status start()
    {
        hipEvent_t e = nullptr;
        zp_status st = on() ? record(s_, &e) : ZP_OK;
        if (!e) return st;
        open_ = true;
        return wait(h_, e);
    }
    zp_status before_basis(int chunk) { return on() && prev_ ? wait(stream(chunk), prev_) : ZP_OK; }
    zp_status after_basis(int chunk) { return on() ? record(stream(chunk), &prev_) : ZP_OK; }
    zp_status finish()
    {
        open_ = false;
        hipEvent_t e = nullptr;
        zp_status st = on() ? record(h_, &e) : ZP_OK;
        return e ? wait(s_, e) : st;
    }

private:
    zp_status record(hipStream_t st, hipEvent_t *out)
    {
        hipEvent_t e;
        zp_status r = hip_check(hipEventCreateWithFlags(&e, hipEventDisableTiming), "hipEventCreate");
        if (r != ZP_OK) return r;
        ev_.push_back(e);
        r = hip_check(hipEventRecord(e, st), "hipEventRecord");
        if (r == ZP_OK) *out = e;
        return r;
    }
    static zp_status wait(hipStream_t st, hipEvent_t e)
    {
        return hip_check(hipStreamWaitEvent(st, e, 0), "hipStreamWaitEvent");
    }

    hipStream_t s_, h_;
    hipEvent_t prev_ = nullptr;
    bool open_ = false;
    std::vector<hipEvent_t> ev_;
};

// Basis of points [p0, p0+Pc) into [Mp][ld] planes: Z as the backward reads
// it (zct_of; pad zeroed), dZ/dr and dZ/dtheta (if not null) in FP64 / FP32.
zp_status basis_into(const Plan &plan, const double *r, const double *th, int64_t p0, int64_t Pc, int ct,
                     void *z, void *zr, void *zt, int64_t ld, int64_t Mp, int64_t M, hipStream_t s)
{
    Planes o{};
    o.ld = ld;
    o.sub = Mp * ld;
    o.plane[0] = z;
    o.fmt[0] = ct == CT_F64 ? F64 : F32;
    const int dfmt = ct == CT_F64 ? F64 : F32;
    o.plane[1] = zr;
    o.fmt[1] = dfmt;
    o.plane[4] = zt;
    o.fmt[4] = dfmt;
    zp_status st = launch_zero_pad(z, zct_of(ct), M, Pc, Mp, ld, Mp * ld, s);
    if (st != ZP_OK) return st;
    return launch_chain_kernel(plan, r + p0, th + p0, Pc, zr ? 1 : 0, true, o, s);
}

} // namespace

extern "C" {

zp_status zp_series_cache_bytes(int64_t M, int64_t P, int32_t prec, size_t *bytes)
{
    if (!bytes || M < 0 || P < 0) return set_error(ZP_ERR_ARG, "bad argument");
    if (prec < ZP_FP64 || prec > ZP_BF16X3) return set_error(ZP_ERR_PREC, "unknown prec");
    *bytes = CacheLayout(M, P, ct_of(prec)).total;
    return ZP_OK;
}

zp_status zp_series_workspace(int64_t M, int64_t P, int64_t B, int32_t prec, size_t *full_bytes, size_t *min_bytes)
{
    if (!full_bytes || M < 0 || P < 0 || B < 0) return set_error(ZP_ERR_ARG, "bad argument");
    if (prec < ZP_FP64 || prec > ZP_BF16X3) return set_error(ZP_ERR_PREC, "unknown prec");
    const int ct = ct_of(prec);
    // Sized for the most demanding use: backward without a cache, or the
    // forward-mode derivative.
    const int64_t P1 = std::min<int64_t>(P, kPad);
    *full_bytes = std::max({WsLayout(M, P, B, ct, true, true, false).total, JvpLayout(M, P, B, ct).total, (size_t)256});
    if (min_bytes)
        *min_bytes = std::max({WsLayout(M, P1, B, ct, true, true, false).total, JvpLayout(M, P1, B, ct).total, (size_t)256});
    return ZP_OK;
}

} // extern "C"

namespace zp {

zp_status series_fwd_checks(const int32_t *h_n, const int32_t *h_m, int64_t M, const double *d_r,
                            const double *d_theta, int64_t P, const double *d_c, int64_t B, int32_t prec,
                            const double *d_f)
{
    zp_status st = common_checks(h_n, h_m, M, P, B, prec);
    if (st != ZP_OK) return st;
    if (M == 0 || P == 0 || B == 0) return ZP_OK;
    if (!d_r || !d_theta || !d_c || !d_f) return set_error(ZP_ERR_ARG, "null pointer");
    return ZP_OK;
}

size_t series_fwd_min_ws(int64_t M, int64_t P, int64_t B, int32_t prec)
{
    return WsLayout(M, std::min<int64_t>(P, kPad), B, ct_of(prec), true, false, false).total;
}

zp_status series_fwd_run(const Plan &pl, int64_t M, const double *d_r, const double *d_theta, int64_t P,
                         const double *d_c, int64_t B, int32_t prec, double *d_f, void *d_cache, void *d_ws,
                         size_t ws_bytes, bool allow_pipe, hipStream_t s)
{
    const Plan *plan = &pl;
    zp_status st = ZP_OK;
    const int ct = ct_of(prec);
    const bool have_cache = d_cache != nullptr;
    int64_t Pc = chunk_for(M, P, B, ct, true, false, have_cache, ws_bytes);
    if (Pc <= 0) return set_error(ZP_ERR_WORKSPACE, "workspace smaller than the minimum (zp_series_workspace)");

    // Pipelined chunks when the points are many and the workspace holds two
    // chunk buffers for the basis (bf16, or no cache); otherwise one stream.
    const bool ws_z = ct == CT_BF3 || !have_cache; // the basis goes through the workspace
    bool pipe = false;
    size_t zbuf = 0; // bytes of one chunk's basis buffer
    const int64_t Pq = Pc == P && allow_pipe ? pipe_chunk(P, B, ct) : 0;
    if (Pq > 0) {
        const WsLayout Lq(M, Pq, B, ct, true, false, have_cache);
        zbuf = al(ct_bytes(ct) * (size_t)pad_up(M) * (size_t)Pq);
        if (!ws_z || Lq.total + zbuf <= ws_bytes) {
            pipe = true;
            Pc = Pq;
        }
    }
    ChunkPipe pipeline(s, pipe);
    if (!pipeline.on()) Pc = chunk_for(M, P, B, ct, true, false, have_cache, ws_bytes);

    const WsLayout L(M, Pc, B, ct, true, false, have_cache);
    char *ws = (char *)d_ws;
    const int64_t Mp = L.Mp, Bp = L.Bp;
    void *cbuf = ws + L.c_off;
    if (ct == CT_BF3) // B(k = e, j = b) = c[perm[e]][b], in MFMA fragment order
        st = launch_convert_gather_frag(d_c, plan->d_perm, M, B, B, cbuf, Bp, Mp, Bp * Mp, s);
    else // B(k = q, j = b) = c[q][b]
        st = launch_convert(d_c, M, B, B, ct, cbuf, Bp, Mp, Mp * Bp, false, s);
    if (st != ZP_OK) return st;

    const CacheLayout CL(M, P, ct);
    char *cache = (char *)d_cache;
    const size_t zsz = zsize_of(ct); // the cache's Z element
    if (have_cache) {
        st = launch_zero_pad(cache + CL.z_off, zct_of(ct), M, P, Mp, CL.Pp, Mp * CL.Pp, s);
        if (st != ZP_OK) return st;
    }
    st = pipeline.start();
    if (st != ZP_OK) return st;
    int chunk = 0;
    for (int64_t p0 = 0; p0 < P; p0 += Pc, ++chunk) {
        const int64_t pc = std::min(Pc, P - p0);
        const int64_t pcp = pad_up(pc);
        hipStream_t cs = pipeline.stream(chunk);
        char *zb = ws + L.z_off + (pipeline.on() && (chunk & 1) ? zbuf : 0); // this chunk's basis buffer
        st = pipeline.before_basis(chunk);
        if (st != ZP_OK) return st;
        Planes o{};
        const int zfmt = ct == CT_F64 ? F64 : ct == CT_F32 ? F32 : B16X3;
        const int dfmt = ct == CT_F64 ? F64 : F32;
        int J = 0;
        if (have_cache) { // keep Z, dZ/dr, dZ/dtheta for the backward
            o.ld = CL.Pp;
            o.sub = Mp * CL.Pp;
            o.plane[0] = cache + CL.z_off + zsz * (size_t)p0;
            o.fmt[0] = ct == CT_F64 ? F64 : F32;
            o.plane[1] = cache + CL.zr_off + dsize_of(ct) * (size_t)p0;
            o.fmt[1] = dfmt;
            o.plane[4] = cache + CL.zt_off + dsize_of(ct) * (size_t)p0;
            o.fmt[4] = dfmt;
            J = 1;
        } else if (ct != CT_BF3) {
            o.ld = pcp;
            o.sub = Mp * pcp;
            o.plane[0] = zb;
            o.fmt[0] = zfmt;
            st = launch_zero_pad(zb, ct, M, pc, Mp, pcp, Mp * pcp, cs);
            if (st != ZP_OK) return st;
        }
        if (ct == CT_BF3) {
            o.kb = zb;
            o.kb_ld = pcp;
            o.kb_sub = Mp * pcp;
            st = launch_zero_kb8(o.kb, M, Mp, pc, pcp, Mp * pcp, cs);
            if (st != ZP_OK) return st;
        }
        st = launch_chain_kernel(*plan, d_r + p0, d_theta + p0, pc, J, true, o, cs);
        if (st != ZP_OK) return st;
        st = pipeline.after_basis(chunk); // the next chunk's basis may start now
        if (st != ZP_OK) return st;

        GemmDesc g{};
        g.ct = ct;
        if (ct == CT_BF3) {
            g.a = Operand{zb, pcp, Mp * pcp, LAY_KB8}; // A(i = p, k = e)
            g.b = Operand{cbuf, Bp / 16, Bp * Mp, LAY_FRAG};     // B(k = e, j = b)
        } else if (have_cache) {
            g.a = Operand{cache + CL.z_off + zsz * (size_t)p0, CL.Pp, Mp * CL.Pp, LAY_XC}; // A(i = p, k = q) = Z[q][p]
            g.b = Operand{cbuf, Bp, Mp * Bp, LAY_XC};
        } else {
            g.a = Operand{zb, pcp, Mp * pcp, LAY_XC};
            g.b = Operand{cbuf, Bp, Mp * Bp, LAY_XC};
        }
        g.M = pc;
        g.N = B;
        g.K = Mp;
        g.splits = 1;
        g.epi = EPI_STORE;
        g.C = d_f + p0 * B;
        g.ldc = B;
        st = launch_gemm(g, cs);
        if (st != ZP_OK) return st;
    }
    return pipeline.finish();
}

} // namespace zp

extern "C" {

zp_status zp_series_fwd(const int32_t *h_n, const int32_t *h_m, int64_t M, const double *d_r, const double *d_theta,
                        int64_t P, const double *d_c, int64_t B, int32_t prec, double *d_f, void *d_cache, void *d_ws,
                        size_t ws_bytes, void *stream)
{
    zp_status st = series_fwd_checks(h_n, h_m, M, d_r, d_theta, P, d_c, B, prec, d_f);
    if (st != ZP_OK || M == 0 || P == 0 || B == 0) return st;
    if (!d_ws || ((uintptr_t)d_ws & 255)) return set_error(ZP_ERR_ARG, "workspace must be non-null and 256-byte aligned");
    if ((uintptr_t)d_cache & 255) return set_error(ZP_ERR_ARG, "cache must be 256-byte aligned");
    if (chunk_for(M, P, B, ct_of(prec), true, false, d_cache != nullptr, ws_bytes) <= 0)
        return set_error(ZP_ERR_WORKSPACE, "workspace smaller than the minimum (zp_series_workspace)");
    std::shared_ptr<Plan> plan;
    st = get_plan(h_n, h_m, M, &plan);
    if (st != ZP_OK) return st;
    return series_fwd_run(*plan, M, d_r, d_theta, P, d_c, B, prec, d_f, d_cache, d_ws, ws_bytes, true,
                          (hipStream_t)stream);
}

zp_status zp_series_bwd(const int32_t *h_n, const int32_t *h_m, int64_t M, const double *d_r, const double *d_theta,
                        int64_t P, const double *d_c, int64_t B, int32_t prec, const double *d_g, const void *d_cache,
                        double *d_grad_c, double *d_grad_r, double *d_grad_theta, void *d_ws, size_t ws_bytes,
                        void *stream)
{
    zp_status st = common_checks(h_n, h_m, M, P, B, prec);
    if (st != ZP_OK) return st;
    if (M == 0 || P == 0 || B == 0) return ZP_OK;
    if (!d_r || !d_theta || !d_g) return set_error(ZP_ERR_ARG, "null pointer");
    if (!d_c && (d_grad_r || d_grad_theta)) return set_error(ZP_ERR_ARG, "null coefficients with grad_r or grad_theta");
    if (!d_ws || ((uintptr_t)d_ws & 255)) return set_error(ZP_ERR_ARG, "workspace must be non-null and 256-byte aligned");
    if (!d_grad_c && !d_grad_r && !d_grad_theta) return ZP_OK;
    if ((uintptr_t)d_cache & 255) return set_error(ZP_ERR_ARG, "cache must be 256-byte aligned");
    const int ct = ct_of(prec);
    const bool have_cache = d_cache != nullptr;
    const int64_t Pc = chunk_for(M, P, B, ct, false, true, have_cache, ws_bytes);
    if (Pc <= 0) return set_error(ZP_ERR_WORKSPACE, "workspace smaller than the minimum (zp_series_workspace)");
    hipStream_t s = (hipStream_t)stream;
    std::shared_ptr<Plan> plan;
    st = get_plan(h_n, h_m, M, &plan);
    if (st != ZP_OK) return st;

    const WsLayout L(M, Pc, B, ct, false, true, have_cache);
    char *ws = (char *)d_ws;
    const int64_t Mp = L.Mp, Bp = L.Bp;
    const bool need_rt = d_grad_r || d_grad_theta;
    // c [Mp][Bp]: H's B operand, element (x = q, k = b), k contiguous.
    void *cbuf = ws + L.c_off;
    if (need_rt) {
        st = launch_convert(d_c, M, B, B, ct, cbuf, Bp, Mp, Mp * Bp, false, s);
        if (st != ZP_OK) return st;
    }
    const CacheLayout CL(M, P, ct);
    const size_t zsz = zsize_of(ct);
    // With one chunk and few output tiles (fewer than eight per CU), the
    // dL/dr, dL/dtheta contraction runs on the helper stream beside the dL/dc
    // contraction, since neither fills the chip alone: the n <= 40 series
    // (896 tiles) went 0.61 -> 0.56 ms, n <= 64 on 8192 points (1088 tiles)
    // 4-7% faster; n <= 64 on 65536 points (8704 tiles) lost 5% with the
    // overlap and keeps one stream.
    const int64_t rt_tiles = ((M + 127) / 128) * ((Pc + 127) / 128);
    ChunkPipe side(s, d_grad_c && need_rt && Pc >= P && rt_tiles < 8 * (int64_t)device_cus());
    for (int64_t p0 = 0; p0 < P; p0 += Pc) {
        const int64_t pc = std::min(Pc, P - p0);
        const int64_t pcp = pad_up(pc);
        const void *z, *zr, *zt;
        int64_t ldz, zsub;
        if (have_cache) {
            const char *cache = (const char *)d_cache;
            z = cache + CL.z_off + zsz * (size_t)p0;
            zr = cache + CL.zr_off + dsize_of(ct) * (size_t)p0;
            zt = cache + CL.zt_off + dsize_of(ct) * (size_t)p0;
            ldz = CL.Pp;
            zsub = Mp * CL.Pp;
        } else {
            // the derivative planes only when dL/dr or dL/dtheta is wanted
            st = basis_into(*plan, d_r, d_theta, p0, pc, ct, ws + L.z_off, need_rt ? ws + L.zr_off : nullptr,
                            need_rt ? ws + L.zt_off : nullptr, pcp, Mp, M, s);
            if (st != ZP_OK) return st;
            z = ws + L.z_off;
            zr = ws + L.zr_off;
            zt = ws + L.zt_off;
            ldz = pcp;
            zsub = Mp * pcp;
        }
        // g rows of this chunk: [pcp][Bp] (and MFMA fragment order for bf16's
        // grad_c operand).
        // In FP64, with B and the chunk already multiples of the pad, g itself
        // has that layout and is read in place.
        const bool g_in_place = ct == CT_F64 && B == Bp && pc == pcp && ((uintptr_t)d_g & 15) == 0;
        const void *gbuf = g_in_place ? (const void *)(d_g + p0 * B) : (const void *)(ws + L.g_off);
        if (ct == CT_BF3) { // both contractions' operands from one read of g
            st = launch_convert_g_bwd(d_g + p0 * B, pc, B, B, ws + L.g_off, pcp * Bp,
                                      d_grad_c ? ws + L.gt_off : nullptr, Bp * pcp, pcp, Bp, s);
            if (st != ZP_OK) return st;
        } else if (!g_in_place) {
            st = launch_convert(d_g + p0 * B, pc, B, B, ct, ws + L.g_off, Bp, pcp, pcp * Bp, false, s);
            if (st != ZP_OK) return st;
        }
        st = side.start(); // both contractions' inputs are queued on s
        if (st != ZP_OK) return st;
        if (d_grad_c) {
            GemmDesc g{};
            g.ct = ct;
            g.a = Operand{z, ldz, zsub, zlay_of(ct)}; // A(i=q, k=p) = Z[q][p]
            if (ct == CT_BF3)
                g.b = Operand{ws + L.gt_off, Bp / 16, Bp * pcp, LAY_FRAG}; // B(k=p, j=b) = g[p][b]
            else
                g.b = Operand{gbuf, Bp, pcp * Bp, LAY_XC}; // B(k=p, j=b) = g[p][b]
            g.M = M;
            g.N = B;
            g.K = pcp;
            g.splits = splits_for(M, B, pcp, ct);
            g.epi = EPI_PARTIAL;
            g.C = (double *)(ws + L.pc_off);
            g.ldc = B;
            st = launch_gemm(g, s);
            if (st != ZP_OK) return st;
            st = launch_splitk_reduce(g.C, g.splits, M, B, d_grad_c, B, p0 > 0, s);
            if (st != ZP_OK) return st;
        }
        if (need_rt) {
            // H^T = c g^T tile by tile (modes down, points across), reduced
            // over the modes against dZ/dr and dZ/dtheta in the epilogue
            GemmDesc g{};
            g.ct = ct;
            g.a = Operand{cbuf, Bp, Mp * Bp, LAY_KC}; // A(i=q, k=b) = c[q][b]
            g.b = Operand{gbuf, Bp, pcp * Bp, LAY_KC}; // B(k=b, j=p) = g[p][b]
            g.M = M;
            g.N = pc;
            g.K = Bp;
            g.splits = 1;
            g.epi = EPI_COLDOT;
            g.order = 1; // tiles sharing a point panel of g run together
            g.D1 = zr;
            g.D2 = zt;
            g.ldd = ldz;
            g.d_f32 = ct != CT_F64;
            g.part = (double *)(ws + L.pr_off);
            st = launch_gemm(g, side.stream(1));
            if (st != ZP_OK) return st;
            st = launch_coldot_reduce(g.part, (int)((M + coldot_bm(ct) - 1) / coldot_bm(ct)), pc,
                                      d_grad_r ? d_grad_r + p0 : nullptr, d_grad_theta ? d_grad_theta + p0 : nullptr,
                                      side.stream(1));
            if (st != ZP_OK) return st;
        }
    }
    return side.finish();
}

} // extern "C"

extern "C" zp_status zp_series_jvp(const int32_t *h_n, const int32_t *h_m, int64_t M, const double *d_r,
                                   const double *d_theta, int64_t P, const double *d_c, int64_t B, int32_t prec,
                                   const double *d_tc, const double *d_tr, const double *d_ttheta, double *d_tf,
                                   void *d_ws, size_t ws_bytes, void *stream)
{
    zp_status st = common_checks(h_n, h_m, M, P, B, prec);
    if (st != ZP_OK) return st;
    if (P == 0 || B == 0) return ZP_OK;
    if (!d_tf || !d_r || !d_theta) return set_error(ZP_ERR_ARG, "null pointer");
    const bool with_c = d_tc != nullptr;                     // Z^T tc
    const bool with_dir = d_tr != nullptr || d_ttheta != nullptr; // (dr dZ/dr + dtheta dZ/dtheta)^T c
    if (with_dir && !d_c) return set_error(ZP_ERR_ARG, "null coefficients with a point tangent");
    hipStream_t s = (hipStream_t)stream;
    if (M == 0 || (!with_c && !with_dir)) // the tangent is zero
        return launch_zero_pad(d_tf, CT_F64, 0, 0, P, B, 0, s);
    if (!d_ws || ((uintptr_t)d_ws & 255)) return set_error(ZP_ERR_ARG, "workspace must be non-null and 256-byte aligned");
    const int ct = ct_of(prec);
    int64_t Pc = jvp_chunk_for(M, P, B, ct, ws_bytes);
    if (Pc <= 0) return set_error(ZP_ERR_WORKSPACE, "workspace smaller than the minimum (zp_series_workspace)");
    std::shared_ptr<Plan> plan;
    st = get_plan(h_n, h_m, M, &plan);
    if (st != ZP_OK) return st;
    // pipelined chunks when the workspace holds two chunk buffers (as the forward)
    const int64_t Pq = Pc == P ? pipe_chunk(P, B, ct) : 0;
    const size_t zstride = Pq > 0 ? al(ct_bytes(ct) * (size_t)(2 * pad_up(M)) * (size_t)Pq) : 0;
    ChunkPipe pipeline(s, Pq > 0 && JvpLayout(M, Pq, B, ct).total + zstride <= ws_bytes);
    if (pipeline.on()) Pc = Pq;

    const int64_t Mp = pad_up(M), Bp = pad_up(B);
    const int nblk = (with_c ? 1 : 0) + (with_dir ? 1 : 0);
    const int64_t K = nblk * Mp;
    const size_t esz = ct == CT_BF3 ? 2 : ct_bytes(ct); // per plane element
    const JvpLayout L(M, Pc, B, ct);
    char *ws = (char *)d_ws;
    char *cbuf = ws + L.c_off;
    // stacked coefficients: block 0 = tc (if any), then c (if a point tangent)
    int blk = 0;
    for (int which = 0; which < 2; ++which) {
        const double *src = which == 0 ? (with_c ? d_tc : nullptr) : (with_dir ? d_c : nullptr);
        if (!src) continue;
        if (ct == CT_BF3) // chain-major order, MFMA fragment order (block blk: k steps from blk Mp / 32)
            st = launch_convert_gather_frag(src, plan->d_perm, M, B, B, cbuf + esz * (size_t)(blk * Mp) * (size_t)Bp,
                                            Bp, Mp, Bp * K, s);
        else // [K][Bp]
            st = launch_convert(src, M, B, B, ct, cbuf + esz * (size_t)(blk * Mp) * (size_t)Bp, Bp, Mp, 0, false, s);
        if (st != ZP_OK) return st;
        ++blk;
    }
    st = pipeline.start();
    if (st != ZP_OK) return st;
    int chunk = 0;
    for (int64_t p0 = 0; p0 < P; p0 += Pc, ++chunk) {
        const int64_t pc = std::min(Pc, P - p0);
        const int64_t pcp = pad_up(pc);
        const hipStream_t cs = pipeline.stream(chunk);
        char *zbuf = ws + L.z_off + (pipeline.on() && (chunk & 1) ? zstride : 0);
        st = pipeline.before_basis(chunk);
        if (st != ZP_OK) return st;
        Planes o{};
        o.ld = pcp;
        const int zfmt = ct == CT_F64 ? F64 : F32;
        if (ct == CT_BF3) {
            o.kb_ld = pcp;
            o.kb_sub = K * pcp;
            for (int b2 = 0; b2 < nblk; ++b2) {
                st = launch_zero_kb8(zbuf + esz * (size_t)(b2 * Mp) * (size_t)pcp, M, Mp, pc, pcp, K * pcp, cs);
                if (st != ZP_OK) return st;
            }
            if (with_c) o.kb = zbuf;
            if (with_dir) o.kb_dir = zbuf + esz * (size_t)((with_c ? 1 : 0) * Mp) * (size_t)pcp;
        } else {
            o.sub = K * pcp;
            for (int b2 = 0; b2 < nblk; ++b2) {
                st = launch_zero_pad(zbuf + esz * (size_t)(b2 * Mp) * (size_t)pcp, ct, M, pc, Mp, pcp, 0, cs);
                if (st != ZP_OK) return st;
            }
            if (with_c) {
                o.plane[0] = zbuf;
                o.fmt[0] = zfmt;
            }
            if (with_dir) {
                o.dir = zbuf + esz * (size_t)((with_c ? 1 : 0) * Mp) * (size_t)pcp;
                o.dir_fmt = zfmt;
            }
        }
        if (with_dir) {
            o.dir_r = d_tr ? d_tr + p0 : nullptr;
            o.dir_th = d_ttheta ? d_ttheta + p0 : nullptr;
        }
        st = launch_chain_kernel(*plan, d_r + p0, d_theta + p0, pc, with_dir ? 1 : 0, true, o, cs);
        if (st != ZP_OK) return st;
        st = pipeline.after_basis(chunk);
        if (st != ZP_OK) return st;

        GemmDesc g{};
        g.ct = ct;
        if (ct == CT_BF3) {
            g.a = Operand{zbuf, pcp, K * pcp, LAY_KB8};
            g.b = Operand{cbuf, Bp / 16, Bp * K, LAY_FRAG};
        } else {
            g.a = Operand{zbuf, pcp, K * pcp, LAY_XC};
            g.b = Operand{cbuf, Bp, K * Bp, LAY_XC};
        }
        g.M = pc;
        g.N = B;
        g.K = K;
        g.splits = 1;
        g.epi = EPI_STORE;
        g.C = d_tf + p0 * B;
        g.ldc = B;
        st = launch_gemm(g, cs);
        if (st != ZP_OK) return st;
    }
    return pipeline.finish();
}

// ------------------------------------------------------- second order --
//
// zp_series_bwd2: the adjoint of zp_series_bwd (for double backward /
// Hessian-vector products).  For cotangents (uc, ur, ut) of its outputs
// (grad_c, grad_r, grad_theta), with D = ur dZ/dr + ut dZ/dtheta and
//   Er = ur d2Z/dr2 + ut d2Z/(dr dtheta),  Et = ur d2Z/(dr dtheta) + ut d2Z/dtheta2,
// the derivatives of L2 = <uc, grad_c> + <ur, grad_r> + <ut, grad_theta> are
//   dL2/dg     = Z^T uc + D^T c                        (zp_series_jvp)
//   dL2/dc     = D g                                   (split-K, as grad_c)
//   dL2/dr[p]  = sum_k dZ/dr_k(p) (g uc^T)[p][k] + sum_k Er_k(p) (g c^T)[p][k]
//   dL2/dth[p] = sum_k dZ/dth_k(p) (g uc^T)[p][k] + sum_k Et_k(p) (g c^T)[p][k]
// The last two are two column-dot contractions whose per-tile partials sit one
// after the other and are reduced together in a fixed order.

namespace {

struct Bwd2Layout {
    int64_t Mp, Bp, Pcp;
    int S, T;
    size_t c_off, u_off, d_off, zr_off, zt_off, er_off, et_off, g_off, gt_off, pc_off, pr_off, total;
    Bwd2Layout(int64_t M, int64_t Pc, int64_t B, int ct)
    {
        Mp = pad_up(M);
        Bp = pad_up(B);
        Pcp = pad_up(Pc);
        const size_t e = ct_bytes(ct), dsz = dsize_of(ct);
        S = splits_for(M, B, Pcp, ct);
        T = (int)((M + coldot_bm(ct) - 1) / coldot_bm(ct));
        size_t o = 0;
        c_off = o;
        o += al(e * (size_t)Mp * (size_t)Bp);
        u_off = o;
        o += al(e * (size_t)Mp * (size_t)Bp);
        d_off = o;
        o += al(e * (size_t)Mp * (size_t)Pcp);
        zr_off = o;
        o += al(dsz * (size_t)M * (size_t)Pcp);
        zt_off = o;
        o += al(dsz * (size_t)M * (size_t)Pcp);
        er_off = o;
        o += al(dsz * (size_t)M * (size_t)Pcp);
        et_off = o;
        o += al(dsz * (size_t)M * (size_t)Pcp);
        g_off = o;
        o += al(e * (size_t)Pcp * (size_t)Bp);
        gt_off = o;
        if (ct == CT_BF3) o += al(e * (size_t)Bp * (size_t)Pcp);
        pc_off = o;
        o += al(8 * (size_t)S * (size_t)M * (size_t)B);
        pr_off = o;
        o += al(8 * (size_t)(2 * T) * 2 * (size_t)Pc);
        total = o;
    }
};

int64_t bwd2_chunk_for(int64_t M, int64_t P, int64_t B, int ct, size_t ws_bytes)
{
    if (Bwd2Layout(M, P, B, ct).total <= ws_bytes) return P;
    int64_t lo = 0, hi = pad_up(P) / kPad;
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) / 2;
        if (Bwd2Layout(M, mid * kPad, B, ct).total <= ws_bytes)
            lo = mid;
        else
            hi = mid - 1;
    }
    return std::min<int64_t>(lo * kPad, P);
}

} // namespace

extern "C" {

zp_status zp_series_bwd2_workspace(int64_t M, int64_t P, int64_t B, int32_t prec, size_t *full_bytes,
                                   size_t *min_bytes)
{
    if (!full_bytes || M < 0 || P < 0 || B < 0) return set_error(ZP_ERR_ARG, "bad argument");
    if (prec < ZP_FP64 || prec > ZP_BF16X3) return set_error(ZP_ERR_PREC, "unknown prec");
    const int ct = ct_of(prec);
    const int64_t P1 = std::min<int64_t>(P, kPad);
    *full_bytes = std::max({Bwd2Layout(M, P, B, ct).total, JvpLayout(M, P, B, ct).total, (size_t)256});
    if (min_bytes) *min_bytes = std::max({Bwd2Layout(M, P1, B, ct).total, JvpLayout(M, P1, B, ct).total, (size_t)256});
    return ZP_OK;
}

zp_status zp_series_bwd2(const int32_t *h_n, const int32_t *h_m, int64_t M, const double *d_r, const double *d_theta,
                         int64_t P, const double *d_c, int64_t B, int32_t prec, const double *d_g, const double *d_uc,
                         const double *d_ur, const double *d_ut, double *d_out_g, double *d_out_c, double *d_out_r,
                         double *d_out_t, void *d_ws, size_t ws_bytes, void *stream)
{
    zp_status st = common_checks(h_n, h_m, M, P, B, prec);
    if (st != ZP_OK) return st;
    if (P == 0 || B == 0 || M == 0) return ZP_OK;
    if (!d_r || !d_theta || !d_c || !d_g) return set_error(ZP_ERR_ARG, "null pointer");
    if (!d_out_g && !d_out_c && !d_out_r && !d_out_t) return ZP_OK;
    if (!d_ws || ((uintptr_t)d_ws & 255)) return set_error(ZP_ERR_ARG, "workspace must be non-null and 256-byte aligned");
    const int ct = ct_of(prec);
    const int64_t Pc = bwd2_chunk_for(M, P, B, ct, ws_bytes);
    if (Pc <= 0 || ws_bytes < JvpLayout(M, std::min<int64_t>(P, kPad), B, ct).total)
        return set_error(ZP_ERR_WORKSPACE, "workspace smaller than the minimum (zp_series_bwd2_workspace)");
    hipStream_t s = (hipStream_t)stream;
    std::shared_ptr<Plan> plan;
    st = get_plan(h_n, h_m, M, &plan);
    if (st != ZP_OK) return st;

    const bool need_u = d_uc != nullptr;                  // terms with uc
    const bool need_dir = d_ur != nullptr || d_ut != nullptr; // terms with ur, ut
    const bool want_rt = d_out_r || d_out_t;
    const bool run_c = d_out_c && need_dir;
    const bool run_u = want_rt && need_u;   // column-dot of uc g^T with dZ/dr, dZ/dtheta
    const bool run_e = want_rt && need_dir; // column-dot of c g^T with Er, Et
    if (d_out_c && !need_dir) {
        st = launch_zero_pad(d_out_c, CT_F64, 0, 0, M, B, 0, s);
        if (st != ZP_OK) return st;
    }
    const Bwd2Layout L(M, Pc, B, ct);
    char *ws = (char *)d_ws;
    const int64_t Mp = L.Mp, Bp = L.Bp;
    if (run_e) {
        st = launch_convert(d_c, M, B, B, ct, ws + L.c_off, Bp, Mp, Mp * Bp, false, s);
        if (st != ZP_OK) return st;
    }
    if (run_u) {
        st = launch_convert(d_uc, M, B, B, ct, ws + L.u_off, Bp, Mp, Mp * Bp, false, s);
        if (st != ZP_OK) return st;
    }
    const int zfmt = ct == CT_F64 ? F64 : F32; // D as the split-K contraction reads it
    const int dfmt = ct == CT_F64 ? F64 : F32;
    const int TM = coldot_bm(ct);
    for (int64_t p0 = 0; p0 < P; p0 += Pc) {
        const int64_t pc = std::min(Pc, P - p0);
        const int64_t pcp = pad_up(pc);
        if (!run_c && !run_u && !run_e) { // the r / theta outputs of this chunk are zero
            if (d_out_r) st = launch_zero_pad(d_out_r + p0, CT_F64, 0, 0, 1, pc, 0, s);
            if (st == ZP_OK && d_out_t) st = launch_zero_pad(d_out_t + p0, CT_F64, 0, 0, 1, pc, 0, s);
            if (st != ZP_OK) return st;
            continue;
        }
        // basis-derived planes of the chunk
        Planes o{};
        o.ld = pcp;
        o.sub = Mp * pcp;
        if (run_u) {
            o.plane[1] = ws + L.zr_off;
            o.fmt[1] = dfmt;
            o.plane[4] = ws + L.zt_off;
            o.fmt[4] = dfmt;
        }
        if (run_c) {
            st = launch_zero_pad(ws + L.d_off, zct_of(ct), M, pc, Mp, pcp, Mp * pcp, s);
            if (st != ZP_OK) return st;
            o.dir = ws + L.d_off;
            o.dir_fmt = zfmt;
        }
        if (run_e) {
            o.sec_r = ws + L.er_off;
            o.sec_t = ws + L.et_off;
            o.sec_fmt = dfmt;
        }
        if (run_c || run_e) {
            o.dir_r = d_ur ? d_ur + p0 : nullptr;
            o.dir_th = d_ut ? d_ut + p0 : nullptr;
        }
        st = launch_chain_kernel(*plan, d_r + p0, d_theta + p0, pc, run_e ? 2 : 1, true, o, s);
        if (st != ZP_OK) return st;
        // the chunk's g: [pcp][Bp] (and MFMA fragment order for the bf16 dL/dc
        // operand); read in place in FP64 when it already has that layout
        const bool g_in_place = ct == CT_F64 && B == Bp && pc == pcp && ((uintptr_t)d_g & 15) == 0;
        const void *gbuf = g_in_place ? (const void *)(d_g + p0 * B) : (const void *)(ws + L.g_off);
        if (run_c && ct == CT_BF3) { // both layouts from one read of g
            st = launch_convert_g_bwd(d_g + p0 * B, pc, B, B, ws + L.g_off, pcp * Bp, ws + L.gt_off, Bp * pcp, pcp,
                                      Bp, s);
            if (st != ZP_OK) return st;
        } else if (!g_in_place) {
            st = launch_convert(d_g + p0 * B, pc, B, B, ct, ws + L.g_off, Bp, pcp, pcp * Bp, false, s);
            if (st != ZP_OK) return st;
        }
        if (run_c) {
            GemmDesc g{};
            g.ct = ct;
            g.a = Operand{ws + L.d_off, pcp, Mp * pcp, zlay_of(ct)}; // A(i=q, k=p) = D[q][p]
            if (ct == CT_BF3)
                g.b = Operand{ws + L.gt_off, Bp / 16, Bp * pcp, LAY_FRAG};
            else
                g.b = Operand{gbuf, Bp, pcp * Bp, LAY_XC};
            g.M = M;
            g.N = B;
            g.K = pcp;
            g.splits = splits_for(M, B, pcp, ct);
            g.epi = EPI_PARTIAL;
            g.C = (double *)(ws + L.pc_off);
            g.ldc = B;
            st = launch_gemm(g, s);
            if (st != ZP_OK) return st;
            st = launch_splitk_reduce(g.C, g.splits, M, B, d_out_c, B, p0 > 0, s);
            if (st != ZP_OK) return st;
        }
        if (run_u || run_e) {
            double *part = (double *)(ws + L.pr_off);
            int tiles = 0;
            for (int which = 0; which < 2; ++which) {
                if (which == 0 ? !run_u : !run_e) continue;
                GemmDesc g{};
                g.ct = ct;
                g.a = Operand{ws + (which == 0 ? L.u_off : L.c_off), Bp, Mp * Bp, LAY_KC}; // A(i=q, k=b)
                g.b = Operand{gbuf, Bp, pcp * Bp, LAY_KC};                               // B(k=b, j=p) = g[p][b]
                g.M = M;
                g.N = pc;
                g.K = Bp;
                g.splits = 1;
                g.epi = EPI_COLDOT;
                g.order = 1;
                g.D1 = ws + (which == 0 ? L.zr_off : L.er_off);
                g.D2 = ws + (which == 0 ? L.zt_off : L.et_off);
                g.ldd = pcp;
                g.d_f32 = ct != CT_F64;
                g.part = part + (size_t)tiles * 2 * (size_t)pc;
                st = launch_gemm(g, s);
                if (st != ZP_OK) return st;
                tiles += (int)((M + TM - 1) / TM);
            }
            st = launch_coldot_reduce(part, tiles, pc, d_out_r ? d_out_r + p0 : nullptr,
                                      d_out_t ? d_out_t + p0 : nullptr, s);
            if (st != ZP_OK) return st;
        }
    }
    if (d_out_g) // Z^T uc + (ur dZ/dr + ut dZ/dtheta)^T c
        return zp_series_jvp(h_n, h_m, M, d_r, d_theta, P, d_c, B, prec, d_uc, d_ur, d_ut, d_out_g, d_ws, ws_bytes,
                             stream);
    return ZP_OK;
}

} // extern "C"
