// zp_series_fwd_noalloc: the series forward for callers that cannot allocate
// device memory.  Its workspace and the device tables of its plan live in one
// fixed array per GPU, `scratch`, instead of a caller-provided workspace and
// the library's plan cache; it runs on the caller's stream only (no helper
// stream, no events).
//
// Layout of the array on each device: the plan tables of the mode list of the
// last call (256-byte aligned length), then the forward's workspace.  A call
// with the same mode list as the previous call on that device reuses the
// tables; a new list is copied in (stream-ordered) and the call then waits
// for its stream, so that the host image of the tables outlives the copy.
// Every call on a device shares its array: calls that overlap on one device
// (other streams, other host threads without ordering) race on it.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <mutex>
#include <vector>

#include "series.hpp"

namespace {

// The array's name is a host-side stand-in in host code; kernels get the
// device address that hipGetSymbolAddress returns (DevState::ptr).
__device__ __align__(256) unsigned char scratch[ZP_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;

struct DevState {
    unsigned char *ptr = nullptr;       // device address of this device's scratch
    std::shared_ptr<zp::Plan> plan;     // plan whose tables are in scratch (null: none)
    std::vector<unsigned char> image;   // host image of those tables
};

std::mutex g_mu;
DevState g_dev[kMaxDevices];

} // namespace

using namespace zp;

extern "C" zp_status zp_series_fwd_noalloc(const int32_t *h_n, const int32_t *h_m, int64_t M, const double *d_r,
                                           const double *d_theta, int64_t P, const double *d_c, int64_t B,
                                           int32_t prec, double *d_f, void *stream)
{
    zp_status st = series_fwd_checks(h_n, h_m, M, d_r, d_theta, P, d_c, B, prec, d_f);
    if (st != ZP_OK || M == 0 || P == 0 || B == 0) return st;
    int dev = -1;
    st = hip_check(hipGetDevice(&dev), "hipGetDevice");
    if (st != ZP_OK) return st;
    if (dev < 0 || dev >= kMaxDevices) return set_error(ZP_ERR_ARG, "device ordinal beyond 63");
    hipStream_t s = (hipStream_t)stream;

    std::lock_guard<std::mutex> lock(g_mu);
    DevState &d = g_dev[dev];
    const bool same = d.plan && (int64_t)d.plan->n.size() == M && std::equal(d.plan->n.begin(), d.plan->n.end(), h_n) &&
                      std::equal(d.plan->m.begin(), d.plan->m.end(), h_m);
    std::shared_ptr<Plan> plan = same ? d.plan : build_plan_host(h_n, h_m, M);
    PlanOffsets off{};
    const size_t tables = (plan_image(*plan, nullptr, &off) + 255) / 256 * 256;
    const size_t need = tables + series_fwd_min_ws(M, P, B, prec);
    if (need > (size_t)ZP_NOALLOC_SCRATCH_BYTES) { // before any device work
        char buf[200];
        std::snprintf(buf, sizeof buf,
                      "zp_series_fwd_noalloc: %zu bytes needed (tables + smallest workspace) exceed the fixed "
                      "scratch of %zu bytes; use zp_series_fwd with a workspace",
                      need, (size_t)ZP_NOALLOC_SCRATCH_BYTES);
        return set_error(ZP_ERR_WORKSPACE, buf);
    }
    if (!d.ptr) { // set-up, once per device, with that device current
        void *p = nullptr;
        st = hip_check(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
        if (st != ZP_OK) return st;
        d.ptr = (unsigned char *)p;
    }
    if (!same) {
        d.plan.reset(); // the tables in scratch are about to change
        plan_image(*plan, &d.image, &off);
        st = hip_check(hipMemcpyAsync(d.ptr, d.image.data(), off.total, hipMemcpyHostToDevice, s),
                       "hipMemcpyAsync(plan tables)");
        if (st == ZP_OK) st = hip_check(hipStreamSynchronize(s), "hipStreamSynchronize");
        if (st != ZP_OK) return st;
        plan->device = dev;
        plan_bind(*plan, d.ptr, off);
        d.plan = plan;
    }
    return series_fwd_run(*plan, M, d_r, d_theta, P, d_c, B, prec, d_f, nullptr, d.ptr + tables,
                          (size_t)ZP_NOALLOC_SCRATCH_BYTES - tables, false, s);
}
