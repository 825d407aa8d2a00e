// Streaming fill: the write rate a trivial kernel reaches on this device, the
// reference the HBM-write-bound basis kernel is compared with besides the
// published peak.  One 16-byte store per lane, one lane per 16 bytes (the grid
// covers the buffer once: on gfx950 a grid-stride loop over fewer workgroups
// wrote up to a quarter slower), non-temporal or plain.
#include <hip/hip_runtime.h>

#include "zp_internal.hpp"

namespace zp {
namespace {

typedef double d2 __attribute__((ext_vector_type(2)));

template <bool NT>
__global__ __launch_bounds__(256) void fill_kernel(d2 *__restrict__ out, int64_t n2, double tail_value,
                                                   double *__restrict__ tail, d2 value)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n2) {
        if (NT)
            __builtin_nontemporal_store(value, out + i);
        else
            out[i] = value;
    } else if (i == n2 && tail) {
        *tail = tail_value;
    }
}

} // namespace
} // namespace zp

using namespace zp;

extern "C" zp_status zp_stream_fill(double *d_out, int64_t n, double value, int32_t nontemporal, void *stream)
{
    if (n < 0) return set_error(ZP_ERR_ARG, "n < 0");
    if (n == 0) return ZP_OK;
    if (!d_out || ((uintptr_t)d_out & 15)) return set_error(ZP_ERR_ARG, "output must be non-null and 16-byte aligned");
    const int64_t n2 = n / 2;
    double *tail = (n & 1) ? d_out + (n - 1) : nullptr;
    const int64_t lanes = n2 + (tail ? 1 : 0);
    const int64_t blocks = (lanes + 255) / 256;
    if (blocks > 0x7FFFFFFF) return set_error(ZP_ERR_ARG, "buffer too large for one launch");
    const d2 v = {value, value};
    if (nontemporal)
        hipLaunchKernelGGL(fill_kernel<true>, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, (d2 *)d_out,
                           n2, value, tail, v);
    else
        hipLaunchKernelGGL(fill_kernel<false>, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, (d2 *)d_out,
                           n2, value, tail, v);
    return hip_check(hipGetLastError(), "fill launch");
}
