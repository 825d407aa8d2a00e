// Radial polynomials by the Zernike recursion of Sec. 2 (Eq. zernike-recursion):
//   R_n^a(r) = r [R_{n-1}^{|a-1|}(r) + R_{n-1}^{a+1}(r)] - R_{n-2}^a(r),
// with R_0^0 = 1 and every R_n^a with a > n or n < 0 taken as zero (which
// also gives R_n^n = r^n).  The r-derivatives follow by differentiating the
// product with r:  R^(j) = r X^(j) + j X^(j-1) - Y^(j).
// A comparator for the paper's accuracy study, which contrasts the Jacobi
// recurrence with other evaluation methods; zp_radial is the production path.
//
// Work decomposition: one thread per point walks the whole (n, a) triangle up
// to the largest requested n.  Row n only needs rows n-1 and n-2, and entry a
// of row n replaces entry a of row n-2 in place, so two buffers per point (one
// per parity of n) of nmax/2 + 1 entries x (J+1) orders live in LDS, laid out
// [parity][entry][order][thread] (consecutive threads, consecutive banks).
// Requested modes are stored when their (n, |m|) entry is formed.
#include <hip/hip_runtime.h>

#include "zp_internal.hpp"

namespace zp {
namespace {

template <int J>
__global__ void zrec_kernel(const int32_t *__restrict__ off, const int32_t *__restrict__ cols,
                            const double *__restrict__ r, int64_t P, int64_t M, int nmax, double *__restrict__ out)
{
    extern __shared__ double lds[];
    const int nt = blockDim.x;
    const int tid = threadIdx.x;
    const int E = nmax / 2 + 1;
    const int64_t p = (int64_t)blockIdx.x * nt + tid;
    const bool live = p < P;
    const double x = live ? r[p] : 0.0;
    auto at = [&](int q, int i, int j) -> double & { return lds[((q * E + i) * (J + 1) + j) * nt + tid]; };
    for (int q = 0; q < 2; ++q)
        for (int i = 0; i < E; ++i)
            for (int j = 0; j <= J; ++j) at(q, i, j) = 0.0;
    int t = 0; // triangle entry of (n, a)
    for (int n = 0; n <= nmax; ++n) {
        const int q = n & 1;
        for (int a = q; a <= n; a += 2, ++t) {
            const int i = (a - q) >> 1;
            double v[J + 1];
            if (n == 0) {
                v[0] = 1.0;
#pragma unroll
                for (int j = 1; j <= J; ++j) v[j] = 0.0;
            } else {
                // row n-1 (parity 1-q) holds entries (a' - (1-q))/2; entries
                // beyond its last were never written and are zero
                const int i1 = ((a == 0 ? 1 : a - 1) - (1 - q)) >> 1; // |a-1|
                const int i2 = (a + 1 - (1 - q)) >> 1;                // a+1
                double X[J + 1];
#pragma unroll
                for (int j = 0; j <= J; ++j) X[j] = at(1 - q, i1, j) + (i2 < E ? at(1 - q, i2, j) : 0.0);
#pragma unroll
                for (int j = 0; j <= J; ++j)
                    v[j] = __builtin_fma(x, X[j], (j ? (double)j * X[j > 0 ? j - 1 : 0] : 0.0) - at(q, i, j));
            }
#pragma unroll
            for (int j = 0; j <= J; ++j) at(q, i, j) = v[j];
            for (int c = off[t]; c < off[t + 1]; ++c) {
                if (!live) continue;
                const int64_t col = cols[c];
#pragma unroll
                for (int j = 0; j <= J; ++j) out[((int64_t)j * M + col) * P + p] = v[j];
            }
        }
    }
}

template <int J>
zp_status launch_j(const Plan &plan, const double *r, int64_t P, double *out, hipStream_t s)
{
    int dev = 0, limit = 0;
    zp_status st = hip_check(hipGetDevice(&dev), "hipGetDevice");
    if (st == ZP_OK) st = hip_check(hipDeviceGetAttribute(&limit, hipDeviceAttributeMaxSharedMemoryPerBlock, dev),
                                    "hipDeviceGetAttribute");
    if (st != ZP_OK) return st;
    const int nmax = plan.nmax;
    const size_t per_thread = 2 * (size_t)(nmax / 2 + 1) * (J + 1) * sizeof(double);
    int nt = 64;
    while (nt > 16 && per_thread * (size_t)nt > (size_t)limit) nt /= 2;
    if (per_thread * (size_t)nt > (size_t)limit) return set_error(ZP_ERR_ARG, "recursion triangle too large for LDS");
    const size_t bytes = per_thread * (size_t)nt;
    const int64_t blocks = (P + nt - 1) / nt;
    if (blocks > INT32_MAX) return set_error(ZP_ERR_ARG, "too many points for one launch");
    hipLaunchKernelGGL(zrec_kernel<J>, dim3((unsigned)blocks), dim3(nt), bytes, s, plan.d_zrec_off, plan.d_zrec_cols,
                       r, P, (int64_t)plan.n.size(), nmax, out);
    return hip_check(hipGetLastError(), "recursion kernel launch");
}

} // namespace

zp_status launch_zrec_kernel(const Plan &plan, const double *d_r, int64_t P, int J, double *out, hipStream_t s)
{
    if (plan.nmax > kZrecNmax) return set_error(ZP_ERR_ARG, "the Zernike-recursion comparator takes n <= 60");
    switch (J) {
    case 0: return launch_j<0>(plan, d_r, P, out, s);
    case 1: return launch_j<1>(plan, d_r, P, out, s);
    case 2: return launch_j<2>(plan, d_r, P, out, s);
    default: return launch_j<3>(plan, d_r, P, out, s);
    }
}

} // namespace zp
