// Internal declarations shared by the host API (zp_api.cpp), the plan builder
// (plan.cpp) and the HIP kernels.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/zp.h"

namespace zp {

// ---------------------------------------------------------------- plan --
//
// A plan is everything about a mode list that does not depend on the points:
// the modes grouped by alpha = |m| into recurrence chains (one chain per
// alpha, shared by every n of that alpha, as in Algorithm 1), the per-step
// recurrence coefficients of each chain, and the list of (K, column) pairs
// each chain must emit.
//
// Recurrence (endpoint-anchored difference form of the beta = 0 Jacobi
// recurrence of Sec. 2).  With x = 1 - 2r^2 and v_k the Jacobi polynomial
// P_k^{(alpha,0)}(x) normalised to 1 at one end of [-1, 1]:
//   low anchor (x = +1):  s = 2r^2,      v_k = P_k / C(k+alpha, k)
//   high anchor (x = -1): s = 2(1-r^2),  v_k = (-1)^k P_k
// the three-term recurrence becomes, with d_k = v_k - v_{k-1},
//   d_k = cc_k d_{k-1} - bs_k s v_{k-1},   v_k = v_{k-1} + d_k,
//   v_0 = 1, d_0 = 0, cc_1 = 0,
// low:  cc_k = (k-1)^2 (2k+alpha) / ((k+alpha)^2 (2k+alpha-2)),
//       bs_k = (2k+alpha-1)(2k+alpha) / (2 (k+alpha)^2)
// high: cc_k = (k+alpha-1)(k-1)(2k+alpha) / (k (k+alpha)(2k+alpha-2)),
//       bs_k = (2k+alpha-1)(2k+alpha) / (2k (k+alpha)).
// It is an exact algebraic rewrite of the paper's recurrence (the sum rule
// of its coefficients makes v = 1 at s = 0 a fixed point), so the end point
// is reproduced exactly and rounding errors vanish with s.
constexpr int kSegEmits = 32; // emissions per chain piece

struct Chain {
    int32_t alpha;    // |m| of every mode on this chain
    int32_t kmax;     // largest K requested on this chain
    int32_t coef_off; // first Coef of this chain (entry k-1 holds step k)
    int32_t emit_off; // first Emit of this chain
    int32_t emit_cnt; // number of Emits
    int32_t pad;
};

struct Coef {
    double cc_lo, bs_lo, cc_hi, bs_hi;
};

struct Emit {
    int32_t K;     // Jacobi degree (n - alpha)/2
    int32_t col;   // output column (position in the caller's mode list)
    int32_t flags; // bit 0: m < 0 (sin column of the basis)
    int32_t pad;
    double a_lo; // (-1)^K C(K+alpha, K): low-anchor factor from v_K to R / r^alpha
};

struct Plan {
    int device = -1;
    std::vector<int32_t> n, m; // the key
    std::vector<Chain> chains; // in launch order (most work first)
    // The same chains cut into pieces of at most kSegEmits emissions (piece
    // boundaries on multiples of 8 of the emission index).  A piece walks its
    // chain from k = 0 to its own last K and emits only its range, so it costs
    // a short recurrence prefix again; the launcher uses pieces when there
    // are too few point tiles to fill the chip with whole chains.
    std::vector<Chain> pieces;
    std::vector<Coef> coefs;
    std::vector<Emit> emits;
    int32_t nmax = 0;
    // device copies (one allocation)
    void *dmem = nullptr;
    const Chain *d_chains = nullptr;
    const Chain *d_pieces = nullptr;
    const Coef *d_coefs = nullptr;
    const Emit *d_emits = nullptr;
    const int32_t *d_perm = nullptr; // d_perm[e] = emits[e].col: chain-major order -> column
    // Coefficient table of the direct (closed-form) evaluation, built on first
    // use: per mode, for j = 0..3, the K+1 values c_s (n-2s)!/(n-2s-j)! of
    // d^j/dr^j of Eq. (radial-part-eq), rounded to double.
    std::once_flag direct_once;
    zp_status direct_status = ZP_OK;
    void *d_direct = nullptr;
    const int64_t *d_direct_off = nullptr; // per mode: offset of its 4 (K+1) coefficients
    const int32_t *d_direct_n = nullptr, *d_direct_m = nullptr;
    const double *d_direct_coef = nullptr;
    // Column table of the Zernike-recursion comparator, built on first use:
    // for every (n, alpha) of the triangle n <= nmax in row order (alpha =
    // n%2, n%2+2, ..., n), the output columns of the requested modes with
    // that (n, |m|): zrec_off [entries+1] into zrec_cols [M].
    std::once_flag zrec_once;
    zp_status zrec_status = ZP_OK;
    void *d_zrec = nullptr;
    const int32_t *d_zrec_off = nullptr, *d_zrec_cols = nullptr;
    ~Plan();
};

// Device table for zp_radial_zernike_recursion (uploaded once per plan).
zp_status get_zrec_table(Plan &plan);

// Zernike-recursion evaluation (Eq. zernike-recursion): out[j][i][p], j <= J.
constexpr int kZrecNmax = 60;
zp_status launch_zrec_kernel(const Plan &plan, const double *d_r, int64_t P, int J, double *out, hipStream_t s);

// Device table for zp_radial_direct (uploaded once per plan).
zp_status get_direct_table(Plan &plan);

// Direct evaluation of the closed form: out[j][i][p] for j <= J.
zp_status launch_direct_kernel(const Plan &plan, const double *d_r, int64_t P, int J, double *out, hipStream_t s);

// Validates the modes; returns ZP_OK or ZP_ERR_MODE (with the offending index
// in *bad).
zp_status validate_modes(const int32_t *n, const int32_t *m, int64_t M, int64_t *bad);

// Host-side construction of a plan (no device work).
std::shared_ptr<Plan> build_plan_host(const int32_t *n, const int32_t *m, int64_t M);

// Byte offsets of a plan's device tables within one contiguous image (the
// chains and pieces start at offset 0).
struct PlanOffsets {
    size_t coefs, emits, perm, total;
};
// Size of the image (and, if host is not null, the image itself).
size_t plan_image(const Plan &p, std::vector<unsigned char> *host, PlanOffsets *o);
// Point the plan's device table pointers into an image at base.
void plan_bind(Plan &p, const void *base, const PlanOffsets &o);

// Cached plan for the current device, uploaded on first use.
zp_status get_plan(const int32_t *n, const int32_t *m, int64_t M, std::shared_ptr<Plan> *out);
void clear_plans();
void clear_plans3(); // three-dimensional series tables (series3d.cpp)

// ------------------------------------------------------------- outputs --

enum PlaneFmt : int32_t { F64 = 0, F32 = 1, B16X3 = 2 };

// Where the chain kernel writes.  plane[q] for q = 0..4 is R (or Z), d/dr,
// d2/dr2, d3/dr3, d/dtheta; null planes are not written.  Column i of a plane
// starts ld elements after column i-1.  A B16X3 plane is three bf16 planes
// (hi, mid, lo) sub elements apart.
// kb, if not null, receives Z once more as three bf16 planes (kb_sub apart) in
// the k-blocked layout the series forward contracts over: the mode index is
// the emission index e (chain-major order, see Plan::d_perm) and element
// (e, p) sits at ((e/8)*kb_ld + p)*8 + e%8.
// dir, if not null, receives the directional derivative
//   dZ = dr[p] dZ/dr + dtheta[p] dZ/dtheta
// of the basis along per-point tangents (dr, dtheta; either may be null),
// in format dir_fmt with the planes' ld and sub; kb_dir, if not null, gets its
// k-blocked bf16 copy (like kb).
// sec_r / sec_t, if not null (with J = 2 and the basis), receive the
// derivatives of that directional derivative along r and theta:
//   sec_r = dr[p] d2Z/dr2 + dtheta[p] d2Z/(dr dtheta)
//   sec_t = dr[p] d2Z/(dr dtheta) + dtheta[p] d2Z/dtheta2
// in format sec_fmt with the planes' ld and sub.
struct Planes {
    void *plane[5];
    int64_t ld;
    int64_t sub;
    int32_t fmt[5];
    void *kb;
    int64_t kb_ld;
    int64_t kb_sub;
    void *dir;
    int32_t dir_fmt;
    const double *dir_r;
    const double *dir_th;
    void *kb_dir;
    void *sec_r;
    void *sec_t;
    int32_t sec_fmt;
};

// Launch the chain kernel: radial only (angular = false) or basis.  J is the
// highest radial derivative needed (0..3).
zp_status launch_chain_kernel(const Plan &plan, const double *d_r, const double *d_theta, int64_t P,
                              int J, bool angular, const Planes &out, hipStream_t s);

// The basis on a tensor grid: point p = i * nt + j at radius r[i], angle
// theta[j] (i < nr, j < nt), into plain planes with ld = nr * nt.
zp_status launch_chain_kernel_polar(const Plan &plan, const double *d_r, int64_t nr, const double *d_theta, int64_t nt,
                                    int J, const Planes &out, hipStream_t s);

// Error plumbing.
zp_status set_error(zp_status s, const std::string &msg);
zp_status hip_check(hipError_t e, const char *what);

} // namespace zp
