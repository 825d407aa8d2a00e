// Internal declarations for the three-dimensional spectral series of the
// paper's duplicated-mode use (Sec. 3, footnote): modes (n, m, l), value
// sum_j c_j R_n^|m|(r) F_m(theta) F_l(phi).  Modes that share (n, m) share
// their Zernike factor, so the library evaluates the basis once per distinct
// (n, m) pair ("owner") and folds the Fourier factor of phi into the
// coefficients.
#pragma once

#include <memory>
#include <vector>

#include "series.hpp"

namespace zp {

struct Plan3 {
    std::vector<int32_t> n, m, l; // the caller's mode list (cache key)
    std::vector<int32_t> un, um;  // distinct (n, m) pairs, in order of first appearance
    std::vector<int32_t> owner;   // mode j -> its pair u
    int device = 0;
    void *dmem = nullptr;
    // device: uptr [U+1], jl [J] (modes of pair u at jl[uptr[u] .. uptr[u+1]),
    // ascending j), owner [J], l [J]
    const int32_t *d_uptr = nullptr, *d_jl = nullptr, *d_owner = nullptr, *d_l = nullptr;
    ~Plan3();
};

// Distinct (n, m) pairs of a mode list (host only): owner[j] and the pairs.
void dedup_modes(const int32_t *n, const int32_t *m, int64_t J, std::vector<int32_t> &un, std::vector<int32_t> &um,
                 std::vector<int32_t> &owner);

zp_status get_plan3(const int32_t *n, const int32_t *m, const int32_t *l, int64_t J, std::shared_ptr<Plan3> *out);
void clear_plans3();

// T[u][q*B + b] = sum over modes j of pair u of c[j][b] F_{l_j}(phi_q)
// (deriv: dF/dphi instead of F).  T is [U][Q*B], row-major.
zp_status launch_fourier_mix(const Plan3 &p, const double *c, int64_t B, const double *phi, int64_t Q, bool deriv,
                             double *T, hipStream_t s);

// grad_c[j][b] = sum_q F_{l_j}(phi_q) gT[owner_j][q*B + b].
zp_status launch_fourier_unmix(const Plan3 &p, const double *gT, int64_t B, const double *phi, int64_t Q,
                               double *grad_c, hipStream_t s);

// grad_phi[q] = sum_j sum_b dF_{l_j}/dphi(phi_q) c[j][b] gT[owner_j][q*B + b],
// summed in a fixed order.
zp_status launch_fourier_phi_grad(const Plan3 &p, const double *gT, const double *c, int64_t B, const double *phi,
                                  int64_t Q, double *grad_phi, hipStream_t s);

} // namespace zp
