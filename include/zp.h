/*
 * zp.h -- C ABI of libzp, the MI355X (gfx950) library for radial Zernike
 * polynomials, the full Zernike basis and the differentiable Zernike series.
 *
 * Mathematics (ZERNIPAX paper, Sec. 2):
 *   mode (n, m): n >= 0, |m| <= n, n - |m| even                 (Sec. 2)
 *   R_n^{|m|}(r) = (-1)^K r^|m| P_K^{(|m|,0)}(1 - 2r^2), K = (n - |m|)/2
 *                                                              (Eq. jacobi-relation)
 *   Z_n^m(r, theta) = R_n^{|m|}(r) cos(m theta)       for m >= 0
 *                   = R_n^{|m|}(r) sin(|m| theta)     for m < 0  (Eq. zernike-poly)
 * Polynomials are unnormalised, as in the paper.
 *
 * Conventions shared by every entry point
 *   - Pointers named h_* are host memory, d_* are device memory of the
 *     current HIP device, and `stream` belongs to that device.  The caller
 *     owns every buffer; the library only reads inputs and writes outputs.
 *   - Mode lists are host arrays (they are metadata, like shapes).  Duplicates
 *     are allowed: every column is written, in order (the paper's duplicated-
 *     mode use, Sec. 3 footnote).  n may not exceed ZP_N_MAX.
 *   - Point arrays are FP64 device arrays.  r is meant to lie in [0, 1] and
 *     theta in [0, 2 pi]; values outside are evaluated as polynomials /
 *     trigonometric functions but accuracy is only guaranteed inside.  r is
 *     not range-checked (that would need a device round trip); NaN in gives
 *     NaN out.
 *   - Output planes are laid out [plane][mode][point], point fastest, i.e.
 *     each plane is the paper's (points x modes) output array in column-major
 *     order (Algorithms 1 and 2, "Output").
 *   - Every call is asynchronous on `stream` (a hipStream_t; NULL means the
 *     default stream).  The series forward, backward and forward-mode
 *     derivative may run part of their work on one library-owned stream per
 *     device (default
 *     priority, created on first use); it waits for `stream` through an event
 *     at the start of the call, and `stream` waits for it before the call's
 *     last piece of work, so to the caller the call is ordered on `stream`
 *     alone.  All argument validation happens on the host before
 *     any device work: on error nothing is written and no kernel is launched.
 *     M == 0 or P == 0 (or B == 0 for the series) is a successful no-op.
 *   - The library allocates device memory only for its cached per-mode-list
 *     tables ("plans"), which zp_cache_clear() releases, and holds one fixed
 *     array per GPU for zp_series_fwd_noalloc.  Calls from several
 *     host threads are safe; calls that write the same buffers race, as any
 *     asynchronous work does.
 */
#ifndef ZP_H
#define ZP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum zp_status {
    ZP_OK = 0,
    ZP_ERR_MODE = 1,      /* a mode has n < 0, |m| > n, n - |m| odd, or n > ZP_N_MAX */
    ZP_ERR_ARG = 2,       /* null pointer with work to do, negative size, bad mask */
    ZP_ERR_ORDER = 3,     /* derivative order outside 0..3 */
    ZP_ERR_WORKSPACE = 4, /* workspace smaller than the minimum for this call */
    ZP_ERR_HIP = 5,       /* a HIP runtime call or kernel launch failed */
    ZP_ERR_PREC = 6       /* unknown zp_prec value */
} zp_status;

/* Contraction precision of the series (the basis itself is always evaluated
 * in FP64). */
typedef enum zp_prec {
    ZP_FP64 = 0,  /* FP64 MFMA, FP64 accumulation */
    ZP_FP32 = 1,  /* operands rounded to FP32, FP32 MFMA */
    ZP_BF16X3 = 2 /* operands rounded to FP32 and split into three BF16 parts
                     (hi + mid + lo), six BF16 MFMA cross products with FP32
                     accumulation */
} zp_prec;

#define ZP_N_MAX 1000    /* largest radial order n accepted */
#define ZP_L_MAX 1048576 /* largest |l| of a toroidal Fourier index (zp_series3d_*) */

/* Output selection bits of zp_basis. */
#define ZP_Z 1u       /* Z                        */
#define ZP_DR 2u      /* dZ/dr                    */
#define ZP_DR2 4u     /* d2Z/dr2                  */
#define ZP_DR3 8u     /* d3Z/dr3                  */
#define ZP_DTHETA 16u /* dZ/dtheta                */

/*
 * zp_radial -- radial polynomials and their r-derivatives.
 * Paper: Eq. (jacobi-relation) with the Jacobi recurrence Eq.
 * (jacobi-recursion) / its beta = 0 form, and the derivative identity with
 * the Pochhammer symbol (Sec. 2); one recurrence chain per |m| shared by all n
 * (Algorithm 1).
 *   h_n, h_m  host int32[M]: modes; the sign of m is ignored (R uses |m|)
 *   d_r       device double[P]
 *   max_dr    0..3: highest r-derivative computed
 *   d_out     device double[(max_dr+1) * M * P]: plane j holds d^jR/dr^j,
 *             element (j, i, p) at ((j*M + i)*P + p)
 * Errors: ZP_ERR_MODE, ZP_ERR_ORDER, ZP_ERR_ARG (negative M or P, null
 * pointer with M*P > 0), ZP_ERR_HIP.
 */
zp_status zp_radial(const int32_t *h_n, const int32_t *h_m, int64_t M, const double *d_r, int64_t P,
                    int32_t max_dr, double *d_out, void *stream);

/*
 * zp_basis -- full Zernike basis and selected derivatives, Eq. (zernike-poly).
 *   h_n, h_m  host int32[M]: modes; m >= 0 selects cos(m theta), m < 0
 *             selects sin(|m| theta)
 *   d_r, d_theta  device double[P]
 *   mask      nonzero subset of ZP_Z | ZP_DR | ZP_DR2 | ZP_DR3 | ZP_DTHETA
 *   d_out     device double[popcount(mask) * M * P]: the selected outputs in
 *             increasing bit order, each a [M][P] plane.  dZ/dtheta is
 *             -m R sin(m theta) for m >= 0 and |m| R cos(|m| theta) for m < 0.
 * Errors: as zp_radial; ZP_ERR_ARG also for mask == 0 or bits above 4.
 */
zp_status zp_basis(const int32_t *h_n, const int32_t *h_m, int64_t M, const double *d_r,
                   const double *d_theta, int64_t P, uint32_t mask, double *d_out, void *stream);

/*
 * zp_basis_polar -- zp_basis on a tensor-product polar grid (the grids of the
 * paper's timings and of spectral methods, Sec. 4): NR radii times NT
 * angles, point p = i * NT + j at (r[i], theta[j]), angle fastest.  The
 * output is exactly that of zp_basis given the NR * NT points (r_p, theta_p)
 * (bit for bit): the radial recurrence runs once per radius and lane instead
 * of once per point where NT is even.
 *   d_r       device double[NR]
 *   d_theta   device double[NT]
 *   mask      as zp_basis
 *   d_out     device double[popcount(mask) * M * NR * NT], layout as zp_basis
 * Errors: as zp_basis; ZP_ERR_ARG also for NR or NT negative or NR * NT
 * overflowing int64.
 */
zp_status zp_basis_polar(const int32_t *h_n, const int32_t *h_m, int64_t M, const double *d_r, int64_t NR,
                         const double *d_theta, int64_t NT, uint32_t mask, double *d_out, void *stream);

/*
 * zp_radial_direct -- the same outputs as zp_radial, evaluated directly from
 * the closed form Eq. (radial-part-eq): each term c_s r^(n-2s) (and its
 * r-derivatives) formed in FP64 and summed in order of s.  This is the
 * comparator of the paper's accuracy study (Sec. 4): its error grows quickly
 * with n - |m| (alternating terms of very different size), and for large n
 * the coefficients overflow FP64 (inf / NaN outputs).  For accuracy
 * comparisons only; zp_radial is the accurate path.  Arguments and errors as
 * zp_radial; at most 65535 modes per call.
 */
zp_status zp_radial_direct(const int32_t *h_n, const int32_t *h_m, int64_t M, const double *d_r, int64_t P,
                           int32_t max_dr, double *d_out, void *stream);

/*
 * zp_radial_zernike_recursion -- the same outputs as zp_radial, by the
 * Zernike recursion Eq. (zernike-recursion), R_n^m = r (R_{n-1}^{|m-1|} +
 * R_{n-1}^{m+1}) - R_{n-2}^m, over the whole (n, |m|) triangle up to the
 * largest requested n, with out-of-range terms zero; derivatives by
 * differentiating the recursion.  A second comparator for the paper's
 * accuracy study (Sec. 2 and 4), for n <= 60 only.  Arguments and errors as
 * zp_radial; ZP_ERR_ARG also for n > 60.
 */
zp_status zp_radial_zernike_recursion(const int32_t *h_n, const int32_t *h_m, int64_t M, const double *d_r, int64_t P,
                                      int32_t max_dr, double *d_out, void *stream);

/*
 * Zernike series f(r_p, theta_p)_b = sum_k c[k][b] Z_k(r_p, theta_p) for B
 * coefficient sets at once (the basis contracted with coefficients; the
 * paper's use of Zernike polynomials as a spectral basis, Sec. 1 and 3), and
 * its adjoint.  Layouts: c [M][B], f and g [P][B], all row-major FP64.
 *
 * Memory: the contraction needs a caller-provided device workspace d_ws of
 * ws_bytes.  zp_series_workspace() reports the size that processes all P
 * points in one pass; any smaller size down to the reported minimum is
 * accepted and processes the points in chunks.  d_ws must be 256-byte
 * aligned.  Its contents are scratch between calls.
 *
 * Basis cache: the forward can keep the basis for the backward in a
 * caller-provided device buffer d_cache of zp_series_cache_bytes() bytes
 * (opaque layout, depends on prec).  If the backward receives d_cache == NULL
 * it recomputes the basis chunk by chunk instead (for when points x modes is
 * too large to keep).  A cache is valid only for the same modes, points, and
 * prec as the forward that filled it.
 */
zp_status zp_series_workspace(int64_t M, int64_t P, int64_t B, int32_t prec, size_t *full_bytes,
                              size_t *min_bytes);
zp_status zp_series_cache_bytes(int64_t M, int64_t P, int32_t prec, size_t *bytes);

/*
 * zp_series_fwd -- f = Z^T c (f [P][B] = sum over modes).
 *   d_c       device double[M*B]
 *   d_f       device double[P*B] (output)
 *   d_cache   nullable device buffer of zp_series_cache_bytes(M, P, prec):
 *             filled for a later zp_series_bwd
 * Errors: as zp_basis, plus ZP_ERR_PREC and ZP_ERR_WORKSPACE.
 */
zp_status zp_series_fwd(const int32_t *h_n, const int32_t *h_m, int64_t M, const double *d_r,
                        const double *d_theta, int64_t P, const double *d_c, int64_t B, int32_t prec,
                        double *d_f, void *d_cache, void *d_ws, size_t ws_bytes, void *stream);

/*
 * zp_series_bwd -- adjoint of zp_series_fwd for an upstream gradient g = dL/df:
 *   grad_c[k][b]    = sum_p Z_k(p) g[p][b]
 *   grad_r[p]       = sum_b g[p][b] sum_k dZ_k/dr(p) c[k][b]
 *   grad_theta[p]   = sum_b g[p][b] sum_k dZ_k/dtheta(p) c[k][b]
 * Each of d_grad_c [M*B], d_grad_r [P], d_grad_theta [P] is nullable (not
 * computed when NULL); results are overwritten, not accumulated.  d_c is read
 * only for grad_r / grad_theta and may be NULL when both are NULL.  Sums have
 * a fixed order (no floating-point atomics): repeated calls are bitwise equal.
 */
zp_status zp_series_bwd(const int32_t *h_n, const int32_t *h_m, int64_t M, const double *d_r,
                        const double *d_theta, int64_t P, const double *d_c, int64_t B, int32_t prec,
                        const double *d_g, const void *d_cache, double *d_grad_c, double *d_grad_r,
                        double *d_grad_theta, void *d_ws, size_t ws_bytes, void *stream);

/*
 * zp_series_jvp -- forward-mode derivative (Jacobian-vector product) of
 * zp_series_fwd along tangents (tc, tr, ttheta) of (c, r, theta):
 *   tf[p][b] = sum_k Z_k(p) tc[k][b]
 *            + sum_k (tr[p] dZ_k/dr(p) + ttheta[p] dZ_k/dtheta(p)) c[k][b]
 * (the paper's forward-mode automatic differentiation, Sec. 3).
 *   d_tc      nullable device double[M*B]
 *   d_tr, d_ttheta  nullable device double[P]
 *   d_c       device double[M*B]; may be NULL when tr and ttheta are both NULL
 *   d_tf      device double[P*B] (output; all zeros if every tangent is NULL)
 * The two sums are one contraction over a stacked mode index, in the
 * precision prec.  Workspace as for zp_series_fwd (zp_series_workspace covers
 * it).  Errors: as zp_series_fwd.
 */
zp_status zp_series_jvp(const int32_t *h_n, const int32_t *h_m, int64_t M, const double *d_r,
                        const double *d_theta, int64_t P, const double *d_c, int64_t B, int32_t prec,
                        const double *d_tc, const double *d_tr, const double *d_ttheta, double *d_tf, void *d_ws,
                        size_t ws_bytes, void *stream);

/*
 * zp_series_bwd2 -- adjoint of zp_series_bwd, for second-order derivatives
 * (double backward, Hessian-vector products; the paper's Hessian use of the
 * automatic differentiation, Sec. 3).  Given cotangents uc [M*B], ur [P],
 * ut [P] of zp_series_bwd's outputs (grad_c, grad_r, grad_theta) for the same
 * (modes, r, theta, c, g), it returns the derivatives of
 *   L2 = <uc, grad_c> + <ur, grad_r> + <ut, grad_theta>
 * with respect to g, c, r and theta:
 *   out_g[p][b] = sum_k Z_k(p) uc[k][b] + sum_k D_k(p) c[k][b]
 *   out_c[k][b] = sum_p D_k(p) g[p][b]
 *   out_r[p]    = sum_b g[p][b] sum_k (dZ_k/dr(p) uc[k][b] + Er_k(p) c[k][b])
 *   out_t[p]    = sum_b g[p][b] sum_k (dZ_k/dtheta(p) uc[k][b] + Et_k(p) c[k][b])
 * with D = ur dZ/dr + ut dZ/dtheta, Er = ur d2Z/dr2 + ut d2Z/(dr dtheta),
 * Et = ur d2Z/(dr dtheta) + ut d2Z/dtheta2 (d2Z/dtheta2 = -m^2 Z).
 *   d_c, d_g  device double[M*B], [P*B] (required)
 *   d_uc, d_ur, d_ut  nullable cotangents (NULL = zero)
 *   d_out_g [P*B], d_out_c [M*B], d_out_r [P], d_out_t [P]: nullable outputs,
 *             overwritten
 * Contractions run in prec.  Workspace: zp_series_bwd2_workspace (one pass /
 * minimum).  Sums have a fixed order.  Errors: as zp_series_bwd.
 */
zp_status zp_series_bwd2_workspace(int64_t M, int64_t P, int64_t B, int32_t prec, size_t *full_bytes,
                                   size_t *min_bytes);
zp_status zp_series_bwd2(const int32_t *h_n, const int32_t *h_m, int64_t M, const double *d_r, const double *d_theta,
                         int64_t P, const double *d_c, int64_t B, int32_t prec, const double *d_g, const double *d_uc,
                         const double *d_ur, const double *d_ut, double *d_out_g, double *d_out_c, double *d_out_r,
                         double *d_out_t, void *d_ws, size_t ws_bytes, void *stream);

/*
 * Three-dimensional spectral series (the paper's duplicated-mode use, Sec. 3
 * footnote): a Zernike basis on the polar plane times a Fourier basis in a
 * periodic third coordinate phi,
 *   f[p][q][b] = sum_j c[j][b] R_{n_j}^{|m_j|}(r_p) F_{m_j}(theta_p) F_{l_j}(phi_q),
 * where F_m(theta) is the angular factor of Eq. (zernike-poly) and
 * F_l(phi) = cos(l phi) for l >= 0, sin(|l| phi) for l < 0.  Points form a
 * tensor grid: P polar points (r_p, theta_p) times Q angles phi_q.
 *
 * Modes j = 0..J-1 are triples (n_j, m_j, l_j): host int32 arrays h_n, h_m,
 * h_l.  Modes sharing (n, m) with different l are "duplicated": their
 * Zernike factor is evaluated once, the Fourier factor is folded into the
 * coefficients, and the contraction runs over the U distinct (n, m) pairs
 * (U = J / (2L+1) for every l in [-L, L]).  Any order and any repetition of
 * triples is accepted; |l| <= ZP_L_MAX.
 *
 * Layouts (row-major FP64): c [J][B], f and g [P][Q][B], phi [Q].
 * Workspace: zp_series3d_workspace() reports the size for one pass and the
 * minimum (smaller sizes process the points in chunks); 256-byte aligned.
 * The basis cache (zp_series3d_cache_bytes) works as for the planar series:
 * filled by the forward, used by the backward if non-NULL, valid only for the
 * same modes, polar points and prec.
 * J == 0, P == 0, Q == 0 or B == 0 is a successful no-op.
 * Errors: as zp_series_fwd; ZP_ERR_MODE also for |l| > ZP_L_MAX.
 */
zp_status zp_series3d_workspace(const int32_t *h_n, const int32_t *h_m, const int32_t *h_l, int64_t J, int64_t P,
                                int64_t Q, int64_t B, int32_t prec, size_t *full_bytes, size_t *min_bytes);
zp_status zp_series3d_cache_bytes(const int32_t *h_n, const int32_t *h_m, const int32_t *h_l, int64_t J, int64_t P,
                                  int32_t prec, size_t *bytes);

/* zp_series3d_fwd -- f = the series above; d_f [P][Q][B] is overwritten. */
zp_status zp_series3d_fwd(const int32_t *h_n, const int32_t *h_m, const int32_t *h_l, int64_t J, const double *d_r,
                          const double *d_theta, int64_t P, const double *d_phi, int64_t Q, const double *d_c,
                          int64_t B, int32_t prec, double *d_f, void *d_cache, void *d_ws, size_t ws_bytes,
                          void *stream);

/*
 * zp_series3d_bwd -- adjoint of zp_series3d_fwd for an upstream gradient
 * g = dL/df [P][Q][B]:
 *   grad_c[j][b]   = sum_p sum_q Z_j(p) F_{l_j}(phi_q) g[p][q][b]
 *   grad_r[p]      = sum_q sum_b g[p][q][b] sum_j dZ_j/dr(p) F_{l_j}(phi_q) c[j][b]
 *   grad_theta[p]  likewise with dZ_j/dtheta
 *   grad_phi[q]    = sum_p sum_b g[p][q][b] sum_j Z_j(p) dF_{l_j}/dphi(phi_q) c[j][b]
 * Each output is nullable (not computed when NULL) and overwritten.  Sums
 * have a fixed order: repeated calls are bitwise equal.
 */
zp_status zp_series3d_bwd(const int32_t *h_n, const int32_t *h_m, const int32_t *h_l, int64_t J, const double *d_r,
                          const double *d_theta, int64_t P, const double *d_phi, int64_t Q, const double *d_c,
                          int64_t B, int32_t prec, const double *d_g, const void *d_cache, double *d_grad_c,
                          double *d_grad_r, double *d_grad_theta, double *d_grad_phi, void *d_ws, size_t ws_bytes,
                          void *stream);

/*
 * Analysis transform: Zernike coefficients from samples of a function on the
 * unit disc by quadrature (the inverse of zp_series_fwd for band-limited
 * data; the spectral-method use of the basis, Sec. 1).  The basis is
 * orthogonal over the disc: the integral of Z_k Z_k' dA is delta_kk' N_k with
 * N_k = eps_m pi / (2 (n_k + 1)), eps_m = 2 for m = 0 and 1 otherwise.
 *
 * zp_analysis_grid -- a host-side quadrature rule on nr x nt points
 * (p = i * nt + j, theta fastest): Gauss-Legendre in t = r^2 with nr nodes
 * times the trapezoidal rule at theta_j = 2 pi j / nt.  For modes with n <= L
 * and data that is a series in those modes, nr >= ceil((L + 1) / 2) and
 * nt >= 2 L + 1 make the transform exact.
 *   h_r, h_theta, h_w  host double[nr * nt] (outputs); weights sum to pi.
 * The rule costs O(nr^2) host operations (Newton's method on each node);
 * nr <= 4096 covers every degree the library accepts (n <= 1000 needs 501).
 * Errors: ZP_ERR_ARG (nr or nt < 1, nr > 4096, nt > 2^24, null pointer).
 */
zp_status zp_analysis_grid(int64_t nr, int64_t nt, double *h_r, double *h_theta, double *h_w);

/* Workspace of zp_series_analysis: one pass / minimum (chunked), bytes. */
zp_status zp_series_analysis_workspace(int64_t M, int64_t P, int64_t B, int32_t prec, size_t *full_bytes,
                                       size_t *min_bytes);

/*
 * zp_series_analysis -- c[k][b] = (1 / N_k) sum_p w_p Z_k(r_p, theta_p) f[p][b].
 *   d_r, d_theta, d_w  device double[P]: quadrature points and weights (any
 *                      rule; zp_analysis_grid gives an exact one)
 *   d_f       device double[P*B], samples, row-major [P][B]
 *   d_c       device double[M*B] (output), row-major [M][B]
 * The contraction over points runs in prec, as zp_series_bwd's grad_c.
 * P == 0 gives all-zero coefficients; M == 0 or B == 0 is a no-op.
 * Errors: as zp_series_bwd.
 */
zp_status zp_series_analysis(const int32_t *h_n, const int32_t *h_m, int64_t M, const double *d_r,
                             const double *d_theta, const double *d_w, int64_t P, const double *d_f, int64_t B,
                             int32_t prec, double *d_c, void *d_ws, size_t ws_bytes, void *stream);

/*
 * zp_series_fwd_noalloc -- zp_series_fwd (no basis cache) for callers that
 * cannot allocate device memory: code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc.  It calls no hipMalloc / hipFree
 * and creates no stream or event; its workspace and its plan tables live in a
 * fixed device array of ZP_NOALLOC_SCRATCH_BYTES per GPU, which the library
 * holds until the process ends.  Work runs on `stream` alone, in chunks of
 * points that fit the array.
 *   Arguments and output as zp_series_fwd.
 *   A call whose mode list differs from the previous call's on this GPU
 *   copies the new tables into the array and waits for `stream` once.
 *   Every call on a GPU shares that GPU's array: calls that overlap on one
 *   GPU (on other streams, or from host threads without ordering) race.
 * Errors: as zp_series_fwd; ZP_ERR_WORKSPACE when the tables plus the
 * smallest workspace (one 128-point chunk) exceed ZP_NOALLOC_SCRATCH_BYTES.
 */
#define ZP_NOALLOC_SCRATCH_BYTES (64u << 20)
zp_status zp_series_fwd_noalloc(const int32_t *h_n, const int32_t *h_m, int64_t M, const double *d_r,
                                const double *d_theta, int64_t P, const double *d_c, int64_t B, int32_t prec,
                                double *d_f, void *stream);

/*
 * zp_stream_fill -- d_out[i] = value for i < n: the device's streaming-write
 * rate, measured by a trivial kernel (one 16-byte store per lane), the
 * reference the basis kernel's store rate is compared with besides the
 * published HBM peak (the roofline measurement of the basis, Sec. 4 timings).
 *   d_out  device double[n], 16-byte aligned
 *   nontemporal  nonzero: non-temporal stores; zero: plain stores
 * Errors: ZP_ERR_ARG (n < 0, null or misaligned d_out), ZP_ERR_HIP.
 */
zp_status zp_stream_fill(double *d_out, int64_t n, double value, int32_t nontemporal, void *stream);

/* Static description of a status code. */
const char *zp_status_string(zp_status s);
/* Detail of the last error raised on the calling host thread ("" if none). */
const char *zp_last_error(void);
/* Release every cached plan (waits for the device first). */
void zp_cache_clear(void);
/* ABI version of this header: 1. */
int32_t zp_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* ZP_H */
