/*
 * zpo.c -- quad-precision CPU oracle for radial Zernike polynomials, their
 * r-derivatives, and the full Zernike basis.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header, table or constant
 * generator with the GPU path.
 *
 * What it computes (ZERNIPAX paper, Sec. 2 and Sec. 3):
 *   R_n^{|m|}(r) = (-1)^K r^alpha P_K^{(alpha,0)}(1 - 2 r^2),
 *        alpha = |m|, K = (n - alpha)/2                       (Eq. jacobi-relation)
 *   P_0, P_1 from the explicit Jacobi sum                     (Eq. jacobi)
 *   P_k, k >= 2, from the general three-term recurrence        (Eq. jacobi-recursion)
 *   d^j/dx^j P_K^{(a,b)} = (a+b+K+1)_j / 2^j P_{K-j}^{(a+j,b+j)} (derivative identity
 *        with Pochhammer symbol, Sec. 2)
 *   Z_n^m(r,theta) = R cos(m theta) (m >= 0), R sin(|m| theta) (m < 0)
 *                                                              (Eq. zernike-poly)
 * Structure follows Algorithm 1 ("CPU"): an outer loop over alpha, one
 * recurrence chain per alpha shared by every requested n with that alpha, and
 * the requested (n, m) pairs picked out of the chain.  The derivative chains
 * use beta = j != 0, so the general recurrence (not its beta = 0 expansion) is
 * used for all of them.
 *
 * The paper writes derivatives with respect to the Jacobi variable x; the
 * r-derivatives it plots need the chain rule through x = 1 - 2 r^2, which the
 * paper does not spell out.  Reading used here: x' = -4r, x'' = -4, x''' = 0,
 *   g(r) = P(x(r)):  g'   = -4 r D1
 *                    g''  = 16 r^2 D2 - 4 D1
 *                    g''' = -64 r^3 D3 + 48 r D2
 * and then Leibniz on r^alpha * g(r).
 *
 * Arithmetic is IEEE binary128 (__float128, 113-bit significand).  A double
 * r squared is exact in binary128, so x = 1 - 2r^2 carries at most one
 * rounding.  Each result is returned as an unevaluated sum hi + lo of two
 * doubles (hi = nearest double, lo = nearest double to the remainder), which
 * keeps ~106 bits for the pins that need more than double.
 */
#include <math.h>
#include <quadmath.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef __float128 quad;

/* ---------------------------------------------------------------- Jacobi -- */

/* Explicit sum, Eq. (jacobi):
 *   P_n^{(a,b)}(x) = sum_{s=0}^{n} C(n+a, n-s) C(n+b, s) ((x-1)/2)^s ((x+1)/2)^(n-s)
 * The recurrence below is only seeded from it (n = 0 and n = 1).  Integer a, b
 * >= 0 only, as every chain here has. */
static quad binom_q(int top, int k)
{
    if (k < 0 || k > top) return 0;
    quad v = 1;
    for (int i = 1; i <= k; ++i) v = v * (quad)(top - k + i) / (quad)i;
    return v;
}

static quad jacobi_explicit(int n, int a, int b, quad x)
{
    quad xm = (x - 1) / 2, xp = (x + 1) / 2, sum = 0;
    for (int s = 0; s <= n; ++s) {
        quad t = binom_q(n + a, n - s) * binom_q(n + b, s);
        for (int i = 0; i < s; ++i) t *= xm;
        for (int i = 0; i < n - s; ++i) t *= xp;
        sum += t;
    }
    return sum;
}

/* P_k^{(a,b)}(x) for k = 0..kmax into out[0..kmax].  P_0, P_1 from Eq. (jacobi);
 * k >= 2 from Eq. (jacobi-recursion) with c = 2k+a+b, A = k+a, B = k+b:
 *   2k(c-k)(c-2) P_k = (c-1)[c(c-2)x + (A-B)(c-2k)] P_{k-1} - 2(A-1)(B-1)c P_{k-2}
 * (A, B are the paper's a, b; renamed so they do not clash with alpha, beta.) */
static void jacobi_chain(int kmax, int a, int b, quad x, quad *out)
{
    if (kmax < 0) return;
    out[0] = jacobi_explicit(0, a, b, x);
    if (kmax < 1) return;
    out[1] = jacobi_explicit(1, a, b, x);
    for (int k = 2; k <= kmax; ++k) {
        quad c = 2 * k + a + b, A = k + a, B = k + b;
        quad lhs = 2 * (quad)k * (c - k) * (c - 2);
        quad t1 = (c - 1) * (c * (c - 2) * x + (A - B) * (c - 2 * k));
        quad t2 = 2 * (A - 1) * (B - 1) * c;
        out[k] = (t1 * out[k - 1] - t2 * out[k - 2]) / lhs;
    }
}

/* Pochhammer (rising factorial), Sec. 2: (z)_j = z (z+1) ... (z+j-1). */
static quad pochhammer(int z, int j)
{
    quad v = 1;
    for (int i = 0; i < j; ++i) v *= (quad)(z + i);
    return v;
}

/* alpha! / (alpha - i)!, zero when i > alpha (the i-th derivative of r^alpha
 * is that times r^(alpha-i)). */
static quad falling(int alpha, int i)
{
    if (i > alpha) return 0;
    quad v = 1;
    for (int t = 0; t < i; ++t) v *= (quad)(alpha - t);
    return v;
}

static quad ipow(quad r, int e)
{
    quad v = 1;
    for (int i = 0; i < e; ++i) v *= r;
    return v;
}

static void split(quad v, double *hi, double *lo)
{
    double h = (double)v;
    *hi = h;
    if (lo) *lo = isfinite(h) ? (double)(v - (quad)h) : 0.0;
}

/* d^j/dr^j R for j = 0..J at one point, given the x-derivatives
 * D[j] = d^j/dx^j P_K^{(alpha,0)}(x), r, and w[i] = d^i/dr^i r^alpha.  Chain
 * rule through x = 1 - 2r^2, then Leibniz on r^alpha g(r), then the (-1)^K of
 * Eq. (jacobi-relation). */
static void assemble_radial(int K, int J, quad r, const quad *D, const quad *w, quad *R)
{
    quad g[4];
    g[0] = D[0];
    g[1] = J >= 1 ? -4 * r * D[1] : 0;
    g[2] = J >= 2 ? 16 * r * r * D[2] - 4 * D[1] : 0;
    g[3] = J >= 3 ? -64 * r * r * r * D[3] + 48 * r * D[2] : 0;
    quad sgn = (K % 2) ? -1 : 1;
    for (int j = 0; j <= J; ++j) {
        quad acc = 0;
        for (int i = 0; i <= j; ++i) acc += binom_q(j, i) * w[i] * g[j - i];
        R[j] = sgn * acc;
    }
}

/* Radial values and r-derivatives of every requested mode at one point
 * (Algorithm 1 for one r): for each alpha with requested modes, the chains
 * P^{(alpha+j, j)}_k, k = 0..Kmax(alpha)-j, then each requested (n, m) of that
 * alpha (pair membership, not n and m separately) is assembled and stored.
 * cb(mode, j, value, ctx) receives every result. */
typedef void (*emit_fn)(int64_t mode, int j, quad value, void *ctx);

static void radial_point(const int32_t *n, const int32_t *m, int64_t M, int amax,
                         const int *kmax_of, int J, quad r, quad *chains, int chain_stride,
                         emit_fn cb, void *ctx)
{
    quad x = 1 - 2 * r * r; /* r_jacobi of Algorithm 1 */
    for (int alpha = 0; alpha <= amax; ++alpha) {
        int Kmax = kmax_of[alpha];
        if (Kmax < 0) continue; /* no requested mode has this |m| */
        for (int j = 0; j <= J; ++j)
            jacobi_chain(Kmax - j, alpha + j, j, x, chains + (size_t)j * chain_stride);
        quad w[4]; /* d^i/dr^i r^alpha = alpha!/(alpha-i)! r^(alpha-i), zero for i > alpha */
        for (int i = 0; i <= J; ++i) w[i] = i > alpha ? 0 : falling(alpha, i) * ipow(r, alpha - i);
        for (int64_t i = 0; i < M; ++i) {
            int a = m[i] < 0 ? -m[i] : m[i];
            if (a != alpha) continue;
            int K = (n[i] - a) / 2;
            quad D[4] = {0, 0, 0, 0};
            for (int j = 0; j <= J; ++j)
                if (K - j >= 0)
                    D[j] = pochhammer(alpha + K + 1, j) / ipow(2, j) *
                           chains[(size_t)j * chain_stride + (K - j)];
            quad R[4];
            assemble_radial(K, J, r, D, w, R);
            for (int j = 0; j <= J; ++j) cb(i, j, R[j], ctx);
        }
    }
}

/* ------------------------------------------------------------ public API -- */

/* Return codes: 0 ok; 1 invalid mode (n < 0, |m| > n, n - |m| odd); 2 bad
 * argument (J outside 0..3, negative size, null output with work to do);
 * 3 out of memory. */
static int check_modes(const int32_t *n, const int32_t *m, int64_t M, int *amax, int *nmax)
{
    *amax = -1;
    *nmax = -1;
    for (int64_t i = 0; i < M; ++i) {
        int a = m[i] < 0 ? -m[i] : m[i];
        if (n[i] < 0 || a > n[i] || ((n[i] - a) & 1)) return 1;
        if (a > *amax) *amax = a;
        if (n[i] > *nmax) *nmax = n[i];
    }
    return 0;
}

static int *kmax_table(const int32_t *n, const int32_t *m, int64_t M, int amax)
{
    int *t = (int *)malloc(sizeof(int) * (size_t)(amax + 1));
    if (!t) return NULL;
    for (int a = 0; a <= amax; ++a) t[a] = -1;
    for (int64_t i = 0; i < M; ++i) {
        int a = m[i] < 0 ? -m[i] : m[i];
        int K = (n[i] - a) / 2;
        if (K > t[a]) t[a] = K;
    }
    return t;
}

typedef struct {
    double *hi, *lo;
    int64_t M, P, p;
} radial_ctx;

static void radial_emit(int64_t mode, int j, quad v, void *vctx)
{
    radial_ctx *c = (radial_ctx *)vctx;
    size_t idx = ((size_t)j * (size_t)c->M + (size_t)mode) * (size_t)c->P + (size_t)c->p;
    split(v, &c->hi[idx], c->lo ? &c->lo[idx] : NULL);
}

/* Radial part and its r-derivatives.
 *   n, m  : M mode numbers (|m| is used; the sign of m does not matter here)
 *   r     : P points
 *   J     : highest r-derivative order, 0..3
 *   hi,lo : [J+1][M][P] outputs; lo may be NULL
 *   nthreads <= 0 means the OpenMP default. */
int zpo_radial(const int32_t *n, const int32_t *m, int64_t M, const double *r, int64_t P,
               int J, double *hi, double *lo, int nthreads)
{
    if (J < 0 || J > 3 || M < 0 || P < 0) return 2;
    int amax, nmax;
    if (check_modes(n, m, M, &amax, &nmax)) return 1;
    if (M == 0 || P == 0) return 0;
    if (!hi || !r) return 2;
    int *kt = kmax_table(n, m, M, amax);
    if (!kt) return 3;
    int stride = nmax / 2 + 2;
    int err = 0;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
#pragma omp parallel
    {
        quad *chains = (quad *)malloc(sizeof(quad) * (size_t)stride * 4);
        if (!chains) {
#pragma omp atomic write
            err = 3;
        } else {
#pragma omp for schedule(dynamic, 16)
            for (int64_t p = 0; p < P; ++p) {
                radial_ctx c = {hi, lo, M, P, p};
                radial_point(n, m, M, amax, kt, J, (quad)r[p], chains, stride, radial_emit, &c);
            }
            free(chains);
        }
    }
    free(kt);
    return err;
}

typedef struct {
    double *hi, *lo;
    int64_t M, P, p;
    const int32_t *m;
    int plane[5]; /* output plane for Z, Z_r, Z_rr, Z_rrr, Z_theta or -1 */
    quad theta;
    int ang_alpha; /* |m| the cached angular factors belong to, or -1 */
    quad cs, sn;   /* cos(|m| theta), sin(|m| theta) */
} basis_ctx;

static void basis_store(basis_ctx *c, int plane, int64_t mode, quad v)
{
    size_t idx = ((size_t)plane * (size_t)c->M + (size_t)mode) * (size_t)c->P + (size_t)c->p;
    split(v, &c->hi[idx], c->lo ? &c->lo[idx] : NULL);
}

/* Eq. (zernike-poly): Z = R cos(m theta) for m >= 0 and R sin(|m| theta) for
 * m < 0; d/dr^j Z carries the same angular factor; dZ/dtheta differentiates the
 * angular factor: -m R sin(m theta) for m >= 0, |m| R cos(|m| theta) for m < 0. */
static void basis_emit(int64_t mode, int j, quad R, void *vctx)
{
    basis_ctx *c = (basis_ctx *)vctx;
    int mm = c->m[mode];
    int a = mm < 0 ? -mm : mm;
    if (a != c->ang_alpha) {
        quad ang = (quad)a * c->theta; /* exact: integer times double fits 113 bits */
        c->cs = cosq(ang);
        c->sn = sinq(ang);
        c->ang_alpha = a;
    }
    quad cs = c->cs, sn = c->sn;
    quad f = mm < 0 ? sn : cs;
    if (c->plane[j] >= 0) basis_store(c, c->plane[j], mode, R * f);
    if (j == 0 && c->plane[4] >= 0) {
        quad dth = mm < 0 ? (quad)a * R * cs : -(quad)a * R * sn;
        basis_store(c, c->plane[4], mode, dth);
    }
}

/* Full basis.  mask bit 0: Z, 1: dZ/dr, 2: d2Z/dr2, 3: d3Z/dr3, 4: dZ/dtheta.
 * Outputs [popcount(mask)][M][P] in increasing bit order. */
int zpo_basis(const int32_t *n, const int32_t *m, int64_t M, const double *r,
              const double *theta, int64_t P, uint32_t mask, double *hi, double *lo, int nthreads)
{
    if (M < 0 || P < 0 || mask == 0 || (mask & ~31u)) return 2;
    int amax, nmax;
    if (check_modes(n, m, M, &amax, &nmax)) return 1;
    if (M == 0 || P == 0) return 0;
    if (!hi || !r || !theta) return 2;
    int plane[5], np = 0, J = 0;
    for (int b = 0; b < 5; ++b) {
        plane[b] = (mask >> b) & 1 ? np++ : -1;
        if (b >= 1 && b <= 3 && plane[b] >= 0) J = b;
    }
    int *kt = kmax_table(n, m, M, amax);
    if (!kt) return 3;
    int stride = nmax / 2 + 2;
    int err = 0;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
#pragma omp parallel
    {
        quad *chains = (quad *)malloc(sizeof(quad) * (size_t)stride * 4);
        if (!chains) {
#pragma omp atomic write
            err = 3;
        } else {
#pragma omp for schedule(dynamic, 16)
            for (int64_t p = 0; p < P; ++p) {
                basis_ctx c;
                c.hi = hi;
                c.lo = lo;
                c.M = M;
                c.P = P;
                c.p = p;
                c.m = m;
                memcpy(c.plane, plane, sizeof plane);
                c.theta = (quad)theta[p];
                c.ang_alpha = -1;
                radial_point(n, m, M, amax, kt, J, (quad)r[p], chains, stride, basis_emit, &c);
            }
            free(chains);
        }
    }
    free(kt);
    return err;
}

/* The Jacobi chain itself, for checking against an independent library
 * evaluation: P_k^{(a,b)}(x) for k = 0..kmax, x given as hi + lo. */
int zpo_jacobi_chain(int kmax, int a, int b, double x_hi, double x_lo, double *hi, double *lo)
{
    if (kmax < 0 || a < 0 || b < 0 || !hi) return 2;
    quad *buf = (quad *)malloc(sizeof(quad) * (size_t)(kmax + 1));
    if (!buf) return 3;
    jacobi_chain(kmax, a, b, (quad)x_hi + (quad)x_lo, buf);
    for (int k = 0; k <= kmax; ++k) split(buf[k], &hi[k], lo ? &lo[k] : NULL);
    free(buf);
    return 0;
}

/* Explicit Jacobi sum, Eq. (jacobi), exposed for the same purpose. */
int zpo_jacobi_explicit(int k, int a, int b, double x, double *hi, double *lo)
{
    if (k < 0 || a < 0 || b < 0 || !hi) return 2;
    split(jacobi_explicit(k, a, b, (quad)x), hi, lo);
    return 0;
}

int zpo_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
