// Internal declarations for the Zernike series (contraction of the basis with
// coefficient sets) and its adjoint.
#pragma once

#include "zp_internal.hpp"

namespace zp {

// Contraction element types.  BF3 is a value split into three bf16 planes
// (hi, mid, lo) stored `sub` elements apart.
enum CType : int { CT_F64 = 0, CT_F32 = 1, CT_BF3 = 2 };

inline size_t ct_bytes(int ct) { return ct == CT_F64 ? 8 : ct == CT_F32 ? 4 : 6; }

// All GEMM operands live in zero-padded buffers whose dimensions are
// multiples of kPad, so tile loads never need bounds checks.
constexpr int64_t kPad = 128;
inline int64_t pad_up(int64_t x) { return (x + kPad - 1) / kPad * kPad; }

// Memory layout of a GEMM operand, element (x, k) where x is the operand's
// output index (i for A, j for B):
//   LAY_KC  : base[x*ld + k]                      (contiguous along k)
//   LAY_XC  : base[k*ld + x]                      (contiguous along x)
//   LAY_KB8 : base[((k/8)*ld + x)*8 + k%8]        (k in blocks of eight)
//   LAY_KC32: as LAY_KC, but FP32 values of a BF3 operand; the GEMM splits
//             them into the three bf16 planes on the way into LDS
enum Layout : int { LAY_KC = 0, LAY_XC = 1, LAY_KB8 = 2, LAY_KC32 = 3, LAY_FRAG = 4 };

// Operand of C(i,j) = sum_k A(i,k) B(k,j); `sub` separates the BF3 planes.
struct Operand {
    const void *base;
    int64_t ld;
    int64_t sub;
    int lay;
};

enum Epi : int {
    EPI_STORE = 0,   // C[i*ldc + j] = acc (FP64)
    EPI_PARTIAL = 1, // split-K: C + split*M*ldc, reduced later
    EPI_COLDOT = 2   // part[itile][0|1][j] = sum_i acc(i,j) D1|D2[i*ldd + j]
};

struct GemmDesc {
    int ct;
    Operand a, b;
    int64_t M, N, K; // output M x N (unpadded); K a multiple of kPad
    int splits;      // split-K count (EPI_PARTIAL)
    int epi;
    double *C;
    int64_t ldc;
    const void *D1, *D2; // EPI_COLDOT: derivative planes, FP64 or FP32
    int64_t ldd;
    bool d_f32;
    double *part; // EPI_COLDOT output partials [ceil(M/BM)][2][N]
    // Order of the output tiles over the launch: 0 = along a row of tiles
    // first (workgroups in flight share an A panel), 1 = down a column of
    // tiles first (they share a B panel).
    int order;
};

// Row-tile height of the column-dot epilogue for a compute type (its
// partials buffer has ceil(M / coldot_bm(ct)) tiles).
int coldot_bm(int ct);

zp_status launch_gemm(const GemmDesc &g, hipStream_t s);

// Compute units of the current device (cached per device; 0 if unknown).
int device_cus();

// Series forward pieces shared by zp_series_fwd and its allocation-free
// variant: argument checks (ZP_OK also for the M, P or B == 0 no-op), the
// smallest workspace without a cache, and the work itself for a plan whose
// device tables are in place.  allow_pipe lets the forward overlap chunks on
// the library's helper stream (which it creates on first use).
zp_status series_fwd_checks(const int32_t *h_n, const int32_t *h_m, int64_t M, const double *d_r,
                            const double *d_theta, int64_t P, const double *d_c, int64_t B, int32_t prec,
                            const double *d_f);
size_t series_fwd_min_ws(int64_t M, int64_t P, int64_t B, int32_t prec);
zp_status series_fwd_run(const Plan &plan, int64_t M, const double *d_r, const double *d_theta, int64_t P,
                         const double *d_c, int64_t B, int32_t prec, double *d_f, void *d_cache, void *d_ws,
                         size_t ws_bytes, bool allow_pipe, hipStream_t s);

// dst (compute type, [R_pad][C_pad] or transposed [C_pad][R_pad]) from a
// row-major FP64 src [R][C] (leading dimension lds); zero padding.
zp_status launch_convert(const double *src, int64_t R, int64_t C, int64_t lds, int ct, void *dst, int64_t ldd,
                         int64_t rows_pad, int64_t sub, bool transpose, hipStream_t s);

// bf16 x 3 operand in MFMA fragment order for B(k = e, j = x) = src[perm[e]][x]:
// per k step of 32 and block of 16 columns, 64 lanes x 8 bf16 contiguous (lane
// = 16 (k % 32 / 8) + x % 16), blocks along x fastest (xblocks = xpad / 16);
// three planes sub apart; zero outside R x C.
zp_status launch_convert_gather_frag(const double *src, const int32_t *perm, int64_t R, int64_t C, int64_t lds,
                                     void *dst, int64_t xpad, int64_t kpad, int64_t sub, hipStream_t s);

// The upstream gradient g [R][C] (rows = points) as the backward's bf16 x 3
// operands from one read: [xpad_r][xpad_c] k-contiguous into dst_c (the
// column-dot's B(k = set, j = point)) and, if dst_s is set, MFMA fragment
// order into dst_s (the split-K's B(k = point, j = set)); xpad_r, xpad_c are
// the padded point and set counts (multiples of 32 and 64).
zp_status launch_convert_g_bwd(const double *src, int64_t R, int64_t C, int64_t lds, void *dst_c, int64_t subc,
                               void *dst_s, int64_t subs, int64_t xpad_r, int64_t xpad_c, hipStream_t s);
// Zero the pad (modes >= M, points >= P) of a k-blocked bf16 operand.
zp_status launch_zero_kb8(void *dst, int64_t M, int64_t Mp, int64_t P, int64_t ld, int64_t sub, hipStream_t s);

// Zero the pad region of a [rows_pad][ld] compute-type plane set whose
// valid block is [rows][cols].
zp_status launch_zero_pad(void *dst, int ct, int64_t rows, int64_t cols, int64_t rows_pad, int64_t ld, int64_t sub,
                          hipStream_t s);

// C[i*ldc + j] (=|+=) sum_s part[s][i][j] for s = 0..S-1, fixed order.
zp_status launch_splitk_reduce(const double *part, int S, int64_t M, int64_t N, double *C, int64_t ldc,
                               bool accumulate, hipStream_t s);

// out1[p] = sum_t part[t][0][p], out2[p] = sum_t part[t][1][p] (either nullable).
zp_status launch_coldot_reduce(const double *part, int T, int64_t P, double *out1, double *out2, hipStream_t s);

} // namespace zp
