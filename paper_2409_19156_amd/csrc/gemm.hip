// MFMA contractions for the Zernike series on gfx950, plus the small
// conversion and fixed-order reduction kernels around them.
//
// C(i,j) = sum_k A(i,k) B(k,j) with a 512-thread workgroup (2 x 4 waves) per
// BM x BN output tile (128 x 128, or 128 x 64 with the narrow shape below).
// Operands come from zero-padded buffers (every dimension a multiple of
// kPad), so tile loads need no bounds checks; stores are masked to the true
// output size.  Each operand tile is copied into LDS in its global layout
// (k-contiguous rows, or rows along the other index), with a row swizzle or
// padding that keeps the MFMA fragment reads and the tile stores free of bank
// conflicts; the fragment reads follow the layout.  The bf16 path needs eight
// consecutive k per lane, so an operand that is not k-contiguous in memory is
// transposed while it is written to LDS.  Tiles are double
// buffered: the next tile's global loads are in flight during the current
// tile's MFMAs.
//
// Element types:
//   F64 : v_mfma_f64_16x16x4 (FP64 in, FP64 accumulate)
//   F32 : v_mfma_f32_16x16x4 (FP32 in, FP32 accumulate)
//   BF3 : value = hi + mid + lo (three bf16 planes); six v_mfma_f32_16x16x32_bf16
//         cross products (hi.hi, hi.mid, mid.hi, hi.lo, mid.mid, lo.hi; the
//         three dropped products are below 2^-24 relative)
// The FP32-accumulating types add their FP32 accumulators into FP64 ones
// every kFlush k (below) and restart them, so FP32 rounding acts on partial
// sums of at most kFlush terms.  The bf16 MFMA's accumulation is biased
// toward -infinity (measured on gfx950: about -1.2e-9 per unit-size product,
// the same for positive and negative data, where the FP32 MFMA shows none),
// which adds up over long sums; the bf16 x 3 contraction therefore negates B
// on every other k step and subtracts that step's sums, so that the bias
// alternates in sign and cancels.
//
// MFMA lane layouts (16x16 blocks): lane l supplies A[l%16][k] and B[k][l%16]
// for k = l/16 (x4 shapes) or k = 8(l/16)..8(l/16)+7 (bf16 x32 shape).  It
// receives D[4(l/16)+t][l%16], t = 0..3, for the FP32-accumulating shapes and
// D[l/16+4t][l%16] for the FP64 shape.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "series.hpp"

namespace zp {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef uint32_t u4 __attribute__((ext_vector_type(4)));

constexpr int kThreads = 512; // eight waves per workgroup
// Flush interval (k terms) of the FP32 accumulators: every 16 k for the FP32
// column-dot and every 32 k for the other FP32 contractions (four or eight x4
// products), every k step of 32 for bf16 x 3 (one bf16 product of depth 32
// per cross term).  Sums that cancel after the contraction amplify its
// rounding errors: the column-dot epilogue sums the product weighted by basis
// derivatives over the modes, and the three-dimensional series folds partial
// sums over the planes into Fourier modes.  Measured against the oracle on
// the n <= 40 and n <= 64 series and the three-dimensional L = 32 workload,
// flushing every 128 k left errors of up to 1.2e-6 (FP32) and 1.0e-6 (bf16 x
// 3) relative to the largest output entry.
template <int CT, int EPI>
constexpr int kFlush = CT == CT_F32 ? (EPI == EPI_COLDOT ? 16 : 32) : 32;

template <int CT> struct CTr;
template <> struct CTr<CT_F64> {
    using T = double;
    static constexpr int NP = 1;
};
template <> struct CTr<CT_F32> {
    using T = float;
    static constexpr int NP = 1;
};
template <> struct CTr<CT_BF3> {
    using T = uint16_t;
    static constexpr int NP = 3;
};

__device__ __forceinline__ uint16_t bf16_rne(float f)
{
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ double bf16_val(uint16_t h) { return (double)__uint_as_float((uint32_t)h << 16); }

// x = hi + mid + lo as three bf16 values (the residuals are exact in FP32).
__device__ __forceinline__ void split3f(float x, uint32_t &h, uint32_t &m, uint32_t &l)
{
    h = bf16_rne(x);
    const float r1 = x - __uint_as_float(h << 16);
    m = bf16_rne(r1);
    const float r2 = r1 - __uint_as_float(m << 16);
    l = bf16_rne(r2);
}

// LDS geometry and global->LDS copy of one operand tile (X rows of the output
// index by BK).  LDS holds the tile either as [X][BK] rows (k contiguous: the
// k-contiguous and k-blocked layouts, and every bf16 operand) or as
// [BK][X+16] (x contiguous, the pad keeping the fragment reads conflict-free).
//
// Rows along x are stored unpadded with the k index XOR-swizzled by the row:
// element (x, k) sits at x*BK + (k ^ swz(x)).  swz(x) is a multiple of the
// 16-byte store width, so each global vector lands contiguously, and it
// spreads the rows over the 64 LDS banks:
//   FP64 : swz = x & 14         (8-byte elements, 128-byte rows)
//   FP32 : swz = (x & 14) * 2   (4-byte elements, 128-byte rows)
//   bf16 : swz = 8 * (((x>>1) & 3) ^ 3*((x>>3) & 1)) (16-byte k blocks,
//          64-byte rows)
// With it, the sixteen lanes that read rows x..x+15 of one k (x4 shapes: two
// k per 32-lane half) and the lanes of one store quarter all touch distinct
// banks.  The bf16 swizzle was chosen by measurement on gfx950 among the 256
// XOR swizzles linear in the low four row bits: it reads the 16-byte fragment
// pattern (lane l: row l % 16, block l / 16) at the rate of contiguous lanes
// and stores the k-blocked tile (lane l: row l) at full rate too, where
// (x>>2) & 3 read the fragments 15% slower.
template <int CT> __device__ __forceinline__ constexpr int row_swizzle(int x)
{
    return CT == CT_F64 ? (x & 14) : CT == CT_F32 ? ((x & 14) << 1) : ((((x >> 1) & 3) ^ (3 * ((x >> 3) & 1))) << 3);
}

template <int CT, int X, int BK, int LAY> struct Tile {
    using T = typename CTr<CT>::T;
    static constexpr bool ROWS_X = LAY != LAY_XC || CT == CT_BF3;
    static constexpr int STRIDE = ROWS_X ? BK : X + 16;
    static constexpr int ELEMS = (ROWS_X ? X : BK) * STRIDE;
    static_assert(!ROWS_X || BK == (CT == CT_F64 ? 16 : 32), "row swizzle assumes 128- or 64-byte rows");

    // LDS position of element (x, k) of a row-major (ROWS_X) tile
    static __device__ __forceinline__ int at(int x, int k) { return x * BK + (k ^ row_swizzle<CT>(x)); }
    static constexpr int VEC = 16 / (int)sizeof(T);
    // global tile as GROWS rows of GCOLS contiguous elements
    static constexpr bool KC = LAY == LAY_KC || LAY == LAY_KC32;
    static constexpr int GROWS = KC ? X : LAY == LAY_XC ? BK : BK / VEC;
    static constexpr int GCOLS = KC ? BK : LAY == LAY_XC ? X : X * VEC;
    static constexpr int NV = GROWS * GCOLS / VEC;
    static constexpr int PER = NV / kThreads;
    static_assert(NV % kThreads == 0, "tile not divisible among threads");
    static_assert(LAY != LAY_KB8 || VEC == 8, "k-blocked layout is for bf16 operands");
    static_assert(LAY != LAY_KC32 || CT == CT_BF3, "FP32-source layout is for bf16 operands");

    using Regs = u4[PER][CTr<CT>::NP];

    static __device__ __forceinline__ void coords(int v, int &gr, int &gc)
    {
        const int idx = v * kThreads + (int)threadIdx.x;
        gr = idx / (GCOLS / VEC);
        gc = (idx % (GCOLS / VEC)) * VEC;
    }

    // Global -> registers for the tile at output-index origin x0, k origin k0.
    static __device__ __forceinline__ void load(Regs &reg, const T *base, int64_t ld, int64_t sub, int64_t x0,
                                                int64_t k0)
    {
#pragma unroll
        for (int v = 0; v < PER; ++v) {
            int gr, gc;
            coords(v, gr, gc);
            int64_t off;
            if (LAY == LAY_KC32) { // eight FP32 k values of one row, split at the LDS store
                const float *fb = (const float *)base + (x0 + gr) * ld + (k0 + gc);
                reg[v][0] = *(const u4 *)fb;
                reg[v][1] = *(const u4 *)(fb + 4);
                continue;
            }
            if (LAY == LAY_KC)
                off = (x0 + gr) * ld + (k0 + gc);
            else if (LAY == LAY_XC)
                off = (k0 + gr) * ld + (x0 + gc);
            else // gr = k block within the tile, gc / 8 = x within the tile
                off = ((k0 / 8 + gr) * ld + x0) * 8 + gc;
#pragma unroll
            for (int p = 0; p < CTr<CT>::NP; ++p) reg[v][p] = *(const u4 *)(base + off + p * sub);
        }
    }

    // Registers -> LDS buffer lds[NP][ELEMS].
    static __device__ __forceinline__ void store(const Regs &reg, T *lds)
    {
#pragma unroll
        for (int v = 0; v < PER; ++v) {
            int gr, gc;
            coords(v, gr, gc);
            if constexpr (LAY == LAY_KC32) {
                // 8 floats -> hi, mid, lo planes of 8 bf16 each
                u4 hp, mp, lp;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    uint32_t h0, m0, l0, h1, m1, l1;
                    const uint32_t w0 = reg[v][q >> 1][(q & 1) * 2], w1 = reg[v][q >> 1][(q & 1) * 2 + 1];
                    split3f(__uint_as_float(w0), h0, m0, l0);
                    split3f(__uint_as_float(w1), h1, m1, l1);
                    hp[q] = h0 | (h1 << 16);
                    mp[q] = m0 | (m1 << 16);
                    lp[q] = l0 | (l1 << 16);
                }
                *(u4 *)(lds + at(gr, gc)) = hp;
                *(u4 *)(lds + ELEMS + at(gr, gc)) = mp;
                *(u4 *)(lds + 2 * ELEMS + at(gr, gc)) = lp;
                continue;
            }
#pragma unroll
            for (int p = 0; p < CTr<CT>::NP; ++p) {
                T *L = lds + p * ELEMS;
                if (!ROWS_X) {
                    *(u4 *)(L + gr * STRIDE + gc) = reg[v][p];
                } else if (LAY == LAY_KC) {
                    *(u4 *)(L + at(gr, gc)) = reg[v][p];
                } else if (LAY == LAY_KB8) {
                    *(u4 *)(L + at(gc / 8, gr * 8)) = reg[v][p];
                } else { // bf16 operand contiguous along x: transpose into [x][k]
                    const u4 w = reg[v][p];
#pragma unroll
                    for (int q = 0; q < VEC; ++q)
                        L[at(gc + q, gr)] = (T)((q & 1) ? (w[q >> 1] >> 16) : (w[q >> 1] & 0xFFFFu));
                }
            }
        }
    }
};

// Fragment read for the x4 shapes: element (x, k) of an LDS tile.
template <class TL>
__device__ __forceinline__ typename TL::T frag1(const typename TL::T *L, int x, int k)
{
    return TL::ROWS_X ? L[TL::at(x, k)] : L[k * TL::STRIDE + x];
}

// Tile configuration per element type: BM x BN workgroup tile of eight
// WM x WN wave tiles (two waves per SIMD), BK k per LDS stage.
template <int CT> struct Cfg;
template <> struct Cfg<CT_F64> {
    static constexpr int BM = 128, BN = 128, BK = 16, WM = 64, WN = 32;
};
template <> struct Cfg<CT_F32> {
    static constexpr int BM = 128, BN = 128, BK = 32, WM = 64, WN = 32;
};
template <> struct Cfg<CT_BF3> {
    static constexpr int BM = 128, BN = 128, BK = 32, WM = 64, WN = 32;
};

// Narrow shape: 64 x 16 wave tiles (a 128 x 64 workgroup tile), half the
// accumulators of 64 x 32.  The FP32 split-K and column-dot always take it, so
// that they fit the 128-register build (gemm_kernel_w4) and two workgroups
// share a CU; FP32 operands need few LDS bytes per product, so the narrower
// tiles cost little there (the FP32 forward, narrow, measured 6% slower).  The
// FP64 split-K and column-dot take it on small problems (below), where twice
// the workgroups fill the chip better.
template <int CT, int EPI> constexpr bool kNarrowDefault = CT == CT_F32 && EPI != EPI_STORE;

template <int CT, int EPI, bool NARROW_ = kNarrowDefault<CT, EPI>> struct CfgE : Cfg<CT> {
    static constexpr bool NARROW = NARROW_;
    static constexpr int BN = NARROW ? 64 : Cfg<CT>::BN;
    static constexpr int WN = NARROW ? 16 : Cfg<CT>::WN;
    static constexpr bool W4 = CT == CT_F64 || NARROW; // compiled for four waves per SIMD
};

template <int CT, int ALAY, int BLAY, int EPI, int NSET, bool NARROW>
__device__ __forceinline__ void gemm_body(const GemmDesc &g)
{
    using C = CfgE<CT, EPI, NARROW>;
    constexpr int BM = C::BM, BN = C::BN, BK = C::BK, WM = C::WM, WN = C::WN;
    using TR = CTr<CT>;
    using T = typename TR::T;
    // B in MFMA fragment order (bf16 only) is loaded from global memory into
    // registers a k step ahead and skips LDS.
    constexpr bool BFRAG = BLAY == LAY_FRAG;
    static_assert(!BFRAG || CT == CT_BF3, "fragment-order operands are bf16");
    using TA = Tile<CT, BM, BK, ALAY>;
    using TB = Tile<CT, BN, BK, BFRAG ? LAY_KC : BLAY>;
    constexpr int NP = TR::NP;
    constexpr int FM = WM / 16, FN = WN / 16;
    constexpr bool MIXED = CT != CT_F64;
    static_assert((BM / WM) * (BN / WN) * 64 == kThreads, "one wave tile per wave");
    static_assert(CT != CT_BF3 || kFlush<CT, EPI> == BK, "bf16 steps alternate the sign of B: flush every step");

    __shared__ __attribute__((aligned(16))) T As[2][NP * TA::ELEMS];
    __shared__ __attribute__((aligned(16))) T Bs[2][BFRAG ? 8 : NP * TB::ELEMS];

    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int wm0 = (wave % (BM / WM)) * WM;
    const int wn0 = (wave / (BM / WM)) * WN;

    // Tile this workgroup computes.  Workgroups are dispatched in linear order
    // and dealt round-robin to the 8 XCDs, each with its own L2.  Give every
    // XCD a contiguous range of logical tiles, and order logical tiles split
    // (slowest), then row tile, then column tile (fastest; or the two swapped
    // with g.order = 1): the workgroups that share an A (or B) panel then run
    // together on one XCD and read it from its L2.
    int bx, by, bz;
    {
        const int64_t nx = gridDim.x, ny = gridDim.y;
        const int64_t total = nx * ny * (int64_t)gridDim.z;
        const int64_t id = blockIdx.x + nx * (blockIdx.y + ny * (int64_t)blockIdx.z);
        const int64_t t8 = total / 8 * 8;
        const int64_t lid = id < t8 ? (id % 8) * (t8 / 8) + id / 8 : id;
        if (g.order == 0) {
            by = (int)(lid % ny);
            bx = (int)((lid / ny) % nx);
        } else {
            bx = (int)(lid % nx);
            by = (int)((lid / nx) % ny);
        }
        bz = (int)(lid / (ny * nx));
    }
    const int64_t i0 = (int64_t)bx * BM;
    const int64_t j0 = (int64_t)by * BN;

    // k range of this workgroup (split-K along the third grid dimension)
    const int64_t kchunk = g.K / g.splits;
    const int64_t kbeg = (int64_t)bz * kchunk;
    const int ntiles = (int)(kchunk / BK);

    using Acc = typename std::conditional<CT == CT_F64, d4, f4>::type;
    Acc acc[FM][FN];
    double acc64[MIXED ? FM : 1][MIXED ? FN : 1][4];
#pragma unroll
    for (int a = 0; a < FM; ++a)
#pragma unroll
        for (int b = 0; b < FN; ++b) {
            acc[a][b] = Acc{0, 0, 0, 0};
            if (MIXED)
#pragma unroll
                for (int t = 0; t < 4; ++t) acc64[MIXED ? a : 0][MIXED ? b : 0][t] = 0.0;
        }

    // sign = -1 moves the FP32 sums of a step whose B fragments were negated.
    auto flush = [&](double sign) {
        if (MIXED) {
#pragma unroll
            for (int a = 0; a < FM; ++a)
#pragma unroll
                for (int b = 0; b < FN; ++b) {
#pragma unroll
                    for (int t = 0; t < 4; ++t)
                        acc64[MIXED ? a : 0][MIXED ? b : 0][t] += sign * (double)acc[a][b][t];
                    acc[a][b] = Acc{0, 0, 0, 0};
                }
        }
    };

    const T *a_base = (const T *)g.a.base;
    const T *b_base = (const T *)g.b.base;
    const int64_t a_ld = g.a.ld, a_sub = g.a.sub, b_ld = g.b.ld, b_sub = g.b.sub;
    // Two register sets.  Step t: tile t+1 (fetched during step t-1) goes from
    // registers into the free LDS buffer, tile t+2 is fetched, and tile t is
    // multiplied out of the other buffer, so the LDS writes and the global
    // loads both overlap the MFMAs; one barrier per step.
    // NSET = 1 keeps one set (the store of tile t+1 precedes the load of tile
    // t+2 into the same registers): 8 to 16 fewer registers, for the builds
    // capped at 128.
    typename TA::Regs ra[NSET];
    typename TB::Regs rb[BFRAG ? 1 : NSET];
    // fragment-order B: this wave's FN x 3 fragments of k step t
    bf8 fbr[2][BFRAG ? FN : 1][3];
    auto load_bfrag = [&](int t, bf8(&dst)[BFRAG ? FN : 1][3]) {
        if constexpr (BFRAG) {
            const int64_t blk = (kbeg / BK + t) * b_ld + (j0 + wn0) / 16;
#pragma unroll
            for (int b = 0; b < FN; ++b)
#pragma unroll
                for (int p = 0; p < 3; ++p)
                    dst[b][p] = *(const bf8 *)((const uint16_t *)g.b.base + p * b_sub + ((blk + b) * 64 + lane) * 8);
        }
    };
    if (ntiles > 0) {
        TA::load(ra[0], a_base, a_ld, a_sub, i0, kbeg);
        TA::store(ra[0], As[0]);
        if constexpr (BFRAG) {
            load_bfrag(0, fbr[0]);
        } else {
            TB::load(rb[0], b_base, b_ld, b_sub, j0, kbeg);
            TB::store(rb[0], Bs[0]);
        }
    }
    if (ntiles > 1) {
        TA::load(ra[NSET - 1], a_base, a_ld, a_sub, i0, kbeg + BK);
        if constexpr (!BFRAG) TB::load(rb[NSET - 1], b_base, b_ld, b_sub, j0, kbeg + BK);
    }
    __syncthreads();

    const int lx = lane & 15, lk = lane >> 4;
    auto step = [&](int t, auto cur_c) {
        constexpr int cur = decltype(cur_c)::value;
        if (t + 1 < ntiles) {
            TA::store(ra[(cur ^ 1) % NSET], As[cur ^ 1]);
            if constexpr (BFRAG)
                load_bfrag(t + 1, fbr[cur ^ 1]);
            else
                TB::store(rb[(cur ^ 1) % NSET], Bs[cur ^ 1]);
        }
        if (t + 2 < ntiles) {
            TA::load(ra[cur % NSET], a_base, a_ld, a_sub, i0, kbeg + (int64_t)(t + 2) * BK);
            if constexpr (!BFRAG) TB::load(rb[cur % NSET], b_base, b_ld, b_sub, j0, kbeg + (int64_t)(t + 2) * BK);
        }
        const T *LA = As[cur];
        const T *LB = Bs[cur];
        if constexpr (CT == CT_BF3) {
#pragma unroll
            for (int kk = 0; kk < BK; kk += 32) {
                bf8 fa[FM][3];
#pragma unroll
                for (int a = 0; a < FM; ++a)
#pragma unroll
                    for (int p = 0; p < 3; ++p)
                        fa[a][p] = *(const bf8 *)(LA + p * TA::ELEMS + TA::at(wm0 + a * 16 + lx, kk + 8 * lk));
#pragma unroll
                for (int b = 0; b < FN; ++b) {
                    bf8 fb[3];
#pragma unroll
                    for (int p = 0; p < 3; ++p) {
                        if constexpr (BFRAG)
                            fb[p] = fbr[cur][b][p];
                        else
                            fb[p] = *(const bf8 *)(LB + p * TB::ELEMS + TB::at(wn0 + b * 16 + lx, kk + 8 * lk));
                    }
                    if constexpr (cur == 1) // odd steps: -B (see the flush)
#pragma unroll
                        for (int p = 0; p < 3; ++p)
                            fb[p] = __builtin_bit_cast(bf8, __builtin_bit_cast(u4, fb[p]) ^ 0x80008000u);
#pragma unroll
                    for (int a = 0; a < FM; ++a) {
                        // small cross products first, the leading one last
                        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[a][2], fb[0], acc[a][b], 0, 0, 0);
                        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[a][1], fb[1], acc[a][b], 0, 0, 0);
                        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[a][0], fb[2], acc[a][b], 0, 0, 0);
                        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[a][1], fb[0], acc[a][b], 0, 0, 0);
                        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[a][0], fb[1], acc[a][b], 0, 0, 0);
                        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[a][0], fb[0], acc[a][b], 0, 0, 0);
                    }
                }
            }
        } else {
#pragma unroll
            for (int kk = 0; kk < BK; kk += 4) {
                T fa[FM], fb[FN];
#pragma unroll
                for (int a = 0; a < FM; ++a) fa[a] = frag1<TA>(LA, wm0 + a * 16 + lx, kk + lk);
#pragma unroll
                for (int b = 0; b < FN; ++b) fb[b] = frag1<TB>(LB, wn0 + b * 16 + lx, kk + lk);
#pragma unroll
                for (int a = 0; a < FM; ++a)
#pragma unroll
                    for (int b = 0; b < FN; ++b) {
                        if constexpr (CT == CT_F64)
                            acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[a], fb[b], acc[a][b], 0, 0, 0);
                        else
                            acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[a], fb[b], acc[a][b], 0, 0, 0);
                    }
                if constexpr (MIXED && kFlush<CT, EPI> < BK)
                    if ((kk + 4) % kFlush<CT, EPI> == 0) flush(1.0);
            }
        }
        if constexpr (CT == CT_BF3)
            flush(cur == 1 ? -1.0 : 1.0); // every step (kFlush == BK)
        else if (MIXED && kFlush<CT, EPI> >= BK && ((t + 1) * BK) % kFlush<CT, EPI> == 0)
            flush(1.0);
        __syncthreads();
    };
    for (int t = 0; t < ntiles; t += 2) {
        step(t, std::integral_constant<int, 0>{});
        if (t + 1 < ntiles) step(t + 1, std::integral_constant<int, 1>{});
    }
    flush(1.0);

    // Output row (within the 16-row block) of accumulator element t.
    auto row_of = [&](int t) -> int { return CT == CT_F64 ? lk + 4 * t : 4 * lk + t; };

    auto value = [&](int a, int b, int t) -> double {
        if constexpr (MIXED)
            return acc64[a][b][t];
        else
            return acc[a][b][t];
    };

    if constexpr (EPI == EPI_STORE || EPI == EPI_PARTIAL) {
        double *Cp = g.C + (EPI == EPI_PARTIAL ? (int64_t)bz * g.M * g.ldc : 0);
#pragma unroll
        for (int a = 0; a < FM; ++a)
#pragma unroll
            for (int b = 0; b < FN; ++b) {
                const int64_t j = j0 + wn0 + b * 16 + lx;
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const int64_t i = i0 + wm0 + a * 16 + row_of(t);
                    if (i < g.M && j < g.N) Cp[i * g.ldc + j] = value(a, b, t);
                }
            }
    } else { // EPI_COLDOT
        // Column j of the tile is spread over the lanes lx + 16*lk (lk = 0..3),
        // each holding 16 of its rows (4 fragments x 4 accumulator elements).
        // Each lane forms its 16 products h * d -- sixteen lanes read 16
        // consecutive j of one plane row, 128 contiguous bytes -- then the four
        // lanes of a column are summed with two exchanges, and the wave rows
        // that share the column are added in a fixed order through LDS.
        constexpr int WROWS = BM / WM;
        __shared__ double red[2][WROWS][BN];
        const int wrow = wave % (BM / WM);
        using DT = typename std::conditional<CT == CT_F64, double, float>::type;
        const DT *D1 = (const DT *)g.D1;
        const DT *D2 = (const DT *)g.D2;
#pragma unroll
        for (int b = 0; b < FN; ++b) {
            const int64_t j = j0 + wn0 + b * 16 + lx;
            double s1 = 0.0, s2 = 0.0;
            if (j < g.N) {
#pragma unroll
                for (int a = 0; a < FM; ++a)
#pragma unroll
                    for (int t = 0; t < 4; ++t) {
                        const int64_t i = i0 + wm0 + a * 16 + row_of(t);
                        if (i < g.M) {
                            const int64_t o = i * g.ldd + j;
                            const double h = value(a, b, t);
                            s1 = __builtin_fma(h, (double)D1[o], s1);
                            s2 = __builtin_fma(h, (double)D2[o], s2);
                        }
                    }
            }
            s1 += __shfl_xor(s1, 16);
            s2 += __shfl_xor(s2, 16);
            s1 += __shfl_xor(s1, 32);
            s2 += __shfl_xor(s2, 32);
            if (lk == 0) {
                red[0][wrow][wn0 + b * 16 + lx] = s1;
                red[1][wrow][wn0 + b * 16 + lx] = s2;
            }
        }
        __syncthreads();
        for (int e = threadIdx.x; e < 2 * BN; e += kThreads) {
            const int o = e / BN, jl = e % BN;
            const int64_t j = j0 + jl;
            if (j >= g.N) continue;
            double sum = 0.0;
#pragma unroll
            for (int r = 0; r < WROWS; ++r) sum += red[o][r][jl];
            g.part[((int64_t)bx * 2 + o) * g.N + j] = sum;
        }
    }
}

template <int CT, int ALAY, int BLAY, int EPI>
__global__ __launch_bounds__(kThreads) void gemm_kernel(GemmDesc g)
{
    gemm_body<CT, ALAY, BLAY, EPI, 2, kNarrowDefault<CT, EPI>>(g);
}

// The same kernel compiled for four waves per SIMD (at most 128 registers,
// one prefetch register set), so that two 512-thread workgroups share a CU
// and one's epilogue and LDS phases overlap the other's products.  Used for
// every FP64 contraction, where it fits without spills (the column-dot keeps
// one 8-byte value in scratch across its main loop): forward 6%, split-K 4%
// and column-dot 18% faster than one workgroup per CU.  Also for the FP32
// split-K and column-dot with their narrow tiles (98 and 127 registers): 7%
// and 9% faster than 64 x 32 wave tiles at one workgroup per CU.  The FP32
// forward and the bf16 instances need 170-220 registers and keep one
// workgroup per CU.
template <int CT, int ALAY, int BLAY, int EPI, bool NARROW>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(4))) void gemm_kernel_w4(GemmDesc g)
{
    gemm_body<CT, ALAY, BLAY, EPI, 1, NARROW>(g);
}

template <int CT, int ALAY, int BLAY, int EPI, bool NARROW>
hipError_t launch_shape(const GemmDesc &g, hipStream_t s)
{
    using C = CfgE<CT, EPI, NARROW>;
    const dim3 grid((unsigned)((g.M + C::BM - 1) / C::BM), (unsigned)((g.N + C::BN - 1) / C::BN),
                    (unsigned)g.splits);
    if constexpr (C::W4)
        hipLaunchKernelGGL((gemm_kernel_w4<CT, ALAY, BLAY, EPI, NARROW>), grid, dim3(kThreads), 0, s, g);
    else
        hipLaunchKernelGGL((gemm_kernel<CT, ALAY, BLAY, EPI>), grid, dim3(kThreads), 0, s, g);
    return hipGetLastError();
}

// FP64 split-K and column-dot: the narrow shape when the wide tiles give fewer
// than four workgroups per CU (n <= 40 series, 861 modes x 16 384 points x 256
// sets: forward + backward 0.54 -> 0.50 ms); larger problems keep the wide
// tiles (n <= 64 on 65 536 points was 2% slower narrow).
template <int CT, int ALAY, int BLAY, int EPI>
hipError_t launch_t(const GemmDesc &g, hipStream_t s)
{
    if constexpr (CT == CT_F64 && EPI != EPI_STORE) {
        const int64_t wide = ((g.M + 127) / 128) * ((g.N + 127) / 128) * (int64_t)g.splits;
        if (wide < 4 * (int64_t)device_cus()) return launch_shape<CT, ALAY, BLAY, EPI, true>(g, s);
    }
    return launch_shape<CT, ALAY, BLAY, EPI, kNarrowDefault<CT, EPI>>(g, s);
}

// The operand-layout combinations the series uses (anything else is an
// internal error).
template <int CT, int EPI>
hipError_t launch_e(const GemmDesc &g, hipStream_t s)
{
    const int a = g.a.lay, b = g.b.lay;
    if constexpr (EPI == EPI_STORE) {
        if constexpr (CT == CT_BF3) {
            if (a == LAY_KB8 && b == LAY_FRAG) return launch_t<CT, LAY_KB8, LAY_FRAG, EPI>(g, s);
        } else {
            if (a == LAY_XC && b == LAY_XC) return launch_t<CT, LAY_XC, LAY_XC, EPI>(g, s);
        }
    } else if constexpr (EPI == EPI_PARTIAL) {
        if constexpr (CT == CT_BF3) {
            if (a == LAY_KC32 && b == LAY_FRAG) return launch_t<CT, LAY_KC32, LAY_FRAG, EPI>(g, s);
        } else {
            if (a == LAY_KC && b == LAY_XC) return launch_t<CT, LAY_KC, LAY_XC, EPI>(g, s);
        }
    } else {
        if (a == LAY_KC && b == LAY_KC) return launch_t<CT, LAY_KC, LAY_KC, EPI>(g, s);
    }
    return hipErrorInvalidValue;
}

template <int CT>
hipError_t launch_c(const GemmDesc &g, hipStream_t s)
{
    switch (g.epi) {
    case EPI_STORE: return launch_e<CT, EPI_STORE>(g, s);
    case EPI_PARTIAL: return launch_e<CT, EPI_PARTIAL>(g, s);
    default: return launch_e<CT, EPI_COLDOT>(g, s);
    }
}

// ------------------------------------------------------------ helpers --

__device__ __forceinline__ void put(void *dst, int ct, int64_t idx, int64_t sub, double v)
{
    if (ct == CT_F64) {
        ((double *)dst)[idx] = v;
    } else if (ct == CT_F32) {
        ((float *)dst)[idx] = (float)v;
    } else {
        uint16_t *b = (uint16_t *)dst;
        const uint16_t h = bf16_rne((float)v);
        const double r1 = v - bf16_val(h);
        const uint16_t m = bf16_rne((float)r1);
        const double r2 = r1 - bf16_val(m);
        b[idx] = h;
        b[idx + sub] = m;
        b[idx + 2 * sub] = bf16_rne((float)r2);
    }
}

// put() for the two adjacent elements idx, idx + 1 (idx even, dst aligned):
// one 16-, 8- or 2 x 3 x 2-byte store instead of two, the same values.
__device__ __forceinline__ void put2(void *dst, int ct, int64_t idx, int64_t sub, double v0, double v1)
{
    if (ct == CT_F64) {
        typedef double dd2 __attribute__((ext_vector_type(2)));
        *(dd2 *)((double *)dst + idx) = dd2{v0, v1};
    } else if (ct == CT_F32) {
        typedef float ff2 __attribute__((ext_vector_type(2)));
        *(ff2 *)((float *)dst + idx) = ff2{(float)v0, (float)v1};
    } else {
        uint16_t h[2], m[2], l[2];
        const double v[2] = {v0, v1};
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            h[u] = bf16_rne((float)v[u]);
            const double r1 = v[u] - bf16_val(h[u]);
            m[u] = bf16_rne((float)r1);
            const double r2 = r1 - bf16_val(m[u]);
            l[u] = bf16_rne((float)r2);
        }
        uint32_t *b = (uint32_t *)((uint16_t *)dst + idx);
        const int64_t sub2 = sub / 2; // planes sub elements apart (sub even)
        b[0] = h[0] | ((uint32_t)h[1] << 16);
        b[sub2] = m[0] | ((uint32_t)m[1] << 16);
        b[2 * sub2] = l[0] | ((uint32_t)l[1] << 16);
    }
}

// Row conversion: dst[r][c] for r < gridDim.x (the padded rows), c < ldd
// (even), two columns per lane; zero outside src's R x C.
__global__ __launch_bounds__(256) void convert_rows_kernel(const double *__restrict__ src, int64_t R, int64_t C,
                                                           int64_t lds, int ct, void *dst, int64_t ldd, int64_t sub)
{
    const int64_t r = blockIdx.x;
    const int64_t c = ((int64_t)blockIdx.y * 256 + threadIdx.x) * 2;
    if (c >= ldd) return;
    double v0 = 0.0, v1 = 0.0;
    if (r < R) {
        if (c < C) v0 = src[r * lds + c];
        if (c + 1 < C) v1 = src[r * lds + c + 1];
    }
    put2(dst, ct, r * ldd + c, sub, v0, v1);
}

// Transposing conversion through a 64 x 64 LDS tile: dst_t[c][r] = src[r][c]
// (dst_t [gridDim.y * 64][ldt]).  Zero outside src's R x C; two elements per
// lane on each store.
__global__ __launch_bounds__(256) void convert_t64_kernel(const double *__restrict__ src, int64_t R, int64_t C,
                                                          int64_t lds, int ct, void *dst_t, int64_t ldt,
                                                          int64_t sub_t)
{
    __shared__ double tile[64][65];
    const int64_t r0 = (int64_t)blockIdx.x * 64; // src rows = dst_t columns
    const int64_t c0 = (int64_t)blockIdx.y * 64; // src cols = dst_t rows
    const int t = threadIdx.x;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const int idx = i * 256 + t;
        const int y = idx >> 5, x = (idx & 31) * 2;
        const int64_t r = r0 + y, c = c0 + x;
        const double v0 = (r < R && c < C) ? src[r * lds + c] : 0.0;
        const double v1 = (r < R && c + 1 < C) ? src[r * lds + c + 1] : 0.0;
        tile[y][x] = v0;
        tile[y][x + 1] = v1;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const int idx = i * 256 + t;
        const int cy = idx >> 5, rx = (idx & 31) * 2;
        put2(dst_t, ct, (c0 + cy) * ldt + r0 + rx, sub_t, tile[rx][cy], tile[rx + 1][cy]);
    }
}

// Direct conversion: dst[r][c] for r < rows_pad, c < ldd.
__global__ void convert_kernel(const double *__restrict__ src, int64_t R, int64_t C, int64_t lds, int ct, void *dst,
                               int64_t ldd, int64_t rows_pad, int64_t sub)
{
    const int64_t total = rows_pad * ldd;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = e / ldd, c = e % ldd;
        const double v = (r < R && c < C) ? src[r * lds + c] : 0.0;
        put(dst, ct, e, sub, v);
    }
}

// Transposing conversion through a 32 x 32 LDS tile: dst[c][r] = src[r][c],
// dst is [rows_pad][ldd] with rows indexed by c.
__global__ __launch_bounds__(256) void convert_t_kernel(const double *__restrict__ src, int64_t R, int64_t C,
                                                        int64_t lds, int ct, void *dst, int64_t ldd, int64_t sub)
{
    __shared__ double tile[32][33];
    const int64_t r0 = (int64_t)blockIdx.x * 32; // src rows = dst columns
    const int64_t c0 = (int64_t)blockIdx.y * 32; // src cols = dst rows
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    for (int y = ty; y < 32; y += 8) {
        const int64_t r = r0 + y, c = c0 + tx;
        tile[y][tx] = (r < R && c < C) ? src[r * lds + c] : 0.0;
    }
    __syncthreads();
    for (int y = ty; y < 32; y += 8) {
        const int64_t c = c0 + y, r = r0 + tx; // dst row c, column r
        put(dst, ct, c * ldd + r, sub, tile[tx][y]);
    }
}

// FP64 value -> three bf16 planes, the same split as put()
__device__ __forceinline__ void split3d(double v, uint32_t &h, uint32_t &m, uint32_t &l)
{
    h = bf16_rne((float)v);
    const double r1 = v - bf16_val((uint16_t)h);
    m = bf16_rne((float)r1);
    const double r2 = r1 - bf16_val((uint16_t)m);
    l = bf16_rne((float)r2);
}

// Eight values (k = 8 kg .. 8 kg + 7 of one column) -> one 16-byte fragment
// row per plane at element offset off.
__device__ __forceinline__ void put_frag8(uint16_t *dst, int64_t sub, int64_t off, const double (&v)[8])
{
    u4 w[3] = {};
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        uint32_t h, m, l;
        split3d(v[e], h, m, l);
        const int q = e >> 1, sh = (e & 1) * 16;
        w[0][q] |= h << sh;
        w[1][q] |= m << sh;
        w[2][q] |= l << sh;
    }
#pragma unroll
    for (int p = 0; p < 3; ++p) *(u4 *)(dst + p * sub + off) = w[p];
}

// One lane per (column x, group of 8 k): eight values gathered through perm
// (consecutive lanes read consecutive columns), split into the three bf16
// planes as put() does, and written as one 16-byte fragment row per plane.
__global__ __launch_bounds__(256) void convert_gather_frag_kernel(const double *__restrict__ src,
                                                                  const int32_t *__restrict__ perm, int64_t R,
                                                                  int64_t C, int64_t lds, uint16_t *dst, int64_t xpad,
                                                                  int64_t sub)
{
    const int64_t x = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t kg = blockIdx.y; // k = 8 kg .. 8 kg + 7
    if (x >= xpad) return;
    double v[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const int64_t k = kg * 8 + e;
        v[e] = (k < R && x < C) ? src[(int64_t)perm[k] * lds + x] : 0.0;
    }
    const int64_t lane = (kg & 3) * 16 + (x & 15);
    put_frag8(dst, sub, (((kg >> 2) * (xpad / 16) + (x >> 4)) * 64 + lane) * 8, v);
}

// The upstream gradient g [R][C] (points x sets) as the two bf16 x 3 operands
// of the backward, from one read of each 32 x 64 tile: [points][sets]
// k-contiguous for the column-dot's B(k = set, j = point) (dst_c, rows of
// xpad_c) and, if dst_s is set, MFMA fragment order for the split-K's
// B(k = point, j = set) (xpad_c / 16 column blocks).  Zero outside R x C.
__global__ __launch_bounds__(256) void convert_g_bwd_kernel(const double *__restrict__ src, int64_t R, int64_t C,
                                                            int64_t lds, uint16_t *dst_c, int64_t subc,
                                                            uint16_t *dst_s, int64_t subs, int64_t xpad_c)
{
    __shared__ double tile[32][65];
    const int64_t r0 = (int64_t)blockIdx.x * 32, c0 = (int64_t)blockIdx.y * 64;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    for (int y = ty; y < 32; y += 4) {
        const int64_t r = r0 + y, c = c0 + tx;
        tile[y][tx] = (r < R && c < C) ? src[r * lds + c] : 0.0;
    }
    __syncthreads();
    const int t = threadIdx.x;
    double v[8];
    { // column-dot operand: row r0 + t / 8, sets c0 + 8 (t % 8) ..; eight lanes per 128-byte row
        const int row = t >> 3, q = t & 7;
#pragma unroll
        for (int e = 0; e < 8; ++e) v[e] = tile[row][q * 8 + e];
        put_frag8(dst_c, subc, (r0 + row) * xpad_c + c0 + q * 8, v);
    }
    if (dst_s) { // split-K operand: set c0 + 16 (t / 64) + t % 16, points r0 + 8 ((t % 64) / 16) ..
        const int bb = t >> 6, lane = t & 63, kg = lane >> 4, xl = lane & 15;
#pragma unroll
        for (int e = 0; e < 8; ++e) v[e] = tile[kg * 8 + e][bb * 16 + xl];
        put_frag8(dst_s, subs, (((r0 / 32) * (xpad_c / 16) + c0 / 16 + bb) * 64 + lane) * 8, v);
    }
}

// Zero the pad of a k-blocked bf16 operand [Mp/8][ld][8] (three planes, sub
// apart): every mode e >= M and every point p >= P.
__global__ void zero_kb8_kernel(uint16_t *dst, int64_t M, int64_t Mp, int64_t P, int64_t ld, int64_t sub)
{
    const int64_t total = (Mp / 8) * ld;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t gq = t / ld, p = t % ld;
        if (gq * 8 + 8 <= M && p < P) continue;
        for (int q = 0; q < 8; ++q) {
            if (gq * 8 + q < M && p < P) continue;
            const int64_t idx = t * 8 + q;
            dst[idx] = 0;
            dst[idx + sub] = 0;
            dst[idx + 2 * sub] = 0;
        }
    }
}

__global__ void zero_kernel(void *dst, int ct, int64_t row0, int64_t rows, int64_t col0, int64_t cols, int64_t ld,
                            int64_t sub)
{
    const int64_t total = rows * cols;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t idx = (row0 + e / cols) * ld + col0 + e % cols;
        put(dst, ct, idx, sub, 0.0);
    }
}

__global__ void splitk_reduce_kernel(const double *__restrict__ part, int S, int64_t M, int64_t N, double *C,
                                     int64_t ldc, int accumulate)
{
    const int64_t total = M * N;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e / N, j = e % N;
        double s = 0.0;
        for (int k = 0; k < S; ++k) s += part[(int64_t)k * M * ldc + i * ldc + j];
        double *c = C + i * ldc + j;
        *c = accumulate ? *c + s : s;
    }
}

__global__ void coldot_reduce_kernel(const double *__restrict__ part, int T, int64_t P, double *out1, double *out2)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    double s1 = 0.0, s2 = 0.0;
    for (int t = 0; t < T; ++t) {
        s1 += part[((int64_t)t * 2 + 0) * P + p];
        s2 += part[((int64_t)t * 2 + 1) * P + p];
    }
    if (out1) out1[p] = s1;
    if (out2) out2[p] = s2;
}

unsigned grid_for(int64_t total, int block)
{
    const int64_t g = (total + block - 1) / block;
    return (unsigned)(g < 65536 * 4 ? (g < 1 ? 1 : g) : 65536 * 4);
}

} // namespace

int coldot_bm(int ct)
{
    return ct == CT_F64 ? Cfg<CT_F64>::BM : ct == CT_F32 ? Cfg<CT_F32>::BM : Cfg<CT_BF3>::BM;
}

zp_status launch_gemm(const GemmDesc &g, hipStream_t s)
{
    if (g.M <= 0 || g.N <= 0) return ZP_OK;
    if (g.K % kPad != 0 || g.splits < 1 || (g.K / g.splits) % kPad != 0 || g.K / g.splits * g.splits != g.K)
        return set_error(ZP_ERR_ARG, "internal: GEMM K split is not a multiple of the pad");
    if (g.ct == CT_BF3 ? false : (g.a.lay == LAY_KB8 || g.b.lay == LAY_KB8))
        return set_error(ZP_ERR_ARG, "internal: k-blocked operands are bf16 only");
    hipError_t e;
    switch (g.ct) {
    case CT_F64: e = launch_c<CT_F64>(g, s); break;
    case CT_F32: e = launch_c<CT_F32>(g, s); break;
    default: e = launch_c<CT_BF3>(g, s); break;
    }
    return hip_check(e, "gemm launch");
}

zp_status launch_convert(const double *src, int64_t R, int64_t C, int64_t lds, int ct, void *dst, int64_t ldd,
                         int64_t rows_pad, int64_t sub, bool transpose, hipStream_t s)
{
    if (!transpose) {
        if (ldd % 2 == 0 && sub % 2 == 0 && rows_pad <= 0x7FFFFFFF && ((uintptr_t)dst & 15) == 0) {
            const dim3 grid((unsigned)rows_pad, (unsigned)((ldd / 2 + 255) / 256));
            hipLaunchKernelGGL(convert_rows_kernel, grid, dim3(256), 0, s, src, R, C, lds, ct, dst, ldd, sub);
        } else {
            hipLaunchKernelGGL(convert_kernel, dim3(grid_for(rows_pad * ldd, 256)), dim3(256), 0, s, src, R, C, lds,
                               ct, dst, ldd, rows_pad, sub);
        }
    } else if (ldd % 64 == 0 && rows_pad % 64 == 0 && sub % 2 == 0) {
        // dst is [rows_pad (>= C, padded)][ldd (>= R, padded)]
        const dim3 grid((unsigned)(ldd / 64), (unsigned)(rows_pad / 64));
        hipLaunchKernelGGL(convert_t64_kernel, grid, dim3(256), 0, s, src, R, C, lds, ct, dst, ldd, sub);
    } else {
        // both multiples of 32
        const dim3 grid((unsigned)(ldd / 32), (unsigned)(rows_pad / 32));
        hipLaunchKernelGGL(convert_t_kernel, grid, dim3(256), 0, s, src, R, C, lds, ct, dst, ldd, sub);
    }
    return hip_check(hipGetLastError(), "convert launch");
}

zp_status launch_convert_gather_frag(const double *src, const int32_t *perm, int64_t R, int64_t C, int64_t lds,
                                     void *dst, int64_t xpad, int64_t kpad, int64_t sub, hipStream_t s)
{
    const dim3 grid((unsigned)((xpad + 255) / 256), (unsigned)(kpad / 8));
    hipLaunchKernelGGL(convert_gather_frag_kernel, grid, dim3(256), 0, s, src, perm, R, C, lds, (uint16_t *)dst, xpad,
                       sub);
    return hip_check(hipGetLastError(), "convert launch");
}

zp_status launch_convert_g_bwd(const double *src, int64_t R, int64_t C, int64_t lds, void *dst_c, int64_t subc,
                               void *dst_s, int64_t subs, int64_t xpad_r, int64_t xpad_c, hipStream_t s)
{
    const dim3 grid((unsigned)(xpad_r / 32), (unsigned)(xpad_c / 64));
    hipLaunchKernelGGL(convert_g_bwd_kernel, grid, dim3(256), 0, s, src, R, C, lds, (uint16_t *)dst_c, subc,
                       (uint16_t *)dst_s, subs, xpad_c);
    return hip_check(hipGetLastError(), "convert launch");
}

zp_status launch_zero_kb8(void *dst, int64_t M, int64_t Mp, int64_t P, int64_t ld, int64_t sub, hipStream_t s)
{
    hipLaunchKernelGGL(zero_kb8_kernel, dim3(grid_for((Mp / 8) * ld, 256)), dim3(256), 0, s, (uint16_t *)dst, M, Mp,
                       P, ld, sub);
    return hip_check(hipGetLastError(), "zero-pad launch");
}

zp_status launch_zero_pad(void *dst, int ct, int64_t rows, int64_t cols, int64_t rows_pad, int64_t ld, int64_t sub,
                          hipStream_t s)
{
    if (rows_pad > rows) {
        const int64_t n = (rows_pad - rows) * ld;
        hipLaunchKernelGGL(zero_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, dst, ct, rows, rows_pad - rows,
                           (int64_t)0, ld, ld, sub);
    }
    if (ld > cols && rows > 0) {
        const int64_t n = rows * (ld - cols);
        hipLaunchKernelGGL(zero_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, dst, ct, (int64_t)0, rows, cols,
                           ld - cols, ld, sub);
    }
    return hip_check(hipGetLastError(), "zero-pad launch");
}

zp_status launch_splitk_reduce(const double *part, int S, int64_t M, int64_t N, double *C, int64_t ldc,
                               bool accumulate, hipStream_t s)
{
    hipLaunchKernelGGL(splitk_reduce_kernel, dim3(grid_for(M * N, 256)), dim3(256), 0, s, part, S, M, N, C, ldc,
                       accumulate ? 1 : 0);
    return hip_check(hipGetLastError(), "split-K reduce launch");
}

zp_status launch_coldot_reduce(const double *part, int T, int64_t P, double *out1, double *out2, hipStream_t s)
{
    hipLaunchKernelGGL(coldot_reduce_kernel, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, s, part, T, P, out1,
                       out2);
    return hip_check(hipGetLastError(), "column-dot reduce launch");
}

} // namespace zp
