// Numeric phase: C_s = sum over the products t of segment s (k ascending) of
// A[prodA[t]] * B[prodB[t]], one b x b block per segment, on gfx950 MFMA.
//
// This replaces the paper's leaf library, which ran every outer product
// batch of a leaf through a batched GEMM (Sec. 4.1, Fig. 2) and accumulated
// into C in memory. Here the waves that own a C block keep it in MFMA
// accumulators across all its block products and store it once, so C is
// never re-read and no two waves ever write the same C entry (no atomics).
//
// MFMA operand layout (16 x 16 x 4 for fp64/fp32): lane l = 16*g + r supplies
// A[r][kk = g] and B[kk = g][r] of one 4-deep step; its four accumulator
// values are D[4*g + i][r] (i = 0..3) for fp32, but D[4*i + g][r] for fp64
// (the fp64 instruction interleaves the row groups; checked on gfx950 with a
// known-input product). The inner index is a free summation variable, which
// lets each lane read its A entries with 16-byte loads (see wave_block); the
// output columns are free to permute too, which lets a lane read two adjacent
// B entries for the two column tiles of its wave in one load.
//
// Two launch shapes:
//  * b = 16 and 32: each workgroup is a single wave that owns one C block
//    (the batch kernels use the same shape at b = 64, one wave per 32 x 32
//    tile): a finished wave frees its slot at once, so a short segment never
//    holds a SIMD while a long neighbour runs.
//  * b = 64: one workgroup of four waves per C block, each wave a 32 x 32
//    tile; the block products are staged in LDS once per workgroup and every
//    wave reads its operand panels from there (k_numeric_f64_b64,
//    k_numeric_f32_b64, k_numeric_bf16x3_b64).
// The dispatcher hands workgroup w to XCD w % 8, and each XCD has its own L2.
// Consecutive C blocks in Morton order share most of their A and B blocks,
// so the launch gives each XCD runs of consecutive tiles (1024 single-wave
// tiles, or 256 four-wave C blocks; XCD x takes runs x, x+8, x+16, ...)
// instead of every eighth tile: neighbours then meet in the same L2, while
// the interleaved runs keep the eight XCDs equally loaded. C is written with
// non-temporal stores, since no later step of the multiply reads it.
//
// The same per-wave routines serve one multiply (k_numeric: one launch over
// the C blocks of C) and a batch of independent multiplies (k_batch_*: one
// launch over the C blocks of all of them).
#include "qt_internal.h"

#include <algorithm>
#include <map>
#include <mutex>

namespace qt {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

template <class T> struct Mfma;
template <> struct Mfma<double> {
    typedef v4d acc;
    static __device__ __forceinline__ acc step(double a, double b, acc c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    // row of accumulator value i held by lane group g
    static __device__ __forceinline__ int row(int g, int i) { return 4 * i + g; }
};
template <> struct Mfma<float> {
    typedef v4f acc;
    static __device__ __forceinline__ acc step(float a, float b, acc c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int g, int i) { return 4 * g + i; }
};

// Tile geometry for block size BS: each wave computes a WT x WT tile made of
// MT x MT 16x16 MFMA tiles; WPB waves cover one C block; the inner dimension
// is walked in chunks of KC with KS 4-deep MFMA steps each. All of a chunk's
// loads are issued before its MFMAs (a scheduling barrier keeps the compiler
// from sinking them next to their first use, which left each wave only one
// to three loads in flight); the next chunk's loads may still rise above the
// current chunk's MFMAs. Measured on gfx950 at b = 32 against the compiler's
// own interleaving: fp64 6% and fp32 8% faster on decay32768, fp64 6% faster
// and fp32 6% slower on random65536.
template <int BS> struct Geo {
    static constexpr int WT = BS < 32 ? BS : 32;
    static constexpr int MT = WT / 16;
    static constexpr int WPB = (BS / WT) * (BS / WT);
    static constexpr int KC = 16;
    static constexpr int KS = KC / 4;
    static constexpr int NCH = BS / KC;
};

constexpr int XCD_CHUNK_LOG = 10;

// Logical tile of physical workgroup w; a bijection on [0, grid) when the
// grid is a multiple of 8 << XCD_CHUNK_LOG (xcd_grid pads it so).
template <int LOG = XCD_CHUNK_LOG>
__device__ __forceinline__ int64_t xcd_logical(int64_t w) {
    const int64_t x = w & 7, i = w >> 3;
    return ((((i >> LOG) << 3) + x) << LOG) | (i & ((1 << LOG) - 1));
}

template <int LOG = XCD_CHUNK_LOG>
static unsigned xcd_grid(int64_t tiles) {
    const int64_t q = int64_t(8) << LOG;
    const int64_t g = (tiles + q - 1) / q * q;
    if (g > 0x7fffffffLL) fail(QT_ERR_UNSUPPORTED, "numeric launch too large");
    return (unsigned)g;
}

// One wave: tile `sub` of a C block, over the products t0 .. t1-1. BUF: the
// C tile is written with buffer stores instead of global stores (the same
// non-temporal policy); measured faster when C blocks are launched grouped by
// inner index (about one block product per C block, so the kernel is bound
// by writing C), slower for the FP32 kernel in Morton order.
template <class T, int BS, bool BUF = false>
__device__ __forceinline__ void wave_block(const T* __restrict__ A, const T* __restrict__ B,
                                           const int32_t* __restrict__ prodA, const int32_t* __restrict__ prodB,
                                           int32_t t0, int32_t t1, T* __restrict__ c, int sub, int32_t ia0,
                                           int32_t ib0) {
    typedef Geo<BS> G;
    typedef typename Mfma<T>::acc acc_t;
    constexpr int VEC = 16 / sizeof(T);            // elements per 16-byte load
    constexpr int NV = G::KS / VEC;                // 16-byte loads per A row per chunk
    typedef T vec_t __attribute__((ext_vector_type(VEC)));
    typedef T pair_t __attribute__((ext_vector_type(2)));
    const int lane = threadIdx.x & 63;
    const int r16 = lane & 15;
    const int g = lane >> 4;
    const int wm = (sub / (BS / G::WT)) * G::WT;
    const int wn = (sub % (BS / G::WT)) * G::WT;

    acc_t acc[G::MT][G::MT];
#pragma unroll
    for (int i = 0; i < G::MT; ++i)
#pragma unroll
        for (int j = 0; j < G::MT; ++j) acc[i][j] = acc_t{0, 0, 0, 0};

    // Step ks of a chunk gives lane group g the inner index
    //   k = (ks / VEC) * 4*VEC + g*VEC + ks % VEC,
    // so each 16-byte A load of a lane is VEC consecutive entries of its row
    // and the four lane groups together read one contiguous run per row.
    // Block indices of the next product are fetched while this one runs;
    // the caller gives the first product's (ia0, ib0).
    int32_t ia = ia0, ib = ib0;
    for (int32_t t = t0; t < t1; ++t) {
        const T* a = A + (size_t)ia * (BS * BS);
        const T* b = B + (size_t)ib * (BS * BS);
        if (t + 1 < t1) {
            ia = prodA[t + 1];
            ib = prodB[t + 1];
        }
#pragma unroll
        for (int ch = 0; ch < G::NCH; ++ch) {
            T ar[G::MT][G::KS], br[G::MT][G::KS];
#pragma unroll
            for (int mt = 0; mt < G::MT; ++mt) {
                const T* row = a + (wm + mt * 16 + r16) * BS + ch * G::KC + g * VEC;
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    const vec_t x = *reinterpret_cast<const vec_t*>(row + v * 4 * VEC);
#pragma unroll
                    for (int e = 0; e < VEC; ++e) ar[mt][v * VEC + e] = x[e];
                }
            }
            if constexpr (G::MT == 2) {
                // the two 16-column tiles of a wave interleave: lane r16 holds
                // column 2 r16 of the 32 in tile 0 and 2 r16 + 1 in tile 1, so
                // one load of two adjacent entries feeds both tiles
#pragma unroll
                for (int v = 0; v < NV; ++v)
#pragma unroll
                    for (int e = 0; e < VEC; ++e) {
                        const pair_t x = *reinterpret_cast<const pair_t*>(
                            b + (ch * G::KC + v * 4 * VEC + g * VEC + e) * BS + wn + 2 * r16);
                        br[0][v * VEC + e] = x[0];
                        br[1][v * VEC + e] = x[1];
                    }
            } else {
#pragma unroll
                for (int v = 0; v < NV; ++v)
#pragma unroll
                    for (int e = 0; e < VEC; ++e)
                        br[0][v * VEC + e] = b[(ch * G::KC + v * 4 * VEC + g * VEC + e) * BS + wn + r16];
            }
            __builtin_amdgcn_sched_barrier(0);   // the chunk's loads stay above this point
#pragma unroll
            for (int ks = 0; ks < G::KS; ++ks)
#pragma unroll
                for (int mt = 0; mt < G::MT; ++mt)
#pragma unroll
                    for (int nt = 0; nt < G::MT; ++nt)
                        acc[mt][nt] = Mfma<T>::step(ar[mt][ks], br[nt][ks], acc[mt][nt]);
        }
    }
    if constexpr (G::MT == 2 && BUF) {
        // a buffer over this C block (BS * BS elements; an offset past it
        // would be dropped, none is), non-temporal stores (policy bit 1)
        constexpr int kBufferWord3 = 0x00020000;   // gfx9 raw buffer: 32-bit data format
        constexpr int kNonTemporal = 2;
        const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(c, 0, BS * BS * (int)sizeof(T), kBufferWord3);
#pragma unroll
        for (int mt = 0; mt < G::MT; ++mt)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const pair_t v = {acc[mt][0][i], acc[mt][1][i]};
                const int off = (int)sizeof(T) * ((wm + mt * 16 + Mfma<T>::row(g, i)) * BS + wn + 2 * r16);
                if constexpr (sizeof(T) == 8) {
                    typedef unsigned int u4 __attribute__((ext_vector_type(4)));
                    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u4, v), rs, off, 0, kNonTemporal);
                } else {
                    typedef unsigned int u2 __attribute__((ext_vector_type(2)));
                    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, v), rs, off, 0, kNonTemporal);
                }
            }
    } else if constexpr (G::MT == 2) {
#pragma unroll
        for (int mt = 0; mt < G::MT; ++mt)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const pair_t v = {acc[mt][0][i], acc[mt][1][i]};
                __builtin_nontemporal_store(
                    v, reinterpret_cast<pair_t*>(c + (wm + mt * 16 + Mfma<T>::row(g, i)) * BS + wn + 2 * r16));
            }
    } else {
#pragma unroll
        for (int i = 0; i < 4; ++i)
            __builtin_nontemporal_store(acc[0][0][i], c + (wm + Mfma<T>::row(g, i)) * BS + wn + r16);
    }
}

// As wave_block, for product lists whose block indices may carry the
// transposition bit (PROD_TRANS): the block is then read as its transpose,
// op(A) = A^T or op(B) = B^T for that product, straight from the stored
// block. A lane's rows interleave like its columns (lane r16 holds rows
// 2 r16 and 2 r16 + 1 in tiles 0 and 1), so a transposed A block, whose rows
// of op(A) are stored columns, gives both of a lane's rows in one load of two
// adjacent entries, as an untransposed B block gives both of its columns.
// A transposed B block gives a lane VEC consecutive inner indices of one
// column in one load, as an untransposed A block does for a row. The
// transposition is uniform over the wave (one product at a time), so the
// choice is a scalar branch. The inner index order is wave_block's, so every
// result is bitwise what wave_block gives on transposed copies of the blocks.
template <class T, int BS>
__device__ __forceinline__ void wave_block_op(const T* __restrict__ A, const T* __restrict__ B,
                                              const int32_t* __restrict__ prodA, const int32_t* __restrict__ prodB,
                                              int32_t t0, int32_t t1, T* __restrict__ c, int sub) {
    typedef Geo<BS> G;
    typedef typename Mfma<T>::acc acc_t;
    constexpr int VEC = 16 / sizeof(T);
    constexpr int NV = G::KS / VEC;
    constexpr int RS = G::MT;                      // stride between a lane's rows (and columns)
    typedef T vec_t __attribute__((ext_vector_type(VEC)));
    typedef T pair_t __attribute__((ext_vector_type(2)));
    const int lane = threadIdx.x & 63;
    const int r16 = lane & 15;
    const int g = lane >> 4;
    const int wm = (sub / (BS / G::WT)) * G::WT;
    const int wn = (sub % (BS / G::WT)) * G::WT;

    acc_t acc[G::MT][G::MT];
#pragma unroll
    for (int i = 0; i < G::MT; ++i)
#pragma unroll
        for (int j = 0; j < G::MT; ++j) acc[i][j] = acc_t{0, 0, 0, 0};

    int32_t ia = prodA[t0], ib = prodB[t0];
    for (int32_t t = t0; t < t1; ++t) {
        const bool ta = ia < 0, tb = ib < 0;
        const T* a = A + (size_t)(ia & PROD_INDEX) * (BS * BS);
        const T* b = B + (size_t)(ib & PROD_INDEX) * (BS * BS);
        if (t + 1 < t1) {
            ia = prodA[t + 1];
            ib = prodB[t + 1];
        }
#pragma unroll
        for (int ch = 0; ch < G::NCH; ++ch) {
            T ar[G::MT][G::KS], br[G::MT][G::KS];
            if (!ta) {
#pragma unroll
                for (int mt = 0; mt < G::MT; ++mt) {
                    const T* row = a + (wm + RS * r16 + mt) * BS + ch * G::KC + g * VEC;
#pragma unroll
                    for (int v = 0; v < NV; ++v) {
                        const vec_t x = *reinterpret_cast<const vec_t*>(row + v * 4 * VEC);
#pragma unroll
                        for (int e = 0; e < VEC; ++e) ar[mt][v * VEC + e] = x[e];
                    }
                }
            } else {
#pragma unroll
                for (int ks = 0; ks < G::KS; ++ks) {
                    const int k = ch * G::KC + (ks / VEC) * 4 * VEC + g * VEC + ks % VEC;
                    if constexpr (G::MT == 2) {
                        const pair_t x = *reinterpret_cast<const pair_t*>(a + k * BS + wm + 2 * r16);
                        ar[0][ks] = x[0];
                        ar[1][ks] = x[1];
                    } else {
                        ar[0][ks] = a[k * BS + wm + r16];
                    }
                }
            }
            if (!tb) {
#pragma unroll
                for (int ks = 0; ks < G::KS; ++ks) {
                    const int k = ch * G::KC + (ks / VEC) * 4 * VEC + g * VEC + ks % VEC;
                    if constexpr (G::MT == 2) {
                        const pair_t x = *reinterpret_cast<const pair_t*>(b + k * BS + wn + 2 * r16);
                        br[0][ks] = x[0];
                        br[1][ks] = x[1];
                    } else {
                        br[0][ks] = b[k * BS + wn + r16];
                    }
                }
            } else {
#pragma unroll
                for (int nt = 0; nt < G::MT; ++nt) {
                    const T* col = b + (wn + RS * r16 + nt) * BS + ch * G::KC + g * VEC;
#pragma unroll
                    for (int v = 0; v < NV; ++v) {
                        const vec_t x = *reinterpret_cast<const vec_t*>(col + v * 4 * VEC);
#pragma unroll
                        for (int e = 0; e < VEC; ++e) br[nt][v * VEC + e] = x[e];
                    }
                }
            }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int ks = 0; ks < G::KS; ++ks)
#pragma unroll
                for (int mt = 0; mt < G::MT; ++mt)
#pragma unroll
                    for (int nt = 0; nt < G::MT; ++nt)
                        acc[mt][nt] = Mfma<T>::step(ar[mt][ks], br[nt][ks], acc[mt][nt]);
        }
    }
    if constexpr (G::MT == 2) {
#pragma unroll
        for (int mt = 0; mt < G::MT; ++mt)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const pair_t v = {acc[mt][0][i], acc[mt][1][i]};
                __builtin_nontemporal_store(
                    v, reinterpret_cast<pair_t*>(c + (wm + 2 * Mfma<T>::row(g, i) + mt) * BS + wn + 2 * r16));
            }
    } else {
#pragma unroll
        for (int i = 0; i < 4; ++i)
            __builtin_nontemporal_store(acc[0][0][i], c + (wm + Mfma<T>::row(g, i)) * BS + wn + r16);
    }
}

// Split-bf16 path: per block product, F = lo_a*hi_b + hi_a*lo_b + hi_a*hi_b
// in fp32 MFMA (16 x 16 x 32 bf16: lane 16*g + r supplies A[r][8g .. 8g+7]
// and B[8g .. 8g+7][r]); F is then added into fp64 accumulators, and C is
// stored in fp64. B is read from its transposed copy so both operands are
// 16-byte contiguous loads.
__device__ __forceinline__ v8bf load8(const uint16_t* p) {
    uint4 u = *reinterpret_cast<const uint4*>(p);
    v8bf r;
    __builtin_memcpy(&r, &u, sizeof(r));
    return r;
}

// Split operands of one product: op(A) row-major (A's split, or the split of
// the transposed block) and op(B)^T row-major (B's transposed split, or B's
// own split when the product reads B transposed).
struct SplitOps {
    const uint16_t* Ahi; const uint16_t* Alo;
    const uint16_t* Ahi_t; const uint16_t* Alo_t;
    const uint16_t* Bhi; const uint16_t* Blo;
    const uint16_t* Bhi_t; const uint16_t* Blo_t;
};

template <int BS, bool DYN = false>
__device__ __forceinline__ void wave_block_bf16x3(const uint16_t* __restrict__ Ahi, const uint16_t* __restrict__ Alo,
                                                  const uint16_t* __restrict__ Bhi_t,
                                                  const uint16_t* __restrict__ Blo_t,
                                                  const int32_t* __restrict__ prodA,
                                                  const int32_t* __restrict__ prodB, int32_t t0, int32_t t1,
                                                  double* __restrict__ c, int sub, const SplitOps* ops = nullptr) {
    static_assert(BS == 32 || BS == 64, "split-bf16 path needs b = 32 or 64");
    constexpr int WT = 32, MT = 2;
    const int lane = threadIdx.x & 63;
    const int r16 = lane & 15;
    const int g = lane >> 4;
    const int wm = (sub / (BS / WT)) * WT;
    const int wn = (sub % (BS / WT)) * WT;

    v4d acc[MT][MT];
#pragma unroll
    for (int i = 0; i < MT; ++i)
#pragma unroll
        for (int j = 0; j < MT; ++j) acc[i][j] = v4d{0, 0, 0, 0};

    for (int32_t t = t0; t < t1; ++t) {
        const int32_t ia = prodA[t], ib = prodB[t];
        const size_t oa = (size_t)(ia & PROD_INDEX) * (BS * BS);
        const size_t ob = (size_t)(ib & PROD_INDEX) * (BS * BS);
        if constexpr (DYN) {
            // a transposed block's row-major op form is the other layout of its split
            Ahi = ia < 0 ? ops->Ahi_t : ops->Ahi;
            Alo = ia < 0 ? ops->Alo_t : ops->Alo;
            Bhi_t = ib < 0 ? ops->Bhi : ops->Bhi_t;
            Blo_t = ib < 0 ? ops->Blo : ops->Blo_t;
        }
        v4f f[MT][MT];
#pragma unroll
        for (int i = 0; i < MT; ++i)
#pragma unroll
            for (int j = 0; j < MT; ++j) f[i][j] = v4f{0, 0, 0, 0};
#pragma unroll
        for (int kc = 0; kc < BS / 32; ++kc) {
            v8bf ah[MT], al[MT], bh[MT], bl[MT];
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) {
                const size_t o = oa + (size_t)(wm + mt * 16 + r16) * BS + kc * 32 + g * 8;
                ah[mt] = load8(Ahi + o);
                al[mt] = load8(Alo + o);
            }
#pragma unroll
            for (int nt = 0; nt < MT; ++nt) {
                const size_t o = ob + (size_t)(wn + nt * 16 + r16) * BS + kc * 32 + g * 8;
                bh[nt] = load8(Bhi_t + o);
                bl[nt] = load8(Blo_t + o);
            }
            __builtin_amdgcn_sched_barrier(0);   // as in wave_block: loads first (5% faster at b = 32)
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                for (int nt = 0; nt < MT; ++nt) {
                    f[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[mt], bh[nt], f[mt][nt], 0, 0, 0);
                    f[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[mt], bl[nt], f[mt][nt], 0, 0, 0);
                    f[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[mt], bh[nt], f[mt][nt], 0, 0, 0);
                }
        }
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int nt = 0; nt < MT; ++nt)
#pragma unroll
                for (int i = 0; i < 4; ++i) acc[mt][nt][i] += (double)f[mt][nt][i];
    }
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int nt = 0; nt < MT; ++nt)
#pragma unroll
            for (int i = 0; i < 4; ++i)
                __builtin_nontemporal_store(acc[mt][nt][i], c + (wm + mt * 16 + 4 * g + i) * BS + wn + nt * 16 + r16);
}

// ------------------------------------------------------ one multiply

// Waves per SIMD the compiler must fit: five for the b = 32 fp64 kernel
// (82 VGPRs with a whole chunk's operands in flight), which measured best on
// gfx950 (four and six within 1%, three 7% slower); the other instances fit
// eight by themselves.
template <class T, int BS> struct MinWaves { static constexpr int value = 1; };
template <> struct MinWaves<double, 32> { static constexpr int value = 5; };

template <class T, int BS>
__global__ __launch_bounds__(64, (MinWaves<T, BS>::value)) void k_numeric(const T* __restrict__ A, const T* __restrict__ B,
                                                const int32_t* __restrict__ prodA,
                                                const int32_t* __restrict__ prodB,
                                                const int32_t* __restrict__ seg, int32_t nseg,
                                                const int32_t* __restrict__ order, T* __restrict__ C) {
    typedef Geo<BS> G;
    const int64_t tile = xcd_logical<>(blockIdx.x);
    const int64_t q = tile / G::WPB;
    if (q >= nseg) return;
    const int64_t s = order ? order[q] : q;
    const int32_t t0 = seg[s];
    wave_block<T, BS>(A, B, prodA, prodB, t0, seg[s + 1], C + (size_t)s * (BS * BS), (int)(tile % G::WPB),
                      prodA[t0], prodB[t0]);
}

// k_numeric for C blocks launched grouped by inner index (`order` is that
// order), writing C with buffer stores. Such C blocks average about one block
// product, so the kernel is bound by writing C; fewer waves in flight then
// contend less for HBM and leave slots to the next multiply's traversal. The
// FP32 instance (registers for seven waves per SIMD) is held to five by LDS
// it never touches (ByKCap): random65536 FP32 steps 1.350 instead of 1.402 ms
// in a loop, lone launches 0.96-0.98 instead of 1.00-1.02 ms. At four waves,
// or with the FP64 instance held below its five, it was slower.
template <class T, int BS> struct ByKCap { static constexpr int waves = 0; };
template <> struct ByKCap<float, 32> { static constexpr int waves = 5; };
constexpr int kLdsPerCU = 160 * 1024;   // gfx950

// Dynamic LDS per one-wave workgroup that holds the kernel to `waves` waves
// per SIMD (four SIMDs per CU); 0: no cap.
constexpr size_t occupancy_cap_lds(int waves) { return waves > 0 ? (size_t)(kLdsPerCU / (4 * waves)) : 0; }

template <class T, int BS>
__global__ __launch_bounds__(64, (MinWaves<T, BS>::value)) void k_numeric_byk(const T* __restrict__ A,
                                                                             const T* __restrict__ B,
                                                                             const int32_t* __restrict__ prodA,
                                                                             const int32_t* __restrict__ prodB,
                                                                             const int32_t* __restrict__ seg,
                                                                             int32_t nseg,
                                                                             const int32_t* __restrict__ order,
                                                                             T* __restrict__ C) {
    typedef Geo<BS> G;
    const int64_t tile = xcd_logical<>(blockIdx.x);
    const int64_t q = tile / G::WPB;
    if (q >= nseg) return;
    const int64_t s = order[q];
    const int32_t t0 = seg[s];
    wave_block<T, BS, true>(A, B, prodA, prodB, t0, seg[s + 1], C + (size_t)s * (BS * BS), (int)(tile % G::WPB),
                            prodA[t0], prodB[t0]);
}

template <int BS>
__global__ __launch_bounds__(64) void k_numeric_bf16x3(const uint16_t* __restrict__ Ahi,
                                                       const uint16_t* __restrict__ Alo,
                                                       const uint16_t* __restrict__ Bhi_t,
                                                       const uint16_t* __restrict__ Blo_t,
                                                       const int32_t* __restrict__ prodA,
                                                       const int32_t* __restrict__ prodB,
                                                       const int32_t* __restrict__ seg, int32_t nseg,
                                                       const int32_t* __restrict__ order, double* __restrict__ C) {
    constexpr int WPB = (BS / 32) * (BS / 32);
    const int64_t tile = xcd_logical<>(blockIdx.x);
    const int64_t q = tile / WPB;
    if (q >= nseg) return;
    const int64_t s = order ? order[q] : q;
    wave_block_bf16x3<BS>(Ahi, Alo, Bhi_t, Blo_t, prodA, prodB, seg[s], seg[s + 1], C + (size_t)s * (BS * BS),
                          (int)(tile % WPB));
}

// One multiply whose products may read blocks transposed (transposed
// operands, symmetric operands stored as a triangle): one wave per tile, as
// k_numeric at b = 16 and 32, at every block size.
template <class T, int BS>
__global__ __launch_bounds__(64, (MinWaves<T, BS>::value)) void k_numeric_op(const T* __restrict__ A,
                                                                           const T* __restrict__ B,
                                                                           const int32_t* __restrict__ prodA,
                                                                           const int32_t* __restrict__ prodB,
                                                                           const int32_t* __restrict__ seg,
                                                                           int32_t nseg,
                                                                           const int32_t* __restrict__ order,
                                                                           T* __restrict__ C) {
    typedef Geo<BS> G;
    const int64_t tile = xcd_logical<>(blockIdx.x);
    const int64_t q = tile / G::WPB;
    if (q >= nseg) return;
    const int64_t s = order ? order[q] : q;
    wave_block_op<T, BS>(A, B, prodA, prodB, seg[s], seg[s + 1], C + (size_t)s * (BS * BS), (int)(tile % G::WPB));
}

template <int BS>
__global__ __launch_bounds__(64) void k_numeric_bf16x3_op(SplitOps ops, const int32_t* __restrict__ prodA,
                                                          const int32_t* __restrict__ prodB,
                                                          const int32_t* __restrict__ seg, int32_t nseg,
                                                          const int32_t* __restrict__ order, double* __restrict__ C) {
    constexpr int WPB = (BS / 32) * (BS / 32);
    const int64_t tile = xcd_logical<>(blockIdx.x);
    const int64_t q = tile / WPB;
    if (q >= nseg) return;
    const int64_t s = order ? order[q] : q;
    wave_block_bf16x3<BS, true>(nullptr, nullptr, nullptr, nullptr, prodA, prodB, seg[s], seg[s + 1],
                                C + (size_t)s * (BS * BS), (int)(tile % WPB), &ops);
}

// b = 64 fp64 with the operands shared through LDS, as for the split path
// below: one workgroup of four waves per 64 x 64 C block, wave w the 32 x 32
// tile (w / 2, w % 2). A block product is staged in two halves of the inner
// index: A's 64 x 32 and B's 32 x 64 half (16 KiB each) go to LDS once and
// each wave reads its panels from there (32 KiB per half per workgroup from
// L2 instead of 64 KiB). LDS rows are padded so that the 16 lanes of a group
// reading 16 rows of A hit distinct banks (34 doubles), and the four groups
// reading four rows of B fall in different halves of the banks (72 doubles).
constexpr int F64L_AROW = 34;
constexpr int F64L_BROW = 72;

// One C block of the LDS-sharing kernel below, products t0 .. t1-1, into c
// (all four waves of the workgroup take part).
__device__ __forceinline__ void lds_block_f64(const double* __restrict__ A, const double* __restrict__ B,
        const int32_t* __restrict__ prodA, const int32_t* __restrict__ prodB, int32_t t0, int32_t t1,
        double* __restrict__ c) {
    constexpr int BS = 64, MT = 2, KH = 32;
    typedef double v2d_t __attribute__((ext_vector_type(2)));
    __shared__ __attribute__((aligned(16))) double la[64 * F64L_AROW];   // A[:, half]
    __shared__ __attribute__((aligned(16))) double lb[KH * F64L_BROW];   // B[half, :]
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int r16 = lane & 15, g = lane >> 4;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;

    v4d acc[MT][MT];
#pragma unroll
    for (int i = 0; i < MT; ++i)
#pragma unroll
        for (int j = 0; j < MT; ++j) acc[i][j] = v4d{0, 0, 0, 0};

    // 16-byte pieces: A's half is 64 rows x 16 pieces, B's half 32 rows x 32
    // pieces; thread tid moves pieces tid + 256 r, r = 0..3, of each. The
    // loads of the next half are issued right after the current half is in
    // LDS, so they are in flight during its MFMAs.
    v2d_t pa[4], pb[4];
#define QT_F64L_FETCH(TT, HH)                                                                          \
    do {                                                                                               \
        const double* a_ = A + (size_t)prodA[TT] * (BS * BS);                                          \
        const double* b_ = B + (size_t)prodB[TT] * (BS * BS);                                          \
        _Pragma("unroll") for (int r = 0; r < 4; ++r) {                                                \
            const int pc = tid + 256 * r;                                                              \
            pa[r] = *reinterpret_cast<const v2d_t*>(a_ + (pc >> 4) * BS + (HH) * KH + (pc & 15) * 2);  \
            pb[r] = *reinterpret_cast<const v2d_t*>(b_ + ((HH) * KH + (pc >> 5)) * BS + (pc & 31) * 2); \
        }                                                                                              \
    } while (0)
    QT_F64L_FETCH(t0, 0);   // a segment holds at least one product
    for (int32_t t = t0; t < t1; ++t) {
#pragma unroll 1
        for (int h = 0; h < 2; ++h) {
            __syncthreads();   // every wave is done reading the previous half
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int pc = tid + 256 * r;
                *reinterpret_cast<v2d_t*>(la + (pc >> 4) * F64L_AROW + (pc & 15) * 2) = pa[r];
                *reinterpret_cast<v2d_t*>(lb + (pc >> 5) * F64L_BROW + (pc & 31) * 2) = pb[r];
            }
            __syncthreads();
            if (h == 0)
                QT_F64L_FETCH(t, 1);
            else if (t + 1 < t1)
                QT_F64L_FETCH(t + 1, 0);
            // step ks gives lane group g the inner index k = 8 (ks / 2) + 2 g + ks % 2
            double ar[MT][8], br[MT][8];
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const v2d_t x = *reinterpret_cast<const v2d_t*>(la + (wm + mt * 16 + r16) * F64L_AROW + 8 * v + 2 * g);
                    ar[mt][2 * v] = x[0];
                    ar[mt][2 * v + 1] = x[1];
                }
#pragma unroll
            for (int nt = 0; nt < MT; ++nt)
#pragma unroll
                for (int ks = 0; ks < 8; ++ks)
                    br[nt][ks] = lb[(8 * (ks >> 1) + 2 * g + (ks & 1)) * F64L_BROW + wn + nt * 16 + r16];
#pragma unroll
            for (int ks = 0; ks < 8; ++ks)
#pragma unroll
                for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                    for (int nt = 0; nt < MT; ++nt)
                        acc[mt][nt] = Mfma<double>::step(ar[mt][ks], br[nt][ks], acc[mt][nt]);
        }
    }
#undef QT_F64L_FETCH
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int nt = 0; nt < MT; ++nt)
#pragma unroll
            for (int i = 0; i < 4; ++i)
                __builtin_nontemporal_store(acc[mt][nt][i],
                                            c + (wm + mt * 16 + Mfma<double>::row(g, i)) * BS + wn + nt * 16 + r16);
}

__global__ __launch_bounds__(256, 4) void k_numeric_f64_b64(const double* __restrict__ A, const double* __restrict__ B,
                                                         const int32_t* __restrict__ prodA,
                                                         const int32_t* __restrict__ prodB,
                                                         const int32_t* __restrict__ seg, int32_t nseg,
                                                         const int32_t* __restrict__ order, double* __restrict__ C) {
    const int64_t q = xcd_logical<8>(blockIdx.x);
    if (q >= nseg) return;   // uniform over the workgroup
    const int64_t s = order ? order[q] : q;
    lds_block_f64(A, B, prodA, prodB, seg[s], seg[s + 1], C + (size_t)s * (64 * 64));
}

// b = 64 fp32 with the operands shared through LDS, like the fp64 kernel
// above: halves of the inner index, each loaded once per workgroup, and the
// next half's loads in flight during the current half's MFMAs. A half of A
// is 64 x 32 and a half of B 32 x 64 floats (8 KiB each). LDS rows are padded
// to 36 and 72 floats: the 16 lanes of a group reading 16 rows of A then
// cover the 64 banks once, and the four groups reading rows of B four apart
// touch every bank exactly twice. The two column tiles of a wave interleave
// as in the per-wave kernel and the k order is that kernel's, so the result
// is bitwise the same.
constexpr int F32L_AROW = 36;
constexpr int F32L_BROW = 72;

// One C block of the LDS-sharing kernel below, products t0 .. t1-1, into c
// (all four waves of the workgroup take part).
__device__ __forceinline__ void lds_block_f32(const float* __restrict__ A, const float* __restrict__ B,
        const int32_t* __restrict__ prodA, const int32_t* __restrict__ prodB, int32_t t0, int32_t t1,
        float* __restrict__ c) {
    constexpr int BS = 64, MT = 2, KH = 32;
    typedef float v2f_t __attribute__((ext_vector_type(2)));
    __shared__ __attribute__((aligned(16))) float la[64 * F32L_AROW];   // A[:, half]
    __shared__ __attribute__((aligned(16))) float lb[KH * F32L_BROW];   // B[half, :]
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int r16 = lane & 15, g = lane >> 4;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;

    v4f acc[MT][MT];
#pragma unroll
    for (int i = 0; i < MT; ++i)
#pragma unroll
        for (int j = 0; j < MT; ++j) acc[i][j] = v4f{0, 0, 0, 0};

    // 16-byte pieces: A's half is 64 rows x 8 pieces, B's half 32 rows x 16
    // pieces; thread tid moves pieces tid and tid + 256 of each
    v4f pa[2], pb[2];
#define QT_F32L_FETCH(TT, HH)                                                                         \
    do {                                                                                              \
        const float* a_ = A + (size_t)prodA[TT] * (BS * BS);                                          \
        const float* b_ = B + (size_t)prodB[TT] * (BS * BS);                                          \
        _Pragma("unroll") for (int r = 0; r < 2; ++r) {                                               \
            const int pc = tid + 256 * r;                                                             \
            pa[r] = *reinterpret_cast<const v4f*>(a_ + (pc >> 3) * BS + (HH) * KH + (pc & 7) * 4);    \
            pb[r] = *reinterpret_cast<const v4f*>(b_ + ((HH) * KH + (pc >> 4)) * BS + (pc & 15) * 4); \
        }                                                                                             \
    } while (0)
    QT_F32L_FETCH(t0, 0);   // a segment holds at least one product
    for (int32_t t = t0; t < t1; ++t) {
#pragma unroll 1
        for (int h = 0; h < 2; ++h) {
            __syncthreads();   // every wave is done reading the previous half
#pragma unroll
            for (int r = 0; r < 2; ++r) {
                const int pc = tid + 256 * r;
                *reinterpret_cast<v4f*>(la + (pc >> 3) * F32L_AROW + (pc & 7) * 4) = pa[r];
                *reinterpret_cast<v4f*>(lb + (pc >> 4) * F32L_BROW + (pc & 15) * 4) = pb[r];
            }
            __syncthreads();
            if (h == 0)
                QT_F32L_FETCH(t, 1);
            else if (t + 1 < t1)
                QT_F32L_FETCH(t + 1, 0);
            // step ks gives lane group g the inner index k = 16 (ks / 4) + 4 g + ks % 4;
            // lane r16 holds columns 2 r16 (tile 0) and 2 r16 + 1 (tile 1)
            float ar[MT][8], br[MT][8];
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                for (int v = 0; v < 2; ++v) {
                    const v4f x = *reinterpret_cast<const v4f*>(la + (wm + mt * 16 + r16) * F32L_AROW + 16 * v + 4 * g);
#pragma unroll
                    for (int e = 0; e < 4; ++e) ar[mt][4 * v + e] = x[e];
                }
#pragma unroll
            for (int ks = 0; ks < 8; ++ks) {
                const v2f_t x = *reinterpret_cast<const v2f_t*>(
                    lb + (16 * (ks >> 2) + 4 * g + (ks & 3)) * F32L_BROW + wn + 2 * r16);
                br[0][ks] = x[0];
                br[1][ks] = x[1];
            }
#pragma unroll
            for (int ks = 0; ks < 8; ++ks)
#pragma unroll
                for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                    for (int nt = 0; nt < MT; ++nt)
                        acc[mt][nt] = Mfma<float>::step(ar[mt][ks], br[nt][ks], acc[mt][nt]);
        }
    }
#undef QT_F32L_FETCH
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const v2f_t v = {acc[mt][0][i], acc[mt][1][i]};
            __builtin_nontemporal_store(
                v, reinterpret_cast<v2f_t*>(c + (wm + mt * 16 + Mfma<float>::row(g, i)) * BS + wn + 2 * r16));
        }
}

__global__ __launch_bounds__(256) void k_numeric_f32_b64(const float* __restrict__ A, const float* __restrict__ B,
                                                         const int32_t* __restrict__ prodA,
                                                         const int32_t* __restrict__ prodB,
                                                         const int32_t* __restrict__ seg, int32_t nseg,
                                                         const int32_t* __restrict__ order, float* __restrict__ C) {
    const int64_t q = xcd_logical<8>(blockIdx.x);
    if (q >= nseg) return;   // uniform over the workgroup
    const int64_t s = order ? order[q] : q;
    lds_block_f32(A, B, prodA, prodB, seg[s], seg[s + 1], C + (size_t)s * (64 * 64));
}

template <class T, int BS>
static void launch_t(const NumericArgs& a, hipStream_t s) {
    if (sizeof(T) == 8 && BS == 64) {
        k_numeric_f64_b64<<<xcd_grid<8>(a.nseg), 256, 0, s>>>((const double*)a.A, (const double*)a.B, a.prodA,
                                                             a.prodB, a.seg, a.nseg, a.order, (double*)a.C);
        QT_LAUNCH("k_numeric_f64_b64");
        return;
    }
    if (sizeof(T) == 4 && BS == 64) {
        k_numeric_f32_b64<<<xcd_grid<8>(a.nseg), 256, 0, s>>>((const float*)a.A, (const float*)a.B, a.prodA,
                                                             a.prodB, a.seg, a.nseg, a.order, (float*)a.C);
        QT_LAUNCH("k_numeric_f32_b64");
        return;
    }
    typedef Geo<BS> G;
    const unsigned grid = xcd_grid<>((int64_t)a.nseg * G::WPB);
    if (a.by_k && a.order) {
        const size_t cap = occupancy_cap_lds(ByKCap<T, BS>::waves);
        k_numeric_byk<T, BS><<<grid, 64, cap, s>>>((const T*)a.A, (const T*)a.B, a.prodA, a.prodB, a.seg, a.nseg,
                                                   a.order, (T*)a.C);
        QT_LAUNCH("k_numeric_byk");
        return;
    }
    k_numeric<T, BS><<<grid, 64, 0, s>>>((const T*)a.A, (const T*)a.B, a.prodA, a.prodB, a.seg, a.nseg, a.order,
                                         (T*)a.C);
    QT_LAUNCH("k_numeric");
}

// b = 64 split-bf16 with the operands shared through LDS. One workgroup of
// four waves owns a 64 x 64 C block, wave w the 32 x 32 tile (w / 2, w % 2).
// Per block product the hi and lo parts of A and of B^T (8 KiB each) are
// staged in LDS once and each wave reads its 32-row panels from there, so a
// product moves 32 KiB from L2 instead of 64 KiB (two waves share every A
// panel and every B panel). Four workgroups share a CU (36 KiB of LDS each),
// so one workgroup's loads overlap the others' MFMAs. LDS rows are padded to 72
// elements (144 bytes) so the 16 lanes reading 16 consecutive rows hit
// distinct banks.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));   // a 16-byte piece, kept in VGPRs
constexpr int BFL_ROW = 72;
constexpr int BFL_ARR = 64 * BFL_ROW;      // elements per staged block

// One C block of the LDS-sharing kernel below, products t0 .. t1-1, into c
// (all four waves of the workgroup take part).
__device__ __forceinline__ void lds_block_bf16x3(const uint16_t* __restrict__ Ahi, const uint16_t* __restrict__ Alo, const uint16_t* __restrict__ Bhi_t, const uint16_t* __restrict__ Blo_t,
        const int32_t* __restrict__ prodA, const int32_t* __restrict__ prodB, int32_t t0, int32_t t1,
        double* __restrict__ c) {
    constexpr int BS = 64, MT = 2;
    __shared__ __attribute__((aligned(16))) uint16_t lds[4 * BFL_ARR];   // Ahi, Alo, Bhi^T, Blo^T
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int r16 = lane & 15, g = lane >> 4;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;

    // thread tid moves 16-byte pieces tid and tid + 256 of each 64 x 64 block:
    // piece q is row q / 8, elements 8 * (q % 8) .. + 7
    const uint16_t* const base4[4] = {Ahi, Alo, Bhi_t, Blo_t};
    u32x4 st0, st1, st2, st3, st4, st5, st6, st7;   // [block m][half h] = st(2m + h)
#define QT_BFL_FETCH(t)                                                                             \
    do {                                                                                            \
        const size_t oa_ = (size_t)prodA[t] * (BS * BS), ob_ = (size_t)prodB[t] * (BS * BS);        \
        st0 = *reinterpret_cast<const u32x4*>(base4[0] + oa_ + (size_t)tid * 8);                    \
        st1 = *reinterpret_cast<const u32x4*>(base4[0] + oa_ + (size_t)(tid + 256) * 8);            \
        st2 = *reinterpret_cast<const u32x4*>(base4[1] + oa_ + (size_t)tid * 8);                    \
        st3 = *reinterpret_cast<const u32x4*>(base4[1] + oa_ + (size_t)(tid + 256) * 8);            \
        st4 = *reinterpret_cast<const u32x4*>(base4[2] + ob_ + (size_t)tid * 8);                    \
        st5 = *reinterpret_cast<const u32x4*>(base4[2] + ob_ + (size_t)(tid + 256) * 8);            \
        st6 = *reinterpret_cast<const u32x4*>(base4[3] + ob_ + (size_t)tid * 8);                    \
        st7 = *reinterpret_cast<const u32x4*>(base4[3] + ob_ + (size_t)(tid + 256) * 8);            \
    } while (0)
    const int q0 = ((tid >> 3) * BFL_ROW + (tid & 7) * 8);                  // LDS offset of piece tid
    const int q1 = (((tid + 256) >> 3) * BFL_ROW + (tid & 7) * 8);          // and of piece tid + 256

    v4d acc[MT][MT];
#pragma unroll
    for (int i = 0; i < MT; ++i)
#pragma unroll
        for (int j = 0; j < MT; ++j) acc[i][j] = v4d{0, 0, 0, 0};

    for (int32_t t = t0; t < t1; ++t) {
        QT_BFL_FETCH(t);   // issued before the barrier: overlaps the other waves' previous product
        __syncthreads();   // every wave is done reading the previous product
        *reinterpret_cast<u32x4*>(lds + 0 * BFL_ARR + q0) = st0;
        *reinterpret_cast<u32x4*>(lds + 0 * BFL_ARR + q1) = st1;
        *reinterpret_cast<u32x4*>(lds + 1 * BFL_ARR + q0) = st2;
        *reinterpret_cast<u32x4*>(lds + 1 * BFL_ARR + q1) = st3;
        *reinterpret_cast<u32x4*>(lds + 2 * BFL_ARR + q0) = st4;
        *reinterpret_cast<u32x4*>(lds + 2 * BFL_ARR + q1) = st5;
        *reinterpret_cast<u32x4*>(lds + 3 * BFL_ARR + q0) = st6;
        *reinterpret_cast<u32x4*>(lds + 3 * BFL_ARR + q1) = st7;
        __syncthreads();
        v4f f[MT][MT];
#pragma unroll
        for (int i = 0; i < MT; ++i)
#pragma unroll
            for (int j = 0; j < MT; ++j) f[i][j] = v4f{0, 0, 0, 0};
#pragma unroll
        for (int kc = 0; kc < BS / 32; ++kc) {
            v8bf ah[MT], al[MT], bh[MT], bl[MT];
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) {
                const int o = (wm + mt * 16 + r16) * BFL_ROW + kc * 32 + g * 8;
                __builtin_memcpy(&ah[mt], lds + 0 * BFL_ARR + o, 16);
                __builtin_memcpy(&al[mt], lds + 1 * BFL_ARR + o, 16);
            }
#pragma unroll
            for (int nt = 0; nt < MT; ++nt) {
                const int o = (wn + nt * 16 + r16) * BFL_ROW + kc * 32 + g * 8;
                __builtin_memcpy(&bh[nt], lds + 2 * BFL_ARR + o, 16);
                __builtin_memcpy(&bl[nt], lds + 3 * BFL_ARR + o, 16);
            }
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                for (int nt = 0; nt < MT; ++nt) {
                    f[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[mt], bh[nt], f[mt][nt], 0, 0, 0);
                    f[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[mt], bl[nt], f[mt][nt], 0, 0, 0);
                    f[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[mt], bh[nt], f[mt][nt], 0, 0, 0);
                }
        }
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int nt = 0; nt < MT; ++nt)
#pragma unroll
                for (int i = 0; i < 4; ++i) acc[mt][nt][i] += (double)f[mt][nt][i];
    }
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int nt = 0; nt < MT; ++nt)
#pragma unroll
            for (int i = 0; i < 4; ++i)
                __builtin_nontemporal_store(acc[mt][nt][i], c + (wm + mt * 16 + 4 * g + i) * BS + wn + nt * 16 + r16);
#undef QT_BFL_FETCH
}

__global__ __launch_bounds__(256, 2) void k_numeric_bf16x3_b64(const uint16_t* __restrict__ Ahi,
                                                                const uint16_t* __restrict__ Alo,
                                                                const uint16_t* __restrict__ Bhi_t,
                                                                const uint16_t* __restrict__ Blo_t,
                                                                const int32_t* __restrict__ prodA,
                                                                const int32_t* __restrict__ prodB,
                                                                const int32_t* __restrict__ seg, int32_t nseg,
                                                                const int32_t* __restrict__ order,
                                                                double* __restrict__ C) {
    const int64_t q = xcd_logical<8>(blockIdx.x);
    if (q >= nseg) return;   // uniform over the workgroup
    const int64_t s = order ? order[q] : q;
    lds_block_bf16x3(Ahi, Alo, Bhi_t, Blo_t, prodA, prodB, seg[s], seg[s + 1], C + (size_t)s * (64 * 64));
}

template <int BS>
static void launch_bf(const NumericArgs& a, hipStream_t s) {
    if (BS == 64) {
        const unsigned grid = xcd_grid<8>(a.nseg);
        k_numeric_bf16x3_b64<<<grid, 256, 0, s>>>(a.Ahi, a.Alo, a.Bhi_t, a.Blo_t, a.prodA, a.prodB, a.seg,
                                                  a.nseg, a.order, (double*)a.C);
        QT_LAUNCH("k_numeric_bf16x3_b64");
        return;
    }
    constexpr int WPB = (BS / 32) * (BS / 32);
    const unsigned grid = xcd_grid<>((int64_t)a.nseg * WPB);
    k_numeric_bf16x3<BS><<<grid, 64, 0, s>>>(a.Ahi, a.Alo, a.Bhi_t, a.Blo_t, a.prodA, a.prodB, a.seg, a.nseg,
                                             a.order, (double*)a.C);
    QT_LAUNCH("k_numeric_bf16x3");
}

template <class T, int BS>
static void launch_op(const NumericArgs& a, hipStream_t s) {
    typedef Geo<BS> G;
    const unsigned grid = xcd_grid<>((int64_t)a.nseg * G::WPB);
    k_numeric_op<T, BS><<<grid, 64, 0, s>>>((const T*)a.A, (const T*)a.B, a.prodA, a.prodB, a.seg, a.nseg, a.order,
                                            (T*)a.C);
    QT_LAUNCH("k_numeric_op");
}

template <int BS>
static void launch_bf_op(const NumericArgs& a, hipStream_t s) {
    constexpr int WPB = (BS / 32) * (BS / 32);
    const SplitOps ops{a.Ahi, a.Alo, a.Ahi_t, a.Alo_t, a.Bhi, a.Blo, a.Bhi_t, a.Blo_t};
    const unsigned grid = xcd_grid<>((int64_t)a.nseg * WPB);
    k_numeric_bf16x3_op<BS><<<grid, 64, 0, s>>>(ops, a.prodA, a.prodB, a.seg, a.nseg, a.order, (double*)a.C);
    QT_LAUNCH("k_numeric_bf16x3_op");
}

void launch_numeric(const NumericArgs& a, hipStream_t s) {
    if (a.nseg <= 0) return;
    if (a.dyn) {
        if (a.prec == QT_F64) {
            switch (a.b) {
                case 16: return launch_op<double, 16>(a, s);
                case 32: return launch_op<double, 32>(a, s);
                case 64: return launch_op<double, 64>(a, s);
            }
        } else if (a.prec == QT_F32) {
            switch (a.b) {
                case 16: return launch_op<float, 16>(a, s);
                case 32: return launch_op<float, 32>(a, s);
                case 64: return launch_op<float, 64>(a, s);
            }
        } else if (a.prec == QT_BF16X3) {
            switch (a.b) {
                case 32: return launch_bf_op<32>(a, s);
                case 64: return launch_bf_op<64>(a, s);
            }
        }
        fail(QT_ERR_UNSUPPORTED, "no numeric kernel for this block size and precision");
    }
    if (a.prec == QT_F64) {
        switch (a.b) {
            case 16: return launch_t<double, 16>(a, s);
            case 32: return launch_t<double, 32>(a, s);
            case 64: return launch_t<double, 64>(a, s);
        }
    } else if (a.prec == QT_F32) {
        switch (a.b) {
            case 16: return launch_t<float, 16>(a, s);
            case 32: return launch_t<float, 32>(a, s);
            case 64: return launch_t<float, 64>(a, s);
        }
    } else if (a.prec == QT_BF16X3) {
        switch (a.b) {
            case 32: return launch_bf<32>(a, s);
            case 64: return launch_bf<64>(a, s);
        }
    }
    fail(QT_ERR_UNSUPPORTED, "no numeric kernel for this block size and precision");
}

// ------------------------------------------------- a batch of multiplies
//
// Work item i of the batch is one wave's tile of one C block (or, for the
// b = 64 kernels that share operands through LDS, one C block and its
// four-wave workgroup). Problem p owns items item_base[p] .. item_base[p+1]-1:
// its C blocks in its launch order (Morton order, or grouped by inner index
// where C blocks average under two block products), WPB tiles each. Problems
// come largest first. Four schedules:
//   flat:          one launch whose grid covers every item, one workgroup per
//                  item in the XCD-run order above; the hardware dispatcher
//                  balances the uneven problems;
//   balanced:      a persistent grid of as many workgroups as fit on the GPU
//                  at once; each takes a contiguous run of items holding an
//                  equal share of the work (block products plus one per C
//                  block, summed at plan creation), so no counter, no
//                  dispatch per item and no tail of long items on few waves;
//   xcd-dynamic:   a persistent grid whose workgroups take 2 items at a time
//                  from a counter per XCD, over the flat grid's XCD runs;
//   dynamic-16:    a persistent grid that takes 16 items at a time from one
//                  counter until none are left.
// Every schedule ends: a balanced workgroup after its run, a dynamic one at
// its first grab past the end.

// A problem's arrays are addressed from the launch's base pointer, a kernel
// argument: a pointer read out of memory would be a generic pointer to the
// compiler, which then addresses every operand load and C store through the
// flat address space (flat loads count against both wait counters, and a
// wait for the next operands becomes a wait for all memory traffic, the
// previous block's C stores included).
template <class T>
__device__ __forceinline__ T* at(const char* base, int64_t off) {
    return (T*)(base + off);
}

template <int WPB>
__device__ __forceinline__ int32_t batch_problem(const int64_t* __restrict__ item_base, int32_t nprob, int64_t it) {
    int32_t lo = 0, hi = nprob - 1;                  // last p with item_base[p] <= it
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (item_base[mid] <= it)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

template <class T, int BS, bool BUF>
__device__ __forceinline__ void batch_item(const BatchProblem* __restrict__ probs, const char* __restrict__ base,
                                           const int64_t* __restrict__ item_base, int32_t nprob, int64_t it) {
    constexpr int WPB = Geo<BS>::WPB;
    const int32_t p = batch_problem<WPB>(item_base, nprob, it);
    const BatchProblem& P = probs[p];
    const int64_t local = it - item_base[p];
    const int64_t q = local / WPB;
    const int sub = (int)(local - q * WPB);
    const int32_t* prodA = at<const int32_t>(base, P.prodA);
    const int32_t* prodB = at<const int32_t>(base, P.prodB);
    const int32_t* seg = at<const int32_t>(base, P.seg);
    const int64_t s = P.order >= 0 ? at<const int32_t>(base, P.order)[q] : q;
    const int32_t t0 = seg[s];
    wave_block<T, BS, BUF>(at<const T>(base, P.A), at<const T>(base, P.B), prodA, prodB, t0, seg[s + 1],
                           at<T>(base, P.C) + (size_t)s * (BS * BS), sub, prodA[t0], prodB[t0]);
}

template <int BS>
__device__ __forceinline__ void batch_item_bf16x3(const BatchProblem* __restrict__ probs,
                                                  const char* __restrict__ base,
                                                  const int64_t* __restrict__ item_base, int32_t nprob,
                                                  int64_t it) {
    constexpr int WPB = (BS / 32) * (BS / 32);
    const int32_t p = batch_problem<WPB>(item_base, nprob, it);
    const BatchProblem& P = probs[p];
    const int64_t local = it - item_base[p];
    const int64_t q = local / WPB;
    const int sub = (int)(local - q * WPB);
    const int32_t* seg = at<const int32_t>(base, P.seg);
    const int64_t s = P.order >= 0 ? at<const int32_t>(base, P.order)[q] : q;
    wave_block_bf16x3<BS>(at<const uint16_t>(base, P.Ahi), at<const uint16_t>(base, P.Alo),
                          at<const uint16_t>(base, P.Bhi_t), at<const uint16_t>(base, P.Blo_t),
                          at<const int32_t>(base, P.prodA), at<const int32_t>(base, P.prodB), seg[s], seg[s + 1],
                          at<double>(base, P.C) + (size_t)s * (BS * BS), sub);
}

// one C block of a b = 64 problem by a whole four-wave workgroup (LDS sharing)
template <int KIND>
__device__ __forceinline__ void batch_item_lds(const BatchProblem* __restrict__ probs, const char* __restrict__ base,
                                               const int64_t* __restrict__ item_base, int32_t nprob, int64_t it) {
    const int32_t p = batch_problem<1>(item_base, nprob, it);
    const BatchProblem& P = probs[p];
    const int64_t q = it - item_base[p];
    const int32_t* seg = at<const int32_t>(base, P.seg);
    const int32_t* prodA = at<const int32_t>(base, P.prodA);
    const int32_t* prodB = at<const int32_t>(base, P.prodB);
    const int64_t s = P.order >= 0 ? at<const int32_t>(base, P.order)[q] : q;
    const int32_t t0 = seg[s], t1 = seg[s + 1];
    if constexpr (KIND == 0)
        lds_block_f64(at<const double>(base, P.A), at<const double>(base, P.B), prodA, prodB, t0, t1,
                      at<double>(base, P.C) + (size_t)s * (64 * 64));
    else if constexpr (KIND == 1)
        lds_block_f32(at<const float>(base, P.A), at<const float>(base, P.B), prodA, prodB, t0, t1,
                      at<float>(base, P.C) + (size_t)s * (64 * 64));
    else
        lds_block_bf16x3(at<const uint16_t>(base, P.Ahi), at<const uint16_t>(base, P.Alo),
                         at<const uint16_t>(base, P.Bhi_t), at<const uint16_t>(base, P.Blo_t), prodA, prodB, t0,
                         t1, at<double>(base, P.C) + (size_t)s * (64 * 64));
}

// Item dispatch for one (precision, block size, LDS sharing) instance; the
// LDS instances exist at b = 64 only and run 256-thread workgroups. BUF: the
// per-wave fp64 / fp32 tiles write C through buffer stores (the flat grid:
// batch64 FP32 6.60 instead of 6.91 ms, FP64 unchanged; the persistent
// schedules are slower with them).
template <int KIND, int BS, bool LDS> struct Item {
    static constexpr int THREADS = LDS ? 256 : 64;
    template <bool BUF = false>
    static __device__ __forceinline__ void run(const BatchProblem* p, const char* base, const int64_t* ib, int32_t n,
                                               int64_t it) {
        if constexpr (LDS)
            batch_item_lds<KIND>(p, base, ib, n, it);
        else if constexpr (KIND == 0)
            batch_item<double, BS, BUF>(p, base, ib, n, it);
        else if constexpr (KIND == 1)
            batch_item<float, BS, BUF>(p, base, ib, n, it);
        else
            batch_item_bf16x3<BS>(p, base, ib, n, it);
    }
};

template <int KIND, int BS, bool LDS>
__global__ __launch_bounds__(LDS ? 256 : 64) void k_batch_flat(const BatchProblem* __restrict__ probs,
                                                                 const char* __restrict__ base,
                                                                 const int64_t* __restrict__ item_base,
                                                                 int32_t nprob) {
    const int64_t it = LDS ? xcd_logical<8>(blockIdx.x) : xcd_logical<>(blockIdx.x);
    if (it >= item_base[nprob]) return;
    Item<KIND, BS, LDS>::template run<true>(probs, base, item_base, nprob, it);
}

// Work of every item, for the balanced schedule: the block products of its
// C block plus one (the C block's own store and set-up).
template <bool LDS>
__global__ void k_batch_item_cost(const BatchProblem* __restrict__ probs, const char* __restrict__ base,
                                  const int64_t* __restrict__ item_base, int32_t nprob, int wpb,
                                  int64_t* __restrict__ cost) {
    const int64_t it = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (it >= item_base[nprob]) return;
    int32_t lo = 0, hi = nprob - 1;
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (item_base[mid] <= it)
            lo = mid;
        else
            hi = mid - 1;
    }
    const BatchProblem& P = probs[lo];
    const int64_t q = (it - item_base[lo]) / wpb;
    const int32_t* seg = at<const int32_t>(base, P.seg);
    const int64_t s = P.order >= 0 ? at<const int32_t>(base, P.order)[q] : q;
    cost[it] = (int64_t)(seg[s + 1] - seg[s]) + 1;
}

// first i in [0, n] with cum[i] >= v (cum ascending, cum[0] = 0)
__device__ __forceinline__ int64_t lower_bound64(const int64_t* __restrict__ cum, int64_t n, int64_t v) {
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (cum[mid] < v)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

// Balanced schedule: workgroup r of the grid takes the items whose work
// starts in [r W / G, (r + 1) W / G), W the batch's total work (cum[n]) --
// a contiguous run, so neighbouring C blocks (and their operands) stay with
// one wave.
template <int KIND, int BS, bool LDS>
__global__ __launch_bounds__(LDS ? 256 : 64) void k_batch_balanced(
    const BatchProblem* __restrict__ probs, const char* __restrict__ base, const int64_t* __restrict__ item_base,
    int32_t nprob, const int64_t* __restrict__ cum) {
    const int64_t n = item_base[nprob];
    const int64_t g = gridDim.x, r = blockIdx.x;
    const int64_t W = cum[n];
    const int64_t i0 = lower_bound64(cum, n, W * r / g);
    const int64_t i1 = lower_bound64(cum, n, W * (r + 1) / g);
    for (int64_t it = i0; it < i1; ++it) Item<KIND, BS, LDS>::run(probs, base, item_base, nprob, it);
}

// Per-XCD dynamic schedule: workgroup w is counted to XCD x = w % 8 and takes
// XCD_GRAB consecutive positions at a time from that XCD's counter; XCD x's
// positions are its runs of items x, x + 8, x + 16, ... (as the flat grid's
// launch order gives them), so the workgroups of an XCD share a window of
// neighbouring items in its L2 while each takes the next work as it gets
// free. The next grab is taken while the current items run. Every item is
// taken exactly once wherever a workgroup really runs (the counters are
// device-wide atomics); a workgroup leaves at its first position past the end.
constexpr int XCD_GRAB = 2;

template <int KIND, int BS, bool LDS>
__global__ __launch_bounds__(LDS ? 256 : 64) void k_batch_xcd(
    const BatchProblem* __restrict__ probs, const char* __restrict__ base, const int64_t* __restrict__ item_base,
    int32_t nprob, unsigned long long* __restrict__ counters) {
    constexpr int LOG = LDS ? 8 : XCD_CHUNK_LOG;
    __shared__ unsigned long long grab[2];
    const int64_t total = item_base[nprob];
    const int64_t x = blockIdx.x & 7;
    unsigned long long* my = counters + 8 * x;   // 64 bytes apart
    if (threadIdx.x == 0) grab[0] = atomicAdd(my, (unsigned long long)XCD_GRAB);
    __syncthreads();
    for (int k = 0;; k ^= 1) {
        const int64_t first = (int64_t)grab[k];
        if (threadIdx.x == 0) grab[k ^ 1] = atomicAdd(my, (unsigned long long)XCD_GRAB);   // the next grab
        bool done = false;
        for (int64_t pos = first; pos < first + XCD_GRAB; ++pos) {
            const int64_t it = ((((pos >> LOG) << 3) + x) << LOG) | (pos & ((int64_t(1) << LOG) - 1));
            if (it >= total) {   // positions map to increasing items: all later ones are past the end too
                done = true;
                break;
            }
            Item<KIND, BS, LDS>::run(probs, base, item_base, nprob, it);
        }
        __syncthreads();   // the next grab is in place, and every wave has read the current one
        if (done) break;
    }
}

template <int KIND, int BS, bool LDS, int CHUNK>
__global__ __launch_bounds__(LDS ? 256 : 64) void k_batch_persistent(
    const BatchProblem* __restrict__ probs, const char* __restrict__ base, const int64_t* __restrict__ item_base,
    int32_t nprob, unsigned long long* __restrict__ counter) {
    __shared__ unsigned long long grab;
    const int64_t total = item_base[nprob];
    while (true) {
        if (threadIdx.x == 0) grab = atomicAdd(counter, (unsigned long long)CHUNK);
        __syncthreads();
        const int64_t first = (int64_t)grab;
        __syncthreads();   // every wave has read grab before the next one is written
        if (first >= total) break;
        const int64_t end = min(first + CHUNK, total);
        for (int64_t it = first; it < end; ++it) Item<KIND, BS, LDS>::run(probs, base, item_base, nprob, it);
    }
}

// Clears the work counters (a kernel rather than a memset, so the launch
// sequence can be captured into a graph and replayed).
__global__ void k_batch_reset(unsigned long long* counter, int n) {
    if ((int)threadIdx.x < n) counter[threadIdx.x] = 0ull;
}

// Workgroups that fit on the GPU at once for a persistent kernel (a multiple of 8).
static int resident_grid(const void* kernel, int threads) {
    static std::mutex mu;
    static std::map<std::pair<const void*, int>, int> cache;
    int dev = 0;
    QT_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find({kernel, dev});
    if (it != cache.end()) return it->second;
    int cus = 0, per_cu = 0;
    QT_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    QT_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0));
    const int g = std::max(8, (cus * std::max(1, per_cu)) / 8 * 8);
    cache[{kernel, dev}] = g;
    return g;
}

template <int KIND, int BS, bool LDS>
static void launch_batch_k(const BatchLaunch& L, hipStream_t s) {
    constexpr int T = Item<KIND, BS, LDS>::THREADS;
    const int64_t items = L.total_items;
    if (L.schedule == 0) {
        const unsigned grid = LDS ? xcd_grid<8>(items) : xcd_grid<>(items);
        k_batch_flat<KIND, BS, LDS><<<grid, T, 0, s>>>(L.probs, L.base, L.item_base, L.nprob);
        QT_LAUNCH("k_batch_flat");
        return;
    }
    if (L.schedule == 1) {
        // every workgroup resident at once (a multiple of 8), at most one per item
        const int64_t res = resident_grid((const void*)k_batch_balanced<KIND, BS, LDS>, T);
        const unsigned g = (unsigned)std::max<int64_t>(8, std::min<int64_t>(res, (items + 7) / 8 * 8));
        k_batch_balanced<KIND, BS, LDS><<<g, T, 0, s>>>(L.probs, L.base, L.item_base, L.nprob, L.cum);
        QT_LAUNCH("k_batch_balanced");
        return;
    }
    if (L.schedule == 2) {
        k_batch_reset<<<1, 64, 0, s>>>(L.counter, 64);
        QT_LAUNCH("k_batch_reset");
        const unsigned g = (unsigned)resident_grid((const void*)k_batch_xcd<KIND, BS, LDS>, T);
        k_batch_xcd<KIND, BS, LDS><<<g, T, 0, s>>>(L.probs, L.base, L.item_base, L.nprob, L.counter);
        QT_LAUNCH("k_batch_xcd");
        return;
    }
    k_batch_reset<<<1, 64, 0, s>>>(L.counter, 1);
    QT_LAUNCH("k_batch_reset");
    const unsigned g = (unsigned)resident_grid((const void*)k_batch_persistent<KIND, BS, LDS, 16>, T);
    k_batch_persistent<KIND, BS, LDS, 16><<<g, T, 0, s>>>(L.probs, L.base, L.item_base, L.nprob, L.counter);
    QT_LAUNCH("k_batch_persistent");
}

void batch_item_costs(const BatchLaunch& L, int64_t* cost, hipStream_t s) {
    if (L.total_items <= 0) return;
    const int wpb = (L.b == 64 && !L.lds) ? 4 : 1;
    const unsigned g = (unsigned)((L.total_items + 255) / 256);
    if (L.lds)
        k_batch_item_cost<true><<<g, 256, 0, s>>>(L.probs, L.base, L.item_base, L.nprob, wpb, cost);
    else
        k_batch_item_cost<false><<<g, 256, 0, s>>>(L.probs, L.base, L.item_base, L.nprob, wpb, cost);
    QT_LAUNCH("k_batch_item_cost");
}

void launch_batch(const BatchLaunch& L, hipStream_t s) {
    if (L.total_items <= 0) return;
    if (L.schedule < 0 || L.schedule >= kBatchSchedules) fail(QT_ERR_ARG, "unknown batch schedule");
    const int kind = (L.prec == QT_F64) ? 0 : (L.prec == QT_F32) ? 1 : 2;
    const int b = L.b;
    if (L.lds && b != 64) fail(QT_ERR_ARG, "LDS-sharing batch kernels need b = 64");
    if (L.lds) {
        if (kind == 0) return launch_batch_k<0, 64, true>(L, s);
        if (kind == 1) return launch_batch_k<1, 64, true>(L, s);
        return launch_batch_k<2, 64, true>(L, s);
    }
    if (kind == 0 && b == 16) return launch_batch_k<0, 16, false>(L, s);
    if (kind == 0 && b == 32) return launch_batch_k<0, 32, false>(L, s);
    if (kind == 0 && b == 64) return launch_batch_k<0, 64, false>(L, s);
    if (kind == 1 && b == 16) return launch_batch_k<1, 16, false>(L, s);
    if (kind == 1 && b == 32) return launch_batch_k<1, 32, false>(L, s);
    if (kind == 1 && b == 64) return launch_batch_k<1, 64, false>(L, s);
    if (kind == 2 && b == 32) return launch_batch_k<2, 32, false>(L, s);
    if (kind == 2 && b == 64) return launch_batch_k<2, 64, false>(L, s);
    fail(QT_ERR_UNSUPPORTED, "no batch kernel for this block size and precision");
}

}  // namespace qt
