// Numeric phase: C_s = sum over the products t of segment s (k ascending) of
// A[prodA[t]] * B[prodB[t]], one b x b block per segment, on gfx950 MFMA.
//
// This replaces the paper's leaf library, which ran every outer product
// batch of a leaf through a batched GEMM (Sec. 4.1, Fig. 2) and accumulated
// into C in memory. Here one wavefront owns a 32 x 32 (or 16 x 16) tile of a
// C block for the whole segment: the tile stays in MFMA accumulators across
// all its block products and is stored once, so C is never re-read and no
// two waves ever write the same C entry (no atomics).
//
// MFMA operand layout (16 x 16 x 4 for fp64/fp32): lane l = 16*g + r supplies
// A[r][kk = g] and B[kk = g][r] of one 4-deep step; its four accumulator
// values are D[4*g + i][r] (i = 0..3) for fp32, but D[4*i + g][r] for fp64
// (the fp64 instruction interleaves the row groups; checked on gfx950 with a
// known-input product). The inner index is a free summation variable, which
// lets each lane read its A entries with 16-byte loads (see k_numeric), while
// the 16 lanes of a group read 16 consecutive entries of one B row.
#include "qt_internal.h"

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
// MT x MT 16x16 MFMA tiles; WPB waves cover one C block; a 256-thread
// workgroup covers SPW segments; the inner dimension is walked in chunks of
// KC with KS 4-deep MFMA steps each.
template <int BS> struct Geo {
    static constexpr int WT = BS < 32 ? BS : 32;
    static constexpr int MT = WT / 16;
    static constexpr int WPB = (BS / WT) * (BS / WT);
    static constexpr int SPW = 4 / WPB;
    static constexpr int KC = BS < 32 ? BS : 32;
    static constexpr int KS = KC / 4;
    static constexpr int NCH = BS / KC;
};

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own
// L2). Remap the hardware workgroup id so that every XCD works through one
// contiguous run of C blocks: neighbouring C blocks in Morton order share
// A block rows and B block columns, which then stay in that XCD's L2.
__device__ __forceinline__ int64_t xcd_remap(int64_t w, int64_t G) {
    const int64_t q = G >> 3, r = G & 7;
    const int64_t x = w & 7, i = w >> 3;
    return x * q + (x < r ? x : r) + i;
}

template <class T, int BS>
__global__ __launch_bounds__(256, 2) void k_numeric(const T* __restrict__ A, const T* __restrict__ B,
                                                 const int32_t* __restrict__ prodA,
                                                 const int32_t* __restrict__ prodB,
                                                 const int32_t* __restrict__ seg, int32_t nseg,
                                                 T* __restrict__ C) {
    typedef Geo<BS> G;
    typedef typename Mfma<T>::acc acc_t;
    constexpr int VEC = 16 / sizeof(T);            // elements per 16-byte load
    constexpr int NV = G::KS / VEC;                // 16-byte loads per A row per chunk
    typedef T vec_t __attribute__((ext_vector_type(VEC)));
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int r16 = lane & 15;
    const int g = lane >> 4;
    const int sub = wave % G::WPB;
    const int64_t wg = xcd_remap(blockIdx.x, gridDim.x);
    const int64_t s = wg * G::SPW + wave / G::WPB;
    if (s >= nseg) return;
    const int wm = (sub / (BS / G::WT)) * G::WT;
    const int wn = (sub % (BS / G::WT)) * G::WT;

    // Step ks of a chunk gives lane group g the inner index
    //   k = (ks / VEC) * 4*VEC + g*VEC + ks % VEC,
    // so each 16-byte A load of a lane is VEC consecutive entries of its row
    // and the four lane groups together read one contiguous run per row.
    struct Ops {
        T a[G::MT][G::KS];
        T b[G::MT][G::KS];
    };
    auto load = [&](Ops& o, const T* __restrict__ a, const T* __restrict__ b, int ch) {
#pragma unroll
        for (int mt = 0; mt < G::MT; ++mt) {
            const T* row = a + (wm + mt * 16 + r16) * BS + ch * G::KC + g * VEC;
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                const vec_t x = *reinterpret_cast<const vec_t*>(row + v * 4 * VEC);
#pragma unroll
                for (int e = 0; e < VEC; ++e) o.a[mt][v * VEC + e] = x[e];
            }
        }
#pragma unroll
        for (int nt = 0; nt < G::MT; ++nt)
#pragma unroll
            for (int v = 0; v < NV; ++v)
#pragma unroll
                for (int e = 0; e < VEC; ++e)
                    o.b[nt][v * VEC + e] = b[(ch * G::KC + v * 4 * VEC + g * VEC + e) * BS + wn + nt * 16 + r16];
    };
    acc_t acc[G::MT][G::MT];
#pragma unroll
    for (int i = 0; i < G::MT; ++i)
#pragma unroll
        for (int j = 0; j < G::MT; ++j) acc[i][j] = acc_t{0, 0, 0, 0};
    auto compute = [&](const Ops& o) {
#pragma unroll
        for (int ks = 0; ks < G::KS; ++ks)
#pragma unroll
            for (int mt = 0; mt < G::MT; ++mt)
#pragma unroll
                for (int nt = 0; nt < G::MT; ++nt)
                    acc[mt][nt] = Mfma<T>::step(o.a[mt][ks], o.b[nt][ks], acc[mt][nt]);
    };

    // Software pipeline over stages (product t, chunk ch): the operands of
    // the next stage are loaded while the MFMAs of this one run; block
    // indices are fetched one product further ahead.
    const int32_t t0 = seg[s], t1 = seg[s + 1];
    const int32_t nstages = (t1 - t0) * G::NCH;
    int32_t tl = t0;
    int chl = 0;
    int32_t ia = prodA[t0], ib = prodB[t0];
    int32_t ia_n = (t0 + 1 < t1) ? prodA[t0 + 1] : 0, ib_n = (t0 + 1 < t1) ? prodB[t0 + 1] : 0;
    auto issue = [&](Ops& o) {
        load(o, A + (size_t)ia * (BS * BS), B + (size_t)ib * (BS * BS), chl);
        if (++chl == G::NCH) {
            chl = 0;
            ++tl;
            ia = ia_n;
            ib = ib_n;
            if (tl + 1 < t1) {
                ia_n = prodA[tl + 1];
                ib_n = prodB[tl + 1];
            }
        }
    };
    Ops o0, o1;
    issue(o0);
    for (int32_t u = 0; u < nstages; u += 2) {
        if (u + 1 < nstages) issue(o1);
        compute(o0);
        if (u + 1 >= nstages) break;
        if (u + 2 < nstages) issue(o0);
        compute(o1);
    }
    T* c = C + (size_t)s * (BS * BS);
#pragma unroll
    for (int mt = 0; mt < G::MT; ++mt)
#pragma unroll
        for (int nt = 0; nt < G::MT; ++nt)
#pragma unroll
            for (int i = 0; i < 4; ++i)
                c[(wm + mt * 16 + Mfma<T>::row(g, i)) * BS + wn + nt * 16 + r16] = acc[mt][nt][i];
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

template <int BS>
__global__ __launch_bounds__(256) void k_numeric_bf16x3(const uint16_t* __restrict__ Ahi,
                                                        const uint16_t* __restrict__ Alo,
                                                        const uint16_t* __restrict__ Bhi_t,
                                                        const uint16_t* __restrict__ Blo_t,
                                                        const int32_t* __restrict__ prodA,
                                                        const int32_t* __restrict__ prodB,
                                                        const int32_t* __restrict__ seg, int32_t nseg,
                                                        double* __restrict__ C) {
    static_assert(BS == 32 || BS == 64, "split-bf16 path needs b = 32 or 64");
    constexpr int WT = 32, MT = 2;
    constexpr int WPB = (BS / WT) * (BS / WT);
    constexpr int SPW = 4 / WPB;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int r16 = lane & 15;
    const int g = lane >> 4;
    const int sub = wave % WPB;
    const int64_t s = xcd_remap(blockIdx.x, gridDim.x) * SPW + wave / WPB;
    if (s >= nseg) return;
    const int wm = (sub / (BS / WT)) * WT;
    const int wn = (sub % (BS / WT)) * WT;

    v4d acc[MT][MT];
#pragma unroll
    for (int i = 0; i < MT; ++i)
#pragma unroll
        for (int j = 0; j < MT; ++j) acc[i][j] = v4d{0, 0, 0, 0};

    const int32_t t0 = seg[s], t1 = seg[s + 1];
    for (int32_t t = t0; t < t1; ++t) {
        const size_t oa = (size_t)prodA[t] * (BS * BS);
        const size_t ob = (size_t)prodB[t] * (BS * BS);
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
    double* c = C + (size_t)s * (BS * BS);
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int nt = 0; nt < MT; ++nt)
#pragma unroll
            for (int i = 0; i < 4; ++i)
                c[(wm + mt * 16 + 4 * g + i) * BS + wn + nt * 16 + r16] = acc[mt][nt][i];
}

template <class T, int BS>
static void launch_t(const NumericArgs& a, hipStream_t s) {
    typedef Geo<BS> G;
    const unsigned grid = (unsigned)((a.nseg + G::SPW - 1) / G::SPW);
    k_numeric<T, BS><<<grid, 256, 0, s>>>((const T*)a.A, (const T*)a.B, a.prodA, a.prodB, a.seg, a.nseg,
                                          (T*)a.C);
    QT_LAUNCH("k_numeric");
}

template <int BS>
static void launch_bf(const NumericArgs& a, hipStream_t s) {
    constexpr int SPW = 4 / ((BS / 32) * (BS / 32));
    const unsigned grid = (unsigned)((a.nseg + SPW - 1) / SPW);
    k_numeric_bf16x3<BS><<<grid, 256, 0, s>>>(a.Ahi, a.Alo, a.Bhi_t, a.Blo_t, a.prodA, a.prodB, a.seg, a.nseg,
                                              (double*)a.C);
    QT_LAUNCH("k_numeric_bf16x3");
}

void launch_numeric(const NumericArgs& a, hipStream_t s) {
    if (a.nseg <= 0) return;
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

}  // namespace qt
