// Attainable MFMA rate of this GPU: a register-only loop of the same MFMA
// instruction each numeric path issues (fp64 16x16x4, fp32 16x16x4, bf16
// 16x16x32), eight independent accumulator chains per wave, enough waves to
// fill every SIMD several times over. No memory traffic inside the loop, so
// the rate it reaches is the ceiling the block GEMMs can approach, to be read
// beside the published peak.
//
// Also the batched-GEMM benchmark of the paper's practical peak figures
// (Sec. 6.1, Table 2): `count` independent block products C_i = A B, one
// pair of b x b operands reused by all, each C_i its own block, run through
// the multiply's own numeric kernels (one C block per product, as in a
// multiply whose C blocks each have one block product).
#include "qt_internal.h"

namespace qt {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

constexpr int PROBE_CHAINS = 8;

template <int KIND> struct ProbeOp;
template <> struct ProbeOp<0> {   // fp64 16x16x4: 2*16*16*4 flops
    typedef v4d acc;
    static constexpr double flops = 2048.0;
    static __device__ __forceinline__ acc step(acc c, float seed) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64((double)seed, 0.5, c, 0, 0, 0);
    }
};
template <> struct ProbeOp<1> {   // fp32 16x16x4
    typedef v4f acc;
    static constexpr double flops = 2048.0;
    static __device__ __forceinline__ acc step(acc c, float seed) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(seed, 0.5f, c, 0, 0, 0);
    }
};
template <> struct ProbeOp<2> {   // bf16 16x16x32: 2*16*16*32 flops
    typedef v4f acc;
    static constexpr double flops = 16384.0;
    static __device__ __forceinline__ acc step(acc c, float seed) {
        v8bf a;
        for (int e = 0; e < 8; ++e) a[e] = (__bf16)(seed + e);
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, a, c, 0, 0, 0);
    }
};

template <int KIND>
__global__ __launch_bounds__(256) void k_probe(float* out, int iters, float seed) {
    typedef typename ProbeOp<KIND>::acc acc_t;
    acc_t acc[PROBE_CHAINS];
#pragma unroll
    for (int c = 0; c < PROBE_CHAINS; ++c) acc[c] = acc_t{0, 0, 0, 0};
    const float s = seed + 1e-7f * threadIdx.x;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int c = 0; c < PROBE_CHAINS; ++c) acc[c] = ProbeOp<KIND>::step(acc[c], s);
    }
    float r = 0;
#pragma unroll
    for (int c = 0; c < PROBE_CHAINS; ++c) r += (float)(acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3]);
    out[(size_t)blockIdx.x * 256 + threadIdx.x] = r;   // keeps the loop live
}

template <int KIND>
static double probe_kind(hipStream_t s) {
    int dev = 0, cus = 0;
    QT_HIP(hipGetDevice(&dev));
    QT_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    const int wgs = cus * 8;   // 8 workgroups of 4 waves per CU: 8 waves per SIMD
    const int iters = (KIND == 2) ? 2048 : 4096;
    DBuf<float> out((size_t)wgs * 256, s);
    hipEvent_t e0, e1;
    timing_event(&e0);
    timing_event(&e1);
    float best = 0;
    for (int rep = 0; rep < 3; ++rep) {   // the first run also warms the clocks
        QT_HIP(hipEventRecord(e0, s));
        k_probe<KIND><<<wgs, 256, 0, s>>>(out.p, iters, 1.0f);
        QT_HIP(hipEventRecord(e1, s));
        QT_HIP(hipEventSynchronize(e1));
        float ms = 0;
        QT_HIP(hipEventElapsedTime(&ms, e0, e1));
        if (rep > 0 && (best == 0 || ms < best)) best = ms;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    const double flops = ProbeOp<KIND>::flops * PROBE_CHAINS * (double)iters * wgs * 4.0;
    return flops / (best * 1e-3) / 1e12;
}

__global__ void k_probe_fill(double* v, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) v[i] = 0.5 + 1e-3 * (double)(i % 97);
}
__global__ void k_probe_fill32(float* v, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) v[i] = 0.5f + 1e-3f * (float)(i % 97);
}
__global__ void k_probe_fill16(uint16_t* v, int64_t n, uint16_t x) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) v[i] = x;
}
__global__ void k_probe_iota(int32_t* seg, int32_t* zeros, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i <= n) seg[i] = (int32_t)i;
    if (i < n) zeros[i] = 0;
}

double probe_batched(qt_prec prec, int b, int64_t count, hipStream_t s) {
    if (prec != QT_F64 && prec != QT_F32 && prec != QT_BF16X3) fail(QT_ERR_ARG, "unknown precision");
    if (b != 16 && b != 32 && b != 64) fail(QT_ERR_SHAPE, "block size must be 16, 32 or 64");
    if (prec == QT_BF16X3 && b == 16) fail(QT_ERR_UNSUPPORTED, "split-bf16 path needs b = 32 or 64");
    if (count < 1 || count > (int64_t(1) << 24)) fail(QT_ERR_ARG, "count must be in 1 .. 2^24");
    const int64_t bb = (int64_t)b * b;
    const unsigned T = 256;
    auto grid = [&](int64_t n) { return (unsigned)((n + T - 1) / T); };
    DBuf<int32_t> seg(count + 1, s), zero(count, s);
    k_probe_iota<<<grid(count + 1), T, 0, s>>>(seg.p, zero.p, count);
    QT_LAUNCH("k_probe_iota");
    NumericArgs na{};
    na.b = b;
    na.prec = prec;
    na.prodA = zero.p;   // every product reads operand block 0 of A and of B
    na.prodB = zero.p;
    na.seg = seg.p;
    na.nseg = (int32_t)count;
    DBuf<double> a64, b64, c64;
    DBuf<float> a32, b32, c32;
    DBuf<uint16_t> split;
    if (prec == QT_F32) {
        a32.alloc(bb, s);
        b32.alloc(bb, s);
        c32.alloc(count * bb, s);
        k_probe_fill32<<<grid(bb), T, 0, s>>>(a32.p, bb);
        k_probe_fill32<<<grid(bb), T, 0, s>>>(b32.p, bb);
        QT_LAUNCH("k_probe_fill32");
        na.A = a32.p;
        na.B = b32.p;
        na.C = c32.p;
    } else {
        c64.alloc(count * bb, s);
        na.C = c64.p;
        if (prec == QT_F64) {
            a64.alloc(bb, s);
            b64.alloc(bb, s);
            k_probe_fill<<<grid(bb), T, 0, s>>>(a64.p, bb);
            k_probe_fill<<<grid(bb), T, 0, s>>>(b64.p, bb);
            QT_LAUNCH("k_probe_fill");
            na.A = a64.p;
            na.B = b64.p;
        } else {
            // hi parts 0.5 (bf16 0x3f00), lo parts 0.25 (0x3e80): the operands' values
            // do not change the MFMA time
            split.alloc(4 * bb, s);
            k_probe_fill16<<<grid(2 * bb), T, 0, s>>>(split.p, 2 * bb, (uint16_t)0x3f00);
            k_probe_fill16<<<grid(2 * bb), T, 0, s>>>(split.p + 2 * bb, 2 * bb, (uint16_t)0x3e80);
            QT_LAUNCH("k_probe_fill16");
            na.Ahi = split.p;
            na.Bhi_t = split.p + bb;
            na.Alo = split.p + 2 * bb;
            na.Blo_t = split.p + 3 * bb;
        }
    }
    hipEvent_t e0, e1;
    timing_event(&e0);
    timing_event(&e1);
    constexpr int kReps = 10;
    launch_numeric(na, s);   // warm-up
    QT_HIP(hipEventRecord(e0, s));
    for (int r = 0; r < kReps; ++r) launch_numeric(na, s);
    QT_HIP(hipEventRecord(e1, s));
    QT_HIP(hipEventSynchronize(e1));
    float ms = 0;
    QT_HIP(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return 2.0 * (double)bb * b * (double)count * kReps / (ms * 1e-3) / 1e12;
}

double probe_mfma(qt_prec prec, hipStream_t s) {
    switch (prec) {
        case QT_F64: return probe_kind<0>(s);
        case QT_F32: return probe_kind<1>(s);
        case QT_BF16X3: return probe_kind<2>(s);
    }
    fail(QT_ERR_ARG, "unknown precision");
}

}  // namespace qt
