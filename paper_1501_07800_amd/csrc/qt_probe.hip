// Attainable MFMA rate of this GPU: a register-only loop of the same MFMA
// instruction each numeric path issues (fp64 16x16x4, fp32 16x16x4, bf16
// 16x16x32), eight independent accumulator chains per wave, enough waves to
// fill every SIMD several times over. No memory traffic inside the loop, so
// the rate it reaches is the ceiling the block GEMMs can approach, to be read
// beside the published peak.
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

double probe_mfma(qt_prec prec, hipStream_t s) {
    switch (prec) {
        case QT_F64: return probe_kind<0>(s);
        case QT_F32: return probe_kind<1>(s);
        case QT_BF16X3: return probe_kind<2>(s);
    }
    fail(QT_ERR_ARG, "unknown precision");
}

}  // namespace qt
