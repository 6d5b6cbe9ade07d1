// Exclusive prefix sums of int32 or int64 counts (reduce / scan block sums /
// rescan).
//
// A tile of SCAN_TILE counts goes to one single-wave workgroup: the tile is
// staged in LDS with coalesced loads, each lane sums 16 consecutive counts,
// the 64 lane sums are scanned across the wave, and the tile is rescanned
// with the tile's global offset. Tiles beyond one are handled by scanning the
// per-tile sums recursively. Single waves, because these scans run in the
// symbolic phase beside the previous multiply's numeric kernel, whose
// single-wave workgroups take every wave slot that frees up: a workgroup of
// several waves would wait until that kernel drained.
#include "qt_internal.h"

namespace qt {

constexpr int SCAN_T = 64;
constexpr int SCAN_I = 16;
constexpr int SCAN_TILE = SCAN_T * SCAN_I;

// Exclusive scan of one value per thread across the workgroup.
template <class T>
__device__ inline T wg_exclusive_scan(T v, T* lds_waves, T* total) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    T x = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        T y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
    }
    if (lane == 63) lds_waves[wave] = x;
    __syncthreads();
    T before = 0, all = 0;
#pragma unroll
    for (int w = 0; w < SCAN_T / 64; ++w) {
        T t = lds_waves[w];
        if (w < wave) before += t;
        all += t;
    }
    *total = all;
    return before + x - v;
}

// Stage counts [tile*SCAN_TILE, +SCAN_TILE) into LDS (zero beyond n).
template <class T>
__device__ inline void load_tile(const T* in, int64_t n, T* lds) {
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
#pragma unroll
    for (int r = 0; r < SCAN_I; ++r) {
        int64_t i = base + r * SCAN_T + threadIdx.x;
        lds[r * SCAN_T + threadIdx.x] = (i < n) ? in[i] : T(0);
    }
    __syncthreads();
}

template <class T>
__global__ __launch_bounds__(SCAN_T) void k_scan_reduce(const T* __restrict__ in, int64_t n, T* __restrict__ sums) {
    __shared__ T lds[SCAN_TILE];
    __shared__ T waves[SCAN_T / 64];
    load_tile(in, n, lds);
    T s = 0;
#pragma unroll
    for (int r = 0; r < SCAN_I; ++r) s += lds[threadIdx.x * SCAN_I + r];
    T total;
    wg_exclusive_scan(s, waves, &total);
    if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

// out[i] = offset(tile) + exclusive prefix within the tile, for i <= n
// (in[n] counts as 0, so out[n] is the grand total).
template <class T>
__global__ __launch_bounds__(SCAN_T) void k_scan_down(const T* __restrict__ in, int64_t n,
                                                      const T* __restrict__ tile_off, T* __restrict__ out) {
    __shared__ T lds[SCAN_TILE];
    __shared__ T waves[SCAN_T / 64];
    load_tile(in, n, lds);
    T v[SCAN_I];
    T s = 0;
#pragma unroll
    for (int r = 0; r < SCAN_I; ++r) {
        v[r] = lds[threadIdx.x * SCAN_I + r];
        s += v[r];
    }
    T total;
    T run = wg_exclusive_scan(s, waves, &total) + (tile_off ? tile_off[blockIdx.x] : T(0));
    __syncthreads();
#pragma unroll
    for (int r = 0; r < SCAN_I; ++r) {
        lds[threadIdx.x * SCAN_I + r] = run;
        run += v[r];
    }
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
#pragma unroll
    for (int r = 0; r < SCAN_I; ++r) {
        int64_t i = base + r * SCAN_T + threadIdx.x;
        if (i <= n) out[i] = lds[r * SCAN_T + threadIdx.x];
    }
}

static int64_t tiles_for(int64_t n) { return (n + 1 + SCAN_TILE - 1) / SCAN_TILE; }

size_t scan_tmp_elems(int64_t n) {
    int64_t nt = tiles_for(n);
    if (nt <= 1) return 0;
    return (size_t)(2 * nt + 1) + scan_tmp_elems(nt);
}

template <class T>
static void scan_impl(const T* in, T* out, int64_t n, T* tmp, hipStream_t s) {
    const int64_t nt = tiles_for(n);
    if (nt <= 1) {
        k_scan_down<T><<<1, SCAN_T, 0, s>>>(in, n, nullptr, out);
        QT_LAUNCH("k_scan_down");
        return;
    }
    T* sums = tmp;
    T* offs = tmp + nt;
    k_scan_reduce<T><<<(unsigned)nt, SCAN_T, 0, s>>>(in, n, sums);
    QT_LAUNCH("k_scan_reduce");
    scan_impl<T>(sums, offs, nt, tmp + 2 * nt + 1, s);
    k_scan_down<T><<<(unsigned)nt, SCAN_T, 0, s>>>(in, n, offs, out);
    QT_LAUNCH("k_scan_down");
}

void exclusive_scan(const int32_t* in, int32_t* out, int64_t n, int32_t* tmp, hipStream_t s) {
    scan_impl<int32_t>(in, out, n, tmp, s);
}

void exclusive_scan(const int64_t* in, int64_t* out, int64_t n, int64_t* tmp, hipStream_t s) {
    scan_impl<int64_t>(in, out, n, tmp, s);
}

void exclusive_scan(const double* in, double* out, int64_t n, double* tmp, hipStream_t s) {
    scan_impl<double>(in, out, n, tmp, s);
}

}  // namespace qt
