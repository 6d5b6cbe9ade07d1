// Key/value sort used when a matrix is built or copied out (outside the
// multiply): a bitonic network over a power-of-two padded array. Pairs are
// ordered by (key, value), so equal keys come out in ascending value order
// (the callers pass positions as values: a deterministic tie-break).
#include "qt_internal.h"

namespace qt {

__global__ void k_bitonic_pad(uint64_t* keys, int32_t* vals, int64_t n, int64_t npow2) {
    int64_t i = n + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < npow2) {
        keys[i] = ~0ull;
        vals[i] = -1;
    }
}

// One compare-exchange stage (distance j) of the merge of sequences of size k.
__global__ void k_bitonic_step(uint64_t* keys, int32_t* vals, int64_t npow2, int64_t j, int64_t k) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npow2) return;
    int64_t l = i ^ j;
    if (l <= i) return;
    const bool up = (i & k) == 0;
    uint64_t ki = keys[i], kl = keys[l];
    const int32_t vi = vals[i], vl = vals[l];
    const bool greater = (ki > kl) || (ki == kl && vi > vl);
    if (greater == up) {
        keys[i] = kl;
        keys[l] = ki;
        vals[i] = vl;
        vals[l] = vi;
    }
}

// Stages with compare distance below SORT_TILE stay inside one tile of
// SORT_TILE entries, so they run in LDS: one launch finishes every such
// stage of a merge step (or, for merge sizes up to the tile, sorts the tile
// outright) instead of one launch per stage.
constexpr int SORT_TILE = 2048;
constexpr int SORT_THREADS = SORT_TILE / 2;

__device__ __forceinline__ void cmp_swap_lds(uint64_t* key, int32_t* val, int64_t gi, int li, int lj, int64_t k) {
    const bool up = (gi & k) == 0;
    const uint64_t ki = key[li], kl = key[lj];
    const int32_t vi = val[li], vl = val[lj];
    const bool greater = (ki > kl) || (ki == kl && vi > vl);
    if (greater == up) {
        key[li] = kl;
        key[lj] = ki;
        val[li] = vl;
        val[lj] = vi;
    }
}

// k_first == 0: every merge size k = 2 .. SORT_TILE on the tile (a full
// bitonic sort of it); otherwise merge size k_first, distances j0 .. 1.
__global__ __launch_bounds__(SORT_THREADS) void k_bitonic_tile(uint64_t* keys, int32_t* vals, int64_t k_first,
                                                               int64_t j0) {
    __shared__ uint64_t key[SORT_TILE];
    __shared__ int32_t val[SORT_TILE];
    const int64_t base = (int64_t)blockIdx.x * SORT_TILE;
    for (int t = threadIdx.x; t < SORT_TILE; t += SORT_THREADS) {
        key[t] = keys[base + t];
        val[t] = vals[base + t];
    }
    __syncthreads();
    const int64_t k_lo = k_first ? k_first : 2, k_hi = k_first ? k_first : SORT_TILE;
    for (int64_t k = k_lo; k <= k_hi; k <<= 1) {
        for (int64_t j = k_first ? j0 : (k >> 1); j > 0; j >>= 1) {
            // thread t handles the pair (i, i + j) with i's bit j clear
            const int t = threadIdx.x;
            const int li = (int)(((t / j) * 2 * j) + (t % j));
            cmp_swap_lds(key, val, base + li, li, li + (int)j, k);
            __syncthreads();
        }
    }
    for (int t = threadIdx.x; t < SORT_TILE; t += SORT_THREADS) {
        keys[base + t] = key[t];
        vals[base + t] = val[t];
    }
}

// keys/vals must hold npow2 = next power of two >= n entries.
void bitonic_sort(uint64_t* keys, int32_t* vals, int64_t n, hipStream_t s) {
    if (n <= 1) return;
    int64_t npow2 = 1;
    while (npow2 < n) npow2 <<= 1;
    const int T = 256;
    if (npow2 > n) {
        k_bitonic_pad<<<(unsigned)((npow2 - n + T - 1) / T), T, 0, s>>>(keys, vals, n, npow2);
        QT_LAUNCH("k_bitonic_pad");
    }
    const unsigned grid = (unsigned)((npow2 + T - 1) / T);
    if (npow2 < SORT_TILE) {   // small: one compare-exchange launch per stage
        for (int64_t k = 2; k <= npow2; k <<= 1)
            for (int64_t j = k >> 1; j > 0; j >>= 1) {
                k_bitonic_step<<<grid, T, 0, s>>>(keys, vals, npow2, j, k);
                QT_LAUNCH("k_bitonic_step");
            }
        return;
    }
    const unsigned tiles = (unsigned)(npow2 / SORT_TILE);
    k_bitonic_tile<<<tiles, SORT_THREADS, 0, s>>>(keys, vals, 0, 0);
    QT_LAUNCH("k_bitonic_tile");
    for (int64_t k = 2 * SORT_TILE; k <= npow2; k <<= 1) {
        int64_t j = k >> 1;
        for (; j >= SORT_TILE; j >>= 1) {
            k_bitonic_step<<<grid, T, 0, s>>>(keys, vals, npow2, j, k);
            QT_LAUNCH("k_bitonic_step");
        }
        k_bitonic_tile<<<tiles, SORT_THREADS, 0, s>>>(keys, vals, k, j);
        QT_LAUNCH("k_bitonic_tile");
    }
}

}  // namespace qt
