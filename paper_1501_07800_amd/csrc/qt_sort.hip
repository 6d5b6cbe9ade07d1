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
    for (int64_t k = 2; k <= npow2; k <<= 1)
        for (int64_t j = k >> 1; j > 0; j >>= 1) {
            k_bitonic_step<<<grid, T, 0, s>>>(keys, vals, npow2, j, k);
            QT_LAUNCH("k_bitonic_step");
        }
}

}  // namespace qt
