// Morton (Z-order) keys for quadtree positions.
//
// A node or block at (row r, column c) of a level gets the key with the bits
// of c at even positions and the bits of r at odd positions. The two lowest
// bits of a key are then the quadrant q = 2*m + n of the position inside its
// parent (m = row half, n = column half), matching the child order
// C_11, C_12, C_21, C_22 of the quadtree, and sorting by key lists every
// subtree contiguously.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace qt {

__host__ __device__ inline uint64_t spread_bits(uint32_t x) {
    uint64_t v = x;
    v = (v | (v << 16)) & 0x0000FFFF0000FFFFull;
    v = (v | (v << 8)) & 0x00FF00FF00FF00FFull;
    v = (v | (v << 4)) & 0x0F0F0F0F0F0F0F0Full;
    v = (v | (v << 2)) & 0x3333333333333333ull;
    v = (v | (v << 1)) & 0x5555555555555555ull;
    return v;
}

__host__ __device__ inline uint32_t compact_bits(uint64_t v) {
    v &= 0x5555555555555555ull;
    v = (v | (v >> 1)) & 0x3333333333333333ull;
    v = (v | (v >> 2)) & 0x0F0F0F0F0F0F0F0Full;
    v = (v | (v >> 4)) & 0x00FF00FF00FF00FFull;
    v = (v | (v >> 8)) & 0x0000FFFF0000FFFFull;
    v = (v | (v >> 16)) & 0x00000000FFFFFFFFull;
    return (uint32_t)v;
}

__host__ __device__ inline uint64_t morton_key(uint32_t r, uint32_t c) {
    return (spread_bits(r) << 1) | spread_bits(c);
}
__host__ __device__ inline uint32_t morton_row(uint64_t k) { return compact_bits(k >> 1); }
__host__ __device__ inline uint32_t morton_col(uint64_t k) { return compact_bits(k); }

}  // namespace qt
