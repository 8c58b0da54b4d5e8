// Hilbert index of a cell of a 2^B x 2^B x 2^B grid (B bits per axis), used
// to order the entries inside each temporal bin in the spatial layout.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace tds {

// Skilling's transform of the axes to the "transposed" Hilbert index
// (J. Skilling, Programming the Hilbert curve, AIP Conf. Proc. 707, 2004):
// undo the excess work of the recursive reflections and rotations, Gray-encode,
// then interleave the bits (axis 0 most significant).  Consecutive indices
// are always adjacent cells, so a run of entries in this order has a compact
// bounding box (unlike the Morton order, which jumps at octant boundaries).
template <int B = 10>
__host__ __device__ inline uint32_t hilbert3(uint32_t x, uint32_t y, uint32_t z) {
    static_assert(B >= 1 && B <= 10, "3 B bits must fit 32 bits");
    uint32_t X[3] = {x, y, z};
    constexpr uint32_t M = 1u << (B - 1);
    for (uint32_t q = M; q > 1; q >>= 1) {
        const uint32_t p = q - 1;
        for (int i = 0; i < 3; ++i) {
            if (X[i] & q) {
                X[0] ^= p;
            } else {
                const uint32_t t = (X[0] ^ X[i]) & p;
                X[0] ^= t;
                X[i] ^= t;
            }
        }
    }
    X[1] ^= X[0];
    X[2] ^= X[1];
    uint32_t t = 0;
    for (uint32_t q = M; q > 1; q >>= 1)
        if (X[2] & q) t ^= q - 1;
    uint32_t key = 0;
    for (int b = B - 1; b >= 0; --b)
        for (int i = 0; i < 3; ++i) key = (key << 1) | (((X[i] ^ t) >> b) & 1u);
    return key;
}

}  // namespace tds
