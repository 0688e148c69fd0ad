// Philox4x32-10 counter-based generator (Salmon, Moraes, Dror and Shaw,
// "Parallel random numbers: as easy as 1, 2, 3", SC 2011): ten rounds of a
// multiply-high/low bijection on a 4 x 32-bit counter, with a 2 x 32-bit key
// bumped by the Weyl constants between rounds.  Compiled for host and device
// from this one definition; the host copy is exported for known-answer tests.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace useries {

struct Philox4 {
    uint32_t v[4];
};

__host__ __device__ inline Philox4 philox4x32_10(Philox4 c, uint32_t k0, uint32_t k1) {
    constexpr uint32_t kM0 = 0xD2511F53u, kM1 = 0xCD9E8D57u;   // round multipliers
    constexpr uint32_t kW0 = 0x9E3779B9u, kW1 = 0xBB67AE85u;   // key schedule increments
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)kM0 * c.v[0];
        const uint64_t p1 = (uint64_t)kM1 * c.v[2];
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        Philox4 n;
        n.v[0] = hi1 ^ c.v[1] ^ k0;
        n.v[1] = lo1;
        n.v[2] = hi0 ^ c.v[3] ^ k1;
        n.v[3] = lo0;
        c = n;
        k0 += kW0;
        k1 += kW1;
    }
    return c;
}

// uniform in (0, 1): the top 24 bits, centred in their interval
__host__ __device__ inline float philox_unit(uint32_t x) {
    return ((float)(x >> 8) + 0.5f) * 5.9604644775390625e-8f;   // 2^-24
}

}  // namespace useries
