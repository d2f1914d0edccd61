// philox.h -- Philox4x32-10 counter-based generator (Salmon, Moraes, Dror,
// Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11), usable on the
// host and on the device.  The key is the 64-bit seed (low word first).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace ftwa {

struct PhiloxCounter {
    uint32_t w0, w1, w2, w3;
};

struct PhiloxBlock {
    uint32_t x[4];
    // 53-bit integers formed from the high bits of the output words
    __host__ __device__ uint64_t bits53_first() const {
        return ((uint64_t)x[0] << 21) | (uint64_t)(x[1] >> 11);
    }
    __host__ __device__ uint64_t bits53_second() const {
        return ((uint64_t)x[2] << 21) | (uint64_t)(x[3] >> 11);
    }
};

__host__ __device__ inline void philox_round(uint32_t& c0, uint32_t& c1, uint32_t& c2,
                                             uint32_t& c3, uint32_t k0, uint32_t k1) {
    const uint64_t p = (uint64_t)0xD2511F53u * c0;
    const uint64_t q = (uint64_t)0xCD9E8D57u * c2;
    const uint32_t nc0 = (uint32_t)(q >> 32) ^ c1 ^ k0;
    const uint32_t nc2 = (uint32_t)(p >> 32) ^ c3 ^ k1;
    c1 = (uint32_t)q;
    c3 = (uint32_t)p;
    c0 = nc0;
    c2 = nc2;
}

__host__ __device__ inline PhiloxBlock philox4x32_10(PhiloxCounter ctr, uint64_t seed) {
    uint32_t c0 = ctr.w0, c1 = ctr.w1, c2 = ctr.w2, c3 = ctr.w3;
    uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    philox_round(c0, c1, c2, c3, k0, k1);
#pragma unroll
    for (int r = 1; r < 10; ++r) {
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
        philox_round(c0, c1, c2, c3, k0, k1);
    }
    PhiloxBlock b;
    b.x[0] = c0;
    b.x[1] = c1;
    b.x[2] = c2;
    b.x[3] = c3;
    return b;
}

}  // namespace ftwa
