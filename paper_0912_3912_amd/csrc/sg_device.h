// sg_device.h -- small device helpers shared by the library's kernels
// (internal; not part of the C-ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sg {

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two 32x32
// multiplies with the high halves folded into the other two counter words and
// the key, key advanced by the two Weyl increments after every round.  Only
// word 0 of the output is used.  Each product is formed as one 64-bit
// multiply (one v_mad_u64_u32 instead of a low and a high multiply).
__device__ __forceinline__ uint32_t philox_word0(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                                 uint32_t k1)
{
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint64_t p0 = (uint64_t)c0 * 0xD2511F53u;
        const uint64_t p1 = (uint64_t)c2 * 0xCD9E8D57u;
        c0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        c1 = (uint32_t)p1;
        c2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        c3 = (uint32_t)p0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c0;
}

// Bit 0 of word 0 for counter (spin, word1, instance id, restart), key = seed.
__device__ __forceinline__ int rng_bit(uint64_t seed, uint32_t spin, uint32_t word1, uint32_t id, uint32_t restart)
{
    return (int)(philox_word0(spin, word1, id, restart, (uint32_t)seed, (uint32_t)(seed >> 32)) & 1u);
}

// Exact floor(a / d) for a * d < 2^32 with m = floor(2^32 / d) + 1 (then
// a*m / 2^32 - a/d < a/2^32 < 1/d, so the floor is unchanged); d = 1 is
// encoded as m = 0.
__device__ __forceinline__ uint32_t fdiv(uint32_t a, uint32_t m) { return m ? __umulhi(a, m) : a; }
__host__ __device__ __forceinline__ uint32_t fdiv_magic(uint32_t d)
{
    return d <= 1 ? 0u : (uint32_t)((0x100000000ull / d) + 1);
}

__device__ __forceinline__ int wrapi(int v, int L) { return v < 0 ? v + L : (v >= L ? v - L : v); }

}  // namespace sg
