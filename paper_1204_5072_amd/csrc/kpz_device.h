// kpz_device.h -- device helpers shared by the lattice and ring kernels:
// the Philox4x32-10 counter-based generator (Salmon, Moraes, Dror, Shaw,
// "Parallel random numbers: as easy as 1, 2, 3", SC'11) and byte-wise
// comparisons used by the SWAR acceptance tests.
#ifndef KPZ_DEVICE_H_
#define KPZ_DEVICE_H_

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace kpzdev {

struct U4 {
    uint32_t x, y, z, w;
};

// Ten rounds of Philox4x32 on counter (c0, c1, c2, c3) with key (k0, k1).
__device__ __forceinline__ U4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                     uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return U4{c0, c1, c2, c3};
}

// 0x80 in every byte of A that is below c (0 <= c <= 256): in 16-bit lanes
// (a | 0x100) - c has bit 8 clear iff a < c.
__device__ __forceinline__ uint32_t byte_lt(uint32_t A, uint32_t c)
{
    const uint32_t cc = c * 0x00010001u;
    const uint32_t even = ((A & 0x00FF00FFu) | 0x01000100u) - cc;
    const uint32_t odd = (((A >> 8) & 0x00FF00FFu) | 0x01000100u) - cc;
    const uint32_t ge = ((even >> 1) & 0x00800080u) | ((odd << 7) & 0x80008000u);
    return ~ge & 0x80808080u;
}

// 0x80 in every byte of A equal to c (0 <= c <= 255).
__device__ __forceinline__ uint32_t byte_eq(uint32_t A, uint32_t c)
{
    const uint32_t z = A ^ (c * 0x01010101u);
    return ~(((z & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | z) & 0x80808080u;
}

}  // namespace kpzdev

#endif  // KPZ_DEVICE_H_
