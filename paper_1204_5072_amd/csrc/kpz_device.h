// kpz_device.h -- device helpers shared by the lattice and ring kernels:
// the Philox4x32 counter-based generator (Salmon, Moraes, Dror, Shaw,
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

// Rounds of the 2+1-d lattice dynamics' draws: seven, the smallest count
// for which the generator's authors found Philox4x32 to pass the BigCrush
// battery (their default, ten, keeps a safety margin and is what the ring
// and KMC draws use).
constexpr int LATTICE_ROUNDS = 7;

// R rounds of Philox4x32 on counter (c0, c1, c2, c3) with key (k0, k1).
// Plain xors: with a wave-uniform counter the compiler keeps the whole call
// on the scalar unit.
template <int R = 10>
__device__ __forceinline__ U4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                     uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < R; ++r) {
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

// The same generator for per-lane counters: each round's two three-input
// xors as single v_bitop3_b32 instructions.  Vector-only, so a wave-uniform
// counter belongs to philox() above.
template <int R = 10>
__device__ __forceinline__ U4 philox_v(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                       uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0 = __builtin_amdgcn_bitop3_b32((uint32_t)(p1 >> 32), c1, k0, 0x96);
        const uint32_t n2 = __builtin_amdgcn_bitop3_b32((uint32_t)(p0 >> 32), c3, k1, 0x96);
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return U4{c0, c1, c2, c3};
}

// 0x80 in every byte of A that is below c (1 <= c <= 256, c uniform), i.e.
// at most t = c - 1.  With t = 128 t7 + t', a byte a = 128 a7 + a' is <= t
// iff a7 < t7, or a7 = t7 and a' <= t'.  In every byte, (a | 0x80) - (t' + 1)
// lies in 0..254 (no borrow between bytes) and has bit 7 clear iff a' <= t'.
// One three-input logic op then takes a7, that bit and t7 (as a uniform mask):
// result bit 7 = ~a7 & ~d7 | t7 & ~(a7 & d7); truth table 0x2B over (A, d, m).
__device__ __forceinline__ uint32_t byte_lt(uint32_t A, uint32_t c)
{
    const uint32_t t = c - 1u;
    const uint32_t d = (A | 0x80808080u) - ((t & 0x7Fu) + 1u) * 0x01010101u;
    const uint32_t m = (t & 0x80u) ? 0xFFFFFFFFu : 0u;
    return __builtin_amdgcn_bitop3_b32(A, d, m, 0x2B) & 0x80808080u;
}

// 0x80 in every byte of A equal to c (0 <= c <= 255).
__device__ __forceinline__ uint32_t byte_eq(uint32_t A, uint32_t c)
{
    const uint32_t z = A ^ (c * 0x01010101u);
    return ~(((z & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | z) & 0x80808080u;
}

}  // namespace kpzdev

#endif  // KPZ_DEVICE_H_
