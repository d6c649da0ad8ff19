// kpz_ring.hip -- gfx950 kernels and the C ABI (include/kpz.h, ring part)
// for the 1+1-dimensional rooftop reduction of the octahedron model.
//
// Paper: Kelling, Odor, Nagy, Schulz, Heinig, "Comparison of different
// parallel implementations of the 2+1-dimensional KPZ model and the
// 3-dimensional KMC model".  Sec. 2.1: the octahedron model is the 2+1-d
// extension of the rooftop (ASEP) model; in one dimension a site is a local
// minimum iff its left bond is down and its right bond up, and a flip
// negates both bonds (probability p for a minimum, q for a maximum).
// Sec. 3 / 3.1: the same two decomposition layers, reduced to one dimension:
// dead-border blocks whose origin moves every MCS, single-hit double tiling
// inside each block.
//
// Layout: bond i (s_i = h(i+1) - h(i)) is bit i mod 32 of word i / 32
// (1 = +1); L / 32 words.
//
// Schedule per MCS t (the oracle implements the same reading):
//   origin    o = w0 * B >> 32 of (ORIGIN1D, t, 0, 0); block b covers sites
//             (o + b B + lx) mod L; lx = 0 is dead when there are >1 blocks
//   tiles     4 sites = two cells of 2 sites (set 0: sites 0,1; set 1: 2,3)
//   4 steps   step k: block set = bit 4 (b mod 8) + k of word (b mod 32) / 8
//             of (SET1D, t, b / 32, 0), one draw per 32 blocks; tile m
//             attempts site 4m + 2 set + r
//   sites     tile m = tile mm (= m mod 8) of block word wl (= m / 8):
//             r = bit 4 mm + k of word wl mod 4 of (SITE1D, t, b B/128 + wl/4, 0),
//             so that the draw bits of step k sit on the tiles' nibbles
//   accept    u = A << 24 | (C & 0xFFFFFF): A = byte mm mod 4 of word
//             2 (wl mod 2) + mm / 4 of (ACC1D, t, b B/64 + wl/2, k);
//             C = w0 of (ACC1D2, t, b B/4 + m, k), drawn only on a tie of A
//
// Kernels
//   kpz_ring_init_kernel      flat start h(i) = i mod 2: words 0x55555555
//   kpz_ring_sweep_kernel<K>  one MCS: every lane one dead-border block of
//                             B = 32 K sites in K registers (no LDS); a wave
//                             takes 64 consecutive blocks, and neighbouring
//                             lanes join their shared words by a shuffle
//   kpz_ring_merge_kernel     the words two blocks share (origin not a
//                             multiple of 32) from both blocks' parts
//   kpz_ring_chunks_kernel    per chunk of 8192 bonds: (sum of bonds, sum of
//                             prefix heights, sum of their squares)
//   kpz_ring_finalize_kernel  chunk prefix, 128-bit totals, flip counters

#include <hip/hip_runtime.h>

#include <stdint.h>
#include <stdio.h>

#include <new>

#include "kpz.h"
#include "kpz_device.h"

namespace {

using kpzdev::byte_eq;
using kpzdev::byte_lt;
using kpzdev::philox;
using kpzdev::philox_v;
using kpzdev::U4;

constexpr uint32_t TAG_ORIGIN1D = 8, TAG_SET1D = 9, TAG_SITE1D = 10, TAG_ACC1D = 11,
                   TAG_ACC1D2 = 12;
constexpr int RING_SLOTS = 1024;       // flip-counter slots
constexpr int RING_HEADER = 256;       // results area
constexpr int CHUNK_WORDS = 256;       // words per chunk of the moment pass (one wave x 4)

struct RingArgs {
    uint32_t *words;
    uint32_t *side;                // [2][nwaves]: a wave's part of its first / after-last word
    unsigned long long *slots;
    uint64_t L;
    uint32_t W;                    // words
    uint32_t B, nb, nwaves;        // block size (sites), blocks, waves (64 blocks each)
    uint32_t seed_lo, seed_hi;
    uint32_t t;
    uint64_t P, Q;
    uint32_t acc;
};

__device__ __forceinline__ uint32_t ring_origin(const RingArgs &a)
{
    const U4 w = philox(0u, 0u, a.t, TAG_ORIGIN1D << 24, a.seed_lo, a.seed_hi);
    return (uint32_t)(((uint64_t)w.x * a.B) >> 32);
}

// 8 flags (bit j of f) -> nibble j (bit 4j).
__device__ __forceinline__ uint32_t spread8(uint32_t f)
{
    uint32_t x = f & 0xFFu;
    x = (x | (x << 12)) & 0x000F000Fu;
    x = (x | (x << 6)) & 0x03030303u;
    x = (x | (x << 3)) & 0x11111111u;
    return x;
}

// byte flags (bit 7 of each byte) of lo (tiles 0..3) and hi (tiles 4..7)
// -> 8-bit tile mask
__device__ __forceinline__ uint32_t gather_bytes(uint32_t lo, uint32_t hi)
{
    const uint32_t a = ((lo >> 7) & 1u) | ((lo >> 14) & 2u) | ((lo >> 21) & 4u) | ((lo >> 28) & 8u);
    const uint32_t b = ((hi >> 7) & 1u) | ((hi >> 14) & 2u) | ((hi >> 21) & 4u) | ((hi >> 28) & 8u);
    return a | (b << 4);
}

struct RingAcc {
    bool fullP;
    bool ties;           // a threshold below 2^32 has nonzero low bits
    uint32_t tP, tQ, lowP, lowQ;
};

// Acceptance of the 8 tiles of one word at step k: nibble masks (0xF per
// accepted tile) for minima (threshold P) and maxima (threshold Q).
__device__ __forceinline__ void ring_accept(uint32_t A0, uint32_t A1, const RingAcc &ac,
                                            uint32_t mn_t, uint32_t mx_t, uint64_t tile0,
                                            uint32_t k, const RingArgs &a, uint32_t &accP,
                                            uint32_t &accQ)
{
    uint32_t p8 = ac.fullP ? 0xFFu : (ac.tP ? gather_bytes(byte_lt(A0, ac.tP), byte_lt(A1, ac.tP)) : 0u);
    uint32_t q8 = ac.tQ ? gather_bytes(byte_lt(A0, ac.tQ), byte_lt(A1, ac.tQ)) : 0u;
    if (ac.ties) {   // uniform: skipped when both thresholds are whole bytes
        const uint32_t tp8 = (!ac.fullP && ac.lowP) ? gather_bytes(byte_eq(A0, ac.tP), byte_eq(A1, ac.tP)) & mn_t : 0u;
        const uint32_t tq8 = ac.lowQ ? gather_bytes(byte_eq(A0, ac.tQ), byte_eq(A1, ac.tQ)) & mx_t : 0u;
        uint32_t ties = tp8 | tq8;
        while (ties) {
            const uint32_t mm = __builtin_ctz(ties);
            ties &= ties - 1;
            const uint64_t g = tile0 + mm;
            const U4 c = philox_v((uint32_t)g, (uint32_t)(g >> 32), a.t, (TAG_ACC1D2 << 24) | k,
                                a.seed_lo, a.seed_hi);
            const uint32_t c24 = c.x & 0xFFFFFFu;
            if (((tp8 >> mm) & 1u) && c24 < ac.lowP) p8 |= 1u << mm;
            if (((tq8 >> mm) & 1u) && c24 < ac.lowQ) q8 |= 1u << mm;
        }
    }
    accP = spread8(p8) * 0xFu;
    accQ = spread8(q8) * 0xFu;
}

// 8 tiles -> 8-bit minimum / maximum flags of the chosen sites (for the
// tie draws): F-mask bit positions 4mm..4mm+3 -> bit mm.
__device__ __forceinline__ uint32_t nibbles_nonzero(uint32_t m)
{
    uint32_t x = (m | (m >> 1) | (m >> 2) | (m >> 3)) & 0x11111111u;
    x = (x | (x >> 3)) & 0x03030303u;
    x = (x | (x >> 6)) & 0x000F000Fu;
    x = (x | (x >> 12)) & 0xFFu;
    return x;
}

// One MCS of the ring.  Every lane is one dead-border block of B = 32 K
// sites held in K registers: blocks are independent within the MCS (site 0
// of a block is dead, so no update touches another block's bonds), and a
// wave handles 64 consecutive blocks.  The words two neighbouring lanes'
// blocks share are assembled with a shuffle; the two at the ends of the
// wave's range go through the side buffer and the merge launch.
template <int K, bool ACC>
__global__ __launch_bounds__(64) void kpz_ring_sweep_kernel(const RingArgs a)
{
    const uint32_t lane = threadIdx.x;
    const uint32_t w = blockIdx.x;                  // wave (range of 64 blocks)
    const uint32_t b = w * 64u + lane;              // this lane's block
    const bool live = b < a.nb;
    const uint32_t last = min(63u, a.nb - 1u - w * 64u);   // last live lane of the wave
    const uint32_t o = ring_origin(a);
    const uint32_t sh = o & 31u;
    // block b starts at site o + b B; its words are gw0 + j, j = 0..K
    const uint64_t g0 = ((uint64_t)o + (uint64_t)b * a.B) % a.L;
    const uint32_t gw0 = (uint32_t)(g0 >> 5);

    uint32_t c[K];
    if (live) {
        uint32_t raw[K + 1];
#pragma unroll
        for (int j = 0; j <= K; ++j) {
            uint32_t gw = gw0 + j;
            if (gw >= a.W) gw -= a.W;
            raw[j] = a.words[gw];
        }
#pragma unroll
        for (int j = 0; j < K; ++j) c[j] = __builtin_amdgcn_alignbit(raw[j + 1], raw[j], sh);
    } else {
#pragma unroll
        for (int j = 0; j < K; ++j) c[j] = 0u;
    }

    // site draws: block word wl uses word wl mod 4 of call (b K/4 + wl/4)
    uint32_t sw[K];
#pragma unroll
    for (int j = 0; j < K; j += 4) {
        const uint64_t qi = (uint64_t)b * (K / 4) + j / 4;
        const U4 s4 = philox_v((uint32_t)qi, (uint32_t)(qi >> 32), a.t, TAG_SITE1D << 24, a.seed_lo,
                             a.seed_hi);
        sw[j] = s4.x;
        sw[j + 1] = s4.y;
        sw[j + 2] = s4.z;
        sw[j + 3] = s4.w;
    }
    // set bits: one draw per 32 blocks; the wave's two draws are uniform
    // (scalar unit), each lane picks its block's 4 bits
    const U4 st0 = philox(2u * w, 0u, a.t, TAG_SET1D << 24, a.seed_lo, a.seed_hi);
    const U4 st1 = philox(2u * w + 1u, 0u, a.t, TAG_SET1D << 24, a.seed_lo, a.seed_hi);
    const bool hi32 = lane >= 32u;
    const uint32_t q8 = (lane >> 3) & 3u;
    const uint32_t sx = hi32 ? st1.x : st0.x, sy = hi32 ? st1.y : st0.y;
    const uint32_t sz = hi32 ? st1.z : st0.z, sww = hi32 ? st1.w : st0.w;
    const uint32_t sword = q8 == 0 ? sx : (q8 == 1 ? sy : (q8 == 2 ? sz : sww));
    const uint32_t setw = sword >> (4u * (lane & 7u));

    RingAcc ac;
    ac.fullP = a.P >= (1ull << 32);
    ac.tP = ac.fullP ? 256u : (uint32_t)(a.P >> 24);
    ac.tQ = (uint32_t)(a.Q >> 24);
    ac.lowP = (uint32_t)(a.P & 0xFFFFFFu);
    ac.lowQ = (uint32_t)(a.Q & 0xFFFFFFu);
    ac.ties = (!ac.fullP && ac.lowP != 0) || ac.lowQ != 0;
    const bool single = a.nb == 1;     // one periodic block: site 0 is live
    int net = 0;

    if (live) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const uint32_t set = (setw >> k) & 1u;
            uint32_t F[K];
#pragma unroll
            for (int j = 0; j < K; ++j) {
                // left neighbour bond of bit 0: bit 31 of the previous word (for
                // j = 0 the block's last bond when the block is the whole ring;
                // otherwise site 0 is dead and the value is not used)
                const uint32_t prev = j ? c[j - 1] : (single ? c[K - 1] : 0u);
                const uint32_t l = (c[j] << 1) | (prev >> 31);
                const uint32_t mn = ~l & c[j];
                const uint32_t R = (sw[j] >> k) & 0x11111111u;
                uint32_t sel = ((0x11111111u & ~R) | (R << 1)) << (2 * set);
                if (j == 0 && !single) sel &= ~1u;
                if (ACC) {
                    const uint32_t mx = l & ~c[j];
                    const uint64_t ai = (uint64_t)b * (K / 2) + j / 2;
                    const U4 aw = philox_v((uint32_t)ai, (uint32_t)(ai >> 32), a.t,
                                         (TAG_ACC1D << 24) | k, a.seed_lo, a.seed_hi);
                    const uint32_t A0 = (j & 1) ? aw.z : aw.x;
                    const uint32_t A1 = (j & 1) ? aw.w : aw.y;
                    uint32_t accP, accQ;
                    const uint64_t tile0 = (uint64_t)b * (a.B / 4) + 8ull * j;
                    ring_accept(A0, A1, ac, nibbles_nonzero(sel & mn), nibbles_nonzero(sel & mx),
                                tile0, k, a, accP, accQ);
                    const uint32_t fmin = sel & mn & accP, fmax = sel & mx & accQ;
                    net += __builtin_popcount(fmin) - __builtin_popcount(fmax);
                    F[j] = fmin | fmax;
                } else {
                    F[j] = sel & mn;
                    net += __builtin_popcount(F[j]);
                }
            }
            // apply: a flip at site i negates bonds i - 1 and i; chosen sites
            // are at least three apart, so the masks never overlap
#pragma unroll
            for (int j = 0; j < K; ++j) {
                c[j] ^= F[j] | (F[j] >> 1);
                const uint32_t in = j + 1 < K ? (F[j + 1] & 1u) : (single ? (F[0] & 1u) : 0u);
                c[j] ^= in << 31;
            }
        }
    }

    // store: global word gw0 + j of block b (j >= 1) = high part of block
    // word j - 1 and low part of block word j; word gw0 is shared with the
    // previous block (its last word's high part comes from lane - 1)
    const uint32_t prev_last = __shfl(c[K - 1], (lane + 63u) & 63u, 64);
    if (live) {
#pragma unroll
        for (int j = 0; j < K; ++j) {
            uint32_t gw = gw0 + j;
            if (gw >= a.W) gw -= a.W;
            if (sh == 0) {
                a.words[gw] = c[j];
            } else if (j > 0) {
                a.words[gw] = __builtin_amdgcn_alignbit(c[j], c[j - 1], 32u - sh);
            } else if (lane > 0) {
                a.words[gw] = __builtin_amdgcn_alignbit(c[0], prev_last, 32u - sh);
            } else {
                a.side[w] = c[0] << sh;
            }
        }
        if (sh && lane == last) a.side[a.nwaves + w] = c[K - 1] >> (32u - sh);
    }

#pragma unroll
    for (int off = 32; off > 0; off >>= 1) net += __shfl_xor(net, off, 64);
    if (lane == 0 && net != 0)
        atomicAdd(a.slots + (w & (RING_SLOTS - 1)), (unsigned long long)(long long)net);
}

// The word at the start of each wave's range: the previous wave's last
// block's high part and this wave's first block's low part.
__global__ void kpz_ring_merge_kernel(const RingArgs a)
{
    const uint32_t o = ring_origin(a);
    const uint32_t sh = o & 31u;
    if (sh == 0) return;
    for (uint32_t w = blockIdx.x * blockDim.x + threadIdx.x; w < a.nwaves;
         w += gridDim.x * blockDim.x) {
        const uint32_t gw = (uint32_t)((((uint64_t)o + (uint64_t)w * 64u * a.B) % a.L) >> 5);
        const uint32_t left = a.side[a.nwaves + (w == 0 ? a.nwaves - 1 : w - 1)];
        a.words[gw] = left | a.side[w];
    }
}

__global__ void kpz_ring_init_kernel(uint32_t *words, uint64_t n)
{
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        words[i] = 0x55555555u;
}

__global__ void kpz_ring_fill_kernel(long long *p, uint32_t n)
{
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        p[i] = 0;
}

// ---- exact moments

// (sum of bonds, sum over positions of the prefix P(p) = sum_{j<p} s_j, sum
// of P^2) of one byte of 8 bonds
__device__ __forceinline__ void byte_sums(uint32_t v, int &d, int &s1, int &s2)
{
    int P = 0;
    s1 = 0;
    s2 = 0;
#pragma unroll
    for (int p = 0; p < 8; ++p) {
        s1 += P;
        s2 += P * P;
        P += ((v >> p) & 1u) ? 1 : -1;
    }
    d = P;
}

// Per chunk of CHUNK_WORDS words (one wave, four words per lane):
// out[3c..3c+2] = (sum of bonds, sum of P, sum of P^2) with P the height
// relative to the chunk's first site.
__global__ __launch_bounds__(256) void kpz_ring_chunks_kernel(const uint32_t *words, uint32_t W,
                                                             long long *out, uint32_t nchunks)
{
    __shared__ int lut_d[256], lut_1[256], lut_2[256];
    {
        int d, s1, s2;
        byte_sums(threadIdx.x, d, s1, s2);
        lut_d[threadIdx.x] = d;
        lut_1[threadIdx.x] = s1;
        lut_2[threadIdx.x] = s2;
    }
    __syncthreads();
    const uint32_t lane = threadIdx.x & 63u;
    for (uint32_t ch = blockIdx.x * 4 + (threadIdx.x >> 6); ch < nchunks; ch += gridDim.x * 4) {
        long long D = 0, S1 = 0, S2 = 0, n = 0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint32_t wi = ch * CHUNK_WORDS + lane * 4 + j;
            if (wi >= W) break;
            const uint32_t w = words[wi];
#pragma unroll
            for (int by = 0; by < 4; ++by) {
                const uint32_t v = (w >> (8 * by)) & 0xFFu;
                const long long e = D;
                S1 += lut_1[v] + 8 * e;
                S2 += lut_2[v] + 2 * e * lut_1[v] + 8 * e * e;
                D += lut_d[v];
                n += 8;
            }
        }
        // exclusive scan of D over the lanes; shift each lane's sums
        long long inc = D;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const long long v = __shfl_up(inc, off, 64);
            if (lane >= (uint32_t)off) inc += v;
        }
        const long long ex = inc - D;
        long long s1 = S1 + n * ex;
        long long s2 = S2 + 2 * ex * S1 + n * ex * ex;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            s1 += __shfl_xor(s1, off, 64);
            s2 += __shfl_xor(s2, off, 64);
        }
        const long long dtot = __shfl(inc, 63, 64);
        if (lane == 0) {
            out[3 * (size_t)ch] = dtot;
            out[3 * (size_t)ch + 1] = s1;
            out[3 * (size_t)ch + 2] = s2;
        }
    }
}

// One work-group: R1 = sum (h - h(0)), R2 = sum (h - h(0))^2 over the ring
// from the chunk triples (prefix of the chunk sums), plus the flip counters.
// res = (R1 lo, R1 hi, R2 lo, R2 hi, net).
__global__ __launch_bounds__(1024) void kpz_ring_finalize_kernel(const long long *ch,
                                                                uint32_t nchunks, uint32_t W,
                                                                const long long *slots,
                                                                long long *res)
{
    __shared__ long long scan[1024];
    __shared__ __int128 r1s[1024], r2s[1024];
    __shared__ long long base;
    const uint32_t tid = threadIdx.x;
    if (tid == 0) base = 0;
    __int128 r1 = 0, r2 = 0;
    __syncthreads();
    for (uint32_t c0 = 0; c0 < nchunks; c0 += 1024) {
        const uint32_t c = c0 + tid;
        const long long d = c < nchunks ? ch[3 * (size_t)c] : 0;
        scan[tid] = d;
        __syncthreads();
        for (uint32_t off = 1; off < 1024; off <<= 1) {
            const long long v = tid >= off ? scan[tid - off] : 0;
            __syncthreads();
            scan[tid] += v;
            __syncthreads();
        }
        const long long ex = base + scan[tid] - d;
        if (c < nchunks) {
            const uint32_t nw = (c + 1) * CHUNK_WORDS <= W ? CHUNK_WORDS : W - c * CHUNK_WORDS;
            const __int128 n = 32 * (__int128)nw;
            const __int128 s1 = ch[3 * (size_t)c + 1], s2 = ch[3 * (size_t)c + 2];
            r1 += s1 + n * ex;
            r2 += s2 + 2 * (__int128)ex * s1 + n * (__int128)ex * ex;
        }
        __syncthreads();
        if (tid == 1023) base += scan[1023];
        __syncthreads();
    }
    r1s[tid] = r1;
    r2s[tid] = r2;
    __syncthreads();
    for (uint32_t s = 512; s > 0; s >>= 1) {
        if (tid < s) {
            r1s[tid] += r1s[tid + s];
            r2s[tid] += r2s[tid + s];
        }
        __syncthreads();
    }
    long long nsum = tid < RING_SLOTS ? slots[tid] : 0;
    scan[tid] = nsum;
    __syncthreads();
    for (uint32_t s = 512; s > 0; s >>= 1) {
        if (tid < s) scan[tid] += scan[tid + s];
        __syncthreads();
    }
    if (tid == 0) {
        const unsigned __int128 u1 = (unsigned __int128)r1s[0], u2 = (unsigned __int128)r2s[0];
        res[0] = (long long)(uint64_t)u1;
        res[1] = (long long)(uint64_t)(u1 >> 64);
        res[2] = (long long)(uint64_t)u2;
        res[3] = (long long)(uint64_t)(u2 >> 64);
        res[4] = scan[0];
    }
}

}  // namespace

// ================================================================ host

struct kpz_ring {
    kpz_ring_params prm;
    uint32_t B;
    uint32_t *words;
    uint8_t *ws;
    hipStream_t stream;
    int64_t t;
    uint64_t P, Q;
    char err[256];
};

namespace {

uint64_t ring_threshold(double prob)
{
    if (prob >= 1.0) return 1ull << 32;
    if (prob <= 0.0) return 0;
    return (uint64_t)(prob * 4294967296.0);
}

kpz_status ring_resolve(const kpz_ring_params *p, uint32_t *B)
{
    if (!p) return KPZ_EINVAL;
    const int64_t L = p->L;
    if (L < 128 || L > (1ll << 32) || L % 128) return KPZ_EINVAL;
    if (!(p->p >= 0.0 && p->p <= 1.0 && p->q >= 0.0 && p->q <= 1.0)) return KPZ_EINVAL;
    if (p->flags != 0) return KPZ_EINVAL;
    const int64_t b = p->block ? p->block : 128;
    if (b != 128 && b != 256 && b != 512 && b != 1024) return KPZ_EINVAL;
    if (L % b) return KPZ_EINVAL;
    *B = (uint32_t)b;
    return KPZ_OK;
}

size_t ring_ws_needed(int64_t L, uint32_t B)
{
    const uint64_t W = (uint64_t)L / 32, nwaves = ((uint64_t)L / B + 63) / 64;
    const uint64_t nchunks = (W + CHUNK_WORDS - 1) / CHUNK_WORDS;
    return (size_t)RING_HEADER + sizeof(long long) * RING_SLOTS + 3 * sizeof(long long) * nchunks +
           2 * sizeof(uint32_t) * nwaves;
}

long long *ring_res(kpz_ring *r) { return (long long *)r->ws; }
long long *ring_slots(kpz_ring *r) { return (long long *)(r->ws + RING_HEADER); }
long long *ring_chunks(kpz_ring *r) { return ring_slots(r) + RING_SLOTS; }
uint32_t *ring_side(kpz_ring *r)
{
    const uint64_t W = (uint64_t)r->prm.L / 32;
    return (uint32_t *)(ring_chunks(r) + 3 * ((W + CHUNK_WORDS - 1) / CHUNK_WORDS));
}

kpz_status ring_fail(kpz_ring *r, hipError_t e, const char *what)
{
    if (r) snprintf(r->err, sizeof r->err, "%s: %s", what, hipGetErrorString(e));
    return KPZ_EHIP;
}

}  // namespace

extern "C" {

kpz_status kpz_ring_workspace_bytes(const kpz_ring_params *p, size_t *bytes)
{
    uint32_t B;
    const kpz_status st = ring_resolve(p, &B);
    if (st != KPZ_OK) return st;
    if (!bytes) return KPZ_EINVAL;
    *bytes = ring_ws_needed(p->L, B);
    return KPZ_OK;
}

kpz_status kpz_ring_init(kpz_ring **out, const kpz_ring_params *p, uint32_t *d_words,
                         size_t words_bytes, void *d_ws, size_t ws_bytes, void *stream)
{
    if (!out) return KPZ_EINVAL;
    *out = nullptr;
    uint32_t B;
    const kpz_status st = ring_resolve(p, &B);
    if (st != KPZ_OK) return st;
    if (!d_words || !d_ws) return KPZ_EINVAL;
    if (words_bytes < (uint64_t)p->L / 8 || ws_bytes < ring_ws_needed(p->L, B)) return KPZ_ESIZE;
    kpz_ring *r = new (std::nothrow) kpz_ring();
    if (!r) return KPZ_EINVAL;
    r->prm = *p;
    r->B = B;
    r->words = d_words;
    r->ws = (uint8_t *)d_ws;
    r->stream = (hipStream_t)stream;
    r->t = 0;
    r->P = ring_threshold(p->p);
    r->Q = ring_threshold(p->q);
    r->err[0] = 0;
    const uint64_t W = (uint64_t)p->L / 32;
    const uint32_t grid = (uint32_t)((W + 255) / 256 < 65536 ? (W + 255) / 256 : 65536);
    hipLaunchKernelGGL(kpz_ring_init_kernel, dim3(grid), dim3(256), 0, r->stream, d_words, W);
    hipLaunchKernelGGL(kpz_ring_fill_kernel, dim3(RING_SLOTS / 256), dim3(256), 0, r->stream,
                       ring_slots(r), (uint32_t)RING_SLOTS);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        ring_fail(r, e, "kpz_ring_init launch");
        delete r;
        return KPZ_EHIP;
    }
    *out = r;
    return KPZ_OK;
}

kpz_status kpz_ring_sweep(kpz_ring *r, int32_t n_mcs)
{
    if (!r || n_mcs < 0) return KPZ_EINVAL;
    if (n_mcs == 0) return KPZ_OK;
    if (r->t + n_mcs > 0xFFFFFFFFll) return KPZ_ERANGE;
    RingArgs a;
    a.words = r->words;
    a.side = ring_side(r);
    a.slots = (unsigned long long *)ring_slots(r);
    a.L = (uint64_t)r->prm.L;
    a.W = (uint32_t)(a.L / 32);
    a.B = r->B;
    a.nb = (uint32_t)(a.L / r->B);
    a.nwaves = (a.nb + 63) / 64;
    a.seed_lo = (uint32_t)r->prm.seed;
    a.seed_hi = (uint32_t)(r->prm.seed >> 32);
    a.P = r->P;
    a.Q = r->Q;
    a.acc = !(r->P == (1ull << 32) && r->Q == 0);
    const uint32_t K = r->B / 32;
    const uint32_t mgrid = (a.nwaves + 255) / 256 < 4096 ? (a.nwaves + 255) / 256 : 4096;
    for (int32_t m = 0; m < n_mcs; ++m) {
        a.t = (uint32_t)(r->t + m);
#define RING_LAUNCH(KK)                                                                      \
    if (a.acc)                                                                               \
        hipLaunchKernelGGL((kpz_ring_sweep_kernel<KK, true>), dim3(a.nwaves), dim3(64), 0,   \
                           r->stream, a);                                                    \
    else                                                                                     \
        hipLaunchKernelGGL((kpz_ring_sweep_kernel<KK, false>), dim3(a.nwaves), dim3(64), 0,  \
                           r->stream, a);
        switch (K) {
        case 4: RING_LAUNCH(4) break;
        case 8: RING_LAUNCH(8) break;
        case 16: RING_LAUNCH(16) break;
        default: RING_LAUNCH(32) break;
        }
#undef RING_LAUNCH
        hipLaunchKernelGGL(kpz_ring_merge_kernel, dim3(mgrid), dim3(256), 0, r->stream, a);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return ring_fail(r, e, "kpz_ring_sweep launch");
    }
    r->t += n_mcs;
    return KPZ_OK;
}

kpz_status kpz_ring_roughness(kpz_ring *r, int64_t *S1o, int64_t *S2o, double *W2o)
{
    if (!r) return KPZ_EINVAL;
    const uint64_t W = (uint64_t)r->prm.L / 32;
    const uint32_t nchunks = (uint32_t)((W + CHUNK_WORDS - 1) / CHUNK_WORDS);
    const uint32_t grid = (nchunks + 3) / 4 < 8192 ? (nchunks + 3) / 4 : 8192;
    hipLaunchKernelGGL(kpz_ring_chunks_kernel, dim3(grid), dim3(256), 0, r->stream, r->words,
                       (uint32_t)W, ring_chunks(r), nchunks);
    hipLaunchKernelGGL(kpz_ring_finalize_kernel, dim3(1), dim3(1024), 0, r->stream,
                       (const long long *)ring_chunks(r), nchunks, (uint32_t)W,
                       (const long long *)ring_slots(r), ring_res(r));
    hipError_t e = hipGetLastError();
    long long res[5];
    if (e == hipSuccess)
        e = hipMemcpyAsync(res, ring_res(r), sizeof res, hipMemcpyDeviceToHost, r->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(r->stream);
    if (e != hipSuccess) return ring_fail(r, e, "kpz_ring_roughness");
    const __int128 L = r->prm.L;
    const __int128 R1 = (__int128)(((unsigned __int128)(uint64_t)res[1] << 64) | (uint64_t)res[0]);
    const __int128 R2 = (__int128)(((unsigned __int128)(uint64_t)res[3] << 64) | (uint64_t)res[2]);
    const __int128 S1 = L / 2 + 2 * (__int128)res[4];
    if ((S1 - R1) % L != 0) {
        snprintf(r->err, sizeof r->err, "height anchor not integral: words and flip count disagree");
        return KPZ_ESTATE;
    }
    const __int128 h0 = (S1 - R1) / L;
    const __int128 S2 = R2 + 2 * h0 * R1 + L * h0 * h0;
    const __int128 num = L * R2 - R1 * R1;
    if (W2o) *W2o = (double)((long double)num / ((long double)L * (long double)L));
    const __int128 lim = (__int128)INT64_MAX;
    if (S1o) *S1o = (int64_t)S1;
    if (S2o) *S2o = (int64_t)S2;
    if (S1 > lim || S1 < -lim - 1 || S2 > lim) return KPZ_ERANGE;
    return KPZ_OK;
}

kpz_status kpz_ring_get_state(kpz_ring *r, int64_t *t, int64_t *net)
{
    if (!r) return KPZ_EINVAL;
    long long s[RING_SLOTS];
    hipError_t e = hipMemcpyAsync(s, ring_slots(r), sizeof s, hipMemcpyDeviceToHost, r->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(r->stream);
    if (e != hipSuccess) return ring_fail(r, e, "kpz_ring_get_state");
    long long n = 0;
    for (int i = 0; i < RING_SLOTS; ++i) n += s[i];
    if (t) *t = r->t;
    if (net) *net = n;
    return KPZ_OK;
}

void kpz_ring_destroy(kpz_ring *r) { delete r; }

const char *kpz_ring_last_error(const kpz_ring *r) { return r ? r->err : ""; }

}  // extern "C"
