// kmc.hip -- kinetic lattice Monte Carlo of a binary alloy on gfx950
// (Sec. 2.2 "Kinetic Monte Carlo", eqs. fcc and metropolis; Sec. 3.2
// "Implementation of KMC").
//
// Kernels:
//   kmc_init_kernel     the homogeneous random mixture, one Philox draw per site
//   kmc_phase_kernel    one block set of one MCS: each work-group copies its
//                       block plus a two-position halo into LDS (one byte per
//                       cubic position), makes the 256 single-hit steps of its
//                       64 tiles in one wave, and writes the block plus a
//                       one-position halo back
//   kmc_count_kernel    number of B and of B-B bonds (64-bit atomics)
//   kmc_fill_kernel     clears counters without hipMemsetAsync
//
// Schedule (both layers doubly tiled; the paper's own GPU scheme): blocks of
// B^3 positions form eight sets by the parities of their block coordinates;
// the sets run one launch each, in an order drawn per MCS; the block grid is
// shifted by a random origin per MCS.  Blocks of one set lie a block apart,
// so what one block reads (two positions beyond its faces) and writes (one
// beyond) never meets another block of the launch.  Inside a block, tiles of
// 8^3 positions are bisected into eight 4^3 cells; step k of 256 picks one
// cell set for the whole block, and every tile makes one attempt at a random
// fcc site of its cell: concurrent attempts are at least five positions
// apart along some axis, more than the three an attempt can reach.
//
// Random numbers (Philox4x32-10, counter (idx lo, idx hi, t, tag << 24 | sub),
// key = seed):
//   origin of MCS t          (18, t, idx 0, sub 0): floor(w_i B / 2^32), i = x, y, z
//   order of the block sets  (19, t, 0, 0): ordering number floor(w0 40320 / 2^32)
//                            of 0..7 in lexicographic order
//   cell set of step k       (20, t, block b, k / 10): bits 3 (k mod 10) .. +2 of w0
//   attempt of step k        (21, t, tile G = b (B/8)^3 + g, k / 2): words
//                            2 (k & 1), 2 (k & 1) + 1 as (wa, wb): site r = wa >> 27
//                            of the cell's 32 fcc sites (x fastest), neighbour
//                            floor((wa mod 2^27) 12 / 2^27), uniform u = wb
//   initial state            (16, 0, site s, 0): B iff w0 < floor(c 2^32)
#include <hip/hip_runtime.h>

#include <math.h>
#include <new>
#include <stdio.h>
#include <string.h>

#include "kmc.h"
#include "kpz_device.h"

namespace {

using kpzdev::philox;
using kpzdev::philox_v;
using kpzdev::U4;

constexpr uint32_t TAG_INIT = 16, TAG_ORIGIN = 18, TAG_ORDER = 19, TAG_SET = 20, TAG_STEP = 21;
constexpr int STEPS = 256;          // fcc sites per 8^3 tile: single-hit steps per block turn
constexpr uint32_t MOVE_SLOTS = 64;  // accepted-jump counters (workspace words 0..63)
constexpr uint32_t COUNT_OFF = 64;   // B and bond counts (workspace words 64, 65)
constexpr uint32_t COUNT_BLOCKS = 1024;

struct PhaseArgs {
    uint8_t *occ;
    unsigned long long *moves;
    unsigned long long T[13];       // T[d] = floor(exp(-d eps) 2^32), T[0] = 2^32
    uint32_t L, nbh;                // lattice edge (power of two); blocks per axis / 2
    uint32_t seed_lo, seed_hi, t, phase;
    uint32_t xcd;                   // 1: XCD-aware work-group -> block map
};

// Ordering number idx (0 <= idx < 8!) of the permutations of 0..7 in
// lexicographic order -> element at position `phase`.
__device__ __forceinline__ uint32_t order_at(uint32_t idx, uint32_t phase)
{
    uint32_t pool = 0x76543210u;    // remaining elements, one nibble each
    uint32_t f = 5040;              // 7!
    uint32_t v = 0;
    for (uint32_t i = 0; i < 8; ++i) {
        const uint32_t pick = idx / f;
        idx -= pick * f;
        v = (pool >> (4 * pick)) & 15u;
        // drop nibble `pick`
        const uint32_t lo = pool & ((1u << (4 * pick)) - 1u);
        const uint32_t hi = pick < 7 ? (pool >> (4 * pick + 4)) << (4 * pick) : 0u;
        pool = lo | hi;
        if (i == phase) break;
        f = i < 7 ? f / (7 - i) : 1;
    }
    return v;
}

// Components + 1 of the twelve neighbour offsets (numbering of kmc.h), two
// bits per neighbour: field nb at bits 2 nb .. 2 nb + 1.
constexpr uint32_t pack2(const int (&v)[12])
{
    uint32_t r = 0;
    for (int k = 0; k < 12; ++k) r |= (uint32_t)v[k] << (2 * k);
    return r;
}
constexpr int NBX1[12] = {2, 2, 0, 0, 2, 2, 0, 0, 1, 1, 1, 1};
constexpr int NBY1[12] = {2, 0, 2, 0, 1, 1, 1, 1, 2, 2, 0, 0};
constexpr int NBZ1[12] = {1, 1, 1, 1, 2, 0, 2, 0, 2, 0, 2, 0};
constexpr uint32_t CXP = pack2(NBX1), CYP = pack2(NBY1), CZP = pack2(NBZ1);

// Number of B among the twelve neighbours of LDS position p + S^2 + S (the
// base p is the position minus S^2 + S, so that every offset is positive
// and folds into the LDS instruction).
template <int S>
__device__ __forceinline__ uint32_t sum12(const uint8_t *p)
{
    constexpr int Z = S * S + S;
    return (uint32_t)p[Z + 1 + S] + p[Z + 1 - S] + p[Z - 1 + S] + p[Z - 1 - S] +
           p[Z + 1 + S * S] + p[Z + 1 - S * S] + p[Z - 1 + S * S] + p[Z - 1 - S * S] +
           p[Z + S + S * S] + p[Z + S - S * S] + p[Z - S + S * S] + p[Z - S - S * S];
}

// One attempt of a tile lane: site r = wa >> 27 of the cell whose corner is
// LDS position `corner` (x fastest over the cell's 32 fcc sites, row r / 2:
// y = (r / 2) mod 4, z = r / 8; x = the fcc parity bit + 2 (r mod 2)),
// neighbour floor((wa mod 2^27) 12 / 2^27), uniform u = wb; T[d] is the
// acceptance threshold for n_b - n_e = d (T[0] = 2^32).  Branch-free: the
// 26 reads are issued together and both positions are always rewritten
// (with their own values when rejected).  Returns 1 if a B jumped.  The
// write is seen by the next step's reads of other lanes: LDS work of one
// wave completes in issue order, and the fences keep the compiler from
// moving memory operations across.
template <int S>
__device__ __forceinline__ uint32_t attempt(uint8_t *lds, int corner, uint32_t par0, uint32_t wa,
                                            uint32_t wb, const unsigned long long *T)
{
    constexpr int Z = S * S + S;
    const uint32_t x4 = wa >> 28;                        // y + 4 z of the row
    const uint32_t ly = x4 & 3u, lz = wa >> 30;
    const uint32_t lx = ((par0 ^ x4 ^ lz) & 1u) | ((wa >> 26) & 2u);
    const int ai = corner + (int)(lx + ly * S + lz * (S * S));
    const uint32_t m = wa & 0x7FFFFFFu;
    const uint32_t sh = ((m + (m << 1)) >> 25) << 1;     // 2 floor(12 m / 2^27)
    const uint32_t X = (CXP >> sh) & 3u, Y = (CYP >> sh) & 3u, Zc = (CZP >> sh) & 3u;
    const int af = ai + (int)(X + Y * S + Zc * (S * S)) - (1 + S + S * S);
    // bases below 2^16: the constant offsets fold into the instructions
    uint8_t *pi = lds + ((uint32_t)(ai - Z) & 0xFFFFu);
    uint8_t *pf = lds + ((uint32_t)(af - Z) & 0xFFFFu);
    const uint32_t oi = pi[Z], of = pf[Z];
    const int si = (int)sum12<S>(pi), sf = (int)sum12<S>(pf);
    int d = oi ? (si - sf + 1) : (sf - si + 1);       // n_b - n_e when oi != of
    d = d < 0 ? 0 : (d > 12 ? 12 : d);
    const uint32_t acc = (uint32_t)(oi != of) & (uint32_t)((unsigned long long)wb < T[d]);
    pi[Z] = (uint8_t)(acc ? of : oi);
    pf[Z] = (uint8_t)(acc ? oi : of);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    return acc;
}

// Cell corners (LDS offsets within a tile) of steps 2j and 2j + 1 of block b,
// in the low and high half-word; the two steps share their cell-set draw
// (k / 10).
template <int S>
__device__ __forceinline__ uint32_t cell_pair(const PhaseArgs &a, uint32_t b, uint32_t j)
{
    const uint32_t k0 = 2 * j;
    const uint32_t sw = philox(b, 0u, a.t, (TAG_SET << 24) | (k0 / 10), a.seed_lo, a.seed_hi).x;
    uint32_t v = 0;
    for (uint32_t h = 0; h < 2; ++h) {
        const uint32_t sc = (sw >> (3 * ((k0 + h) % 10))) & 7u;
        v |= (4u * ((sc & 1u) + ((sc >> 1) & 1u) * S + (sc >> 2) * S * S)) << (16 * h);
    }
    return v;
}

template <int B, int NTHREADS>
__global__ __launch_bounds__(NTHREADS) void kmc_phase_kernel(PhaseArgs a)
{
    constexpr int S = B + 4;                // LDS cube edge: block + halo 2 on each side
    constexpr int NT = B / 8;               // tiles per block edge
    constexpr int TPB = NT * NT * NT;       // tiles (attempting lanes) per block, <= 64
    constexpr int H = S / 2;                // fcc sites per LDS row
    constexpr int SO = B + 2;               // written-back edge: block + halo 1
    constexpr int HO = SO / 2;
    static_assert(TPB <= 64, "all attempting lanes must sit in wave 0");
    __shared__ uint8_t lds[S * S * S];
    __shared__ unsigned long long Ts[13];

    const uint32_t L = a.L, Lm = L - 1, half = L >> 1;
    // per-MCS draws (uniform over the launch)
    const U4 wo = philox(0u, 0u, a.t, TAG_ORIGIN << 24, a.seed_lo, a.seed_hi);
    const uint32_t ox = (uint32_t)(((uint64_t)wo.x * B) >> 32);
    const uint32_t oy = (uint32_t)(((uint64_t)wo.y * B) >> 32);
    const uint32_t oz = (uint32_t)(((uint64_t)wo.z * B) >> 32);
    const uint32_t ordw = philox(0u, 0u, a.t, TAG_ORDER << 24, a.seed_lo, a.seed_hi).x;
    const uint32_t c = order_at((uint32_t)(((uint64_t)ordw * 40320u) >> 32), a.phase);

    // work-group -> block of set c
    const uint32_t nset = a.nbh * a.nbh * a.nbh;
    uint32_t j = blockIdx.x;
    if (a.xcd) j = (j & 7u) * (nset >> 3) + (j >> 3);
    const uint32_t jx = j % a.nbh, jy = (j / a.nbh) % a.nbh, jz = j / (a.nbh * a.nbh);
    const uint32_t nb = 2 * a.nbh;
    const uint32_t bx = 2 * jx + (c & 1u), by = 2 * jy + ((c >> 1) & 1u), bz = 2 * jz + (c >> 2);
    const uint32_t b = (bz * nb + by) * nb + bx;
    const uint32_t X0 = ox + bx * B, Y0 = oy + by * B, Z0 = oz + bz * B;   // < 2L

    if (threadIdx.x < 13) Ts[threadIdx.x] = a.T[threadIdx.x];
    // load block + halo 2 (fcc positions only)
    constexpr int NIT = (S * S + NTHREADS - 1) / NTHREADS;   // LDS rows per thread
    const uint32_t WL = L >> 3, WLm = WL - 1;                 // words per compact row
    uint32_t keep0[NIT], keep4[NIT], keep5[NIT];              // edge words, for the write-back
    if constexpr (TPB == 64) {
        // LDS rows of 36 positions (18 sites), row tid + NTHREADS it: the
        // row's 18 compact bytes lie in 6 aligned global words; realign them
        // and spread each pair of sites over one LDS dword.  Straight-line
        // over all rows (the last row repeated where the count runs out) so
        // that every load is in flight at once.
        const uint32_t *occw = (const uint32_t *)a.occ;
#pragma unroll
        for (int it = 0; it < NIT; ++it) {
            const uint32_t row = min(threadIdx.x + it * NTHREADS, (uint32_t)(S * S - 1));
            const uint32_t ly = row % S, lz = row / S;
            const uint32_t gy = (Y0 + L - 2 + ly) & Lm, gz = (Z0 + L - 2 + lz) & Lm;
            const uint32_t lxo = (X0 + gy + gz) & 1u;
            const uint32_t k0 = ((X0 + L - 2 + lxo) & Lm) >> 1;
            const uint32_t q = k0 >> 2, o = k0 & 3u;
            const uint32_t *rw = occw + ((uint64_t)gz * L + gy) * WL;
            uint32_t w[6], r[5];
#pragma unroll
            for (int i = 0; i < 6; ++i) w[i] = rw[(q + i) & WLm];
            keep0[it] = w[0];
            keep4[it] = w[4];
            keep5[it] = w[5];
#pragma unroll
            for (int i = 0; i < 5; ++i) r[i] = __builtin_amdgcn_alignbyte(w[i + 1], w[i], o);
            const uint32_t se = lxo ? 0x010C000Cu : 0x0C010C00u;
            const uint32_t so = se + (lxo ? 0x02000200u : 0x00020002u);
            uint32_t *dst = (uint32_t *)(lds + (lz * S + ly) * S);
#pragma unroll
            for (int j = 0; j < H / 2; ++j)
                dst[j] = __builtin_amdgcn_perm(0u, r[j >> 1], (j & 1) ? so : se);
        }
    } else {
        for (uint32_t e = threadIdx.x; e < (uint32_t)(S * S * H); e += NTHREADS) {
            const uint32_t row = e / H, k = e - row * H;
            const uint32_t ly = row % S, lz = row / S;
            const uint32_t gy = (Y0 + L - 2 + ly) & Lm, gz = (Z0 + L - 2 + lz) & Lm;
            const uint32_t lxo = (X0 + gy + gz) & 1u;
            const uint32_t gx = (X0 + L - 2 + lxo + 2 * k) & Lm;
            const uint64_t gi = ((uint64_t)gz * L + gy) * half + (gx >> 1);
            lds[(lz * S + ly) * S + lxo + 2 * k] = a.occ[gi];
        }
    }
    __syncthreads();

    uint32_t mv = 0;
    const uint32_t par0 = (ox + oy + oz) & 1u;
    if constexpr (TPB == 64) {
        // 32^3 blocks: wave 0 makes every attempt of the block, one lane per
        // tile; the other waves only load and store.
        if (threadIdx.x < 64) {
            const uint32_t g = threadIdx.x;
            const uint32_t tx = g % NT, ty = (g / NT) % NT, tz = g / (NT * NT);
            const uint64_t G = (uint64_t)b * TPB + g;
            const int tbase = (int)(((8 * tz + 2) * S + (8 * ty + 2)) * S + 8 * tx + 2);
            // the 128 pairs of cell corners in two registers: lane l holds
            // pairs l and 64 + l; each is read uniformly with v_readlane (no
            // LDS read, whose wait would also wait for the last step's writes)
            static_assert(STEPS == 256, "two 64-lane tables of step pairs");
            const uint32_t ct[2] = {cell_pair<S>(a, b, g), cell_pair<S>(a, b, 64u + g)};
            U4 w = philox_v((uint32_t)G, (uint32_t)(G >> 32), a.t, TAG_STEP << 24, a.seed_lo,
                             a.seed_hi);
#pragma unroll
            for (uint32_t hv = 0; hv < 2; ++hv) {
                for (uint32_t q = 0; q < 64; ++q) {
                    const uint32_t kk = 64 * hv + q;
                    // draws of the next pair of steps, independent of the
                    // lattice: their arithmetic fills the LDS latency of this pair
                    const U4 wn = philox_v((uint32_t)G, (uint32_t)(G >> 32), a.t,
                                            (TAG_STEP << 24) | (kk + 1), a.seed_lo, a.seed_hi);
                    const uint32_t cw = (uint32_t)__builtin_amdgcn_readlane((int)ct[hv], (int)q);
                    mv += attempt<S>(lds, tbase + (int)(cw & 0xFFFFu), par0, w.x, w.y, Ts);
                    mv += attempt<S>(lds, tbase + (int)(cw >> 16), par0, w.z, w.w, Ts);
                    w = wn;
                }
            }
        }
    } else {
        // smaller blocks (small lattices): TPB lanes of wave 0
        if (threadIdx.x < TPB) {
            const uint32_t g = threadIdx.x;
            const uint32_t tx = g % NT, ty = (g / NT) % NT, tz = g / (NT * NT);
            const uint64_t G = (uint64_t)b * TPB + g;
            const int tbase = (int)(((8 * tz + 2) * S + (8 * ty + 2)) * S + 8 * tx + 2);
            uint32_t sw = 0;
            U4 w = philox_v((uint32_t)G, (uint32_t)(G >> 32), a.t, TAG_STEP << 24, a.seed_lo,
                             a.seed_hi);
            for (uint32_t kk = 0; kk < STEPS / 2; ++kk) {
                const U4 wn = philox_v((uint32_t)G, (uint32_t)(G >> 32), a.t,
                                        (TAG_STEP << 24) | (kk + 1), a.seed_lo, a.seed_hi);
#pragma unroll
                for (uint32_t h = 0; h < 2; ++h) {
                    const uint32_t k = 2 * kk + h;
                    if (k % 10 == 0)
                        sw = philox(b, 0u, a.t, (TAG_SET << 24) | (k / 10), a.seed_lo,
                                    a.seed_hi).x;
                    const uint32_t sc = (sw >> (3 * (k % 10))) & 7u;
                    const int cell =
                        4 * (int)((sc & 1u) + ((sc >> 1) & 1u) * S + (sc >> 2) * S * S);
                    mv += attempt<S>(lds, tbase + cell, par0, h ? w.z : w.x, h ? w.w : w.y, Ts);
                }
                w = wn;
            }
        }
    }
    __syncthreads();

    // write back block + halo 1 (the halo may have received jumps)
    if constexpr (TPB == 64) {
        // rows -1..B in y and z, each by the thread that loaded it: the row's
        // whole loaded segment (x = -2..B+1) goes back in the same 6 aligned
        // words; the bytes of the edge words outside the segment get the
        // values loaded before.  No other work-group of the launch writes any
        // byte of these words, nor reads one our block changes: blocks of one
        // set are 32 positions apart and the words reach at most 8 positions
        // beyond the segment.
        uint32_t *occw = (uint32_t *)a.occ;
#pragma unroll
        for (int it = 0; it < NIT; ++it) {
            const uint32_t row = threadIdx.x + it * NTHREADS;
            const uint32_t ly = row % S, lz = row / S;
            if (row >= (uint32_t)(S * S) || ly < 1 || ly > S - 2 || lz < 1 || lz > S - 2) continue;
            const uint32_t gy = (Y0 + L - 2 + ly) & Lm, gz = (Z0 + L - 2 + lz) & Lm;
            const uint32_t lxo = (X0 + gy + gz) & 1u;
            const uint32_t k0 = ((X0 + L - 2 + lxo) & Lm) >> 1;
            const uint32_t q = k0 >> 2, o = k0 & 3u;
            uint32_t *rw = occw + ((uint64_t)gz * L + gy) * WL;
            const uint32_t *src = (const uint32_t *)(lds + (lz * S + ly) * S);
            uint32_t dd[H / 2 + 1], seg[6];
#pragma unroll
            for (int j = 0; j < H / 2; ++j) dd[j] = src[j];
            dd[H / 2] = 0;
            const uint32_t sel = lxo ? 0x07050301u : 0x06040200u;
#pragma unroll
            for (int m = 0; m < 5; ++m) seg[m] = __builtin_amdgcn_perm(dd[2 * m + 1], dd[2 * m], sel);
            seg[5] = 0;
            // window word i holds segment bytes 4 i - o .. 4 i - o + 3
            const uint32_t sh = (4u - o) & 3u;
            uint32_t out[6];
#pragma unroll
            for (int i = 0; i < 6; ++i) {
                const uint32_t lo = o ? (i ? seg[i - 1] : 0u) : seg[i];
                out[i] = __builtin_amdgcn_alignbyte(seg[i], lo, sh);
            }
            const uint32_t m0 = 0xFFFFFFFFu << (8 * o);
            rw[q & WLm] = (out[0] & m0) | (keep0[it] & ~m0);
#pragma unroll
            for (int i = 1; i < 4; ++i) rw[(q + i) & WLm] = out[i];
            // bytes of words 4 and 5 inside the segment: below o + 2 and o - 2
            const uint32_t m4 = o < 2 ? (1u << (8 * (o + 2))) - 1u : 0xFFFFFFFFu;
            rw[(q + 4) & WLm] = (out[4] & m4) | (keep4[it] & ~m4);
            if (o == 3) rw[(q + 5) & WLm] = (out[5] & 0xFFu) | (keep5[it] & ~0xFFu);
        }
    } else {
        for (uint32_t e = threadIdx.x; e < (uint32_t)(SO * SO * HO); e += NTHREADS) {
            const uint32_t row = e / HO, k = e - row * HO;
            const uint32_t ly = row % SO, lz = row / SO;
            const uint32_t gy = (Y0 + L - 1 + ly) & Lm, gz = (Z0 + L - 1 + lz) & Lm;
            const uint32_t lxo = (X0 + 1 + gy + gz) & 1u;
            const uint32_t gx = (X0 + L - 1 + lxo + 2 * k) & Lm;
            const uint64_t gi = ((uint64_t)gz * L + gy) * half + (gx >> 1);
            a.occ[gi] = lds[((lz + 1) * S + ly + 1) * S + 1 + lxo + 2 * k];
        }
    }

    // accepted jumps: wave 0 holds them all
    if (threadIdx.x < 64) {
        for (int off = 32; off > 0; off >>= 1) mv += __shfl_xor(mv, off, 64);
        // spread over MOVE_SLOTS counters: same-address atomics from every
        // work-group of a launch would serialise in L2
        if (threadIdx.x == 0 && mv)
            atomicAdd(a.moves + (blockIdx.x & (MOVE_SLOTS - 1)), (unsigned long long)mv);
    }
}

__global__ void kmc_init_kernel(uint8_t *occ, uint64_t n, unsigned long long C, uint32_t seed_lo,
                                uint32_t seed_hi)
{
    for (uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; s < n;
         s += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t w0 = philox((uint32_t)s, (uint32_t)(s >> 32), 0u, TAG_INIT << 24, seed_lo,
                                   seed_hi).x;
        occ[s] = (unsigned long long)w0 < C ? 1 : 0;
    }
}

__global__ void kmc_fill_kernel(unsigned long long *p, uint32_t n, unsigned long long v)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// res[0] += number of B, res[1] += B-B bonds, each bond counted once through
// the six neighbours (+1,+1,0) (+1,-1,0) (+1,0,+1) (+1,0,-1) (0,+1,+1)
// (0,+1,-1).  A thread takes one compact word (4 sites x = 2(4w + j) + p of
// row (y, z), p = (y + z) mod 2).  The x+1 neighbours lie in rows of the
// other parity at compact index 4w + j + p: bytes p.. of words w, w + 1 of
// those rows; the (0, +1, +-1) neighbours lie at index 4w + j of rows of the
// same parity.  Sites are bytes 0/1, so a bond is a byte of (own & other)
// and the byte sums never carry (at most 6 per byte).
__device__ __forceinline__ uint32_t byte_sum(uint32_t v) { return (v * 0x01010101u) >> 24; }

__global__ void kmc_count_kernel(const uint8_t *occ, uint32_t L, uint32_t log2L,
                                 unsigned long long *res)
{
    const uint32_t *occw = (const uint32_t *)occ;
    const uint32_t Lm = L - 1, WL = L >> 3, WLm = WL - 1;
    const uint64_t n = (uint64_t)L * L * WL;            // words
    unsigned long long nb = 0, bonds = 0;
    for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
         e += (uint64_t)gridDim.x * blockDim.x) {
        // L is a power of two: rows and planes by shifts
        const uint32_t row = (uint32_t)(e >> (log2L - 3));
        const uint32_t w = (uint32_t)e & WLm;
        const uint32_t y = row & Lm, z = row >> log2L;
        const uint32_t p = (y + z) & 1u;
        const uint32_t own = occw[e];
        const uint32_t yp = (y + 1) & Lm, ym = (y + Lm) & Lm, zp = (z + 1) & Lm, zm = (z + Lm) & Lm;
        const uint32_t w1 = (w + 1) & WLm;
        const uint64_t r1 = ((uint64_t)z * L + yp) * WL, r2 = ((uint64_t)z * L + ym) * WL;
        const uint64_t r3 = ((uint64_t)zp * L + y) * WL, r4 = ((uint64_t)zm * L + y) * WL;
        const uint64_t r5 = ((uint64_t)zp * L + yp) * WL, r6 = ((uint64_t)zm * L + yp) * WL;
        const uint32_t a = __builtin_amdgcn_alignbyte(occw[r1 + w1], occw[r1 + w], p);
        const uint32_t b = __builtin_amdgcn_alignbyte(occw[r2 + w1], occw[r2 + w], p);
        const uint32_t c = __builtin_amdgcn_alignbyte(occw[r3 + w1], occw[r3 + w], p);
        const uint32_t d = __builtin_amdgcn_alignbyte(occw[r4 + w1], occw[r4 + w], p);
        const uint32_t f = occw[r5 + w], g = occw[r6 + w];
        const uint32_t m = (own & a) + (own & b) + (own & c) + (own & d) + (own & f) + (own & g);
        nb += byte_sum(own);
        bonds += byte_sum(m);
    }
    for (int off = 32; off > 0; off >>= 1) {
        nb += __shfl_xor(nb, off, 64);
        bonds += __shfl_xor(bonds, off, 64);
    }
    // one atomic pair per work-group (at most COUNT_BLOCKS of them)
    __shared__ unsigned long long part[2][4];
    if ((threadIdx.x & 63) == 0) {
        part[0][threadIdx.x >> 6] = nb;
        part[1][threadIdx.x >> 6] = bonds;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long a = 0, b = 0;
        for (uint32_t i = 0; i < blockDim.x / 64; ++i) {
            a += part[0][i];
            b += part[1][i];
        }
        if (a) atomicAdd(&res[0], a);
        if (b) atomicAdd(&res[1], b);
    }
}

}  // namespace

// ================================================================ host

struct kmc_sim {
    kmc_params prm;
    int32_t B;
    uint8_t *occ;
    unsigned long long *ws;         // [0, 64) accepted-jump slots, [64] n_b, [65] bonds
    hipStream_t stream;
    int64_t t;
    unsigned long long T[13];
    char err[256];
};

namespace {

constexpr size_t KMC_WS = 8 * (COUNT_OFF + 2);

kpz_status kmc_resolve(const kmc_params *p, int32_t *B)
{
    if (!p) return KPZ_EINVAL;
    const int64_t L = p->L;
    if (L < 16 || L > 2048 || (L & (L - 1))) return KPZ_EINVAL;
    if (!(p->c >= 0.0 && p->c <= 1.0) || !(p->eps >= 0.0) || !isfinite(p->eps)) return KPZ_EINVAL;
    if (p->flags != 0) return KPZ_EINVAL;
    int32_t b = p->block;
    if (b == 0) b = L >= 64 ? 32 : (L >= 32 ? 16 : 8);
    if (b != 8 && b != 16 && b != 32) return KPZ_EINVAL;
    if (L / b < 2) return KPZ_EINVAL;
    *B = b;
    return KPZ_OK;
}

kpz_status kmc_fail(kmc_sim *s, hipError_t e, const char *what)
{
    if (s) snprintf(s->err, sizeof s->err, "%s: %s", what, hipGetErrorString(e));
    return KPZ_EHIP;
}

unsigned long long prob_threshold(double prob)
{
    if (prob >= 1.0) return 1ull << 32;
    if (prob <= 0.0) return 0;
    return (unsigned long long)(prob * 4294967296.0);
}

}  // namespace

extern "C" {

kpz_status kmc_workspace_bytes(const kmc_params *p, size_t *bytes)
{
    int32_t B;
    const kpz_status st = kmc_resolve(p, &B);
    if (st != KPZ_OK) return st;
    if (!bytes) return KPZ_EINVAL;
    *bytes = KMC_WS;
    return KPZ_OK;
}

kpz_status kmc_init(kmc_sim **out, const kmc_params *p, uint8_t *d_occ, size_t occ_bytes,
                    void *d_ws, size_t ws_bytes, void *stream)
{
    if (!out) return KPZ_EINVAL;
    *out = nullptr;
    int32_t B;
    const kpz_status st = kmc_resolve(p, &B);
    if (st != KPZ_OK) return st;
    if (!d_occ || !d_ws || ((uintptr_t)d_occ & 3u) || ((uintptr_t)d_ws & 7u)) return KPZ_EINVAL;
    const uint64_t n = (uint64_t)p->L * p->L * p->L / 2;
    if (occ_bytes < n || ws_bytes < KMC_WS) return KPZ_ESIZE;
    kmc_sim *s = new (std::nothrow) kmc_sim();
    if (!s) return KPZ_EINVAL;
    s->prm = *p;
    s->B = B;
    s->occ = d_occ;
    s->ws = (unsigned long long *)d_ws;
    s->stream = (hipStream_t)stream;
    s->t = 0;
    s->err[0] = 0;
    s->T[0] = 1ull << 32;
    for (int d = 1; d <= 12; ++d) s->T[d] = prob_threshold(exp(-(double)d * p->eps));
    const unsigned long long C = prob_threshold(p->c);
    const uint32_t grid = (uint32_t)((n + 255) / 256 < 16384 ? (n + 255) / 256 : 16384);
    hipLaunchKernelGGL(kmc_init_kernel, dim3(grid), dim3(256), 0, s->stream, d_occ, n, C,
                       (uint32_t)p->seed, (uint32_t)(p->seed >> 32));
    hipLaunchKernelGGL(kmc_fill_kernel, dim3(1), dim3(128), 0, s->stream, s->ws, COUNT_OFF + 2,
                       0ull);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        kmc_fail(s, e, "kmc_init launch");
        delete s;
        return KPZ_EHIP;
    }
    *out = s;
    return KPZ_OK;
}

kpz_status kmc_sweep(kmc_sim *s, int32_t n_mcs)
{
    if (!s || n_mcs < 0) return KPZ_EINVAL;
    if (n_mcs == 0) return KPZ_OK;
    if (s->t + n_mcs > 0xFFFFFFFFll) return KPZ_ERANGE;
    PhaseArgs a;
    a.occ = s->occ;
    a.moves = s->ws;
    memcpy(a.T, s->T, sizeof a.T);
    a.L = (uint32_t)s->prm.L;
    a.nbh = a.L / (2u * (uint32_t)s->B);
    a.seed_lo = (uint32_t)s->prm.seed;
    a.seed_hi = (uint32_t)(s->prm.seed >> 32);
    const uint32_t nset = a.nbh * a.nbh * a.nbh;
    a.xcd = (nset % 8 == 0) ? 1u : 0u;
    for (int32_t m = 0; m < n_mcs; ++m) {
        a.t = (uint32_t)(s->t + m);
        for (uint32_t ph = 0; ph < 8; ++ph) {
            a.phase = ph;
            switch (s->B) {
            case 8: hipLaunchKernelGGL((kmc_phase_kernel<8, 64>), dim3(nset), dim3(64), 0, s->stream, a); break;
            case 16: hipLaunchKernelGGL((kmc_phase_kernel<16, 64>), dim3(nset), dim3(64), 0, s->stream, a); break;
            default: hipLaunchKernelGGL((kmc_phase_kernel<32, 256>), dim3(nset), dim3(256), 0, s->stream, a); break;
            }
        }
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return kmc_fail(s, e, "kmc_sweep launch");
    }
    s->t += n_mcs;
    return KPZ_OK;
}

kpz_status kmc_counts(kmc_sim *s, int64_t *n_b, int64_t *bonds)
{
    if (!s) return KPZ_EINVAL;
    const uint32_t L = (uint32_t)s->prm.L;
    const uint64_t n = (uint64_t)L * L * L / 2;
    const uint32_t grid = (uint32_t)((n / 4 + 255) / 256 < COUNT_BLOCKS ? (n / 4 + 255) / 256
                                                                         : COUNT_BLOCKS);
    hipLaunchKernelGGL(kmc_fill_kernel, dim3(1), dim3(64), 0, s->stream, s->ws + COUNT_OFF, 2u,
                       0ull);
    hipLaunchKernelGGL(kmc_count_kernel, dim3(grid), dim3(256), 0, s->stream,
                       (const uint8_t *)s->occ, L, (uint32_t)__builtin_ctz(L), s->ws + COUNT_OFF);
    hipError_t e = hipGetLastError();
    unsigned long long r[2] = {0, 0};
    if (e == hipSuccess)
        e = hipMemcpyAsync(r, s->ws + COUNT_OFF, sizeof r, hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return kmc_fail(s, e, "kmc_counts");
    if (n_b) *n_b = (int64_t)r[0];
    if (bonds) *bonds = (int64_t)r[1];
    return KPZ_OK;
}

kpz_status kmc_get_state(kmc_sim *s, int64_t *t, int64_t *moves)
{
    if (!s) return KPZ_EINVAL;
    unsigned long long slots[MOVE_SLOTS];
    hipError_t e = hipMemcpyAsync(slots, s->ws, sizeof slots, hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return kmc_fail(s, e, "kmc_get_state");
    unsigned long long m = 0;
    for (uint32_t i = 0; i < MOVE_SLOTS; ++i) m += slots[i];
    if (t) *t = s->t;
    if (moves) *moves = (int64_t)m;
    return KPZ_OK;
}

kpz_status kmc_set_state(kmc_sim *s, int64_t t, int64_t moves)
{
    if (!s || t < 0 || t > 0xFFFFFFFFll || moves < 0) return KPZ_EINVAL;
    hipLaunchKernelGGL(kmc_fill_kernel, dim3(1), dim3(64), 0, s->stream, s->ws, MOVE_SLOTS, 0ull);
    hipLaunchKernelGGL(kmc_fill_kernel, dim3(1), dim3(64), 0, s->stream, s->ws, 1u,
                       (unsigned long long)moves);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return kmc_fail(s, e, "kmc_set_state");
    s->t = t;
    return KPZ_OK;
}

void kmc_destroy(kmc_sim *s) { delete s; }

const char *kmc_last_error(const kmc_sim *s) { return s ? s->err : ""; }

}  // extern "C"
