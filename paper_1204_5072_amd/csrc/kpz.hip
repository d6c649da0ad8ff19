// kpz.hip -- gfx950 kernels and the C ABI (include/kpz.h) for the Monte
// Carlo sweep of the 2+1-d KPZ octahedron model.
//
// Paper: Kelling, Odor, Nagy, Schulz, Heinig, "Comparison of different
// parallel implementations of the 2+1-dimensional KPZ model and the
// 3-dimensional KMC model".  Sec. 2.1 (slopes, eq. "rule", heights, eq.
// "Wdef"), Sec. 3 (dead-border and double-tiling decomposition, the two
// layers), Sec. 3.1 (single-hit double tiling at the work-group layer, one
// domain set chosen collectively per work-group and step, several domains
// per work-item).
//
// Kernels (the hot path)
//   kpz_init_kernel          flat start, HBM write stream
//   kpz_sweep_kernel         one MCS: one wave64 per dead-border block, the
//                            block held in registers as bit planes (the
//                            step code is in kpz_slice.h); 16 single-hit
//                            steps; two-buffer store rotated by the origin
//   kpz_row_moments_kernel   per-row (sum, sum of squares) of the x-prefix
//                            heights, a lane group per row (a wave for long
//                            rows), HBM read stream
//   kpz_finalize_kernel      column-0 prefix, 128-bit totals, flip counters,
//                            one work-group, one pass over the row sums
// and around it: the in-place merge, device-layer double tiling
// (kpz_dt_kernel, one launch per block set), the batched ensemble and the
// job pool (kpz_batch_round_kernel), block residency below one MCS.
//
// Random numbers: Philox4x32-7 (Salmon et al., SC'11) keyed by the seed,
// counter (idx_lo, idx_hi, t, tag << 24 | sub).  Tile row ty of block b is
// cut into row groups of 32 tiles, G = (b nty + ty) nqx + tx / 32, and tile
// tx owns bit pi(tx) = 8 (tx mod 4) + (tx mod 32) / 4 of every word drawn for
// its group:
//   origin  (ORIGIN, t, res): ox = w0 Bx >> 32, oy = w1 By >> 32
//   sets    (SET, t, b, res): step k takes bits 2k..2k+1 of w0
//   sites   (SITE, t, G, k/2): rx from word 2 (k mod 2), ry from the next
//   accept  bit j (most significant first) of the 32-bit uniform: word
//           k mod 4 of (ACC1, t, G, 4 (k/4) + j) for j < 4, word j mod 4 of
//           (ACC2, t, G, 8k + j/4 - 1) beyond; the kernel compares bit by
//           bit and draws the later words only while some tile is undecided.

#include <hip/hip_runtime.h>
#include <type_traits>

#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <utility>
#include <vector>

#include "kpz.h"
#include "kpz_device.h"
#include "kpz_slice.h"

namespace {

using kpzdev::philox;
using kpzdev::philox_v;
using kpzdev::LATTICE_ROUNDS;
using kpzdev::U4;

constexpr uint32_t TAG_ORIGIN = 1, TAG_SET = 2, TAG_SITE = 3, TAG_ACC1 = 4, TAG_ACC2 = 5;
constexpr int NSLOTS = 1024;          // flip-counter slots in the workspace
constexpr int WS_HEADER = 256;        // results area at the start of the workspace
constexpr int TILE = 4;               // tile edge (sites)
constexpr uint32_t GROUP_SITES = 128; // sites of a row group (32 tiles, one bit each per plane word)
// Staged sweep loads: a block row spans at most U = floor((nw + 7) / 4)
// 16-byte units; R = floor(64 / U) rows per load instruction, so the nty
// tile rows of one row offset take ceil(nty / R) <= STAGE_NC instructions
// for every valid shape (at most 64 lanes: By = 4 nty, nw <= 8 nqx,
// nty nqx <= 64), and a block takes By U <= STAGE_UNITS units of LDS.
constexpr uint32_t STAGE_UNITS = 768;
constexpr uint32_t STAGE_NC = 4;
// global and LDS pointers of the global-to-LDS load
typedef const __attribute__((address_space(1))) void *gptr_t;
typedef __attribute__((address_space(3))) void *lptr_t;
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
// s_waitcnt vmcnt(0) (expcnt and lgkmcnt not waited for)
constexpr int WAIT_VMCNT0 = 0x0F70;

// ---------------------------------------------------------------- init

__global__ void kpz_init_kernel(uint4 *words4, uint64_t n4, uint32_t w4)
{
    // words4: the lattice as uint4 (4 words); a row has w4 = W/4 of them
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n4;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t v = ((i / w4) & 1) ? 0xCCCCCCCCu : 0x33333333u;
        words4[i] = make_uint4(v, v, v, v);
    }
}

__global__ void kpz_init_small_kernel(uint32_t *words, uint32_t n, uint32_t w)
{
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        words[i] = ((i / w) & 1) ? 0xCCCCCCCCu : 0x33333333u;
}

__global__ void kpz_fill_counters_kernel(long long *slots, long long first)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < NSLOTS) slots[i] = i == 0 ? first : 0;
}

// --------------------------------------------------------------- sweep

struct SweepArgs {
    uint32_t *words;             // output lattice (and input when src == words)
    const uint32_t *src;         // input lattice
    uint32_t *side;              // [2][L][nbx]: straddling-word parts (left edge, right edge)
    unsigned long long *slots;   // flip counters
    uint32_t L, W;               // size, words per row
    uint32_t Bx, By;             // block shape
    uint32_t nbx, nby;           // blocks per direction
    uint32_t nw;                 // words per block row (Bx / 16)
    uint32_t nqx;                // row groups per tile row (Bx / 128, at least 1)
    uint32_t ntg, nwg;           // tiles and lattice words per row group
    uint32_t nty, mnty;          // tile rows per block (By / 4); ceil(2^16 / nty)
    // staged sweep loads: units per block row floor((nw + 7) / 4), ceil(2^16
    // / su_u), rows per load instruction floor(64 / su_u), load instructions
    // per row offset ceil(nty / su_r), units of LDS per block By su_u
    uint32_t su_u, su_m, su_r, su_nc, su;
    uint32_t seed_lo, seed_hi;
    uint32_t t;
    uint32_t res;                // residency of MCS t (origin move), 0 .. moves - 1
    uint32_t nsteps;             // single-hit steps per residency (16 / moves)
    uint32_t slot_mask;          // flip-counter slots - 1 (power of two)
    uint32_t acc;                // 1 unless P = 2^32 and Q = 0 (acceptance draws needed)
    // Two-buffer mode (db = 1): the launch reads src and writes words, a
    // different buffer.  src is stored rotated by s_in sites (word w of a row
    // holds sites 16 w + s_in ..), s_in = (x origin of launch (prev_t,
    // prev_res)) mod 64 when prev_valid, else 0; the output is stored rotated
    // by this launch's x origin mod 64, so every block writes whole words of
    // its own (16-byte aligned for blocks of 64 sites or more) and no word is
    // shared.  db = 0: in place, shared words through the side buffer.
    uint32_t db, prev_valid, prev_t, prev_res;
    uint32_t xcd;                // 1: map work-groups so that consecutive blocks share an XCD
    // ensemble members in two-buffer mode: buffer 0 is `words`, buffer 1 is
    // `alt`; at the start of a call the state is in buffer cur0, rotated as
    // written by launch (prev_t, prev_res) when prev_valid
    uint32_t *alt;
    uint32_t cur0;
    uint64_t P, Q;               // acceptance thresholds over 2^32
    // Device-layer double tiling: 1 when the launch runs a block set together
    // with its diagonal partner set.  The four words at a block's corners in
    // its top row and in the halo row below it are then shared with a
    // diagonal block of the same launch (each changes only its own bits) and
    // are written by atomic xor of the change; every other word stays one
    // block's.
    uint32_t ahead;
};

// Storage rotation of a lattice buffer written in two-buffer mode: the x
// origin of the launch that wrote it, mod 64 (0 for a buffer in the
// documented layout, valid = 0).  Word w of a row then holds sites 16 w + s
// .. 16 w + s + 15 (mod L); with blocks at least 64 sites wide every block
// starts on a 16-byte boundary of the output.
struct Rot {
    uint32_t valid, t, res, Bx, seed_lo, seed_hi;
};

__device__ __forceinline__ uint32_t rot_sites(const Rot &r)
{
    if (!r.valid) return 0u;
    const U4 w = philox<LATTICE_ROUNDS>(r.res, 0u, r.t, TAG_ORIGIN << 24, r.seed_lo, r.seed_hi);
    return (uint32_t)(((uint64_t)w.x * r.Bx) >> 32) & 63u;
}

// Index i + d of a periodic row of W words (i < W, d <= W).
__device__ __forceinline__ uint32_t wrap_add(uint32_t i, uint32_t d, uint32_t W)
{
    const uint32_t j = i + d;
    return j >= W ? j - W : j;
}

// The nwg (1 .. 8) lattice words of a row group whose first site is bit sh2
// of storage word gw of row `row`, realigned so that A[i] holds the group's
// sites 16 i .. 16 i + 15; A[i] = 0 for i >= nwg.  R[i], i <= nwg: storage
// word gw + i as loaded (the words the group shares with its neighbours are
// R[0] and R[nwg]).  VEC (W % 4 == 0): three 16-byte loads of the aligned
// words around the group, the funnel shift chosen by gw mod 4 (uniform).
template <int O>
__device__ __forceinline__ void funnel8(const uint32_t (&v)[12], uint32_t sh2, uint32_t nwg,
                                        uint32_t (&A)[8], uint32_t (&R)[9])
{
#pragma unroll
    for (int i = 0; i < 8; ++i)
        A[i] = (uint32_t)i < nwg ? __builtin_amdgcn_alignbit(v[O + i + 1], v[O + i], sh2) : 0u;
#pragma unroll
    for (int i = 0; i < 9; ++i) R[i] = v[O + i];
}

// The raw words of a row group: VEC, the three aligned 16-byte units from
// word gw - (gw mod 4) on (all three always loaded, so the loads of several
// rows can be issued before the first wait; words beyond the group are
// neighbours' and unused; W >= 4); otherwise the nwg + 1 words gw .. gw + nwg
// (nwg + 1 <= W + 1, so one wrap suffices), zero beyond.
template <bool VEC>
struct GroupRaw {
    uint32_t v[12];
};

template <bool VEC>
__device__ __forceinline__ void load_raw(const uint32_t *row, uint32_t gw, uint32_t W,
                                         uint32_t nwg, GroupRaw<VEC> &g)
{
    if constexpr (VEC) {
        const uint32_t g0 = gw - (gw & 3u);
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            uint32_t idx = g0 + 4u * m;
            if (idx >= W) idx -= W;
            if (idx >= W) idx -= W;
            const uint4 x = *(const uint4 *)(row + idx);
            g.v[4 * m] = x.x; g.v[4 * m + 1] = x.y; g.v[4 * m + 2] = x.z; g.v[4 * m + 3] = x.w;
        }
    } else {
#pragma unroll
        for (uint32_t i = 0; i < 9; ++i) g.v[i] = i <= nwg ? row[wrap_add(gw, i, W)] : 0u;
#pragma unroll
        for (uint32_t i = 9; i < 12; ++i) g.v[i] = 0u;
    }
}

// Realigns loaded words (see load_raw) into A and R as load_group does.
template <bool VEC>
__device__ __forceinline__ void funnel_group(const GroupRaw<VEC> &g, uint32_t gw, uint32_t nwg,
                                             uint32_t sh2, uint32_t (&A)[8], uint32_t (&R)[9])
{
    if constexpr (VEC) {
        switch (__builtin_amdgcn_readfirstlane(gw & 3u)) {
        case 0: funnel8<0>(g.v, sh2, nwg, A, R); break;
        case 1: funnel8<1>(g.v, sh2, nwg, A, R); break;
        case 2: funnel8<2>(g.v, sh2, nwg, A, R); break;
        default: funnel8<3>(g.v, sh2, nwg, A, R); break;
        }
    } else {
        funnel8<0>(g.v, sh2, nwg, A, R);
    }
}

// load_raw and funnel_group of one row group, with the loads the group does
// not need skipped.
template <bool VEC>
__device__ __forceinline__ void load_group(const uint32_t *row, uint32_t gw, uint32_t W,
                                           uint32_t nwg, uint32_t sh2, uint32_t (&A)[8],
                                           uint32_t (&R)[9])
{
    if constexpr (VEC) {
        const uint32_t o = __builtin_amdgcn_readfirstlane(gw & 3u);
        const uint32_t g0 = gw - o;
        uint32_t v[12];
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            uint4 x = make_uint4(0u, 0u, 0u, 0u);
            if (4u * m < o + nwg + 1u) {
                uint32_t idx = g0 + 4u * m;
                if (idx >= W) idx -= W;
                if (idx >= W) idx -= W;
                x = *(const uint4 *)(row + idx);
            }
            v[4 * m] = x.x; v[4 * m + 1] = x.y; v[4 * m + 2] = x.z; v[4 * m + 3] = x.w;
        }
        switch (o) {
        case 0: funnel8<0>(v, sh2, nwg, A, R); break;
        case 1: funnel8<1>(v, sh2, nwg, A, R); break;
        case 2: funnel8<2>(v, sh2, nwg, A, R); break;
        default: funnel8<3>(v, sh2, nwg, A, R); break;
        }
    } else {
#pragma unroll
        for (uint32_t i = 0; i < 9; ++i) R[i] = i <= nwg ? row[wrap_add(gw, i, W)] : 0u;
#pragma unroll
        for (uint32_t i = 0; i < 8; ++i)
            A[i] = i < nwg ? __builtin_amdgcn_alignbit(R[i + 1], R[i], sh2) : 0u;
    }
}

// R[n] for a runtime n <= 8.
__device__ __forceinline__ uint32_t pick9(const uint32_t (&R)[9], uint32_t n)
{
    uint32_t v = R[0];
#pragma unroll
    for (uint32_t i = 1; i < 9; ++i)
        if (i == n) v = R[i];
    return v;
}

// One MCS residency of dead-border block b (DT: block b of a double-tiling
// set, no dead sites, halos from the idle neighbours) by the calling wave;
// the bit-sliced step is in kpz_slice.h.
//
// Device layer: origin (ox, oy) of residency res of MCS t; block (bx, by)
// covers sites ((ox + bx Bx + lx) mod L, (oy + by By + ly) mod L).
// Work-group layer: steps k = res * nsteps .. + nsteps - 1 of the MCS's 16;
// step k takes cell set bits 2k.. of (SET, t, b, res).w0 and, for row group
// G = (b nty + ty) nqx + q, the tile's bit of words 2 (k mod 2), +1 of
// (SITE, t, G, k / 2) as the site (rx, ry) in its cell.
template <bool ACC, bool DT, bool VEC, int XN = 2, int WY = 2, bool STG = false>
__device__ __forceinline__ void sweep_block(const SweepArgs &a, uint32_t b, uint4 *stg = nullptr)
{
    using namespace kpzslice;
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t bx = b % a.nbx, by = b / a.nbx;

    const U4 wo = philox<LATTICE_ROUNDS>(a.res, 0u, a.t, TAG_ORIGIN << 24, a.seed_lo, a.seed_hi);
    const uint32_t ox = (uint32_t)(((uint64_t)wo.x * a.Bx) >> 32);
    const uint32_t oy = (uint32_t)(((uint64_t)wo.y * a.By) >> 32);
    uint32_t gx0 = ox + bx * a.Bx;
    if (gx0 >= a.L) gx0 -= a.L;
    uint32_t gy0 = oy + by * a.By;
    if (gy0 >= a.L) gy0 -= a.L;
    const uint32_t s_in =
        rot_sites(Rot{a.db & a.prev_valid, a.prev_t, a.prev_res, a.Bx, a.seed_lo, a.seed_hi});
    uint32_t px0 = gx0 + (a.L - s_in);          // storage position of the block's first site
    if (px0 >= a.L) px0 -= a.L;
    const uint32_t sh2 = 2u * (px0 & 15u);
    const uint32_t gw0 = px0 >> 4;

    // lane = q nty + ty: q = floor(lane / nty) = lane ceil(2^16 / nty) >> 16
    // for lane < 64 and nty <= 64 (the error lane / 2^16 stays below 1 / nty)
    const uint32_t q = __umul24(lane, a.mnty) >> 16, ty = lane - __umul24(q, a.nty);
    // XN = 1: several row groups per tile row, so every group has 8 words
    const uint32_t nwg = XN == 1 ? 8u : a.nwg;
    const bool active = q < a.nqx;
    const uint32_t qw = active ? q * nwg : 0u;
    const uint32_t gwq = wrap_add(gw0, qw, a.W);   // storage word of the group's first site

    // ---- load: four rows of the group, transposed into planes.  DT keeps
    // the words the block shares with its idle neighbours as loaded: their
    // neighbours' bits do not change during the launch, so the store merges
    // into these copies instead of reading the words again.
    uint32_t X[4][4], Y[4][4];
    uint32_t w0r[4], wnr[4];
    if constexpr (STG) {
        // Staged load (VEC): the wave reads the block's By rows of su_u
        // aligned 16-byte units (from the unit holding the block's first
        // word), su_r rows per load instruction with consecutive lanes on
        // consecutive units of a row, and keeps them in its LDS region with
        // row 4 ty + r at position r nty + ty; every lane then takes its
        // group's three units of each of its four rows (lanes of consecutive
        // tile rows read units su_u apart: no bank conflicts for odd su_u).
        const uint32_t U = a.su_u, R = a.su_r;
        const uint32_t rs = __umul24(lane, a.su_m) >> 16, col = lane - __umul24(rs, U);
        const uint32_t rsv = rs < R ? rs : 0xffffu;        // lanes past R U idle
        const uint32_t xin = wrap_add(gw0 >> 2, col, a.W >> 2);
        const char *base = (const char *)a.src + 16u * xin;    // the lane's unit in row 0
        const uint32_t pitch = 4u * a.W;                       // bytes per row
        // each load goes straight to LDS (global_load_lds_dwordx4: lane i's
        // 16 bytes at the wave-uniform destination + 16 i)
        // (the row index wraps only in blocks that cross the lattice's edge)
        auto issue = [&](auto wrap) {
#pragma unroll
            for (uint32_t cc = 0; cc < STAGE_NC; ++cc) {
                if (cc < a.su_nc) {
                    const uint32_t tyc = cc * R + rsv;
#pragma unroll
                    for (uint32_t r = 0; r < 4; ++r) {
                        if (tyc < a.nty) {
                            uint32_t gy = gy0 + 4u * tyc + r;
                            if (decltype(wrap)::value && gy >= a.L) gy -= a.L;
                            __builtin_amdgcn_global_load_lds(
                                (const gptr_t)(base + (uint64_t)gy * pitch),
                                (lptr_t)(stg + (r * a.nty + cc * R) * U), 16, 0, 0);
                        }
                    }
                }
            }
        };
        if (gy0 + a.By > a.L) issue(std::true_type{});
        else issue(std::false_type{});
        __builtin_amdgcn_s_waitcnt(WAIT_VMCNT0);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        // the group's first unit; with one group per tile row the third unit
        // exists only when U > 2 (it is needed only then)
        const uint32_t j0 = ((gw0 & 3u) + q * nwg) >> 2;
        const bool third = XN == 1 || U > 2u;
        // whole 16-byte reads, all twelve issued before the first is used (a
        // volatile vector load is not cut into the words one funnel case
        // uses): lanes of consecutive tile rows then meet no bank conflict
        u32x4 v[4][3];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const uint4 *srow = stg + (r * a.nty + ty) * U + j0;
#pragma unroll
            for (uint32_t m = 0; m < 3; ++m) {
                v[r][m] = u32x4{0u, 0u, 0u, 0u};
                if (active && (m < 2 || third))
                    v[r][m] = *(const volatile __attribute__((address_space(3))) u32x4 *)(srow + m);
            }
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            uint32_t A[8] = {0u, 0u, 0u, 0u, 0u, 0u, 0u, 0u}, R9[9];
            if (active) {
                GroupRaw<VEC> g;
#pragma unroll
                for (uint32_t m = 0; m < 3; ++m) {
                    g.v[4 * m] = v[r][m].x; g.v[4 * m + 1] = v[r][m].y;
                    g.v[4 * m + 2] = v[r][m].z; g.v[4 * m + 3] = v[r][m].w;
                }
                funnel_group<VEC>(g, gwq, nwg, sh2, A, R9);
            }
            w0r[r] = 0u;
            wnr[r] = 0u;
            transpose8(A);
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                X[r][c] = A[2 * c];
                Y[r][c] = A[2 * c + 1];
            }
        }
    } else {
        // the loads of HR rows at a time are issued before the first is used
        // (all four in the dead-border sweep; one at a time with DT, whose
        // halo copies leave no registers for more); idle lanes read the
        // group 0 words of their tile row's rows
        constexpr int HR = DT ? 1 : 4;
        const uint32_t gwl = active ? gwq : gw0;
#pragma unroll
        for (int r0 = 0; r0 < 4; r0 += HR) {
        GroupRaw<VEC> g[HR];
        if (HR > 1) {
#pragma unroll
            for (int h = 0; h < HR; ++h) {
                const uint32_t gy = wrap_add(gy0, 4u * (active ? ty : 0u) + r0 + h, a.L);
                load_raw<VEC>(a.src + (size_t)gy * a.W, gwl, a.W, nwg, g[h]);
            }
        }
#pragma unroll
        for (int h = 0; h < HR; ++h) {
            const int r = r0 + h;
            uint32_t A[8], R[9];
            if (HR > 1) {
                funnel_group<VEC>(g[h], gwl, nwg, sh2, A, R);
            } else {
                const uint32_t gy = wrap_add(gy0, 4u * (active ? ty : 0u) + r, a.L);
                load_group<VEC>(a.src + (size_t)gy * a.W, gwl, a.W, nwg, sh2, A, R);
            }
            w0r[r] = R[0];
            wnr[r] = DT ? pick9(R, nwg) : 0u;
            if (!active) {
#pragma unroll
                for (int i = 0; i < 8; ++i) A[i] = 0u;
            }
            transpose8(A);
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                X[r][c] = A[2 * c];
                Y[r][c] = A[2 * c + 1];
            }
        }
        }
    }
    // DT halos: sigma_x of the column left of the block (lanes of group 0,
    // bit r = row r of the tile row; with sh2 = 0 it lies in the word before
    // the block, kept in hw) and sigma_y of the row below it (lanes of tile
    // row 0, as planes; its words as loaded in hr)
    uint32_t hx = 0u, hy[4] = {0u, 0u, 0u, 0u};
    uint32_t hw[4] = {0u, 0u, 0u, 0u};
    uint32_t hr[9] = {0u, 0u, 0u, 0u, 0u, 0u, 0u, 0u, 0u};
    if constexpr (DT) {
        if (active && q == 0) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                uint32_t wl = w0r[r];
                if (sh2 == 0) {
                    const uint32_t gy = wrap_add(gy0, 4u * ty + r, a.L);
                    wl = a.src[(size_t)gy * a.W + (gw0 == 0 ? a.W - 1 : gw0 - 1)];
                    hw[r] = wl;
                }
                const uint32_t bit = sh2 ? sh2 - 2u : 30u;
                hx |= ((wl >> bit) & 1u) << r;
            }
        }
        if (active && ty == 0) {
            uint32_t A[8] = {0u, 0u, 0u, 0u, 0u, 0u, 0u, 0u};
            const uint32_t gy = gy0 == 0 ? a.L - 1 : gy0 - 1;
            load_group<VEC>(a.src + (size_t)gy * a.W, gwq, a.W, nwg, sh2, A, hr);
            transpose8(A);
#pragma unroll
            for (int c = 0; c < 4; ++c) hy[c] = A[2 * c + 1];
        }
    }

    // ---- per-lane constants
    LaneCtx c;
    c.vm = active ? ((1u << (a.ntg >> 2)) - 1u) * 0x01010101u : 0u;
    c.dxm = (!DT && q == 0 && a.nbx > 1) ? 1u : 0u;
    c.dym = (!DT && ty == 0 && a.nby > 1) ? ~0u : 0u;
    c.xn = (a.nqx > 1 || a.nbx == 1) ? 1u : 0u;
    const uint32_t span = (a.nqx - 1u) * a.nty;
    // the groups of a tile row exchange with their neighbours cyclically:
    // with several blocks along x, group 0's tile 0 is dead at its left
    // column (its read is masked, its flip bit there is always 0)
    const uint32_t srcL = q > 0 ? lane - a.nty : lane + span;
    const uint32_t srcR = q + 1 < a.nqx ? lane + a.nty : lane - span;
    c.srcL4 = 4u * srcL;
    c.srcR4 = 4u * srcR;
    c.rmask = q + 1 < a.nqx ? ~0u : 0u;
    c.pb = 24u + (a.ntg >> 2) - 1u;
    c.wrapy = a.nby == 1 ? 1u : 0u;
    c.srcD4 = 4u * (ty > 0 ? lane - 1u : lane + a.nty - 1u);
    c.srcU4 = 4u * (ty + 1 < a.nty ? lane + 1u : lane - (a.nty - 1u));
    c.hxl = (DT && q == 0) ? ~0u : 0u;
    c.hyl = (DT && ty == 0) ? ~0u : 0u;
    c.uym = (DT && ty + 1 == a.nty) ? 0u : ~0u;

    const uint64_t G = ((uint64_t)b * a.nty + ty) * a.nqx + (active ? q : 0u);
    AccDraw d;
    d.P = a.P;
    d.Q = a.Q;
    d.nlP = levels_of(a.P);
    d.nlQ = levels_of(a.Q);
    d.nl = d.nlP > d.nlQ ? d.nlP : d.nlQ;
    d.seed_lo = a.seed_lo;
    d.seed_hi = a.seed_hi;
    d.t = a.t;
    d.G = (uint32_t)G;

    // ---- work-group layer: single-hit steps k0 .. k1 - 1
    const uint32_t setw = philox<LATTICE_ROUNDS>(b, 0u, a.t, (TAG_SET << 24) | a.res, a.seed_lo, a.seed_hi).x;
    const uint32_t k0 = a.res * a.nsteps, k1 = k0 + a.nsteps;
    const bool xn = XN == 2 ? c.xn != 0u : (XN == 1 || XN == 3);
    constexpr bool XBC = DT || XN != 0;        // the group boundary bond is kept (hl)
    int net = 0;
    U4 sw = {0u, 0u, 0u, 0u};
    uint32_t l1[4][4] = {{0u, 0u, 0u, 0u}, {0u, 0u, 0u, 0u}, {0u, 0u, 0u, 0u}, {0u, 0u, 0u, 0u}};
    uint32_t hl = 0u;
    bool own = false;   // hl holds the bond (a run of sx = 0 steps is on)
    for (uint32_t kq = k0 >> 2; 4u * kq < k1; ++kq) {
        if (ACC) {
#pragma unroll
            for (uint32_t j = 0; j < 4; ++j) {
                if (j < d.nl) {
                    const U4 v = philox_v<LATTICE_ROUNDS>((uint32_t)G, (uint32_t)(G >> 32), a.t,
                                        (TAG_ACC1 << 24) | (4u * kq + j), a.seed_lo, a.seed_hi);
                    l1[j][0] = v.x; l1[j][1] = v.y; l1[j][2] = v.z; l1[j][3] = v.w;
                }
            }
        }
#pragma unroll
        for (uint32_t kr = 0; kr < 4; ++kr) {
            const uint32_t k = 4u * kq + kr;
            if (k < k0 || k >= k1) continue;
            if ((kr & 1u) == 0 || k == k0)
                sw = philox_v<LATTICE_ROUNDS>((uint32_t)G, (uint32_t)(G >> 32), a.t, (TAG_SITE << 24) | (k >> 1),
                            a.seed_lo, a.seed_hi);
            const uint32_t RX = (kr & 1u) ? sw.z : sw.x;
            const uint32_t RY = (kr & 1u) ? sw.w : sw.y;
            const uint32_t lev[4] = {l1[0][kr], l1[1][kr], l1[2][kr], l1[3][kr]};
            const uint32_t s = (setw >> (2u * k)) & 3u;
            if (XBC && (xn || DT)) {
                if ((s & 1u) == 0 && !own) {
                    pull_bond(X, c, xn, DT, hx, hl);
                    own = true;
                } else if ((s & 1u) && own) {
                    push_bond(X, c, xn, DT, hx, hl);
                    own = false;
                }
            }
            switch (s) {
            case 0: step<0, 0, ACC, DT, XBC, WY, TAG_ACC2>(X, Y, RX, RY, c, lev, d, k, net, hl, hy); break;
            case 1: step<1, 0, ACC, DT, XBC, WY, TAG_ACC2>(X, Y, RX, RY, c, lev, d, k, net, hl, hy); break;
            case 2: step<0, 1, ACC, DT, XBC, WY, TAG_ACC2>(X, Y, RX, RY, c, lev, d, k, net, hl, hy); break;
            default: step<1, 1, ACC, DT, XBC, WY, TAG_ACC2>(X, Y, RX, RY, c, lev, d, k, net, hl, hy); break;
            }
        }
    }
    if (XBC && own) push_bond(X, c, xn, DT, hx, hl);

    // ---- store.  Two-buffer mode: the group's words are whole output words
    // (the output is rotated by the origin).  In place: words wholly inside
    // the block are stored (the word a group shares with the group to its
    // left is assembled from that group's last word); the block's parts of
    // the two words it shares with its neighbours go to the side buffer and
    // are merged by a separate launch.  DT: those two words are merged in
    // place (the neighbours are idle), and the halos are written back.
    // output word of the block's first site: storage position ox + bx Bx -
    // (ox mod 64)
    uint32_t gwo = 4u * (ox >> 6) + bx * a.nw;
    if (gwo >= a.W) gwo -= a.W;
    const uint32_t gwoq = wrap_add(gwo, qw, a.W);
    const bool ovec = VEC && (gwoq & 3u) == 0 && (nwg & 3u) == 0;
    const uint32_t lowm = sh2 ? (1u << sh2) - 1u : 0u;
    if (STG && a.db && (a.nw & 3u) == 0) {
        // Staged store (two-buffer mode, whole units per row): every lane
        // puts its group's output units into the wave's LDS region (the
        // layout of the staged load, nw / 4 of the su_u units of a row in
        // use), then the wave writes the block's rows as it read them.
        const uint32_t U = a.su_u, R = a.su_r;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            uint32_t A[8];
#pragma unroll
            for (int cc = 0; cc < 4; ++cc) {
                A[2 * cc] = X[r][cc];
                A[2 * cc + 1] = Y[r][cc];
            }
            transpose8(A);
            if (active) {
                uint4 *srow = stg + (r * a.nty + ty) * U + ((q * nwg) >> 2);
#pragma unroll
                for (uint32_t m = 0; m < 2; ++m)
                    if (4u * m < nwg)
                        srow[m] = make_uint4(A[4 * m], A[4 * m + 1], A[4 * m + 2], A[4 * m + 3]);
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const uint32_t rs = __umul24(lane, a.su_m) >> 16, col = lane - __umul24(rs, U);
        const uint32_t rsv = (rs < R && col + 1u < U) ? rs : 0xffffu;
        const uint32_t xout = wrap_add(gwo >> 2, col, a.W >> 2);
        char *base = (char *)a.words + 16u * xout;             // the lane's unit in row 0
        const uint32_t pitch = 4u * a.W;
        auto put = [&](auto wrap) {
#pragma unroll
            for (uint32_t cc = 0; cc < STAGE_NC; ++cc) {
                if (cc < a.su_nc) {
                    const uint32_t tyc = cc * R + rsv;
#pragma unroll
                    for (uint32_t r = 0; r < 4; ++r) {
                        if (tyc < a.nty) {
                            uint32_t gy = gy0 + 4u * tyc + r;
                            if (decltype(wrap)::value && gy >= a.L) gy -= a.L;
                            *(uint4 *)(base + (uint64_t)gy * pitch) =
                                stg[(r * a.nty + cc * R) * U + lane];
                        }
                    }
                }
            }
        };
        if (gy0 + a.By > a.L) put(std::true_type{});
        else put(std::false_type{});
    } else
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        uint32_t A[8];
#pragma unroll
        for (int cc = 0; cc < 4; ++cc) {
            A[2 * cc] = X[r][cc];
            A[2 * cc + 1] = Y[r][cc];
        }
        transpose8(A);
        const uint32_t gy = wrap_add(gy0, 4u * ty + r, a.L);
        uint32_t *row = a.words + (size_t)gy * a.W;
        if (a.db) {
            if (!active) continue;
            if (ovec) {
#pragma unroll
                for (uint32_t m = 0; m < 2; ++m)
                    if (4u * m < nwg)
                        *(uint4 *)(row + wrap_add(gwoq, 4u * m, a.W)) =
                            make_uint4(A[4 * m], A[4 * m + 1], A[4 * m + 2], A[4 * m + 3]);
            } else {
#pragma unroll
                for (uint32_t i = 0; i < 8; ++i)
                    if (i < nwg) row[wrap_add(gwoq, i, a.W)] = A[i];
            }
            continue;
        }
        // in place (and DT): every lane takes part in the exchange
        uint32_t lastA = A[0];
#pragma unroll
        for (uint32_t i = 1; i < 8; ++i)
            if (i + 1 == nwg) lastA = A[i];
        const uint32_t prevLast = bperm(c.srcL4, lastA);
        if (!active) continue;
        // DT with the diagonal partner set in the launch: the block's top
        // row shares its corner words with the partner blocks above-left
        // and above-right
        const bool corner = DT && a.ahead && r == 3 && ty + 1u == a.nty;
        if (sh2 == 0) {
#pragma unroll
            for (uint32_t i = 0; i < 8; ++i)
                if (i < nwg) row[wrap_add(gwq, i, a.W)] = A[i];
            if (DT && q == 0) {
                // halo column in the previous word, bit 30
                const uint32_t w = hw[r];
                const uint32_t nwv = (w & ~(1u << 30)) | (((hx >> r) & 1u) << 30);
                uint32_t *hp = row + (gw0 == 0 ? a.W - 1 : gw0 - 1);
                if (nwv != w) {
                    if (corner) atomicXor(hp, nwv ^ w);
                    else *hp = nwv;
                }
            }
            continue;
        }
#pragma unroll
        for (uint32_t i = 1; i < 8; ++i)
            if (i < nwg)
                row[wrap_add(gwq, i, a.W)] = __builtin_amdgcn_alignbit(A[i], A[i - 1], 32u - sh2);
        if (q > 0) {
            row[gwq] = __builtin_amdgcn_alignbit(A[0], prevLast, 32u - sh2);
        } else if (DT) {
            const uint32_t hb = sh2 - 2u;
            const uint32_t nwv =
                (w0r[r] & lowm & ~(1u << hb)) | (((hx >> r) & 1u) << hb) | (A[0] << sh2);
            if (corner) atomicXor(row + gwq, nwv ^ w0r[r]);
            else row[gwq] = nwv;
        } else {
            a.side[(size_t)gy * a.nbx + bx] = A[0] << sh2;
        }
        if (q + 1 == a.nqx) {
            if (DT) {
                const uint32_t nwv = (wnr[r] & ~lowm) | (lastA >> (32u - sh2));
                uint32_t *ep = row + wrap_add(gwq, nwg, a.W);
                if (corner) atomicXor(ep, nwv ^ wnr[r]);
                else *ep = nwv;
            } else {
                a.side[((size_t)a.L + gy) * a.nbx + bx] = lastA >> (32u - sh2);
            }
        }
    }

    if constexpr (DT) {
        // halo row: the sigma_y bits of the block's columns in the row below
        uint32_t B[8];
#pragma unroll
        for (int cc = 0; cc < 4; ++cc) {
            B[2 * cc] = 0u;
            B[2 * cc + 1] = hy[cc];
        }
        transpose8(B);
        uint32_t lastB = B[0];
#pragma unroll
        for (uint32_t i = 1; i < 8; ++i)
            if (i + 1 == nwg) lastB = B[i];
        const uint32_t prevLastB = bperm(c.srcL4, lastB);
        if (active && ty == 0) {
            const uint32_t gy = gy0 == 0 ? a.L - 1 : gy0 - 1;
            uint32_t *row = a.words + (size_t)gy * a.W;
            const uint32_t YM = 0xAAAAAAAAu;
            // with the diagonal partner set in the launch, the halo row's
            // end words are shared with the partner blocks below-left and
            // below-right (atomic xor of this block's change)
            const bool corner = a.ahead != 0u;
            if (sh2 == 0) {
#pragma unroll
                for (uint32_t i = 0; i < 8; ++i)
                    if (i < nwg) {
                        const uint32_t nwv = (hr[i] & ~YM) | B[i];
                        uint32_t *wp = row + wrap_add(gwq, i, a.W);
                        if (corner && q + 1 == a.nqx && i + 1 == nwg) atomicXor(wp, nwv ^ hr[i]);
                        else *wp = nwv;
                    }
            } else {
#pragma unroll
                for (uint32_t i = 1; i < 8; ++i)
                    if (i < nwg)
                        row[wrap_add(gwq, i, a.W)] =
                            (hr[i] & ~YM) | __builtin_amdgcn_alignbit(B[i], B[i - 1], 32u - sh2);
                if (q > 0) {
                    row[gwq] = (hr[0] & ~YM) | __builtin_amdgcn_alignbit(B[0], prevLastB, 32u - sh2);
                } else {
                    const uint32_t nwv = (hr[0] & ~(YM & ~lowm)) | (B[0] << sh2);
                    if (corner) atomicXor(row + gwq, nwv ^ hr[0]);
                    else row[gwq] = nwv;
                }
                if (q + 1 == a.nqx) {
                    const uint32_t lw = pick9(hr, nwg);
                    const uint32_t nwv = (lw & ~(YM & lowm)) | (lastB >> (32u - sh2));
                    uint32_t *ep = row + wrap_add(gwq, nwg, a.W);
                    if (corner) atomicXor(ep, nwv ^ lw);
                    else *ep = nwv;
                }
            }
        }
    }

    // ---- flip counter of this block: wave sum, one atomic per block
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) net += __shfl_xor(net, off, 64);
    if (lane == 0 && net != 0)
        atomicAdd(a.slots + (b & a.slot_mask), (unsigned long long)(long long)net);
}

// One MCS residency of every block: one wave per block, four waves per
// work-group (one when the block count is not a multiple of four).
// Work-groups are dealt to the 8 XCDs round-robin (group i to XCD i mod 8);
// with xcd set, group i takes the blocks of virtual group (i mod 8) n/8 +
// i/8, so each XCD runs one contiguous range of blocks and neighbouring
// blocks, which share cache lines at their edges, meet in the same L2.
// XN = 1: several row groups per tile row (8 words each), which exchange
// tile 0's left neighbour; 3: one block along x and one row group per tile
// row (tile 0's left neighbour wraps around to the same lane's group); 0: one
// group per tile row and several blocks along x; 2: decided at run time.
// WY: one block along y (the tile row below tile row 0 wraps around); 2 = at
// run time.
// VEC: every wave stages its block's rows in its own a.su 16-byte units of
// the dynamic LDS.
template <bool ACC, bool VEC, int XN, int WY>
__global__ __launch_bounds__(256) void kpz_sweep_kernel(const SweepArgs a, uint32_t nblocks)
{
    extern __shared__ uint4 kpz_stage[];
    uint32_t g = blockIdx.x;
    if (a.xcd) g = (g & 7u) * (gridDim.x >> 3) + (g >> 3);
    const uint32_t wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t b = g * (blockDim.x >> 6) + wv;
    if (b >= nblocks) return;
    sweep_block<ACC, false, VEC, XN, WY, VEC>(a, b, kpz_stage + wv * a.su);
}

// Straddling word j = gy * nbx + bx of MCS a.t: the word at the left edge of
// block column bx in row gy holds the last sites of block bx-1 (low bits) and
// the first sites of block bx (high bits); both parts are in the side buffer.
__device__ __forceinline__ void merge_one(const SweepArgs &a, uint32_t ox, uint64_t j)
{
    const uint32_t gy = (uint32_t)(j / a.nbx), bx = (uint32_t)(j % a.nbx);
    uint32_t gw = (ox >> 4) + bx * a.nw;
    if (gw >= a.W) gw -= a.W;
    const uint32_t left = a.side[((size_t)a.L + gy) * a.nbx + (bx == 0 ? a.nbx - 1 : bx - 1)];
    const uint32_t right = a.side[(size_t)gy * a.nbx + bx];
    a.words[(size_t)gy * a.W + gw] = left | right;
}

__device__ __forceinline__ uint32_t origin_x(const SweepArgs &a)
{
    const U4 wo = philox<LATTICE_ROUNDS>(a.res, 0u, a.t, TAG_ORIGIN << 24, a.seed_lo, a.seed_hi);
    return (uint32_t)(((uint64_t)wo.x * a.Bx) >> 32);
}

__global__ void kpz_merge_kernel(const SweepArgs a)
{
    const uint32_t ox = origin_x(a);
    if ((ox & 15u) == 0) return;
    const uint64_t n = (uint64_t)a.L * a.nbx;
    for (uint64_t j = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; j < n;
         j += (uint64_t)gridDim.x * blockDim.x)
        merge_one(a, ox, j);
}

// ------------------------------------ double tiling at the device layer
//
// Alternative device layer (Sec. 3): the blocks (same frames as above, nbx
// and nby even) form four sets (bx mod 2, by mod 2) of non-adjacent
// blocks; an MCS runs the sets in the order perm[(DTORDER, t).w0 * 24 >>
// 32] (the 24 orderings of 0..3 in lexicographic order), one launch per
// set.  A block of the active set makes its 16 single-hit steps with the
// same draws as under dead borders but has no dead sites: an update at its
// left column or bottom row flips a slope stored in the idle block to the
// left or below.  Blocks of one set touch disjoint words (for Bx >= 16), so
// every launch updates the lattice in place with no merge.

constexpr uint32_t TAG_DTORDER = 13;

// Block set (bx mod 2 + 2 (by mod 2)) of position `phase` in MCS t: the
// ordering floor(w0 24 / 2^32) of (DTORDER, t), orderings of 0..3 numbered
// lexicographically.
__device__ __forceinline__ uint32_t dt_set(uint32_t t, uint32_t seed_lo, uint32_t seed_hi,
                                           uint32_t phase)
{
    uint32_t idx = (uint32_t)(((uint64_t)philox<LATTICE_ROUNDS>(0u, 0u, t, TAG_DTORDER << 24, seed_lo,
                                                seed_hi).x * 24u) >> 32);
    uint32_t pool = 0x3210u;             // remaining set codes, one per nibble
    uint32_t n = 4, c = 0;
    const uint32_t fact[4] = {1u, 1u, 2u, 6u};
    for (uint32_t i = 0; i <= phase; ++i) {
        const uint32_t f = fact[n - 1];
        const uint32_t pick = idx / f;
        idx %= f;
        c = (pool >> (4 * pick)) & 15u;
        // remove nibble `pick`
        const uint32_t lowmask = (1u << (4 * pick)) - 1u;
        pool = (pool & lowmask) | ((pool >> 4) & ~lowmask);
        --n;
    }
    return c;
}

// One launch per block set; the blocks of set c are (2 i + (c & 1), 2 j +
// (c >> 1)), one wave each.  a.ahead: the launch also runs the set of the
// next phase, the diagonal partner (c ^ 3) of this one, in waves nset ..
// 2 nset - 1 (Sec. 3.2, blocks updated ahead of time): the two sets touch
// no common slope, so this equals running them one after the other.
template <bool ACC, bool VEC, int XN>
__global__ __launch_bounds__(256) void kpz_dt_kernel(const SweepArgs a, uint32_t phase,
                                                     uint32_t nset)
{
    uint32_t g = blockIdx.x;
    if ((gridDim.x & 7u) == 0) g = (g & 7u) * (gridDim.x >> 3) + (g >> 3);
    uint32_t w = g * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (w >= (a.ahead ? 2u * nset : nset)) return;
    if (w >= nset) {   // wave-uniform
        w -= nset;
        ++phase;
    }
    const uint32_t c = dt_set(a.t, a.seed_lo, a.seed_hi, phase);
    const uint32_t hx = a.nbx >> 1;
    const uint32_t bx = 2 * (w % hx) + (c & 1u), by = 2 * (w / hx) + (c >> 1);
    sweep_block<ACC, true, VEC, XN, 0>(a, __builtin_amdgcn_readfirstlane(by * a.nbx + bx));
}


// ------------------------------------------------------------ roughness

// Per row y: with P(x) = sum_{l<x} sigma_x(l,y) (height relative to the row
// start), A_y = sum_x P(x) and B_y = sum_x P(x)^2, a group of lanes per row.
//
// A word's 16 sites are taken as two halves of 8; a 256-entry LDS table gives,
// for 8 sites with local prefix p_k (k = 0..7), d = p_8, a = sum p_k and
// c = sum p_k^2.  A half's table index is gathered from the word with two
// masks and a shift: bit 2i of the index is sigma_x of site i and bit 2i+1
// that of site i + 4 (i = 0..3), i.e. the index interleaves the half's first
// and last four sites, and the table is filled in that order.  The large row
// passes hold the table in LUT_COPIES copies, entry e of copy j at index
// e LUT_COPIES + j, and lane l reads copy l mod LUT_COPIES: the 64 lookups of
// a wave then never meet in one bank.  The one-work-group passes of small
// lattices, whose table fill would outlast their few lookups, keep one copy
// (C = 1).
constexpr uint32_t LUT_COPIES = 32;
constexpr uint32_t LUT_WORDS = 256 * LUT_COPIES;
constexpr int LUT_ABIAS = 28;   // a + LUT_ABIAS >= 0

// Entry layout: c (0..140) in bits 0..7 with bits 8..12 zero and a + 28
// (0..56) in bits 13..18 with bits 19..23 zero, so the plain sum of up to 32
// entries holds the sums of c and of a + 28 exactly in bits 0..12 and
// 13..23; d (-8..8) in bits 27..31, two's complement (one arithmetic shift).
__device__ __forceinline__ uint32_t lut8_entry(uint32_t idx)
{
    int p = 0, a = 0, c = 0;
    for (int k = 0; k < 8; ++k) {
        a += p;
        c += p * p;
        const uint32_t bit = k < 4 ? 2 * k : 2 * (k - 4) + 1;   // interleaved index
        p += ((idx >> bit) & 1u) ? 1 : -1;
    }
    return (uint32_t)c | ((uint32_t)(a + LUT_ABIAS) << 13) | ((uint32_t)p << 27);
}

// Fills the replicated table (every thread of the work-group takes part;
// the caller synchronises before the first lookup).
template <uint32_t C = LUT_COPIES>
__device__ __forceinline__ void fill_row_lut(uint32_t *lut)
{
    for (uint32_t i = threadIdx.x; i < 256u; i += blockDim.x) {
        const uint32_t e = lut8_entry(i);
        if constexpr (C == 1) {
            lut[i] = e;
        } else {
            const uint4 v = make_uint4(e, e, e, e);
#pragma unroll
            for (uint32_t j = 0; j < C / 4; ++j)
                ((uint4 *)(lut + i * C))[(j + i) & (C / 4 - 1u)] = v;
        }
    }
}

// Sums of a lane over the halves of consecutive words, the heights of a half
// being o + p_k with o its offset from the lane's first site: T = sum o,
// Q = sum o^2, R = sum o (a + 28), csum = sum of the table entries (at most
// 32 halves between two calls of lane_totals).
struct LaneSums {
    int o, T, Q, R;
    uint32_t csum;
};

__device__ __forceinline__ void add_half(LaneSums &r, uint32_t e)
{
    const int ab = (int)__builtin_amdgcn_ubfe(e, 13, 6);
    r.T += r.o;
    r.Q = __mul24(r.o, r.o) + r.Q;
    r.R = __mul24(r.o, ab) + r.R;
    r.csum += e;
    r.o += (int)e >> 27;
}

// Byte offsets into the table of the two halves of word w, for copy offset
// `copy4x2` = 4 copy (0x10001): the interleaved index of each half times
// 4 C, computed for both halves at once, the first in the low and the second
// in the high 16 bits (the sites of the second half sit 16 bits above those
// of the first, and every offset stays below 2^15).
template <uint32_t C>
__device__ __forceinline__ void lut_addrs(uint32_t w, uint32_t copy4x2, uint32_t &a0, uint32_t &a1)
{
    constexpr uint32_t S = C == 1 ? 2 : C == 32 ? 7 : 0;   // log2(4 C)
    static_assert(S != 0, "one or 32 copies");
    constexpr uint32_t M1 = (0x55u << S) * 0x10001u, M2 = (0xAAu << S) * 0x10001u;
    // index bits 0,2,4,6 <- sites 0..3 (w bits 0,2,4,6); bits 1,3,5,7 <-
    // sites 4..7 (w bits 8,10,12,14); likewise 16 bits up
    const uint32_t P = ((w << S) & M1) | ((w >> (7 - S)) & M2) | copy4x2;
    a0 = P & 0xFFFFu;
    a1 = P >> 16;
}

template <uint32_t C>
__device__ __forceinline__ void add_word(LaneSums &r, uint32_t w, const uint32_t *lut,
                                         uint32_t copy4x2)
{
    uint32_t a0, a1;
    lut_addrs<C>(w, copy4x2, a0, a1);
    const uint32_t e0 = *(const uint32_t *)((const char *)lut + a0);
    const uint32_t e1 = *(const uint32_t *)((const char *)lut + a1);
    add_half(r, e0);
    add_half(r, e1);
}

// (o, sum of heights, sum of squared heights) of the lane's nh halves,
// heights relative to its first site: sum over halves of 8 o + a and of
// 8 o^2 + 2 o a + c.
__device__ __forceinline__ void lane_totals(const LaneSums &r, int nh, int &l1, int &l2)
{
    const int sa = (int)((r.csum >> 13) & 0x7FFu) - LUT_ABIAS * nh;
    const int sc = (int)(r.csum & 0x1FFFu);
    l1 = 8 * r.T + sa;
    l2 = 8 * r.Q + 2 * (r.R - LUT_ABIAS * r.T) + sc;
}

// Lanes per row (a power of two, for the width of the group shuffles): a
// row of W words, W a power of two from 4 to 128, is taken by W / 4 lanes,
// one 16-byte load each, so a wave holds 256 / W rows; every other row takes
// a whole wave.
__host__ __device__ __forceinline__ uint32_t row_lanes(uint32_t W)
{
    return (W >= 4u && W < 256u && (W & (W - 1u)) == 0) ? W / 4u : 64u;
}

// Wave tasks of the row-moment pass for an L x L lattice: L / R, R = 64 /
// row_lanes(L / 16) rows per wave (R > 1 only for L a power of two from 64
// to 2048, where R = 4096 / L divides L).
__host__ __device__ __forceinline__ uint32_t row_tasks(uint32_t L)
{
    const uint32_t R = 64u / row_lanes(L / 16u);
    return (L + R - 1u) / R;
}

// Inclusive sum over the 64 lanes of a wave: shifts by 1, 2, 4 and 8 lanes
// within each row of 16 lanes, then the last lane of row 0 added to row 1 and
// of row 2 to row 3, then lane 31 added to rows 2 and 3 (DPP).
__device__ __forceinline__ int wave_incl_sum(int x)
{
    x += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xf, 0xf, false);   // row_shr:1
    x += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xf, 0xf, false);   // row_shr:2
    x += __builtin_amdgcn_update_dpp(0, x, 0x114, 0xf, 0xf, false);   // row_shr:4
    x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xf, 0xf, false);   // row_shr:8
    x += __builtin_amdgcn_update_dpp(0, x, 0x142, 0xa, 0xf, false);   // row_bcast:15
    x += __builtin_amdgcn_update_dpp(0, x, 0x143, 0xc, 0xf, false);   // row_bcast:31
    return x;
}

// Moments of one row in stored order, taken by a group of G lanes (G =
// row_lanes(W), the group's lanes gl = 0..G-1 aligned to G in the wave), NV
// consecutive words per lane and chunk (NV = 8 only for W % 512 == 0, where
// G = 64 and every lane is full): returns (A_y, B_y), the sums of the
// heights relative to the row's first stored site and of their squares, in
// lane gl = 0 and, in `first`, the row's first stored word.  A row stored
// rotated by s sites starts at site s; the finalize pass takes column s as
// the reference column and shifts the totals to h(0, 0).  A lane's local
// sums stay below 2^24 and heights within a row below L, so they are
// 32-bit; only the row totals are 64-bit.
// Words idx .. idx + NV - 1 of a row of W words (zero beyond W); *nv = how
// many lie in the row.
template <int NV>
__device__ __forceinline__ void row_chunk(const uint32_t *rp, uint32_t W, uint32_t idx,
                                          uint32_t (&v)[NV], int &nv)
{
    nv = 0;
    if (NV == 8) {
#pragma unroll
        for (int j = 0; j < NV / 4; ++j) {
            const uint4 q = *(const uint4 *)(rp + idx + 4 * j);
            v[4 * j] = q.x; v[4 * j + 1] = q.y; v[4 * j + 2] = q.z; v[4 * j + 3] = q.w;
        }
        nv = NV;
    } else {
#pragma unroll
        for (int m = 0; m < NV; ++m) v[m] = 0u;
        if ((W & 3u) == 0) {
            if (idx < W) {
                const uint4 q = *(const uint4 *)(rp + idx);
                v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
                nv = 4;
            }
        } else {
#pragma unroll
            for (int m = 0; m < 4; ++m)
                if (idx + m < W) { v[m] = rp[idx + m]; nv = m + 1; }
        }
    }
}

template <int NV, uint32_t C = LUT_COPIES>
__device__ __forceinline__ void row_moments(const uint32_t *rp, uint32_t W, const uint32_t *lut,
                                            uint32_t gl, uint32_t G, long long &A, long long &B,
                                            uint32_t &first)
{
    static_assert(NV == 4 || NV == 8, "four or eight words per lane");
    const uint32_t copy4x2 = (threadIdx.x & (C - 1u)) * 0x40004u;   // work-groups of whole waves
    long long s1 = 0, s2 = 0;
    int carry = 0;
    first = 0u;
    for (uint32_t base = 0; base < W; base += NV * G) {
        uint32_t v[NV];
        int nv;
        row_chunk<NV>(rp, W, base + NV * gl, v, nv);
        if (base == 0) first = v[0];
        // this lane's words relative to its own start
        LaneSums ls = {0, 0, 0, 0, 0u};
#pragma unroll
        for (int m = 0; m < NV; ++m)
            if (NV == 8 || m < nv) add_word<C>(ls, v[m], lut, copy4x2);
        int l1, l2;
        lane_totals(ls, 2 * nv, l1, l2);
        const int o = ls.o;
        // lane offsets within the chunk: exclusive scan of o over the group
        int incl, total;
        if (G == 64u) {
            incl = wave_incl_sum(o);
            total = __builtin_amdgcn_readlane(incl, 63);
        } else {
            incl = o;
            for (uint32_t off = 1; off < G; off <<= 1) {
                const int t = __shfl_up(incl, off, G);
                if (gl >= off) incl += t;
            }
            total = __shfl(incl, G - 1u, G);
        }
        const int c = carry + incl - o;
        s1 += (long long)(16 * nv) * c + l1;
        s2 += (long long)(16 * nv) * ((long long)c * c) + 2LL * c * l1 + l2;
        carry += total;
    }
    for (uint32_t off = G >> 1; off > 0; off >>= 1) {
        s1 += __shfl_xor(s1, off, G);
        s2 += __shfl_xor(s2, off, G);
    }
    A = s1;
    B = s2;
}

// One wave per 64 / row_lanes(W) rows; work-groups of ROW_WAVES waves share
// one table, so that its LDS (32 KiB) admits eight waves per SIMD.
constexpr uint32_t ROW_WAVES = 8;
__global__ __launch_bounds__(64 * ROW_WAVES) __attribute__((amdgpu_waves_per_eu(8)))
void kpz_row_moments_kernel(const uint32_t *words, uint32_t L, uint32_t W, long long *rowA,
                            long long *rowB)
{
    __shared__ uint32_t lut[LUT_WORDS];
    fill_row_lut(lut);
    __syncthreads();
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t G = row_lanes(W), R = 64u / G;
    const uint32_t gl = lane & (G - 1u);
    const uint32_t tasks = (L + R - 1u) / R;
    for (uint32_t task = blockIdx.x * ROW_WAVES + wv; task < tasks;
         task += gridDim.x * ROW_WAVES) {
        const uint32_t row = task * R + lane / G;
        if (row < L) {   // a whole lane group is in or out
            long long A, B;
            uint32_t first;
            if ((W & 511u) == 0)
                row_moments<8>(words + (size_t)row * W, W, lut, gl, G, A, B, first);
            else
                row_moments<4>(words + (size_t)row * W, W, lut, gl, G, A, B, first);
            if (gl == 0) {
                rowA[row] = A;
                rowB[row] = (B << 1) | ((first >> 1) & 1u);   // + sigma_y of the first stored site
            }
        }
    }
}

// Work-groups of a row-moment launch over `tasks` wave tasks.
__host__ __forceinline__ uint32_t row_grid(uint32_t tasks)
{
    const uint32_t g = (tasks + ROW_WAVES - 1u) / ROW_WAVES;
    return g < 2048u ? g : 2048u;
}

// A lattice buffer in the documented layout from one stored rotated by
// rot_sites(rot) (src != dst).
__global__ void kpz_rotate_kernel(const uint32_t *src, uint32_t *dst, uint32_t L, uint32_t W,
                                  const Rot rot)
{
    const uint32_t s = rot_sites(rot);
    const uint32_t sw = s >> 4, rot2 = 2u * (s & 15u);
    const uint64_t n = (uint64_t)L * W;
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x) {
        // layout word w: sites 16 w .. = stored positions 16 (w - sw) - s mod 16
        const uint32_t w = (uint32_t)(i % W);
        const uint64_t rowb = i - w;
        const uint32_t w1 = w >= sw ? w - sw : w + W - sw;
        const uint32_t w0 = w1 ? w1 - 1 : W - 1;
        dst[i] = rot2 ? __builtin_amdgcn_alignbit(src[rowb + w1], src[rowb + w0], 32u - rot2)
                      : src[rowb + w1];
    }
}

// One work-group of NT threads: c_y = sum_{k<y} sigma_y(0,k) (column-0
// heights), R1 = sum_y (L c_y + A_y), R2 = sum_y (L c_y^2 + 2 c_y A_y + B_y)
// in 128-bit, and the sum of the flip-counter slots.  The row pass stores
// rowB[y] = 2 B_y + [sigma_y(0,y) = +1] (B_y <= L^3/4 leaves the room), so
// this pass reads two contiguous arrays and never the lattice.  Wave w takes
// one contiguous range of rows [y0, y1), 64 consecutive rows per load
// (coalesced), in one pass: with d_y = c_y - c_{y0} (from a ballot of the
// sigma_y bits and a count of the set bits below each lane), a lane sums
// r1 = sum (L d_y + A_y) and r2 = sum (L d_y^2 + 2 d_y A_y + B_y) over its n
// rows; once c_{y0} = C is known from the waves' totals, its share of R1 is
// r1 + n L C and of R2 is r2 + 2 C r1 + n L C^2.
template <int NT>
__device__ __forceinline__ void finalize_moments(uint32_t L, const long long *rowA,
                                                 const long long *rowB, const long long *slots,
                                                 uint32_t nslots, long long *res,
                                                 const uint32_t *row0, uint32_t s)
{
    constexpr uint32_t NWV = NT / 64;
    __shared__ long long wsum[NWV];
    __shared__ __int128 r2s[NT];
    __shared__ long long r1s[NT];
    __shared__ long long ns[NT];
    const uint32_t tid = threadIdx.x, lane = tid & 63u;
    const uint32_t wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const uint32_t per = (L + NWV - 1) / NWV;
    const uint32_t y0 = min(L, wv * per);
    const uint32_t y1 = min(L, y0 + per);
    // with |c| <= L/2, |A_y| <= L^2/2 and B_y <= L^3/4 every row's term fits
    // int64 for L <= 2^20; sums over rows are kept in 128-bit
    long long d = 0;   // sum of sigma_y(0, .) over the wave's rows before `base`
    long long r1 = 0, nr = 0;
    __int128 r2 = 0;
    constexpr int U = 8;   // loads of U groups of 64 rows in flight
    for (uint32_t base = y0; base < y1; base += 64u * U) {
        long long Av[U], Bv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint32_t y = base + 64u * u + lane;
            const uint32_t yy = y < y1 ? y : base;   // in range: base < y1
            Av[u] = rowA[yy];
            Bv[u] = rowB[yy];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint32_t y = base + 64u * u + lane;
            const bool ok = y < y1;
            const uint64_t upm = __ballot(ok && (Bv[u] & 1));
            // the lanes below this one hold rows y - lane .. y - 1, all in range
            const uint32_t below = __builtin_amdgcn_mbcnt_hi(
                (uint32_t)(upm >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)upm, 0u));
            const long long dy = d + 2 * (long long)below - (long long)lane;
            if (ok) {
                r1 += (long long)L * dy + Av[u];
                r2 += (__int128)((long long)L * dy * dy + 2 * dy * Av[u] + (Bv[u] >> 1));
                nr += 1;
            }
            d += 2 * (long long)__popcll(upm) - (long long)__popcll(__ballot(ok));
        }
    }
    if (lane == 0) wsum[wv] = d;
    __syncthreads();
    long long C = 0;   // c_{y0}
    for (uint32_t w = 0; w < wv; ++w) C += wsum[w];
    r2 += (__int128)(2 * C) * r1 + (__int128)((long long)L * nr) * ((__int128)C * C);
    r1 += (long long)L * nr * C;
    long long n = 0;
    for (uint32_t i = tid; i < nslots; i += NT) n += slots[i];
    r1s[tid] = r1;
    r2s[tid] = r2;
    ns[tid] = n;
    __syncthreads();
    for (uint32_t off = NT / 2; off > 0; off >>= 1) {
        if (tid < off) {
            r1s[tid] += r1s[tid + off];
            r2s[tid] += r2s[tid + off];
            ns[tid] += ns[tid + off];
        }
        __syncthreads();
    }
    if (tid == 0) {
        // rows stored rotated by s sites: the sums above are relative to
        // h(s, 0); h(s, 0) - h(0, 0) = P0 = the slopes of sites 0 .. s - 1 of
        // row 0, stored at positions L - s .. L - 1
        long long P0 = 0;
        for (uint32_t i = L - s; i < L; ++i)
            P0 += 2 * (long long)((row0[i >> 4] >> (2u * (i & 15u))) & 1u) - 1;
        const long long N = (long long)L * L;
        const __int128 R1p = r1s[0];
        const __int128 R2 = r2s[0] + 2 * (__int128)P0 * R1p + (__int128)N * P0 * P0;
        const unsigned __int128 u2 = (unsigned __int128)R2;
        res[0] = (long long)(R1p + (__int128)N * P0);
        res[1] = (long long)(uint64_t)u2;
        res[2] = (long long)(uint64_t)(u2 >> 64);
        res[3] = ns[0];
    }
}

__global__ __launch_bounds__(1024) void kpz_finalize_kernel(uint32_t L, const long long *rowA,
                                                            const long long *rowB,
                                                            const long long *slots,
                                                            long long *res, const uint32_t *words,
                                                            const Rot rot)
{
    finalize_moments<1024>(L, rowA, rowB, slots, NSLOTS, res, words, rot_sites(rot));
}

// Lattices of at most SMALL_ROWS rows: the row pass and the finalize in one
// work-group, the row sums in LDS (one launch per sample instead of two).
constexpr uint32_t SMALL_ROWS = 1024;

// Row sums of a lattice of L <= SMALL_ROWS rows by the 16 waves of one
// work-group of 1024 threads, into rA / rB (LDS); `lut` filled.
__device__ __forceinline__ void small_rows(const uint32_t *words, uint32_t L, uint32_t W,
                                           const uint32_t *lut, long long *rA, long long *rB)
{
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t G = row_lanes(W), R = 64u / G;
    const uint32_t gl = lane & (G - 1u);
    const uint32_t tasks = (L + R - 1u) / R;
    for (uint32_t task = wv; task < tasks; task += 16u) {
        const uint32_t row = task * R + lane / G;
        if (row < L) {   // a whole lane group is in or out
            long long A, B;
            uint32_t first;
            row_moments<4, 1>(words + (size_t)row * W, W, lut, gl, G, A, B, first);
            if (gl == 0) {
                rA[row] = A;
                rB[row] = (B << 1) | ((first >> 1) & 1u);   // + sigma_y of the first stored site
            }
        }
    }
}

__global__ __launch_bounds__(1024) void kpz_roughness_small_kernel(const uint32_t *words,
                                                                   uint32_t L, uint32_t W,
                                                                   const long long *slots,
                                                                   long long *res, const Rot rot)
{
    __shared__ uint32_t lut[256];
    __shared__ long long rA[SMALL_ROWS], rB[SMALL_ROWS];
    fill_row_lut<1>(lut);
    __syncthreads();
    small_rows(words, L, W, lut, rA, rB);
    __syncthreads();
    finalize_moments<1024>(L, rA, rB, slots, NSLOTS, res, words, rot_sites(rot));
}


// ------------------------------------------------ height moments to order 4
//
// Exact sums M_k = sum over sites of (h - h(0,0))^k, k = 1..4 (the one-point
// functions of the height distribution), with the same row scheme as W^2:
// per 8 sites a table entry (d, sum p, ..., sum p^4) of the local prefix
// p, combined by binomial shifts sum (c + v)^k = sum_j C(k,j) c^(k-j) S_j.

struct Mom4 {
    long long n;                  // number of values
    long long s1;
    long long s2;
    __int128 s3, s4;
};

__device__ __forceinline__ Mom4 mom4_shift(const Mom4 &m, long long c)
{
    // moments of (v + c) from those of v
    Mom4 r;
    const __int128 C = c, C2 = C * C, C3 = C2 * C, C4 = C3 * C;
    r.n = m.n;
    r.s1 = m.s1 + m.n * c;
    r.s2 = m.s2 + 2 * c * m.s1 + m.n * c * c;
    r.s3 = m.s3 + 3 * C * m.s2 + 3 * C2 * m.s1 + C3 * m.n;
    r.s4 = m.s4 + 4 * C * m.s3 + 6 * C2 * m.s2 + 4 * C3 * m.s1 + C4 * m.n;
    return r;
}

__device__ __forceinline__ void mom4_add(Mom4 &a, const Mom4 &b)
{
    a.n += b.n;
    a.s1 += b.s1;
    a.s2 += b.s2;
    a.s3 += b.s3;
    a.s4 += b.s4;
}

// 8 sites: local prefix p_k (k = 0..7) -> d = p_8 and sum p^j, j = 1..4
// (|sum p| <= 28, sum p^2 <= 140, |sum p^3| <= 784, sum p^4 <= 4676)
__device__ __forceinline__ uint2 lut8_mom4(uint32_t byte)
{
    int p = 0, a1 = 0, a2 = 0, a3 = 0, a4 = 0;
    for (int i = 0; i < 8; ++i) {
        a1 += p;
        a2 += p * p;
        a3 += p * p * p;
        a4 += p * p * p * p;
        p += ((byte >> i) & 1u) ? 1 : -1;
    }
    // x: d + 8 (5 bits) | a1 + 28 (6) | a2 (8) ; y: a3 + 1024 (11) | a4 (13)
    return make_uint2((uint32_t)(p + 8) | ((uint32_t)(a1 + 28) << 5) | ((uint32_t)a2 << 11),
                      (uint32_t)(a3 + 1024) | ((uint32_t)a4 << 11));
}

__device__ __forceinline__ Mom4 chunk8(uint2 e, int &d)
{
    Mom4 m;
    d = (int)(e.x & 31u) - 8;
    m.n = 8;
    m.s1 = (int)((e.x >> 5) & 63u) - 28;
    m.s2 = (int)(e.x >> 11);
    m.s3 = (int)(e.y & 2047u) - 1024;
    m.s4 = (int)(e.y >> 11);
    return m;
}

__device__ void row_mom4(const uint32_t *rp, uint32_t W, const uint2 *lut, uint32_t lane, Mom4 &out)
{
    Mom4 tot = {0, 0, 0, 0, 0};
    long long carry = 0;
    for (uint32_t base = 0; base < W; base += 64) {
        const uint32_t idx = base + lane;
        Mom4 w = {0, 0, 0, 0, 0};
        int dw = 0;
        if (idx < W) {
            uint32_t x = rp[idx] & 0x55555555u;
            x = (x | (x >> 1)) & 0x33333333u;
            x = (x | (x >> 2)) & 0x0F0F0F0Fu;
            x = (x | (x >> 4)) & 0x00FF00FFu;
            int d0, d1;
            const Mom4 lo = chunk8(lut[x & 0xFFu], d0);
            Mom4 hi = chunk8(lut[(x >> 16) & 0xFFu], d1);
            hi = mom4_shift(hi, d0);
            w = lo;
            mom4_add(w, hi);
            dw = d0 + d1;
        }
        int incl = dw;
        for (int off = 1; off < 64; off <<= 1) {
            const int t = __shfl_up(incl, off, 64);
            if ((int)lane >= off) incl += t;
        }
        mom4_add(tot, mom4_shift(w, carry + incl - dw));
        carry += __shfl(incl, 63, 64);
    }
    // wave sum
    for (int off = 32; off > 0; off >>= 1) {
        tot.n += __shfl_xor(tot.n, off, 64);
        tot.s1 += __shfl_xor(tot.s1, off, 64);
        tot.s2 += __shfl_xor(tot.s2, off, 64);
        long long lo3 = (long long)(uint64_t)(unsigned __int128)tot.s3;
        long long hi3 = (long long)(uint64_t)((unsigned __int128)tot.s3 >> 64);
        long long lo4 = (long long)(uint64_t)(unsigned __int128)tot.s4;
        long long hi4 = (long long)(uint64_t)((unsigned __int128)tot.s4 >> 64);
        const __int128 o3 = (__int128)(((unsigned __int128)(uint64_t)__shfl_xor(hi3, off, 64) << 64) |
                                       (uint64_t)__shfl_xor(lo3, off, 64));
        const __int128 o4 = (__int128)(((unsigned __int128)(uint64_t)__shfl_xor(hi4, off, 64) << 64) |
                                       (uint64_t)__shfl_xor(lo4, off, 64));
        tot.s3 += o3;
        tot.s4 += o4;
    }
    out = tot;
}

// Per row y (relative to the row start): (sum P, sum P^2, sum P^3, sum P^4),
// 6 int64 per row: s1, s2, s3 lo/hi, s4 lo/hi.
__global__ __launch_bounds__(256) void kpz_row_mom4_kernel(const uint32_t *words, uint32_t L,
                                                           uint32_t W, long long *rows6)
{
    __shared__ uint2 lut[256];
    lut[threadIdx.x] = lut8_mom4(threadIdx.x);
    __syncthreads();
    const uint32_t lane = threadIdx.x & 63u;
    for (uint32_t row = blockIdx.x * 4u + (threadIdx.x >> 6); row < L; row += gridDim.x * 4u) {
        Mom4 m;
        row_mom4(words + (size_t)row * W, W, lut, lane, m);
        if (lane == 0) {
            long long *o = rows6 + 6 * (size_t)row;
            o[0] = m.s1;
            o[1] = m.s2;
            o[2] = (long long)(uint64_t)(unsigned __int128)m.s3;
            o[3] = (long long)(uint64_t)((unsigned __int128)m.s3 >> 64);
            o[4] = (long long)(uint64_t)(unsigned __int128)m.s4;
            o[5] = (long long)(uint64_t)((unsigned __int128)m.s4 >> 64);
        }
    }
}

// One work-group: rows shifted by their column-0 height c_y and summed;
// res = M1..M4 as (lo, hi) pairs.
__global__ __launch_bounds__(256) void kpz_mom4_finalize_kernel(const uint32_t *words, uint32_t L,
                                                                uint32_t W, const long long *rows6,
                                                                long long *res)
{
    constexpr int NT = 256;
    __shared__ long long sc[NT];
    __shared__ __int128 acc[4][NT];
    const uint32_t tid = threadIdx.x;
    const uint32_t per = (L + NT - 1) / NT;
    const uint32_t y0 = min(L, tid * per), y1 = min(L, y0 + per);
    long long loc = 0;
    for (uint32_t y = y0; y < y1; ++y) loc += ((words[(size_t)y * W] >> 1) & 1u) ? 1 : -1;
    sc[tid] = loc;
    __syncthreads();
    for (uint32_t off = 1; off < NT; off <<= 1) {
        const long long v = tid >= off ? sc[tid - off] : 0;
        __syncthreads();
        sc[tid] += v;
        __syncthreads();
    }
    long long c = sc[tid] - loc;
    __int128 t1 = 0, t2 = 0, t3 = 0, t4 = 0;
    for (uint32_t y = y0; y < y1; ++y) {
        const long long *o = rows6 + 6 * (size_t)y;
        Mom4 m;
        m.n = L;
        m.s1 = o[0];
        m.s2 = o[1];
        m.s3 = (__int128)(((unsigned __int128)(uint64_t)o[3] << 64) | (uint64_t)o[2]);
        m.s4 = (__int128)(((unsigned __int128)(uint64_t)o[5] << 64) | (uint64_t)o[4]);
        const Mom4 r = mom4_shift(m, c);
        t1 += r.s1;
        t2 += r.s2;
        t3 += r.s3;
        t4 += r.s4;
        c += ((words[(size_t)y * W] >> 1) & 1u) ? 1 : -1;
    }
    acc[0][tid] = t1;
    acc[1][tid] = t2;
    acc[2][tid] = t3;
    acc[3][tid] = t4;
    __syncthreads();
    for (uint32_t off = NT / 2; off > 0; off >>= 1) {
        if (tid < off)
            for (int k = 0; k < 4; ++k) acc[k][tid] += acc[k][tid + off];
        __syncthreads();
    }
    if (tid == 0)
        for (int k = 0; k < 4; ++k) {
            const unsigned __int128 u = (unsigned __int128)acc[k][0];
            res[2 * k] = (long long)(uint64_t)u;
            res[2 * k + 1] = (long long)(uint64_t)(u >> 64);
        }
}

// ------------------------------------------------------------ invariants
//
// The surface constraints of Sec. 2.1 on the stored slopes: around every
// plaquette the four slopes sum to zero, sigma_x(x,y) + sigma_y(x+1,y) =
// sigma_y(x,y) + sigma_x(x,y+1), and along the periodic row 0 (column 0)
// the sigma_x (sigma_y) sum to zero.  With every plaquette closed, the
// sigma_x sums of rows y and y+1 differ by the sum of sigma_y(x+1,y) -
// sigma_y(x,y) over the periodic row, which is zero, so all rows (and
// likewise all columns) share the sums of row 0 and column 0.
//
// In bits (a = sigma_x(x,y) > 0, b = sigma_y(x+1,y) > 0, c = sigma_x(x,y+1)
// > 0, d = sigma_y(x,y) > 0) a plaquette is closed iff {a, b} = {c, d} as
// multisets: a ^ b = c ^ d and a & b = c & d.  A thread takes U consecutive
// words of a row (one 16-byte load for U = 4) and walks down R rows, keeping
// the row above from one iteration to the next; the word to the right of its
// last word gives sigma_y(x+1,y) of the last site.  out[0] counts open
// plaquettes, out[1] the sigma_x = +1 bonds of row 0, out[2] the sigma_y = +1
// bonds of column 0 (one atomic per wave each).
template <int U>
__global__ __launch_bounds__(256) void kpz_check_kernel(const uint32_t *words, uint32_t L,
                                                        uint32_t W, uint32_t R,
                                                        unsigned long long *out)
{
    const uint32_t ng = W / U;
    const uint64_t gid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t chunk = gid / ng;
    const uint32_t g = (uint32_t)(gid - chunk * ng);
    uint32_t open = 0, row0 = 0, col0 = 0;
    if (chunk * R < L) {
        const uint32_t y0 = (uint32_t)chunk * R, y1 = min(L, y0 + R);
        const uint32_t xn = (g + 1 == ng) ? 0u : (g + 1) * U;   // word right of the last
        uint32_t cur[U], cn;
        auto load = [&](uint32_t y, uint32_t (&v)[U], uint32_t &n) {
            const uint32_t *rp = words + (size_t)y * W;
            if constexpr (U == 4) {
                const uint4 q = *(const uint4 *)(rp + g * 4u);
                v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
            } else {
#pragma unroll
                for (int u = 0; u < U; ++u) v[u] = rp[g * U + u];
            }
            n = rp[xn];
        };
        load(y0, cur, cn);
        for (uint32_t y = y0; y < y1; ++y) {
            uint32_t up[U], un;
            load(y + 1 == L ? 0u : y + 1, up, un);
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const uint32_t w = cur[u], wn = (u + 1 < U) ? cur[u + 1] : cn;
                const uint32_t a = w, d = w >> 1, c = up[u];
                const uint32_t b = __builtin_amdgcn_alignbit(wn, w, 3);   // sigma_y(x+1, y)
                open += __popc(((a ^ b ^ c ^ d) | ((a & b) ^ (c & d))) & 0x55555555u);
                if (y == 0) row0 += __popc(w & 0x55555555u);
            }
            if (g == 0) col0 += (cur[0] >> 1) & 1u;
#pragma unroll
            for (int u = 0; u < U; ++u) cur[u] = up[u];
            cn = un;
        }
    }
    for (int off = 32; off > 0; off >>= 1) {
        open += __shfl_xor(open, off);
        row0 += __shfl_xor(row0, off);
        col0 += __shfl_xor(col0, off);
    }
    if ((threadIdx.x & 63u) == 0) {
        if (open) atomicAdd(out, (unsigned long long)open);
        if (row0) atomicAdd(out + 1, (unsigned long long)row0);
        if (col0) atomicAdd(out + 2, (unsigned long long)col0);
    }
}

// ------------------------------------------------------------ calibration
//
// VALU issue rate of the sweep's instruction mix, measured: each wave runs
// `iters` rounds of VALU_PROBE_OPS independent 32-bit bitwise instructions
// (v_bfi_b32, v_xor_b32, v_bitop3_b32 on eight registers, written in asm so
// the count is exact), the only other work being the scalar loop counter.
// Wave instructions per second = waves * iters * VALU_PROBE_OPS / time.

constexpr uint32_t VALU_PROBE_OPS = 192;

__global__ __launch_bounds__(256) void kpz_valu_probe_kernel(uint32_t *out, uint32_t iters)
{
    uint32_t a0 = threadIdx.x, a1 = a0 * 3u, a2 = a0 * 5u, a3 = a0 * 7u;
    uint32_t a4 = a0 ^ 0x55u, a5 = a0 ^ 0xAAu, a6 = a0 + 11u, a7 = a0 + 13u;
    const uint32_t m = 0x0F0F3355u ^ blockIdx.x;
    for (uint32_t it = 0; it < iters; ++it) {
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            asm volatile(
                "v_bfi_b32 %0, %8, %0, %1\n\t"
                "v_bfi_b32 %1, %8, %1, %2\n\t"
                "v_bfi_b32 %2, %8, %2, %3\n\t"
                "v_bfi_b32 %3, %8, %3, %4\n\t"
                "v_bfi_b32 %4, %8, %4, %5\n\t"
                "v_bfi_b32 %5, %8, %5, %6\n\t"
                "v_bfi_b32 %6, %8, %6, %7\n\t"
                "v_bfi_b32 %7, %8, %7, %0\n\t"
                "v_xor_b32 %0, %0, %2\n\t"
                "v_xor_b32 %1, %1, %3\n\t"
                "v_xor_b32 %2, %2, %4\n\t"
                "v_xor_b32 %3, %3, %5\n\t"
                "v_xor_b32 %4, %4, %6\n\t"
                "v_xor_b32 %5, %5, %7\n\t"
                "v_xor_b32 %6, %6, %0\n\t"
                "v_xor_b32 %7, %7, %1\n\t"
                "v_bitop3_b32 %0, %0, %3, %8 bitop3:0x96\n\t"
                "v_bitop3_b32 %1, %1, %4, %8 bitop3:0x96\n\t"
                "v_bitop3_b32 %2, %2, %5, %8 bitop3:0x96\n\t"
                "v_bitop3_b32 %3, %3, %6, %8 bitop3:0x96\n\t"
                "v_bitop3_b32 %4, %4, %7, %8 bitop3:0x96\n\t"
                "v_bitop3_b32 %5, %5, %0, %8 bitop3:0x96\n\t"
                "v_bitop3_b32 %6, %6, %1, %8 bitop3:0x96\n\t"
                "v_bitop3_b32 %7, %7, %2, %8 bitop3:0x96"
                : "+v"(a0), "+v"(a1), "+v"(a2), "+v"(a3), "+v"(a4), "+v"(a5), "+v"(a6), "+v"(a7)
                : "v"(m));
        }
    }
    out[blockIdx.x * blockDim.x + threadIdx.x] = a0 ^ a1 ^ a2 ^ a3 ^ a4 ^ a5 ^ a6 ^ a7;
}

// ------------------------------------------------------------ ensemble
//
// Many independent lattices ("members", each with its own L, p, q and seed,
// one common block shape) advance together: one launch runs one MCS of
// every member (all their blocks in one grid); in-place members need one
// more launch that merges their straddling words, two-buffer members none.
// Rounds are separated by kernel boundaries, which make each round's words
// visible to the next at no extra cost.

// Moment pass inputs of one member.  With `state` set (ensembles) the
// current buffer and its rotation come from the member's sweep arguments;
// otherwise `words` is the current buffer and `rot` its rotation (pool jobs,
// filled by the host).
struct MemberRows {
    const uint32_t *words;
    long long *rowA, *rowB;
    const long long *slots;
    uint32_t L, W;
    const SweepArgs *state;
    Rot rot;
};

__device__ __forceinline__ const uint32_t *member_current(const MemberRows &m, Rot &rot)
{
    if (!m.state) {
        rot = m.rot;
        return m.words;
    }
    const SweepArgs &a = *m.state;
    if (!a.db) {
        rot = Rot{0u, 0u, 0u, a.Bx, 0u, 0u};
        return a.words;
    }
    rot = Rot{a.prev_valid, a.prev_t, a.prev_res, a.Bx, a.seed_lo, a.seed_hi};
    return a.cur0 ? a.alt : a.words;
}

// The arguments of launch (k, res) of a call for a member whose state at the
// call's start is in `a` (two-buffer mode: which buffer to read and write,
// and how the input is rotated).
__device__ __forceinline__ void member_launch_args(SweepArgs &a, uint32_t k, uint32_t res)
{
    if (a.db) {
        const uint32_t moves = 16u / a.nsteps;
        const uint32_t n = k * moves + res;            // launches before this one
        const uint32_t cur = a.cur0 ^ (n & 1u);
        uint32_t *b0 = a.words, *b1 = a.alt;
        a.src = cur ? b1 : b0;
        a.words = cur ? b0 : b1;
        if (n > 0) {
            a.prev_valid = 1u;
            a.prev_t = a.t + (n - 1) / moves;
            a.prev_res = (n - 1) % moves;
        }
    }
    a.t += k;
    a.res = res;
}

// One round of the ensemble: every block of members [0, nmem) runs MCS
// t_r + k (t_r = the member's t at the start of the call), one wave per
// block.  Wave g of the grid is block g - bprefix[r] of member r (bprefix =
// prefix sums of the members' block counts); each member has its own block
// shape.
__global__ __launch_bounds__(256) void kpz_batch_round_kernel(const SweepArgs *members,
                                                              const uint32_t *bprefix,
                                                              uint32_t nmem, uint32_t k,
                                                              uint32_t res)
{
    // XCD-aware order (the grid is padded to a multiple of 8 work-groups):
    // group i takes the waves of virtual group (i mod 8) n/8 + i/8
    const uint32_t wg = (blockIdx.x & 7u) * (gridDim.x >> 3) + (blockIdx.x >> 3);
    const uint32_t g = __builtin_amdgcn_readfirstlane(wg * 4u + (threadIdx.x >> 6));
    if (g >= bprefix[nmem]) return;
    uint32_t lo = 0, hi = nmem;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (bprefix[mid] <= g) lo = mid;
        else hi = mid;
    }
    const uint32_t r = __builtin_amdgcn_readfirstlane(lo);
    SweepArgs a = members[r];
    member_launch_args(a, k, res);
    const uint32_t b = g - bprefix[r];
    if (a.W % 4 == 0) {
        if (a.acc) sweep_block<true, false, true>(a, b);
        else sweep_block<false, false, true>(a, b);
    } else {
        if (a.acc) sweep_block<true, false, false>(a, b);
        else sweep_block<false, false, false>(a, b);
    }
}

// Straddling words of members [0, nmem) after round (k, res); sprefix =
// prefix sums of L_r * nbx_r.
__global__ void kpz_batch_merge_kernel(const SweepArgs *members, const unsigned long long *sprefix,
                                       uint32_t nmem, uint32_t k, uint32_t res)
{
    const uint64_t total = sprefix[nmem];
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < total;
         i += (uint64_t)gridDim.x * blockDim.x) {
        uint32_t lo = 0, hi = nmem;
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (sprefix[mid] <= i) lo = mid;
            else hi = mid;
        }
        SweepArgs a = members[lo];
        if (a.db) continue;                       // two-buffer members share no words
        a.t += k;
        a.res = res;
        const uint32_t ox = origin_x(a);
        if ((ox & 15u) != 0) merge_one(a, ox, i - sprefix[lo]);
    }
}

__global__ void kpz_zero_kernel(uint32_t *p, uint64_t n)
{
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

__global__ void kpz_batch_advance_kernel(SweepArgs *members, uint32_t n, uint32_t dt)
{
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        SweepArgs &a = members[i];
        if (a.db && dt) {
            const uint32_t moves = 16u / a.nsteps;
            a.cur0 ^= (dt * moves) & 1u;
            a.prev_valid = 1u;
            a.prev_t = a.t + dt - 1u;
            a.prev_res = moves - 1u;
        }
        a.t += dt;
    }
}

// Ensemble members' `words` in the documented layout: one work-group per
// row (rows numbered over the members as in the moment pass) copies the
// current buffer's row through LDS, undoing the rotation; then
// kpz_batch_settle_kernel marks every member as held in buffer 0.
__global__ __launch_bounds__(256) void kpz_batch_sync_kernel(const MemberRows *mr,
                                                             const uint32_t *rprefix, uint32_t n)
{
    extern __shared__ uint32_t rowbuf[];
    const uint32_t total = rprefix[n];
    for (uint32_t g = blockIdx.x; g < total; g += gridDim.x) {
        uint32_t lo = 0, hi = n;
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (rprefix[mid] <= g) lo = mid;
            else hi = mid;
        }
        const MemberRows m = mr[lo];
        const uint32_t row = g - rprefix[lo];
        Rot rot;
        const uint32_t *cur = member_current(m, rot);
        const uint32_t s = rot_sites(rot);
        const uint32_t sw = s >> 4, rot2 = 2u * (s & 15u);
        const uint32_t *src = cur + (size_t)row * m.W;
        for (uint32_t w = threadIdx.x; w < m.W; w += blockDim.x) rowbuf[w] = src[w];
        __syncthreads();
        uint32_t *dst = (m.state ? m.state->words : (uint32_t *)m.words) + (size_t)row * m.W;
        for (uint32_t w = threadIdx.x; w < m.W; w += blockDim.x) {
            const uint32_t w1 = w >= sw ? w - sw : w + m.W - sw;
            const uint32_t pv = rowbuf[w1 ? w1 - 1 : m.W - 1];
            dst[w] = rot2 ? __builtin_amdgcn_alignbit(rowbuf[w1], pv, 32u - rot2) : rowbuf[w1];
        }
        __syncthreads();
    }
}

__global__ void kpz_batch_settle_kernel(SweepArgs *members, uint32_t n)
{
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        members[i].cur0 = 0u;
        members[i].prev_valid = 0u;
    }
}

// Row moments of all members: wave tasks numbered consecutively over the
// members (tprefix = prefix sums of L / R, R = 64 / row_lanes(W) rows per
// task, one member per task).
__global__ __launch_bounds__(256) void kpz_batch_rows_kernel(const MemberRows *mr,
                                                             const uint32_t *tprefix, uint32_t n)
{
    __shared__ uint32_t lut[LUT_WORDS];
    fill_row_lut(lut);
    __syncthreads();
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t total = tprefix[n];
    for (uint32_t g = blockIdx.x * 4u + wv; g < total; g += gridDim.x * 4u) {
        uint32_t lo = 0, hi = n;
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (tprefix[mid] <= g) lo = mid;
            else hi = mid;
        }
        const MemberRows m = mr[lo];
        const uint32_t G = row_lanes(m.W), R = 64u / G;
        const uint32_t row = (g - tprefix[lo]) * R + lane / G;
        if (row < m.L) {   // a whole lane group is in or out
            Rot rot;
            const uint32_t *cur = member_current(m, rot);
            long long A, B;
            uint32_t first;
            const uint32_t *rp = cur + (size_t)row * m.W;
            if ((m.W & 511u) == 0)
                row_moments<8>(rp, m.W, lut, lane & (G - 1u), G, A, B, first);
            else
                row_moments<4>(rp, m.W, lut, lane & (G - 1u), G, A, B, first);
            if ((lane & (G - 1u)) == 0) {
                m.rowA[row] = A;
                m.rowB[row] = (B << 1) | ((first >> 1) & 1u);   // + sigma_y of the first stored site
            }
        }
    }
}

// Members of at most SMALL_ROWS rows: one work-group of 1024 threads per
// member computes the row sums into LDS and finalizes them (one launch per
// sample instead of two); results as for kpz_batch_finalize_kernel.
__global__ __launch_bounds__(1024) void kpz_batch_moments_small_kernel(const MemberRows *mr,
                                                                       uint32_t n, uint32_t nslots,
                                                                       long long *res, uint32_t k)
{
    __shared__ uint32_t lut[256];
    __shared__ long long rA[SMALL_ROWS], rB[SMALL_ROWS];
    fill_row_lut<1>(lut);
    __syncthreads();
    const uint32_t r = blockIdx.x;
    const MemberRows m = mr[r];
    Rot rot;
    const uint32_t *cur = member_current(m, rot);
    small_rows(cur, m.L, m.W, lut, rA, rB);
    __syncthreads();
    finalize_moments<1024>(m.L, rA, rB, m.slots, nslots, res + ((size_t)k * n + r) * 4, cur,
                           rot_sites(rot));
}

// One work-group per member; results of sample `k` go to res[(k n + r) 4 ..].
__global__ __launch_bounds__(256) void kpz_batch_finalize_kernel(const MemberRows *mr, uint32_t n,
                                                                 uint32_t nslots, long long *res,
                                                                 uint32_t k)
{
    const uint32_t r = blockIdx.x;
    const MemberRows m = mr[r];
    Rot rot;
    const uint32_t *cur = member_current(m, rot);
    finalize_moments<256>(m.L, m.rowA, m.rowB, m.slots, nslots, res + ((size_t)k * n + r) * 4, cur,
                          rot_sites(rot));
}

}  // namespace

// ================================================================ host

struct kpz_sim {
    kpz_params prm;
    uint32_t Bx, By;
    uint32_t *words;
    size_t words_bytes;
    uint8_t *ws;
    size_t ws_bytes;
    hipStream_t stream;
    int64_t t;
    uint64_t P, Q;
    // two-buffer mode: buf[cur] holds the state, rotated as written by the
    // launch (rot_t, rot_res) when rot_valid
    bool db;
    bool dt;                       // double tiling at the device layer
    bool dt_ahead;                 // ... with diagonal partner sets run together
    uint32_t *buf[2];
    int cur;
    uint32_t rot_valid, rot_t, rot_res;
    char err[256];
};

namespace {

bool is_pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }

int ilog2(uint32_t v)
{
    int r = 0;
    while ((1u << r) < v) ++r;
    return r;
}

uint64_t threshold(double prob)
{
    if (prob >= 1.0) return 1ull << 32;
    if (prob <= 0.0) return 0;
    return (uint64_t)(prob * 4294967296.0);
}

// A block shape the sweep takes: whole words per row (Bx a multiple of 16),
// whole tiles (By a multiple of 4), a row of at most 32 tiles or of whole row
// groups of 32 tiles (Bx <= 128 or a multiple of 128, at most 1024), and at
// most 64 (row group, tile row) pairs, one per lane of the block's wave.
bool block_ok(int64_t bx, int64_t by)
{
    if (bx < 16 || bx > 1024 || bx % 16 || by < TILE || by % TILE) return false;
    if (bx > (int64_t)GROUP_SITES && bx % GROUP_SITES) return false;
    const int64_t lanes = (bx > (int64_t)GROUP_SITES ? bx / GROUP_SITES : 1) * (by / TILE);
    return lanes <= 64;
}

// Default block shape for L.  L a multiple of 128: Bx the largest power of
// two <= 256 dividing L, By the largest <= 128 (one full wave per block where
// L allows: two row groups of 128 sites in 32 tile rows; the fastest of the
// full shapes at L = 65536).  Other L (multiples of 16): the valid shape
// dividing L with the most tiles per wave, then the widest.
std::pair<int64_t, int64_t> default_block(int64_t L)
{
    if (L % 128 == 0) {
        int64_t dx = 256, dy = 128;
        while (L % dx) dx >>= 1;
        while (L % dy) dy >>= 1;
        return {dx, dy};
    }
    int64_t best_x = 16, best_y = TILE, best_area = 0;
    for (int64_t bx = 16; bx <= 512 && bx <= L; bx += 16) {
        if (L % bx) continue;
        for (int64_t by = TILE; by <= L && by <= 64 * TILE; by += TILE) {
            if (L % by || !block_ok(bx, by)) continue;
            const int64_t area = bx * by;
            if (area > best_area || (area == best_area && bx > best_x)) {
                best_area = area;
                best_x = bx;
                best_y = by;
            }
        }
    }
    return {best_x, best_y};
}

// Philox4x32 with the lattice draws' round count, on the host: the order of
// the block sets of an MCS is needed before its launches are issued.
void philox_host(uint32_t c[4], uint32_t k0, uint32_t k1)
{
    for (int r = 0; r < kpzdev::LATTICE_ROUNDS; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c[1] ^ k0;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c[3] ^ k1;
        c[1] = (uint32_t)p1;
        c[3] = (uint32_t)p0;
        c[0] = n0;
        c[2] = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

// The four block sets of MCS t in launch order: ordering number
// floor(w0 24 / 2^32) of draw (DTORDER, t), the 24 orderings of 0..3 in
// lexicographic order (the device's dt_set for every phase at once).
void dt_order_host(uint32_t t, uint64_t seed, uint32_t perm[4])
{
    uint32_t c[4] = {0u, 0u, t, TAG_DTORDER << 24};
    philox_host(c, (uint32_t)seed, (uint32_t)(seed >> 32));
    uint32_t idx = (uint32_t)(((uint64_t)c[0] * 24u) >> 32);
    uint32_t pool[4] = {0u, 1u, 2u, 3u};
    uint32_t n = 4;
    const uint32_t fact[4] = {1u, 1u, 2u, 6u};
    for (uint32_t i = 0; i < 4; ++i) {
        const uint32_t f = fact[n - 1];
        const uint32_t pick = idx / f;
        idx %= f;
        perm[i] = pool[pick];
        for (uint32_t k = pick; k + 1 < n; ++k) pool[k] = pool[k + 1];
        --n;
    }
}

// Resolves defaults and validates; fills block shape.
kpz_status resolve(const kpz_params *p, uint32_t *Bx, uint32_t *By)
{
    if (!p) return KPZ_EINVAL;
    if (p->L < 16 || (p->L % 16) != 0) return KPZ_EINVAL;
    if (!(p->p >= 0.0 && p->p <= 1.0 && p->q >= 0.0 && p->q <= 1.0)) return KPZ_EINVAL;
    if ((p->flags & ~(KPZ_FLAG_IN_PLACE | KPZ_FLAG_DEVICE_DT | KPZ_FLAG_DT_AHEAD)) != 0)
        return KPZ_EINVAL;
    if ((p->flags & KPZ_FLAG_DT_AHEAD) && !(p->flags & KPZ_FLAG_DEVICE_DT)) return KPZ_EINVAL;
    if (p->moves != 0 && p->moves != 1 && p->moves != 2 && p->moves != 4 && p->moves != 8 &&
        p->moves != 16)
        return KPZ_EINVAL;
    const int tx = p->tile_x ? p->tile_x : TILE, ty = p->tile_y ? p->tile_y : TILE;
    if (tx != TILE || ty != TILE) return KPZ_EINVAL;
    const int64_t L = p->L;
    const int64_t bx = p->block_x ? p->block_x : default_block(L).first;
    const int64_t by = p->block_y ? p->block_y : default_block(L).second;
    if (!block_ok(bx, by)) return KPZ_EINVAL;
    if (L % bx || L % by) return KPZ_EINVAL;
    if (p->flags & KPZ_FLAG_DEVICE_DT) {
        // four block sets need an even number of blocks along both axes
        const int64_t nbx = L / bx, nby = L / by;
        if (nbx < 2 || nby < 2 || (nbx & 1) || (nby & 1)) return KPZ_EINVAL;
        if (p->moves > 1) return KPZ_EINVAL;
    }
    *Bx = (uint32_t)bx;
    *By = (uint32_t)by;
    return KPZ_OK;
}

uint32_t moves_of(const kpz_params *p) { return p->moves ? (uint32_t)p->moves : 1u; }

size_t ws_side_end(int64_t L, int64_t Bx)
{
    // header, flip-counter slots, six int64 per row (row moments: two for
    // W^2, six for the fourth-order moments) and the side buffer of the
    // straddling words (two uint32 per row and block column)
    return (size_t)WS_HEADER + sizeof(long long) * NSLOTS + 6 * sizeof(long long) * (size_t)L +
           2 * sizeof(uint32_t) * (size_t)L * (size_t)(L / Bx);
}

size_t ws_needed(int64_t L, int64_t Bx, uint32_t flags)
{
    // plus, in two-buffer mode, the second lattice buffer (256-byte aligned)
    const size_t side_end = ws_side_end(L, Bx);
    if (flags & (KPZ_FLAG_IN_PLACE | KPZ_FLAG_DEVICE_DT)) return side_end;
    return ((side_end + 255) & ~(size_t)255) + (size_t)L * (size_t)L / 4;
}

kpz_status hip_fail(kpz_sim *s, hipError_t e, const char *what)
{
    if (s) snprintf(s->err, sizeof s->err, "%s: %s", what, hipGetErrorString(e));
    return KPZ_EHIP;
}

long long *ws_res(kpz_sim *s) { return (long long *)s->ws; }
long long *ws_slots(kpz_sim *s) { return (long long *)(s->ws + WS_HEADER); }
long long *ws_rowA(kpz_sim *s) { return ws_slots(s) + NSLOTS; }
long long *ws_rowB(kpz_sim *s) { return ws_rowA(s) + s->prm.L; }
uint32_t *ws_side(kpz_sim *s) { return (uint32_t *)(ws_rowA(s) + 6 * (size_t)s->prm.L); }
uint32_t *ws_alt(kpz_sim *s)
{
    return (uint32_t *)(s->ws + ((ws_side_end(s->prm.L, s->Bx) + 255) & ~(size_t)255));
}
Rot sim_rot(const kpz_sim *s)
{
    return Rot{s->rot_valid, s->rot_t, s->rot_res, s->Bx, (uint32_t)s->prm.seed,
               (uint32_t)(s->prm.seed >> 32)};
}

// Block shape fields of the sweep arguments (shape validated by resolve).
void set_shape(SweepArgs &a, uint32_t L, uint32_t Bx, uint32_t By)
{
    a.L = L;
    a.W = L / 16;
    a.Bx = Bx;
    a.By = By;
    a.nbx = L / Bx;
    a.nby = L / By;
    a.nw = Bx / 16;
    a.nqx = Bx > GROUP_SITES ? Bx / GROUP_SITES : 1u;
    a.ntg = (Bx > GROUP_SITES ? GROUP_SITES : Bx) / TILE;
    a.nwg = a.ntg / 4;
    a.nty = By / TILE;
    a.mnty = (65536u + a.nty - 1u) / a.nty;
    a.su_u = (a.nw + 7u) / 4u;
    a.su_m = (65536u + a.su_u - 1u) / a.su_u;
    a.su_r = 64u / a.su_u;
    a.su_nc = (a.nty + a.su_r - 1u) / a.su_r;
    a.su = a.By * a.su_u;
}

// Waves (blocks) per work-group: four when the block count allows;
// KPZ_WAVES_PER_GROUP=1 selects one.  The launch shape changes no result.
uint32_t waves_per_group(uint32_t nblocks)
{
    if (const char *env = getenv("KPZ_WAVES_PER_GROUP"))
        if (atoi(env) == 1) return 1u;
    return nblocks % 4 == 0 ? 4u : 1u;
}

// One wave per block.
template <bool ACC, bool VEC, int XN, int WY>
hipError_t launch_sweep_v(const SweepArgs &a, uint32_t nblocks, hipStream_t st)
{
    const uint32_t wpg = waves_per_group(nblocks);
    const uint32_t grid = nblocks / wpg;
    SweepArgs b = a;
    b.xcd = (grid % 8u) == 0 ? a.xcd : 0u;
    if (VEC && (b.su > STAGE_UNITS || b.su_nc > STAGE_NC)) return hipErrorInvalidValue;
    hipLaunchKernelGGL((kpz_sweep_kernel<ACC, VEC, XN, WY>), dim3(grid), dim3(64 * wpg),
                       VEC ? (size_t)wpg * b.su * sizeof(uint4) : 0, st, b, nblocks);
    return hipGetLastError();
}

template <bool ACC, bool VEC>
hipError_t launch_sweep_x(const SweepArgs &a, uint32_t nblocks, hipStream_t st)
{
    // XN = 1 only with several row groups per tile row (8 words per group);
    // a single block along x with one group is XN = 3
    const bool wy = a.nby == 1;
    if (a.nqx > 1) return wy ? launch_sweep_v<ACC, VEC, 1, 1>(a, nblocks, st)
                             : launch_sweep_v<ACC, VEC, 1, 0>(a, nblocks, st);
    if (a.nbx == 1) return wy ? launch_sweep_v<ACC, VEC, 3, 1>(a, nblocks, st)
                              : launch_sweep_v<ACC, VEC, 3, 0>(a, nblocks, st);
    return wy ? launch_sweep_v<ACC, VEC, 0, 1>(a, nblocks, st)
              : launch_sweep_v<ACC, VEC, 0, 0>(a, nblocks, st);
}

template <bool ACC>
hipError_t launch_sweep(const SweepArgs &a, uint32_t nblocks, hipStream_t st)
{
    return (a.W % 4 == 0) ? launch_sweep_x<ACC, true>(a, nblocks, st)
                          : launch_sweep_x<ACC, false>(a, nblocks, st);
}

template <bool ACC, bool VEC, int XN>
hipError_t launch_dt_v(const SweepArgs &a, uint32_t phase, uint32_t nset, hipStream_t st)
{
    const uint32_t wpg = waves_per_group(nset);
    const uint32_t waves = a.ahead ? 2u * nset : nset;
    hipLaunchKernelGGL((kpz_dt_kernel<ACC, VEC, XN>), dim3(waves / wpg), dim3(64 * wpg), 0, st,
                       a, phase, nset);
    return hipGetLastError();
}

template <bool ACC>
hipError_t launch_dt(const SweepArgs &a, uint32_t phase, uint32_t nset, hipStream_t st)
{
    // double tiling needs at least two blocks along each axis: no wrap
    const bool xn = a.nqx > 1;
    if (a.W % 4 == 0)
        return xn ? launch_dt_v<ACC, true, 1>(a, phase, nset, st)
                  : launch_dt_v<ACC, true, 0>(a, phase, nset, st);
    return xn ? launch_dt_v<ACC, false, 1>(a, phase, nset, st)
              : launch_dt_v<ACC, false, 0>(a, phase, nset, st);
}

}  // namespace


// ------------------------------------------------------------ ensemble host

namespace {

constexpr int BATCH_SLOTS = 64;   // flip-counter slots per member

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

struct BatchLayout {
    std::vector<uint32_t> Bx, By;   // block shape of each member
    uint32_t moves;                 // origin moves per MCS, common to all members
    bool db;                        // two-buffer members (every L <= 65536)
    uint32_t maxW;                  // longest row (words)
    std::vector<size_t> off_alt;    // second lattice buffer of each member (two-buffer mode)
    std::vector<size_t> word_off;   // per member, in words
    size_t words_bytes;
    size_t off_members, off_bprefix, off_sprefix, off_rprefix, off_tprefix, off_rows, off_res,
        off_slots;
    std::vector<size_t> off_rowA, off_rowB, off_side;
    size_t ws_bytes;
};

kpz_status batch_layout(const kpz_params *m, int32_t n, BatchLayout *lay)
{
    if (!m || n < 1) return KPZ_EINVAL;
    for (int32_t r = 0; r < n; ++r)
        if (moves_of(&m[r]) != moves_of(&m[0])) return KPZ_EINVAL;
    lay->moves = moves_of(&m[0]);
    lay->Bx.resize(n);
    lay->By.resize(n);
    for (int32_t r = 0; r < n; ++r) {
        const kpz_status st = resolve(&m[r], &lay->Bx[r], &lay->By[r]);
        if (st != KPZ_OK) return st;
    }
    lay->word_off.resize(n);
    size_t w = 0;
    for (int32_t r = 0; r < n; ++r) {
        lay->word_off[r] = w;
        w += align256((size_t)m[r].L * m[r].L / 4) / 4;
    }
    lay->words_bytes = 4 * w;
    lay->db = true;
    lay->maxW = 0;
    for (int32_t r = 0; r < n; ++r) {
        if (m[r].flags & KPZ_FLAG_DEVICE_DT) return KPZ_EINVAL;   // dead borders only
        if (m[r].L > 65536 || (m[r].flags & KPZ_FLAG_IN_PLACE)) lay->db = false;
        lay->maxW = std::max(lay->maxW, (uint32_t)(m[r].L / 16));
    }
    size_t o = 0;
    lay->off_members = o;  o = align256(o + sizeof(SweepArgs) * (size_t)n);
    lay->off_bprefix = o;  o = align256(o + 4 * ((size_t)n + 1));
    lay->off_sprefix = o;  o = align256(o + 8 * ((size_t)n + 1));
    lay->off_rprefix = o;  o = align256(o + 4 * ((size_t)n + 1));
    lay->off_tprefix = o;  o = align256(o + 4 * ((size_t)n + 1));
    lay->off_rows = o;     o = align256(o + sizeof(MemberRows) * (size_t)n);
    lay->off_res = o;      o = align256(o + 4 * sizeof(long long) * (size_t)n * KPZ_BATCH_MAX_SAMPLES);
    lay->off_slots = o;    o = align256(o + sizeof(long long) * BATCH_SLOTS * (size_t)n);
    lay->off_rowA.resize(n);
    lay->off_rowB.resize(n);
    lay->off_side.resize(n);
    for (int32_t r = 0; r < n; ++r) {
        const size_t L = (size_t)m[r].L;
        lay->off_rowA[r] = o; o = align256(o + 8 * L);
        lay->off_rowB[r] = o; o = align256(o + 8 * L);
        lay->off_side[r] = o; o = align256(o + 4 * 2 * L * (L / lay->Bx[r]));
    }
    lay->off_alt.assign(n, 0);
    if (lay->db)
        for (int32_t r = 0; r < n; ++r) {
            const size_t L = (size_t)m[r].L;
            lay->off_alt[r] = o; o = align256(o + L * L / 4);
        }
    lay->ws_bytes = o;
    return KPZ_OK;
}

// One round (residency res of MCS k of the call) of members [0, nmem) plus
// the merge of their straddling words.  nblocks = bprefix[nmem], mwords =
// sprefix[nmem].
hipError_t round_launch(uint32_t nblocks, uint64_t mwords, hipStream_t st,
                        const SweepArgs *members, const uint32_t *bprefix,
                        const unsigned long long *sprefix, uint32_t nmem, uint32_t k,
                        uint32_t res, bool merge)
{
    // four waves (blocks) per work-group; the kernel's XCD map needs a
    // multiple of 8 work-groups
    const uint32_t grid = (((nblocks + 3u) / 4u) + 7u) & ~7u;
    hipLaunchKernelGGL(kpz_batch_round_kernel, dim3(grid), dim3(256), 0, st, members, bprefix,
                       nmem, k, res);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !merge) return e;
    const uint32_t mgrid = (uint32_t)((mwords + 255) / 256 < 8192 ? (mwords + 255) / 256 : 8192);
    hipLaunchKernelGGL(kpz_batch_merge_kernel, dim3(mgrid), dim3(256), 0, st, members, sprefix,
                       nmem, k, res);
    return hipGetLastError();
}

}  // namespace

struct kpz_batch {
    int32_t n;
    std::vector<kpz_params> prm;
    BatchLayout lay;
    uint32_t *words;
    uint8_t *ws;
    hipStream_t stream;
    int64_t t;
    uint32_t per_round;
    uint64_t merge_words;
    uint32_t total_rows, total_row_tasks;
    char err[256];
};

namespace {

kpz_status batch_fail(kpz_batch *b, hipError_t e, const char *what)
{
    if (b) snprintf(b->err, sizeof b->err, "%s: %s", what, hipGetErrorString(e));
    return KPZ_EHIP;
}

SweepArgs *batch_members(kpz_batch *b) { return (SweepArgs *)(b->ws + b->lay.off_members); }
long long *batch_res(kpz_batch *b) { return (long long *)(b->ws + b->lay.off_res); }

// sweep n_mcs on stream st (kernels only: capturable)
kpz_status batch_sweep_on(kpz_batch *b, int32_t n_mcs, hipStream_t st)
{
    if (n_mcs <= 0) return KPZ_OK;
    const uint32_t *bp = (const uint32_t *)(b->ws + b->lay.off_bprefix);
    const unsigned long long *sp = (const unsigned long long *)(b->ws + b->lay.off_sprefix);
    for (int32_t k = 0; k < n_mcs; ++k)
        for (uint32_t r = 0; r < b->lay.moves; ++r) {
            const hipError_t e = round_launch(b->per_round, b->merge_words, st,
                                              batch_members(b), bp, sp, (uint32_t)b->n,
                                              (uint32_t)k, r, !b->lay.db);
            if (e != hipSuccess) return batch_fail(b, e, "kpz_batch_sweep launch");
        }
    hipLaunchKernelGGL(kpz_batch_advance_kernel, dim3((b->n + 255) / 256), dim3(256), 0, st,
                       batch_members(b), (uint32_t)b->n, (uint32_t)n_mcs);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return batch_fail(b, e, "kpz_batch_sweep launch");
    return KPZ_OK;
}

kpz_status batch_moments_on(kpz_batch *b, uint32_t k, hipStream_t st)
{
    const MemberRows *mr = (const MemberRows *)(b->ws + b->lay.off_rows);
    if (16u * b->lay.maxW <= SMALL_ROWS) {
        hipLaunchKernelGGL(kpz_batch_moments_small_kernel, dim3(b->n), dim3(1024), 0, st, mr,
                           (uint32_t)b->n, (uint32_t)BATCH_SLOTS, batch_res(b), k);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return batch_fail(b, e, "kpz_batch moments launch");
        return KPZ_OK;
    }
    const uint32_t nt = b->total_row_tasks;
    const uint32_t rgrid = (nt + 3) / 4 < 8192 ? (nt + 3) / 4 : 8192;
    hipLaunchKernelGGL(kpz_batch_rows_kernel, dim3(rgrid), dim3(256), 0, st, mr,
                       (const uint32_t *)(b->ws + b->lay.off_tprefix), (uint32_t)b->n);
    hipLaunchKernelGGL(kpz_batch_finalize_kernel, dim3(b->n), dim3(256), 0, st, mr,
                       (uint32_t)b->n, (uint32_t)BATCH_SLOTS, batch_res(b), k);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return batch_fail(b, e, "kpz_batch moments launch");
    return KPZ_OK;
}

// Converts (R1, R2 lo, R2 hi, net) of member r into S1, S2, W2.
kpz_status convert_moments(const long long *res, int64_t L, int64_t *S1o, int64_t *S2o,
                           double *W2o, char *err, size_t errn)
{
    const __int128 N = (__int128)L * L;
    const __int128 R1 = res[0];
    const __int128 R2 = (__int128)(((unsigned __int128)(uint64_t)res[2] << 64) | (uint64_t)res[1]);
    const __int128 net = res[3];
    const __int128 S1 = N / 2 + 2 * net;
    const __int128 num = S1 - R1;
    if (num % N != 0) {
        snprintf(err, errn, "height anchor not integral: words and flip count disagree");
        return KPZ_ESTATE;
    }
    const __int128 ha = num / N;
    const __int128 S2 = R2 + 2 * ha * R1 + N * ha * ha;
    const __int128 wnum = N * R2 - R1 * R1;
    if (W2o) *W2o = (double)((long double)wnum / ((long double)N * (long double)N));
    const __int128 lim = (__int128)INT64_MAX;
    kpz_status st = KPZ_OK;
    if (S1 > lim || S1 < -lim - 1 || S2 > lim || S2 < 0) st = KPZ_ERANGE;
    if (S1o) *S1o = (int64_t)S1;
    if (S2o) *S2o = (int64_t)S2;
    return st;
}

}  // namespace


// ------------------------------------------------------------ job pool host

namespace {

struct PoolJob {
    int64_t id;
    kpz_params prm;
    int64_t t, n_mcs;
    size_t off, bytes;        // arena extent
    size_t off_words, off_slots, off_rowA, off_rowB, off_alt;
    // two-buffer state: the lattice is in buffer cur (0 = words, 1 = alt),
    // rotated as written by launch (rot_t, rot_res) when rot_valid
    uint32_t cur, rot_valid, rot_t, rot_res;
};

struct PoolResult {
    int64_t id, S1, S2;
    double W2;
    kpz_status st;
};

// a job: its lattice twice (two-buffer mode), flip counters, row moments
size_t pool_job_bytes_raw(int64_t L, uint32_t Bx, uint32_t By)
{
    (void)Bx;
    (void)By;
    return 2 * align256((size_t)L * L / 4) + align256(sizeof(long long) * BATCH_SLOTS) +
           2 * align256(8 * (size_t)L);
}

struct PoolCtl {
    size_t off_members, off_bprefix, off_sprefix, off_tprefix, off_rows, off_res, bytes;
};

PoolCtl pool_ctl_layout(int32_t max_jobs)
{
    PoolCtl c;
    size_t o = 0;
    c.off_members = o;  o = align256(o + sizeof(SweepArgs) * (size_t)max_jobs);
    c.off_bprefix = o;  o = align256(o + 4 * ((size_t)max_jobs + 1));
    c.off_sprefix = o;  o = align256(o + 8 * ((size_t)max_jobs + 1));
    c.off_tprefix = o;  o = align256(o + 4 * ((size_t)max_jobs + 1));
    c.off_rows = o;     o = align256(o + sizeof(MemberRows) * (size_t)max_jobs);
    c.off_res = o;      o = align256(o + 4 * sizeof(long long) * (size_t)max_jobs);
    c.bytes = o;
    return c;
}

}  // namespace

struct kpz_pool {
    uint8_t *arena;
    size_t arena_bytes;
    int32_t max_jobs, max_quantum;
    uint32_t Bx, By;                      // block shape of every job; 0: each job's default
    hipStream_t stream;
    PoolCtl ctl;
    std::map<size_t, size_t> free_list;   // offset -> bytes (heap part of the arena)
    std::vector<PoolJob> jobs;            // resident
    std::deque<PoolResult> done;
    int64_t next_id;
    char err[256];
};

namespace {

bool pool_alloc(kpz_pool *p, size_t bytes, size_t *off)
{
    for (auto it = p->free_list.begin(); it != p->free_list.end(); ++it) {
        if (it->second >= bytes) {
            *off = it->first;
            const size_t rest = it->second - bytes;
            const size_t roff = it->first + bytes;
            p->free_list.erase(it);
            if (rest) p->free_list[roff] = rest;
            return true;
        }
    }
    return false;
}

void pool_free(kpz_pool *p, size_t off, size_t bytes)
{
    auto it = p->free_list.emplace(off, bytes).first;
    // merge with the following and the preceding extents
    auto nx = std::next(it);
    if (nx != p->free_list.end() && it->first + it->second == nx->first) {
        it->second += nx->second;
        p->free_list.erase(nx);
    }
    if (it != p->free_list.begin()) {
        auto pv = std::prev(it);
        if (pv->first + pv->second == it->first) {
            pv->second += it->second;
            p->free_list.erase(it);
        }
    }
}

kpz_status pool_fail(kpz_pool *p, hipError_t e, const char *what)
{
    if (p) snprintf(p->err, sizeof p->err, "%s: %s", what, hipGetErrorString(e));
    return KPZ_EHIP;
}

SweepArgs pool_args(const kpz_pool *p, const PoolJob &j)
{
    SweepArgs a;
    const uint32_t L = (uint32_t)j.prm.L;
    a.words = (uint32_t *)(p->arena + j.off_words);
    a.src = a.words;
    a.db = 1;
    a.alt = (uint32_t *)(p->arena + j.off_alt);
    a.cur0 = j.cur;
    a.prev_valid = j.rot_valid;
    a.prev_t = j.rot_t;
    a.prev_res = j.rot_res;
    a.xcd = 0;
    a.side = nullptr;
    a.slots = (unsigned long long *)(p->arena + j.off_slots);
    set_shape(a, L, (uint32_t)j.prm.block_x, (uint32_t)j.prm.block_y);
    a.seed_lo = (uint32_t)j.prm.seed;
    a.seed_hi = (uint32_t)(j.prm.seed >> 32);
    a.t = (uint32_t)j.t;
    a.res = 0;
    a.nsteps = 16;
    a.slot_mask = BATCH_SLOTS - 1;
    a.P = threshold(j.prm.p);
    a.Q = threshold(j.prm.q);
    a.acc = !(a.P == (1ull << 32) && a.Q == 0);
    return a;
}

}  // namespace

namespace {

// A non-sticky error left pending on this thread by another library's HIP
// call (a query that returned "not ready", a failed allocation that was
// retried) would be reported by the hipGetLastError after our own launches;
// entry points that launch clear it first.  Errors of a faulted context are
// sticky and still surface.
void clear_pending_error() { (void)hipGetLastError(); }

// Text of the last failed kpz_init / kpz_batch_init / kpz_pool_init on this
// thread (those return no handle to hold it).
thread_local char g_init_err[256];

void set_init_error(hipError_t e, const char *what)
{
    snprintf(g_init_err, sizeof g_init_err, "%s: %s", what, hipGetErrorString(e));
}

}  // namespace

// ------------------------------------------------ no-allocation roughness
//
// Scratch of kpz_roughness_noalloc: the results header (WS_HEADER bytes),
// NSLOTS flip-counter slots (slot 0 = the caller's flip count, the rest 0)
// and two int64 row sums per row for L up to KPZ_NOALLOC_MAX_L.  One copy per
// device, held until the process ends.  In host code `scratch` names a
// host-side stand-in, never a device address: the address on each device
// comes from hipGetSymbolAddress, looked up once per device with that device
// current, and only that pointer is passed to kernels.
namespace {

constexpr size_t NOALLOC_SCRATCH_BYTES =
    WS_HEADER + sizeof(long long) * NSLOTS + 2 * sizeof(long long) * KPZ_NOALLOC_MAX_L;

__device__ __align__(256) uint8_t scratch[NOALLOC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[MAX_DEVICES];   // device address of `scratch` per device ordinal

// The current device's scratch address (looked up on the first call on it).
kpz_status scratch_on_current_device(void **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        set_init_error(e, "kpz_roughness_noalloc: hipGetDevice");
        return KPZ_EHIP;
    }
    if (dev < 0 || dev >= MAX_DEVICES) {
        snprintf(g_init_err, sizeof g_init_err, "kpz_roughness_noalloc: device %d out of range", dev);
        return KPZ_EINVAL;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            set_init_error(e, "kpz_roughness_noalloc: hipGetSymbolAddress(scratch)");
            return KPZ_EHIP;
        }
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return KPZ_OK;
}

}  // namespace

extern "C" {

kpz_status kpz_dt_order(uint64_t seed, uint32_t t, int32_t *perm)
{
    if (!perm) return KPZ_EINVAL;
    uint32_t o[4];
    dt_order_host(t, seed, o);
    for (int i = 0; i < 4; ++i) perm[i] = (int32_t)o[i];
    return KPZ_OK;
}

const char *kpz_status_str(kpz_status s)
{
    switch (s) {
    case KPZ_OK: return "ok";
    case KPZ_EINVAL: return "invalid argument";
    case KPZ_ESIZE: return "buffer too small";
    case KPZ_EHIP: return "HIP runtime error";
    case KPZ_ESTATE: return "inconsistent device state";
    case KPZ_ERANGE: return "result out of range";
    }
    return "unknown status";
}

const char *kpz_last_error(const kpz_sim *s) { return s ? s->err : g_init_err; }

kpz_status kpz_workspace_bytes(const kpz_params *p, size_t *bytes)
{
    uint32_t bx, by;
    const kpz_status st = resolve(p, &bx, &by);
    if (st != KPZ_OK) return st;
    if (!bytes) return KPZ_EINVAL;
    *bytes = ws_needed(p->L, bx, p->flags);
    return KPZ_OK;
}

kpz_status kpz_block_shape(const kpz_params *p, int32_t *block_x, int32_t *block_y)
{
    uint32_t bx, by;
    const kpz_status st = resolve(p, &bx, &by);
    if (st != KPZ_OK) return st;
    if (!block_x || !block_y) return KPZ_EINVAL;
    *block_x = (int32_t)bx;
    *block_y = (int32_t)by;
    return KPZ_OK;
}

kpz_status kpz_init(kpz_sim **out, const kpz_params *p, uint32_t *d_words, size_t words_bytes,
                    void *d_ws, size_t ws_bytes, void *stream)
{
    clear_pending_error();
    if (!out) return KPZ_EINVAL;
    *out = nullptr;
    uint32_t bx, by;
    kpz_status st = resolve(p, &bx, &by);
    if (st != KPZ_OK) return st;
    if (!d_words || !d_ws) return KPZ_EINVAL;
    const uint64_t L = (uint64_t)p->L;
    if (words_bytes < L * L / 4 || ws_bytes < ws_needed(p->L, bx, p->flags)) return KPZ_ESIZE;
    kpz_sim *s = new (std::nothrow) kpz_sim();
    if (!s) return KPZ_EINVAL;
    s->prm = *p;
    s->Bx = bx;
    s->By = by;
    s->words = d_words;
    s->words_bytes = words_bytes;
    s->ws = (uint8_t *)d_ws;
    s->ws_bytes = ws_bytes;
    s->stream = (hipStream_t)stream;
    s->t = 0;
    s->P = threshold(p->p);
    s->Q = threshold(p->q);
    s->db = !(p->flags & (KPZ_FLAG_IN_PLACE | KPZ_FLAG_DEVICE_DT));
    s->dt = (p->flags & KPZ_FLAG_DEVICE_DT) != 0;
    s->dt_ahead = (p->flags & KPZ_FLAG_DT_AHEAD) != 0;
    s->buf[0] = d_words;
    s->buf[1] = s->db ? ws_alt(s) : d_words;
    s->cur = 0;
    s->rot_valid = s->rot_t = s->rot_res = 0;
    s->err[0] = 0;
    const uint64_t nwords = L * L / 16;
    const uint32_t W = (uint32_t)(L / 16);
    if (W % 4 == 0) {
        const uint64_t n4 = nwords / 4;
        const uint32_t blocks = (uint32_t)((n4 + 255) / 256 < 65536 ? (n4 + 255) / 256 : 65536);
        hipLaunchKernelGGL(kpz_init_kernel, dim3(blocks), dim3(256), 0, s->stream,
                           (uint4 *)d_words, n4, W / 4);
    } else {
        hipLaunchKernelGGL(kpz_init_small_kernel, dim3(1), dim3(256), 0, s->stream, d_words,
                           (uint32_t)nwords, W);
    }
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) {
        hipLaunchKernelGGL(kpz_fill_counters_kernel, dim3(NSLOTS / 256), dim3(256), 0, s->stream,
                           ws_slots(s), 0LL);
        e = hipGetLastError();
    }
    if (e != hipSuccess) {
        set_init_error(e, "kpz_init launch");
        delete s;
        return KPZ_EHIP;
    }
    *out = s;
    return KPZ_OK;
}

kpz_status kpz_sweep(kpz_sim *s, int32_t n_mcs)
{
    clear_pending_error();
    if (!s || n_mcs < 0) return KPZ_EINVAL;
    if (n_mcs == 0) return KPZ_OK;
    if (s->t + n_mcs > 0xFFFFFFFFll) return KPZ_ERANGE;
    const uint32_t L = (uint32_t)s->prm.L;
    SweepArgs a;
    a.words = s->words;
    a.src = s->words;
    a.alt = nullptr;
    a.cur0 = 0;
    a.ahead = 0;
    a.db = 0;
    a.prev_valid = a.prev_t = a.prev_res = 0;
    a.side = ws_side(s);
    a.slots = (unsigned long long *)ws_slots(s);
    set_shape(a, L, s->Bx, s->By);
    a.seed_lo = (uint32_t)s->prm.seed;
    a.seed_hi = (uint32_t)(s->prm.seed >> 32);
    a.P = s->P;
    a.Q = s->Q;
    a.slot_mask = NSLOTS - 1;
    a.acc = !(s->P == (1ull << 32) && s->Q == 0);
    const uint32_t moves = moves_of(&s->prm);
    a.nsteps = 16u / moves;
    const uint32_t nblocks = a.nbx * a.nby;
    const uint64_t nstraddle = (uint64_t)L * a.nbx;
    const uint32_t mgrid = (uint32_t)((nstraddle + 255) / 256 < 8192 ? (nstraddle + 255) / 256 : 8192);
    a.xcd = 1;
    if (s->dt) {
        // double tiling at the device layer: four launches per MCS, one per
        // block set in the order drawn for the MCS, in place
        // (with dt_ahead, a set whose successor in the order is its diagonal
        // partner shares its launch with it: two to four launches per MCS)
        const uint32_t nset = nblocks / 4;
        a.res = 0;
        for (int32_t m = 0; m < n_mcs; ++m) {
            a.t = (uint32_t)(s->t + m);
            uint32_t perm[4];
            dt_order_host(a.t, s->prm.seed, perm);
            for (uint32_t ph = 0; ph < 4; ++ph) {
                a.ahead = (s->dt_ahead && ph + 1 < 4 && perm[ph + 1] == (perm[ph] ^ 3u)) ? 1u : 0u;
                const hipError_t e = a.acc ? launch_dt<true>(a, ph, nset, s->stream)
                                           : launch_dt<false>(a, ph, nset, s->stream);
                if (e != hipSuccess) return hip_fail(s, e, "kpz_sweep launch");
                ph += a.ahead;
            }
        }
        s->t += n_mcs;
        return KPZ_OK;
    }
    for (int32_t m = 0; m < n_mcs; ++m) {
        a.t = (uint32_t)(s->t + m);
        for (uint32_t r = 0; r < moves; ++r) {
            a.res = r;
            if (s->db) {
                // read buf[cur] (rotated as last written), write the other buffer
                a.db = 1;
                a.src = s->buf[s->cur];
                a.words = s->buf[s->cur ^ 1];
                a.prev_valid = s->rot_valid;
                a.prev_t = s->rot_t;
                a.prev_res = s->rot_res;
            }
            hipError_t e = a.acc ? launch_sweep<true>(a, nblocks, s->stream)
                                 : launch_sweep<false>(a, nblocks, s->stream);
            if (e != hipSuccess) return hip_fail(s, e, "kpz_sweep launch");
            if (s->db) {
                s->cur ^= 1;
                s->rot_valid = 1;
                s->rot_t = a.t;
                s->rot_res = r;
            } else {
                hipLaunchKernelGGL(kpz_merge_kernel, dim3(mgrid), dim3(256), 0, s->stream, a);
                e = hipGetLastError();
                if (e != hipSuccess) return hip_fail(s, e, "kpz_sweep merge launch");
            }
        }
    }
    s->t += n_mcs;
    return KPZ_OK;
}

kpz_status kpz_roughness(kpz_sim *s, int64_t *S1o, int64_t *S2o, double *W2o)
{
    clear_pending_error();
    if (!s) return KPZ_EINVAL;
    const uint32_t L = (uint32_t)s->prm.L, W = L / 16;
    hipError_t e = hipSuccess;
    if (L <= SMALL_ROWS) {
        hipLaunchKernelGGL(kpz_roughness_small_kernel, dim3(1), dim3(1024), 0, s->stream,
                           s->buf[s->cur], L, W, ws_slots(s), ws_res(s), sim_rot(s));
        e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(s, e, "kpz_roughness launch");
    } else {
        hipLaunchKernelGGL(kpz_row_moments_kernel, dim3(row_grid(row_tasks(L))),
                           dim3(64 * ROW_WAVES), 0, s->stream,
                           s->buf[s->cur], L, W, ws_rowA(s), ws_rowB(s));
        e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(s, e, "kpz_roughness launch");
        hipLaunchKernelGGL(kpz_finalize_kernel, dim3(1), dim3(1024), 0, s->stream, L, ws_rowA(s),
                           ws_rowB(s), ws_slots(s), ws_res(s), s->buf[s->cur], sim_rot(s));
        e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(s, e, "kpz_roughness launch");
    }
    long long res[4];
    e = hipMemcpyAsync(res, ws_res(s), sizeof res, hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return hip_fail(s, e, "kpz_roughness copy");
    const __int128 N = (__int128)L * L;
    const __int128 R1 = res[0];
    const __int128 R2 = (__int128)(((unsigned __int128)(uint64_t)res[2] << 64) | (uint64_t)res[1]);
    const __int128 net = res[3];
    // absolute heights: S1 = N/2 + 2 net; h(0,0) = (S1 - R1) / N
    const __int128 S1 = N / 2 + 2 * net;
    const __int128 num = S1 - R1;
    if (num % N != 0) {
        snprintf(s->err, sizeof s->err, "height anchor not integral: words and flip count disagree");
        return KPZ_ESTATE;
    }
    const __int128 ha = num / N;
    const __int128 S2 = R2 + 2 * ha * R1 + N * ha * ha;
    const __int128 wnum = N * R2 - R1 * R1;   // = N^2 W^2
    if (W2o) *W2o = (double)((long double)wnum / ((long double)N * (long double)N));
    const __int128 lim = (__int128)INT64_MAX;
    kpz_status st = KPZ_OK;
    if (S1 > lim || S1 < -lim - 1 || S2 > lim || S2 < 0) st = KPZ_ERANGE;
    if (S1o) *S1o = (int64_t)S1;
    if (S2o) *S2o = (int64_t)S2;
    return st;
}

kpz_status kpz_height_moments(kpz_sim *s, int64_t sums[8], double *W2, double *skewness,
                              double *kurtosis)
{
    clear_pending_error();
    if (!s) return KPZ_EINVAL;
    const kpz_status sst = kpz_sync_words(s);
    if (sst != KPZ_OK) return sst;
    const uint32_t L = (uint32_t)s->prm.L, W = L / 16;
    long long *rows6 = ws_rowA(s);   // 6 int64 per row
    const uint32_t rgrid = (L + 3) / 4 < 4096 ? (L + 3) / 4 : 4096;
    hipLaunchKernelGGL(kpz_row_mom4_kernel, dim3(rgrid), dim3(256), 0, s->stream, s->words, L, W,
                       rows6);
    hipLaunchKernelGGL(kpz_mom4_finalize_kernel, dim3(1), dim3(256), 0, s->stream, s->words, L, W,
                       (const long long *)rows6, ws_res(s) + 4);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(s, e, "kpz_height_moments launch");
    long long res[8];
    e = hipMemcpyAsync(res, ws_res(s) + 4, sizeof res, hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return hip_fail(s, e, "kpz_height_moments copy");
    if (sums)
        for (int k = 0; k < 8; ++k) sums[k] = res[k];
    __int128 M[4];
    for (int k = 0; k < 4; ++k)
        M[k] = (__int128)(((unsigned __int128)(uint64_t)res[2 * k + 1] << 64) | (uint64_t)res[2 * k]);
    // central moments (shift invariant) in extended precision
    const long double N = (long double)L * (long double)L;
    const long double mu = (long double)M[0] / N;
    const long double e2 = (long double)M[1] / N, e3 = (long double)M[2] / N,
                      e4 = (long double)M[3] / N;
    const long double m2 = e2 - mu * mu;
    const long double m3 = e3 - 3 * mu * e2 + 2 * mu * mu * mu;
    const long double m4 = e4 - 4 * mu * e3 + 6 * mu * mu * e2 - 3 * mu * mu * mu * mu;
    if (W2) *W2 = (double)m2;
    if (skewness) *skewness = m2 > 0 ? (double)(m3 / powl(m2, 1.5L)) : 0.0;
    if (kurtosis) *kurtosis = m2 > 0 ? (double)(m4 / (m2 * m2) - 3) : 0.0;
    return KPZ_OK;
}

// Header slots of the invariant counters (after the moments of
// kpz_roughness and kpz_height_moments).
constexpr int RES_CHECK = 16;
constexpr uint32_t CHECK_ROWS = 64;   // rows a thread walks

kpz_status kpz_check_invariants(kpz_sim *s, int64_t counts[3])
{
    clear_pending_error();
    if (!s || !counts) return KPZ_EINVAL;
    const kpz_status sst = kpz_sync_words(s);
    if (sst != KPZ_OK) return sst;
    const uint32_t L = (uint32_t)s->prm.L, W = L / 16;
    unsigned long long *d = (unsigned long long *)(ws_res(s) + RES_CHECK);
    hipLaunchKernelGGL(kpz_zero_kernel, dim3(1), dim3(64), 0, s->stream, (uint32_t *)d,
                       (uint64_t)6);
    const uint32_t R = L < CHECK_ROWS ? L : CHECK_ROWS;
    const uint64_t chunks = (L + R - 1) / R;
    if ((W & 3u) == 0) {
        const uint64_t th = (uint64_t)(W / 4) * chunks;
        hipLaunchKernelGGL(kpz_check_kernel<4>, dim3((uint32_t)((th + 255) / 256)), dim3(256), 0,
                           s->stream, s->words, L, W, R, d);
    } else {
        const uint64_t th = (uint64_t)W * chunks;
        hipLaunchKernelGGL(kpz_check_kernel<1>, dim3((uint32_t)((th + 255) / 256)), dim3(256), 0,
                           s->stream, s->words, L, W, R, d);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(s, e, "kpz_check_invariants launch");
    unsigned long long v[3];
    e = hipMemcpyAsync(v, d, sizeof v, hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return hip_fail(s, e, "kpz_check_invariants copy");
    counts[0] = (int64_t)v[0];
    counts[1] = 2 * (int64_t)v[1] - (int64_t)L;
    counts[2] = 2 * (int64_t)v[2] - (int64_t)L;
    if (counts[0] || counts[1] || counts[2]) {
        snprintf(s->err, sizeof s->err,
                 "invalid surface: %lld open plaquettes, row-0 slope sum %lld, column-0 slope sum "
                 "%lld", (long long)counts[0], (long long)counts[1], (long long)counts[2]);
        return KPZ_ESTATE;
    }
    return KPZ_OK;
}

kpz_status kpz_get_state(kpz_sim *s, int64_t *t, int64_t *net)
{
    if (!s) return KPZ_EINVAL;
    if (t) *t = s->t;
    if (net) {
        long long slots[NSLOTS];
        hipError_t e = hipMemcpyAsync(slots, ws_slots(s), sizeof slots, hipMemcpyDeviceToHost,
                                      s->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
        if (e != hipSuccess) return hip_fail(s, e, "kpz_get_state copy");
        long long n = 0;
        for (int i = 0; i < NSLOTS; ++i) n += slots[i];
        *net = n;
    }
    return KPZ_OK;
}

kpz_status kpz_set_state(kpz_sim *s, int64_t t, int64_t net)
{
    if (!s || t < 0 || t > 0xFFFFFFFFll) return KPZ_EINVAL;
    hipLaunchKernelGGL(kpz_fill_counters_kernel, dim3(NSLOTS / 256), dim3(256), 0, s->stream,
                       ws_slots(s), (long long)net);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(s, e, "kpz_set_state launch");
    s->t = t;
    // `words` holds the state in the documented layout from here on
    s->cur = 0;
    s->rot_valid = 0;
    return KPZ_OK;
}

kpz_status kpz_sync_words(kpz_sim *s)
{
    clear_pending_error();
    if (!s) return KPZ_EINVAL;
    if (!s->db || (s->cur == 0 && !s->rot_valid)) return KPZ_OK;
    const uint32_t L = (uint32_t)s->prm.L, W = L / 16;
    const uint64_t n = (uint64_t)L * W;
    const uint32_t grid = (uint32_t)((n + 255) / 256 < 65536 ? (n + 255) / 256 : 65536);
    if (s->cur == 1) {
        // the other buffer -> words, undoing the rotation on the way
        hipLaunchKernelGGL(kpz_rotate_kernel, dim3(grid), dim3(256), 0, s->stream, s->buf[1],
                           s->buf[0], L, W, sim_rot(s));
    } else {
        // words is rotated: through the other buffer and back
        hipLaunchKernelGGL(kpz_rotate_kernel, dim3(grid), dim3(256), 0, s->stream, s->buf[0],
                           s->buf[1], L, W, sim_rot(s));
        hipLaunchKernelGGL(kpz_rotate_kernel, dim3(grid), dim3(256), 0, s->stream, s->buf[1],
                           s->buf[0], L, W, Rot{0u, 0u, 0u, s->Bx, 0u, 0u});
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(s, e, "kpz_sync_words launch");
    s->cur = 0;
    s->rot_valid = 0;
    return KPZ_OK;
}

void kpz_destroy(kpz_sim *s) { delete s; }


kpz_status kpz_batch_sizes(const kpz_params *members, int32_t n, size_t *words_bytes,
                           size_t *ws_bytes)
{
    BatchLayout lay;
    const kpz_status st = batch_layout(members, n, &lay);
    if (st != KPZ_OK) return st;
    if (words_bytes) *words_bytes = lay.words_bytes;
    if (ws_bytes) *ws_bytes = lay.ws_bytes;
    return KPZ_OK;
}

kpz_status kpz_batch_init(kpz_batch **out, const kpz_params *members, int32_t n, uint32_t *d_words,
                          size_t words_bytes, void *d_ws, size_t ws_bytes, void *stream)
{
    clear_pending_error();
    if (!out) return KPZ_EINVAL;
    *out = nullptr;
    BatchLayout lay;
    kpz_status st = batch_layout(members, n, &lay);
    if (st != KPZ_OK) return st;
    if (!d_words || !d_ws) return KPZ_EINVAL;
    if (words_bytes < lay.words_bytes || ws_bytes < lay.ws_bytes) return KPZ_ESIZE;
    kpz_batch *b = new (std::nothrow) kpz_batch();
    if (!b) return KPZ_EINVAL;
    b->n = n;
    b->prm.assign(members, members + n);
    b->lay = lay;
    b->words = d_words;
    b->ws = (uint8_t *)d_ws;
    b->stream = (hipStream_t)stream;
    b->t = 0;
    b->err[0] = 0;

    std::vector<SweepArgs> args(n);
    std::vector<MemberRows> rows(n);
    std::vector<uint32_t> bprefix(n + 1, 0), rprefix(n + 1, 0), tprefix(n + 1, 0);
    std::vector<unsigned long long> sprefix(n + 1, 0);
    long long *slots = (long long *)(b->ws + lay.off_slots);
    for (int32_t r = 0; r < n; ++r) {
        const kpz_params &p = members[r];
        const uint32_t L = (uint32_t)p.L;
        SweepArgs &a = args[r];
        a.words = d_words + lay.word_off[r];
        a.src = a.words;
        a.db = lay.db ? 1u : 0u;
        a.prev_valid = a.prev_t = a.prev_res = a.xcd = 0;
        a.alt = lay.db ? (uint32_t *)(b->ws + lay.off_alt[r]) : nullptr;
        a.cur0 = 0;
        a.side = (uint32_t *)(b->ws + lay.off_side[r]);
        a.slots = (unsigned long long *)(slots + (size_t)BATCH_SLOTS * r);
        set_shape(a, L, lay.Bx[r], lay.By[r]);
        a.seed_lo = (uint32_t)p.seed;
        a.seed_hi = (uint32_t)(p.seed >> 32);
        a.t = 0;
        a.res = 0;
        a.nsteps = 16u / lay.moves;
        a.slot_mask = BATCH_SLOTS - 1;
        a.P = threshold(p.p);
        a.Q = threshold(p.q);
        a.acc = !(a.P == (1ull << 32) && a.Q == 0);
        rows[r].words = a.words;
        rows[r].rowA = (long long *)(b->ws + lay.off_rowA[r]);
        rows[r].rowB = (long long *)(b->ws + lay.off_rowB[r]);
        rows[r].slots = slots + (size_t)BATCH_SLOTS * r;
        rows[r].L = L;
        rows[r].W = L / 16;
        rows[r].state = (const SweepArgs *)(b->ws + lay.off_members) + r;
        rows[r].rot = Rot{0u, 0u, 0u, lay.Bx[r], 0u, 0u};
        bprefix[r + 1] = bprefix[r] + a.nbx * a.nby;
        sprefix[r + 1] = sprefix[r] + (unsigned long long)L * a.nbx;
        rprefix[r + 1] = rprefix[r] + L;
        tprefix[r + 1] = tprefix[r] + row_tasks(L);
    }
    b->per_round = bprefix[n];
    b->merge_words = sprefix[n];
    b->total_rows = rprefix[n];
    b->total_row_tasks = tprefix[n];
    hipError_t e = hipSuccess;
    auto h2d = [&](size_t off, const void *src, size_t bytes) {
        if (e == hipSuccess)
            e = hipMemcpyAsync(b->ws + off, src, bytes, hipMemcpyHostToDevice, b->stream);
    };
    h2d(lay.off_members, args.data(), sizeof(SweepArgs) * n);
    h2d(lay.off_bprefix, bprefix.data(), 4 * (n + 1));
    h2d(lay.off_sprefix, sprefix.data(), 8 * (n + 1));
    h2d(lay.off_rprefix, rprefix.data(), 4 * (n + 1));
    h2d(lay.off_tprefix, tprefix.data(), 4 * (n + 1));
    h2d(lay.off_rows, rows.data(), sizeof(MemberRows) * n);
    for (int32_t r = 0; r < n && e == hipSuccess; ++r) {
        const uint64_t L = (uint64_t)members[r].L;
        const uint32_t W = (uint32_t)(L / 16);
        if (W % 4 == 0) {
            const uint64_t n4 = L * L / 64;
            const uint32_t blocks = (uint32_t)((n4 + 255) / 256 < 65536 ? (n4 + 255) / 256 : 65536);
            hipLaunchKernelGGL(kpz_init_kernel, dim3(blocks), dim3(256), 0, b->stream,
                               (uint4 *)(d_words + lay.word_off[r]), n4, W / 4);
        } else {
            hipLaunchKernelGGL(kpz_init_small_kernel, dim3(1), dim3(256), 0, b->stream,
                               d_words + lay.word_off[r], (uint32_t)(L * L / 16), W);
        }
        e = hipGetLastError();
    }
    if (e == hipSuccess) {
        const uint32_t ns = (uint32_t)BATCH_SLOTS * (uint32_t)n;
        hipLaunchKernelGGL(kpz_zero_kernel, dim3((2 * ns + 255) / 256), dim3(256), 0, b->stream,
                           (uint32_t *)slots, (uint64_t)2 * ns);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) {
        set_init_error(e, "kpz_batch_init");
        delete b;
        return KPZ_EHIP;
    }
    *out = b;
    return KPZ_OK;
}

kpz_status kpz_batch_word_offset(const kpz_batch *b, int32_t r, size_t *off)
{
    if (!b || !off || r < 0 || r >= b->n) return KPZ_EINVAL;
    *off = b->lay.word_off[r];
    return KPZ_OK;
}

kpz_status kpz_batch_sync_words(kpz_batch *b)
{
    clear_pending_error();
    if (!b) return KPZ_EINVAL;
    if (!b->lay.db) return KPZ_OK;
    const uint32_t grid = b->total_rows < 8192 ? b->total_rows : 8192;
    hipLaunchKernelGGL(kpz_batch_sync_kernel, dim3(grid), dim3(256), sizeof(uint32_t) * b->lay.maxW,
                       b->stream, (const MemberRows *)(b->ws + b->lay.off_rows),
                       (const uint32_t *)(b->ws + b->lay.off_rprefix), (uint32_t)b->n);
    hipLaunchKernelGGL(kpz_batch_settle_kernel, dim3((b->n + 255) / 256), dim3(256), 0, b->stream,
                       batch_members(b), (uint32_t)b->n);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return batch_fail(b, e, "kpz_batch_sync_words launch");
    return KPZ_OK;
}

kpz_status kpz_batch_sweep(kpz_batch *b, int32_t n_mcs)
{
    clear_pending_error();
    if (!b || n_mcs < 0) return KPZ_EINVAL;
    if (b->t + n_mcs > 0xFFFFFFFFll) return KPZ_ERANGE;
    const kpz_status st = batch_sweep_on(b, n_mcs, b->stream);
    if (st == KPZ_OK) b->t += n_mcs;
    return st;
}

kpz_status kpz_batch_roughness(kpz_batch *b, int64_t *S1, int64_t *S2, double *W2)
{
    clear_pending_error();
    if (!b) return KPZ_EINVAL;
    kpz_status st = batch_moments_on(b, 0, b->stream);
    if (st != KPZ_OK) return st;
    std::vector<long long> res(4 * (size_t)b->n);
    hipError_t e = hipMemcpyAsync(res.data(), batch_res(b), res.size() * sizeof(long long),
                                  hipMemcpyDeviceToHost, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return batch_fail(b, e, "kpz_batch_roughness copy");
    kpz_status worst = KPZ_OK;
    for (int32_t r = 0; r < b->n; ++r) {
        const kpz_status s = convert_moments(&res[4 * (size_t)r], b->prm[r].L, S1 ? S1 + r : nullptr,
                                             S2 ? S2 + r : nullptr, W2 ? W2 + r : nullptr, b->err,
                                             sizeof b->err);
        if (s != KPZ_OK && worst == KPZ_OK) worst = s;
    }
    return worst;
}

kpz_status kpz_batch_run(kpz_batch *b, const int32_t *times, int32_t n_times, int64_t *S1,
                         int64_t *S2, double *W2)
{
    clear_pending_error();
    if (!b || !times || n_times < 1 || n_times > KPZ_BATCH_MAX_SAMPLES) return KPZ_EINVAL;
    int64_t prev = b->t;
    for (int32_t k = 0; k < n_times; ++k) {
        if (times[k] <= prev) return KPZ_EINVAL;
        prev = times[k];
    }
    if (prev > 0xFFFFFFFFll) return KPZ_ERANGE;
    // capture the schedule on a private stream, ordered after the caller's stream
    hipStream_t cs = nullptr;
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ev_in, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ev_out, hipEventDisableTiming);
    kpz_status st = KPZ_OK;
    if (e == hipSuccess) e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        int64_t t = b->t;
        for (int32_t k = 0; k < n_times && st == KPZ_OK; ++k) {
            st = batch_sweep_on(b, (int32_t)(times[k] - t), cs);
            t = times[k];
            if (st == KPZ_OK) st = batch_moments_on(b, (uint32_t)k, cs);
        }
        const hipError_t e2 = hipStreamEndCapture(cs, &graph);
        if (e == hipSuccess) e = e2;
    }
    if (e == hipSuccess && st == KPZ_OK) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (e == hipSuccess && st == KPZ_OK) e = hipEventRecord(ev_in, b->stream);
    if (e == hipSuccess && st == KPZ_OK) e = hipStreamWaitEvent(cs, ev_in, 0);
    if (e == hipSuccess && st == KPZ_OK) e = hipGraphLaunch(exec, cs);
    if (e == hipSuccess && st == KPZ_OK) e = hipEventRecord(ev_out, cs);
    if (e == hipSuccess && st == KPZ_OK) e = hipStreamWaitEvent(b->stream, ev_out, 0);
    std::vector<long long> res(4 * (size_t)b->n * n_times);
    if (e == hipSuccess && st == KPZ_OK)
        e = hipMemcpyAsync(res.data(), batch_res(b), res.size() * sizeof(long long),
                           hipMemcpyDeviceToHost, b->stream);
    if (e == hipSuccess && st == KPZ_OK) e = hipStreamSynchronize(b->stream);
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (ev_in) (void)hipEventDestroy(ev_in);
    if (ev_out) (void)hipEventDestroy(ev_out);
    if (cs) (void)hipStreamDestroy(cs);
    if (st != KPZ_OK) return st;
    if (e != hipSuccess) return batch_fail(b, e, "kpz_batch_run");
    b->t = times[n_times - 1];
    kpz_status worst = KPZ_OK;
    for (int32_t k = 0; k < n_times; ++k)
        for (int32_t r = 0; r < b->n; ++r) {
            const size_t i = (size_t)k * b->n + r;
            const kpz_status s = convert_moments(&res[4 * i], b->prm[r].L, S1 ? S1 + i : nullptr,
                                                 S2 ? S2 + i : nullptr, W2 ? W2 + i : nullptr,
                                                 b->err, sizeof b->err);
            if (s != KPZ_OK && worst == KPZ_OK) worst = s;
        }
    return worst;
}

kpz_status kpz_batch_get_t(const kpz_batch *b, int64_t *t)
{
    if (!b || !t) return KPZ_EINVAL;
    *t = b->t;
    return KPZ_OK;
}

void kpz_batch_destroy(kpz_batch *b) { delete b; }

const char *kpz_batch_last_error(const kpz_batch *b) { return b ? b->err : g_init_err; }


kpz_status kpz_pool_job_bytes(const kpz_params *job, int32_t bx, int32_t by, size_t *bytes)
{
    if (!job || !bytes) return KPZ_EINVAL;
    kpz_params q = *job;
    q.block_x = bx;
    q.block_y = by;
    uint32_t rbx, rby;
    const kpz_status st = resolve(&q, &rbx, &rby);
    if (st != KPZ_OK) return st;
    *bytes = pool_job_bytes_raw(job->L, rbx, rby);
    return KPZ_OK;
}

kpz_status kpz_pool_control_bytes(int32_t max_jobs, size_t *bytes)
{
    if (max_jobs < 1 || !bytes) return KPZ_EINVAL;
    *bytes = pool_ctl_layout(max_jobs).bytes;
    return KPZ_OK;
}

kpz_status kpz_pool_init(kpz_pool **out, void *d_arena, size_t arena_bytes, int32_t max_jobs,
                         int32_t max_quantum, int32_t bx, int32_t by, void *stream)
{
    if (!out) return KPZ_EINVAL;
    *out = nullptr;
    if (!d_arena || ((uintptr_t)d_arena & 255) || max_jobs < 1 || max_quantum < 1) return KPZ_EINVAL;
    if ((bx == 0) != (by == 0)) return KPZ_EINVAL;
    if (bx) {
        // the shape rules of resolve() for a lattice the block fits
        kpz_params t = {};
        t.L = bx * by;   // a multiple of both sides and of 16
        t.p = 1.0;
        t.block_x = bx;
        t.block_y = by;
        uint32_t rbx, rby;
        if (resolve(&t, &rbx, &rby) != KPZ_OK) return KPZ_EINVAL;
    }
    const PoolCtl ctl = pool_ctl_layout(max_jobs);
    if (arena_bytes < ctl.bytes) return KPZ_ESIZE;
    kpz_pool *p = new (std::nothrow) kpz_pool();
    if (!p) return KPZ_EINVAL;
    p->arena = (uint8_t *)d_arena;
    p->arena_bytes = arena_bytes;
    p->max_jobs = max_jobs;
    p->max_quantum = max_quantum;
    p->Bx = (uint32_t)bx;
    p->By = (uint32_t)by;
    p->stream = (hipStream_t)stream;
    p->ctl = ctl;
    p->next_id = 0;
    p->err[0] = 0;
    if (arena_bytes > ctl.bytes) p->free_list[ctl.bytes] = arena_bytes - ctl.bytes;
    *out = p;
    return KPZ_OK;
}

kpz_status kpz_pool_submit(kpz_pool *p, const kpz_params *job, int64_t n_mcs, int64_t *id)
{
    clear_pending_error();
    if (!p || !job || n_mcs < 1 || n_mcs > 0xFFFFFFFFll) return KPZ_EINVAL;
    kpz_params q = *job;
    if (p->Bx) {
        if ((job->block_x && job->block_x != (int32_t)p->Bx) ||
            (job->block_y && job->block_y != (int32_t)p->By))
            return KPZ_EINVAL;
        q.block_x = (int32_t)p->Bx;
        q.block_y = (int32_t)p->By;
    }
    if (moves_of(job) != 1) return KPZ_EINVAL;
    uint32_t rbx, rby;
    kpz_status st = resolve(&q, &rbx, &rby);
    if (st != KPZ_OK) return st;
    q.block_x = (int32_t)rbx;
    q.block_y = (int32_t)rby;
    const size_t bytes = pool_job_bytes_raw(q.L, rbx, rby);
    if (bytes > p->arena_bytes - p->ctl.bytes) return KPZ_EINVAL;
    if ((int32_t)p->jobs.size() >= p->max_jobs) return KPZ_ESIZE;
    size_t off;
    if (!pool_alloc(p, bytes, &off)) return KPZ_ESIZE;
    PoolJob j;
    j.id = p->next_id++;
    j.prm = q;
    j.t = 0;
    j.n_mcs = n_mcs;
    j.off = off;
    j.bytes = bytes;
    const size_t L = (size_t)q.L;
    size_t o = off;
    j.off_words = o; o += align256(L * L / 4);
    j.off_slots = o; o += align256(sizeof(long long) * BATCH_SLOTS);
    j.off_rowA = o;  o += align256(8 * L);
    j.off_rowB = o;  o += align256(8 * L);
    j.off_alt = o;
    j.cur = j.rot_valid = j.rot_t = j.rot_res = 0;
    const uint32_t W = (uint32_t)(L / 16);
    uint32_t *words = (uint32_t *)(p->arena + j.off_words);
    if (W % 4 == 0) {
        const uint64_t n4 = (uint64_t)L * L / 64;
        const uint32_t blocks = (uint32_t)((n4 + 255) / 256 < 65536 ? (n4 + 255) / 256 : 65536);
        hipLaunchKernelGGL(kpz_init_kernel, dim3(blocks), dim3(256), 0, p->stream, (uint4 *)words, n4,
                           W / 4);
    } else {
        hipLaunchKernelGGL(kpz_init_small_kernel, dim3(1), dim3(256), 0, p->stream, words,
                           (uint32_t)(L * L / 16), W);
    }
    hipLaunchKernelGGL(kpz_zero_kernel, dim3(1), dim3(256), 0, p->stream,
                       (uint32_t *)(p->arena + j.off_slots), (uint64_t)2 * BATCH_SLOTS);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        pool_free(p, off, bytes);
        return pool_fail(p, e, "kpz_pool_submit launch");
    }
    p->jobs.push_back(j);
    if (id) *id = j.id;
    return KPZ_OK;
}

kpz_status kpz_pool_step(kpz_pool *p, int32_t quantum, int32_t *n_active)
{
    clear_pending_error();
    if (!p || quantum < 1 || quantum > p->max_quantum) return KPZ_EINVAL;
    const size_t n = p->jobs.size();
    if (n == 0) {
        if (n_active) *n_active = 0;
        return KPZ_OK;
    }
    // members sorted by decreasing rounds this step
    std::vector<size_t> order(n);
    for (size_t i = 0; i < n; ++i) order[i] = i;
    auto rounds_of = [&](size_t i) {
        const int64_t rem = p->jobs[i].n_mcs - p->jobs[i].t;
        return (uint32_t)(rem < quantum ? rem : quantum);
    };
    std::stable_sort(order.begin(), order.end(),
                     [&](size_t a, size_t b) { return rounds_of(a) > rounds_of(b); });
    std::vector<SweepArgs> args(n);
    std::vector<uint32_t> bprefix(n + 1, 0), rounds(n);
    std::vector<unsigned long long> sprefix(n + 1, 0);
    for (size_t k = 0; k < n; ++k) {
        const PoolJob &j = p->jobs[order[k]];
        args[k] = pool_args(p, j);
        rounds[k] = rounds_of(order[k]);
        bprefix[k + 1] = bprefix[k] + args[k].nbx * args[k].nby;
        sprefix[k + 1] = sprefix[k] + (unsigned long long)args[k].L * args[k].nbx;
    }
    hipError_t e = hipSuccess;
    auto h2d = [&](size_t off, const void *src, size_t bytes) {
        if (e == hipSuccess)
            e = hipMemcpyAsync(p->arena + off, src, bytes, hipMemcpyHostToDevice, p->stream);
    };
    h2d(p->ctl.off_members, args.data(), sizeof(SweepArgs) * n);
    h2d(p->ctl.off_bprefix, bprefix.data(), 4 * (n + 1));
    h2d(p->ctl.off_sprefix, sprefix.data(), 8 * (n + 1));
    if (e != hipSuccess) return pool_fail(p, e, "kpz_pool_step copy");
    // round k runs the members with more than k rounds this step: a prefix
    // [0, m) of the sorted table, so its grid is bprefix[m]
    const SweepArgs *d_members = (const SweepArgs *)(p->arena + p->ctl.off_members);
    const uint32_t *d_bprefix = (const uint32_t *)(p->arena + p->ctl.off_bprefix);
    const unsigned long long *d_sprefix = (const unsigned long long *)(p->arena + p->ctl.off_sprefix);
    size_t m = n;
    for (uint32_t k = 0; k < rounds[0]; ++k) {
        while (m > 0 && rounds[m - 1] <= k) --m;
        e = round_launch(bprefix[m], sprefix[m], p->stream, d_members, d_bprefix, d_sprefix,
                         (uint32_t)m, k, 0u, false);
        if (e != hipSuccess) return pool_fail(p, e, "kpz_pool_step launch");
    }
    for (size_t k = 0; k < n; ++k) {
        PoolJob &j = p->jobs[order[k]];
        // two-buffer state after rounds[k] launches
        j.cur ^= rounds[k] & 1u;
        j.rot_valid = 1;
        j.rot_t = (uint32_t)(j.t + rounds[k] - 1);
        j.rot_res = 0;
        j.t += rounds[k];
    }
    // sample and release the jobs that reached their n_mcs
    std::vector<size_t> fin;
    for (size_t i = 0; i < n; ++i)
        if (p->jobs[i].t >= p->jobs[i].n_mcs) fin.push_back(i);
    if (!fin.empty()) {
        std::vector<MemberRows> rows(fin.size());
        std::vector<uint32_t> tprefix(fin.size() + 1, 0);
        for (size_t f = 0; f < fin.size(); ++f) {
            const PoolJob &j = p->jobs[fin[f]];
            rows[f].words = (const uint32_t *)(p->arena + (j.cur ? j.off_alt : j.off_words));
            rows[f].state = nullptr;
            rows[f].rot = Rot{j.rot_valid, j.rot_t, j.rot_res, (uint32_t)j.prm.block_x, (uint32_t)j.prm.seed,
                              (uint32_t)(j.prm.seed >> 32)};
            rows[f].rowA = (long long *)(p->arena + j.off_rowA);
            rows[f].rowB = (long long *)(p->arena + j.off_rowB);
            rows[f].slots = (const long long *)(p->arena + j.off_slots);
            rows[f].L = (uint32_t)j.prm.L;
            rows[f].W = (uint32_t)(j.prm.L / 16);
            tprefix[f + 1] = tprefix[f] + row_tasks((uint32_t)j.prm.L);
        }
        h2d(p->ctl.off_rows, rows.data(), sizeof(MemberRows) * fin.size());
        h2d(p->ctl.off_tprefix, tprefix.data(), 4 * (fin.size() + 1));
        if (e != hipSuccess) return pool_fail(p, e, "kpz_pool_step copy");
        const uint32_t nt = tprefix[fin.size()];
        const uint32_t rgrid = (nt + 3) / 4 < 8192 ? (nt + 3) / 4 : 8192;
        const MemberRows *mr = (const MemberRows *)(p->arena + p->ctl.off_rows);
        hipLaunchKernelGGL(kpz_batch_rows_kernel, dim3(rgrid), dim3(256), 0, p->stream, mr,
                           (const uint32_t *)(p->arena + p->ctl.off_tprefix), (uint32_t)fin.size());
        hipLaunchKernelGGL(kpz_batch_finalize_kernel, dim3((uint32_t)fin.size()), dim3(256), 0,
                           p->stream, mr, (uint32_t)fin.size(), (uint32_t)BATCH_SLOTS,
                           (long long *)(p->arena + p->ctl.off_res), 0u);
        e = hipGetLastError();
        std::vector<long long> res(4 * fin.size());
        if (e == hipSuccess)
            e = hipMemcpyAsync(res.data(), p->arena + p->ctl.off_res, res.size() * sizeof(long long),
                               hipMemcpyDeviceToHost, p->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
        if (e != hipSuccess) return pool_fail(p, e, "kpz_pool_step sample");
        for (size_t f = 0; f < fin.size(); ++f) {
            const PoolJob &j = p->jobs[fin[f]];
            PoolResult r;
            r.id = j.id;
            r.st = convert_moments(&res[4 * f], j.prm.L, &r.S1, &r.S2, &r.W2, p->err, sizeof p->err);
            p->done.push_back(r);
            pool_free(p, j.off, j.bytes);
        }
        std::vector<PoolJob> keep;
        keep.reserve(n - fin.size());
        size_t f = 0;
        for (size_t i = 0; i < n; ++i) {
            if (f < fin.size() && fin[f] == i) { ++f; continue; }
            keep.push_back(p->jobs[i]);
        }
        p->jobs.swap(keep);
    }
    if (n_active) *n_active = (int32_t)p->jobs.size();
    return KPZ_OK;
}

kpz_status kpz_pool_poll(kpz_pool *p, int32_t max_results, int64_t *ids, int64_t *S1, int64_t *S2,
                         double *W2, int32_t *status, int32_t *n_results)
{
    if (!p || max_results < 0) return KPZ_EINVAL;
    int32_t k = 0;
    while (k < max_results && !p->done.empty()) {
        const PoolResult &r = p->done.front();
        if (ids) ids[k] = r.id;
        if (S1) S1[k] = r.S1;
        if (S2) S2[k] = r.S2;
        if (W2) W2[k] = r.W2;
        if (status) status[k] = (int32_t)r.st;
        p->done.pop_front();
        ++k;
    }
    if (n_results) *n_results = k;
    return KPZ_OK;
}

kpz_status kpz_pool_stats(const kpz_pool *p, int32_t *n_active, size_t *largest_free)
{
    if (!p) return KPZ_EINVAL;
    if (n_active) *n_active = (int32_t)p->jobs.size();
    if (largest_free) {
        size_t m = 0;
        for (const auto &kv : p->free_list) m = kv.second > m ? kv.second : m;
        *largest_free = m;
    }
    return KPZ_OK;
}

void kpz_pool_destroy(kpz_pool *p) { delete p; }

const char *kpz_pool_last_error(const kpz_pool *p) { return p ? p->err : g_init_err; }

kpz_status kpz_valu_probe(uint32_t *d_out, int32_t n_groups, int32_t iters,
                          int32_t *ops_per_iter, void *stream)
{
    clear_pending_error();
    if (!d_out || n_groups < 1 || iters < 1) return KPZ_EINVAL;
    if (ops_per_iter) *ops_per_iter = (int32_t)VALU_PROBE_OPS;
    hipLaunchKernelGGL(kpz_valu_probe_kernel, dim3((uint32_t)n_groups), dim3(256), 0,
                       (hipStream_t)stream, d_out, (uint32_t)iters);
    return hipGetLastError() == hipSuccess ? KPZ_OK : KPZ_EHIP;
}

kpz_status kpz_roughness_noalloc(const uint32_t *d_words, int64_t L, int64_t net, int64_t *S1o,
                                 int64_t *S2o, double *W2o, void *stream)
{
    clear_pending_error();
    if (!d_words || L < 16 || (L % 16) != 0) return KPZ_EINVAL;
    if (L > KPZ_NOALLOC_MAX_L) {
        snprintf(g_init_err, sizeof g_init_err,
                 "kpz_roughness_noalloc: L = %lld exceeds the scratch maximum %d",
                 (long long)L, KPZ_NOALLOC_MAX_L);
        return KPZ_ESIZE;
    }
    void *base = nullptr;
    const kpz_status sst = scratch_on_current_device(&base);
    if (sst != KPZ_OK) return sst;
    hipStream_t st = (hipStream_t)stream;
    long long *res = (long long *)base;
    long long *slots = (long long *)((uint8_t *)base + WS_HEADER);
    long long *rowA = slots + NSLOTS, *rowB = rowA + L;
    const uint32_t Lu = (uint32_t)L, W = Lu / 16;
    const Rot none = {0u, 0u, 0u, 16u, 0u, 0u};
    // every slot is rewritten (slot 0 = net) before the moments read them;
    // the header and row sums are written before they are read
    hipLaunchKernelGGL(kpz_fill_counters_kernel, dim3(NSLOTS / 256), dim3(256), 0, st, slots,
                       (long long)net);
    if (Lu <= SMALL_ROWS) {
        hipLaunchKernelGGL(kpz_roughness_small_kernel, dim3(1), dim3(1024), 0, st, d_words, Lu, W,
                           (const long long *)slots, res, none);
    } else {
        hipLaunchKernelGGL(kpz_row_moments_kernel, dim3(row_grid(row_tasks(Lu))),
                           dim3(64 * ROW_WAVES), 0, st, d_words, Lu, W,
                           rowA, rowB);
        hipLaunchKernelGGL(kpz_finalize_kernel, dim3(1), dim3(1024), 0, st, Lu,
                           (const long long *)rowA, (const long long *)rowB,
                           (const long long *)slots, res, d_words, none);
    }
    hipError_t e = hipGetLastError();
    long long h[4];
    if (e == hipSuccess) e = hipMemcpyAsync(h, res, sizeof h, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        set_init_error(e, "kpz_roughness_noalloc");
        return KPZ_EHIP;
    }
    return convert_moments(h, L, S1o, S2o, W2o, g_init_err, sizeof g_init_err);
}

}  // extern "C"
