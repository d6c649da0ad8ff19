// kpz_slice.h -- bit-sliced single-hit double tiling of one dead-border block
// per wave64 (gfx950).
//
// Paper: Sec. 3 (dead-border blocks, origin moved between residencies),
// Sec. 3.1 (single-hit double tiling: every tile of a work-group updates one
// site of the cell set chosen for the step, the cells of one set never
// touch), Sec. 2.1 eq. "rule" (a local minimum becomes a maximum with
// probability p, a maximum a minimum with probability q).
//
// Layout in registers.  Tiles are 4 x 4 sites, split into four 2 x 2 cells
// (set s = sx + 2 sy).  A block of Bx x By sites has nty = By / 4 tile rows;
// each tile row is cut into nqx = max(1, Bx / 128) row groups of up to 32
// tiles.  Lane q * nty + ty of the wave holds row group q of tile row ty as
// 32 "plane" words: X[r][c] holds sigma_x and Y[r][c] sigma_y of the sites
// (4 tx + c, 4 ty + r) of every tile tx of the group, tile tx at bit
// pi(tx) = 8 (tx mod 4) + tx / 4.  With that bit order a group's eight
// packed lattice words (16 sites of 2 bits each) become its eight plane words
// of one row by one 8 x 8 bit transpose done in the four bytes at once.
//
// A step then updates the 32 tiles of a group with whole-word logic: the
// chosen site of every tile (rx, ry from the tile's bit of two random words)
// is selected from the planes by bit-select, the minimum and maximum tests
// and the flip are bitwise.  Neighbours outside the lane: the slope one tile
// to the left (bit shift within the word; the group's first tile takes it
// from the group to the left, a ds_bpermute), the slope one row below the
// tile row (the lane below, a DPP wave shift).  The attempts of a step never
// share a slope (Sec. 3.1), so one pass of reads then one pass of writes is
// exact.
#ifndef KPZ_SLICE_H_
#define KPZ_SLICE_H_

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kpz_device.h"

namespace kpzslice {

using kpzdev::philox_v;
using kpzdev::U4;

// (m & a) | (~m & b): one v_bfi_b32
__device__ __forceinline__ uint32_t bsel(uint32_t m, uint32_t a, uint32_t b)
{
    return (m & a) | (~m & b);
}

// Swap the bits of `hi` under mask m with the bits of `lo` under m << s.
__device__ __forceinline__ void swap_bits(uint32_t &lo, uint32_t &hi, int s, uint32_t m)
{
    const uint32_t l = lo, h = hi;
    lo = bsel(m << s, h << s, l);
    hi = bsel(m, l >> s, h);
}

// In each of the four bytes at once, transposes the 8 x 8 bit matrix whose
// row i is byte j of w[i]: afterwards bit i of byte j of w[p] is the former
// bit p of byte j of w[i].  Three stages of block swaps (4, 2, 1); the
// transpose is its own inverse.
__device__ __forceinline__ void transpose8(uint32_t (&w)[8])
{
#pragma unroll
    for (int i = 0; i < 4; ++i) swap_bits(w[i], w[i + 4], 4, 0x0F0F0F0Fu);
#pragma unroll
    for (int i = 0; i < 8; i += 4) {
        swap_bits(w[i], w[i + 2], 2, 0x33333333u);
        swap_bits(w[i + 1], w[i + 3], 2, 0x33333333u);
    }
#pragma unroll
    for (int i = 0; i < 8; i += 2) swap_bits(w[i], w[i + 1], 1, 0x55555555u);
}

// Tile shifts in the pi bit order.  prev_tile: bit pi(tx) <- bit pi(tx - 1)
// (tile 0 gets an arbitrary bit, replaced or masked by the caller).
// next_tile: bit pi(tx) <- bit pi(tx + 1), tile 0's own bit dropped.
__device__ __forceinline__ uint32_t prev_tile(uint32_t v)
{
    return (v << 8) | __builtin_amdgcn_ubfe(v, 23u, 8u);
}

__device__ __forceinline__ uint32_t next_tile(uint32_t v)
{
    return (v >> 8) | (__builtin_amdgcn_ubfe(v, 1u, 7u) << 24);
}

// Lane exchanges.  dpp_down: value of lane l - 1 (0 in lane 0); dpp_up:
// value of lane l + 1 (0 in lane 63).
__device__ __forceinline__ uint32_t dpp_down(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x138, 0xf, 0xf, true);   // wave_shr:1
}

__device__ __forceinline__ uint32_t dpp_up(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x130, 0xf, 0xf, true);   // wave_shl:1
}

__device__ __forceinline__ uint32_t bperm(uint32_t addr4, uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_ds_bpermute((int)addr4, (int)v);
}

// Per-lane constants of a block's steps.
struct LaneCtx {
    uint32_t vm;      // tiles of the lane's group (0 for idle lanes)
    uint32_t dxm;     // 1: tile 0's left column is the dead border
    uint32_t dym;     // ~0: the tile row's bottom row is the dead border
    uint32_t xn;      // (uniform) tile 0's left neighbour is in another lane / wraps
                      // (read when the XN template argument is 2)
    uint32_t srcL4;   // ds_bpermute address of the lane holding the left group (the
                      // block's last group for group 0: its wrap, or unused when the
                      // left column is the dead border)
    uint32_t srcR4;   // ... the right group (group 0 for the last group: its wrap, or
                      // a dead tile 0 that never flips)
    uint32_t rmask;   // DT: ~0 when the right group is in the block
    uint32_t pb;      // bit of the group's last tile
    uint32_t wrapy;   // (uniform) one block along y: the tile row below wraps
                      // (read when the step's WY template argument is 2)
    uint32_t srcD4;   // wrapy: lane holding the tile row below
    uint32_t srcU4;   // wrapy: lane holding the tile row above
    // double tiling at the device layer (no dead sites): halos of group 0 /
    // tile row 0 come from the idle neighbour blocks
    uint32_t hxl;     // ~0 in lanes of group 0 (left halo column)
    uint32_t hyl;     // ~0 in lanes of tile row 0 (halo row below)
    uint32_t uym;     // 0 in lanes of the last tile row (flips from above are not theirs)
};

// Acceptance state of an MCS (thresholds over 2^32, Sec. 2.1 p and q).
struct AccDraw {
    uint64_t P, Q;
    uint32_t nlP, nlQ;   // levels after which a tie means u >= threshold (0: no draw)
    uint32_t nl;         // max(nlP, nlQ)
    uint32_t seed_lo, seed_hi, t;
    uint32_t G;          // this lane's row group
};

// Number of uniform bits that decide u < T for 0 < T < 2^32: 32 - ctz(T).
__host__ __device__ __forceinline__ uint32_t levels_of(uint64_t T)
{
    if (T == 0 || T >= (1ull << 32)) return 0;
    uint32_t n = 32;
    while (!((T >> (32 - n)) & 1u)) --n;
    return n;
}

// The tiles of `mn` (minima) accepted with probability p and of `mx`
// (maxima) with probability q.  The uniform u of a tile is compared with
// the threshold bit by bit from the top: level j (j = 0..31) is bit 31 - j
// of u, the tile's bit of word (k mod 4) of draw (ACC1, t, G, 4 (k / 4) + j)
// for j < 4 (lev[j], drawn for the four steps of k / 4) and of word j mod 4
// of draw (ACC2, t, G, 8 k + j / 4 - 1) beyond.  Levels are drawn only while
// a tile of the wave is still tied with its threshold.
template <uint32_t TAG_ACC2>
__device__ __forceinline__ uint32_t accept(uint32_t mn, uint32_t mx, const uint32_t (&lev)[4],
                                           const AccDraw &d, uint32_t k, int &net)
{
    const uint64_t FULL = 1ull << 32;
    uint32_t fP = d.P >= FULL ? mn : 0u, eqP = d.nlP ? mn : 0u;
    uint32_t fQ = d.Q >= FULL ? mx : 0u, eqQ = d.nlQ ? mx : 0u;
    const uint32_t P = (uint32_t)d.P, Q = (uint32_t)d.Q;
#pragma unroll
    for (uint32_t j = 0; j < 4; ++j) {
        if (j >= d.nl || !__any((eqP | eqQ) != 0u)) break;
        const uint32_t U = lev[j];
        if ((P >> (31 - j)) & 1u) { fP |= eqP & ~U; eqP &= U; } else { eqP &= ~U; }
        if ((Q >> (31 - j)) & 1u) { fQ |= eqQ & ~U; eqQ &= U; } else { eqQ &= ~U; }
        if (j + 1 >= d.nlP) eqP = 0u;
        if (j + 1 >= d.nlQ) eqQ = 0u;
    }
    for (uint32_t jb = 4; jb < d.nl; jb += 4) {
        if (!__any((eqP | eqQ) != 0u)) break;
        const U4 w = philox_v<kpzdev::LATTICE_ROUNDS>(d.G, 0u, d.t, (TAG_ACC2 << 24) | (8u * k + jb / 4u - 1u), d.seed_lo,
                              d.seed_hi);
        const uint32_t ws[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
        for (uint32_t jj = 0; jj < 4; ++jj) {
            const uint32_t j = jb + jj;
            if (j >= d.nl) break;
            const uint32_t U = ws[jj];
            if ((P >> (31 - j)) & 1u) { fP |= eqP & ~U; eqP &= U; } else { eqP &= ~U; }
            if ((Q >> (31 - j)) & 1u) { fQ |= eqQ & ~U; eqQ &= U; } else { eqQ &= ~U; }
            if (j + 1 >= d.nlP) eqP = 0u;
            if (j + 1 >= d.nlQ) eqQ = 0u;
        }
    }
    net += __builtin_popcount(fP) - __builtin_popcount(fQ);
    return fP | fQ;
}

// The slope bond between the last tile of a row group and the first tile of
// the next group (sigma_x at the group boundary, one bit per row) is written
// by the left group's last tile in steps with sx = 1 and by the right group's
// first tile in steps with sx = 0, and read likewise.  The left group keeps it
// as bit pb of X[r][3]; the right group keeps a copy `hl` (bit r for row r)
// that is authoritative during a run of sx = 0 steps: pull_bond copies it
// from the left lane before such a run, push_bond copies it back after it,
// one lane exchange per change of sx instead of two per step.  DT: group 0's
// bond is the halo column hx of the idle block to the left.
__device__ __forceinline__ void pull_bond(const uint32_t (&X)[4][4], const LaneCtx &c, bool xn,
                                          bool dt, uint32_t hx, uint32_t &hl)
{
    uint32_t v = 0u;
    if (xn) {
        const uint32_t e = __builtin_amdgcn_ubfe(X[0][3], c.pb, 1u) |
                           (__builtin_amdgcn_ubfe(X[1][3], c.pb, 1u) << 1) |
                           (__builtin_amdgcn_ubfe(X[2][3], c.pb, 1u) << 2) |
                           (__builtin_amdgcn_ubfe(X[3][3], c.pb, 1u) << 3);
        v = bperm(c.srcL4, e);
    }
    hl = dt ? bsel(c.hxl, hx, v) : v;
}

__device__ __forceinline__ void push_bond(uint32_t (&X)[4][4], const LaneCtx &c, bool xn, bool dt,
                                          uint32_t &hx, uint32_t hl)
{
    if (dt) hx = bsel(c.hxl, hl, hx);
    if (!xn) return;
    const uint32_t v = bperm(c.srcR4, hl);
    // DT: the last group's right bond stays its own (idle block beyond)
    const uint32_t m = (1u << c.pb) & (dt ? c.rmask : ~0u);
#pragma unroll
    for (int r = 0; r < 4; ++r)
        X[r][3] = bsel(m, __builtin_amdgcn_alignbit(v, v, ((uint32_t)r - c.pb) & 31u), X[r][3]);
}

// One single-hit step with cell set (SX, SY) for the 32 tiles of this lane's
// row group.  RX, RY: the site of every tile in its 2 x 2 cell (tile bit).
// hl: the group's left boundary bond (see pull_bond; used when XB).  DT: halo
// row hy[c] (sigma_y below tile row 0, lanes of tile row 0).  WY: 0 or 1 fix
// the wrapped tile row below at compile time; 2 reads it from the context.
template <int SX, int SY, bool ACC, bool DT, bool XB, int WY, uint32_t TAG_ACC2>
__device__ __forceinline__ void step(uint32_t (&X)[4][4], uint32_t (&Y)[4][4], uint32_t RX,
                                     uint32_t RY, const LaneCtx &c, const uint32_t (&lev)[4],
                                     const AccDraw &d, uint32_t k, int &net, uint32_t &hl,
                                     uint32_t (&hy)[4])
{
    constexpr int R0 = 2 * SY, C0 = 2 * SX;
    const bool wrapy = !DT && (WY == 2 ? c.wrapy != 0u : WY == 1);
    // sigma_x one column left of C0, rows R0 and R0 + 1
    uint32_t xm0, xm1;
    if (SX) {
        xm0 = X[R0][1];
        xm1 = X[R0 + 1][1];
    } else {
        xm0 = prev_tile(X[R0][3]);
        xm1 = prev_tile(X[R0 + 1][3]);
        if (XB) {
            // tile 0: the bond to the group on the left
            xm0 = bsel(1u, hl >> R0, xm0);
            xm1 = bsel(1u, hl >> (R0 + 1), xm1);
        }
    }
    // sigma_y one row below R0, columns C0 and C0 + 1
    uint32_t yd0, yd1;
    if (SY) {
        yd0 = Y[1][C0];
        yd1 = Y[1][C0 + 1];
    } else if (wrapy) {
        yd0 = bperm(c.srcD4, Y[3][C0]);
        yd1 = bperm(c.srcD4, Y[3][C0 + 1]);
    } else {
        yd0 = dpp_down(Y[3][C0]);
        yd1 = dpp_down(Y[3][C0 + 1]);
        if (DT) {
            yd0 = bsel(c.hyl, hy[C0], yd0);
            yd1 = bsel(c.hyl, hy[C0 + 1], yd1);
        }
    }
    const uint32_t xa0 = bsel(RX, X[R0][C0 + 1], X[R0][C0]);
    const uint32_t xa1 = bsel(RX, X[R0 + 1][C0 + 1], X[R0 + 1][C0]);
    const uint32_t xc0 = bsel(RX, X[R0][C0], xm0);
    const uint32_t xc1 = bsel(RX, X[R0 + 1][C0], xm1);
    const uint32_t yb0 = bsel(RX, Y[R0][C0 + 1], Y[R0][C0]);
    const uint32_t yb1 = bsel(RX, Y[R0 + 1][C0 + 1], Y[R0 + 1][C0]);
    const uint32_t ydm = bsel(RX, yd1, yd0);
    const uint32_t sa = bsel(RY, xa1, xa0);   // sigma_x(x, y)
    const uint32_t sb = bsel(RY, yb1, yb0);   // sigma_y(x, y)
    const uint32_t sc = bsel(RY, xc1, xc0);   // sigma_x(x - 1, y)
    const uint32_t sd = bsel(RY, yb0, ydm);   // sigma_y(x, y - 1)
    // live tiles: the dead border (site lx = 0 or ly = 0) is never updated
    uint32_t lm = c.vm;
    if (!DT) {
        if (!SX) lm = bsel(c.dxm, RX, lm);
        if (!SY) lm &= RY | ~c.dym;
    }
    // minimum: own slopes +1, incoming slopes -1; maximum: the reverse
    const uint32_t mn = sa & sb & ~(sc | sd) & lm;
    uint32_t F;
    if (ACC) {
        const uint32_t mx = sc & sd & ~(sa | sb) & lm;
        F = accept<TAG_ACC2>(mn, mx, lev, d, k, net);
    } else {
        F = mn;
        net += __builtin_popcount(mn);
    }
    // flip: sigma_x(x), sigma_x(x - 1), sigma_y(x), sigma_y(x, y - 1)
    const uint32_t F1 = F & RY, F0 = F ^ F1;
    const uint32_t F01 = F0 & RX, F00 = F0 ^ F01;
    const uint32_t F11 = F1 & RX, F10 = F1 ^ F11;
    X[R0][C0] ^= F0;
    X[R0][C0 + 1] ^= F01;
    X[R0 + 1][C0] ^= F1;
    X[R0 + 1][C0 + 1] ^= F11;
    if (SX) {
        X[R0][1] ^= F00;
        X[R0 + 1][1] ^= F10;
    } else {
        X[R0][3] ^= next_tile(F00);
        X[R0 + 1][3] ^= next_tile(F10);
        if (XB) hl ^= ((F00 & 1u) | ((F10 & 1u) << 1)) << R0;
    }
    Y[R0][C0] ^= F00 ^ F10;
    Y[R0][C0 + 1] ^= F01 ^ F11;
    Y[R0 + 1][C0] ^= F10;
    Y[R0 + 1][C0 + 1] ^= F11;
    if (SY) {
        Y[1][C0] ^= F00;
        Y[1][C0 + 1] ^= F01;
    } else if (wrapy) {
        Y[3][C0] ^= bperm(c.srcU4, F00);
        Y[3][C0 + 1] ^= bperm(c.srcU4, F01);
    } else {
        uint32_t u0 = dpp_up(F00), u1 = dpp_up(F01);
        if (DT) {
            u0 &= c.uym;
            u1 &= c.uym;
            hy[C0] ^= F00 & c.hyl;
            hy[C0 + 1] ^= F01 & c.hyl;
        }
        Y[3][C0] ^= u0;
        Y[3][C0 + 1] ^= u1;
    }
}

}  // namespace kpzslice

#endif  // KPZ_SLICE_H_
