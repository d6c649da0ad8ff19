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
// Kernels
//   kpz_init_kernel         flat start, HBM write stream
//   kpz_sweep_kernel<K,ACC> one MCS: one wave64 work-group per dead-border
//                           block; block in LDS; 16 single-hit steps
//   kpz_row_moments_kernel  per-row (sum, sum of squares) of the x-prefix
//                           heights, a lane group per row (a wave for long
//                           rows), HBM read stream
//   kpz_finalize_kernel     column-0 prefix, 128-bit totals, flip counters,
//                           one work-group, one pass over the row sums
//
// LDS layout of a block in the sweep.  Tiles are 4 x 4 sites, each split
// into four 2 x 2 cells; cell set s = sx + 2 sy.  A cell is one byte: site
// (rx, ry) of the cell at bits 2(2 ry + rx) (sigma_x) and +1 (sigma_y).
// Four tiles of one tile column, (tx, qy + j H) for j = 0..3 with
// H = nty / 4, share one dword ("quad"), byte j; the LDS holds four planes
// (one per cell set) of nq = ntx * H quads.  Every bitwise operation of the
// update therefore serves four tiles at once (the paper's several domains
// per work-item, realised as SIMD within a 32-bit register), and the 64
// lanes of a wave read consecutive dwords (no bank conflicts).
//
// Random numbers: Philox4x32-10 (Salmon et al., SC'11) keyed by the seed,
// counter (idx_lo, idx_hi, t, tag << 24 | sub):
//   origin    (ORIGIN, t, 0, 0):  ox = w0*Bx >> 32, oy = w1*By >> 32
//   sets      (SET, t, block, 0): step k uses bits 2k..2k+1 of w0
//   sites     (SITE, t, G, 0):    G = block*nq + quad; tile j of the quad,
//                                 step k: bits 8j + 2(k&3) of word k>>2
//   accept    u = A << 24 | (B & 0xFFFFFF), A = byte j of word k&3 of
//             (ACC1, t, G, k>>2), B = word j of (ACC2, t, G, k); B is
//             generated only when A alone cannot decide u < threshold.

#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <deque>
#include <map>
#include <new>
#include <vector>

#include "kpz.h"
#include "kpz_device.h"

namespace {

using kpzdev::byte_eq;
using kpzdev::byte_lt;
using kpzdev::philox;
using kpzdev::U4;

constexpr uint32_t TAG_ORIGIN = 1, TAG_SET = 2, TAG_SITE = 3, TAG_ACC1 = 4, TAG_ACC2 = 5;
constexpr int NSLOTS = 1024;          // flip-counter slots in the workspace
constexpr int WS_HEADER = 256;        // results area at the start of the workspace
constexpr int TILE = 4;               // tile edge (sites)

// ------------------------------------------------------------ bit helpers

__device__ __forceinline__ uint32_t rotr(uint32_t x, uint32_t s)
{
    return __builtin_amdgcn_alignbit(x, x, s);
}

// 4 x 4 byte transpose: out[m].byte[j] = in[j].byte[m].
__device__ __forceinline__ void transpose_bytes(uint32_t v[4])
{
    const uint32_t t0 = __builtin_amdgcn_perm(v[1], v[0], 0x05010400u);
    const uint32_t t1 = __builtin_amdgcn_perm(v[1], v[0], 0x07030602u);
    const uint32_t t2 = __builtin_amdgcn_perm(v[3], v[2], 0x05010400u);
    const uint32_t t3 = __builtin_amdgcn_perm(v[3], v[2], 0x07030602u);
    v[0] = __builtin_amdgcn_perm(t2, t0, 0x05040100u);
    v[1] = __builtin_amdgcn_perm(t2, t0, 0x07060302u);
    v[2] = __builtin_amdgcn_perm(t3, t1, 0x05040100u);
    v[3] = __builtin_amdgcn_perm(t3, t1, 0x07060302u);
}

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
    unsigned long long *slots;   // NSLOTS flip counters
    uint32_t L, W;               // size, words per row
    uint32_t Bx, By;             // block shape
    uint32_t nbx, nby;           // blocks per direction
    uint32_t ntx, log2ntx;       // tiles per block row
    uint32_t H, log2H;           // quad rows per plane (nty / 4)
    uint32_t nq;                 // quads per plane
    uint32_t nw, log2nw;         // aligned words per block row (Bx / 16)
    uint32_t units;              // load/store units per block (nq / 2)
    uint32_t seed_lo, seed_hi;
    uint32_t t;
    uint32_t res;                // residency of MCS t (origin move), 0 .. moves - 1
    uint32_t nsteps;             // single-hit steps per residency (16 / moves)
    uint32_t slot_mask;          // flip-counter slots - 1 (power of two)
    uint32_t acc;                // 1 unless P = 2^32 and Q = 0 (acceptance draws needed)
    // Two-buffer mode (db = 1): the launch reads src and writes words, a
    // different buffer.  src is stored rotated by s_in sites (word w of a row
    // holds sites 16 w + s_in ..), s_in = (x origin of launch (prev_t,
    // prev_res)) mod 16 when prev_valid, else 0; the output is stored rotated
    // by this launch's x origin mod 16, so every block writes whole words of
    // its own and no word is shared.  db = 0: in place, shared words through
    // the side buffer.
    uint32_t db, prev_valid, prev_t, prev_res;
    uint32_t xcd;                // 1: map work-groups so that consecutive blocks share an XCD
    // ensemble members in two-buffer mode: buffer 0 is `words`, buffer 1 is
    // `alt`; at the start of a call the state is in buffer cur0, rotated as
    // written by launch (prev_t, prev_res) when prev_valid
    uint32_t *alt;
    uint32_t cur0;
    uint64_t P, Q;               // acceptance thresholds over 2^32
};

// Storage rotation of a lattice buffer written in two-buffer mode: the x
// origin of the launch that wrote it, mod 16 (0 for a buffer in the
// documented layout, valid = 0).
struct Rot {
    uint32_t valid, t, res, Bx, seed_lo, seed_hi;
};

__device__ __forceinline__ uint32_t rot_sites(const Rot &r)
{
    if (!r.valid) return 0u;
    const U4 w = philox(r.res, 0u, r.t, TAG_ORIGIN << 24, r.seed_lo, r.seed_hi);
    return (uint32_t)(((uint64_t)w.x * r.Bx) >> 32) & 15u;
}

// Quad q = tid + TPB i (tid = thread in the block) has tile column
// qx = q mod ntx and quad row qy = q / ntx.  With NTX (= ntx) known at
// compile time both tests below fold to constants or a single lane compare.
template <int TPB, int NTX>
__device__ __forceinline__ bool quad_left_edge(uint32_t tid, int i, const SweepArgs &a)
{
    if constexpr (NTX >= TPB) return (i % (NTX / TPB)) == 0 && tid == 0;
    else if constexpr (NTX > 0) return (tid & (NTX - 1)) == 0;
    else return ((tid + (uint32_t)TPB * i) & (a.ntx - 1)) == 0;
}

template <int TPB, int NTX>
__device__ __forceinline__ bool quad_bottom_row(uint32_t tid, int i, const SweepArgs &a)
{
    if constexpr (NTX >= TPB) return i < NTX / TPB;
    else if constexpr (NTX > 0) return i == 0 && tid < (uint32_t)NTX;
    else return tid + (uint32_t)TPB * i < a.ntx;
}

// Byte-wise helpers for the acceptance test of four tiles at once (byte_lt
// and byte_eq are in kpz_device.h).
__device__ __forceinline__ uint32_t bytes_nonzero(uint32_t F)
{
    // F has at most one bit per byte, at position 0, 2, 4 or 6
    return (F + 0x7F7F7F7Fu) & 0x80808080u;
}

__device__ __forceinline__ uint32_t expand_bit7(uint32_t m7)
{
    const uint32_t m = m7 >> 7;
    return (m << 8) - m;
}

struct AccCtx {
    bool fullP;          // P = 2^32: every minimum is accepted
    bool ties;           // a threshold below 2^32 has nonzero low bits: A equal
                         // to its top byte needs the second draw
    uint32_t tP, tQ;     // top bytes of P and Q
    uint32_t lowP, lowQ; // low 24 bits of P and Q
};

// One single-hit attempt in each of the four tiles of a quad.  ca, la, da:
// LDS indices of the quad's own cells (set s), the cells to the left (set
// s^1) and the cells below (set s^2).
//
// DT (double tiling at the device layer): with splice set (a bottom-row quad
// and sy = 0) the lower cell of byte 0 is the halo byte at LDS index hb (the
// block below), not byte 3 of the block's top quad row.
template <int SX, int SY, bool ACC, bool DT>
__device__ __forceinline__ void quad_update(uint32_t *lds, uint32_t ca, uint32_t la, uint32_t da,
                                            uint32_t rot, uint32_t D, uint32_t dm, bool lok,
                                            uint32_t Aw, const AccCtx &ac, uint64_t G, uint32_t k,
                                            const SweepArgs &a, int &net, bool splice = false,
                                            uint32_t hb = 0)
{
    const uint32_t c = lds[ca];
    const uint32_t l = lds[la];
    const uint32_t top = SY ? 0u : lds[da];
    uint32_t d = SY ? lds[da] : rotr(top, rot);
    if (DT && !SY && splice) d = (d & ~0xFFu) | (lds[hb] & 0xFFu);
    // one-hot sigma_x position 2r of each tile's chosen site
    const uint32_t oh = __builtin_amdgcn_perm(0u, 0x40100401u, D) & ~dm;
    // neighbour slopes moved onto each site's own bit positions:
    // sigma_x(x-1,y) at 2r, sigma_y(x,y-1) at 2r+1
    const uint32_t X = ((c << 2) & 0x44444444u) | ((l >> 2) & 0x11111111u);
    const uint32_t Y = ((c << 4) & 0xA0A0A0A0u) | ((d >> 4) & 0x0A0A0A0Au);
    const uint32_t N = X | Y;
    // minimum: own slopes (+1,+1), incoming slopes (-1,-1)
    const uint32_t zmin = c & ~N;
    uint32_t F = zmin & (zmin >> 1) & oh;
    if (ACC) {
        // maximum: own slopes (-1,-1), incoming slopes (+1,+1).  A byte (tile)
        // holds a minimum flip in F or a maximum flip in Fx, never both, so
        // the P test applies to F and the Q test to Fx byte by byte
        const uint32_t zmax = N & ~c;
        const uint32_t Fx = zmax & (zmax >> 1) & oh;
        // bit 7 of each byte: the tile's uniform A accepts
        uint32_t accP = ac.fullP ? 0x80808080u : (ac.tP ? byte_lt(Aw, ac.tP) : 0u);
        uint32_t accQ = ac.tQ ? byte_lt(Aw, ac.tQ) : 0u;
        if (ac.ties) {
            const uint32_t tieP = (!ac.fullP && ac.lowP) ? (bytes_nonzero(F) & byte_eq(Aw, ac.tP)) : 0u;
            const uint32_t tieQ = ac.lowQ ? (bytes_nonzero(Fx) & byte_eq(Aw, ac.tQ)) : 0u;
            if (__any((tieP | tieQ) != 0)) {
                const U4 w2 = philox((uint32_t)G, (uint32_t)(G >> 32), a.t,
                                     (TAG_ACC2 << 24) | (16u * a.res + k),
                                     a.seed_lo, a.seed_hi);
                const uint32_t Bw[4] = {w2.x, w2.y, w2.z, w2.w};
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const uint32_t b24 = Bw[j] & 0xFFFFFFu;
                    if (((tieP >> (8 * j + 7)) & 1u) && b24 < ac.lowP) accP |= 0x80u << (8 * j);
                    if (((tieQ >> (8 * j + 7)) & 1u) && b24 < ac.lowQ) accQ |= 0x80u << (8 * j);
                }
            }
        }
        const uint32_t fmin = F & expand_bit7(accP), fmax = Fx & expand_bit7(accQ);
        net += __builtin_popcount(fmin) - __builtin_popcount(fmax);
        F = fmin | fmax;
    } else {
        net += __builtin_popcount(F);
    }
    // flip: own sigma_x, sigma_y; sigma_x of the left site; sigma_y of the lower site
    const uint32_t mc = F | (F << 1) | ((F >> 2) & 0x11111111u) | ((F >> 3) & 0x0A0A0A0Au);
    const uint32_t ml = (F & 0x11111111u) << 2;
    const uint32_t md = (F & 0x05050505u) << 5;
    lds[ca] = c ^ mc;
    if (SX || lok) lds[la] = l ^ ml;
    if (SY) {
        lds[da] = d ^ md;
    } else if (DT && splice) {
        // bytes 1..3 go back to the top quad row (bytes 0..2), byte 0 to the
        // halo; the top row's byte 3 keeps its value
        const uint32_t nd = d ^ md;
        lds[da] = (rotr(nd, 8u) & 0x00FFFFFFu) | (top & 0xFF000000u);
        lds[hb] = nd & 0xFFu;
    } else {
        lds[da] = rotr(d ^ md, (32u - rot) & 31u);
    }
}

// All quads of this thread for one step with cell set (SX, SY).
template <int TPB, int K, int NTX, int SX, int SY, bool ACC, bool DT>
__device__ __forceinline__ void step_quads(uint32_t *lds, uint32_t tid, uint32_t kr,
                                           const uint32_t (&sw)[K][4], const uint32_t (&aw)[K][4],
                                           const AccCtx &ac, uint64_t Gbase, uint32_t k,
                                           const SweepArgs &a, int &net)
{
    constexpr uint32_t S = SX + 2 * SY;
    const uint32_t ntx = NTX ? (uint32_t)NTX : a.ntx;
    const uint32_t nq = NTX ? (uint32_t)NTX * a.H : a.nq;
    const uint32_t pc = S * nq, pl = (S ^ 1u) * nq, pd = (S ^ 2u) * nq;
#pragma unroll
    for (int i = 0; i < K; ++i) {
        const uint32_t q = tid + (uint32_t)TPB * i;
        const bool ledge = SX ? false : quad_left_edge<TPB, NTX>(tid, i, a);
        const bool bottom = SY ? false : quad_bottom_row<TPB, NTX>(tid, i, a);
        // left quad (tile tx-1) for sx = 0: q-1, or the wrap-around quad of
        // a single periodic block, or (dead left edge) the quad itself,
        // which is then only read
        const uint32_t lq = SX ? q : (ledge ? (a.nbx == 1 ? q + ntx - 1 : q) : q - 1);
        // lower quad (tile ty-1) for sy = 0: q - ntx, or for the bottom quad
        // row the top quad row, one byte down
        const uint32_t dq = SY ? q : (bottom ? q + (a.H - 1) * ntx : q - ntx);
        const uint32_t rot = bottom ? 24u : 0u;
        if constexpr (DT) {
            // no dead sites: the left cells of the left edge are the halo
            // column (hcol[sy][qy] after the four planes), the lower cells of
            // the bottom row's first tile row the halo row (hrow[sx][tx])
            const uint32_t la = ledge ? 4 * nq + SY * a.H + q / ntx : pl + lq;
            const uint32_t hb = 4 * nq + 2 * a.H + SX * ntx + (q & (ntx - 1));
            const uint32_t D = (sw[i][0] >> (2 * kr)) & 0x03030303u;
            quad_update<SX, SY, ACC, true>(lds, pc + q, la, pd + dq, rot, D, 0u, true,
                                           ACC ? aw[i][0] : 0u, ac, Gbase + q, k, a, net, bottom,
                                           hb);
        } else {
            const uint32_t dm = (ledge && a.nbx > 1 ? 0x11111111u : 0u) |
                                (bottom && a.nby > 1 ? 0x00000005u : 0u);
            const bool lok = !ledge || a.nbx == 1;
            const uint32_t D = (sw[i][0] >> (2 * kr)) & 0x03030303u;
            quad_update<SX, SY, ACC, false>(lds, pc + q, pl + lq, pd + dq, rot, D, dm, lok,
                                            ACC ? aw[i][0] : 0u, ac, Gbase + q, k, a, net);
        }
    }
}

// One MCS of dead-border block b (device layer) with the block in LDS.  DT:
// block b of a double-tiling set instead (no dead sites, in place): the
// left neighbour's last column and the lower neighbour's top row are loaded
// as halos after the four planes, and written back (read-modify-write of
// the slopes this block may flip) after the block's own words.
template <int TPB, int K, int NTX, bool ACC, bool DT = false>
__device__ __forceinline__ void sweep_block(const SweepArgs &a, uint32_t b, uint32_t *lds)
{
    const uint32_t tid = threadIdx.x;
    const uint32_t bx = b % a.nbx, by = b / a.nbx;
    const uint32_t ntx = NTX ? (uint32_t)NTX : a.ntx;
    const uint32_t nq = NTX ? (uint32_t)NTX * a.H : a.nq;
    const uint32_t nw = ntx / 4;

    // device layer: origin of this residency, then this block's frame
    const U4 wo = philox(a.res, 0u, a.t, TAG_ORIGIN << 24, a.seed_lo, a.seed_hi);
    const uint32_t ox = (uint32_t)(((uint64_t)wo.x * a.Bx) >> 32);
    const uint32_t oy = (uint32_t)(((uint64_t)wo.y * a.By) >> 32);
    uint32_t gx0 = ox + bx * a.Bx;
    if (gx0 >= a.L) gx0 -= a.L;
    uint32_t gy0 = oy + by * a.By;
    if (gy0 >= a.L) gy0 -= a.L;
    // storage rotation of the input (two-buffer mode)
    const uint32_t s_in =
        rot_sites(Rot{a.db & a.prev_valid, a.prev_t, a.prev_res, a.Bx, a.seed_lo, a.seed_hi});
    uint32_t px0 = gx0 + (a.L - s_in);          // storage position of the block's first site
    if (px0 >= a.L) px0 -= a.L;
    const uint32_t sh2 = 2u * (px0 & 15u);
    const uint32_t gw0 = px0 >> 4;
    // two-buffer mode: the output is rotated by ox mod 16, so the block's
    // first site starts output word (ox >> 4) + bx nw
    uint32_t gwo = (ox >> 4) + bx * nw;
    if (gwo >= a.W) gwo -= a.W;

    // ---- load: HBM row words -> aligned block words -> cells -> quads.
    // Unit u = (wx, qy, sy): aligned word column wx of the two rows of cell
    // row sy in the tile rows qy + j H, j = 0..3.  The nw units of one row
    // group sit in consecutive lanes of one wave (nw divides 64), so the next
    // word of a row comes from the next lane.
    constexpr int UIT = (K * TPB / 2 + TPB - 1) / TPB;
    for (int it = 0; it < UIT; ++it) {
        const uint32_t u = tid + (uint32_t)TPB * it;
        const bool uok = u < a.units;
        const uint32_t wx = u & (nw - 1);
        const uint32_t rest = u >> a.log2nw;
        const uint32_t qy = rest & (a.H - 1);
        const uint32_t sy = rest >> a.log2H;
        uint32_t gw = gw0 + wx;
        if (gw >= a.W) gw -= a.W;
        const uint32_t gw1 = gw + 1 == a.W ? 0 : gw + 1;
        uint32_t E[4], O[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint32_t r0 = 4 * (qy + j * a.H) + 2 * sy;
            uint32_t A[2];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                uint32_t gy = gy0 + r0 + h;
                if (gy >= a.L) gy -= a.L;
                const uint32_t *row = a.src + (size_t)gy * a.W;
                const uint32_t lo = uok ? row[gw] : 0u;
                uint32_t hi = __shfl_down(lo, 1, 64);
                if (uok && wx == nw - 1 && sh2) hi = row[gw1];
                A[h] = __builtin_amdgcn_alignbit(hi, lo, sh2);
            }
            E[j] = (A[0] & 0x0F0F0F0Fu) | ((A[1] & 0x0F0F0F0Fu) << 4);
            O[j] = ((A[0] >> 4) & 0x0F0F0F0Fu) | (A[1] & 0xF0F0F0F0u);
        }
        transpose_bytes(E);
        transpose_bytes(O);
        if (uok) {
            const uint32_t q0 = qy * ntx + 4 * wx;
            *(uint4 *)(lds + (2 * sy) * nq + q0) = make_uint4(E[0], E[1], E[2], E[3]);
            *(uint4 *)(lds + (2 * sy + 1) * nq + q0) = make_uint4(O[0], O[1], O[2], O[3]);
        }
    }

    if constexpr (DT) {
        // halo column: sigma_x(gx0 - 1, y) of the block's rows, at the bits of
        // the sx = 1 cells' right-hand sites (2 + 4 ry) of tile j = byte j
        const uint32_t xh = gx0 == 0 ? a.L - 1 : gx0 - 1;
        const uint32_t hw = xh >> 4, hbit = 2u * (xh & 15u);
        for (uint32_t e = tid; e < 2 * a.H; e += TPB) {
            const uint32_t sy = e / a.H, qy = e - sy * a.H;
            uint32_t v = 0;
            for (uint32_t j = 0; j < 4; ++j)
                for (uint32_t ry = 0; ry < 2; ++ry) {
                    uint32_t gy = gy0 + 4 * (qy + j * a.H) + 2 * sy + ry;
                    if (gy >= a.L) gy -= a.L;
                    const uint32_t bit = (a.src[(size_t)gy * a.W + hw] >> hbit) & 1u;
                    v |= bit << (8 * j + 2 + 4 * ry);
                }
            lds[4 * nq + e] = v;
        }
        // halo row: sigma_y(x, gy0 - 1) of the block's columns, at the bits of
        // the sy = 1 cells' upper sites (5 + 2 rx)
        const uint32_t yh = gy0 == 0 ? a.L - 1 : gy0 - 1;
        const uint32_t *hrowp = a.src + (size_t)yh * a.W;
        for (uint32_t e = tid; e < 2 * ntx; e += TPB) {
            const uint32_t sx = e / ntx, tx = e - sx * ntx;
            uint32_t v = 0;
            for (uint32_t rx = 0; rx < 2; ++rx) {
                uint32_t x = gx0 + 4 * tx + 2 * sx + rx;
                if (x >= a.L) x -= a.L;
                v |= ((hrowp[x >> 4] >> (2u * (x & 15u) + 1u)) & 1u) << (5 + 2 * rx);
            }
            lds[4 * nq + 2 * a.H + e] = v;
        }
    }

    // ---- site draws of this MCS for this thread's quads
    const uint64_t Gbase = (uint64_t)b * nq;
    uint32_t sw[K][4];
    uint32_t aw[K][4];
#pragma unroll
    for (int i = 0; i < K; ++i) {
        const uint64_t G = Gbase + tid + (uint32_t)TPB * i;
        const U4 s4 = philox((uint32_t)G, (uint32_t)(G >> 32), a.t, (TAG_SITE << 24) | a.res,
                             a.seed_lo, a.seed_hi);
        sw[i][0] = s4.x;
        sw[i][1] = s4.y;
        sw[i][2] = s4.z;
        sw[i][3] = s4.w;
        aw[i][0] = aw[i][1] = aw[i][2] = aw[i][3] = 0u;
    }
    const uint32_t setw = philox(b, 0u, a.t, (TAG_SET << 24) | a.res, a.seed_lo, a.seed_hi).x;
    // steps of this residency: [k0, k1) of the MCS's 16
    const uint32_t k0 = a.res * a.nsteps, k1 = k0 + a.nsteps;
    AccCtx ac;
    ac.fullP = a.P >= (1ull << 32);
    ac.tP = ac.fullP ? 256u : (uint32_t)(a.P >> 24);
    ac.tQ = (uint32_t)(a.Q >> 24);
    ac.lowP = (uint32_t)(a.P & 0xFFFFFFu);
    ac.lowQ = (uint32_t)(a.Q & 0xFFFFFFu);
    ac.ties = (!ac.fullP && ac.lowP != 0) || ac.lowQ != 0;
    const bool active = K * TPB == (int)nq || tid < nq;
    int net = 0;

    __syncthreads();

    // ---- work-group layer: single-hit steps k = 4 kq + kr in [k0, k1)
    // (all 16 when the origin moves once per MCS); the step range is the
    // same for the whole block, so skipping steps never splits a barrier
    for (int kq = 0; kq < 4; ++kq) {
        if (ACC && 4u * kq + 3u >= k0 && 4u * kq < k1) {
#pragma unroll
            for (int i = 0; i < K; ++i) {
                const uint64_t G = Gbase + tid + (uint32_t)TPB * i;
                const U4 w1 = philox((uint32_t)G, (uint32_t)(G >> 32), a.t,
                                     (TAG_ACC1 << 24) | (4u * a.res + (uint32_t)kq), a.seed_lo,
                                     a.seed_hi);
                aw[i][0] = w1.x;
                aw[i][1] = w1.y;
                aw[i][2] = w1.z;
                aw[i][3] = w1.w;
            }
        }
        for (uint32_t kr = 0; kr < 4; ++kr) {
            const uint32_t k = 4u * kq + kr;
            const uint32_t s = (setw >> (2 * k)) & 3u;
            if (k >= k0 && k < k1) {
                if (active) {
                    switch (s) {
                    case 0: step_quads<TPB, K, NTX, 0, 0, ACC, DT>(lds, tid, kr, sw, aw, ac, Gbase, k, a, net); break;
                    case 1: step_quads<TPB, K, NTX, 1, 0, ACC, DT>(lds, tid, kr, sw, aw, ac, Gbase, k, a, net); break;
                    case 2: step_quads<TPB, K, NTX, 0, 1, ACC, DT>(lds, tid, kr, sw, aw, ac, Gbase, k, a, net); break;
                    default: step_quads<TPB, K, NTX, 1, 1, ACC, DT>(lds, tid, kr, sw, aw, ac, Gbase, k, a, net); break;
                    }
                }
                __syncthreads();
            }
            if (ACC) {
#pragma unroll
                for (int i = 0; i < K; ++i) {
                    aw[i][0] = aw[i][1];
                    aw[i][1] = aw[i][2];
                    aw[i][2] = aw[i][3];
                }
            }
        }
#pragma unroll
        for (int i = 0; i < K; ++i) {
            sw[i][0] = sw[i][1];
            sw[i][1] = sw[i][2];
            sw[i][2] = sw[i][3];
        }
    }

    // ---- store: quads -> cells -> aligned block words -> HBM row words.
    // Two-buffer mode: the block's words are whole output words (the output
    // is rotated by the origin), stored as they are.  In place: words wholly
    // inside the block are stored; the block's parts of the two words it
    // shares with its left and right neighbours go to the side buffer and
    // are merged by a separate launch (the kernel boundary makes both parts
    // visible; a release/acquire between work-groups inside the launch would
    // write back the whole L2 per block).
    for (int it = 0; it < UIT; ++it) {
        const uint32_t u = tid + (uint32_t)TPB * it;
        const bool uok = u < a.units;
        const uint32_t wx = u & (nw - 1);
        const uint32_t rest = u >> a.log2nw;
        const uint32_t qy = rest & (a.H - 1);
        const uint32_t sy = rest >> a.log2H;
        const uint32_t q0 = qy * ntx + 4 * wx;
        uint32_t E[4] = {0u, 0u, 0u, 0u}, O[4] = {0u, 0u, 0u, 0u};
        if (uok) {
            const uint4 e = *(const uint4 *)(lds + (2 * sy) * nq + q0);
            const uint4 o = *(const uint4 *)(lds + (2 * sy + 1) * nq + q0);
            E[0] = e.x; E[1] = e.y; E[2] = e.z; E[3] = e.w;
            O[0] = o.x; O[1] = o.y; O[2] = o.z; O[3] = o.w;
        }
        transpose_bytes(E);
        transpose_bytes(O);
        uint32_t gw = (a.db ? gwo : gw0) + wx;
        if (gw >= a.W) gw -= a.W;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint32_t r0 = 4 * (qy + j * a.H) + 2 * sy;
            uint32_t A[2];
            A[0] = (E[j] & 0x0F0F0F0Fu) | ((O[j] & 0x0F0F0F0Fu) << 4);
            A[1] = ((E[j] >> 4) & 0x0F0F0F0Fu) | (O[j] & 0xF0F0F0F0u);
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                uint32_t gy = gy0 + r0 + h;
                if (gy >= a.L) gy -= a.L;
                uint32_t *row = a.words + (size_t)gy * a.W;
                if (a.db) {
                    if (uok) row[gw] = A[h];
                    continue;
                }
                const uint32_t prev = __shfl_up(A[h], 1, 64);
                if (!uok) continue;
                if (sh2 == 0) {
                    row[gw] = A[h];
                } else if (DT) {
                    // the neighbours sharing the end words are idle (blocks of
                    // one set are not adjacent): merge in place
                    const uint32_t lowm = (1u << sh2) - 1u;
                    if (wx > 0) row[gw] = __builtin_amdgcn_alignbit(A[h], prev, 32u - sh2);
                    else row[gw] = (row[gw] & lowm) | (A[h] << sh2);
                    if (wx == nw - 1) {
                        const uint32_t gwn = gw + 1 == a.W ? 0u : gw + 1;
                        row[gwn] = (row[gwn] & ~lowm) | (A[h] >> (32u - sh2));
                    }
                } else {
                    if (wx > 0) row[gw] = __builtin_amdgcn_alignbit(A[h], prev, 32u - sh2);
                    else a.side[(size_t)gy * a.nbx + bx] = A[h] << sh2;
                    if (wx == nw - 1)
                        a.side[((size_t)a.L + gy) * a.nbx + bx] = A[h] >> (32u - sh2);
                }
            }
        }
    }

    if constexpr (DT) {
        // ---- halo write-back, after this block's own words (one of which
        // may hold the halo column's bit)
        __syncthreads();
        const uint32_t xh = gx0 == 0 ? a.L - 1 : gx0 - 1;
        const uint32_t hw = xh >> 4, hbit = 2u * (xh & 15u);
        for (uint32_t e = tid; e < a.By; e += TPB) {
            const uint32_t ty = e >> 2, sy = (e >> 1) & 1u, ry = e & 1u;
            const uint32_t j = ty / a.H, qy = ty - j * a.H;
            const uint32_t bit = (lds[4 * nq + sy * a.H + qy] >> (8 * j + 2 + 4 * ry)) & 1u;
            uint32_t gy = gy0 + e;
            if (gy >= a.L) gy -= a.L;
            uint32_t *wp = a.words + (size_t)gy * a.W + hw;
            const uint32_t w0 = *wp;
            const uint32_t w1 = (w0 & ~(1u << hbit)) | (bit << hbit);
            if (w1 != w0) *wp = w1;
        }
        const uint32_t yh = gy0 == 0 ? a.L - 1 : gy0 - 1;
        uint32_t *hrowp = a.words + (size_t)yh * a.W;
        const uint32_t nwr = nw + (sh2 ? 1u : 0u);      // words holding the block's columns
        for (uint32_t m = tid; m < nwr; m += TPB) {
            uint32_t gwm = gw0 + m;
            if (gwm >= a.W) gwm -= a.W;
            uint32_t val = 0, mask = 0;
            for (uint32_t i = 0; i < 16; ++i) {
                uint32_t e = 16 * gwm + i + (a.L - gx0);
                if (e >= a.L) e -= a.L;
                if (e >= a.Bx) continue;
                const uint32_t tx = e >> 2, sx = (e >> 1) & 1u, rx = e & 1u;
                const uint32_t bit = (lds[4 * nq + 2 * a.H + sx * ntx + tx] >> (5 + 2 * rx)) & 1u;
                val |= bit << (2 * i + 1);
                mask |= 1u << (2 * i + 1);
            }
            const uint32_t w0 = hrowp[gwm];
            const uint32_t w1 = (w0 & ~mask) | val;
            if (w1 != w0) hrowp[gwm] = w1;
        }
    }

    // ---- flip counter of this block: wave sums, one atomic per wave
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) net += __shfl_xor(net, off, 64);
    if ((tid & 63u) == 0 && net != 0)
        atomicAdd(a.slots + ((b * (TPB / 64) + tid / 64) & a.slot_mask),
                  (unsigned long long)(long long)net);
}

template <int TPB, int K, int NTX, bool ACC>
__global__ __launch_bounds__(TPB) void kpz_sweep_kernel(const SweepArgs a)
{
    extern __shared__ uint32_t lds[];
    // Work-groups are dealt to the 8 XCDs round-robin (group i to XCD i mod
    // 8); with xcd set, group i takes block (i mod 8) n/8 + i/8, so each XCD
    // runs one contiguous range of blocks and neighbouring blocks, which
    // share cache lines at their edges, meet in the same L2.
    uint32_t b = blockIdx.x;
    if (a.xcd) b = (b & 7u) * (gridDim.x >> 3) + (b >> 3);
    sweep_block<TPB, K, NTX, ACC>(a, b, lds);
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
    const U4 wo = philox(a.res, 0u, a.t, TAG_ORIGIN << 24, a.seed_lo, a.seed_hi);
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
// every launch updates the lattice in place with no merge.  The block runs
// in the SWAR kernel above (sweep_block with DT), the left and lower
// neighbours' slopes as halos.

constexpr uint32_t TAG_DTORDER = 13;

// Block set (bx mod 2 + 2 (by mod 2)) of position `phase` in MCS t: the
// ordering floor(w0 24 / 2^32) of (DTORDER, t), orderings of 0..3 numbered
// lexicographically.
__device__ __forceinline__ uint32_t dt_set(uint32_t t, uint32_t seed_lo, uint32_t seed_hi,
                                           uint32_t phase)
{
    uint32_t idx = (uint32_t)(((uint64_t)philox(0u, 0u, t, TAG_DTORDER << 24, seed_lo,
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

// The same schedule with the SWAR block kernel: one launch per block set; the
// blocks of set c are (2 i + (c & 1), 2 j + (c >> 1)).  LDS: the block's four
// cell planes plus the halo column (2 H words) and row (2 ntx words).
template <int TPB, int K, int NTX, bool ACC>
__global__ __launch_bounds__(TPB) void kpz_dt_swar_kernel(const SweepArgs a, uint32_t phase)
{
    extern __shared__ uint32_t lds[];
    uint32_t g = blockIdx.x;
    if ((gridDim.x & 7u) == 0) g = (g & 7u) * (gridDim.x >> 3) + (g >> 3);
    const uint32_t c = dt_set(a.t, a.seed_lo, a.seed_hi, phase);
    const uint32_t hx = a.nbx >> 1;
    const uint32_t bx = 2 * (g % hx) + (c & 1u), by = 2 * (g / hx) + (c >> 1);
    sweep_block<TPB, K, NTX, ACC, true>(a, by * a.nbx + bx, lds);
}


// ------------------------------------------------------------ roughness

// Per row y: with P(x) = sum_{l<x} sigma_x(l,y) (height relative to the row
// start), A_y = sum_x P(x) and B_y = sum_x P(x)^2, a group of lanes per row.
//
// A word's 16 sigma_x bits are compacted into two bytes of 8 sites; a
// 256-entry LDS table gives, for 8 sites with local prefix p_k (k = 0..7),
// d = p_8, a = sum p_k and c = sum p_k^2.  Each lane takes four consecutive
// words (one 16-byte load); one wave scan per 256 words places the lanes.
__device__ __forceinline__ uint32_t lut8_entry(uint32_t byte)
{
    int p = 0, a = 0, c = 0;
    for (int i = 0; i < 8; ++i) {
        a += p;
        c += p * p;
        p += ((byte >> i) & 1u) ? 1 : -1;
    }
    // two's complement d (-8..8) in bits 0..4 and a (-28..28) in bits 5..11,
    // c (0..140) in bits 12..19: one signed or unsigned field extract each
    return ((uint32_t)p & 31u) | (((uint32_t)a & 127u) << 5) | ((uint32_t)c << 12);
}

struct WordSums {
    int d, s1, s2;   // increment, sum of prefixes, sum of squared prefixes (16 sites)
};

__device__ __forceinline__ WordSums word_sums(uint32_t w, const uint32_t *lut)
{
    uint32_t x = w & 0x55555555u;              // sigma_x of site i at bit 2i
    x = (x | (x >> 1)) & 0x33333333u;
    x = (x | (x >> 2)) & 0x0F0F0F0Fu;
    x = (x | (x >> 4)) & 0x00FF00FFu;          // sites 0..7 in byte 0, 8..15 in byte 2
    const uint32_t e0 = lut[x & 0xFFu], e1 = lut[(x >> 16) & 0xFFu];
    const int d0 = (int)(e0 << 27) >> 27, a0 = (int)(e0 << 20) >> 25, c0 = (int)(e0 >> 12);
    const int d1 = (int)(e1 << 27) >> 27, a1 = (int)(e1 << 20) >> 25, c1 = (int)(e1 >> 12);
    WordSums r;
    r.d = d0 + d1;
    r.s1 = a0 + 8 * d0 + a1;
    r.s2 = c0 + 8 * d0 * d0 + 2 * d0 * a1 + c1;
    return r;
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

// Moments of one row, taken by a group of G lanes (G = row_lanes(W), the
// group's lanes gl = 0..G-1 aligned to G in the wave), NV consecutive words
// per lane and chunk (NV = 16 only for W % 1024 == 0, where G = 64 and every
// lane is full): returns (A_y, B_y) in lane gl = 0 and, in `first`, the
// row's first word in the documented layout.  rot2 = twice the storage
// rotation (a row stored rotated by s sites holds sites s.. in its word 0;
// word w of the layout is then bits of stored words w - 1 and w).  A lane's
// local sums stay below 2^24 and heights within a row below L, so they are
// 32-bit; only the row totals are 64-bit.
template <int NV>
__device__ __forceinline__ void row_moments(const uint32_t *rp, uint32_t W, const uint32_t *lut,
                                            uint32_t gl, uint32_t G, uint32_t rot2, long long &A,
                                            long long &B, uint32_t &first)
{
    static_assert(NV == 4 || NV == 16, "four or sixteen words per lane");
    const bool vec = (W & 3u) == 0;
    long long s1 = 0, s2 = 0;
    int carry = 0;
    uint32_t carry_w = rot2 ? rp[W - 1] : 0u;   // stored word before word 0 (periodic row)
    first = 0u;
    for (uint32_t base = 0; base < W; base += NV * G) {
        const uint32_t idx = base + NV * gl;
        uint32_t v[NV];
        int nv = 0;
        if (NV == 16) {
#pragma unroll
            for (int j = 0; j < NV / 4; ++j) {
                const uint4 q = *(const uint4 *)(rp + idx + 4 * j);
                v[4 * j] = q.x; v[4 * j + 1] = q.y; v[4 * j + 2] = q.z; v[4 * j + 3] = q.w;
            }
            nv = NV;
        } else {
#pragma unroll
            for (int m = 0; m < NV; ++m) v[m] = 0u;
            if (vec) {
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
        if (rot2) {
            // the previous stored word of each lane's first word: the previous
            // lane's last (full lanes precede any lane with words), or the
            // carried word for the group's lane 0
            uint32_t pv = __shfl(v[NV - 1], (gl + G - 1u) & (G - 1u), G);
            if (gl == 0) pv = carry_w;
            carry_w = __shfl(v[NV - 1], G - 1u, G);
#pragma unroll
            for (int m = NV - 1; m > 0; --m)
                v[m] = __builtin_amdgcn_alignbit(v[m], v[m - 1], 32u - rot2);
            v[0] = __builtin_amdgcn_alignbit(v[0], pv, 32u - rot2);
        }
        if (base == 0) first = v[0];
        // this lane's words relative to its own start
        int o = 0, l1 = 0, l2 = 0;
#pragma unroll
        for (int m = 0; m < NV; ++m) {
            if (NV == 16 || m < nv) {
                const WordSums ws = word_sums(v[m], lut);
                l1 += 16 * o + ws.s1;
                l2 += 16 * o * o + 2 * o * ws.s1 + ws.s2;
                o += ws.d;
            }
        }
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

// One wave per 64 / row_lanes(W) rows.
__global__ __launch_bounds__(256) void kpz_row_moments_kernel(const uint32_t *words, uint32_t L,
                                                              uint32_t W, long long *rowA,
                                                              long long *rowB, const Rot rot)
{
    __shared__ uint32_t lut[256];
    lut[threadIdx.x] = lut8_entry(threadIdx.x);
    __syncthreads();
    const uint32_t rot2 = 2u * rot_sites(rot);
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t G = row_lanes(W), R = 64u / G;
    const uint32_t gl = lane & (G - 1u);
    const uint32_t tasks = (L + R - 1u) / R;
    for (uint32_t task = blockIdx.x * 4u + wv; task < tasks; task += gridDim.x * 4u) {
        const uint32_t row = task * R + lane / G;
        if (row < L) {   // a whole lane group is in or out
            long long A, B;
            uint32_t first;
            if ((W & 1023u) == 0)
                row_moments<16>(words + (size_t)row * W, W, lut, gl, G, rot2, A, B, first);
            else
                row_moments<4>(words + (size_t)row * W, W, lut, gl, G, rot2, A, B, first);
            if (gl == 0) {
                rowA[row] = A;
                rowB[row] = (B << 1) | ((first >> 1) & 1u);   // + sigma_y(0, row)
            }
        }
    }
}

// A lattice buffer in the documented layout from one stored rotated by
// rot_sites(rot) (src != dst).
__global__ void kpz_rotate_kernel(const uint32_t *src, uint32_t *dst, uint32_t L, uint32_t W,
                                  const Rot rot)
{
    const uint32_t rot2 = 2u * rot_sites(rot);
    const uint64_t n = (uint64_t)L * W;
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t w = (uint32_t)(i % W);
        const uint64_t pi = w ? i - 1 : i + W - 1;
        dst[i] = rot2 ? __builtin_amdgcn_alignbit(src[i], src[pi], 32u - rot2) : src[i];
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
                                                 uint32_t nslots, long long *res)
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
        const unsigned __int128 u2 = (unsigned __int128)r2s[0];
        res[0] = r1s[0];
        res[1] = (long long)(uint64_t)u2;
        res[2] = (long long)(uint64_t)(u2 >> 64);
        res[3] = ns[0];
    }
}

__global__ __launch_bounds__(1024) void kpz_finalize_kernel(uint32_t L, const long long *rowA,
                                                            const long long *rowB,
                                                            const long long *slots,
                                                            long long *res)
{
    finalize_moments<1024>(L, rowA, rowB, slots, NSLOTS, res);
}

// Lattices of at most SMALL_ROWS rows: the row pass and the finalize in one
// work-group, the row sums in LDS (one launch per sample instead of two).
constexpr uint32_t SMALL_ROWS = 1024;

// Row sums of a lattice of L <= SMALL_ROWS rows by the 16 waves of one
// work-group of 1024 threads, into rA / rB (LDS); `lut` filled.
__device__ __forceinline__ void small_rows(const uint32_t *words, uint32_t L, uint32_t W,
                                           uint32_t rot2, const uint32_t *lut, long long *rA,
                                           long long *rB)
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
            row_moments<4>(words + (size_t)row * W, W, lut, gl, G, rot2, A, B, first);
            if (gl == 0) {
                rA[row] = A;
                rB[row] = (B << 1) | ((first >> 1) & 1u);   // + sigma_y(0, row)
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
    if (threadIdx.x < 256) lut[threadIdx.x] = lut8_entry(threadIdx.x);
    __syncthreads();
    small_rows(words, L, W, 2u * rot_sites(rot), lut, rA, rB);
    __syncthreads();
    finalize_moments<1024>(L, rA, rB, slots, NSLOTS, res);
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
// t_r + k (t_r = the member's t at the start of the call).  Block g of the
// grid is block g - bprefix[r] of member r (bprefix = prefix sums of the
// members' block counts).
template <int TPB, int K, int NTX>
__global__ __launch_bounds__(TPB) void kpz_batch_round_kernel(const SweepArgs *members,
                                                              const uint32_t *bprefix,
                                                              uint32_t nmem, uint32_t k,
                                                              uint32_t res)
{
    extern __shared__ uint32_t lds[];
    // XCD-aware order (the grid is padded to a multiple of 8): group i takes
    // block (i mod 8) n/8 + i/8 of the concatenated members
    const uint32_t g = (blockIdx.x & 7u) * (gridDim.x >> 3) + (blockIdx.x >> 3);
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
    if (a.acc) sweep_block<TPB, K, NTX, true>(a, b, lds);
    else sweep_block<TPB, K, NTX, false>(a, b, lds);
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
        const uint32_t rot2 = 2u * rot_sites(rot);
        const uint32_t *src = cur + (size_t)row * m.W;
        for (uint32_t w = threadIdx.x; w < m.W; w += blockDim.x) rowbuf[w] = src[w];
        __syncthreads();
        uint32_t *dst = (m.state ? m.state->words : (uint32_t *)m.words) + (size_t)row * m.W;
        for (uint32_t w = threadIdx.x; w < m.W; w += blockDim.x) {
            const uint32_t pv = rowbuf[w ? w - 1 : m.W - 1];
            dst[w] = rot2 ? __builtin_amdgcn_alignbit(rowbuf[w], pv, 32u - rot2) : rowbuf[w];
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
    __shared__ uint32_t lut[256];
    lut[threadIdx.x] = lut8_entry(threadIdx.x);
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
            if ((m.W & 1023u) == 0)
                row_moments<16>(rp, m.W, lut, lane & (G - 1u), G, 2u * rot_sites(rot), A, B, first);
            else
                row_moments<4>(rp, m.W, lut, lane & (G - 1u), G, 2u * rot_sites(rot), A, B, first);
            if ((lane & (G - 1u)) == 0) {
                m.rowA[row] = A;
                m.rowB[row] = (B << 1) | ((first >> 1) & 1u);   // + sigma_y(0, row)
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
    if (threadIdx.x < 256) lut[threadIdx.x] = lut8_entry(threadIdx.x);
    __syncthreads();
    const uint32_t r = blockIdx.x;
    const MemberRows m = mr[r];
    Rot rot;
    const uint32_t *cur = member_current(m, rot);
    small_rows(cur, m.L, m.W, 2u * rot_sites(rot), lut, rA, rB);
    __syncthreads();
    finalize_moments<1024>(m.L, rA, rB, m.slots, nslots, res + ((size_t)k * n + r) * 4);
}

// One work-group per member; results of sample `k` go to res[(k n + r) 4 ..].
__global__ __launch_bounds__(256) void kpz_batch_finalize_kernel(const MemberRows *mr, uint32_t n,
                                                                 uint32_t nslots, long long *res,
                                                                 uint32_t k)
{
    const uint32_t r = blockIdx.x;
    const MemberRows m = mr[r];
    finalize_moments<256>(m.L, m.rowA, m.rowB, m.slots, nslots, res + ((size_t)k * n + r) * 4);
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

// Resolves defaults and validates; fills block shape.
kpz_status resolve(const kpz_params *p, uint32_t *Bx, uint32_t *By)
{
    if (!p) return KPZ_EINVAL;
    if (p->L < 16 || (p->L % 16) != 0) return KPZ_EINVAL;
    if (!(p->p >= 0.0 && p->p <= 1.0 && p->q >= 0.0 && p->q <= 1.0)) return KPZ_EINVAL;
    if ((p->flags & ~(KPZ_FLAG_IN_PLACE | KPZ_FLAG_DEVICE_DT)) != 0) return KPZ_EINVAL;
    if (p->moves != 0 && p->moves != 1 && p->moves != 2 && p->moves != 4 && p->moves != 8 &&
        p->moves != 16)
        return KPZ_EINVAL;
    const int tx = p->tile_x ? p->tile_x : TILE, ty = p->tile_y ? p->tile_y : TILE;
    if (tx != TILE || ty != TILE) return KPZ_EINVAL;
    const int64_t L = p->L;
    // default: the largest power of two <= 256 that divides L (L % 16 == 0)
    int64_t dflt = 256;
    while (L % dflt) dflt >>= 1;
    const int64_t bx = p->block_x ? p->block_x : dflt;
    const int64_t by = p->block_y ? p->block_y : dflt;
    if (!is_pow2(bx) || !is_pow2(by)) return KPZ_EINVAL;
    if (bx < 16 || by < 16 || bx > 1024 || bx * by > 65536) return KPZ_EINVAL;
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

template <int TPB, int K, int NTX, bool ACC>
hipError_t launch_sweep_k(const SweepArgs &a, uint32_t nblocks, size_t shmem, hipStream_t st)
{
    hipLaunchKernelGGL((kpz_sweep_kernel<TPB, K, NTX, ACC>), dim3(nblocks), dim3(TPB), shmem, st, a);
    return hipGetLastError();
}

// Shape-specialised kernels for the tile-column counts of the common block
// widths (256, 512, 1024 sites); every other width runs the runtime-width
// kernel (NTX = 0).
template <int TPB, int K, bool ACC>
hipError_t launch_sweep_ntx(const SweepArgs &a, uint32_t nblocks, size_t shmem, hipStream_t st)
{
    switch (a.ntx) {
    case 64: return launch_sweep_k<TPB, K, 64, ACC>(a, nblocks, shmem, st);
    case 128: return launch_sweep_k<TPB, K, 128, ACC>(a, nblocks, shmem, st);
    case 256: return launch_sweep_k<TPB, K, 256, ACC>(a, nblocks, shmem, st);
    default: return launch_sweep_k<TPB, K, 0, ACC>(a, nblocks, shmem, st);
    }
}

template <int TPB, int K, int NTX, bool ACC>
hipError_t launch_dt_k(const SweepArgs &a, uint32_t phase, uint32_t nblocks, size_t shmem,
                       hipStream_t st)
{
    hipLaunchKernelGGL((kpz_dt_swar_kernel<TPB, K, NTX, ACC>), dim3(nblocks), dim3(TPB), shmem, st,
                       a, phase);
    return hipGetLastError();
}

template <int TPB, int K, bool ACC>
hipError_t launch_dt_ntx(const SweepArgs &a, uint32_t phase, uint32_t nblocks, size_t shmem,
                         hipStream_t st)
{
    switch (a.ntx) {
    case 64: return launch_dt_k<TPB, K, 64, ACC>(a, phase, nblocks, shmem, st);
    case 128: return launch_dt_k<TPB, K, 128, ACC>(a, phase, nblocks, shmem, st);
    case 256: return launch_dt_k<TPB, K, 256, ACC>(a, phase, nblocks, shmem, st);
    default: return launch_dt_k<TPB, K, 0, ACC>(a, phase, nblocks, shmem, st);
    }
}

template <bool ACC>
hipError_t launch_dt(const SweepArgs &a, uint32_t phase, uint32_t tpb, uint32_t K,
                     uint32_t nblocks, size_t shmem, hipStream_t st)
{
    if (tpb == 256) {
        switch (K) {
        case 1: return launch_dt_ntx<256, 1, ACC>(a, phase, nblocks, shmem, st);
        case 2: return launch_dt_ntx<256, 2, ACC>(a, phase, nblocks, shmem, st);
        case 4: return launch_dt_ntx<256, 4, ACC>(a, phase, nblocks, shmem, st);
        default: return hipErrorInvalidValue;
        }
    }
    switch (K) {
    case 1: return launch_dt_ntx<64, 1, ACC>(a, phase, nblocks, shmem, st);
    case 2: return launch_dt_ntx<64, 2, ACC>(a, phase, nblocks, shmem, st);
    case 4: return launch_dt_ntx<64, 4, ACC>(a, phase, nblocks, shmem, st);
    case 8: return launch_dt_ntx<64, 8, ACC>(a, phase, nblocks, shmem, st);
    case 16: return launch_dt_ntx<64, 16, ACC>(a, phase, nblocks, shmem, st);
    default: return hipErrorInvalidValue;
    }
}

// tpb threads per block, K = nq / tpb quads per thread (K = 1 with idle
// lanes for blocks of fewer than 64 quads).
template <bool ACC>
hipError_t launch_sweep(const SweepArgs &a, uint32_t tpb, uint32_t K, uint32_t nblocks,
                        size_t shmem, hipStream_t st)
{
    if (tpb == 256) {
        switch (K) {
        case 1: return launch_sweep_ntx<256, 1, ACC>(a, nblocks, shmem, st);
        case 2: return launch_sweep_ntx<256, 2, ACC>(a, nblocks, shmem, st);
        case 4: return launch_sweep_ntx<256, 4, ACC>(a, nblocks, shmem, st);
        default: return hipErrorInvalidValue;
        }
    }
    switch (K) {
    case 1: return launch_sweep_ntx<64, 1, ACC>(a, nblocks, shmem, st);
    case 2: return launch_sweep_ntx<64, 2, ACC>(a, nblocks, shmem, st);
    case 4: return launch_sweep_ntx<64, 4, ACC>(a, nblocks, shmem, st);
    case 8: return launch_sweep_ntx<64, 8, ACC>(a, nblocks, shmem, st);
    case 16: return launch_sweep_ntx<64, 16, ACC>(a, nblocks, shmem, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace


// ------------------------------------------------------------ ensemble host

namespace {

constexpr int BATCH_SLOTS = 64;   // flip-counter slots per member

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

struct BatchLayout {
    uint32_t Bx, By;
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
    int64_t Lmin = INT64_MAX;
    for (int32_t r = 0; r < n; ++r) Lmin = m[r].L < Lmin ? m[r].L : Lmin;
    if (Lmin < 16 || Lmin % 16) return KPZ_EINVAL;
    int64_t dflt = 256;
    while (Lmin % dflt) dflt >>= 1;
    int64_t bx = -1, by = -1;
    for (int32_t r = 0; r < n; ++r)
        if (moves_of(&m[r]) != moves_of(&m[0])) return KPZ_EINVAL;
    lay->moves = moves_of(&m[0]);
    for (int32_t r = 0; r < n; ++r) {
        kpz_params q = m[r];
        if (!q.block_x) q.block_x = (int32_t)dflt;
        if (!q.block_y) q.block_y = (int32_t)dflt;
        uint32_t rbx, rby;
        const kpz_status st = resolve(&q, &rbx, &rby);
        if (st != KPZ_OK) return st;
        if (bx < 0) { bx = rbx; by = rby; }
        if ((int64_t)rbx != bx || (int64_t)rby != by) return KPZ_EINVAL;
    }
    lay->Bx = (uint32_t)bx;
    lay->By = (uint32_t)by;
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
        lay->off_side[r] = o; o = align256(o + 4 * 2 * L * (L / lay->Bx));
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

// Kernel shape shared by every member of an ensemble or pool.
struct RoundShape {
    uint32_t tpb, K, ntx;
    size_t shmem;
};

bool round_shape(uint32_t Bx, uint32_t By, RoundShape *rs)
{
    rs->ntx = Bx / TILE;
    const uint32_t nq = rs->ntx * (By / 16);
    rs->tpb = nq >= 256 ? 256u : 64u;
    rs->K = nq <= rs->tpb ? 1u : nq / rs->tpb;
    rs->shmem = sizeof(uint32_t) * 4 * (size_t)nq;
    return (rs->tpb == 256 && rs->K <= 4) || (rs->tpb == 64 && rs->K <= 2);
}

// The ensemble's round kernel is specialised for the tile-column counts of
// block widths 64 to 1024 (the autotuner's candidates); others run the
// runtime-width kernel.
template <int TPB, int K>
void round_launch_k(const RoundShape &rs, uint32_t grid, hipStream_t st, const SweepArgs *members,
                    const uint32_t *bprefix, uint32_t nmem, uint32_t k, uint32_t res)
{
    switch (rs.ntx) {
    case 16:
        hipLaunchKernelGGL((kpz_batch_round_kernel<TPB, K, 16>), dim3(grid), dim3(TPB), rs.shmem,
                           st, members, bprefix, nmem, k, res);
        break;
    case 32:
        hipLaunchKernelGGL((kpz_batch_round_kernel<TPB, K, 32>), dim3(grid), dim3(TPB), rs.shmem,
                           st, members, bprefix, nmem, k, res);
        break;
    case 64:
        hipLaunchKernelGGL((kpz_batch_round_kernel<TPB, K, 64>), dim3(grid), dim3(TPB), rs.shmem,
                           st, members, bprefix, nmem, k, res);
        break;
    case 128:
        hipLaunchKernelGGL((kpz_batch_round_kernel<TPB, K, 128>), dim3(grid), dim3(TPB), rs.shmem,
                           st, members, bprefix, nmem, k, res);
        break;
    case 256:
        hipLaunchKernelGGL((kpz_batch_round_kernel<TPB, K, 256>), dim3(grid), dim3(TPB), rs.shmem,
                           st, members, bprefix, nmem, k, res);
        break;
    default:
        hipLaunchKernelGGL((kpz_batch_round_kernel<TPB, K, 0>), dim3(grid), dim3(TPB), rs.shmem,
                           st, members, bprefix, nmem, k, res);
        break;
    }
}

// One round (residency res of MCS k of the call) of members [0, nmem) plus
// the merge of their straddling words.  grid = bprefix[nmem], mwords =
// sprefix[nmem].
hipError_t round_launch(const RoundShape &rs, uint32_t nblocks, uint64_t mwords, hipStream_t st,
                        const SweepArgs *members, const uint32_t *bprefix,
                        const unsigned long long *sprefix, uint32_t nmem, uint32_t k,
                        uint32_t res, bool merge)
{
    const uint32_t grid = (nblocks + 7u) & ~7u;   // the kernel's XCD map needs a multiple of 8
    if (rs.tpb == 256) {
        if (rs.K == 1) round_launch_k<256, 1>(rs, grid, st, members, bprefix, nmem, k, res);
        else if (rs.K == 2) round_launch_k<256, 2>(rs, grid, st, members, bprefix, nmem, k, res);
        else round_launch_k<256, 4>(rs, grid, st, members, bprefix, nmem, k, res);
    } else {
        if (rs.K == 1) round_launch_k<64, 1>(rs, grid, st, members, bprefix, nmem, k, res);
        else round_launch_k<64, 2>(rs, grid, st, members, bprefix, nmem, k, res);
    }
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
    RoundShape rs;
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
            const hipError_t e = round_launch(b->rs, b->per_round, b->merge_words, st,
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
    uint32_t Bx, By;
    RoundShape rs;
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
    a.L = L;
    a.W = L / 16;
    a.Bx = p->Bx;
    a.By = p->By;
    a.nbx = L / p->Bx;
    a.nby = L / p->By;
    a.ntx = p->Bx / TILE;
    a.log2ntx = (uint32_t)ilog2(a.ntx);
    a.H = p->By / 16;
    a.log2H = (uint32_t)ilog2(a.H);
    a.nq = a.ntx * a.H;
    a.nw = p->Bx / 16;
    a.log2nw = (uint32_t)ilog2(a.nw);
    a.units = a.nw * a.H * 2;
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

extern "C" {

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
    a.db = 0;
    a.prev_valid = a.prev_t = a.prev_res = 0;
    a.xcd = 0;
    a.side = ws_side(s);
    a.slots = (unsigned long long *)ws_slots(s);
    a.L = L;
    a.W = L / 16;
    a.Bx = s->Bx;
    a.By = s->By;
    a.nbx = L / s->Bx;
    a.nby = L / s->By;
    a.ntx = s->Bx / TILE;
    a.log2ntx = (uint32_t)ilog2(a.ntx);
    a.H = s->By / 16;
    a.log2H = (uint32_t)ilog2(a.H);
    a.nq = a.ntx * a.H;
    a.nw = s->Bx / 16;
    a.log2nw = (uint32_t)ilog2(a.nw);
    a.units = a.nw * a.H * 2;
    a.seed_lo = (uint32_t)s->prm.seed;
    a.seed_hi = (uint32_t)(s->prm.seed >> 32);
    a.P = s->P;
    a.Q = s->Q;
    a.slot_mask = NSLOTS - 1;
    a.acc = !(s->P == (1ull << 32) && s->Q == 0);
    const uint32_t moves = moves_of(&s->prm);
    a.nsteps = 16u / moves;
    // threads per block: four waves when the block has at least 256 quads
    // (fewer registers per lane, more waves to hide LDS and HBM latency);
    // KPZ_THREADS_PER_BLOCK=64 selects one wave per block.  The launch shape
    // does not change any result.
    uint32_t tpb = a.nq >= 256 ? 256u : 64u;
    if (const char *env = getenv("KPZ_THREADS_PER_BLOCK"))
        if (atoi(env) == 64) tpb = 64u;
    const uint32_t K = a.nq <= tpb ? 1u : a.nq / tpb;
    const uint32_t nblocks = a.nbx * a.nby;
    const size_t shmem = sizeof(uint32_t) * 4 * (size_t)a.nq;
    const uint64_t nstraddle = (uint64_t)L * a.nbx;
    const uint32_t mgrid = (uint32_t)((nstraddle + 255) / 256 < 8192 ? (nstraddle + 255) / 256 : 8192);
    a.xcd = (nblocks % 8u) == 0;
    if (s->dt) {
        // double tiling at the device layer: four launches per MCS, one per
        // block set in the order drawn for the MCS, in place
        const uint32_t grid = a.nbx * a.nby / 4;
        const size_t dshmem = shmem + sizeof(uint32_t) * (2 * (size_t)a.H + 2 * (size_t)a.ntx);
        a.res = 0;
        for (int32_t m = 0; m < n_mcs; ++m) {
            a.t = (uint32_t)(s->t + m);
            for (uint32_t ph = 0; ph < 4; ++ph) {
                const hipError_t e = a.acc ? launch_dt<true>(a, ph, tpb, K, grid, dshmem, s->stream)
                                           : launch_dt<false>(a, ph, tpb, K, grid, dshmem, s->stream);
                if (e != hipSuccess) return hip_fail(s, e, "kpz_sweep launch");
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
            hipError_t e = a.acc ? launch_sweep<true>(a, tpb, K, nblocks, shmem, s->stream)
                                 : launch_sweep<false>(a, tpb, K, nblocks, shmem, s->stream);
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
        const uint32_t nt = row_tasks(L);
        const uint32_t rgrid = (nt + 3) / 4 < 4096 ? (nt + 3) / 4 : 4096;
        hipLaunchKernelGGL(kpz_row_moments_kernel, dim3(rgrid), dim3(256), 0, s->stream,
                           s->buf[s->cur], L, W, ws_rowA(s), ws_rowB(s), sim_rot(s));
        e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(s, e, "kpz_roughness launch");
        hipLaunchKernelGGL(kpz_finalize_kernel, dim3(1), dim3(1024), 0, s->stream, L, ws_rowA(s),
                           ws_rowB(s), ws_slots(s), ws_res(s));
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
    if (!round_shape(lay.Bx, lay.By, &b->rs)) { delete b; return KPZ_EINVAL; }

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
        a.L = L;
        a.W = L / 16;
        a.Bx = lay.Bx;
        a.By = lay.By;
        a.nbx = L / lay.Bx;
        a.nby = L / lay.By;
        a.ntx = lay.Bx / TILE;
        a.log2ntx = (uint32_t)ilog2(a.ntx);
        a.H = lay.By / 16;
        a.log2H = (uint32_t)ilog2(a.H);
        a.nq = a.ntx * a.H;
        a.nw = lay.Bx / 16;
        a.log2nw = (uint32_t)ilog2(a.nw);
        a.units = a.nw * a.H * 2;
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
        rows[r].rot = Rot{0u, 0u, 0u, lay.Bx, 0u, 0u};
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
    if (!is_pow2(bx) || !is_pow2(by) || bx < 16 || by < 16 || bx > 1024 || (int64_t)bx * by > 65536)
        return KPZ_EINVAL;
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
    if (!round_shape(p->Bx, p->By, &p->rs)) {
        delete p;
        return KPZ_EINVAL;
    }
    if (arena_bytes > ctl.bytes) p->free_list[ctl.bytes] = arena_bytes - ctl.bytes;
    *out = p;
    return KPZ_OK;
}

kpz_status kpz_pool_submit(kpz_pool *p, const kpz_params *job, int64_t n_mcs, int64_t *id)
{
    clear_pending_error();
    if (!p || !job || n_mcs < 1 || n_mcs > 0xFFFFFFFFll) return KPZ_EINVAL;
    kpz_params q = *job;
    q.block_x = (int32_t)p->Bx;
    q.block_y = (int32_t)p->By;
    if ((job->block_x && job->block_x != (int32_t)p->Bx) ||
        (job->block_y && job->block_y != (int32_t)p->By))
        return KPZ_EINVAL;
    if (moves_of(job) != 1) return KPZ_EINVAL;
    uint32_t rbx, rby;
    kpz_status st = resolve(&q, &rbx, &rby);
    if (st != KPZ_OK) return st;
    const size_t bytes = pool_job_bytes_raw(q.L, p->Bx, p->By);
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
        e = round_launch(p->rs, bprefix[m], sprefix[m], p->stream, d_members, d_bprefix, d_sprefix,
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
            rows[f].rot = Rot{j.rot_valid, j.rot_t, j.rot_res, p->Bx, (uint32_t)j.prm.seed,
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

}  // extern "C"
