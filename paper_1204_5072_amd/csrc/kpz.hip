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
//                           heights, one wave per row, HBM read stream
//   kpz_finalize_kernel     column-0 prefix, 128-bit totals, flip counters
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

#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <new>

#include "kpz.h"

namespace {

constexpr uint32_t TAG_ORIGIN = 1, TAG_SET = 2, TAG_SITE = 3, TAG_ACC1 = 4, TAG_ACC2 = 5;
constexpr int NSLOTS = 1024;          // flip-counter slots in the workspace
constexpr int WS_HEADER = 256;        // results area at the start of the workspace
constexpr int TILE = 4;               // tile edge (sites)
constexpr int STEPS = TILE * TILE;    // single-hit steps per MCS

// ------------------------------------------------------------------ Philox

struct U4 {
    uint32_t x, y, z, w;
};

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
    uint32_t *words;
    unsigned long long *slots;   // NSLOTS flip counters
    uint32_t L, W;               // size, words per row
    uint32_t Bx, By;             // block shape
    uint32_t nbx, nby;           // blocks per direction
    uint32_t ntx, log2ntx;       // tiles per block row
    uint32_t H;                  // tile rows per quad row (nty / 4)
    uint32_t nq;                 // quads per plane
    uint32_t nw;                 // aligned words per block row (Bx / 16)
    uint32_t units;              // load/store units per block
    uint32_t seed_lo, seed_hi;
    uint32_t t;
    uint64_t P, Q;               // acceptance thresholds over 2^32
};

template <int K, bool ACC>
__global__ __launch_bounds__(64) void kpz_sweep_kernel(const SweepArgs a)
{
    extern __shared__ uint32_t lds[];
    const uint32_t lane = threadIdx.x;
    const uint32_t b = blockIdx.x;
    const uint32_t bx = b % a.nbx, by = b / a.nbx;
    const uint32_t nq = a.nq;

    // device layer: origin of this MCS, then this block's frame
    const U4 wo = philox(0u, 0u, a.t, TAG_ORIGIN << 24, a.seed_lo, a.seed_hi);
    const uint32_t ox = (uint32_t)(((uint64_t)wo.x * a.Bx) >> 32);
    const uint32_t oy = (uint32_t)(((uint64_t)wo.y * a.By) >> 32);
    uint32_t gx0 = ox + bx * a.Bx;
    if (gx0 >= a.L) gx0 -= a.L;
    uint32_t gy0 = oy + by * a.By;
    if (gy0 >= a.L) gy0 -= a.L;
    const uint32_t sh2 = 2u * (gx0 & 15u);
    const uint32_t gw0 = gx0 >> 4;

    uint32_t *edge = lds + 4 * nq;   // [2][By]: original first / last aligned word of each row

    // ---- load: HBM row words -> aligned block words -> cells -> quads
    for (uint32_t u = lane; u < a.units; u += 64) {
        const uint32_t wx = u % a.nw;
        const uint32_t rest = u / a.nw;
        const uint32_t qy = rest % a.H;
        const uint32_t sy = rest / a.H;
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
                const uint32_t *row = a.words + (size_t)gy * a.W;
                const uint32_t lo = row[gw];
                const uint32_t hi = sh2 ? row[gw1] : 0u;
                A[h] = __builtin_amdgcn_alignbit(hi, lo, sh2);
                if (wx == 0) edge[r0 + h] = A[h];
                if (wx == a.nw - 1) edge[a.By + r0 + h] = A[h];
            }
            E[j] = (A[0] & 0x0F0F0F0Fu) | ((A[1] & 0x0F0F0F0Fu) << 4);
            O[j] = ((A[0] >> 4) & 0x0F0F0F0Fu) | (A[1] & 0xF0F0F0F0u);
        }
        transpose_bytes(E);
        transpose_bytes(O);
        const uint32_t q0 = qy * a.ntx + 4 * wx;
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            lds[(2 * sy) * nq + q0 + m] = E[m];
            lds[(2 * sy + 1) * nq + q0 + m] = O[m];
        }
    }

    // ---- per-quad constants and random words of this MCS
    uint32_t own[K], lft[K], dwn[K], rl[K], dmx[K], dmy[K], sw[K][4];
    bool lok[K], valid[K];
#pragma unroll
    for (int i = 0; i < K; ++i) {
        const uint32_t q = lane + 64u * i;
        valid[i] = q < nq;
        const uint32_t qx = q & (a.ntx - 1), qy = q >> a.log2ntx;
        own[i] = q;
        // left neighbour quad for set sx = 0 (tile tx-1); wraps if one block per row
        lok[i] = qx > 0 || a.nbx == 1;
        lft[i] = qx > 0 ? q - 1 : (a.nbx == 1 ? q + a.ntx - 1 : q);
        // lower neighbour quad for set sy = 0 (tile ty-1): for qy = 0 it is the
        // last quad row, shifted by one byte
        dwn[i] = qy > 0 ? q - a.ntx : q + (a.H - 1) * a.ntx;
        rl[i] = qy > 0 ? 0u : 24u;
        // dead border: local x = 0 (rx = 0 sites of tiles tx = 0), local y = 0
        // (ry = 0 sites of tile ty = 0, i.e. byte 0 of quad row 0)
        dmx[i] = (qx == 0 && a.nbx > 1) ? 0x11111111u : 0u;
        dmy[i] = (qy == 0 && a.nby > 1) ? 0x00000005u : 0u;
        const uint64_t G = (uint64_t)b * nq + q;
        const U4 s4 = philox((uint32_t)G, (uint32_t)(G >> 32), a.t, TAG_SITE << 24, a.seed_lo,
                             a.seed_hi);
        sw[i][0] = s4.x;
        sw[i][1] = s4.y;
        sw[i][2] = s4.z;
        sw[i][3] = s4.w;
    }
    const uint32_t setw = philox(b, 0u, a.t, TAG_SET << 24, a.seed_lo, a.seed_hi).x;
    int net = 0;

    __syncthreads();

    // ---- work-group layer: 16 single-hit steps k = 4 kq + kr; sw[i][0] holds
    // the site word of the current group of four steps
    for (int kq = 0; kq < 4; ++kq) {
        for (int kr = 0; kr < 4; ++kr) {
            const int k = 4 * kq + kr;
            const uint32_t s = (setw >> (2 * k)) & 3u;
            const bool sx = s & 1u, sy = s >> 1;
            const uint32_t pc = s * nq, pl = (s ^ 1u) * nq, pd = (s ^ 2u) * nq;
#pragma unroll
            for (int i = 0; i < K; ++i) {
                if (K == 1 && !valid[i]) continue;
                const uint32_t ca = pc + own[i];
                const uint32_t la = pl + (sx ? own[i] : lft[i]);
                const uint32_t da = pd + (sy ? own[i] : dwn[i]);
                const uint32_t rot = sy ? 0u : rl[i];
                const uint32_t c = lds[ca];
                const uint32_t l = lds[la];
                const uint32_t d = rotr(lds[da], rot);
                // site of each tile's cell: r = 2 ry + rx in byte j
                const uint32_t D = (sw[i][0] >> (2 * kr)) & 0x03030303u;
                // one-hot sigma_x position 2r of the chosen site in every byte
                uint32_t oh = __builtin_amdgcn_perm(0u, 0x40100401u, D);
                oh &= ~((sx ? 0u : dmx[i]) | (sy ? 0u : dmy[i]));
                // neighbour slopes moved onto each site's own bit positions:
                // sigma_x(x-1,y) at 2r, sigma_y(x,y-1) at 2r+1
                const uint32_t X = ((c << 2) & 0x44444444u) | ((l >> 2) & 0x11111111u);
                const uint32_t Y = ((c << 4) & 0xA0A0A0A0u) | ((d >> 4) & 0x0A0A0A0Au);
                const uint32_t N = X | Y;
                // minimum: own slopes (+1,+1), incoming slopes (-1,-1)
                const uint32_t zmin = c & ~N;
                uint32_t F = zmin & (zmin >> 1) & oh;
                if (ACC) {
                    // maximum: own slopes (-1,-1), incoming slopes (+1,+1)
                    const uint32_t zmax = N & ~c;
                    const uint32_t Fx = zmax & (zmax >> 1) & oh;
                    uint32_t keep = 0;
                    if (__any((F | Fx) != 0)) {
                        const uint64_t G = (uint64_t)b * nq + own[i];
                        const U4 w1 = philox((uint32_t)G, (uint32_t)(G >> 32), a.t,
                                             (TAG_ACC1 << 24) | (uint32_t)kq, a.seed_lo,
                                             a.seed_hi);
                        const uint32_t Aw = kr == 0 ? w1.x : kr == 1 ? w1.y : kr == 2 ? w1.z : w1.w;
                        uint32_t tie = 0;
#pragma unroll
                        for (int j = 0; j < 4; ++j) {
                            const bool is_min = (F >> (8 * j)) & 0xFFu;
                            const bool is_max = (Fx >> (8 * j)) & 0xFFu;
                            const uint64_t thr = is_min ? a.P : a.Q;
                            const uint32_t Aj = (Aw >> (8 * j)) & 0xFFu;
                            const uint32_t t8 = (uint32_t)(thr >> 24);   // 256 for thr = 2^32
                            if ((is_min || is_max) && thr != 0) {
                                if (Aj < t8) keep |= 0xFFu << (8 * j);
                                else if (Aj == t8 && (thr & 0xFFFFFFu)) tie |= 1u << j;
                            }
                        }
                        if (__any(tie != 0)) {
                            const U4 w2 = philox((uint32_t)G, (uint32_t)(G >> 32), a.t,
                                                 (TAG_ACC2 << 24) | (uint32_t)k, a.seed_lo,
                                                 a.seed_hi);
                            const uint32_t Bw[4] = {w2.x, w2.y, w2.z, w2.w};
#pragma unroll
                            for (int j = 0; j < 4; ++j) {
                                const bool is_min = (F >> (8 * j)) & 0xFFu;
                                const uint64_t thr = is_min ? a.P : a.Q;
                                if ((tie >> j) & 1u && (Bw[j] & 0xFFFFFFu) < (uint32_t)(thr & 0xFFFFFFu))
                                    keep |= 0xFFu << (8 * j);
                            }
                        }
                    }
                    const uint32_t fmin = F & keep, fmax = Fx & keep;
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
                if (sx || lok[i]) lds[la] = l ^ ml;
                lds[da] = rotr(d ^ md, (32u - rot) & 31u);
            }
            __syncthreads();
        }
#pragma unroll
        for (int i = 0; i < K; ++i) {
            sw[i][0] = sw[i][1];
            sw[i][1] = sw[i][2];
            sw[i][2] = sw[i][3];
        }
    }

    // ---- store: quads -> cells -> aligned block words -> HBM row words
    for (uint32_t u = lane; u < a.units; u += 64) {
        const uint32_t wx = u % a.nw;
        const uint32_t rest = u / a.nw;
        const uint32_t qy = rest % a.H;
        const uint32_t sy = rest / a.H;
        const uint32_t q0 = qy * a.ntx + 4 * wx;
        uint32_t E[4], O[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            E[m] = lds[(2 * sy) * nq + q0 + m];
            O[m] = lds[(2 * sy + 1) * nq + q0 + m];
        }
        transpose_bytes(E);
        transpose_bytes(O);
        uint32_t gw = gw0 + wx;
        if (gw >= a.W) gw -= a.W;
        uint32_t gwe = gw0 + a.nw;
        if (gwe >= a.W) gwe -= a.W;
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
                // aligned word of the left neighbour unit (same row)
                const uint32_t prev = __shfl_up(A[h], 1, 64);
                if (sh2 == 0) {
                    row[gw] = A[h];
                } else {
                    if (wx == 0) {
                        const uint32_t delta = (A[h] ^ edge[r0 + h]) << sh2;
                        if (delta) atomicXor(row + gw, delta);
                    } else {
                        row[gw] = __builtin_amdgcn_alignbit(A[h], prev, 32u - sh2);
                    }
                    if (wx == a.nw - 1) {
                        const uint32_t delta = (A[h] ^ edge[a.By + r0 + h]) >> (32u - sh2);
                        if (delta) atomicXor(row + gwe, delta);
                    }
                }
            }
        }
    }

    // ---- flip counter of this block
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) net += __shfl_xor(net, off, 64);
    if (lane == 0 && net != 0)
        atomicAdd(a.slots + (b & (NSLOTS - 1)), (unsigned long long)(long long)net);
}

// ------------------------------------------------------------ roughness

// Per row y: with P(x) = sum_{l<x} sigma_x(l,y) (height relative to the row
// start), A_y = sum_x P(x) and B_y = sum_x P(x)^2.  One wave per row.
__global__ __launch_bounds__(256) void kpz_row_moments_kernel(const uint32_t *words, uint32_t L,
                                                              uint32_t W, long long *rowA,
                                                              long long *rowB)
{
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t row = blockIdx.x * 4u + (threadIdx.x >> 6);
    if (row >= L) return;
    const uint32_t *rp = words + (size_t)row * W;
    long long s1 = 0, s2 = 0;
    int carry = 0;
    for (uint32_t base = 0; base < W; base += 64) {
        const uint32_t idx = base + lane;
        const bool ok = idx < W;
        const uint32_t w = ok ? rp[idx] : 0u;
        int cur = 0, p1 = 0, p2 = 0;
        if (ok) {
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                p1 += cur;
                p2 += cur * cur;
                cur += ((w >> (2 * k)) & 1u) ? 1 : -1;
            }
        }
        // exclusive prefix of the word increments across the wave
        int incl = cur;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const int v = __shfl_up(incl, off, 64);
            if ((int)lane >= off) incl += v;
        }
        const int total = __shfl(incl, 63, 64);
        const long long o = carry + incl - cur;
        if (ok) {
            s1 += 16 * o + p1;
            s2 += 16 * o * o + 2 * o * p1 + p2;
        }
        carry += total;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        s1 += __shfl_xor(s1, off, 64);
        s2 += __shfl_xor(s2, off, 64);
    }
    if (lane == 0) {
        rowA[row] = s1;
        rowB[row] = s2;
    }
}

// One work-group of 1024 threads: c_y = sum_{k<y} sigma_y(0,k) (column-0
// heights), R1 = sum_y (L c_y + A_y), R2 = sum_y (L c_y^2 + 2 c_y A_y + B_y)
// in 128-bit, and the sum of the flip-counter slots.
__global__ __launch_bounds__(1024) void kpz_finalize_kernel(const uint32_t *words, uint32_t L,
                                                            uint32_t W, const long long *rowA,
                                                            const long long *rowB,
                                                            const long long *slots,
                                                            long long *res)
{
    __shared__ long long sc[1024];
    __shared__ __int128 r2s[1024];
    __shared__ long long r1s[1024];
    __shared__ long long ns[1024];
    const uint32_t tid = threadIdx.x;
    const uint32_t per = (L + 1023) / 1024;
    const uint32_t y0 = tid * per;
    const uint32_t y1 = min(L, y0 + per);
    long long loc = 0;
    for (uint32_t y = y0; y < y1; ++y) loc += ((words[(size_t)y * W] >> 1) & 1u) ? 1 : -1;
    sc[tid] = loc;
    __syncthreads();
    // inclusive Hillis-Steele scan over the 1024 thread sums
    for (uint32_t off = 1; off < 1024; off <<= 1) {
        const long long v = tid >= off ? sc[tid - off] : 0;
        __syncthreads();
        sc[tid] += v;
        __syncthreads();
    }
    long long c = sc[tid] - loc;
    long long r1 = 0;
    __int128 r2 = 0;
    for (uint32_t y = y0; y < y1; ++y) {
        const long long Ay = rowA[y], By = rowB[y];
        r1 += (long long)L * c + Ay;
        r2 += (__int128)L * c * c + (__int128)2 * c * Ay + By;
        c += ((words[(size_t)y * W] >> 1) & 1u) ? 1 : -1;
    }
    long long n = 0;
    for (uint32_t i = tid; i < NSLOTS; i += 1024) n += slots[i];
    r1s[tid] = r1;
    r2s[tid] = r2;
    ns[tid] = n;
    __syncthreads();
    for (uint32_t off = 512; off > 0; off >>= 1) {
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
    if (p->flags != 0) return KPZ_EINVAL;
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
    *Bx = (uint32_t)bx;
    *By = (uint32_t)by;
    return KPZ_OK;
}

size_t ws_needed(int64_t L)
{
    return (size_t)WS_HEADER + sizeof(long long) * NSLOTS + 2 * sizeof(long long) * (size_t)L;
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

template <int K, bool ACC>
hipError_t launch_sweep_k(const SweepArgs &a, uint32_t nblocks, size_t shmem, hipStream_t st)
{
    hipLaunchKernelGGL((kpz_sweep_kernel<K, ACC>), dim3(nblocks), dim3(64), shmem, st, a);
    return hipGetLastError();
}

template <bool ACC>
hipError_t launch_sweep(const SweepArgs &a, uint32_t K, uint32_t nblocks, size_t shmem,
                        hipStream_t st)
{
    switch (K) {
    case 1: return launch_sweep_k<1, ACC>(a, nblocks, shmem, st);
    case 2: return launch_sweep_k<2, ACC>(a, nblocks, shmem, st);
    case 4: return launch_sweep_k<4, ACC>(a, nblocks, shmem, st);
    case 8: return launch_sweep_k<8, ACC>(a, nblocks, shmem, st);
    case 16: return launch_sweep_k<16, ACC>(a, nblocks, shmem, st);
    default: return hipErrorInvalidValue;
    }
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

const char *kpz_last_error(const kpz_sim *s) { return s ? s->err : ""; }

kpz_status kpz_workspace_bytes(const kpz_params *p, size_t *bytes)
{
    uint32_t bx, by;
    const kpz_status st = resolve(p, &bx, &by);
    if (st != KPZ_OK) return st;
    if (!bytes) return KPZ_EINVAL;
    *bytes = ws_needed(p->L);
    return KPZ_OK;
}

kpz_status kpz_init(kpz_sim **out, const kpz_params *p, uint32_t *d_words, size_t words_bytes,
                    void *d_ws, size_t ws_bytes, void *stream)
{
    if (!out) return KPZ_EINVAL;
    *out = nullptr;
    uint32_t bx, by;
    kpz_status st = resolve(p, &bx, &by);
    if (st != KPZ_OK) return st;
    if (!d_words || !d_ws) return KPZ_EINVAL;
    const uint64_t L = (uint64_t)p->L;
    if (words_bytes < L * L / 4 || ws_bytes < ws_needed(p->L)) return KPZ_ESIZE;
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
        hip_fail(s, e, "kpz_init launch");
        delete s;
        return KPZ_EHIP;
    }
    *out = s;
    return KPZ_OK;
}

kpz_status kpz_sweep(kpz_sim *s, int32_t n_mcs)
{
    if (!s || n_mcs < 0) return KPZ_EINVAL;
    if (n_mcs == 0) return KPZ_OK;
    if (s->t + n_mcs > 0xFFFFFFFFll) return KPZ_ERANGE;
    const uint32_t L = (uint32_t)s->prm.L;
    SweepArgs a;
    a.words = s->words;
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
    a.nq = a.ntx * a.H;
    a.nw = s->Bx / 16;
    a.units = a.nw * a.H * 2;
    a.seed_lo = (uint32_t)s->prm.seed;
    a.seed_hi = (uint32_t)(s->prm.seed >> 32);
    a.P = s->P;
    a.Q = s->Q;
    const uint32_t K = a.nq <= 64 ? 1u : a.nq / 64u;
    const uint32_t nblocks = a.nbx * a.nby;
    const size_t shmem = sizeof(uint32_t) * (4 * (size_t)a.nq + 2 * (size_t)s->By);
    const bool acc = !(s->P == (1ull << 32) && s->Q == 0);
    for (int32_t m = 0; m < n_mcs; ++m) {
        a.t = (uint32_t)(s->t + m);
        const hipError_t e = acc ? launch_sweep<true>(a, K, nblocks, shmem, s->stream)
                                 : launch_sweep<false>(a, K, nblocks, shmem, s->stream);
        if (e != hipSuccess) return hip_fail(s, e, "kpz_sweep launch");
    }
    s->t += n_mcs;
    return KPZ_OK;
}

kpz_status kpz_roughness(kpz_sim *s, int64_t *S1o, int64_t *S2o, double *W2o)
{
    if (!s) return KPZ_EINVAL;
    const uint32_t L = (uint32_t)s->prm.L, W = L / 16;
    hipLaunchKernelGGL(kpz_row_moments_kernel, dim3((L + 3) / 4), dim3(256), 0, s->stream,
                       s->words, L, W, ws_rowA(s), ws_rowB(s));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(s, e, "kpz_roughness launch");
    hipLaunchKernelGGL(kpz_finalize_kernel, dim3(1), dim3(1024), 0, s->stream, s->words, L, W,
                       ws_rowA(s), ws_rowB(s), ws_slots(s), ws_res(s));
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(s, e, "kpz_roughness launch");
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
    return KPZ_OK;
}

void kpz_destroy(kpz_sim *s) { delete s; }

}  // extern "C"
