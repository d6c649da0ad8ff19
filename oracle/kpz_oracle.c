/*
 * kpz_oracle.c -- TEST INFRASTRUCTURE, NOT PRODUCT CODE.
 *
 * Plain, slow, obviously-correct CPU oracle for the 2+1-d KPZ octahedron
 * model (Kelling, Odor, Nagy, Schulz, Heinig, "Comparison of different
 * parallel implementations of the 2+1-dimensional KPZ model and the
 * 3-dimensional KMC model", Sec. 2.1 and Sec. 3.1).  Only the tests, the
 * smoke check and the CPU-baseline leg of the benchmark may load this
 * library; the GPU path shares no code with it.
 *
 * State: two int8 arrays sx[y*L+x], sy[y*L+x] in {-1,+1} holding the
 * forward slopes sigma_x(x,y) = h(x+1,y)-h(x,y) and sigma_y(x,y) =
 * h(x,y+1)-h(x,y) on the periodic L x L lattice (Sec. 2.1, the slope
 * description of the octahedron surface), plus the anchor height h(0,0).
 *
 * Update rule (Sec. 2.1, eq. "rule"): a site whose four nearest neighbours
 * are all one unit higher (a local minimum) is raised by two with
 * probability p; a site whose four neighbours are all one unit lower (a
 * local maximum) is lowered by two with probability q.  In slope terms
 * both moves negate sigma_x(x,y), sigma_x(x-1,y), sigma_y(x,y) and
 * sigma_y(x,y-1).
 *
 * Dynamics provided:
 *   or_rs_heights_run  random-sequential updates on an int64 height field
 *   or_rs_slopes_run   the same draws applied to the slope arrays
 *   or_dd_run          the two-layer decomposition of Sec. 3 / 3.1:
 *                      dead-border blocks with a random origin every MCS
 *                      (device layer), single-hit double tiling inside each
 *                      block (work-group layer)
 *   or_dd_run_par      the same, blocks of a residency on several threads
 *   or_strat_run       a control for the schedule studies: random-sequential
 *                      updates with exactly Tx*Ty attempts per tile per MCS
 *   or_rs1d_run        the 1+1-d rooftop (ASEP) reduction (Sec. 2.1),
 *                      random-sequential
 *   or_dd1d_run        the same ring under the decomposition of Sec. 3 / 3.1
 *                      reduced to one dimension
 * One Monte Carlo step (MCS) is N = L*L update attempts (Sec. 2.2).
 *
 * Random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel
 * random numbers: as easy as 1, 2, 3", SC'11), written out here from its
 * published definition.  The paper used LCGs / Mersenne Twister and found
 * the choice immaterial (Sec. 3.1); the counter layout below is this
 * project's own reading of the unspecified stream structure.
 *   ctr = (idx_lo, idx_hi, t, tag<<24 | sub),  key = (seed_lo, seed_hi)
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_TAG_ORIGIN 1u
#define OR_TAG_SET    2u
#define OR_TAG_SITE   3u
#define OR_TAG_ACC1   4u
#define OR_TAG_ACC2   5u
#define OR_TAG_RS     6u
#define OR_TAG_RS1D   7u
#define OR_TAG_ORIGIN1D 8u
#define OR_TAG_SET1D    9u
#define OR_TAG_SITE1D  10u
#define OR_TAG_ACC1D   11u
#define OR_TAG_ACC1D2  12u
#define OR_TAG_STRAT   14u
#define OR_TAG_STRAT2  15u

#define OR_OK       0
#define OR_EINVAL  -1
#define OR_ENOMEM  -2
#define OR_ECHECK  -3

/* ---------------------------------------------------------------- Philox */

/* R rounds of Philox4x32 on counter ctr with key key, the key advanced by
 * its Weyl increments before each round after the first.  R = 10 is the
 * published default; the 2+1-d lattice dynamics draw with R = 7. */
void or_philox4x32_r(const uint32_t ctr[4], const uint32_t key[2], int rounds, uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < rounds; ++round) {
        uint64_t prod0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t prod1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(prod0 >> 32), lo0 = (uint32_t)prod0;
        uint32_t hi1 = (uint32_t)(prod1 >> 32), lo1 = (uint32_t)prod1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += 0x9E3779B9u;   /* key schedule: golden-ratio Weyl increments */
        k1 += 0xBB67AE85u;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    or_philox4x32_r(ctr, key, 10, out);
}

/* Rounds per tag: the draws of the 2+1-d lattice dynamics (its decomposed
 * schedules, their random-sequential and stratified references: tags 1..6
 * and 13..15) use Philox4x32-7, the smallest round count its authors found
 * to pass the BigCrush battery; the ring (7..12) and KMC (16..) draws keep
 * the ten-round default. */
int or_tag_rounds(uint32_t tag)
{
    return ((tag >= 1u && tag <= 6u) || (tag >= 13u && tag <= 15u)) ? 7 : 10;
}

void or_draw(uint64_t seed, uint32_t tag, uint32_t t, uint64_t idx, uint32_t sub, uint32_t w[4])
{
    uint32_t ctr[4] = { (uint32_t)idx, (uint32_t)(idx >> 32), t, (tag << 24) | (sub & 0xFFFFFFu) };
    uint32_t key[2] = { (uint32_t)seed, (uint32_t)(seed >> 32) };
    or_philox4x32_r(ctr, key, or_tag_rounds(tag), w);
}

/* Acceptance threshold: an attempt with 32-bit uniform u is accepted iff
 * u < floor(prob * 2^32); prob = 1 gives 2^32 (always), prob = 0 gives 0. */
static uint64_t threshold(double prob)
{
    if (prob >= 1.0) return (uint64_t)1 << 32;
    if (prob <= 0.0) return 0;
    return (uint64_t)(prob * 4294967296.0);
}

/* ------------------------------------------------------------ the rule */

enum { SITE_NONE = 0, SITE_MIN = 1, SITE_MAX = 2 };

static int classify(int L, const int8_t *sx, const int8_t *sy, int x, int y)
{
    int xm = (x + L - 1) % L, ym = (y + L - 1) % L;
    int a = sx[y * L + x];    /* h(x+1,y) - h(x,y)  */
    int b = sy[y * L + x];    /* h(x,y+1) - h(x,y)  */
    int c = sx[y * L + xm];   /* h(x,y) - h(x-1,y)  */
    int d = sy[ym * L + x];   /* h(x,y) - h(x,y-1)  */
    if (a == 1 && b == 1 && c == -1 && d == -1) return SITE_MIN;
    if (a == -1 && b == -1 && c == 1 && d == 1) return SITE_MAX;
    return SITE_NONE;
}

static void flip(int L, int8_t *sx, int8_t *sy, int x, int y)
{
    int xm = (x + L - 1) % L, ym = (y + L - 1) % L;
    sx[y * L + x] = (int8_t)-sx[y * L + x];
    sy[y * L + x] = (int8_t)-sy[y * L + x];
    sx[y * L + xm] = (int8_t)-sx[y * L + xm];
    sy[ym * L + x] = (int8_t)-sy[ym * L + x];
}

/* ------------------------------------------------- flat initial state */

/* Flat start (Sec. 2.1): heights h(x,y) = (x+y) mod 2, h(0,0) = 0. */
int or_flat(int L, int8_t *sx, int8_t *sy)
{
    if (L <= 0 || (L & 1)) return OR_EINVAL;
    for (int y = 0; y < L; ++y)
        for (int x = 0; x < L; ++x) {
            int h = (x + y) & 1;
            int hx = ((x + 1) % L + y) & 1;   /* L even: parity is periodic */
            int hy = (x + (y + 1) % L) & 1;
            sx[y * L + x] = (int8_t)(hx - h);
            sy[y * L + x] = (int8_t)(hy - h);
        }
    return OR_OK;
}

/* ------------------------------------------- random-sequential dynamics */

/* One attempt of MCS t with index a in [0, N): site = floor(w0 * N / 2^32),
 * uniform u = w1. */
int or_rs_heights_run(int L, double p, double q, uint64_t seed, uint32_t t0, int n_mcs,
                      int64_t *h)
{
    if (L <= 0 || (L & 1) || n_mcs < 0) return OR_EINVAL;
    const uint64_t N = (uint64_t)L * (uint64_t)L;
    const uint64_t P = threshold(p), Q = threshold(q);
    uint32_t w[4];
    for (int m = 0; m < n_mcs; ++m) {
        uint32_t t = t0 + (uint32_t)m;
        for (uint64_t a = 0; a < N; ++a) {
            or_draw(seed, OR_TAG_RS, t, a, 0, w);
            uint64_t site = ((uint64_t)w[0] * N) >> 32;
            int x = (int)(site % (uint64_t)L), y = (int)(site / (uint64_t)L);
            int64_t hh = h[site];
            int64_t hl = h[(uint64_t)y * L + (x + L - 1) % L];
            int64_t hr = h[(uint64_t)y * L + (x + 1) % L];
            int64_t hd = h[(uint64_t)((y + L - 1) % L) * L + x];
            int64_t hu = h[(uint64_t)((y + 1) % L) * L + x];
            if (hl == hh + 1 && hr == hh + 1 && hd == hh + 1 && hu == hh + 1) {
                if ((uint64_t)w[1] < P) h[site] = hh + 2;
            } else if (hl == hh - 1 && hr == hh - 1 && hd == hh - 1 && hu == hh - 1) {
                if ((uint64_t)w[1] < Q) h[site] = hh - 2;
            }
        }
    }
    return OR_OK;
}

int or_rs_slopes_run(int L, double p, double q, uint64_t seed, uint32_t t0, int n_mcs,
                     int8_t *sx, int8_t *sy, int64_t *h00, int64_t *net)
{
    if (L <= 0 || (L & 1) || n_mcs < 0) return OR_EINVAL;
    const uint64_t N = (uint64_t)L * (uint64_t)L;
    const uint64_t P = threshold(p), Q = threshold(q);
    uint32_t w[4];
    for (int m = 0; m < n_mcs; ++m) {
        uint32_t t = t0 + (uint32_t)m;
        for (uint64_t a = 0; a < N; ++a) {
            or_draw(seed, OR_TAG_RS, t, a, 0, w);
            uint64_t site = ((uint64_t)w[0] * N) >> 32;
            int x = (int)(site % (uint64_t)L), y = (int)(site / (uint64_t)L);
            int kind = classify(L, sx, sy, x, y);
            int dh = 0;
            if (kind == SITE_MIN && (uint64_t)w[1] < P) dh = 2;
            if (kind == SITE_MAX && (uint64_t)w[1] < Q) dh = -2;
            if (dh) {
                flip(L, sx, sy, x, y);
                *net += dh / 2;
                if (x == 0 && y == 0) *h00 += dh;
            }
        }
    }
    return OR_OK;
}

/*
 * Stratified random-sequential control (an experiment, not a schedule of
 * the paper): per MCS every Tx x Ty tile of the fixed tiling receives
 * exactly Tx*Ty attempts, at uniformly random sites of the tile, and all N
 * attempts run one at a time in a uniformly random order.  It differs from
 * random-sequential updates only in the exact per-tile attempt count, and
 * from the decomposed schedule in having no cells, sets, single hits or
 * dead borders, so it isolates the effect of the exact count on W^2(t).
 * Order: Fisher-Yates over the attempt list (tile-major), position i
 * drawing j = floor(w0 (i+1) / 2^32) from (STRAT, t, i, 0); attempt a (tile
 * a / S) takes its site floor(w0 S / 2^32) in the tile and u = w1 from
 * (STRAT2, t, a, 0).
 */
int or_strat_run(int L, double p, double q, uint64_t seed, int Tx, int Ty, uint32_t t0,
                 int n_mcs, int8_t *sx, int8_t *sy, int64_t *h00, int64_t *net)
{
    if (L <= 0 || (L & 1) || n_mcs < 0 || Tx <= 0 || Ty <= 0 || L % Tx || L % Ty) return OR_EINVAL;
    const uint64_t N = (uint64_t)L * (uint64_t)L;
    const int S = Tx * Ty, ntx = L / Tx;
    const uint64_t P = threshold(p), Q = threshold(q);
    uint32_t *order = (uint32_t *)malloc(sizeof(uint32_t) * N);
    if (!order) return OR_ENOMEM;
    uint32_t w[4];
    for (int m = 0; m < n_mcs; ++m) {
        const uint32_t t = t0 + (uint32_t)m;
        for (uint64_t a = 0; a < N; ++a) order[a] = (uint32_t)a;
        for (uint64_t i = N - 1; i > 0; --i) {
            or_draw(seed, OR_TAG_STRAT, t, i, 0, w);
            const uint64_t j = ((uint64_t)w[0] * (i + 1)) >> 32;
            const uint32_t tmp = order[i];
            order[i] = order[j];
            order[j] = tmp;
        }
        for (uint64_t i = 0; i < N; ++i) {
            const uint32_t a = order[i];
            or_draw(seed, OR_TAG_STRAT2, t, a, 0, w);
            const int tile = (int)(a / (uint32_t)S);
            const int r = (int)(((uint64_t)w[0] * (uint64_t)S) >> 32);
            const int x = (tile % ntx) * Tx + r % Tx, y = (tile / ntx) * Ty + r / Tx;
            const int kind = classify(L, sx, sy, x, y);
            int dh = 0;
            if (kind == SITE_MIN && (uint64_t)w[1] < P) dh = 2;
            if (kind == SITE_MAX && (uint64_t)w[1] < Q) dh = -2;
            if (dh) {
                flip(L, sx, sy, x, y);
                *net += dh / 2;
                if (x == 0 && y == 0) *h00 += dh;
            }
        }
    }
    free(order);
    return OR_OK;
}

/* ---------------------------------------- decomposed (DB + DT) dynamics */

/*
 * One MCS t of the two-layer schedule (Sec. 3 and 3.1):
 *
 * Device layer, dead border.  Origin (ox, oy) = (floor(w0*Bx/2^32),
 * floor(w1*By/2^32)) from draw (ORIGIN, t, 0, 0); it moves every MCS.
 * Block (bx, by), b = by*nbx + bx, covers global sites
 * ((ox + bx*Bx + lx) mod L, (oy + by*By + ly) mod L), 0 <= lx < Bx,
 * 0 <= ly < By.  Sites with lx = 0 (when nbx > 1) or ly = 0 (when
 * nby > 1) are the dead border: they are never updated, but an attempt
 * that lands there still counts.  With width one on the low side, every
 * update of a block reads and writes only slopes stored at its own sites.
 *
 * Work-group layer, single-hit double tiling.  Tiles Tx x Ty, each bisected
 * in both directions into four cells of cx x cy = Tx/2 x Ty/2 sites; cell
 * set s = sx + 2 sy.  A block makes S = Tx*Ty single-hit steps per MCS, so
 * every site of the block had on average one chance.  In step k the block
 * draws one set s_k (uniform, with replacement) = bits 2k..2k+1 of w0 of
 * draw (SET, t, b, 0); every tile then makes one attempt at a site of its
 * set-s_k cell.  Cells of one set are at least cx+1 (cy+1) sites apart, so
 * the attempts of a step never touch each other.
 *
 * Draw numbering (this project's layout; the paper leaves the random
 * streams open).  Tile row ty of block b is cut into row groups of 32
 * tiles, G = (b*nty + ty)*nqx + tx/32 (nty = By/Ty tile rows per block,
 * nqx = ntx/32 groups per tile row, or one group of all ntx tiles when
 * ntx <= 32); tile tx owns bit pi(tx) = 8*(tx mod 4) + (tx mod 32)/4 of
 * every 32-bit word drawn for its group.
 *   Site in a 2x2 cell at step k: rx = bit pi(tx) of word 2*(k mod 2), ry =
 *   bit pi(tx) of word 2*(k mod 2) + 1 of draw (SITE, t, G, k/2).  1x1
 *   cells (2x2 tiles) draw no site.
 *   Acceptance uniform at step k: u = sum_j b_j 2^(31-j), j = 0..31, b_j =
 *   bit pi(tx) of word (k mod 4) of draw (ACC1, t, G, 4*(k/4) + j) for
 *   j < 4, and of word (j mod 4) of draw (ACC2, t, G, 8*k + j/4 - 1) for
 *   j >= 4.  The attempt is accepted iff u < P (at a minimum) or u < Q (at a
 *   maximum), P = floor(p*2^32) (2^32 for p = 1), Q likewise.
 *
 * Block residency (Sec. 3: the origin is moved after some time).  With
 * `moves` = m > 1 the origin moves m times per MCS: residency i = 0..m-1
 * of MCS t has its own origin from draw (ORIGIN, t, i, 0) and set word
 * from (SET, t, b, i), and runs steps k = i S/m .. (i+1) S/m - 1 in the
 * blocks of that origin; site and acceptance draws are numbered by the
 * step k within the MCS as above.  m = 1 is the schedule above.
 */
/* Cell set of step k from the block's set draw w[0..3]: bits 2 (k mod 16)
 * .. +1 of word k / 16 (word 0 for the 16 steps of 4 x 4 tiles). */
static int step_set(const uint32_t w[4], int k)
{
    return (int)((w[k >> 4] >> (2 * (k & 15))) & 3u);
}

static int dd_validate(int L, int Bx, int By, int Tx, int Ty, int moves)
{
    if (L <= 0 || (L & 1)) return 0;
    if (moves < 1 || (moves & (moves - 1)) || (Tx * Ty) % moves) return 0;
    if (Bx <= 0 || By <= 0 || L % Bx || L % By) return 0;
    if (!((Tx == 4 && Ty == 4) || (Tx == 2 && Ty == 2) || (Tx == 8 && Ty == 8))) return 0;
    if (Bx % Tx || By % Ty) return 0;
    /* a tile row is one row group of at most 32 tiles or whole groups of 32 */
    if (Bx / Tx > 32 && (Bx / Tx) % 32) return 0;
    return 1;
}

/* Bit of tile tx (tile tx mod 32 of its row group) in every word drawn
 * for the group. */
static int tile_bit(int tx) { return 8 * (tx & 3) + ((tx & 31) >> 2); }

/* Row group of tile (tx, ty) of block b: tile row ty of the block cut into
 * groups of 32 tiles (one group when the row has at most 32). */
static uint64_t row_group(int b, int ty, int tx, int nty, int ntx)
{
    const uint64_t nqx = ntx > 32 ? (uint64_t)(ntx / 32) : 1u;
    return ((uint64_t)b * (uint64_t)nty + (uint64_t)ty) * nqx + (uint64_t)(tx / 32);
}

/* Bit i of the site draw of step k, tile tx of row group G, for cells of
 * 2^a sites: word a*k + i of the group's site stream, i.e. word
 * (a*k + i) mod 4 of draw (SITE, t, G, (a*k + i) / 4). */
static int site_bit(uint64_t seed, uint32_t t, uint64_t G, int k, int a, int i, int tx)
{
    uint32_t w[4];
    const uint32_t n = (uint32_t)(a * k + i);
    or_draw(seed, OR_TAG_SITE, t, G, n >> 2, w);
    return (int)((w[n & 3u] >> tile_bit(tx)) & 1u);
}

/* Site (rx, ry) in the cell of tile tx of row group G at step k: for 2x2
 * cells rx = bit 0, ry = bit 1; for 4x4 cells rx = bit 0 + 2 bit 1, ry =
 * bit 2 + 2 bit 3 (the 4x4 cells of 8x8 tiles, an oracle-only variant). */
static void cell_site(uint64_t seed, uint32_t t, uint64_t G, int k, int cx, int tx, int *rx,
                      int *ry)
{
    if (cx == 2) {
        *rx = site_bit(seed, t, G, k, 2, 0, tx);
        *ry = site_bit(seed, t, G, k, 2, 1, tx);
    } else {
        *rx = site_bit(seed, t, G, k, 4, 0, tx) + 2 * site_bit(seed, t, G, k, 4, 1, tx);
        *ry = site_bit(seed, t, G, k, 4, 2, tx) + 2 * site_bit(seed, t, G, k, 4, 3, tx);
    }
}

/* The 32-bit acceptance uniform of tile tx of row group G at step k. */
static uint32_t acc_uniform(uint64_t seed, uint32_t t, uint64_t G, int k, int tx)
{
    const int bit = tile_bit(tx);
    uint32_t u = 0, w[4];
    for (int j = 0; j < 32; ++j) {
        uint32_t word;
        if (j < 4) {
            or_draw(seed, OR_TAG_ACC1, t, G, (uint32_t)(4 * (k >> 2) + j), w);
            word = w[k & 3];
        } else {
            or_draw(seed, OR_TAG_ACC2, t, G, (uint32_t)(8 * k + (j >> 2) - 1), w);
            word = w[j & 3];
        }
        u |= ((word >> bit) & 1u) << (31 - j);
    }
    return u;
}

/* Whether an attempt at a site of kind `kind` is accepted. */
static int accepted(int kind, uint64_t P, uint64_t Q, uint64_t seed, uint32_t t, uint64_t G,
                    int k, int tx)
{
    const uint64_t thr = kind == SITE_MIN ? P : Q;
    if (thr == 0) return 0;
    if (thr >= ((uint64_t)1 << 32)) return 1;
    return (uint64_t)acc_uniform(seed, t, G, k, tx) < thr;
}

/* Block-local site (lx, ly) of tile (tx, ty) of row group G at step k with
 * cell set s. */
static void attempt_site(uint64_t seed, uint32_t t, uint64_t G, int k, int s, int tx, int ty,
                         int Tx, int Ty, int *lx, int *ly)
{
    const int cx = Tx / 2, cy = Ty / 2;
    int rx = 0, ry = 0;
    if (cx * cy > 1) cell_site(seed, t, G, k, cx, tx, &rx, &ry);
    *lx = tx * Tx + (s & 1) * cx + rx;
    *ly = ty * Ty + (s >> 1) * cy + ry;
}

int or_dd_run(int L, double p, double q, uint64_t seed, int Bx, int By, int Tx, int Ty,
              int moves, uint32_t t0, int n_mcs, int8_t *sx, int8_t *sy, int64_t *h00,
              int64_t *net, int check)
{
    if (!dd_validate(L, Bx, By, Tx, Ty, moves) || n_mcs < 0) return OR_EINVAL;
    const int nbx = L / Bx, nby = L / By;
    const int ntx = Bx / Tx, nty = By / Ty;
    const int S = Tx * Ty;
    const uint64_t P = threshold(p), Q = threshold(q);
    const int nblocks = nbx * nby;
    uint32_t *setw = (uint32_t *)malloc(sizeof(uint32_t) * 4 * (size_t)nblocks);
    int64_t *stamp = check ? (int64_t *)malloc(sizeof(int64_t) * (size_t)L * (size_t)L) : NULL;
    if (!setw || (check && !stamp)) {
        free(setw); free(stamp);
        return OR_ENOMEM;
    }
    if (check)
        for (size_t i = 0; i < (size_t)L * (size_t)L; ++i) stamp[i] = -1;
    int64_t step_id = 0;
    int status = OR_OK;
    uint32_t w[4];

    const int per_res = S / moves;
    for (int m = 0; m < n_mcs && status == OR_OK; ++m) {
      const uint32_t t = t0 + (uint32_t)m;
      for (int res = 0; res < moves && status == OR_OK; ++res) {
        or_draw(seed, OR_TAG_ORIGIN, t, (uint64_t)res, 0, w);
        const int ox = (int)(((uint64_t)w[0] * (uint64_t)Bx) >> 32);
        const int oy = (int)(((uint64_t)w[1] * (uint64_t)By) >> 32);
        for (int b = 0; b < nblocks; ++b) {
            or_draw(seed, OR_TAG_SET, t, (uint64_t)b, (uint32_t)res, &setw[4 * b]);
        }
        /* all blocks make step k "at the same time"; blocks are independent,
           so visiting them one after the other gives the same result */
        for (int k = res * per_res; k < (res + 1) * per_res && status == OR_OK; ++k, ++step_id) {
            for (int by = 0; by < nby; ++by)
                for (int bx = 0; bx < nbx; ++bx) {
                    const int b = by * nbx + bx;
                    const int s = step_set(&setw[4 * b], k);
                    for (int ty = 0; ty < nty; ++ty)
                        for (int tx = 0; tx < ntx; ++tx) {
                            const uint64_t G = row_group(b, ty, tx, nty, ntx);
                            int lx, ly;
                            attempt_site(seed, t, G, k, s, tx, ty, Tx, Ty, &lx, &ly);
                            if ((nbx > 1 && lx == 0) || (nby > 1 && ly == 0)) continue;
                            const int gx = (ox + bx * Bx + lx) % L;
                            const int gy = (oy + by * By + ly) % L;
                            if (check) {
                                /* no two attempts of one step are equal or neighbours */
                                const int nx[5] = { gx, (gx + 1) % L, (gx + L - 1) % L, gx, gx };
                                const int ny[5] = { gy, gy, gy, (gy + 1) % L, (gy + L - 1) % L };
                                for (int e = 0; e < 5; ++e)
                                    if (stamp[(size_t)ny[e] * L + nx[e]] == step_id) status = OR_ECHECK;
                                stamp[(size_t)gy * L + gx] = step_id;
                            }
                            const int kind = classify(L, sx, sy, gx, gy);
                            if (kind == SITE_NONE) continue;
                            if (!accepted(kind, P, Q, seed, t, G, k, tx)) continue;
                            flip(L, sx, sy, gx, gy);
                            const int dh = kind == SITE_MIN ? 2 : -2;
                            *net += dh / 2;
                            if (gx == 0 && gy == 0) *h00 += dh;
                        }
                }
        }
      }
    }
    free(setw); free(stamp);
    return status;
}

/*
 * The same schedule visited block by block: within one residency the
 * blocks never touch each other's slopes (dead borders; a block that spans
 * a whole axis wraps onto itself), so a residency may run its blocks in any
 * order, here in parallel over `threads` OpenMP threads, each block making
 * all its steps before the next.  Equal to or_dd_run (tested); used to time
 * the oracle on all host cores and to reach larger lattices in the tests.
 */
int or_dd_run_par(int L, double p, double q, uint64_t seed, int Bx, int By, int Tx, int Ty,
                  int moves, uint32_t t0, int n_mcs, int8_t *sx, int8_t *sy, int64_t *h00,
                  int64_t *net, int threads)
{
    if (!dd_validate(L, Bx, By, Tx, Ty, moves) || n_mcs < 0 || threads < 1) return OR_EINVAL;
    const int nbx = L / Bx, nby = L / By;
    const int ntx = Bx / Tx, nty = By / Ty;
    const int S = Tx * Ty;
    const uint64_t P = threshold(p), Q = threshold(q);
    const int nblocks = nbx * nby;
    const int per_res = S / moves;
    for (int m = 0; m < n_mcs; ++m) {
        const uint32_t t = t0 + (uint32_t)m;
        for (int res = 0; res < moves; ++res) {
            uint32_t w[4];
            or_draw(seed, OR_TAG_ORIGIN, t, (uint64_t)res, 0, w);
            const int ox = (int)(((uint64_t)w[0] * (uint64_t)Bx) >> 32);
            const int oy = (int)(((uint64_t)w[1] * (uint64_t)By) >> 32);
            int64_t dnet = 0, dh00 = 0;
#pragma omp parallel for schedule(dynamic, 16) num_threads(threads) reduction(+ : dnet, dh00)
            for (int b = 0; b < nblocks; ++b) {
                const int bx = b % nbx, by = b / nbx;
                uint32_t ws[4];
                or_draw(seed, OR_TAG_SET, t, (uint64_t)b, (uint32_t)res, ws);
                for (int k = res * per_res; k < (res + 1) * per_res; ++k) {
                    const int s = step_set(ws, k);
                    for (int ty = 0; ty < nty; ++ty)
                        for (int tx = 0; tx < ntx; ++tx) {
                            const uint64_t G = row_group(b, ty, tx, nty, ntx);
                            int lx, ly;
                            attempt_site(seed, t, G, k, s, tx, ty, Tx, Ty, &lx, &ly);
                            if ((nbx > 1 && lx == 0) || (nby > 1 && ly == 0)) continue;
                            const int gx = (ox + bx * Bx + lx) % L;
                            const int gy = (oy + by * By + ly) % L;
                            const int kind = classify(L, sx, sy, gx, gy);
                            if (kind == SITE_NONE) continue;
                            if (!accepted(kind, P, Q, seed, t, G, k, tx)) continue;
                            flip(L, sx, sy, gx, gy);
                            const int dh = kind == SITE_MIN ? 2 : -2;
                            dnet += dh / 2;
                            if (gx == 0 && gy == 0) dh00 += dh;
                        }
                }
            }
            *net += dnet;
            *h00 += dh00;
        }
    }
    return OR_OK;
}

/* -------------------------------------------- 1+1-d rooftop reduction */

/* Ring of L bonds s[i] = h(i+1) - h(i) in {-1,+1}; site i is a minimum iff
 * s[i-1] = -1 and s[i] = +1.  Attempt a of MCS t: site floor(w0*L/2^32),
 * u = w1 of draw (RS1D, t, a, 0). */
int or_rs1d_run(int L, double p, double q, uint64_t seed, uint32_t t0, int n_mcs,
                int8_t *s, int64_t *h0, int64_t *net)
{
    if (L <= 0 || (L & 1) || n_mcs < 0) return OR_EINVAL;
    const uint64_t P = threshold(p), Q = threshold(q);
    uint32_t w[4];
    for (int m = 0; m < n_mcs; ++m) {
        uint32_t t = t0 + (uint32_t)m;
        for (uint64_t a = 0; a < (uint64_t)L; ++a) {
            or_draw(seed, OR_TAG_RS1D, t, a, 0, w);
            int i = (int)(((uint64_t)w[0] * (uint64_t)L) >> 32);
            int im = (i + L - 1) % L;
            int dh = 0;
            if (s[im] == -1 && s[i] == 1 && (uint64_t)w[1] < P) dh = 2;
            else if (s[im] == 1 && s[i] == -1 && (uint64_t)w[1] < Q) dh = -2;
            if (dh) {
                s[im] = (int8_t)-s[im];
                s[i] = (int8_t)-s[i];
                *net += dh / 2;
                if (i == 0) *h0 += dh;
            }
        }
    }
    return OR_OK;
}

/* ------------------------------------------- one block, on its own copy */

/*
 * Residency res of MCS t of the decomposed schedule (the whole MCS when
 * moves = 1) restricted to block (bx, by) of that residency's origin, run on
 * a copy of that block's sites: bsx[ly*Bx+lx], bsy[ly*Bx+lx] hold sigma_x,
 * sigma_y of block-local site (lx, ly), i.e. global site
 * ((ox + bx*Bx + lx) mod L, (oy + by*By + ly) mod L).  Requires more than one
 * block along both axes: then the dead border (lx = 0, ly = 0) keeps every
 * update inside the block's own sites, so this equals the block's part of
 * or_dd_run.  Same draws and the same step order as or_dd_run.
 */
int or_dd_block_mcs(int L, double p, double q, uint64_t seed, int Bx, int By, int Tx, int Ty,
                    int moves, uint32_t t, int res, int bx, int by, int8_t *bsx, int8_t *bsy,
                    int64_t *net)
{
    if (!dd_validate(L, Bx, By, Tx, Ty, moves) || res < 0 || res >= moves) return OR_EINVAL;
    const int nbx = L / Bx, nby = L / By;
    if (nbx < 2 || nby < 2 || bx < 0 || by < 0 || bx >= nbx || by >= nby) return OR_EINVAL;
    const int ntx = Bx / Tx, nty = By / Ty;
    const int S = Tx * Ty;
    const uint64_t P = threshold(p), Q = threshold(q);
    const int b = by * nbx + bx;
    const int per_res = S / moves;
    uint32_t w[4];
    or_draw(seed, OR_TAG_SET, t, (uint64_t)b, (uint32_t)res, w);
    for (int k = res * per_res; k < (res + 1) * per_res; ++k) {
        const int s = step_set(w, k);
        for (int ty = 0; ty < nty; ++ty)
            for (int tx = 0; tx < ntx; ++tx) {
                const uint64_t G = row_group(b, ty, tx, nty, ntx);
                int lx, ly;
                attempt_site(seed, t, G, k, s, tx, ty, Tx, Ty, &lx, &ly);
                if (lx == 0 || ly == 0) continue;   /* dead border */
                int8_t *a = &bsx[ly * Bx + lx], *bb = &bsy[ly * Bx + lx];
                int8_t *c = &bsx[ly * Bx + lx - 1], *d = &bsy[(ly - 1) * Bx + lx];
                int kind = SITE_NONE;
                if (*a == 1 && *bb == 1 && *c == -1 && *d == -1) kind = SITE_MIN;
                if (*a == -1 && *bb == -1 && *c == 1 && *d == 1) kind = SITE_MAX;
                if (kind == SITE_NONE) continue;
                if (!accepted(kind, P, Q, seed, t, G, k, tx)) continue;
                *a = (int8_t)-*a; *bb = (int8_t)-*bb; *c = (int8_t)-*c; *d = (int8_t)-*d;
                *net += kind == SITE_MIN ? 1 : -1;
            }
    }
    return OR_OK;
}

/* Origin of residency res of MCS t: ox = floor(w0 * Bx / 2^32),
 * oy = floor(w1 * By / 2^32) of draw (ORIGIN, t, res, 0). */
void or_dd_origin(uint64_t seed, uint32_t t, int res, int Bx, int By, int *ox, int *oy)
{
    uint32_t w[4];
    or_draw(seed, OR_TAG_ORIGIN, t, (uint64_t)res, 0, w);
    *ox = (int)(((uint64_t)w[0] * (uint64_t)Bx) >> 32);
    *oy = (int)(((uint64_t)w[1] * (uint64_t)By) >> 32);
}

/* ------------------------------------ 1+1-d decomposed schedule */

/*
 * The rooftop ring (bonds s[i] = h(i+1) - h(i), site i touches bonds i-1
 * and i) under the two-layer decomposition of Sec. 3 / 3.1 reduced to one
 * dimension:
 *
 * Device layer.  Origin o = floor(w0 * B / 2^32) of draw (ORIGIN1D, t, 0, 0),
 * once per MCS; block b covers sites (o + b B + lx) mod L, 0 <= lx < B.  With
 * more than one block, site lx = 0 is the dead border: every update of a
 * block then reads and writes only the block's own bonds.
 *
 * Work-group layer.  Tiles of 4 sites, bisected into two cells of 2 sites
 * (set 0: sites 0, 1; set 1: sites 2, 3 of the tile); S = 4 single-hit
 * steps per MCS.  In step k block b uses set bit 4 (b mod 8) + k of word
 * (b mod 32) / 8 of draw (SET1D, t, b / 32, 0) (one draw serves 32 blocks)
 * and tile m attempts site 4 m + 2 set + r.  Attempts of one step are at
 * least three sites apart.
 *
 * Draws.  Tile m of block b is tile mm = m mod 8 of block word wl = m / 8
 * (a packed word holds 32 sites = 8 tiles); with nt = B/4 tiles per block,
 * n4 = ceil(nt/32) and n2 = ceil(nt/16):
 *   r = bit 4 mm + k of word (wl mod 4) of draw (SITE1D, t, b n4 + wl/4, 0);
 *   u = A << 24 | (C & 0xFFFFFF) with A = byte (mm mod 4) of word
 *       2 (wl mod 2) + mm/4 of draw (ACC1D, t, b n2 + wl/2, k) and
 *       C = w0 of draw (ACC1D2, t, b nt + m, k) (needed only on a tie of A).
 */
static int dd1d_validate(int L, int B)
{
    return L > 0 && !(L & 1) && B >= 4 && B % 4 == 0 && L % B == 0;
}

static int dd1d_attempt(int L, int8_t *s, int i, uint64_t P, uint64_t Q, uint64_t seed,
                        uint32_t t, int k, uint64_t acc_idx, int acc_word, int acc_shift,
                        uint64_t tie_idx, int64_t *h0, int64_t *net)
{
    const int im = (i + L - 1) % L;
    int kind = SITE_NONE;
    if (s[im] == -1 && s[i] == 1) kind = SITE_MIN;
    if (s[im] == 1 && s[i] == -1) kind = SITE_MAX;
    if (kind == SITE_NONE) return 0;
    const uint64_t thr = kind == SITE_MIN ? P : Q;
    if (thr == 0) return 0;
    if (thr < ((uint64_t)1 << 32)) {
        uint32_t wa[4], wc[4];
        or_draw(seed, OR_TAG_ACC1D, t, acc_idx, (uint32_t)k, wa);
        const uint32_t A = (wa[acc_word] >> acc_shift) & 0xFFu;
        or_draw(seed, OR_TAG_ACC1D2, t, tie_idx, (uint32_t)k, wc);
        const uint32_t u = (A << 24) | (wc[0] & 0xFFFFFFu);
        if ((uint64_t)u >= thr) return 0;
    }
    s[im] = (int8_t)-s[im];
    s[i] = (int8_t)-s[i];
    const int dh = kind == SITE_MIN ? 2 : -2;
    *net += dh / 2;
    if (i == 0) *h0 += dh;
    return 1;
}

int or_dd1d_run(int L, double p, double q, uint64_t seed, int B, uint32_t t0, int n_mcs,
                int8_t *s, int64_t *h0, int64_t *net, int check)
{
    if (!dd1d_validate(L, B) || n_mcs < 0) return OR_EINVAL;
    const int nb = L / B, nt = B / 4;
    const uint64_t n4 = (uint64_t)(nt + 31) / 32, n2 = (uint64_t)(nt + 15) / 16;
    const uint64_t P = threshold(p), Q = threshold(q);
    int64_t *stamp = check ? (int64_t *)malloc(sizeof(int64_t) * (size_t)L) : NULL;
    if (check && !stamp) return OR_ENOMEM;
    if (check)
        for (int i = 0; i < L; ++i) stamp[i] = -1;
    int64_t step_id = 0;
    int status = OR_OK;
    uint32_t w[4];
    for (int mc = 0; mc < n_mcs && status == OR_OK; ++mc) {
        const uint32_t t = t0 + (uint32_t)mc;
        or_draw(seed, OR_TAG_ORIGIN1D, t, 0, 0, w);
        const int o = (int)(((uint64_t)w[0] * (uint64_t)B) >> 32);
        for (int k = 0; k < 4 && status == OR_OK; ++k, ++step_id) {
            for (int b = 0; b < nb; ++b) {
                or_draw(seed, OR_TAG_SET1D, t, (uint64_t)(b / 32), 0, w);
                const int set = (int)((w[(b % 32) / 8] >> (4 * (b % 8) + k)) & 1u);
                for (int m = 0; m < nt; ++m) {
                    const int wl = m / 8, mm = m % 8;
                    or_draw(seed, OR_TAG_SITE1D, t, (uint64_t)b * n4 + (uint64_t)(wl / 4), 0, w);
                    const int r = (int)((w[wl % 4] >> (4 * mm + k)) & 1u);
                    const int lx = 4 * m + 2 * set + r;
                    if (nb > 1 && lx == 0) continue;
                    const int i = (int)(((int64_t)o + (int64_t)b * B + lx) % L);
                    if (check) {
                        const int nbr[3] = { i, (i + 1) % L, (i + L - 1) % L };
                        for (int e = 0; e < 3; ++e)
                            if (stamp[nbr[e]] == step_id) status = OR_ECHECK;
                        stamp[i] = step_id;
                    }
                    dd1d_attempt(L, s, i, P, Q, seed, t, k, (uint64_t)b * n2 + (uint64_t)(wl / 2),
                                 2 * (wl % 2) + mm / 4, 8 * (mm % 4),
                                 (uint64_t)b * (uint64_t)nt + (uint64_t)m, h0, net);
                }
            }
        }
    }
    free(stamp);
    return status;
}

/* One MCS t of block b of the 1+1-d schedule on its own copy bs[lx] of the
 * block's bonds (global bond (o + b B + lx) mod L); needs two or more
 * blocks, so that the dead border keeps every update inside the block. */
int or_dd1d_block_mcs(int L, double p, double q, uint64_t seed, int B, uint32_t t, int b,
                      int8_t *bs, int64_t *net)
{
    if (!dd1d_validate(L, B)) return OR_EINVAL;
    const int nb = L / B, nt = B / 4;
    if (nb < 2 || b < 0 || b >= nb) return OR_EINVAL;
    const uint64_t n4 = (uint64_t)(nt + 31) / 32, n2 = (uint64_t)(nt + 15) / 16;
    const uint64_t P = threshold(p), Q = threshold(q);
    uint32_t w[4];
    int64_t h0_unused = 0;
    for (int k = 0; k < 4; ++k) {
        or_draw(seed, OR_TAG_SET1D, t, (uint64_t)(b / 32), 0, w);
        const int set = (int)((w[(b % 32) / 8] >> (4 * (b % 8) + k)) & 1u);
        for (int m = 0; m < nt; ++m) {
            const int wl = m / 8, mm = m % 8;
            or_draw(seed, OR_TAG_SITE1D, t, (uint64_t)b * n4 + (uint64_t)(wl / 4), 0, w);
            const int r = (int)((w[wl % 4] >> (4 * mm + k)) & 1u);
            const int lx = 4 * m + 2 * set + r;
            if (lx == 0) continue;
            /* block-local ring of B bonds; lx >= 1 never wraps */
            dd1d_attempt(B, bs, lx, P, Q, seed, t, k, (uint64_t)b * n2 + (uint64_t)(wl / 2),
                         2 * (wl % 2) + mm / 4, 8 * (mm % 4),
                         (uint64_t)b * (uint64_t)nt + (uint64_t)m, &h0_unused, net);
        }
    }
    return OR_OK;
}

/* Origin of MCS t of the 1+1-d schedule. */
int or_dd1d_origin(uint64_t seed, uint32_t t, int B)
{
    uint32_t w[4];
    or_draw(seed, OR_TAG_ORIGIN1D, t, 0, 0, w);
    return (int)(((uint64_t)w[0] * (uint64_t)B) >> 32);
}

/* Flat rooftop: s[i] = +1 for even i, -1 for odd i (h(i) = i mod 2). */
int or_flat1d(int L, int8_t *s)
{
    if (L <= 0 || (L & 1)) return OR_EINVAL;
    for (int i = 0; i < L; ++i) s[i] = (i & 1) ? -1 : 1;
    return OR_OK;
}

/* ------------------------------- double tiling at both layers (2+1-d) */

/*
 * The device layer as double tiling instead of dead borders (Sec. 3: the
 * blocks are bisected in both directions into 2^2 sets of non-interacting
 * blocks, the sets updated in turn in a sequence randomized every MCS; the
 * paper uses this for its KMC code and notes that KPZ inherited the
 * work-group scheme from it):
 *
 * MCS t: origin (ox, oy) from (ORIGIN, t, 0, 0) as for dead borders, so the
 * block boundaries move every MCS; block (bx, by) covers the same sites as
 * there, with nbx, nby even.  The four block sets c = (bx mod 2) + 2 (by
 * mod 2) run in the order perm[floor(w0 * 24 / 2^32)] of draw
 * (DTORDER, t, 0, 0), perm = the 24 orderings of (0, 1, 2, 3) in
 * lexicographic order.  In its phase every block of the set makes its 16
 * single-hit steps with the same set, site and acceptance draws as under
 * dead borders, and no site is dead: an update at the block's left column
 * or bottom row flips a slope stored at a site of the (idle) block to the
 * left or below.  Blocks of one set share no slope, so a phase is the same
 * whether its blocks run in parallel or one after the other.
 *
 * Blocks of the next set updated ahead of time (Sec. 3.2, the KMC code's
 * way to fill the device; Sec. 4, the fraction f): with `ahead`, a phase
 * whose next set is its diagonal partner (c ^ 3: both block coordinates of
 * the other parity) takes that set too.  A block's update touches its own
 * sites, the sigma_x column of the block to its left and the sigma_y row of
 * the block below, so diagonal neighbours touch no common slope and the two
 * sets commute.  This mode runs them interleaved, each step first over the
 * partner's blocks and then over the current set's, an order unlike the
 * plain one; the result must equal the plain run exactly.
 */
#define OR_TAG_DTORDER 13u

static void dt_perm(uint32_t w0, int perm[4])
{
    int idx = (int)(((uint64_t)w0 * 24u) >> 32);
    int pool[4] = { 0, 1, 2, 3 };
    int n = 4;
    for (int i = 0; i < 4; ++i) {
        int f = 1;
        for (int k = 2; k < n; ++k) f *= k;          /* (n-1)! */
        const int pick = idx / f;
        idx %= f;
        perm[i] = pool[pick];
        for (int k = pick; k < n - 1; ++k) pool[k] = pool[k + 1];
        --n;
    }
}

int or_dt_perm(uint64_t seed, uint32_t t, int perm[4])
{
    uint32_t w[4];
    or_draw(seed, OR_TAG_DTORDER, t, 0, 0, w);
    dt_perm(w[0], perm);
    return OR_OK;
}

int or_dt_run(int L, double p, double q, uint64_t seed, int Bx, int By, int Tx, int Ty,
              uint32_t t0, int n_mcs, int8_t *sx, int8_t *sy, int64_t *h00, int64_t *net,
              int check, int ahead)
{
    if (!dd_validate(L, Bx, By, Tx, Ty, 1) || n_mcs < 0) return OR_EINVAL;
    const int nbx = L / Bx, nby = L / By;
    if (nbx < 2 || nby < 2 || (nbx & 1) || (nby & 1)) return OR_EINVAL;
    const int ntx = Bx / Tx, nty = By / Ty;
    const int S = Tx * Ty;
    const uint64_t P = threshold(p), Q = threshold(q);
    int64_t *stamp = check ? (int64_t *)malloc(sizeof(int64_t) * (size_t)L * (size_t)L) : NULL;
    if (check && !stamp) return OR_ENOMEM;
    if (check)
        for (size_t i = 0; i < (size_t)L * (size_t)L; ++i) stamp[i] = -1;
    int64_t step_id = 0;
    int status = OR_OK;
    uint32_t w[4];
    for (int m = 0; m < n_mcs && status == OR_OK; ++m) {
        const uint32_t t = t0 + (uint32_t)m;
        or_draw(seed, OR_TAG_ORIGIN, t, 0, 0, w);
        const int ox = (int)(((uint64_t)w[0] * (uint64_t)Bx) >> 32);
        const int oy = (int)(((uint64_t)w[1] * (uint64_t)By) >> 32);
        int perm[4];
        or_dt_perm(seed, t, perm);
        for (int ph = 0; ph < 4 && status == OR_OK; ++ph) {
            /* sets of this phase: the partner first when it is taken ahead */
            int sets[2] = { perm[ph], -1 }, nsets = 1;
            /* ahead = 2 pairs a set with its x neighbour set (c ^ 1) instead:
             * not exact, the negative control of the tests */
            const int partner = perm[ph] ^ (ahead == 2 ? 1 : 3);
            if (ahead && ph + 1 < 4 && perm[ph + 1] == partner) {
                sets[0] = perm[ph + 1];
                sets[1] = perm[ph];
                nsets = 2;
            }
            for (int k = 0; k < S && status == OR_OK; ++k, ++step_id)
              for (int si = 0; si < nsets; ++si) {
                const int csx = sets[si] & 1, csy = sets[si] >> 1;
                for (int by = csy; by < nby; by += 2)
                    for (int bx = csx; bx < nbx; bx += 2) {
                        const int b = by * nbx + bx;
                        or_draw(seed, OR_TAG_SET, t, (uint64_t)b, 0, w);
                        const int s = step_set(w, k);
                        for (int ty = 0; ty < nty; ++ty)
                            for (int tx = 0; tx < ntx; ++tx) {
                                const uint64_t G = row_group(b, ty, tx, nty, ntx);
                                int lx, ly;
                                attempt_site(seed, t, G, k, s, tx, ty, Tx, Ty, &lx, &ly);
                                const int gx = (ox + bx * Bx + lx) % L;
                                const int gy = (oy + by * By + ly) % L;
                                if (check) {
                                    const int nx[5] = { gx, (gx + 1) % L, (gx + L - 1) % L, gx, gx };
                                    const int ny[5] = { gy, gy, gy, (gy + 1) % L, (gy + L - 1) % L };
                                    for (int e = 0; e < 5; ++e)
                                        if (stamp[(size_t)ny[e] * L + nx[e]] == step_id) status = OR_ECHECK;
                                    stamp[(size_t)gy * L + gx] = step_id;
                                }
                                const int kind = classify(L, sx, sy, gx, gy);
                                if (kind == SITE_NONE) continue;
                                if (!accepted(kind, P, Q, seed, t, G, k, tx)) continue;
                                flip(L, sx, sy, gx, gy);
                                const int dh = kind == SITE_MIN ? 2 : -2;
                                *net += dh / 2;
                                if (gx == 0 && gy == 0) *h00 += dh;
                            }
                    }
            }
            if (nsets == 2) ++ph;   /* the partner's phase is done */
        }
    }
    free(stamp);
    return status;
}
