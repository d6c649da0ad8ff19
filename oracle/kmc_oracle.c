/*
 * kmc_oracle.c -- TEST INFRASTRUCTURE, NOT PRODUCT CODE.
 *
 * Plain CPU oracle for the paper's second workload, the kinetic lattice
 * Monte Carlo model of a binary alloy (Kelling, Odor, Nagy, Schulz, Heinig,
 * Sec. 2.2 "Kinetic Monte Carlo" and Sec. 3.2 "Implementation of KMC"):
 *
 * Lattice.  An fcc lattice stored as the sub-lattice of an L x L x L simple
 * cubic grid (L even, periodic): position (x, y, z) is a site iff
 * (x ^ y ^ z) & 1 == 0 (eq. "fcc"), i.e. x + y + z even.  Each site holds
 * species A (0) or B (1); the twelve nearest neighbours are the offsets
 * with two coordinates +-1 and one 0, numbered
 *   0..3  (+1,+1,0) (+1,-1,0) (-1,+1,0) (-1,-1,0)
 *   4..7  (+1,0,+1) (+1,0,-1) (-1,0,+1) (-1,0,-1)
 *   8..11 (0,+1,+1) (0,+1,-1) (0,-1,+1) (0,-1,-1).
 *
 * Update attempt (eq. "metropolis" with Gamma = 1, both species active as
 * in the paper's GPU code): a site i and one of its neighbours f are
 * chosen; if they hold the same species nothing happens; otherwise let b be
 * the one holding B and e the one holding A.  With n_b = number of B among
 * b's neighbours and n_e = number of B among e's neighbours other than b
 * (the B's neighbour count after the jump), the B jumps from b to e with
 * probability 1 if n_e >= n_b, else exp(-(n_b - n_e) eps).  (This reading
 * of n_f makes the dynamics satisfy detailed balance with respect to
 * exp(eps * #BB bonds), which the tests check exactly.)  The probabilities
 * are integer thresholds T[d] = floor(exp(-d eps) 2^32), d = 1..12
 * (T[0] = 2^32), compared with a 32-bit uniform.  One MCS = N attempts,
 * N = L^3 / 2 sites.
 *
 * Random numbers: Philox4x32-10, as in kpz_oracle.c (tags 16..20 here).
 *   initial state: site s (fcc index, x fastest) is B iff w0 of
 *                  (KMC_INIT, 0, s, 0) < floor(c 2^32)
 *   random-sequential attempt a of MCS t: (KMC_RS, t, a, 0): site
 *                  floor(w0 N / 2^32), neighbour floor(w1 12 / 2^32), u = w2
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

void or_draw(uint64_t seed, uint32_t tag, uint32_t t, uint64_t idx, uint32_t sub, uint32_t w[4]);

#define KMC_TAG_INIT    16u
#define KMC_TAG_RS      17u
#define KMC_TAG_ORIGIN  18u
#define KMC_TAG_ORDER   19u
#define KMC_TAG_SET     20u
#define KMC_TAG_STEP    21u

#define KMC_OK       0
#define KMC_EINVAL  -1
#define KMC_ENOMEM  -2
#define KMC_ECHECK  -3

static const int NB[12][3] = {
    { 1, 1, 0 }, { 1, -1, 0 }, { -1, 1, 0 }, { -1, -1, 0 },
    { 1, 0, 1 }, { 1, 0, -1 }, { -1, 0, 1 }, { -1, 0, -1 },
    { 0, 1, 1 }, { 0, 1, -1 }, { 0, -1, 1 }, { 0, -1, -1 },
};

static inline int wrap(int v, int L) { return ((v % L) + L) % L; }
static inline size_t pos(int L, int x, int y, int z)
{
    return ((size_t)z * (size_t)L + (size_t)y) * (size_t)L + (size_t)x;
}

/* Thresholds T[d] = floor(exp(-d eps) 2^32) for d = 0..12 (T[0] = 2^32). */
void or_kmc_thresholds(double eps, uint64_t T[13])
{
    T[0] = (uint64_t)1 << 32;
    for (int d = 1; d <= 12; ++d) {
        const double v = exp(-(double)d * eps);
        T[d] = v >= 1.0 ? ((uint64_t)1 << 32) : (uint64_t)(v * 4294967296.0);
    }
}

/* fcc index s -> position: sites in x-fastest order over (z, y, x) with
 * x + y + z even; each row (y, z) holds L/2 sites x = (y + z) % 2 + 2k. */
static void site_pos(int L, uint64_t s, int *x, int *y, int *z)
{
    const uint64_t half = (uint64_t)L / 2;
    const uint64_t row = s / half, k = s % half;
    *y = (int)(row % (uint64_t)L);
    *z = (int)(row / (uint64_t)L);
    *x = (int)(2 * k + (uint64_t)((*y + *z) & 1));
}

int or_kmc_init(int L, double c, uint64_t seed, uint8_t *occ)
{
    if (L < 4 || (L & 1)) return KMC_EINVAL;
    const uint64_t C = c >= 1.0 ? ((uint64_t)1 << 32) : (c <= 0.0 ? 0 : (uint64_t)(c * 4294967296.0));
    memset(occ, 0, (size_t)L * L * L);
    const uint64_t N = (uint64_t)L * L * L / 2;
    uint32_t w[4];
    for (uint64_t s = 0; s < N; ++s) {
        int x, y, z;
        site_pos(L, s, &x, &y, &z);
        or_draw(seed, KMC_TAG_INIT, 0, s, 0, w);
        occ[pos(L, x, y, z)] = (uint64_t)w[0] < C ? 1 : 0;
    }
    return KMC_OK;
}

static int count_b(int L, const uint8_t *occ, int x, int y, int z, int skip_x, int skip_y,
                   int skip_z)
{
    int n = 0;
    for (int k = 0; k < 12; ++k) {
        const int nx = wrap(x + NB[k][0], L), ny = wrap(y + NB[k][1], L), nz = wrap(z + NB[k][2], L);
        if (nx == skip_x && ny == skip_y && nz == skip_z) continue;
        n += occ[pos(L, nx, ny, nz)];
    }
    return n;
}

/* One attempt at site (x, y, z) towards neighbour nb with uniform u;
 * returns 1 if the B moved. */
static int attempt(int L, uint8_t *occ, const uint64_t T[13], int x, int y, int z, int nb,
                   uint32_t u)
{
    const int fx = wrap(x + NB[nb][0], L), fy = wrap(y + NB[nb][1], L), fz = wrap(z + NB[nb][2], L);
    const size_t pi = pos(L, x, y, z), pf = pos(L, fx, fy, fz);
    if (occ[pi] == occ[pf]) return 0;
    int bx = x, by = y, bz = z, ex = fx, ey = fy, ez = fz;
    if (!occ[pi]) {
        bx = fx; by = fy; bz = fz;
        ex = x; ey = y; ez = z;
    }
    const int nb_b = count_b(L, occ, bx, by, bz, -1, -1, -1);
    const int nb_e = count_b(L, occ, ex, ey, ez, bx, by, bz);
    const int d = nb_b - nb_e;
    if (d > 0 && (uint64_t)u >= T[d]) return 0;
    occ[pos(L, bx, by, bz)] = 0;
    occ[pos(L, ex, ey, ez)] = 1;
    return 1;
}

/* Random-sequential dynamics: MCS t0 .. t0 + n_mcs - 1.  *moves counts the
 * accepted jumps. */
int or_kmc_rs_run(int L, double eps, uint64_t seed, uint32_t t0, int n_mcs, uint8_t *occ,
               int64_t *moves)
{
    if (L < 4 || (L & 1) || n_mcs < 0) return KMC_EINVAL;
    uint64_t T[13];
    or_kmc_thresholds(eps, T);
    const uint64_t N = (uint64_t)L * L * L / 2;
    uint32_t w[4];
    for (int m = 0; m < n_mcs; ++m) {
        const uint32_t t = t0 + (uint32_t)m;
        for (uint64_t a = 0; a < N; ++a) {
            or_draw(seed, KMC_TAG_RS, t, a, 0, w);
            const uint64_t s = ((uint64_t)w[0] * N) >> 32;
            const int nb = (int)(((uint64_t)w[1] * 12u) >> 32);
            int x, y, z;
            site_pos(L, s, &x, &y, &z);
            *moves += attempt(L, occ, T, x, y, z, nb, w[2]);
        }
    }
    return KMC_OK;
}

/* Number of B sites and of B-B nearest-neighbour bonds. */
void or_kmc_counts(int L, const uint8_t *occ, int64_t *nB, int64_t *bonds)
{
    int64_t b = 0, e = 0;
    for (int z = 0; z < L; ++z)
        for (int y = 0; y < L; ++y)
            for (int x = (y + z) & 1; x < L; x += 2) {
                if (!occ[pos(L, x, y, z)]) continue;
                ++b;
                e += count_b(L, occ, x, y, z, -1, -1, -1);
            }
    *nB = b;
    *bonds = e / 2;
}

/* One attempt (exported for the tests): site (x, y, z) must be an fcc
 * position; returns 1 if a B jumped, 0 if not, KMC_EINVAL on bad input. */
int or_kmc_attempt(int L, double eps, uint8_t *occ, int x, int y, int z, int nb, uint32_t u)
{
    if (L < 4 || (L & 1) || x < 0 || y < 0 || z < 0 || x >= L || y >= L || z >= L ||
        ((x ^ y ^ z) & 1) || nb < 0 || nb > 11)
        return KMC_EINVAL;
    uint64_t T[13];
    or_kmc_thresholds(eps, T);
    return attempt(L, occ, T, x, y, z, nb, u);
}

/* ------------------------------------------ decomposed schedule (Sec. 3) */

/*
 * Double tiling at both layers, as in the paper's GPU KMC code (Sec. 3.2,
 * "Implementation of KMC"):
 *
 * Device layer.  Blocks of B x B x B cubic positions (B a multiple of 8,
 * L / B even); MCS t shifts the block grid by (ox, oy, oz) =
 * floor(w0..w2 B / 2^32) of (KMC_ORIGIN, t, 0, 0); block (bx, by, bz) covers
 * positions o + (bx, by, bz) B + [0, B)^3 (mod L).  The eight block sets
 * c = (bx & 1) + 2 (by & 1) + 4 (bz & 1) are updated one after the other in
 * the order given by the ordering number floor(w0 40320 / 2^32) of
 * (KMC_ORDER, t, 0, 0), orderings of 0..7 numbered in lexicographic order.
 * Blocks of one set are a whole block apart, so the positions one of them
 * reads or writes (at most two beyond its faces) never meet another's.
 *
 * Work-group layer.  Tiles of 8^3 positions, each bisected into eight cells
 * of 4^3 (cell set s = sx + 2 sy + 4 sz); during its set's turn a block
 * makes 256 single-hit steps (a tile holds 256 sites).  Step k: the block,
 * b = (bz nb + by) nb + bx, takes its cell set from bits 3 (k mod 10) .. +2
 * of w0 of (KMC_SET, t, b, k / 10); tile g (x fastest within the block) of
 * block b, G = b (B/8)^3 + g, takes words 2 (k & 1) and 2 (k & 1) + 1 of
 * (KMC_STEP, t, G, k / 2) as (wa, wb): the site is the r-th fcc site of its
 * set-s cell, r = wa >> 27 (x fastest over the cell's 32 sites), the
 * neighbour floor((wa mod 2^27) 12 / 2^27), u = wb.  Attempts of one step
 * are at least five positions apart along some axis.
 *
 * check != 0 verifies that no two attempts of one step lie within
 * Chebyshev distance 3 (an attempt reads at most two and writes at most one
 * position away from its site); counts, if not NULL, receives per fcc site
 * (fcc index) the number of attempts made at it.
 */
static void or_kmc_perm8(uint32_t w0, int perm[8])
{
    uint64_t idx = ((uint64_t)w0 * 40320u) >> 32;
    int pool[8] = { 0, 1, 2, 3, 4, 5, 6, 7 };
    int n = 8;
    for (int i = 0; i < 8; ++i) {
        uint64_t f = 1;
        for (int k = 2; k < n; ++k) f *= (uint64_t)k;    /* (n-1)! */
        const int pick = (int)(idx / f);
        idx %= f;
        perm[i] = pool[pick];
        for (int k = pick; k < n - 1; ++k) pool[k] = pool[k + 1];
        --n;
    }
}

/* Order of the eight block sets in MCS t. */
void or_kmc_order(uint64_t seed, uint32_t t, int32_t perm[8])
{
    uint32_t w[4];
    int p[8];
    or_draw(seed, KMC_TAG_ORDER, t, 0, 0, w);
    or_kmc_perm8(w[0], p);
    for (int i = 0; i < 8; ++i) perm[i] = p[i];
}

/* Block-grid shift of MCS t. */
void or_kmc_origin(uint64_t seed, uint32_t t, int B, int32_t o[3])
{
    uint32_t w[4];
    or_draw(seed, KMC_TAG_ORIGIN, t, 0, 0, w);
    for (int i = 0; i < 3; ++i) o[i] = (int32_t)(((uint64_t)w[i] * (uint64_t)B) >> 32);
}

int or_kmc_dt_run(int L, double eps, uint64_t seed, int B, uint32_t t0, int n_mcs, uint8_t *occ,
               int64_t *moves, int check, int32_t *counts)
{
    if (L < 16 || (L & 1) || B < 8 || (B & 7) || L % B || ((L / B) & 1) || n_mcs < 0)
        return KMC_EINVAL;
    const int nb = L / B, nt = B / 8, tpb = nt * nt * nt;
    uint64_t T[13];
    or_kmc_thresholds(eps, T);
    int64_t *stamp = check ? (int64_t *)malloc(sizeof(int64_t) * (size_t)L * L * L) : NULL;
    if (check && !stamp) return KMC_ENOMEM;
    if (check)
        for (size_t i = 0; i < (size_t)L * L * L; ++i) stamp[i] = -1;
    int64_t step_id = 0;
    int status = KMC_OK;
    uint32_t w[4], ws[4];
    for (int m = 0; m < n_mcs && status == KMC_OK; ++m) {
        const uint32_t t = t0 + (uint32_t)m;
        int32_t o[3], perm[8];
        or_kmc_origin(seed, t, B, o);
        or_kmc_order(seed, t, perm);
        for (int ph = 0; ph < 8 && status == KMC_OK; ++ph) {
            const int c = perm[ph];
            for (int k = 0; k < 256 && status == KMC_OK; ++k, ++step_id) {
                for (int bz = (c >> 2) & 1; bz < nb; bz += 2)
                    for (int by = (c >> 1) & 1; by < nb; by += 2)
                        for (int bx = c & 1; bx < nb; bx += 2) {
                            const uint64_t b = ((uint64_t)bz * nb + by) * nb + bx;
                            or_draw(seed, KMC_TAG_SET, t, b, (uint32_t)(k / 10), ws);
                            const int s = (int)((ws[0] >> (3 * (k % 10))) & 7u);
                            const int sx = s & 1, sy = (s >> 1) & 1, sz = s >> 2;
                            for (int g = 0; g < tpb; ++g) {
                                const int tx = g % nt, ty = (g / nt) % nt, tz = g / (nt * nt);
                                const uint64_t G = b * (uint64_t)tpb + (uint64_t)g;
                                or_draw(seed, KMC_TAG_STEP, t, G, (uint32_t)(k / 2), w);
                                const uint32_t wa = w[2 * (k & 1)], wb = w[2 * (k & 1) + 1];
                                const int r = (int)(wa >> 27);
                                const int nbr = (int)(((uint64_t)(wa & 0x7FFFFFFu) * 12u) >> 27);
                                /* cell corner (unwrapped) and the r-th fcc site in it */
                                const int X0 = o[0] + bx * B + 8 * tx + 4 * sx;
                                const int Y0 = o[1] + by * B + 8 * ty + 4 * sy;
                                const int Z0 = o[2] + bz * B + 8 * tz + 4 * sz;
                                const int row = r >> 1, ly = row & 3, lz = row >> 2;
                                const int lx = ((X0 + Y0 + Z0 + ly + lz) & 1) + 2 * (r & 1);
                                const int x = wrap(X0 + lx, L), y = wrap(Y0 + ly, L),
                                          z = wrap(Z0 + lz, L);
                                if (check) {
                                    for (int dz = -3; dz <= 3; ++dz)
                                        for (int dy = -3; dy <= 3; ++dy)
                                            for (int dx = -3; dx <= 3; ++dx)
                                                if (stamp[pos(L, wrap(x + dx, L), wrap(y + dy, L),
                                                              wrap(z + dz, L))] == step_id)
                                                    status = KMC_ECHECK;
                                    stamp[pos(L, x, y, z)] = step_id;
                                }
                                if (counts)
                                    ++counts[((size_t)z * L + (size_t)y) * (size_t)(L / 2) +
                                             (size_t)(x >> 1)];
                                *moves += attempt(L, occ, T, x, y, z, nbr, wb);
                            }
                        }
            }
        }
    }
    free(stamp);
    return status;
}
