/*
 * kmc.h -- C ABI of the gfx950 kinetic lattice Monte Carlo of a binary alloy
 * (Kelling, Odor, Nagy, Schulz, Heinig, Sec. 2.2 "Kinetic Monte Carlo" and
 * Sec. 3.2 "Implementation of KMC").  Part of libkpz.so.
 *
 * Model:
 *   - Sites: the fcc lattice stored as the sub-lattice of an L x L x L
 *     periodic simple cubic grid, position (x, y, z) being a site iff
 *     (x ^ y ^ z) & 1 == 0 (eq. "fcc"); N = L^3 / 2 sites, each holding
 *     species A (0) or B (1); twelve nearest neighbours, the offsets with two
 *     coordinates +-1 and one 0, numbered
 *       0..3  (+1,+1,0) (+1,-1,0) (-1,+1,0) (-1,-1,0)
 *       4..7  (+1,0,+1) (+1,0,-1) (-1,0,+1) (-1,0,-1)
 *       8..11 (0,+1,+1) (0,+1,-1) (0,-1,+1) (0,-1,-1).
 *   - Attempt (eq. "metropolis", Gamma = 1, both species active as in the
 *     paper's GPU code): site i and neighbour f; if both hold the same
 *     species nothing happens, else the B (on b) jumps to the A (on e) with
 *     probability 1 if n_e >= n_b and exp(-(n_b - n_e) eps) otherwise, n_b =
 *     number of B among b's neighbours and n_e = number of B among e's
 *     neighbours other than b.  The probability is applied as a 32-bit
 *     integer test u < floor(exp(-d eps) 2^32).  This dynamics keeps the
 *     Boltzmann law exp(eps * #B-B bonds) stationary.
 *   - One MCS = N attempts, made by double tiling at both layers: blocks of
 *     B^3 positions in eight sets (block parities), updated set after set in
 *     an order drawn per MCS, the block grid shifted by a random origin per
 *     MCS; inside a block, tiles of 8^3 positions bisected into eight cells
 *     of 4^3, 256 single-hit steps per block (Sec. 3.2, "Implementation of
 *     KMC").  All random numbers are Philox4x32-10 draws keyed by the seed;
 *     results are reproducible and independent of the device.
 *
 * Data layout ("occ"): N bytes, one per fcc site, value 0 (A) or 1 (B).
 * Site (x, y, z) is byte ((z L + y) L/2 + x/2): x fastest, row (y, z)
 * holding the L/2 sites x = (y + z) mod 2 + 2k.
 *
 * Memory, streams and errors follow kpz.h: the caller owns `occ` and the
 * workspace (kmc_workspace_bytes()), the library never allocates device
 * memory, all work goes to the stream given to kmc_init, entry points
 * return a kpz_status and keep HIP error text in the handle.
 */
#ifndef KMC_H_
#define KMC_H_

#include <stddef.h>
#include <stdint.h>

#include "kpz.h"

#ifdef __cplusplus
extern "C" {
#endif

/* L: a power of two, 16 <= L <= 2048.  c: initial concentration of B in
 * [0, 1] (each site is B independently with probability c).  eps: the
 * coupling (inverse effective temperature) of eq. "metropolis", >= 0.
 * block: the device-layer block edge B, 8, 16 or 32 with L / B >= 2;
 * 0 = the largest allowed.  flags must be 0. */
typedef struct {
    int64_t L;
    double c;
    double eps;
    uint64_t seed;
    int32_t block;
    uint32_t flags;
} kmc_params;

typedef struct kmc_sim kmc_sim;

/* Device workspace bytes for these parameters (KPZ_EINVAL if invalid). */
kpz_status kmc_workspace_bytes(const kmc_params *params, size_t *ws_bytes);

/* Creates a handle and enqueues the initial random mixture into d_occ (at
 * least L^3/2 bytes, 4-byte aligned): site s is B iff the first word of the
 * draw (tag 16, t = 0, index s) is below floor(c 2^32).  t = 0, accepted
 * jumps = 0.  d_workspace: kmc_workspace_bytes() bytes, 8-byte aligned.
 * KPZ_EINVAL for a NULL or misaligned buffer, KPZ_ESIZE if one is too
 * small; nothing is enqueued then. */
kpz_status kmc_init(kmc_sim **out, const kmc_params *params, uint8_t *d_occ, size_t occ_bytes,
                    void *d_workspace, size_t workspace_bytes, void *stream);

/* Enqueues n_mcs MCS: eight launches per MCS, one per block set. */
kpz_status kmc_sweep(kmc_sim *sim, int32_t n_mcs);

/* Number of B sites and of B-B nearest-neighbour bonds (exact integers);
 * synchronises the stream. */
kpz_status kmc_counts(kmc_sim *sim, int64_t *n_b, int64_t *bonds);

/* MCS counter and number of accepted jumps so far; synchronises. */
kpz_status kmc_get_state(kmc_sim *sim, int64_t *t, int64_t *moves);

/* Declares that `occ` now holds the state after t MCS with `moves`
 * accepted jumps (for a state the caller wrote into occ); enqueues. */
kpz_status kmc_set_state(kmc_sim *sim, int64_t t, int64_t moves);

void kmc_destroy(kmc_sim *sim);

const char *kmc_last_error(const kmc_sim *sim);

#ifdef __cplusplus
}
#endif

#endif /* KMC_H_ */
