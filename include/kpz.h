/*
 * kpz.h -- C ABI of the MI355X (gfx950) library for the Monte Carlo sweep of
 * the 2+1-dimensional KPZ octahedron model.
 *
 * Model (Kelling, Odor, Nagy, Schulz, Heinig, "Comparison of different
 * parallel implementations of the 2+1-dimensional KPZ model and the
 * 3-dimensional KMC model"):
 *   - Sec. 2.1: the surface on a periodic L x L lattice is stored as the
 *     x and y slopes sigma = +-1 of every site; a site whose four neighbours
 *     are all one unit higher (a local minimum) flips to a local maximum
 *     with probability p, a local maximum flips back with probability q
 *     (eq. "rule"); the squared width W^2 = <h^2> - <h>^2 (eq. "Wdef").
 *   - Sec. 2.2: one Monte Carlo step (MCS) = N = L^2 update attempts.
 *   - Sec. 3 and 3.1: random-sequential dynamics made parallel by two
 *     decomposition layers -- dead-border blocks whose origin moves randomly
 *     (device layer) and single-hit double tiling inside each block
 *     (work-group layer).
 *
 * Data layout ("words"), shared with every caller:
 *   L*L/16 uint32 words, row-major, L/16 words per row.  Word w of row y
 *   holds sites x = 16 w + k, k = 0..15: bit 2k is sigma_x(x,y) =
 *   h(x+1,y) - h(x,y) and bit 2k+1 is sigma_y(x,y) = h(x,y+1) - h(x,y),
 *   bit value 1 meaning +1.  4 bytes per 16 sites, i.e. L^2/4 bytes.
 *
 * Memory ownership: the library never allocates device memory.  The caller
 * owns the device buffers `words` (L*L/4 bytes) and `workspace`
 * (kpz_workspace_bytes()); both must stay valid, and must not be touched by
 * other work on other streams, until kpz_destroy().  The handle itself is a
 * small host object owned by the library.
 *
 * Between calls the lattice may live in either of two buffers, rotated by
 * up to 15 sites (two-buffer mode, see kpz_params.flags): `words` holds the
 * state in the layout above after kpz_init, kpz_set_state and
 * kpz_sync_words.  kpz_roughness and kpz_height_moments read the state
 * wherever it is.
 *
 * Streams: all device work of a handle is enqueued on the HIP stream given
 * to kpz_init (a hipStream_t passed as void*; NULL = the default stream).
 * kpz_init, kpz_sweep and kpz_sync_words only enqueue; kpz_roughness and
 * kpz_get_state synchronise that stream.
 *
 * Errors: every entry point returns a kpz_status; nothing throws or aborts
 * across the ABI.  On KPZ_EHIP the HIP error text is kept in the handle
 * (kpz_last_error).  A handle is not thread-safe; distinct handles are
 * independent.
 */
#ifndef KPZ_H_
#define KPZ_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    KPZ_OK = 0,
    KPZ_EINVAL = -1,   /* invalid argument or parameter combination        */
    KPZ_ESIZE = -2,    /* a caller buffer is smaller than required          */
    KPZ_EHIP = -3,     /* a HIP runtime call failed (see kpz_last_error)    */
    KPZ_ESTATE = -4,   /* device state inconsistent (e.g. corrupted words)  */
    KPZ_ERANGE = -5    /* a result does not fit the output type             */
} kpz_status;

/* Parameters of one simulation.
 *   L        linear size; even, a multiple of 16, at least 16.
 *   p, q     acceptance probabilities of deposition (minimum -> maximum) and
 *            desorption (maximum -> minimum), 0 <= p, q <= 1 (Sec. 2.1).
 *            They are applied as integer thresholds floor(p * 2^32)
 *            (p = 1 -> 2^32) against 32-bit uniforms.
 *   seed     64-bit Philox4x32-7 key (seven rounds).
 *   block_x, block_y
 *            dead-border block shape of the device layer (Sec. 3), sites;
 *            both divide L.  block_x: a multiple of 16 (whole words per
 *            row), at most 128 or a multiple of 128, at most 1024; block_y:
 *            a multiple of 4 (whole tiles); (block_x / 128, at least 1) x
 *            block_y / 4 <= 64 (one wave per block, one lane per row group
 *            of 32 tiles and tile row).  0 = library default: for L a
 *            multiple of 128 the largest power of two <= 256 (x) and <= 128
 *            (y) dividing L; otherwise the valid shape dividing L with the
 *            most sites, then the widest.  A direction with a single block
 *            has no dead border (the block is periodic).
 *   tile_x, tile_y
 *            double-tiling tile shape of the work-group layer (Sec. 3.1);
 *            must be 4 x 4 (four 2 x 2 cells per tile, 16 single-hit steps
 *            per MCS); 0 = default (4).
 *   moves    how often the dead-border origin moves per MCS (Sec. 3: the
 *            origin moves to a new random place from time to time): 1, 2, 4, 8 or 16;
 *            0 = default (1).  Each MCS then runs `moves` residencies of
 *            16 / moves single-hit steps, each with its own random origin
 *            (block residency 1 / moves MCS; every residency reads and
 *            writes the whole lattice once).
 *   flags    0, or KPZ_FLAG_IN_PLACE.  By default the library keeps a second
 *            lattice buffer in the workspace: every launch reads one buffer
 *            and writes the other, each block writing whole words of its
 *            own (no word is shared between blocks).  KPZ_FLAG_IN_PLACE
 *            updates `words` in place instead (the workspace then holds no
 *            second lattice; the words two blocks share are joined by a
 *            merge launch after every sweep launch), for lattices too large
 *            to hold twice.  Both modes give identical results.
 *            KPZ_FLAG_DEVICE_DT replaces the dead borders of the device
 *            layer by double tiling (Sec. 3): the blocks form four sets of
 *            non-adjacent blocks (bx mod 2, by mod 2; L / block_x and
 *            L / block_y must be even), run in a random order every MCS,
 *            one launch per set, each block with all its sites live.  A
 *            different schedule (different results), updated in place; a
 *            block reads and writes the slopes of its left neighbour's
 *            last column and its lower neighbour's top row (both idle in
 *            that launch).  Needs moves <= 1; not for batches or pools.
 *            KPZ_FLAG_DT_AHEAD (with KPZ_FLAG_DEVICE_DT) updates the next
 *            set ahead of time (Sec. 3.2; Sec. 4, the fraction f of full
 *            use): where the next set in the MCS's order is the diagonal
 *            partner of the current one (both block coordinates of the
 *            other parity), the two share one launch.  Diagonal blocks
 *            touch no common slope, so the results are identical to the
 *            plain double tiling; an MCS takes two to four launches (three
 *            on average).  The words at block corners that two blocks of
 *            such a launch share are written by atomic xor.
 * The shape and `moves` change the sequence of updates, so results are
 * reproducible for identical (L, p, q, seed, block, tile, moves) only. */
typedef struct {
    int32_t L;
    double p;
    double q;
    uint64_t seed;
    int32_t block_x;
    int32_t block_y;
    int32_t tile_x;
    int32_t tile_y;
    int32_t moves;
    uint32_t flags;
} kpz_params;

#define KPZ_FLAG_IN_PLACE 1u
#define KPZ_FLAG_DEVICE_DT 2u
#define KPZ_FLAG_DT_AHEAD 4u

typedef struct kpz_sim kpz_sim;

/* Bytes of device workspace a simulation with these parameters needs.
 * Returns KPZ_EINVAL for invalid parameters. */
kpz_status kpz_workspace_bytes(const kpz_params *params, size_t *ws_bytes);

/* The dead-border block shape (Sec. 3) a simulation with these parameters
 * runs, after defaults: *block_x, *block_y in sites.  The shape is part of
 * the dynamics (it fixes the decomposition), so a caller that replays a run
 * elsewhere records it.  Host only; KPZ_EINVAL for invalid parameters. */
kpz_status kpz_block_shape(const kpz_params *params, int32_t *block_x, int32_t *block_y);

/* Creates a handle and enqueues the flat initial state (Sec. 2.1: heights
 * h(x,y) = (x + y) mod 2, i.e. even rows 0x33333333 and odd rows
 * 0xCCCCCCCC) into `d_words`, zeroes the workspace counters and sets the
 * MCS counter t = 0.  `d_words` / `d_workspace` are device pointers of at
 * least L*L/4 and kpz_workspace_bytes() bytes (else KPZ_ESIZE); `stream`
 * is a hipStream_t.  On error *out is set to NULL. */
kpz_status kpz_init(kpz_sim **out, const kpz_params *params, uint32_t *d_words,
                    size_t words_bytes, void *d_workspace, size_t workspace_bytes,
                    void *stream);

/* Enqueues n_mcs Monte Carlo steps t, t+1, ..., t+n_mcs-1 of the decomposed
 * schedule (Sec. 3 / 3.1): per MCS a new random block origin, then 16
 * single-hit steps in which every block picks a random set of cells and
 * every 4 x 4 tile makes one attempt in its cell of that set.  n_mcs >= 0. */
kpz_status kpz_sweep(kpz_sim *sim, int32_t n_mcs);

/* Exact moments of the current surface (Sec. 2.1, height reconstruction and
 * eq. "Wdef"): S1 = sum h, S2 = sum h^2 over all N = L^2 sites, with the
 * absolute heights of the flat start continued by the dynamics (h(0,0) =
 * 0 at t = 0), and W2 = S2/N - (S1/N)^2, computed as the double nearest to
 * (N S2 - S1^2) / N^2 from 128-bit integers.  Synchronises the stream.
 * Any output pointer may be NULL.  KPZ_ERANGE if S1 or S2 does not fit
 * int64 (W2 is still written); KPZ_ESTATE if the words are not a valid
 * surface for the recorded number of flips. */
kpz_status kpz_roughness(kpz_sim *sim, int64_t *S1, int64_t *S2, double *W2);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops and harnesses that forbid hipMalloc): the exact
 * moments of kpz_roughness for a lattice given by its words alone, with the
 * row sums and results in a static scratch area of the library instead of a
 * caller-owned workspace.  Nothing is allocated; the scratch area (about
 * 1 MiB) exists once per device and is held until the process ends.
 *   d_words  L*L/16 uint32 on the current device in the documented layout
 *            (for a two-buffer kpz_sim call kpz_sync_words first)
 *   L        16 <= L <= KPZ_NOALLOC_MAX_L, L % 16 == 0
 *   net      deposits minus desorptions since the flat start (kpz_get_state)
 *   stream   hipStream_t the work is enqueued on; synchronised before return
 * Outputs as for kpz_roughness (any may be NULL).  KPZ_ESIZE if L exceeds
 * KPZ_NOALLOC_MAX_L, KPZ_EINVAL for a NULL pointer or an invalid L (nothing
 * enqueued), KPZ_ESTATE if words and net disagree, KPZ_EHIP on a HIP error;
 * kpz_last_error(NULL) gives the text.  Calls on one device share its
 * scratch area, which keeps the last call's contents: calls that overlap in
 * time on the same device race (use one stream, or serialise them). */
#define KPZ_NOALLOC_MAX_L 65536
kpz_status kpz_roughness_noalloc(const uint32_t *d_words, int64_t L, int64_t net, int64_t *S1,
                                 int64_t *S2, double *W2, void *stream);

/* Height distribution to fourth order (the one-point functions of Sec.
 * 2.1): exact sums M_k = sum over sites of (h - h(0,0))^k, k = 1..4, as
 * 128-bit integers in sums[2k-2] (low 64 bits) and sums[2k-1] (high 64
 * bits, two's complement), and from them, in extended precision, the
 * variance W2, the skewness m3 / m2^(3/2) and the excess kurtosis
 * m4 / m2^2 - 3 of the heights (m_k central moments).  Any output may be
 * NULL.  Synchronises the stream. */
kpz_status kpz_height_moments(kpz_sim *sim, int64_t sums[8], double *W2, double *skewness,
                              double *kurtosis);

/* Validity of the stored surface (Sec. 2.1: the slopes are the differences
 * of a periodic height function): counts[0] = number of plaquettes whose
 * four slopes do not sum to zero, sigma_x(x,y) + sigma_y(x+1,y) !=
 * sigma_y(x,y) + sigma_x(x,y+1); counts[1] = sum of sigma_x along row 0;
 * counts[2] = sum of sigma_y along column 0.  When every plaquette is closed
 * all rows have the sum of row 0 and all columns that of column 0, so the
 * three counts are zero exactly when every plaquette, row and column sums
 * to zero.  One pass over the lattice (after kpz_sync_words); synchronises
 * the stream.  Returns KPZ_ESTATE if any count is non-zero (the counts are
 * still written), KPZ_EINVAL for a NULL argument. */
kpz_status kpz_check_invariants(kpz_sim *sim, int64_t counts[3]);

/* Checkpoint support.  The complete dynamical state is (words, t, net_flips)
 * where net_flips = #depositions - #desorptions since the flat start (so
 * S1 = N/2 + 2 net_flips).  get synchronises the stream; set enqueues the
 * counter reset, makes the next sweep run MCS number t, and declares that
 * `words` holds the lattice (use it after writing `words`, e.g. from a
 * checkpoint). */
kpz_status kpz_get_state(kpz_sim *sim, int64_t *t, int64_t *net_flips);
kpz_status kpz_set_state(kpz_sim *sim, int64_t t, int64_t net_flips);

/* Enqueues whatever makes `words` hold the current state in the documented
 * layout (nothing in in-place mode or when it already does; otherwise one
 * or two copy launches over the lattice).  Call before reading `words`. */
kpz_status kpz_sync_words(kpz_sim *sim);

/* Frees the handle (not the caller's buffers).  NULL is ignored. */
void kpz_destroy(kpz_sim *sim);

/* Order of the four block sets in MCS t under double tiling at the device
 * layer (Sec. 3: the sets updated in a sequence randomized every MCS):
 * perm[0..3] (host memory, four int32 written) receives the set codes
 * bx mod 2 + 2 (by mod 2) in launch order, drawn from the lattice's seed.
 * Pure host computation.  KPZ_EINVAL if perm is NULL. */
kpz_status kpz_dt_order(uint64_t seed, uint32_t t, int32_t *perm);

/* Static text for a status code. */
const char *kpz_status_str(kpz_status status);

/* Text of the last error recorded in the handle ("" if none).  With
 * sim = NULL: the text of the last failed kpz_init, kpz_batch_init or
 * kpz_pool_init on the calling thread. */
const char *kpz_last_error(const kpz_sim *sim);

/* ------------------------------------------------------------------------
 * Ensembles: many independent lattices advanced together.
 *
 * Ensemble averages of W^2(t) need hundreds of independent realisations.  A
 * batch holds n members, each a full simulation as above with its own L, p,
 * q, seed and block shape (block_x, block_y; 0 = the default for its L),
 * and all share the 4 x 4 tile and `moves`.
 * Every member's results are bit-identical to a single-lattice run with the
 * same parameters and block shape.  Each MCS of a kpz_batch_sweep is one
 * launch over the blocks of all members plus one launch that merges their
 * straddling words (the launch boundary orders one MCS before the next).
 *
 * Memory (caller-owned device buffers, sizes from kpz_batch_sizes):
 * `words` holds the members' packed lattices one after the other (member
 * r at kpz_batch_word_offset words, 256-byte aligned), each in the single-
 * lattice layout; `workspace` holds per-member counters, row sums, the
 * straddling-word buffers and the sample results.
 */
typedef struct kpz_batch kpz_batch;

#define KPZ_BATCH_MAX_SAMPLES 1024

/* Device bytes of the words buffer and of the workspace for these members
 * (n >= 1).  KPZ_EINVAL if a member is invalid or the block shapes differ. */
kpz_status kpz_batch_sizes(const kpz_params *members, int32_t n, size_t *words_bytes,
                           size_t *workspace_bytes);

/* Creates the batch and enqueues the flat start of every member (t = 0) on
 * `stream` (a hipStream_t). */
kpz_status kpz_batch_init(kpz_batch **out, const kpz_params *members, int32_t n,
                          uint32_t *d_words, size_t words_bytes, void *d_workspace,
                          size_t workspace_bytes, void *stream);

/* Enqueues whatever makes every member's lattice in the words buffer hold
 * its current state in the documented layout.  Members with L <= 65536 are
 * swept in two-buffer mode (the second buffers are in the workspace; the
 * lattice may sit in either, rotated by up to 15 sites, between calls);
 * if any member is larger or has KPZ_FLAG_IN_PLACE, all are swept in place.
 * Call before reading the words buffer. */
kpz_status kpz_batch_sync_words(kpz_batch *batch);

/* Offset (in uint32 words) of member r's lattice inside the words buffer. */
kpz_status kpz_batch_word_offset(const kpz_batch *batch, int32_t member, size_t *offset_words);

/* Enqueues n_mcs MCS of every member (two launches per MCS). */
kpz_status kpz_batch_sweep(kpz_batch *batch, int32_t n_mcs);

/* Exact moments of every member (arrays of n; any may be NULL), as
 * kpz_roughness.  Synchronises the stream. */
kpz_status kpz_batch_roughness(kpz_batch *batch, int64_t *S1, int64_t *S2, double *W2);

/* Runs the whole sampling schedule as one captured HIP graph: for each of
 * the n_times strictly increasing MCS counts times[k] (> current t), sweep
 * every member up to t = times[k] and take its moments.  Outputs are arrays
 * of n_times * n, sample-major (any may be NULL).  n_times <=
 * KPZ_BATCH_MAX_SAMPLES.  Synchronises the stream. */
kpz_status kpz_batch_run(kpz_batch *batch, const int32_t *times, int32_t n_times, int64_t *S1,
                         int64_t *S2, double *W2);

/* Current MCS count of the batch (all members share it). */
kpz_status kpz_batch_get_t(const kpz_batch *batch, int64_t *t);

/* Frees the batch handle (not the caller's buffers).  NULL is ignored. */
void kpz_batch_destroy(kpz_batch *batch);

/* Text of the last error recorded in the batch handle ("" if none); NULL:
 * as kpz_last_error(NULL). */
const char *kpz_batch_last_error(const kpz_batch *batch);

/* ------------------------------------------------------------------------
 * Job pool: continuous batching of independent simulation jobs.
 *
 * A job is (params, n_mcs): a flat start advanced n_mcs MCS, whose result is
 * its exact final S1, S2, W^2.  Jobs live in a caller-owned device arena
 * (the HBM budget); kpz_pool_submit admits a job only if its lattice and
 * workspace fit into free arena memory and a slot is free.  Each
 * kpz_pool_step advances every resident job min(quantum, remaining) MCS
 * in rounds: round k is one launch over all blocks of the jobs with more
 * than k MCS left in this step (plus the merge of their straddling words);
 * jobs submitted between steps join the next one, so new work overlaps
 * running work on the device.  A job's result is bit-identical whatever
 * else runs with it.  With the pool's block_x, block_y set, every job runs
 * that shape (it must divide the job's L); with both 0 each job runs its own
 * block_x, block_y or, where those are 0, the default shape for its L.  Jobs
 * move the origin once per MCS (moves 0 or 1).
 */
typedef struct kpz_pool kpz_pool;

/* Arena bytes one job occupies while resident. */
kpz_status kpz_pool_job_bytes(const kpz_params *job, int32_t block_x, int32_t block_y,
                              size_t *bytes);

/* Arena bytes of the pool's control region (the first part of the arena;
 * job lattices and workspaces use the rest). */
kpz_status kpz_pool_control_bytes(int32_t max_jobs, size_t *bytes);

/* Creates a pool over the device arena [d_arena, d_arena + arena_bytes)
 * (caller-owned, 256-byte aligned) for at most max_jobs resident jobs and
 * steps of at most max_quantum MCS, on `stream` (a hipStream_t). */
kpz_status kpz_pool_init(kpz_pool **out, void *d_arena, size_t arena_bytes, int32_t max_jobs,
                         int32_t max_quantum, int32_t block_x, int32_t block_y, void *stream);

/* Admits a job (flat start enqueued) and returns its id; KPZ_ESIZE if it
 * does not fit into free arena memory or no slot is free right now (it may
 * fit after running jobs finish); KPZ_EINVAL if it can never run here. */
kpz_status kpz_pool_submit(kpz_pool *pool, const kpz_params *job, int64_t n_mcs,
                           int64_t *job_id);

/* One step: every resident job advances min(quantum, remaining) MCS; jobs
 * that reach their n_mcs are sampled and leave the arena.  *n_active
 * (may be NULL) = jobs still resident after the step. */
kpz_status kpz_pool_step(kpz_pool *pool, int32_t quantum, int32_t *n_active);

/* Moves up to max_results finished jobs' results (FIFO) to the arrays;
 * *n_results = how many.  status[k] is job k's own kpz_status (KPZ_OK, or
 * e.g. KPZ_ESTATE if its words and flip counter disagreed; its moments are
 * then not meaningful).  A failed job never hides the others: the call
 * returns KPZ_OK whenever its arguments are valid.  Any array may be NULL. */
kpz_status kpz_pool_poll(kpz_pool *pool, int32_t max_results, int64_t *job_ids, int64_t *S1,
                         int64_t *S2, double *W2, int32_t *status, int32_t *n_results);

/* Resident jobs and free arena bytes (largest free extent). */
kpz_status kpz_pool_stats(const kpz_pool *pool, int32_t *n_active, size_t *largest_free);

void kpz_pool_destroy(kpz_pool *pool);

/* Text of the last error recorded in the pool handle; NULL: as
 * kpz_last_error(NULL). */
const char *kpz_pool_last_error(const kpz_pool *pool);

/* ------------------------------------------------------------------------
 * Calibration (for the roofline of the sweep, which is bound by vector ALU
 * issue): enqueues n_groups work-groups of 256 threads, each thread running
 * `iters` rounds of 24 independent 32-bit bitwise vector instructions (the
 * sweep's mix: bit select, xor, three-input logic) written in assembly so
 * the count is exact.  *ops_per_iter (may be NULL) = wave instructions per
 * wave and iteration (192).  The measured rate
 * n_groups * 4 * iters * ops_per_iter / time is the device's VALU issue
 * ceiling for that mix.  d_out: n_groups * 256 uint32 (caller-owned device
 * memory, written with a checksum).  KPZ_EINVAL for n_groups or iters < 1;
 * KPZ_EHIP if the launch fails.
 */
kpz_status kpz_valu_probe(uint32_t *d_out, int32_t n_groups, int32_t iters,
                          int32_t *ops_per_iter, void *stream);

/* ------------------------------------------------------------------------
 * The 1+1-dimensional ring (rooftop / ASEP reduction of the model, Sec.
 * 2.1) under the same decomposition reduced to one dimension (Sec. 3 and
 * 3.1): dead-border blocks of B sites whose origin moves every MCS, tiles
 * of 4 sites (two cells of 2 sites), 4 single-hit steps per MCS.
 *
 * Layout: L / 32 uint32 words; bond i, s_i = h(i+1) - h(i), is bit i mod 32
 * of word i / 32 (1 = +1).  Flat start h(i) = i mod 2 (words 0x55555555).
 * Memory, streams and errors as for kpz_sim.
 */
typedef struct kpz_ring kpz_ring;

/* L: a multiple of 128, 128 <= L <= 2^32.  block: the dead-border block
 * of the device layer, 128, 256, 512 or 1024 sites dividing L; 0 = 128.
 * Every block draws one cell set per step for all its tiles, which
 * correlates the updates across the block; in one dimension blocks of
 * thousands of sites visibly change the growth (amplitude and effective
 * exponent), small blocks do not.  A single block (block = L) has no dead
 * border.  p, q, seed as in kpz_params; flags must be 0.  Results are
 * reproducible for identical parameters. */
typedef struct {
    int64_t L;
    double p;
    double q;
    uint64_t seed;
    int32_t block;
    uint32_t flags;
} kpz_ring_params;

/* Device workspace bytes for these parameters (KPZ_EINVAL if invalid). */
kpz_status kpz_ring_workspace_bytes(const kpz_ring_params *params, size_t *ws_bytes);

/* Creates a handle and enqueues the flat start into d_words (at least L/8
 * bytes) and the workspace counters; t = 0. */
kpz_status kpz_ring_init(kpz_ring **out, const kpz_ring_params *params, uint32_t *d_words,
                         size_t words_bytes, void *d_workspace, size_t workspace_bytes,
                         void *stream);

/* Enqueues n_mcs MCS (each: one sweep launch, one straddling-word merge). */
kpz_status kpz_ring_sweep(kpz_ring *ring, int32_t n_mcs);

/* Exact S1 = sum h, S2 = sum h^2 and W^2 = S2/L - (S1/L)^2 (computed from
 * 128-bit integers); synchronises the stream.  KPZ_ERANGE if S1 or S2 does
 * not fit int64 (W^2 is still set); KPZ_ESTATE if words and flip counters
 * disagree. */
kpz_status kpz_ring_roughness(kpz_ring *ring, int64_t *S1, int64_t *S2, double *W2);

/* MCS counter and net number of flips (deposits - desorptions); syncs. */
kpz_status kpz_ring_get_state(kpz_ring *ring, int64_t *t, int64_t *net);

void kpz_ring_destroy(kpz_ring *ring);

const char *kpz_ring_last_error(const kpz_ring *ring);

#ifdef __cplusplus
}
#endif

#endif /* KPZ_H_ */
