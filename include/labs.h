/*
 * labs.h -- C ABI of the MI355X (gfx950) LABS dual-step library, liblabs.so.
 *
 * The operations follow the problem statement of Psenicnik, Mlinaric, Brest and
 * Boskovic, "Dual-Step Optimization for Binary Sequences with High Merit
 * Factors" (arXiv 2409.07222):
 *   Sec. 1    S = (s_1..s_L), s_i in {+1,-1}; C_k(S) = sum_{i=1}^{L-k} s_i s_{i+k};
 *             E(S) = sum_{k=1}^{L-1} C_k^2; Eq. (1) F = L^2 / (2E).
 *   Eq. (2)   skew-symmetry for L = 2k+1: s_{k+1+i} = (-1)^i s_{k+1-i}, i = 1..k.
 *   Eq. (3)   restriction classes: s_1..s_p fixed, s_{p+1}..s_{k+1} free, the
 *             last k elements set by Eq. (2).
 *   Alg. 1    first step: walks over skew neighbours (one free element and its
 *             Eq. (2) partner flipped), best neighbour each step, sieve by energy.
 *   Alg. 2    second step: best-first search over all L single flips, driven by
 *             a priority queue keyed by E.
 *
 * Conventions shared by every entry point
 *   Packed sequences: W = labs_words(L) = ceil(L/32) uint32 words per sequence;
 *     s_i is bit 31 - ((i-1) mod 32) of word (i-1)/32, set for +1, clear for -1;
 *     the unused low bits of the last word must be zero.  Sequence j of a batch
 *     starts at word j*W.  Read MSB first the words spell s_1, s_2, ... -- the
 *     digit order of the paper's hexadecimal coding (Sec. 4).
 *   Order of sequences ("key order"): ascending (E, key) where key is the packed
 *     words compared as unsigned integers, word 0 first.
 *   Pointers: every array argument is DEVICE memory unless marked "host".  The
 *     caller owns all memory; the library allocates nothing except where an entry
 *     point says so.
 *   Streams: `stream` is a hipStream_t passed as void* (NULL = default stream).
 *     Calls enqueue work and return; results are valid once the stream has
 *     synchronised, except where an entry point says it synchronises.
 *   Errors: arguments are validated before anything is enqueued; on
 *     LABS_E_INVALID nothing was written.  HIP failures return LABS_E_DEVICE.
 *     labs_last_error() returns a description of the last failure on the
 *     calling thread.  No C++ exception crosses this interface.
 *   Limits: odd L for skew operations; 1 <= L <= 1023 for energies and deltas;
 *     first-step walks need 5 <= L <= 639 (at most 10 words of even lags);
 *     second-step searches 2 <= L <= 1023;
 *     |C_k| <= L-1 and E < 2^31 for every L accepted.
 */
#ifndef LABS_H
#define LABS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LABS_ABI_VERSION 2

typedef int32_t labs_status;
enum {
    LABS_OK = 0,
    LABS_E_INVALID = -1,     /* bad argument; nothing enqueued */
    LABS_E_DEVICE = -2,      /* HIP runtime or launch failure */
    LABS_E_NOMEM = -3,       /* workspace too small */
    LABS_E_UNSUPPORTED = -4  /* valid request outside what the library implements */
};

int32_t labs_abi_version(void);
const char* labs_status_str(labs_status s);
/* Text of the last failure on this thread ("" when none).  The pointer stays
 * valid until the next library call on the same thread. */
const char* labs_last_error(void);
/* ceil(L/32): words per packed sequence. */
int32_t labs_words(int32_t L);

/* ----------------------------------------------------------------------------
 * labs_energy -- Sec. 1 definitions: E(S) and optionally every C_k(S).
 *   L       sequence length, 1..1023
 *   n       number of sequences (0 allowed: nothing is done)
 *   seqs    [n*W] packed sequences (device, read)
 *   E       [n] int32 energies (device, written)
 *   C       [n*(L-1)] int32, C_1..C_{L-1} of sequence j at j*(L-1) (device,
 *           written; may be NULL)
 */
labs_status labs_energy(int32_t L, int64_t n, const uint32_t* seqs, int32_t* E, int32_t* C,
                        void* stream);

/* ----------------------------------------------------------------------------
 * labs_flip_deltas -- exact energy change of every neighbour, E(S') - E(S).
 *   skew = 0: the L single flips of Alg. 2's neighbourhood; dE is [n*L], entry
 *             j*L + (i-1) for the flip of s_i.  p is ignored.
 *   skew = 1: the skew neighbours of Alg. 1 over the free positions of Eq. (3):
 *             a = p+1..k+1 (k = (L-1)/2, L odd), flipping s_a together with its
 *             Eq. (2) partner s_{L+1-a} (the centre a = k+1 alone); dE is
 *             [n*(k+1-p)], entry j*(k+1-p) + (a-p-1).  The change is exact for
 *             any input sequence, skew-symmetric or not.
 */
labs_status labs_flip_deltas(int32_t L, int32_t p, int32_t skew, int64_t n,
                             const uint32_t* seqs, int32_t* dE, void* stream);

/* ----------------------------------------------------------------------------
 * First step (Alg. 1 with a tabu tenure in place of the Bloom filter).
 *
 * Walker w (global id walker_begin + j, j = 0..n_walkers-1) starts from a
 * seeded skew-symmetric sequence in a seeded restriction class: it reads the
 * SplitMix64 stream (Steele, Lea, Flood 2014) whose state starts at
 *   key = mix(seed ^ mix((L << 32) ^ (w + 1))),  mix = SplitMix64's finaliser,
 * output i (i = 0, 1, ...) being mix(key + (i+1) * 0x9E3779B97F4A7C15).
 * Output i-1 sets s_i (+1 when its top bit is set) for i = 1..k+1, except that
 * s_1 = +1 when p >= 1; output k+1 draws the tenure
 * tenure_lo + (output mod (tenure_hi - tenure_lo + 1)).  Eq. (2) sets the rest.
 * Then, for t = 1..steps: every free position a = p+1..k+1 is evaluated
 * (dE_a = E(flip_skew_a S) - E(S)); the admissible ones are those with
 * tabu_until[a] < t (initially 0); the walker takes the admissible a with the
 * lowest (dE_a, a), even uphill, sets tabu_until[a] = t + tenure and E += dE_a.
 * With no admissible position the walk stops; its remaining trajectory is -1.
 * Sieve: after each move, a sequence with E <= e_max is offered to the pool.
 * Results depend only on (seed, L, p, tenures, steps, walker id): any split of
 * the walker range gives the same per-walker results.
 */
typedef struct {
    int32_t L;            /* odd, 5..639 */
    int32_t p;            /* restriction prefix length, 0..k-1 (at least 2 free positions) */
    int32_t steps;        /* steps per walker; 0 = the paper's default 4(L+1) */
    int32_t tenure_lo;    /* tabu tenure range, 0 <= lo <= hi < k+1-p */
    int32_t tenure_hi;
    int32_t e_max;        /* sieve threshold (E <= e_max enters the pool); < 0: no pool */
    int64_t walker_begin; /* first global walker id, >= 0 */
    int64_t n_walkers;    /* >= 1; walker ids must stay below 2^31 */
    uint64_t seed;
    uint32_t flags;       /* bit 0 LABS_POOL_WALKER_BEST: also offer each walker's best
                             sequence (the first step reaching its lowest energy, the
                             initial sequence counted as step 0) to the pool at the end */
    int32_t reserved;     /* must be 0 */
} labs_step1_cfg;

#define LABS_POOL_WALKER_BEST 1u

/* Candidate pool (caller-allocated, device).  On return from a call that fills
 * it, the pool holds the min(capacity, D) smallest, in key order, of the D
 * distinct sequences in (its previous contents) U (this call's offers), sorted
 * ascending; `walker`/`step` of an entry are those of its earliest offer in
 * (walker, step) order.  Overflow is not an error: *dropped grows by D minus
 * the entries kept, the number of distinct sequences the capacity cut (a
 * sequence offered again after it was cut counts once).  The library keeps the
 * cut sequences of the call in a set inside the workspace, exact for up to
 * capacity + staging (>= capacity + 65536) distinct cut sequences per call;
 * beyond that the call completes the walk and the pool but returns
 * LABS_E_NOMEM, since *dropped is then not exact. */
typedef struct {
    uint32_t* seqs;     /* [capacity*W] */
    int32_t* E;         /* [capacity] */
    int64_t* walker;    /* [capacity], may be NULL */
    int32_t* step;      /* [capacity], may be NULL */
    int64_t capacity;   /* >= 1 */
    int64_t* count;     /* device int64: entries held (read on entry, written) */
    int64_t* dropped;   /* device int64: incremented */
} labs_pool;

typedef struct {
    uint32_t* final_seqs;  /* [n*W] sequence after the last step */
    int32_t* final_E;      /* [n] */
    uint32_t* best_seqs;   /* [n*W] first sequence of least energy (may be NULL) */
    int32_t* best_E;       /* [n] (may be NULL) */
    int32_t* best_step;    /* [n] step of best (0 = initial), may be NULL */
    int32_t* traj_E;       /* [n*steps] energy after step t at j*steps + t-1, may be NULL */
    int64_t* flip_evals;   /* device int64, incremented by (steps taken)*(k+1-p) per walker;
                              may be NULL */
    /* First-hit stamps of the device's constant-rate real-time counter (the
     * s_memrealtime clock; labs_realtime_hz gives its rate).  With n_levels in
     * 1..LABS_MAX_LEVELS, first_hit_ticks[l] (device uint64, caller-initialised,
     * e.g. to UINT64_MAX) is lowered, by atomic min, to the counter's value when a
     * walker's energy first reaches E <= level_E[l] (the initial sequence
     * counted); start_ticks (device uint64, caller-initialised) is lowered to the
     * counter's value as the call's walker-init kernel starts.  A walker that
     * stays at or below a level re-stamps it at most once per launch, later, so
     * the minimum is its first hit.  The stamps accumulate across calls that
     * share the buffers.  n_levels = 0: no stamps (both pointers ignored). */
    int32_t n_levels;
    int32_t level_E[16];
    uint64_t* first_hit_ticks;
    uint64_t* start_ticks;
} labs_step1_out;

#define LABS_MAX_LEVELS 16

/* Rate of the real-time counter the first-hit stamps read, in ticks per second,
 * for the current device.  Host call. */
labs_status labs_realtime_hz(int64_t* hz);

/* Workspace bytes for labs_walk_step1 with these configurations and pools of at
 * most pool_capacity entries (ignored when no cfg has e_max >= 0).  Host call. */
labs_status labs_walk_step1_workspace(const labs_step1_cfg* cfg, int32_t n_cfg,
                                      int64_t pool_capacity, size_t* bytes);

/* Run the first step.  cfg, pools and outs are HOST arrays of n_cfg structs;
 * prop must be NULL (plain walker).
 *   n_cfg = 1: one configuration in segmented launches of one wavefront per
 *     walker; pools may be NULL when e_max < 0.  When a pool is used the call
 *     synchronises `stream` between walk segments and returns after the pool is
 *     final.
 *   n_cfg > 1: a batch of configurations of any (odd) lengths in one
 *     hipGraph-captured launch: per shape class of the walker kernel, a
 *     persistent kernel drains a queue of (configuration, walker) items, the
 *     most expensive first.  Every cfg must have e_max < 0 and flags = 0, and
 *     pools must be NULL.  The graph is cached per (cfg, outs, workspace) and
 *     replayed on identical calls; the call returns without synchronising.
 *   Per-walker results are identical in both forms. */
labs_status labs_walk_step1(const labs_step1_cfg* cfg, int32_t n_cfg, const void* prop,
                            labs_pool* pools, labs_step1_out* outs, void* ws, size_t ws_bytes,
                            void* stream);

/* ----------------------------------------------------------------------------
 * First step with the Bloom filter of Alg. 1 (Sec. 3) in place of the tabu
 * tenure.  The walker, its stream, its initial sequence and the sieve are those
 * of labs_walk_step1; tenure_lo and tenure_hi must be 0.  Each walker owns a
 * Bloom filter (Bloom 1970) of m = 2^log2_bits bits.  A sequence is keyed by
 *   h(S) = XOR of Z_i over i = 1..k+1 with s_i = +1,
 * Z_i being output i-1 of the SplitMix64 stream whose state starts at
 * 0x6A09E667F3BCC909 (the table the second step keys sequences with), and a key
 * sets / tests the n_hash bits (g1 + j g2) mod m, j = 0..n_hash-1, with g1 the
 * low 32 bits of h, g2 its high 32 bits with the lowest bit set, arithmetic
 * modulo 2^32 (double hashing, Kirsch and Mitzenmacher 2006).  The initial
 * sequence is inserted; at step t every free position a = p+1..k+1 is evaluated,
 * a neighbour is unexplored when its key is not in the filter, the walker takes
 * the unexplored a with the lowest (dE_a, a), even uphill, inserts the new
 * sequence and E += dE_a; with no unexplored neighbour the walk stops (its
 * remaining trajectory is -1).  The filter sits in LDS for each launch segment
 * and in the workspace (n_walkers * m / 8 bytes) between segments.
 * steps = 0 is the paper's T_i = 4(L+1).  One configuration per call; pool and
 * outputs as in labs_walk_step1 with n_cfg = 1, results again independent of
 * how the walker range is split.
 */
typedef struct {
    int32_t log2_bits;    /* filter bits per walker m = 2^log2_bits, 6..18 */
    int32_t n_hash;       /* bits set and tested per key, 1..16 */
    int32_t reserved[2];  /* must be 0 */
} labs_bloom;

labs_status labs_walk_step1_bloom_workspace(const labs_step1_cfg* cfg, const labs_bloom* bloom,
                                            int64_t pool_capacity, size_t* bytes);
labs_status labs_walk_step1_bloom(const labs_step1_cfg* cfg, const labs_bloom* bloom, labs_pool* pool,
                                  labs_step1_out* out, void* ws, size_t ws_bytes, void* stream);

/* ----------------------------------------------------------------------------
 * Autotuner of the walker's tiles.  A shape class is (NW, R): NW = ceil(k/32)
 * words of even lags and R = ceil((k+1-p)/64) free positions per lane.  Its tile
 * is RB, the slots a lane scans per pass (R, or ceil(R/2) to free registers for
 * occupancy), and the resident waves per SIMD requested by persistent launches
 * (1, 2, 3, 4 or 8).  Untuned, RB is R unless that kernel keeps at most three
 * waves per SIMD resident and the ceil(R/2) kernel keeps more, and persistent
 * launches request 2 waves per SIMD.  labs_autotune_step1 times every candidate tile on the largest
 * length of each class among Ls (host array of n_L odd lengths) with `walkers`
 * walkers x `steps` steps, and keeps the fastest in a process-wide table used by
 * every later walk.  It allocates and frees its own scratch and synchronises
 * `stream`.  The table can be written to / read from a JSON file; labs_autotune_get
 * reports the tile used for (L, p) (host outputs).
 */
labs_status labs_autotune_step1(const int32_t* Ls, int32_t n_L, int32_t p, int32_t walkers,
                                int32_t steps, void* stream);
labs_status labs_autotune_save(const char* path);
labs_status labs_autotune_load(const char* path);
labs_status labs_autotune_get(int32_t L, int32_t p, int32_t* rb, int32_t* waves_per_simd);

/* ----------------------------------------------------------------------------
 * labs_pool_topk -- the k smallest distinct sequences of a pool in key order.
 *   pool     as above; reads pool->count (entries 0..count-1, any order, duplicates
 *            allowed)
 *   out_seqs [k*W], out_E [k] (device, written), out_n (device int64: number written,
 *            min(k, distinct))
 *   ws       workspace of labs_pool_topk_workspace(pool->capacity, L) bytes
 * Synchronises `stream` (it reads pool->count).
 */
labs_status labs_pool_topk_workspace(int64_t capacity, int32_t L, size_t* bytes);
labs_status labs_pool_topk(const labs_pool* pool, int32_t L, int32_t k, uint32_t* out_seqs,
                           int32_t* out_E, int64_t* out_n, void* ws, size_t ws_bytes,
                           void* stream);

/* labs_pool_topk_noalloc -- labs_pool_topk for callers that cannot allocate
 * device memory (code under stream capture, tight serving loops, harnesses that
 * forbid allocation).  Same arguments, results and ordering, without the
 * workspace: the sort's scratch is a fixed 64 MiB device array inside the
 * library, one per GPU, held until the process ends.  A pool whose count needs
 * more scratch than that (about 700,000 entries at L = 501) is rejected with
 * LABS_E_INVALID before any launch.  Calls on one GPU share that array, so calls
 * that overlap in time on one GPU (several streams or host threads) race; the
 * library keeps no state between calls in it.  Allocates nothing; synchronises
 * `stream` (it reads pool->count).
 */
labs_status labs_pool_topk_noalloc(const labs_pool* pool, int32_t L, int32_t k, uint32_t* out_seqs,
                                   int32_t* out_E, int64_t* out_n, void* stream);

/* ----------------------------------------------------------------------------
 * Second step (Alg. 2) as a batch-synchronous best-first search.
 *
 * Order in this step: (E, z, sequence) with z the sequence's Zobrist key: the
 * XOR, over the positions i with s_i = +1, of output i-1 of the SplitMix64
 * stream started at state 0x6A09E667F3BCC909, with its lowest bit set.  (Ties in
 * energy are unspecified by the paper; a pseudo-random tie order keeps the
 * selection cheap on the GPU.)
 * Open (the priority queue) starts as the distinct candidates, cut to the
 * pq_capacity smallest; Closed starts empty; best = min(Open).
 * While Open is non-empty, expansions < max_expansions and u < T_u, a round:
 *   - pops the min(batch, max_expansions - expansions) smallest Open entries
 *     into Closed (expansions grows by their number);
 *   - expands every single flip s_i -> -s_i (i = 1..L) of every popped pivot; a
 *     neighbour already in Closed, in Open or produced earlier in this round is
 *     skipped (Alg. 2's PQ.contains test, by exact sequence); the others are
 *     pushed with their exact energy;
 *   - with T_r > 0 (MAKE_ROTATIONS, rotations of the pivot), after every single
 *     flip of the round each pivot also produces its cyclic rotations left by
 *     1..T_r (the first element moved to the end, repeatedly), then right by
 *     1..T_r, skipped or pushed by the same rule;
 *   - if the round's smallest pushed energy is below best's, best becomes the
 *     smallest pushed entry and u = 0; otherwise u grows by the
 *     number of pivots (u counts pops since the last strict improvement; with
 *     batch = 1 this is Alg. 2's dynamic depth exactly);
 *   - cuts Open to the pq_capacity smallest (evicted sequences are forgotten
 *     and may be pushed again later).
 * Alg. 2's queue has no capacity: that is the case pq_capacity >= n_cand +
 * max_expansions (L + 2 T_r), where no cut ever evicts (Open cannot outgrow it),
 * so a sequence is pushed at most once.
 * Results do not depend on scheduling.  The call synchronises `stream`.
 * Memory: the workspace holds two hash tables of next_pow2(4 x (n_cand +
 * max_expansions + pq_capacity + 9 batch (L + 2 T_r))) slots of 16 + 4W bytes
 * (10.7 GB at 10^7 expansions of L = 501); configurations whose table would pass
 * 2^31 slots are rejected (LABS_E_INVALID).
 */
typedef struct {
    int32_t L;               /* 2..1023 */
    int32_t batch;           /* pivots per round, >= 1 */
    int32_t T_r;             /* rotations per side, 0..32 with 2 T_r < L (0: none) */
    int32_t reserved;        /* must be 0 */
    int64_t pq_capacity;     /* Q >= 1 */
    int64_t max_expansions;  /* >= 0 */
    int64_t T_u;             /* >= 1 */
} labs_step2_cfg;

typedef struct {
    int64_t expansions;      /* pivots popped */
    int64_t pushes;          /* neighbours pushed (new or re-pushed after eviction) */
    int64_t dup_skips;       /* neighbours skipped as already present */
    int64_t evictions;       /* entries cut by the capacity in the rounds (seeds beyond Q are
                                not admitted, not evicted) */
    int64_t rounds;
    int64_t open_count;      /* Open entries at the end */
    int32_t best_E;
    int32_t best_round;      /* round of the last improvement, -1 if none */
    int64_t rebuilds;        /* rebuilds of the hash set (evicted tombstones dropped); they
                                change no result */
} labs_step2_stats;

typedef struct {
    uint32_t* best_seq;      /* [W] (device) */
    int32_t* best_E;         /* [1] (device) */
    labs_step2_stats* stats; /* device */
    uint32_t* open_seqs;     /* [open_capacity*W] Open at exit, any order (may be NULL) */
    int32_t* open_E;         /* [open_capacity] (may be NULL) */
    int64_t open_capacity;   /* entries written: min(open_count, open_capacity) */
} labs_step2_out;

labs_status labs_refine_step2_workspace(const labs_step2_cfg* cfg, int64_t n_cand, size_t* bytes);
/* cand_seqs: [n_cand*W] packed candidates (device), n_cand >= 1. */
labs_status labs_refine_step2(const labs_step2_cfg* cfg, int64_t n_cand, const uint32_t* cand_seqs,
                              const labs_step2_out* out, void* ws, size_t ws_bytes, void* stream);

/* ----------------------------------------------------------------------------
 * Legendre-construction seeds of the second step (Sec. 4.1).  A pair (n, o) of
 * an odd prime n and a rotation 0 <= o < n gives the length-L sequence
 *   s_j = chi((j + o) mod n),  j = 0..L-1,
 * chi(a) = +1 for the non-zero quadratic residues mod n and -1 otherwise,
 * chi(0) = -1: a Legendre sequence rotated by o with its first L - n elements
 * appended (periodic extension).  The sweep (a reading of the section's ranges,
 * which hold no prime at most lengths) takes every odd prime n <= L with
 * t_lo <= 10^4 (L - n)/n <= t_hi and every o with r_lo <= 10^4 o/n <= r_hi, in
 * (n, o) order; sweep = NULL means {0, 900, 1800, 2600}, whose best pair gives
 * the construction column of the section's table at L = 450, 471, 491, 526.
 *
 * labs_legendre_pairs (host only): writes up to `capacity` pairs to the HOST
 * arrays n_out / o_out and sets *count to the number of pairs in the sweep.
 * labs_legendre_build: for the n_pairs HOST pairs (validated: n an odd prime <=
 * 1023, 0 <= o < n), writes the packed sequences [n_pairs*W] and their energies
 * [n_pairs] to DEVICE arrays; the workspace (labs_legendre_build_workspace
 * bytes, device) holds the pairs on the device.  2 <= L <= 1023.  The call
 * synchronises `stream`.  The sequences feed labs_refine_step2 as candidates.
 */
typedef struct {
    int32_t t_lo, t_hi;   /* appended fraction (L - n)/n, in 1/10^4 */
    int32_t r_lo, r_hi;   /* rotation o/n, in 1/10^4, <= 10^4 */
} labs_legendre_sweep;

labs_status labs_legendre_pairs(int32_t L, const labs_legendre_sweep* sweep, int32_t* n_out,
                                int32_t* o_out, int64_t capacity, int64_t* count);
labs_status labs_legendre_build_workspace(int64_t n_pairs, size_t* bytes);
labs_status labs_legendre_build(int32_t L, int64_t n_pairs, const int32_t* n, const int32_t* o,
                                uint32_t* seqs, int32_t* E, void* ws, size_t ws_bytes, void* stream);

/* ----------------------------------------------------------------------------
 * End operators (Sec. 3: the operators that extend the search to even lengths
 * by removing or appending elements at either end of a sequence).  For each of
 * the n packed sequences of length L (device), writes
 *   minus[(2j + q)*W(L-1)]: q = 0 without its first element, q = 1 without its last;
 *   plus [(4j + q)*W(L+1)]: q = 0 +1 before the first element, q = 1 -1 before it,
 *                           q = 2 +1 after the last element,   q = 3 -1 after it;
 * and their energies E_minus[2n], E_plus[4n] (all device).  1 <= L <= 1022; for
 * L = 1 minus and E_minus are not written (may be NULL).  Asynchronous on `stream`.
 * The results feed labs_refine_step2 at L - 1 and L + 1.
 */
labs_status labs_length_operators(int32_t L, int64_t n, const uint32_t* seqs, uint32_t* minus,
                                  int32_t* E_minus, uint32_t* plus, int32_t* E_plus, void* stream);

/* ----------------------------------------------------------------------------
 * Launch timing (diagnostics).  While enabled, every launch of a timed kernel
 * is bracketed by HIP events on the stream it runs on, and the entry point
 * that launched it synchronises that stream before returning and adds the
 * elapsed times to a process-wide table.  Timed kernel names: "walk" (the
 * first-step scan/apply kernel), "walk_batched" (a whole batched launch),
 * "expand" (the second-step expansion kernel).  total_ms and launches are HOST outputs.
 */
labs_status labs_timing_enable(int32_t on);
labs_status labs_timing_reset(void);
labs_status labs_timing_read(const char* kernel, double* total_ms, int64_t* launches);


/* ============================================================================
 * Learned flip proposal.  Not part of the paper's method: a small network
 * reorders which skew flips (Alg. 1 neighbourhood, Eq. (2) partners) receive an
 * exact energy evaluation; every accepted move is still scored exactly.
 *
 * Network: x -> GELU(W1 x + b1) -> GELU(W2 h1 + b2) -> W3 h2 + b3, GELU in its
 * tanh form.  For odd L = 2k+1:
 *   x  (d_in = L + k values)   s_1..s_L as +1/-1, then C_{2m}/(L-2m), m = 1..k
 *   z  (d_out = k + 1 logits)  logit j scores the skew flip of position j+1
 * Products take bfloat16 operands (round to nearest even) and accumulate in
 * FP32; biases, pre-activations and logits are FP32; hidden activations are
 * stored as bf16.
 *
 * Parameter blob: one FP32 array of n_params elements (the masters) and a bf16
 * copy with the same offsets (the product operands; its bias slots are unused):
 *   W1 [hidden][ld_in] at off_W1     b1 [hidden] at off_b1
 *   W2 [hidden][hidden] at off_W2    b2 [hidden] at off_b2
 *   W3 [ld_out][hidden] at off_W3    b3 [ld_out] at off_b3
 * Pad columns of W1 (d_in..ld_in-1) and pad rows of W3 / entries of b3
 * (d_out..ld_out-1) do not affect any result.
 * Feature rows X are bf16 (uint16 bit patterns) with row stride ld_in, pads 0.
 * Logit rows have stride ld_out; their pad columns are not written.
 * Admissibility masks: mask_words uint32 per row, bit (j mod 32) of word j/32
 * set when logit j may be chosen.  Labels: int32 in [0, d_out).
 * -------------------------------------------------------------------------- */
typedef struct {
    int32_t L, k, d_in, d_out, hidden;
    int32_t ld_in;        /* d_in rounded up to a multiple of 64 */
    int32_t ld_out;       /* d_out rounded up to a multiple of 64 */
    int32_t mask_words;   /* ceil(d_out / 32) */
    int64_t off_W1, off_b1, off_W2, off_b2, off_W3, off_b3;
    int64_t n_params;     /* elements of the blob (each slice 64-aligned) */
} labs_mlp_layout;

/* Host-only.  L odd in [5, 1023]; hidden a multiple of 64 in [64, 1024]. */
labs_status labs_mlp_layout_of(int32_t L, int32_t hidden, labs_mlp_layout* out);

/* Features of n packed sequences of length L (odd): X [n*ld_in] bf16, written. */
labs_status labs_mlp_features(int32_t L, int64_t n, const uint32_t* seqs, uint16_t* X, void* stream);

/* Forward pass: logits [n*ld_out] FP32 from features X [n*ld_in].
 *   params       FP32 blob (biases are read from it)
 *   params_bf16  bf16 blob (weights are read from it)
 *   ws           scratch of labs_mlp_forward_workspace bytes (device) */
labs_status labs_mlp_forward_workspace(const labs_mlp_layout* lay, int64_t n, size_t* bytes);
labs_status labs_mlp_forward(const labs_mlp_layout* lay, const float* params, const uint16_t* params_bf16,
                             int64_t n, const uint16_t* X, float* logits, void* ws, size_t ws_bytes,
                             void* stream);

/* Gradients of the mean masked softmax cross-entropy over n rows:
 *   loss_r = logsumexp_{j admissible} z_rj - z_r,label   (the label always counts
 *   as admissible), loss = mean_r loss_r.
 * grads (FP32 blob, every element overwritten; pads 0) and *loss (device float)
 * are written.  The backward products use the same bf16 rounding as the
 * forward, applied to the upstream gradient too; bias gradients sum FP32 values. */
labs_status labs_mlp_grads_workspace(const labs_mlp_layout* lay, int64_t n, size_t* bytes);
labs_status labs_mlp_grads(const labs_mlp_layout* lay, const float* params, const uint16_t* params_bf16,
                           int64_t n, const uint16_t* X, const uint32_t* mask, const int32_t* labels,
                           float* grads, float* loss, void* ws, size_t ws_bytes, void* stream);

/* One Adam step (Kingma and Ba 2015) over the whole blob, t >= 1 counting from 1:
 *   m = b1 m + (1-b1) g;  v = b2 v + ((1-b2) g) g;
 *   p -= lr (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps)
 * in FP32 with each operation rounded separately (constants rounded to FP32
 * once: b1, 1-b1, b2, 1-b2, 1-b^t, lr, eps); params_bf16 is refreshed. */
labs_status labs_mlp_adam(const labs_mlp_layout* lay, float* params, uint16_t* params_bf16,
                          const float* grads, float* m, float* v, int32_t t, double lr, double beta1,
                          double beta2, double eps, void* stream);

/* params_bf16 = bf16(params), elementwise. */
labs_status labs_mlp_cast(const labs_mlp_layout* lay, const float* params, uint16_t* params_bf16,
                          void* stream);

/* One training step on logged walker states: features of seqs [n*W], then
 * labs_mlp_grads, then labs_mlp_adam with step t.  grads is written. */
labs_status labs_mlp_train_workspace(const labs_mlp_layout* lay, int64_t n, size_t* bytes);
labs_status labs_mlp_train_step(const labs_mlp_layout* lay, float* params, uint16_t* params_bf16,
                                float* grads, float* m, float* v, int32_t t, double lr, double beta1,
                                double beta2, double eps, int64_t n, const uint32_t* seqs,
                                const uint32_t* mask, const int32_t* labels, float* loss, void* ws,
                                size_t ws_bytes, void* stream);


/* ----------------------------------------------------------------------------
 * labs_learned_walk -- the first-step walk (Alg. 1 neighbourhood: skew flips of
 * the free positions p+1..k+1, Eq. (3)) with the candidate set narrowed by a
 * proposer.  Walkers start exactly as in labs_walk_step1 (same seed, walker ids,
 * initial sequences and tenures).  At step t (from 1) of a walker:
 *   admissible  = free positions a with tabu_until(a) < t
 *   candidates  = every admissible position when (t-1) mod fallback_every == 0
 *                 (a full exact scan: the plain walker's step), otherwise the
 *                 top_m admissible positions by proposer score (ties: lower a)
 *   move        = the candidate of least exact integer dE (ties: lower a),
 *                 dE computed from the current C table by definition
 *   then E += dE, tabu_until(a) = t + tenure, as in the plain walker.
 * With fallback_every = 1, or top_m >= k+1-p, every step is the plain walker's.
 * Proposers:
 *   LABS_PROPOSE_MLP     score = logit a-1 of the network (labs_mlp_* layout,
 *                        hidden width prop->hidden) on the current state
 *   LABS_PROPOSE_RANDOM  score = a SplitMix64 draw keyed by (prop->seed,
 *                        walker, t, a): top_m uniformly random admissible
 *                        positions (the ablation without a network)
 * Training log (prop->log_every > 0): n_log = steps / log_every records per
 * walker, stored step-major (record r of walker j at index r*n + j, so that
 * consecutive records come from different walkers); it describes step
 * t = (r+1)*log_every: the packed state before the move (W words), the
 * admissible positions (mask_words words, bit (a-1) mod 32 of word (a-1)/32)
 * and the label a-1 of the chosen move.  Logged from a walker with
 * fallback_every = 1 the label is the plain walker's best admissible flip.
 * Outputs (device, nullable except flip_evals):
 *   final_seqs/final_E, best_seqs/best_E/best_step as labs_walk_step1
 *   hit_step  [n]  first step with E <= cfg->e_max (-1 if none or e_max < 0)
 *   traj_E    [n*steps] E after each step (-1 after a halt)
 *   moves     [n*steps] moved position a (-1 after a halt)
 *   cands     [n*steps*top_m] the rescored positions of each non-full step in
 *             descending score order (-1 on full-scan steps and as padding)
 *   flip_evals [1] exact dE evaluations over all walkers and steps
 * cfg: as labs_walk_step1 with n_cfg = 1; flags must be 0.  Limits: L <= 639,
 * 1 <= top_m <= 64, fallback_every >= 1.  The network weights must not change
 * while the call runs.
 * -------------------------------------------------------------------------- */
#define LABS_PROPOSE_MLP 0
#define LABS_PROPOSE_RANDOM 1

typedef struct {
    int32_t mode;
    int32_t top_m;
    int32_t fallback_every;
    int32_t hidden;
    const float* params;          /* FP32 blob (MLP mode) */
    const uint16_t* params_bf16;  /* bf16 blob (MLP mode) */
    uint64_t seed;                /* RANDOM mode */
    int32_t log_every;
    int32_t reserved;             /* must be 0 */
} labs_proposer;

typedef struct {
    uint32_t* final_seqs;
    int32_t* final_E;
    uint32_t* best_seqs;
    int32_t* best_E;
    int32_t* best_step;
    int32_t* hit_step;
    int32_t* traj_E;
    int32_t* moves;
    int16_t* cands;
    uint32_t* log_seqs;
    uint32_t* log_mask;
    int32_t* log_label;
    int64_t* flip_evals;
    /* first-hit stamps, as in labs_step1_out */
    int32_t n_levels;
    int32_t level_E[16];
    uint64_t* first_hit_ticks;
    uint64_t* start_ticks;
} labs_learned_out;

labs_status labs_learned_walk_workspace(const labs_step1_cfg* cfg, const labs_proposer* prop, size_t* bytes);
labs_status labs_learned_walk(const labs_step1_cfg* cfg, const labs_proposer* prop, const labs_learned_out* out,
                              void* ws, size_t ws_bytes, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* LABS_H */
