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

#define LABS_ABI_VERSION 1

typedef int32_t labs_status;
enum {
    LABS_OK = 0,
    LABS_E_INVALID = -1,     /* bad argument; nothing enqueued */
    LABS_E_DEVICE = -2,      /* HIP runtime or launch failure */
    LABS_E_NOMEM = -3,       /* workspace too small */
    LABS_E_UNSUPPORTED = -4  /* valid request outside what this build implements */
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
 * (walker, step) order.  Overflow is not an error: *dropped grows by the number
 * of distinct sequences cut by the capacity. */
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
} labs_step1_out;

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
 * Autotuner of the walker's tiles.  A shape class is (NW, R): NW = ceil(k/32)
 * words of even lags and R = ceil((k+1-p)/64) free positions per lane.  Its tile
 * is RB, the slots a lane scans per pass (R, or ceil(R/2) to free registers for
 * occupancy), and the resident waves per SIMD requested by persistent launches
 * (1, 2, 4 or 8).  labs_autotune_step1 times every candidate tile on the largest
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
 *   - if the round's smallest pushed energy is below best's, best becomes the
 *     smallest pushed entry and u = 0; otherwise u grows by the
 *     number of pivots (u counts pops since the last strict improvement; with
 *     batch = 1 this is Alg. 2's dynamic depth exactly);
 *   - cuts Open to the pq_capacity smallest (evicted sequences are forgotten
 *     and may be pushed again later).
 * Results do not depend on scheduling.  The call synchronises `stream`.
 */
typedef struct {
    int32_t L;               /* 2..1023 */
    int32_t batch;           /* pivots per round, >= 1 */
    int32_t T_r;             /* rotations; must be 0 in this build */
    int32_t reserved;        /* must be 0 */
    int64_t pq_capacity;     /* Q >= 1 */
    int64_t max_expansions;  /* >= 0 */
    int64_t T_u;             /* >= 1 */
} labs_step2_cfg;

typedef struct {
    int64_t expansions;      /* pivots popped */
    int64_t pushes;          /* neighbours pushed (new or re-pushed after eviction) */
    int64_t dup_skips;       /* neighbours skipped as already present */
    int64_t evictions;       /* entries cut by the capacity */
    int64_t rounds;
    int64_t open_count;      /* Open entries at the end */
    int32_t best_E;
    int32_t best_round;      /* round of the last improvement, -1 if none */
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

#ifdef __cplusplus
}
#endif
#endif /* LABS_H */
