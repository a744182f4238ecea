// Internal declarations of liblabs.so (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include "../../include/labs.h"

namespace labsdev {

// ---------------------------------------------------------------- host errors
void set_error(const char* fmt, ...);
void clear_error();
labs_status invalid(const char* fmt, ...);   // sets the message, returns LABS_E_INVALID
labs_status device_error(hipError_t e, const char* what);
const char* last_error();

#define LABS_HIP(call)                                                      \
    do {                                                                    \
        hipError_t _e = (call);                                             \
        if (_e != hipSuccess) return ::labsdev::device_error(_e, #call);       \
    } while (0)

#define LABS_LAUNCHED(what)                                                 \
    do {                                                                    \
        hipError_t _e = hipGetLastError();                                  \
        if (_e != hipSuccess) return ::labsdev::device_error(_e, what);        \
    } while (0)

inline int32_t words_of(int32_t L) { return (L + 31) / 32; }
inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Bump allocator over a caller workspace (256-byte aligned slices).
struct Carve {
    char* base;
    size_t size, used;
    explicit Carve(void* b, size_t s) : base((char*)b), size(s), used(0) {}
    template <class T> T* take(size_t count) {
        size_t off = align_up(used, 256);
        used = off + count * sizeof(T);
        return (base && used <= size) ? (T*)(base + off) : nullptr;
    }
    bool ok() const { return used <= size; }
};

// ---------------------------------------------------------------- device helpers
extern "C" __device__ int __ockl_wfred_min_i32(int);
extern "C" __device__ unsigned int __ockl_wfred_or_u32(unsigned int);
extern "C" __device__ int __ockl_wfred_add_i32(int);
extern "C" __device__ unsigned int __ockl_wfred_max_u32(unsigned int);
extern "C" __device__ int __ockl_wfred_max_i32(int);
extern "C" __device__ int __ockl_wfscan_add_i32(int, bool);

// popcount(x) + acc in one instruction: bit-plane sums chain through the
// accumulator operand of v_bcnt_u32_b32 (written out, because the compiler splits
// such chains into separate popcounts and three-way adds)
__device__ __forceinline__ uint32_t bcnt_add(uint32_t x, uint32_t acc) {
    uint32_t r;
    asm("v_bcnt_u32_b32 %0, %1, %2" : "=v"(r) : "v"(x), "v"(acc));
    return r;
}

// SplitMix64 (Steele, Lea, Flood 2014): finaliser and the counter form of its
// stream, output i of the stream started at `key` is mix(key + (i+1)*gamma).
__device__ __forceinline__ uint64_t sm64_mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
__device__ __forceinline__ uint64_t sm64_at(uint64_t key, uint64_t i) {
    return sm64_mix(key + (i + 1ull) * 0x9E3779B97F4A7C15ull);
}
// Zobrist table of sequence keys (Zobrist 1970): Z for position i+1 is output i
// of the SplitMix64 stream started at kZobristState.  The second step keys whole
// sequences with it, the first step's Bloom filter the first k+1 elements.
constexpr uint64_t kZobristState = 0x6A09E667F3BCC909ull;
__device__ __forceinline__ uint64_t zobrist_at(int i) { return sm64_at(kZobristState, (uint64_t)i); }
__device__ __forceinline__ uint64_t walker_key(uint64_t seed, int32_t L, int64_t w) {
    uint64_t lw = ((uint64_t)(uint32_t)L << 32) ^ (uint64_t)(w + 1);
    return sm64_mix(seed ^ sm64_mix(lw));
}

// bfloat16 bit pattern of an FP32 value, round to nearest even.
__device__ __forceinline__ uint16_t f2bf(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// Packed wire format: s_i (1-based) is bit 31-((i-1)&31) of word (i-1)>>5.
__device__ __forceinline__ int packed_bit(const uint32_t* w, int i) {
    return (w[(i - 1) >> 5] >> (31 - ((i - 1) & 31))) & 1;
}

// ---------------------------------------------------------------- launchers
labs_status launch_energy(int32_t L, int64_t n, const uint32_t* seqs, int32_t* E, int32_t* C,
                          hipStream_t st);
labs_status launch_flip_deltas(int32_t L, int32_t p, int32_t skew, int64_t n,
                               const uint32_t* seqs, int32_t* dE, hipStream_t st);

// Records for sorting/pooling: KW = W + 3 uint32 key words per record, stored
// word-major: key word q of record i at rec[q*stride + i]. Word 0 is E, words
// 1..W the packed sequence, word W+1 the walker id, word W+2 the step.
struct RecBuf {
    uint32_t* rec;
    int64_t stride;
    int32_t KW;
};

// The distinct sequences a pool's capacity cut within one call (the pool's
// `dropped` count): an open-addressing set of packed sequences, a non-zero
// 64-bit hash per slot (0 = empty) and the sequence's words beside it.
// status[0] is set when an insert found the set too full, status[1] counts
// the entries.
struct CutSet {
    uint64_t* keys;      // [slots]
    uint32_t* words;     // [slots * W]
    uint32_t* status;    // [2]
    int64_t slots;       // power of two
};
// Slots for a pool of capacity `cap` fed by staging batches of up to `staged`
// records: one batch always fits while the set is at most half full.
int64_t cutset_slots(int64_t cap, int64_t staged);
size_t cutset_bytes(int64_t slots, int32_t W);
CutSet cutset_carve(Carve& cv, int64_t slots, int32_t W);
labs_status cutset_clear(const CutSet& cs, hipStream_t st);

size_t sort_workspace_bytes(int64_t nmax, int32_t KW);
size_t compact_workspace_bytes(int64_t nmax, int32_t KW);
// Sort records [0, n) of rb, keep the first min(cap, D) distinct sequences in the
// output arrays and set count / out_n.  With `cut`, every distinct sequence beyond
// the capacity that the set does not hold yet is added to it and counted in
// *dropped (so a sequence cut in several compactions of one call counts once).
labs_status compact_records(const RecBuf& rb, int32_t W, int64_t n, int64_t cap, uint32_t* out_seqs,
                            int32_t* out_E, int64_t* out_walker, int32_t* out_step, int64_t* count,
                            int64_t* dropped, int64_t* out_n, const CutSet* cut, void* ws,
                            size_t ws_bytes, hipStream_t st);
labs_status pool_to_rec(const labs_pool& pool, int64_t n, int32_t W, const RecBuf& rb, int64_t off,
                        hipStream_t st);

// First-step walker state and launch arguments (walk.hip).
struct WalkArgs {
    int32_t L, p, k, nf, W;
    int32_t t0, t1, steps_total;
    int64_t n, walker_begin;
    uint64_t seed;
    int32_t tenure_lo, tenure_hi;
    uint32_t* seq;      // [n*W] packed current sequence
    int32_t* E;         // [n]
    int32_t* tenure;    // [n]
    int32_t* halted;    // [n] 0 = running, else the step that found no admissible move
    int32_t* tabu;      // [n*nf] tabu_until per free position
    int32_t* bestE;     // [n]
    int32_t* bestT;     // [n]
    uint32_t* bestSeq;  // [n*W]
    int32_t* traj;      // [n*steps_total] or null
    int32_t e_max;      // < 0: sieve off
    uint32_t* rec;      // staging records, word-major
    int64_t rec_stride;
    uint32_t* st_count;
    uint32_t st_cap;
    // Bloom-filter self-avoidance (null bloom: the tabu tenure)
    uint64_t* zh;          // [n] Zobrist key of the current sequence's first k+1 elements
    uint32_t* bloom;       // [n << (bloom_log2 - 5)] filter words per walker
    int32_t bloom_log2;    // filter bits per walker = 2^bloom_log2
    int32_t bloom_hashes;  // bits set / tested per key
    // first-hit stamps of the real-time counter (n_levels = 0: off)
    int32_t n_levels;
    int32_t level_E[16];
    unsigned long long* hit_ticks;    // [n_levels], atomic min
    unsigned long long* start_ticks;  // [1], atomic min, stamped by the init kernel
};

// Stamp every level l that energy E reaches (E <= level_E[l]) with the real-time
// counter (lane 0, atomic min: a level reached again later keeps its first stamp)
// and return the largest level energy below E (-1: none), which the caller
// compares E against before calling again.  Wave-uniform.
__device__ __forceinline__ int stamp_levels(const WalkArgs& A, int E, int lane) {
    const unsigned long long now = __builtin_amdgcn_s_memrealtime();
    int pend = -1;
    for (int l = 0; l < A.n_levels; ++l) {
        const int lv = A.level_E[l];
        if (E <= lv) {
            if (lane == 0) atomicMin(&A.hit_ticks[l], now);
        } else {
            pend = lv > pend ? lv : pend;
        }
    }
    return __builtin_amdgcn_readfirstlane(pend);
}
// Copies the first-hit stamp request of an output struct into walker arguments
// (n_levels, level_E, first_hit_ticks, start_ticks), validating it.
template <class Out>
inline labs_status set_stamps(WalkArgs& A, const Out& o) {
    A.n_levels = 0;
    A.hit_ticks = nullptr;
    A.start_ticks = nullptr;
    if (o.n_levels == 0) return LABS_OK;
    if (o.n_levels < 0 || o.n_levels > LABS_MAX_LEVELS)
        return invalid("n_levels must be in [0, %d], got %d", LABS_MAX_LEVELS, o.n_levels);
    if (!o.first_hit_ticks) return invalid("first_hit_ticks must not be NULL when n_levels > 0");
    A.n_levels = o.n_levels;
    for (int l = 0; l < LABS_MAX_LEVELS; ++l) A.level_E[l] = l < o.n_levels ? o.level_E[l] : -1;
    A.hit_ticks = (unsigned long long*)o.first_hit_ticks;
    A.start_ticks = (unsigned long long*)o.start_ticks;
    return LABS_OK;
}
__device__ __forceinline__ int pending_level(const WalkArgs& A) {
    int pend = -1;
    for (int l = 0; l < A.n_levels; ++l) pend = A.level_E[l] > pend ? A.level_E[l] : pend;
    return __builtin_amdgcn_readfirstlane(pend);
}
bool walk_shape_supported(int L, int p);
size_t step2_workspace_bytes(const labs_step2_cfg& c, long long n_cand);
bool step2_fits(const labs_step2_cfg& c, long long n_cand);   // hash-set slots fit int32 indices
labs_status step2_run(const labs_step2_cfg& cfg, long long n_cand, const uint32_t* cand_seqs,
                      const labs_step2_out& out, void* ws, size_t ws_bytes, hipStream_t st,
                      labs_status (*tb)(void*, hipStream_t), labs_status (*te)(void*, hipStream_t),
                      void* tctx);
labs_status launch_walker_init(const WalkArgs& A, hipStream_t st);
labs_status launch_bloom_init(const WalkArgs& A, hipStream_t st);
labs_status legendre_pairs(int32_t L, const labs_legendre_sweep& sw, int32_t* n_out, int32_t* o_out,
                           int64_t capacity, int64_t* count);
size_t legendre_workspace_bytes(int64_t n_pairs);
labs_status length_operators(int32_t L, int64_t n, const uint32_t* seqs, uint32_t* minus, int32_t* E_minus,
                             uint32_t* plus, int32_t* E_plus, hipStream_t st);
labs_status legendre_build(int32_t L, int64_t n_pairs, const int32_t* n_host, const int32_t* o_host,
                           uint32_t* seqs, int32_t* E, void* ws, size_t ws_bytes, hipStream_t st);
labs_status launch_walker_init_items(const WalkArgs* args, const int2* items, int n_items, hipStream_t st);
// Autotuned register tile (slots per pass) for the walker of (L, p); R when untuned.
int walk_tile_rb(int L, int p, int R);
size_t batch_workspace_bytes(const labs_step1_cfg* c, int n);
labs_status batch_walk(const labs_step1_cfg* c, int n, const labs_step1_out* outs, void* ws, size_t wsb,
                       hipStream_t st, const void* tile_override, bool use_graph);
labs_status autotune_step1(const int32_t* Ls, int n_L, int p, int walkers, int steps, hipStream_t st);
labs_status autotune_save(const char* path);
labs_status autotune_load(const char* path);
labs_status autotune_get(int L, int p, int* rb, int* waves);
labs_status launch_walk(const WalkArgs& A, hipStream_t st);
labs_status launch_offer_best(const WalkArgs& A, hipStream_t st);
labs_status launch_walk_outputs(const WalkArgs& A, const labs_step1_out& o, hipStream_t st);
// Sorts records [0, n) of `rb` by key words 0..nkeys-1 (word 0 most significant),
// leaving the permutation in *perm_out (device array of n uint32, inside ws).
labs_status radix_sort_records(const RecBuf& rb, int64_t n, int32_t nkeys, void* ws,
                               size_t ws_bytes, uint32_t** perm_out, hipStream_t st);

// Learned proposal network (mlp.hip).
bool mlp_layout(int L, int hidden, labs_mlp_layout* o);
labs_status launch_features(int L, int64_t n, const uint32_t* seqs, uint16_t* X, int ld_in, hipStream_t st);
size_t mlp_forward_ws(const labs_mlp_layout& y, int64_t n);
labs_status mlp_forward(const labs_mlp_layout& y, const float* P, const uint16_t* Pb, int64_t n, const uint16_t* X,
                        float* logits, void* ws, size_t wsb, hipStream_t st);
size_t mlp_grads_ws(const labs_mlp_layout& y, int64_t n);
labs_status mlp_grads(const labs_mlp_layout& y, const float* P, const uint16_t* Pb, int64_t n, const uint16_t* X,
                      const uint32_t* mask, const int32_t* labels, float* G, float* loss, void* ws, size_t wsb,
                      hipStream_t st);
labs_status mlp_adam(const labs_mlp_layout& y, float* P, uint16_t* Pb, const float* G, float* M, float* V, int t,
                     double lr, double b1, double b2, double eps, hipStream_t st);
labs_status mlp_cast(const labs_mlp_layout& y, const float* P, uint16_t* Pb, hipStream_t st);

// First-step walk with a proposer (learned.hip).
labs_status validate_step1_cfg(const labs_step1_cfg& c);
bool learned_walk_supported(int L);
size_t learned_walk_ws(const labs_step1_cfg& c, const labs_proposer& pr);
labs_status learned_walk(const labs_step1_cfg& c, const labs_proposer& pr, const labs_learned_out& o, void* ws,
                         size_t wsb, hipStream_t st);

}  // namespace labsdev
