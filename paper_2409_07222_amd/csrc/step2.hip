// Second step (Algorithm 2) as a device-resident, batch-synchronous best-first
// search.  Every round is a fixed sequence of kernels that read a control block
// in device memory; the host enqueues rounds and looks at the stop flag every
// few rounds.
//
// Data structures (all in the caller's workspace):
//  * a hash set H keyed by the exact sequence (open addressing, linear probing,
//    four slots per live entry).  A slot holds a 64-bit Zobrist key (0 = empty),
//    a one-byte tag of the key that lets most probes stop without touching the
//    key array, a state (OPEN, CLOSED, EVICTED), E and the packed sequence (key, E
//    and state share one 16-byte record).
//    Zobrist keys make a neighbour's key one XOR away from its pivot's (Alg. 2's
//    HASH_FLIP).  H holds Closed U Open U evicted sequences; an EVICTED slot
//    counts as absent and is re-opened when its sequence is pushed again.  When
//    half of H is claimed it is rebuilt without the evicted tombstones.
//  * the Open list: (E, slot, key) entries, unordered.  Pops mark entries dead;
//    the capacity cut at the end of each round compacts the list into the other
//    buffer, so every round starts from a dense list.  A round's neighbours sit
//    at fixed positions (pivot b, flip i) after the surviving old entries.
//  * an exact "T smallest" selection in the order (E, Zobrist key, sequence):
//    energies of one length are congruent mod 4, so (E - emin)/4 is selected by
//    one 14-bit radix level (a bin it leaves unresolved is finished by the tie
//    select), then the entries tied at the threshold energy are split byte by
//    byte on the Zobrist key (and, if keys collide, the sequence).
//    The energy window of the last cut is carried to the next round as the
//    starting bounds.
//
// A round's neighbours do not enter H when they are generated.  The expansion
// only reads H (no writer runs beside it): a neighbour whose sequence H holds as
// OPEN or CLOSED is a duplicate.  Two pivots of one round produce a common
// neighbour exactly when they differ in two positions (each flips the other's
// position), so the in-round repeats are found by comparing the pivots pairwise:
// each expansion workgroup compares its pivot with the lower-numbered ones and
// skips the copies they also produce (the direct expansion for long sequences
// takes them from k_repeats, 64 x 64 tiles in LDS).  The capacity cut runs over
// old and new entries alike, and only the new entries that survive it are
// written into H (the tombstone re-opened, or an empty slot claimed by CAS).
// Neighbours cut in their own round never touch H, so H holds little more than
// Closed U Open and rarely needs a rebuild.
//
// A round's launches: k_expand (repeats, then the single flips; the direct
// expansion for long sequences adds k_clear_repeats and k_repeats), the rotation
// kernels when T_r > 0, k_mid_hist (the round's counts and statistics, the cut
// setup, the radix level), k_sel_classify (threshold bins, flags, tie lists, the
// tied entries' top key bytes; in an improving round each workgroup's best
// candidate), k_sel_keys (the two tie selects; a third workgroup takes an
// improving round's best), k_keep (the cut; it also takes the next round's pivots
// out of Open: CLOSED in the table, their slots and words copied to the next
// round's pivot arrays), k_round_next (end of this round, start of the next).
// The seeding insertions are exact and use no fences: a candidate walks its
// probe sequence with 64-bit CAS on the key word; an empty slot is claimed, a
// slot already holding its key makes the candidate "pending".  After the kernel
// boundary the pending candidates are compared with the slot's sequence; a
// mismatch is a true 64-bit key collision, finished one at a time by a single
// thread.
#include "labs_internal.h"

#include <climits>

namespace labsdev {

namespace {

constexpr int32_t DEAD = INT32_MAX;
constexpr uint32_t ST_OPEN = 1, ST_CLOSED = 2, ST_EVICTED = 3;
// Radix digit of the energy select.  All energies of one length L are congruent
// mod 4 (C_k has the parity of L-k, so C_k^2 is 0 mod 4 or 1 mod 8), so the
// select works on (E - emin)/4.  E <= sum_{j<L} j^2 = (L-1)L(2L-1)/6 < 2^29 for
// L <= 1023, so (E - emin)/4 < 2^27.
constexpr int kSelBits = 14;
// One radix level of kSelBits over D = (E - emin)/4 (< 2^27 for L <= 1023); when it
// leaves a bin of 2^ls values (ls = bit length of the range - kSelBits), the cut
// takes everything below the bin and the tie select resolves the bin's values
// (at most 2^kSubBits of them) before the key bytes.
constexpr int kSubBits = 13;
static_assert(kSelBits + kSubBits >= 27, "the sub-bins must cover (E - emin)/4 for L <= 1023");
constexpr int kSelBins = 1 << kSelBits;
// After the energy histogram, two 256-bin histograms of the top Zobrist-key byte of
// the entries tied at the cut's energy (first) and at the pivots' energy (second),
// in kZCopies copies (workgroup b adds into copy b mod kZCopies, so that few
// workgroups add into one counter; the tie select sums the copies).
constexpr int kZBins = 256;
constexpr int kZCopies = 16;
constexpr int kHistWords = kSelBins + kZCopies * 2 * kZBins;
constexpr int kSelBlocks = 256;
constexpr int kSelThreads = 512;
constexpr int kGridBlocks = 1024;                    // grid-stride kernels over the Open list
// The classify pass and the cut with as many workgroups as stay resident together
// (two, three per CU at their register use), so that no workgroup waits for a slot.
constexpr int kClassifyBlocks = 512;
constexpr int kKeepBlocks = 768;
constexpr int kCheck = 8;    // rounds between host looks at the control block
constexpr int kMaxL = 1023;
constexpr int kPad = 1024;
constexpr int kSv = kMaxL + 2 * kPad + 2;
constexpr int kExThreads = 256;
constexpr int kExWaves = kExThreads / 64;
constexpr int kItems = 8;                            // list entries per thread per pass (filters)
constexpr int kKeepItems = 2;
constexpr int kHistItems = 12;                       // the radix histogram: 256 x 512 x 12 entries a pass                        // the cut: fewer, so inserts overlap across threads

// A slot's key, energy and state in one 16-byte record, so that a claim (CAS on
// the key) and the writes of E and state touch one cache line, as do a probe's
// key compare and state read.
struct SlotRec {
    unsigned long long key;   // Zobrist key, 0 = empty
    int32_t E;
    uint32_t state;           // ST_OPEN, ST_CLOSED, ST_EVICTED
};

struct Table {
    SlotRec* rec;
    uint8_t* tag;          // 0 for an empty slot, else tag_of(key): a byte-wide filter
    uint32_t* seq;
    uint64_t mask;
    int32_t W;
};

// One byte per slot (64 MB at 2^26 slots, small enough to stay in the on-package
// cache): read-only probes stop at an empty tag and read the 8-byte key only on
// a tag match.  Written once, right after the slot's key is claimed.
__device__ __forceinline__ uint8_t tag_of(unsigned long long key) { return (uint8_t)(0x80u | (key >> 57)); }

struct Ctl {
    // persistent
    long long n_tot, n_live;
    long long expansions, pushes, dups, evictions, rounds, u;
    int32_t best_E, best_slot, best_round, stop;
    int32_t error, which, pad0, pad1;
    // per round
    long long n_piv, batch_begin, n_pend, n_slow, survivors;
    int32_t batch_minE, improved, pad2, pad3;
    // selection
    long long T, c_lt, need;
    uint32_t emin, emax;
    int32_t sel_enabled, sel_all;
    int32_t hi_shift, pad4;   // hi_shift: bin width (bits of D) of an unresolved select
    uint32_t prefix, Dt;
    int32_t resolved, n_cand;
    // table occupancy (claimed slots, tombstones included) and rebuild scratch
    long long claimed, claimed_new;
    long long out_count;
    uint32_t blo, bhi;     // bounds of the live Open energies (blo is one of them)
    // A cut that also selects the next round's T2 pivots (the T2 smallest of the
    // survivors are the T2 smallest before the cut): their own threshold; the cut
    // takes them out of Open for the next round (n_pivpos); presel: this round's pivots
    // were selected so.
    long long T2, c_lt2, out_count2, n_pivpos;
    uint32_t Dt2, prefix2;
    int32_t resolved2, dual, presel, dual_all;   // dual_all: T2 takes every survivor
    // A tie select that split its tied entries on the top key byte first: the
    // entries tied at the cut's (zv) / the pivots' (zv2) energy whose top byte is
    // below the threshold byte are taken by the cut itself (flag bits 2 / 3 mark
    // the tied entries); 0 when unused.
    uint32_t zv, zv2;
    // n_live and expansions as the round began (read by every workgroup of the
    // histogram pass, whose workgroup 0 updates the live fields)
    long long n_live0, expansions0;
    long long n_bestc;   // workgroups' candidates for an improving round's best (bestc)
};

// The control block as a kernel found it at its start, copied to LDS by the first
// threads of each workgroup: one round trip instead of a chain of dependent scalar
// loads.  The round kernels read their inputs from the copy and write through
// P.ctl; a field a kernel writes is not read back through the copy.
__device__ __forceinline__ void snap_ctl(Ctl& cs, const Ctl* c) {
    static_assert(sizeof(Ctl) % 8 == 0, "the control block is copied in 8-byte words");
    constexpr int n = (int)(sizeof(Ctl) / 8);
    static_assert(n <= 64, "one wavefront copies the control block");
    if (threadIdx.x < (unsigned)n)
        reinterpret_cast<unsigned long long*>(&cs)[threadIdx.x] =
            reinterpret_cast<const unsigned long long*>(c)[threadIdx.x];
    __syncthreads();
}

// A pending insertion: the slot whose key matched, the source of the sequence
// (a pivot slot and a flip position, or a candidate index when src < 0) and E.
struct Pend {
    int32_t slot, src, flip, E;
};

struct Params {
    int32_t L, W, B;
    long long Q, X, T_u;
    long long cap_o, cap_pend;
    Table H;
    Ctl* ctl;
    int32_t* oE[2];
    int32_t* oS[2];
    unsigned long long* oZ[2];   // Zobrist key of each Open entry (tie order without table reads)
    uint32_t* flag;        // [cap_o]
    int32_t* cand[2];      // [cap_o] each: Open positions of tied entries
    unsigned long long* candz[2];   // [cap_o] each: their Zobrist keys
    int32_t* cand2[2];     // the same for the next round's pivots (dual cut)
    unsigned long long* candz2[2];
    int32_t* piv;          // [B] table slots of this round's pivots
    int32_t* pivn;         // [B] the next round's (written by the cut; the host alternates the two)
    // [kCheck][kKeepBlocks]: hash-set slots claimed by each workgroup of the cut in
    // the rounds of a batch (round r writes row r mod kCheck); the host copies the
    // rows with the batch's flags and sums them (no atomics on one counter)
    int32_t* kclaims;
    int32_t* pivE;         // [B] energies of this round's pivots, and of the next round's
    int32_t* pivEn;
    unsigned long long* pivK;   // [B] their Zobrist keys (as stored with their slots)
    unsigned long long* pivKn;
    uint32_t* ghist;       // [kHistWords]: energy bins, then the two key-byte histograms; zero between selections
    uint32_t* best_seq;    // [W] copy of the best sequence
    Pend* pend;            // [cap_pend]
    Pend* slow;            // [cap_pend]
    const uint32_t* cands; // seeding input
    // This round's neighbours occupy Open positions batch_begin + b*L + (i-1) for
    // pivot b and flip position i (DEAD when not pushed); by that offset:
    int32_t* ntomb;        // slot of the sequence's evicted tombstone, or -1
    int32_t* bcnt;         // [B] neighbours pushed by pivot b
    int32_t* bmin;         // [B] their least energy
    int32_t* bmax;         // [B] their greatest energy
    // [B*L] 1 when neighbour (b, i) repeats a neighbour of a lower-numbered pivot
    // (the direct expansion only; the bit-sliced one finds its repeats itself)
    uint8_t* repeat;
    int32_t direct;        // the direct expansion is in use
    uint32_t* pseq;        // [B*W] packed sequences of the round's pivots
    uint32_t* pseqn;       // [B*W] the next round's (written by the cut)
    int32_t* pivpos;       // [B] the next round's pivots' Open positions (the cut)
    int32_t best_in_classify;   // rounds: an improving round's best is found by the classify pass and the tie select
    int32_t* bestc;             // [kClassifyBlocks] each classify workgroup's least entry at the round's least energy
    int32_t take_pivots;   // the cut takes its pivots out of Open (rounds; not the seeding cut,
                           // whose pivots leave after the initial best is found)
    // MAKE_ROTATIONS: rotation q of pivot b sits at Open position batch_begin +
    // n_piv*L + b*R2 + q (after every single flip of the round); q < Tr rotates
    // left by q+1, else right by q-Tr+1.
    int32_t Tr, R2;
    unsigned long long* rkey;   // [B*R2] their Zobrist keys
    int32_t* rE;                // [B*R2] their energies
    uint32_t* pw0;              // [B] first packed word of each pivot of the round
};

__device__ __forceinline__ uint64_t zob(int i) { return zobrist_at(i); }

__device__ void best_scan(const Params& P, int initial);

// Block-aggregated append: every thread of the block must call it (uniformly).
__device__ long long block_append(long long* counter, bool take) {
    __shared__ int wcnt[16];
    __shared__ long long bbase;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int nw = (blockDim.x + 63) >> 6;
    const uint64_t m = __ballot(take);
    const uint64_t lt = lane ? (~0ull >> (64 - lane)) : 0ull;
    if (lane == 0) wcnt[wv] = __popcll(m);
    __syncthreads();
    if (threadIdx.x == 0) {
        int run = 0;
        for (int k = 0; k < nw; ++k) {
            const int t = wcnt[k];
            wcnt[k] = run;
            run += t;
        }
        bbase = run ? (long long)atomicAdd((unsigned long long*)counter, (unsigned long long)run) : 0;
    }
    __syncthreads();
    const long long idx = bbase + wcnt[wv] + __popcll(m & lt);
    __syncthreads();
    return take ? idx : -1;
}

// Block-aggregated append of n >= 0 items per thread (one atomic per block);
// every thread of the block must call it.  Returns the thread's first index.
__device__ long long block_append_n(long long* counter, int n) {
    __shared__ int wsum[16];
    __shared__ long long bbase;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int nw = (blockDim.x + 63) >> 6;
    int x = n;
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) wsum[wv] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        int run = 0;
        for (int k = 0; k < nw; ++k) {
            const int t = wsum[k];
            wsum[k] = run;
            run += t;
        }
        bbase = run ? (long long)atomicAdd((unsigned long long*)counter, (unsigned long long)run) : 0;
    }
    __syncthreads();
    const long long r = bbase + wsum[wv] + (x - n);
    __syncthreads();
    return r;
}

// Two block-aggregated appends in one pass (every thread calls it uniformly):
// *oa, *ob receive this thread's first positions in the two lists.
__device__ void block_append2(long long* ca, int na, long long* cb, int nb, long long* oa, long long* ob) {
    __shared__ int wa[16], wb[16];
    __shared__ long long ba, bbq;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int nw = (blockDim.x + 63) >> 6;
    int x = na, y = nb;
    for (int o = 1; o < 64; o <<= 1) {
        const int u = __shfl_up(x, o, 64), v = __shfl_up(y, o, 64);
        if (lane >= o) {
            x += u;
            y += v;
        }
    }
    if (lane == 63) {
        wa[wv] = x;
        wb[wv] = y;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int ra = 0, rb = 0;
        for (int k = 0; k < nw; ++k) {
            const int ta = wa[k], tb = wb[k];
            wa[k] = ra;
            wb[k] = rb;
            ra += ta;
            rb += tb;
        }
        ba = ra ? (long long)atomicAdd((unsigned long long*)ca, (unsigned long long)ra) : 0;
        bbq = rb ? (long long)atomicAdd((unsigned long long*)cb, (unsigned long long)rb) : 0;
    }
    __syncthreads();
    *oa = ba + wa[wv] + (x - na);
    *ob = bbq + wb[wv] + (y - nb);
    __syncthreads();
}

__device__ __forceinline__ void atomic_min_batch(Ctl* c, bool take, int32_t E) {
    const int mn = __ockl_wfred_min_i32(take ? E : INT32_MAX);
    if ((threadIdx.x & 63) == 0 && mn != INT32_MAX) atomicMin(&c->batch_minE, mn);
}

// Tie order between two slots of equal energy: Zobrist key, then the sequence
// (words compared as unsigned).
__device__ __forceinline__ bool key_less(const Table& H, int a, int b) {
    if (H.rec[a].key != H.rec[b].key) return H.rec[a].key < H.rec[b].key;
    for (int w = 0; w < H.W; ++w) {
        uint32_t x = H.seq[(size_t)a * H.W + w], y = H.seq[(size_t)b * H.W + w];
        if (x != y) return x < y;
    }
    return false;
}

__device__ __forceinline__ uint32_t src_word(const Params& P, int src, int flip, int w) {
    if (src < 0) return P.cands[(size_t)(-src - 1) * P.W + w];
    uint32_t x = P.H.seq[(size_t)src * P.W + w];
    if (flip > 0 && w == ((flip - 1) >> 5)) x ^= 1u << (31 - ((flip - 1) & 31));
    return x;
}

// 32 elements of a packed sequence from element a (0-based) on, first element in
// the top bit (elements past the last word read as 0).
__device__ __forceinline__ uint32_t read32(const uint32_t* p, int W, int a) {
    const int q = a >> 5, h = a & 31;
    const uint32_t hi = p[q];
    if (!h) return hi;
    const uint32_t lo = q + 1 < W ? p[q + 1] : 0u;
    return (hi << h) | (lo >> (32 - h));
}

// Word w of the left rotation by r (0 < r < L) of a packed sequence: element i
// is element (i + r) mod L of the original; bits past element L-1 are 0.
__device__ __forceinline__ uint32_t rot_word(const uint32_t* p, int L, int W, int r, int w) {
    const int a = (32 * w + r) % L;
    const int n1 = L - a;   // elements before the wrap
    uint32_t x = read32(p, W, a);
    if (n1 < 32) x = (x & (~0u << (32 - n1))) | (read32(p, W, 0) >> n1);
    if (w == W - 1 && (L & 31)) x &= ~0u << (32 - (L & 31));
    return x;
}

// Left shift of rotation q of a pivot.
__device__ __forceinline__ int rot_shift(const Params& P, int q) { return q < P.Tr ? q + 1 : P.L - (q - P.Tr + 1); }

// Word w of this round's new entry at offset j from batch_begin: a single flip
// of a pivot, or (past every flip) a rotation of one.
__device__ __forceinline__ uint32_t new_word(const Params& P, long long j, int w) {
    // from the round's compact copy of its pivots' words
    const long long nf = P.ctl->n_piv * P.L;
    if (j < nf) {
        const int flip = (int)(j % P.L) + 1;
        uint32_t x = P.pseq[(size_t)(j / P.L) * P.W + w];
        if (w == ((flip - 1) >> 5)) x ^= 1u << (31 - ((flip - 1) & 31));
        return x;
    }
    const long long jr = j - nf;
    return rot_word(P.pseq + (size_t)(jr / P.R2) * P.W, P.L, P.W, rot_shift(P, (int)(jr % P.R2)), w);
}

// Word w of the sequence of Open entry o (table slot `slot`, or a new entry of
// this round when slot < 0).
__device__ __forceinline__ uint32_t entry_word(const Params& P, int slot, long long o, int w) {
    if (slot >= 0) return P.H.seq[(size_t)slot * P.W + w];
    return new_word(P, o - P.ctl->batch_begin, w);
}

__device__ __forceinline__ bool entries_equal(const Params& P, int sa, long long a, int sb, long long b) {
    for (int w = 0; w < P.W; ++w)
        if (entry_word(P, sa, a, w) != entry_word(P, sb, b, w)) return false;
    return true;
}

enum { INS_NONE = 0, INS_CLAIMED = 1, INS_PENDING = 2 };

// Phase 1: claim an empty slot or stop at a slot holding the same key.
__device__ int claim_or_pend(const Params& P, unsigned long long key, int src, int flip, int32_t E,
                             int* slot_out) {
    const Table& H = P.H;
    uint64_t s = key & H.mask;
    for (uint64_t probe = 0; probe <= H.mask; ++probe) {
        const unsigned long long prev = atomicCAS(&H.rec[s].key, 0ull, key);
        if (prev == 0ull) {
            H.tag[s] = tag_of(key);
            for (int w = 0; w < H.W; ++w) H.seq[s * H.W + w] = src_word(P, src, flip, w);
            H.rec[s].E = E;
            H.rec[s].state = ST_OPEN;
            *slot_out = (int)s;
            return INS_CLAIMED;
        }
        if (prev == key) {
            *slot_out = (int)s;
            return INS_PENDING;
        }
        s = (s + 1) & H.mask;
    }
    atomicExch(&P.ctl->error, 2);
    return INS_NONE;
}

__device__ __forceinline__ void push_open(const Params& P, bool take, int32_t E, int slot,
                                          unsigned long long key) {
    Ctl* c = P.ctl;
    const long long o = block_append(&c->n_tot, take);
    if (take && o >= P.cap_o) atomicExch(&c->error, 4);
    if (take && o < P.cap_o) {
        P.oE[c->which][o] = E;
        P.oS[c->which][o] = slot;
        P.oZ[c->which][o] = key;
    }
    atomic_min_batch(c, take, E);
}

__device__ __forceinline__ void push_pending(const Params& P, bool take, const Pend& pd) {
    Ctl* c = P.ctl;
    const long long o = block_append(&c->n_pend, take);
    if (take && o >= P.cap_pend) atomicExch(&c->error, 5);
    if (take && o < P.cap_pend) P.pend[o] = pd;
}

// Words a sequence compare or copy loads together before it uses them (a loop that
// uses each word as it loads it waits for every load in turn); small, as the
// registers they take count against every kernel's occupancy.
constexpr int kWordChunk = 8;

// Whether table slot s holds pivot slot ps's sequence with element `flip` (1-based)
// flipped.  The pivot's words come from `pkl` (a copy in LDS) when given, else from
// its table row.
__device__ __forceinline__ bool flip_equal(const Params& P, uint64_t s, int ps, int flip, const uint32_t* pkl) {
    const int W = P.H.W;
    const uint32_t* row = P.H.seq + s * W;
    const uint32_t* pr = P.H.seq + (size_t)ps * W;
    const int fw = (flip - 1) >> 5;
    const uint32_t fm = 1u << (31 - ((flip - 1) & 31));
    bool eq = true;
    for (int w0 = 0; w0 < W && eq; w0 += kWordChunk) {
        uint32_t a[kWordChunk], b[kWordChunk];
#pragma unroll
        for (int w = 0; w < kWordChunk; ++w) {
            a[w] = w0 + w < W ? row[w0 + w] : 0u;
            b[w] = w0 + w < W ? (pkl ? pkl[w0 + w] : pr[w0 + w]) : 0u;
        }
#pragma unroll
        for (int w = 0; w < kWordChunk; ++w) eq &= (a[w] ^ b[w]) == (w0 + w == fw ? fm : 0u);
    }
    return eq;
}

// A generated neighbour (flip position `flip` of the block's pivot, slot ps;
// energy En; Zobrist key): its Open position is fixed by (pivot, flip).  It is
// DEAD when a lower-numbered pivot of the round produces the same sequence
// (`repeated`) or when H holds its sequence as OPEN or CLOSED; otherwise it is a
// new entry.  `taken`, `mn` and `mx` accumulate per thread; `home_tag` is the home
// slot's tag when the caller loaded it ahead (else -1), `pkl` the pivot's words in
// LDS when the caller holds them (else null).
__device__ __forceinline__ void stage_neighbour(const Params& P, int cur, long long batch_begin, bool valid,
                                                bool repeated, unsigned long long key, int ps, int flip,
                                                int32_t En, int& taken, int32_t& mn, int32_t& mx,
                                                int home_tag = -1, const uint32_t* pkl = nullptr) {
    if (!valid) return;
    const long long j = (long long)blockIdx.x * P.L + (flip - 1);
    int tomb = -1;
    bool take = !repeated;
    if (take) {
        const Table& H = P.H;
        const uint8_t tg = tag_of(key);
        uint64_t s = key & H.mask;
        for (uint64_t probe = 0; probe <= H.mask; ++probe, s = (s + 1) & H.mask) {
            // the home slot's tag may have been loaded ahead by the caller
            const uint8_t ts = (probe == 0 && home_tag >= 0) ? (uint8_t)home_tag : H.tag[s];
            if (ts == 0) break;
            if (ts != tg) continue;
            const SlotRec rc = H.rec[s];   // key and state in one load (no slot changes here)
            if (rc.key != key || !flip_equal(P, s, ps, flip, pkl)) continue;
            if (rc.state == ST_EVICTED) tomb = (int)s;
            else take = false;
            break;
        }
    }
    const long long o = batch_begin + j;
    if (!take) {
        P.oE[cur][o] = DEAD;
        return;
    }
    P.oE[cur][o] = En;
    P.oS[cur][o] = -1;
    P.oZ[cur][o] = key;
    P.ntomb[j] = tomb;
    ++taken;
    mn = En < mn ? En : mn;
    mx = En > mx ? En : mx;
}

// The block's pushed count and least energy (every thread calls it once).
__device__ void stage_finish(const Params& P, int taken, int32_t mn, int32_t mx) {
    __shared__ int s_cnt[16];
    __shared__ int32_t s_min[16], s_max[16];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int nw = (blockDim.x + 63) >> 6;
    taken = __ockl_wfred_add_i32(taken);
    mn = __ockl_wfred_min_i32(mn);
    mx = (int32_t)__ockl_wfred_max_u32((uint32_t)mx);   // energies are >= 0
    if (lane == 0) {
        s_cnt[wv] = taken;
        s_min[wv] = mn;
        s_max[wv] = mx;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int t = 0;
        int32_t m = INT32_MAX, x = 0;
        for (int k = 0; k < nw; ++k) {
            t += s_cnt[k];
            m = s_min[k] < m ? s_min[k] : m;
            x = s_max[k] > x ? s_max[k] : x;
        }
        P.bcnt[blockIdx.x] = t;
        P.bmin[blockIdx.x] = m;
        P.bmax[blockIdx.x] = x;
    }
}

// ---------------------------------------------------------------- seeding
__global__ __launch_bounds__(64) void k_seed(Params P, long long n_cand) {
    __shared__ int8_t sv[kSv];
    const int lane = threadIdx.x;
    const long long j = blockIdx.x;
    const int L = P.L, W = P.W;
    const uint32_t* wrd = P.cands + j * W;
    for (int i = lane; i < kSv; i += 64) sv[i] = 0;
    __syncthreads();
    for (int x = 1 + lane; x <= L; x += 64) sv[kPad + x] = packed_bit(wrd, x) ? 1 : -1;
    __syncthreads();
    int e = 0;
    for (int d = 1 + lane; d <= L - 1; d += 64) {
        int cd = 0;
        for (int i = 1; i <= L - d; ++i) cd += (int)sv[kPad + i] * (int)sv[kPad + i + d];
        e += cd * cd;
    }
    e = __ockl_wfred_add_i32(e);
    unsigned long long h = 0;
    for (int x = 1 + lane; x <= L; x += 64)
        if (sv[kPad + x] > 0) h ^= zob(x - 1);
    for (int o = 32; o > 0; o >>= 1) h ^= __shfl_xor(h, o, 64);
    const unsigned long long key = h | 1ull;
    int slot = -1, res = INS_NONE;
    if (lane == 0) res = claim_or_pend(P, key, (int)(-j - 1), 0, e, &slot);
    push_open(P, res == INS_CLAIMED, e, slot, key);
    Pend pd{slot, (int)(-j - 1), 0, e};
    push_pending(P, res == INS_PENDING, pd);
}

// ---------------------------------------------------------------- phases 2 and 3
__global__ __launch_bounds__(512) void k_resolve(Params P) {
    Ctl* c = P.ctl;
    if (c->stop) return;
    const long long n = c->n_pend < P.cap_pend ? c->n_pend : P.cap_pend;
    for (long long base = (long long)blockIdx.x * blockDim.x; base < n;
         base += (long long)gridDim.x * blockDim.x) {
        const long long q = base + threadIdx.x;
        bool pushed = false, coll = false;
        Pend pd{0, 0, 0, 0};
        if (q < n) {
            pd = P.pend[q];
            bool eq = true;
            for (int w = 0; w < P.W; ++w)
                if (P.H.seq[(size_t)pd.slot * P.W + w] != src_word(P, pd.src, pd.flip, w)) {
                    eq = false;
                    break;
                }
            if (!eq) coll = true;
            else if (P.H.rec[pd.slot].state == ST_EVICTED &&
                     atomicCAS(&P.H.rec[pd.slot].state, ST_EVICTED, ST_OPEN) == ST_EVICTED)
                pushed = true;
        }
        push_open(P, pushed, pd.E, pd.slot, pushed ? P.H.rec[pd.slot].key : 0ull);
        const long long o = block_append(&c->n_slow, coll);
        if (coll && o < P.cap_pend) P.slow[o] = pd;
    }
}

// Phase 3: key collisions, one at a time (no concurrency, so plain accesses).
__global__ void k_slow(Params P) {
    Ctl* c = P.ctl;
    if (c->stop || c->n_slow == 0) return;
    const Table& H = P.H;
    const long long n = c->n_slow < P.cap_pend ? c->n_slow : P.cap_pend;
    for (long long q = 0; q < n; ++q) {
        const Pend pd = P.slow[q];
        const unsigned long long key = H.rec[pd.slot].key;
        uint64_t s = (pd.slot + 1) & H.mask;
        for (uint64_t probe = 0; probe <= H.mask; ++probe, s = (s + 1) & H.mask) {
            if (H.rec[s].key == 0ull) {
                H.rec[s].key = key;
                H.tag[s] = tag_of(key);
                for (int w = 0; w < H.W; ++w) H.seq[s * H.W + w] = src_word(P, pd.src, pd.flip, w);
                H.rec[s].E = pd.E;
                H.rec[s].state = ST_OPEN;
                const long long o = c->n_tot++;
                if (o < P.cap_o) {
                    P.oE[c->which][o] = pd.E;
                    P.oS[c->which][o] = (int)s;
                    P.oZ[c->which][o] = key;
                }
                if (pd.E < c->batch_minE) c->batch_minE = pd.E;
                break;
            }
            if (H.rec[s].key != key) continue;
            bool eq = true;
            for (int w = 0; w < H.W; ++w)
                if (H.seq[s * H.W + w] != src_word(P, pd.src, pd.flip, w)) { eq = false; break; }
            if (!eq) continue;
            if (H.rec[s].state == ST_EVICTED) {
                H.rec[s].state = ST_OPEN;
                const long long o = c->n_tot++;
                if (o < P.cap_o) {
                    P.oE[c->which][o] = pd.E;
                    P.oS[c->which][o] = (int)s;
                    P.oZ[c->which][o] = key;
                }
                if (pd.E < c->batch_minE) c->batch_minE = pd.E;
            }
            break;
        }
    }
}

// Repeats within a round: a neighbour y = p_b (+) e_i equals a neighbour of pivot
// b' exactly when p_b (+) p_b' = e_i (+) e_i' with i != i', i.e. the two pivots
// are at Hamming distance 2 and i is one of the two positions where they differ
// (y equal to a pivot itself is a CLOSED entry of H).  Block b compares its pivot
// with every lower-numbered pivot and marks its copies of the shared neighbours,
// so of every repeated sequence exactly the copy of the lowest pivot is kept.
// The direct expansion's repeat map (the bit-sliced one compares in its own block).
constexpr int kRepTile = 64;

__global__ __launch_bounds__(256) void k_repeats(Params P) {
    Ctl* c = P.ctl;
    const int tb = blockIdx.y, tq = blockIdx.x;   // pivot tiles: higher (b) and lower (q)
    if (c->stop || tq > tb) return;
    const long long n = c->n_piv;
    const int b0 = tb * kRepTile, q0 = tq * kRepTile;
    if (b0 >= n) return;
    const int L = P.L, W = P.W;
    __shared__ uint32_t sb[kRepTile][33], sq[kRepTile][33];
    for (int e = threadIdx.x; e < kRepTile * W; e += blockDim.x) {
        const int r = e / W, w = e % W;
        sb[r][w] = (b0 + r < n) ? P.H.seq[(size_t)P.piv[b0 + r] * W + w] : 0u;
        sq[r][w] = (q0 + r < n) ? P.H.seq[(size_t)P.piv[q0 + r] * W + w] : 0u;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < kRepTile * kRepTile; e += blockDim.x) {
        const int rb = e / kRepTile, rq = e % kRepTile;
        const long long bi = b0 + rb, qi = q0 + rq;
        if (bi >= n || qi >= bi) continue;
        int d = 0;
        for (int w = 0; w < W; ++w) d += __popc(sb[rb][w] ^ sq[rq][w]);
        if (d != 2) continue;
        int first = -1, second = -1;
        for (int w = 0; w < W; ++w) {
            uint32_t x = sb[rb][w] ^ sq[rq][w];
            while (x) {
                const int k = __clz((int)x);
                const int pos = 32 * w + k + 1;   // 1-based position, MSB first
                if (first < 0) first = pos;
                else second = pos;
                x &= ~(0x80000000u >> k);
            }
        }
        uint8_t* row = P.repeat + bi * L;
        row[first - 1] = 1;
        row[second - 1] = 1;
    }
}

// ---------------------------------------------------------------- round control
// The capacity cut (T = Q smallest survive; sel_all: nothing is evicted) together
// with the next round's pivots (T2 = min(B, X - expansions) smallest of the
// survivors, which are the T2 smallest overall).  sel_enabled: some threshold
// needs the histogram.
__device__ void cut_setup(const Params& P) {
    Ctl* c = P.ctl;
    c->T = P.Q;
    c->sel_all = c->n_live > P.Q ? 0 : 1;
    long long T2 = P.X - c->expansions;
    if (T2 > P.B) T2 = P.B;
    const long long surv = c->sel_all ? c->n_live : P.Q;
    c->T2 = T2;
    c->dual = T2 > 0 ? 1 : 0;
    c->dual_all = T2 >= surv ? 1 : 0;
    c->sel_enabled = (!c->sel_all || (c->dual && !c->dual_all)) ? 1 : 0;
    c->c_lt2 = 0;
    c->out_count2 = 0;
    c->resolved2 = 1;
    c->Dt2 = 0;
    c->prefix2 = 0;
    c->survivors = 0;
    c->n_pivpos = 0;
    c->out_count = 0;
    c->zv = 0;
    c->zv2 = 0;
    c->n_bestc = 0;
}

// next_piv: the table slots of the pivots the last cut took out of Open for the
// coming round.  One thread.
__device__ void round_begin(const Params& P, const int32_t* next_piv, Ctl* c) {
    if (c->stop) return;
    if (c->n_live == 0 || c->expansions >= P.X || c->u >= P.T_u) {
        // the search ends: pivots taken out for a round that does not run go back
        // into Open (OPEN in the table, their energies in the list)
        const int cur = c->which;
        const long long n = c->n_pivpos < P.B ? c->n_pivpos : P.B;
        for (long long b = 0; b < n; ++b) {
            const int sl = next_piv[b];
            P.H.rec[sl].state = ST_OPEN;
            P.oE[cur][P.pivpos[b]] = P.H.rec[sl].E;
        }
        c->n_pivpos = 0;
        c->stop = 1;
        return;
    }
    long long T = P.X - c->expansions;
    if (T > P.B) T = P.B;
    c->T = T;
    // the last cut selected this round's T pivots and listed their positions
    c->presel = c->dual && c->T2 == T ? 1 : 0;
    c->dual = 0;
    c->sel_enabled = 0;
    c->sel_all = 0;
    if (!c->presel) {   // cannot happen while the search goes on
        atomicExch(&c->error, 7);
        c->stop = 1;
        return;
    }
    // the last cut took this round's pivots out of Open (CLOSED in the table, DEAD
    // in the list) and copied their slots and words
    if (c->n_pivpos > P.B) atomicExch(&c->error, 3);
    c->n_piv = c->n_pivpos < P.B ? c->n_pivpos : P.B;
    c->n_live0 = c->n_live;
    c->expansions0 = c->expansions;
    c->n_pend = 0;
    c->n_slow = 0;
    c->batch_begin = c->n_tot;
    c->batch_minE = INT32_MAX;
    c->improved = 0;
    c->emin = c->blo;   // the live entries are a subset of the last cut's survivors
    c->emax = c->bhi;
    c->out_count = 0;
}

__global__ void k_round_begin(Params P) { round_begin(P, P.piv, P.ctl); }

// ---------------------------------------------------------------- selection
// Selects the T smallest live Open entries in key order into flag[].
__global__ __launch_bounds__(kSelThreads) void k_sel_minmax(Params P) {
    Ctl* c = P.ctl;
    if (c->stop || !c->sel_enabled) return;
    __shared__ uint32_t smn, smx;
    if (threadIdx.x == 0) {
        smn = UINT32_MAX;
        smx = 0;
    }
    __syncthreads();
    const int cur = c->which;
    uint32_t mn = UINT32_MAX, mx = 0;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < c->n_tot;
         i += (long long)gridDim.x * blockDim.x) {
        const int32_t e = P.oE[cur][i];
        if (e != DEAD) {
            mn = min(mn, (uint32_t)e);
            mx = max(mx, (uint32_t)e);
        }
    }
    mn = (uint32_t)__ockl_wfred_min_i32((int)min(mn, (uint32_t)INT32_MAX));
    mx = __ockl_wfred_max_u32(mx);
    if ((threadIdx.x & 63) == 0) {
        atomicMin(&smn, mn);
        atomicMax(&smx, mx);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        atomicMin(&c->emin, smn);
        atomicMax(&c->emax, smx);
    }
}

// The digit layout from [emin, emax]: D has hs bits; the histogram bins D >> ls.
__device__ __forceinline__ void digit_shifts(const Ctl* c, int* hs, int* ls) {
    const uint32_t R = (c->emax - c->emin) >> 2;
    const int nbits = R ? 32 - __clz((int)R) : 0;
    *hs = nbits;
    *ls = nbits > kSelBits ? nbits - kSelBits : 0;
}

// Block histograms of D >> ls over the live Open entries, merged into one.
__global__ __launch_bounds__(kSelThreads) void k_sel_hist(Params P) {
    Ctl* c = P.ctl;
    if (c->stop || !c->sel_enabled) return;
    if (c->emax == c->emin) return;
    __shared__ uint32_t h[kSelBins];
    int hs, ls;
    digit_shifts(c, &hs, &ls);
    const int nbins = 1 << (hs - ls);   // bins in use
    for (int b = threadIdx.x; b < nbins; b += blockDim.x) h[b] = 0;
    __syncthreads();
    const int cur = c->which;
    const uint32_t emin = c->emin;
    const uint32_t dmask = (1u << (hs - ls)) - 1u;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < c->n_tot;
         i += (long long)gridDim.x * blockDim.x) {
        const int32_t e = P.oE[cur][i];
        if (e == DEAD) continue;
        const uint32_t D = ((uint32_t)e - emin) >> 2;
        if (hs < 32 && (D >> hs) != 0u) continue;
        atomicAdd(&h[(D >> ls) & dmask], 1u);
    }
    __syncthreads();
    for (int b = threadIdx.x; b < nbins; b += blockDim.x)
        if (h[b]) atomicAdd(&P.ghist[b], h[b]);
}

// The round's counts and the histogram in one launch.  Every workgroup reduces
// the expansion's per-pivot counts and energy bounds and derives the round's
// values (the statistics and cut_setup's decisions) from fields no workgroup
// writes here; workgroup 0 stores them in the control block; then the energy
// histogram of the live entries, as k_sel_hist.  (The best sequence of an
// improving round is found by the classify pass and the tie select.)
struct MidVals {
    long long n_tot, n_live, expansions, cnt, T2;
    int32_t mn, mx, sel_all, dual, dual_all, sel_enabled;
    uint32_t emin, emax;
};

__global__ __launch_bounds__(kSelThreads) void k_mid_hist(Params P) {
    __shared__ long long s_cnt[kSelThreads / 64];
    __shared__ int32_t s_min[kSelThreads / 64], s_max[kSelThreads / 64];
    __shared__ MidVals m;
    __shared__ Ctl cs;
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    // the first pivots' counts (in bounds for any count) load with the control block
    const bool pre = t < P.B;
    const int32_t pc0 = pre ? P.bcnt[t] : 0, pmn0 = pre ? P.bmin[t] : INT32_MAX, pmx0 = pre ? P.bmax[t] : 0;
    snap_ctl(cs, P.ctl);
    const Ctl* c = &cs;
    Ctl* cg = P.ctl;
    if (c->stop) return;
    const long long np = c->n_piv;
    // this workgroup's first kHistItems entries per thread, loaded while the round's
    // counts are reduced (the list's length needs only the pivot count)
    const int cur = c->which;
    const long long n_tot = c->batch_begin + np * (P.L + P.R2);
    int32_t ev[kHistItems];
    const long long hbase = (long long)blockIdx.x * blockDim.x * kHistItems + t;
#pragma unroll
    for (int k = 0; k < kHistItems; ++k) {
        const long long i = hbase + (long long)k * blockDim.x;
        ev[k] = i < n_tot ? P.oE[cur][i] : DEAD;
    }
    long long cnt = 0;
    int32_t mn = INT32_MAX, mx = 0;
    for (long long b = t; b < np; b += blockDim.x) {
        const int32_t bc = b == t ? pc0 : P.bcnt[b];
        const int32_t bn = b == t ? pmn0 : P.bmin[b];
        const int32_t bx = b == t ? pmx0 : P.bmax[b];
        cnt += bc;
        mn = bn < mn ? bn : mn;
        mx = bx > mx ? bx : mx;
    }
    for (int o = 32; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o, 64);
    mn = __ockl_wfred_min_i32(mn);
    mx = (int32_t)__ockl_wfred_max_u32((uint32_t)mx);
    if (lane == 0) {
        s_cnt[wv] = cnt;
        s_min[wv] = mn;
        s_max[wv] = mx;
    }
    __syncthreads();
    if (t == 0) {
        cnt = s_cnt[0];
        mn = s_min[0];
        mx = s_max[0];
        for (int k = 1; k < (int)(blockDim.x >> 6); ++k) {
            cnt += s_cnt[k];
            mn = s_min[k] < mn ? s_min[k] : mn;
            mx = s_max[k] > mx ? s_max[k] : mx;
        }
        m.cnt = cnt;
        m.mn = mn;
        m.mx = mx;
        m.n_tot = c->batch_begin + np * (P.L + P.R2);
        m.n_live = c->n_live0 - np + cnt;
        m.expansions = c->expansions0 + np;
        // cut_setup's decisions on the round's values
        m.sel_all = m.n_live > P.Q ? 0 : 1;
        long long T2 = P.X - m.expansions;
        if (T2 > P.B) T2 = P.B;
        const long long surv = m.sel_all ? m.n_live : P.Q;
        m.T2 = T2;
        m.dual = T2 > 0 ? 1 : 0;
        m.dual_all = T2 >= surv ? 1 : 0;
        m.sel_enabled = (!m.sel_all || (m.dual && !m.dual_all)) ? 1 : 0;
        m.emin = (uint32_t)mn < c->blo ? (uint32_t)mn : c->blo;
        m.emax = (uint32_t)mx > c->bhi ? (uint32_t)mx : c->bhi;
        if (blockIdx.x == 0) {
            cg->n_tot = m.n_tot;
            cg->batch_minE = mn;
            cg->expansions = m.expansions;
            cg->n_live = m.n_live;
            cg->pushes = c->pushes + cnt;
            cg->dups = c->dups + np * (P.L + P.R2) - cnt;
            if (mn < c->best_E) cg->improved = 1;
            else cg->u = c->u + np;
            cut_setup(P);
            cg->emin = m.emin;
            cg->emax = m.emax;
        }
    }
    __syncthreads();
    if (!m.sel_enabled || m.emax == m.emin) return;
    __shared__ uint32_t h[kSelBins];
    const uint32_t R = (m.emax - m.emin) >> 2;
    const int hs = R ? 32 - __clz((int)R) : 0;
    const int ls = hs > kSelBits ? hs - kSelBits : 0;
    const int nbins = 1 << (hs - ls);   // bins in use
    for (int b = t; b < nbins; b += blockDim.x) h[b] = 0;
    __syncthreads();
    const uint32_t emin = m.emin;
    const uint32_t dmask = (1u << (hs - ls)) - 1u;
    auto add = [&](int32_t e) {
        if (e == DEAD) return;
        const uint32_t D = ((uint32_t)e - emin) >> 2;
        if (hs < 32 && (D >> hs) != 0u) return;
        atomicAdd(&h[(D >> ls) & dmask], 1u);
    };
#pragma unroll
    for (int k = 0; k < kHistItems; ++k) add(ev[k]);
    // longer lists: the rest in passes of kHistItems loads per thread
    const long long stride = (long long)gridDim.x * blockDim.x * kHistItems;
    for (long long base = hbase + stride; base < n_tot; base += stride) {
#pragma unroll
        for (int k = 0; k < kHistItems; ++k) {
            const long long i = base + (long long)k * blockDim.x;
            ev[k] = i < n_tot ? P.oE[cur][i] : DEAD;
        }
#pragma unroll
        for (int k = 0; k < kHistItems; ++k) add(ev[k]);
    }
    __syncthreads();
    for (int b = t; b < nbins; b += blockDim.x)
        if (h[b]) atomicAdd(&P.ghist[b], h[b]);
}

// The cut from the histogram: the bin holding the T-th smallest entry (and, for a
// dual cut, the T2-th).  A bin is resolved when bins are single values of D
// (ls = 0); otherwise the bin [prefix << ls, (prefix + 1) << ls) is left to the tie
// select.  Every workgroup of the classify pass computes it (the histogram is
// read-only there); workgroup 0 stores it for the tie select and the cut.
struct SelCut {
    long long c_lt, c_lt2;
    uint32_t prefix, prefix2, Dt, Dt2;
    int32_t resolved, resolved2, hi_shift;
};

__device__ void find_cut(const Params& P, const Ctl* c, SelCut* out) {
    __shared__ uint32_t part[kSelThreads / 64];
    const int t = threadIdx.x;
    if (t == 0) {
        out->c_lt = 0;
        out->c_lt2 = 0;
        out->prefix = 0;
        out->prefix2 = 0;
        out->Dt = 0;
        out->Dt2 = 0;
        out->resolved = 1;
        out->resolved2 = 1;
        out->hi_shift = 0;
    }
    __syncthreads();
    if (c->emax == c->emin) return;   // every live entry has one energy
    int hs, ls;
    digit_shifts(c, &hs, &ls);
    const int nb = 1 << (hs - ls);      // bins in use
    const int per = (nb + (int)blockDim.x - 1) / (int)blockDim.x;
    const int b0 = t * per;
    uint32_t a = 0;
    for (int k = 0; k < per; ++k)
        if (b0 + k < nb) a += P.ghist[b0 + k];
    // exclusive prefix of the chunk sums: within the wave by shuffles, then the
    // totals of the lower waves
    const int lane = t & 63, wv = t >> 6;
    uint32_t incl = a;
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(incl, o, 64);
        if (lane >= o) incl += y;
    }
    if (lane == 63) part[wv] = incl;
    __syncthreads();
    uint32_t below = 0;
    for (int k = 0; k < wv; ++k) below += part[k];
    const long long first = (long long)below + incl - a;   // entries in the bins before this chunk
    if (t == 0) out->hi_shift = ls;
    // the chunk holding the need-th smallest entry finds its bin
    auto locate = [&](long long need, long long* c_lt, uint32_t* prefix, uint32_t* Dt, int32_t* resolved) {
        if (!(first < need && need <= first + a)) return;
        long long before = first;
        int v = b0;
        for (int k = 0; k < per && b0 + k < nb; ++k) {
            const uint32_t cnt = P.ghist[b0 + k];
            if (before + cnt >= need) {
                v = b0 + k;
                break;
            }
            before += cnt;
        }
        *c_lt = before;
        *prefix = (uint32_t)v;
        *Dt = (uint32_t)v;
        *resolved = ls == 0 ? 1 : 0;
    };
    if (!c->sel_all) locate(c->T, &out->c_lt, &out->prefix, &out->Dt, &out->resolved);
    if (c->dual && !c->dual_all) locate(c->T2, &out->c_lt2, &out->prefix2, &out->Dt2, &out->resolved2);
    __syncthreads();
}

__device__ __forceinline__ bool entry_less(const Params& P, int cur, long long a, long long b);

// This workgroup's least entry (by key, then sequence) among the round's new
// entries of the round's least energy, in the classify pass's entry layout.
__device__ void best_offer(const Params& P, const Ctl* c) {
    __shared__ long long best[kSelThreads];
    const int cur = c->which;
    const int32_t target = c->batch_minE;
    const long long lo = c->batch_begin, n_tot = c->n_tot;
    long long mine = -1;
    const long long stride = (long long)gridDim.x * blockDim.x * kItems;
    for (long long base = (long long)blockIdx.x * blockDim.x * kItems; base < n_tot; base += stride)
        for (int k = 0; k < kItems; ++k) {
            const long long i = base + threadIdx.x + (long long)k * blockDim.x;
            if (i < lo || i >= n_tot || P.oE[cur][i] != target) continue;
            if (mine < 0 || entry_less(P, cur, i, mine)) mine = i;
        }
    best[threadIdx.x] = mine;
    __syncthreads();
    for (int o = (int)blockDim.x >> 1; o > 0; o >>= 1) {
        if (threadIdx.x < (unsigned)o) {
            const long long x = best[threadIdx.x], y = best[threadIdx.x + o];
            if (x < 0 || (y >= 0 && entry_less(P, cur, y, x))) best[threadIdx.x] = y;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0 && best[0] >= 0)
        P.bestc[atomicAdd((unsigned long long*)&P.ctl->n_bestc, 1ull)] = (int32_t)best[0];
    __syncthreads();
}

// The tie select's third workgroup: the least offer becomes the best.
__device__ void best_take(const Params& P, const Ctl* c) {
    Ctl* cg = P.ctl;
    __shared__ long long best[1024];
    const int cur = c->which;
    const long long n = c->n_bestc;
    long long mine = -1;
    for (long long q = threadIdx.x; q < n; q += blockDim.x) {
        const long long i = P.bestc[q];
        if (mine < 0 || entry_less(P, cur, i, mine)) mine = i;
    }
    best[threadIdx.x] = mine;
    __syncthreads();
    for (int o = (int)blockDim.x >> 1; o > 0; o >>= 1) {
        if (threadIdx.x < (unsigned)o) {
            const long long x = best[threadIdx.x], y = best[threadIdx.x + o];
            if (x < 0 || (y >= 0 && entry_less(P, cur, y, x))) best[threadIdx.x] = y;
        }
        __syncthreads();
    }
    const long long b = best[0];
    if (b >= 0 && threadIdx.x < (unsigned)P.W)
        P.best_seq[threadIdx.x] = entry_word(P, P.oS[cur][b], b, threadIdx.x);
    if (threadIdx.x == 0 && b >= 0) {
        cg->best_slot = 1;
        cg->best_E = c->batch_minE;
        cg->best_round = (int32_t)c->rounds;
        cg->u = 0;
    }
}

__global__ __launch_bounds__(kSelThreads) void k_sel_classify(Params P) {
    __shared__ Ctl cs;
    snap_ctl(cs, P.ctl);
    const Ctl* c = &cs;
    Ctl* cg = P.ctl;
    if (c->stop) return;
    const int nblk = (int)gridDim.x;
    // the first pass's energies load while the cut is found
    const int cur = c->which;
    const long long n_tot = c->n_tot;
    const long long base0 = (long long)blockIdx.x * blockDim.x * kItems;
    int32_t e0[kItems];
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        const long long i = base0 + threadIdx.x + (long long)k * blockDim.x;
        e0[k] = i < n_tot ? P.oE[cur][i] : DEAD;
    }
    // a round that improved on the best: every workgroup offers its least (key,
    // sequence) among its new entries at the round's least energy; the tie select
    // takes the least of the offers
    if (P.best_in_classify && c->improved) best_offer(P, c);
    if (!c->sel_enabled) return;
    __shared__ SelCut cut;
    find_cut(P, c, &cut);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        cg->c_lt = cut.c_lt;
        cg->prefix = cut.prefix;
        cg->Dt = cut.Dt;
        cg->resolved = cut.resolved;
        cg->hi_shift = cut.hi_shift;
        cg->c_lt2 = cut.c_lt2;
        cg->prefix2 = cut.prefix2;
        cg->Dt2 = cut.Dt2;
        cg->resolved2 = cut.resolved2;
    }
    const bool all = c->sel_all;
    // resolved: the threshold energy Et; otherwise the threshold bin [Dlo, Dhi) of D
    const bool res = cut.resolved;
    const uint32_t Et = c->emin + (cut.Dt << 2);
    const uint32_t emin = c->emin;
    const uint32_t Dlo = res ? 0u : cut.prefix << cut.hi_shift;
    const uint32_t Dhi = res ? 0u : (cut.prefix + 1u) << cut.hi_shift;
    // the dual cut's second threshold (bit 1 of flag: the next round's pivots)
    const bool dual = c->dual;
    const bool dual_all = c->dual_all;
    const bool res2 = cut.resolved2;
    const uint32_t Et2 = c->emin + (cut.Dt2 << 2);
    const uint32_t D2lo = cut.prefix2 << cut.hi_shift;
    const uint32_t D2hi = (cut.prefix2 + 1u) << cut.hi_shift;
    // top key bytes of the entries tied at a resolved threshold energy
    __shared__ uint32_t zh[2 * kZBins];
    for (int b = threadIdx.x; b < 2 * kZBins; b += blockDim.x) zh[b] = 0;
    __syncthreads();
    const long long stride = (long long)nblk * blockDim.x * kItems;
    for (long long base = (long long)blockIdx.x * blockDim.x * kItems; base < n_tot; base += stride) {
        bool tie[kItems], tie2[kItems];
        int cnt = 0, cnt2 = 0;
#pragma unroll
        for (int k = 0; k < kItems; ++k) {
            const long long i = base + threadIdx.x + (long long)k * blockDim.x;
            tie[k] = false;
            tie2[k] = false;
            if (i < n_tot) {
                const int32_t e = base == base0 ? e0[k] : P.oE[cur][i];
                uint32_t f = 0;
                if (e != DEAD) {
                    const uint32_t D = ((uint32_t)e - emin) >> 2;
                    if (all) {
                        f = 1;
                    } else if (res) {
                        if ((uint32_t)e < Et) f = 1;
                        else if ((uint32_t)e == Et) {
                            tie[k] = true;
                            f = 4u;
                        }
                    } else {
                        if (D < Dlo) f = 1;
                        else if (D < Dhi) tie[k] = true;
                    }
                    if (dual && dual_all) {
                        f |= 2u;
                    } else if (dual) {
                        if (res2) {
                            if ((uint32_t)e < Et2) f |= 2u;
                            else if ((uint32_t)e == Et2) {
                                tie2[k] = true;
                                f |= 8u;
                            }
                        } else {
                            if (D < D2lo) f |= 2u;
                            else if (D < D2hi) tie2[k] = true;
                        }
                    }
                }
                P.flag[i] = f;
            }
            cnt += tie[k] ? 1 : 0;
            cnt2 += tie2[k] ? 1 : 0;
        }
        long long o, o2;
        if (dual && !dual_all) block_append2(&cg->out_count, cnt, &cg->out_count2, cnt2, &o, &o2);   // uniform
        else o = block_append_n(&cg->out_count, cnt);
#pragma unroll
        for (int k = 0; k < kItems; ++k)
            if (tie[k]) {
                const long long i = base + threadIdx.x + (long long)k * blockDim.x;
                const unsigned long long z = P.oZ[cur][i];
                P.cand[0][o] = (int32_t)i;
                P.candz[0][o] = z;
                if (res) atomicAdd(&zh[z >> 56], 1u);
                ++o;
            }
        if (dual && !dual_all) {   // uniform
#pragma unroll
            for (int k = 0; k < kItems; ++k)
                if (tie2[k]) {
                    const long long i = base + threadIdx.x + (long long)k * blockDim.x;
                    const unsigned long long z = P.oZ[cur][i];
                    P.cand2[0][o2] = (int32_t)i;
                    P.candz2[0][o2] = z;
                    if (res2) atomicAdd(&zh[kZBins + (z >> 56)], 1u);
                    ++o2;
                }
        }
    }
    __syncthreads();
    uint32_t* zcopy = P.ghist + kSelBins + (blockIdx.x % kZCopies) * 2 * kZBins;
    for (int b = threadIdx.x; b < 2 * kZBins; b += blockDim.x)
        if (zh[b]) atomicAdd(&zcopy[b], zh[b]);
}

// Tie digits of Open entry o: bytes 0..7 are its Zobrist key (most significant
// first), bytes 8.. its packed sequence.
__device__ __forceinline__ int tie_digit(const Params& P, int cur, long long o, int pos) {
    if (pos < 8) return (int)((P.oZ[cur][o] >> (56 - 8 * pos)) & 255ull);
    const int q = pos - 8;
    return (int)((entry_word(P, P.oS[cur][o], o, q >> 2) >> (24 - 8 * (q & 3))) & 255u);
}

// First tie-digit position >= pos at which Open entries a and b differ (npos if none).
__device__ __forceinline__ int first_diff(const Params& P, int cur, long long a, long long b, int pos, int npos) {
    if (pos < 8) {
        unsigned long long x = P.oZ[cur][a] ^ P.oZ[cur][b];
        x &= ~0ull >> (8 * pos);
        if (x) return __clzll((long long)x) >> 3;
        pos = 8;
    }
    const int q0 = pos - 8;
    const int sa = P.oS[cur][a], sb = P.oS[cur][b];
    for (int w = q0 >> 2; w < P.W; ++w) {
        uint32_t x = entry_word(P, sa, a, w) ^ entry_word(P, sb, b, w);
        if (w == (q0 >> 2)) x &= 0xffffffffu >> (8 * (q0 & 3));
        if (x) return 8 + 4 * w + (__clz((int)x) >> 3);
    }
    return npos;
}

// Among the tied candidates, flag the `T - c_lt` smallest in tie order: an MSD
// byte-wise radix select over the tie digits.  Each iteration first finds, in one
// pass, the first digit position (from `pos` on) at which any candidate differs
// from the first one, then partitions the candidates on that digit.
constexpr int kTieLds = 2048;   // ties resolved on Zobrist bytes in LDS up to this count
constexpr int kTieU = 8;        // candidates loaded ahead per thread in the global passes

// Block 0: the selection's own threshold (flag bit 0); block 1 (dual cuts): the
// second threshold, the next round's pivots (flag bit 1).  The two blocks share no
// state but the flag words, which they update by atomic ORs of different bits.
__global__ __launch_bounds__(1024) void k_sel_keys(Params P) {
    const int which = blockIdx.x;
    __shared__ Ctl cs;
    snap_ctl(cs, P.ctl);
    const Ctl* c = &cs;
    Ctl* cg = P.ctl;
    if (which == 2) {
        if (!c->stop && P.best_in_classify && c->improved) best_take(P, c);
        return;
    }
    if (c->stop || !c->sel_enabled) return;
    if (which ? (!c->dual || c->dual_all) : c->sel_all) return;
    int32_t* const* CA = which ? P.cand2 : P.cand;
    unsigned long long* const* CZ = which ? P.candz2 : P.candz;
    const uint32_t bit = which ? 2u : 1u;
    const uint32_t prefix = which ? c->prefix2 : c->prefix;
    __shared__ uint32_t h[256];
    __shared__ int s_pos, s_v, s_m2;
    __shared__ long long s_r;
    __shared__ unsigned long long zs[2][kTieLds];
    __shared__ int32_t is[2][kTieLds];
    const int cur = c->which;
    const int t = threadIdx.x;
    const int npos = 8 + 4 * P.W;
    int m = (int)(which ? c->out_count2 : c->out_count);
    long long r = which ? c->T2 - c->c_lt2 : c->T - c->c_lt;
    int src = 0;
    int pos = 0;
    // every thread reads the control block before thread 0 updates it below
    const bool unres = which ? !c->resolved2 : !c->resolved;
    const int ls = c->hi_shift;
    __syncthreads();
    if (unres && (ls > kSubBits || r >= m)) {
        // the whole bin is taken (or its width is out of range: an error the host sees)
        if (t == 0) {
            if (ls > kSubBits) atomicExch(&cg->error, 6);
            if (!which) {
                cg->Dt = ((prefix + 1u) << ls) - 1u;
                cg->resolved = 1;
            }
        }
        if (ls > kSubBits) return;
    } else if (unres && r > 0) {
        // The one radix level left a bin of 2^ls values of D: select its r smallest
        // values exactly (a histogram of D - Dlo in LDS, over the zs storage), keep
        // the entries below the threshold value, and go on with the tied ones.
        const uint32_t Dlo = prefix << ls;
        const uint32_t emin = c->emin;
        const int nsub = 1 << ls;
        uint32_t* hs = (uint32_t*)&zs[0][0];   // 2 * kTieLds * 8 bytes = 2^kSubBits counts
        for (int k = t; k < nsub; k += blockDim.x) hs[k] = 0;
        if (t == 0) s_m2 = 0;
        __syncthreads();
        for (int q0 = t; q0 < m; q0 += kTieU * blockDim.x) {
            uint32_t e[kTieU];
#pragma unroll
            for (int u = 0; u < kTieU; ++u) {
                const int q = q0 + u * blockDim.x;
                e[u] = q < m ? (uint32_t)P.oE[cur][CA[src][q]] : 0u;
            }
#pragma unroll
            for (int u = 0; u < kTieU; ++u)
                if (q0 + u * blockDim.x < m) atomicAdd(&hs[(e[u] - emin) / 4u - Dlo], 1u);
        }
        __syncthreads();
        if (t == 0) {
            long long cum = 0;
            int v = 0;
            for (; v < nsub; ++v) {
                if (cum + hs[v] >= r) break;
                cum += hs[v];
            }
            s_v = v;
            s_r = r - cum;
            if (!which) {
                cg->Dt = Dlo + (uint32_t)v;   // the cut's energy, for the next round's bounds
                cg->resolved = 1;
            }
        }
        __syncthreads();
        const uint32_t Dv = Dlo + (uint32_t)s_v;
        for (int q0 = t; q0 < m; q0 += kTieU * blockDim.x) {
            int idx[kTieU];
            uint32_t e[kTieU];
#pragma unroll
            for (int u = 0; u < kTieU; ++u) {
                const int q = q0 + u * blockDim.x;
                idx[u] = q < m ? CA[src][q] : -1;
            }
#pragma unroll
            for (int u = 0; u < kTieU; ++u) e[u] = idx[u] >= 0 ? (uint32_t)P.oE[cur][idx[u]] : 0u;
#pragma unroll
            for (int u = 0; u < kTieU; ++u) {
                if (idx[u] < 0) continue;
                const uint32_t D = (e[u] - emin) / 4u;
                if (D < Dv) atomicOr(&P.flag[idx[u]], bit);
                else if (D == Dv) {
                    const int o2 = atomicAdd(&s_m2, 1);
                    CA[1 - src][o2] = idx[u];
                    CZ[1 - src][o2] = CZ[src][q0 + u * blockDim.x];
                }
            }
        }
        __syncthreads();
        m = s_m2;
        r = s_r;
        src = 1 - src;
        __syncthreads();
    }
    if (!unres && m > kTieLds && r > 0 && r < m) {
        // The classify pass counted the tied entries' top key bytes: the threshold
        // byte v comes from that histogram, the tied entries below it are taken by
        // the cut itself (zv / zv2, flag bits 2 / 3), and one pass over the tied
        // entries keeps those of byte v.
        if (t < kZBins) {
            uint32_t v = 0;
            for (int cp = 0; cp < kZCopies; ++cp) v += P.ghist[kSelBins + cp * 2 * kZBins + kZBins * which + t];
            h[t] = v;
        }
        if (t == 0) s_m2 = 0;
        __syncthreads();
        if (t < 64) {
            const uint32_t c0 = h[4 * t], c1 = h[4 * t + 1], c2 = h[4 * t + 2], c3 = h[4 * t + 3];
            uint32_t inc = c0 + c1 + c2 + c3;
            for (int o = 1; o < 64; o <<= 1) {
                const uint32_t y = __shfl_up(inc, o, 64);
                if (t >= o) inc += y;
            }
            long long cum = (long long)inc - (c0 + c1 + c2 + c3);
            const uint32_t cs[4] = {c0, c1, c2, c3};
            for (int k = 0; k < 4; ++k) {
                if (cum < r && r <= cum + cs[k]) {
                    s_v = 4 * t + k;
                    s_r = r - cum;
                }
                cum += cs[k];
            }
        }
        __syncthreads();
        const int v = s_v;
        if (t == 0) {
            if (which) cg->zv2 = (uint32_t)v;
            else cg->zv = (uint32_t)v;
        }
        for (int q0 = t; q0 < m; q0 += kTieU * blockDim.x) {
            unsigned long long z[kTieU];
#pragma unroll
            for (int u = 0; u < kTieU; ++u) {
                const int q = q0 + u * blockDim.x;
                z[u] = q < m ? CZ[src][q] : 0ull;
            }
#pragma unroll
            for (int u = 0; u < kTieU; ++u) {
                const int q = q0 + u * blockDim.x;
                if (q < m && (int)(z[u] >> 56) == v) {
                    const int o2 = atomicAdd(&s_m2, 1);
                    CA[1 - src][o2] = CA[src][q];
                    CZ[1 - src][o2] = z[u];
                }
            }
        }
        __syncthreads();
        m = s_m2;
        r = s_r;
        src = 1 - src;
        pos = 1;
        __syncthreads();
    }
    // Large tie sets: partition on key bytes read from the Open list until the
    // remaining set fits in LDS (keys are pseudo-random, so one byte divides
    // the set by about 256).
    while (m > kTieLds && pos < 8 && r > 0 && r < m) {
        const int sh = 56 - 8 * pos;
        if (t < 256) h[t] = 0;
        if (t == 0) s_m2 = 0;
        __syncthreads();
        for (int q0 = t; q0 < m; q0 += kTieU * blockDim.x) {
            unsigned long long z[kTieU];
#pragma unroll
            for (int u = 0; u < kTieU; ++u) {
                const int q = q0 + u * blockDim.x;
                z[u] = q < m ? CZ[src][q] : 0ull;
            }
#pragma unroll
            for (int u = 0; u < kTieU; ++u)
                if (q0 + u * blockDim.x < m) atomicAdd(&h[(z[u] >> sh) & 255ull], 1u);
        }
        __syncthreads();
        if (t < 64) {
            const uint32_t c0 = h[4 * t], c1 = h[4 * t + 1], c2 = h[4 * t + 2], c3 = h[4 * t + 3];
            uint32_t inc = c0 + c1 + c2 + c3;
            for (int o = 1; o < 64; o <<= 1) {
                const uint32_t y = __shfl_up(inc, o, 64);
                if (t >= o) inc += y;
            }
            long long cum = (long long)inc - (c0 + c1 + c2 + c3);
            const uint32_t cs[4] = {c0, c1, c2, c3};
            for (int k = 0; k < 4; ++k) {
                if (cum < r && r <= cum + cs[k]) {
                    s_v = 4 * t + k;
                    s_r = r - cum;
                }
                cum += cs[k];
            }
        }
        __syncthreads();
        const int v = s_v;
        for (int q0 = t; q0 < m; q0 += kTieU * blockDim.x) {
            int idx[kTieU];
            unsigned long long z[kTieU];
#pragma unroll
            for (int u = 0; u < kTieU; ++u) {
                const int q = q0 + u * blockDim.x;
                idx[u] = q < m ? CA[src][q] : -1;
                z[u] = q < m ? CZ[src][q] : 0ull;
            }
#pragma unroll
            for (int u = 0; u < kTieU; ++u) {
                if (idx[u] < 0) continue;
                const int dgt = (int)((z[u] >> sh) & 255ull);
                if (dgt < v) {
                    atomicOr(&P.flag[idx[u]], bit);
                } else if (dgt == v) {
                    const int o2 = atomicAdd(&s_m2, 1);
                    CA[1 - src][o2] = idx[u];
                    CZ[1 - src][o2] = z[u];
                }
            }
        }
        __syncthreads();
        m = s_m2;
        r = s_r;
        src = 1 - src;
        pos += 1;
        __syncthreads();
    }
    if (m <= kTieLds && pos < 8 && r > 0 && r < m) {
        // Fast path: the tied entries' keys in LDS, one byte of the key per pass.
        int b = 0;
        for (int q = t; q < m; q += blockDim.x) {
            is[0][q] = CA[src][q];
            zs[0][q] = CZ[src][q];
        }
        __syncthreads();
        while (pos < 8 && r > 0 && r < m) {
            if (t == 0) s_pos = 8;
            __syncthreads();
            const unsigned long long z0 = zs[b][0], keep_mask = ~0ull >> (8 * pos);
            int first = 8;
            for (int q = t; q < m; q += blockDim.x) {
                const unsigned long long x = (zs[b][q] ^ z0) & keep_mask;
                const int d = x ? (__clzll((long long)x) >> 3) : 8;
                first = d < first ? d : first;
            }
            first = __ockl_wfred_min_i32(first);
            if ((t & 63) == 0) atomicMin(&s_pos, first);
            if (t < 256) h[t] = 0;
            if (t == 0) s_m2 = 0;
            __syncthreads();
            pos = s_pos;
            if (pos >= 8) break;   // equal keys: finish on the sequences below
            const int sh = 56 - 8 * pos;
            for (int q = t; q < m; q += blockDim.x) atomicAdd(&h[(zs[b][q] >> sh) & 255ull], 1u);
            __syncthreads();
            if (t < 64) {   // one wave scans the 256 counts (4 per lane)
                const uint32_t c0 = h[4 * t], c1 = h[4 * t + 1], c2 = h[4 * t + 2], c3 = h[4 * t + 3];
                uint32_t inc = c0 + c1 + c2 + c3;
                for (int o = 1; o < 64; o <<= 1) {
                    const uint32_t y = __shfl_up(inc, o, 64);
                    if (t >= o) inc += y;
                }
                long long cum = (long long)inc - (c0 + c1 + c2 + c3);
                const uint32_t cs[4] = {c0, c1, c2, c3};
                for (int k = 0; k < 4; ++k) {
                    if (cum < r && r <= cum + cs[k]) {
                        s_v = 4 * t + k;
                        s_r = r - cum;
                    }
                    cum += cs[k];
                }
            }
            __syncthreads();
            const int v = s_v;
            for (int q = t; q < m; q += blockDim.x) {
                const int dgt = (int)((zs[b][q] >> sh) & 255ull);
                if (dgt < v) atomicOr(&P.flag[is[b][q]], bit);
                else if (dgt == v) {
                    const int o2 = atomicAdd(&s_m2, 1);
                    zs[1 - b][o2] = zs[b][q];
                    is[1 - b][o2] = is[b][q];
                }
            }
            __syncthreads();
            m = s_m2;
            r = s_r;
            b = 1 - b;
            pos += 1;
            __syncthreads();
        }
        if (pos < 8 || r <= 0 || r >= m) {
            if (r > 0)
                for (int q = t; q < m; q += blockDim.x) atomicOr(&P.flag[is[b][q]], bit);
            return;
        }
        // the remaining m entries share their whole key: continue on the sequences
        __syncthreads();
        for (int q = t; q < m; q += blockDim.x) CA[1 - src][q] = is[b][q];
        __syncthreads();
        src = 1 - src;
        pos = 8;
    }
    while (pos < npos && r > 0 && r < m) {
        if (t == 0) s_pos = npos;
        __syncthreads();
        const int ref_i = CA[src][0];
        int first = npos;
        for (int q = t; q < m; q += blockDim.x) {
            const int d = first_diff(P, cur, CA[src][q], ref_i, pos, npos);
            first = d < first ? d : first;
        }
        first = __ockl_wfred_min_i32(first);
        if ((t & 63) == 0) atomicMin(&s_pos, first);
        __syncthreads();
        pos = s_pos;
        if (pos >= npos) break;   // all remaining candidates equal: cannot happen for a set
        for (int k = t; k < 256; k += blockDim.x) h[k] = 0;
        if (t == 0) s_m2 = 0;
        __syncthreads();
        for (int q = t; q < m; q += blockDim.x)
            atomicAdd(&h[tie_digit(P, cur, CA[src][q], pos)], 1u);
        __syncthreads();
        if (t == 0) {
            long long cum = 0;
            int v = 0;
            for (; v < 256; ++v) {
                if (cum + h[v] >= r) break;
                cum += h[v];
            }
            s_v = v;
            s_r = r - cum;
        }
        __syncthreads();
        const int v = s_v;
        for (int q = t; q < m; q += blockDim.x) {
            const int idx = CA[src][q];
            const int dgt = tie_digit(P, cur, idx, pos);
            if (dgt < v) atomicOr(&P.flag[idx], bit);
            else if (dgt == v) CA[1 - src][atomicAdd(&s_m2, 1)] = idx;
        }
        __syncthreads();
        m = s_m2;
        r = s_r;
        src = 1 - src;
        pos += 1;
        __syncthreads();
    }
    if (r > 0)
        for (int q = t; q < m; q += blockDim.x) atomicOr(&P.flag[CA[src][q]], bit);
}

// ---------------------------------------------------------------- pop / expand
// The direct expansion's repeat map starts each round clear.
__global__ __launch_bounds__(kSelThreads) void k_clear_repeats(Params P) {
    Ctl* c = P.ctl;
    if (c->stop) return;
    uint32_t* rw = (uint32_t*)P.repeat;
    const long long nw = ((long long)P.B * P.L + 3) / 4;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < nw;
         i += (long long)gridDim.x * blockDim.x)
        rw[i] = 0u;
}

// Direct O(L^2) expansion, one wavefront per pivot: the fallback for L > 641.
__global__ __launch_bounds__(64) void k_expand_direct(Params P) {
    Ctl* c = P.ctl;
    if (c->stop || (long long)blockIdx.x >= c->n_piv) return;
    const int cur = c->which;
    const long long bb = c->batch_begin;
    __shared__ int8_t sv[kSv];
    __shared__ int32_t Cl[kMaxL + 1];
    __shared__ uint32_t pk[32];
    const int lane = threadIdx.x;
    const int L = P.L, W = P.W;
    const int ps = P.piv[blockIdx.x];
    const int32_t Ep = P.H.rec[ps].E;
    if (lane < W) pk[lane] = P.H.seq[(size_t)ps * W + lane];
    for (int i = lane; i < kSv; i += 64) sv[i] = 0;
    __syncthreads();
    for (int x = 1 + lane; x <= L; x += 64) sv[kPad + x] = packed_bit(pk, x) ? 1 : -1;
    __syncthreads();
    for (int d = 1 + lane; d <= L - 1; d += 64) {
        int cd = 0;
        for (int i = 1; i <= L - d; ++i) cd += (int)sv[kPad + i] * (int)sv[kPad + i + d];
        Cl[d] = cd;
    }
    __syncthreads();
    unsigned long long hp = 0;
    for (int x = 1 + lane; x <= L; x += 64)
        if (sv[kPad + x] > 0) hp ^= zob(x - 1);
    for (int o = 32; o > 0; o >>= 1) hp ^= __shfl_xor(hp, o, 64);
    int taken = 0;
    int32_t mn = INT32_MAX, mx = 0;
    for (int r0 = 0; r0 < L; r0 += 64) {
        const int i = 1 + r0 + lane;
        const bool valid = i <= L;
        int32_t En = 0;
        unsigned long long key = 0;
        if (valid) {
            const int si = sv[kPad + i];
            int g = 0, q = 0;
            for (int d = 1; d <= L - 1; ++d) {
                const int t = sv[kPad + i + d] + sv[kPad + i - d];
                g += Cl[d] * t;
                q += t * t;
            }
            En = Ep - 4 * si * g + 4 * q;
            key = (hp ^ zob(i - 1)) | 1ull;
        }
        stage_neighbour(P, cur, bb, valid, valid && P.repeat[(long long)blockIdx.x * L + (i - 1)], key, ps,
                        i, En, taken, mn, mx);
    }
    stage_finish(P, taken, mn, mx);
}

// Bit-sliced expansion, 4 wavefronts per pivot.  For the single flip of s_i:
//   dE_i = sum_d dC_d (2 C_d + dC_d),  dC_d = -2 s_i t_d,  t_d = s_{i+d}[valid] + s_{i-d}[valid]
//        = -4 s_i G_i + 4 Q_i,   G_i = sum_d C_d t_d,   Q_i = sum_d t_d^2.
// With windows F_i = V >> i and B_i = VR >> (N-i+1) (bit d-1 = digit of s_{i+d} /
// s_{i-d}, 0 outside 1..L) and the two's-complement bit planes P_j of (C_d)_d:
//   G_i = 2 sum_j w_j (popc(P_j & F_i) + popc(P_j & B_i)) - PC[L-i] - PC[i-1],
//   Q_i = (L-1) + 2 (M - 2 popc((F_i ^ B_i) & [d <= M])),  M = min(L-i, i-1),
// PC being the prefix sums of C_d.  C_d itself is (L-d) - 2 popc((V ^ V>>d) & [j < L-d]).
// Window words that can hold lags in lane group r of the expansion (positions
// i in [1 + S r, S (r + 1)], S = 64 kExWaves): backward lags reach i - 1 < S (r + 1),
// forward lags L - i <= 32 NW2 - S r, and the groups before the last hold only
// valid positions (the last may clamp to i = L, which reaches no forward lag).
// Words past these are zero for every lane of the group and are skipped.
constexpr int kExSpanW = 2 * kExWaves;   // 32-bit words per lane group's span
template <int NW2>
__device__ constexpr int ex_fwords(int r) { return NW2 - kExSpanW * r > 0 ? NW2 - kExSpanW * r : 0; }
template <int NW2>
__device__ constexpr int ex_bwords(int r) { return kExSpanW * (r + 1) < NW2 ? kExSpanW * (r + 1) : NW2; }

template <int NW2, int R2>
__global__ __launch_bounds__(kExThreads) void k_expand(Params P) {
    // The pivot's slot, energy and key (as stored with its slot: lowest bit 1, as
    // the neighbours' keys), its words and the lower-numbered pivots' first words
    // come from the round's compact copies, in bounds for every workgroup of the
    // launch: they are loaded before the control block says whether this
    // workgroup has a pivot.
    const int ps = P.piv[blockIdx.x];
    const int32_t Ep = P.pivE[blockIdx.x];
    const unsigned long long hp = P.pivK[blockIdx.x];
    constexpr int NQ2 = (NW2 + 1) / 2;      // chunks of 64 lags
    constexpr int NVW = 2 * NW2 + 8;
    __shared__ uint32_t V[NVW], VR[NVW], pk[32];
    __shared__ int32_t Cl[32 * NW2 + 1], PC[32 * NW2 + 1];
    __shared__ uint8_t srep[32 * NW2 + 4];   // flip i repeats a lower-numbered pivot's neighbour
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int L = P.L, W = P.W;
    const uint32_t* pw = P.pseq + (size_t)blockIdx.x * W;
    static_assert(2 * NW2 + 8 <= kExThreads, "one word of V and VR per thread");
    const uint32_t wx = tid < W ? pw[tid] : 0u, wy = tid < W ? pw[W - 1 - tid] : 0u;
    constexpr int kRepU = 4;
    uint32_t f0[kRepU];
#pragma unroll
    for (int u = 0; u < kRepU; ++u) {
        const int q = tid + u * kExThreads;
        f0[u] = q < (int)blockIdx.x ? P.pseq[(size_t)q * W] : 0u;
    }
    Ctl* c = P.ctl;
    if (c->stop || (long long)blockIdx.x >= c->n_piv) return;
    const int cur = c->which;
    const long long bb = c->batch_begin;
    // V bit j = digit of s_{j+1} (LSB first): word w is the bit-reversed packed word;
    // VR (reversal over N = 32W bits): word W-1-w is the packed word itself.
    if (tid < NVW) {
        if (tid < W) pk[tid] = wx;
        V[tid] = __builtin_bitreverse32(wx);
        VR[tid] = wy;
    }
    for (int x = tid; x < 32 * NW2 + 4; x += kExThreads) srep[x] = 0;
    __syncthreads();
    // In-round repeats: the neighbour p_b (+) e_i equals a neighbour of pivot q
    // exactly when p_b and p_q are at Hamming distance 2 and i is one of the two
    // positions where they differ (p_b (+) e_i = p_q (+) e_i' with i' the other).
    // Of every repeated sequence the copy of the lowest-numbered pivot is kept, so
    // pivot b compares itself with every q < b.
    // The first words of four rows are loaded together (those of the first pass at
    // the start); a pair whose first words alone differ in more than 2 places is
    // not at distance 2.
    for (int q0 = tid; q0 < (int)blockIdx.x; q0 += kRepU * kExThreads) {
        if (q0 != tid) {
#pragma unroll
            for (int u = 0; u < kRepU; ++u) {
                const int q = q0 + u * kExThreads;
                f0[u] = q < (int)blockIdx.x ? P.pseq[(size_t)q * W] : 0u;
            }
        }
#pragma unroll
        for (int u = 0; u < kRepU; ++u) {
            if (q0 + u * kExThreads >= (int)blockIdx.x || __popc(f0[u] ^ pk[0]) > 2) continue;
            const uint32_t* row = P.pseq + (size_t)(q0 + u * kExThreads) * W;
            int d = 0;
            for (int w = 0; w < W; ++w) d += __popc(row[w] ^ pk[w]);
            if (d != 2) continue;
            for (int w = 0; w < W; ++w) {
                uint32_t x = row[w] ^ pk[w];
                while (x) {
                    const int k = __clz((int)x);
                    const int pos = 32 * w + k + 1;   // 1-based position, MSB first
                    if (pos <= L) srep[pos - 1] = 1;
                    x &= ~(0x80000000u >> k);
                }
            }
        }
    }
    for (int d = 1 + tid; d <= 32 * NW2; d += kExThreads) {
        int cd = 0;
        if (d <= L - 1) {
            const int q = d >> 5, r = d & 31, n = L - d;
            int dis = 0;
            for (int w = 0; w * 32 < n; ++w) {
                const uint32_t sh = __builtin_amdgcn_alignbit(V[w + q + 1], V[w + q], r);
                const int left = n - 32 * w;
                const uint32_t m = left >= 32 ? 0xffffffffu : ((1u << left) - 1u);
                dis += __popc((V[w] ^ sh) & m);
            }
            cd = n - 2 * dis;
        }
        Cl[d] = cd;
    }
    if (tid == 0) Cl[0] = 0;
    __syncthreads();
    if (wv == 0) {
        int carry = 0;
        for (int base = 0; base <= 32 * NW2; base += 64) {
            int v = (base + lane <= 32 * NW2 && base + lane >= 1) ? Cl[base + lane] : 0;
            for (int o = 1; o < 64; o <<= 1) {
                int u = __shfl_up(v, o, 64);
                if (lane >= o) v += u;
            }
            if (base + lane <= 32 * NW2) PC[base + lane] = carry + v;
            carry += __shfl(v, 63, 64);
        }
    }
    __syncthreads();
    // the neighbours' keys, and their home slots' tags loaded now: the loads land
    // while the energies are computed
    unsigned long long nkey[R2];
    int htag[R2];
#pragma unroll
    for (int r = 0; r < R2; ++r) {
        const int i0 = 1 + lane + 64 * (wv + kExWaves * r);
        nkey[r] = (hp ^ zob((i0 <= L ? i0 : L) - 1)) | 1ull;
        htag[r] = (i0 <= L && !srep[i0 - 1]) ? (int)P.H.tag[nkey[r] & P.H.mask] : 0;
    }
    int32_t Cq[NQ2];
    uint32_t orv = 0;
#pragma unroll
    for (int q = 0; q < NQ2; ++q) {
        const int d = 64 * q + lane + 1;
        Cq[q] = d <= 32 * NW2 ? Cl[d] : 0;
        orv |= (uint32_t)(Cq[q] ^ (Cq[q] >> 31));
    }
    orv = __ockl_wfred_or_u32(orv);
    const int nb = (32 - __clz((int)orv)) + 1;
    const int N = 32 * W;
    uint32_t F[R2][NW2], B[R2][NW2];
#pragma unroll
    for (int r = 0; r < R2; ++r) {
        int i = 1 + lane + 64 * (wv + kExWaves * r);
        if (i > L) i = L;
        const int qf = i >> 5, hf = i & 31;
        const int sb = N - i + 1, qb = sb >> 5, hb = sb & 31;
#pragma unroll
        for (int w = 0; w < NW2; ++w) {
            F[r][w] = w < ex_fwords<NW2>(r) ? __builtin_amdgcn_alignbit(V[qf + w + 1], V[qf + w], hf) : 0u;
            B[r][w] = w < ex_bwords<NW2>(r) ? __builtin_amdgcn_alignbit(VR[qb + w + 1], VR[qb + w], hb) : 0u;
        }
    }
    int32_t H[R2];
#pragma unroll
    for (int r = 0; r < R2; ++r) H[r] = 0;
    for (int jp = 0; jp < nb; ++jp) {
        uint32_t acc[R2];
#pragma unroll
        for (int r = 0; r < R2; ++r) acc[r] = 0;
#pragma unroll
        for (int q = 0; q < NQ2; ++q) {
            const uint64_t bal = __ballot((Cq[q] >> jp) & 1);
            const uint32_t lo = (uint32_t)bal, hi = (uint32_t)(bal >> 32);
#pragma unroll
            for (int r = 0; r < R2; ++r) {
                if (2 * q < ex_fwords<NW2>(r)) acc[r] = bcnt_add(lo & F[r][2 * q], acc[r]);
                if (2 * q < ex_bwords<NW2>(r)) acc[r] = bcnt_add(lo & B[r][2 * q], acc[r]);
                if (2 * q + 1 < ex_fwords<NW2>(r)) acc[r] = bcnt_add(hi & F[r][2 * q + 1], acc[r]);
                if (2 * q + 1 < ex_bwords<NW2>(r)) acc[r] = bcnt_add(hi & B[r][2 * q + 1], acc[r]);
            }
        }
        const int wgt = (jp == nb - 1) ? -(1 << jp) : (1 << jp);
#pragma unroll
        for (int r = 0; r < R2; ++r) H[r] += wgt * (int)acc[r];
    }
    int taken = 0;
    int32_t mn = INT32_MAX, mx = 0;
#pragma unroll
    for (int r = 0; r < R2; ++r) {
        const int i0 = 1 + lane + 64 * (wv + kExWaves * r);
        const bool valid = i0 <= L;
        const int i = valid ? i0 : L;
        const int Mf = L - i, Mb = i - 1, M = Mf < Mb ? Mf : Mb;
        int dis = 0;
#pragma unroll
        for (int w = 0; w < NW2; ++w) {
            if (w >= ex_fwords<NW2>(r) || w >= ex_bwords<NW2>(r)) continue;   // M is below
            const int left = M - 32 * w;
            const uint32_t m = left >= 32 ? 0xffffffffu : (left <= 0 ? 0u : ((1u << left) - 1u));
            dis += __popc((F[r][w] ^ B[r][w]) & m);
        }
        const int si = ((pk[(i - 1) >> 5] >> (31 - ((i - 1) & 31))) & 1u) ? 1 : -1;
        const int G = 2 * H[r] - PC[Mf] - PC[Mb];
        const int Q = (L - 1) + 2 * (M - 2 * dis);
        const int32_t En = Ep - 4 * si * G + 4 * Q;
        stage_neighbour(P, cur, bb, valid, srep[i - 1] != 0, nkey[r], ps, i, En, taken, mn, mx, htag[r], pk);
    }
    stage_finish(P, taken, mn, mx);
}

typedef void (*expand_kernel_t)(Params);

expand_kernel_t pick_expand(int L, unsigned* threads) {
    const int nw2 = (L - 1 + 31) / 32;
    const int r2 = (L + kExThreads - 1) / kExThreads;
    *threads = kExThreads;
#define EXP(NWV, RV) if (nw2 <= NWV && r2 <= RV) return k_expand<NWV, RV>;
    EXP(2, 1) EXP(4, 1) EXP(8, 1) EXP(12, 2) EXP(16, 2) EXP(17, 3) EXP(20, 3)
#undef EXP
    *threads = 64;
    return k_expand_direct;
}

// ---------------------------------------------------------------- rotations
constexpr int kRotThreads = 256;
constexpr int kMaxTr = 32;

// Energies and keys of the rotations of each pivot (MAKE_ROTATIONS).  C_k of the
// pivot is computed once; moving the first element x_1 of a sequence to its end
// changes C_k by x_1 (x_{L+1-k} - x_{1+k}), moving the last element x_L to its
// front by x_L (x_k - x_{L-k}), so each rotation costs O(L) after the previous
// one.  Keys are the Zobrist XOR of the rotated sequence.
__global__ __launch_bounds__(kRotThreads) void k_rot_build(Params P) {
    Ctl* c = P.ctl;
    if (c->stop) return;
    const long long b = blockIdx.x;
    if (b >= c->n_piv) return;
    __shared__ int8_t s[kMaxL];
    __shared__ int32_t C0[kMaxL], C[kMaxL];
    __shared__ uint32_t V[40];
    __shared__ int32_t red_e[kRotThreads / 64];
    __shared__ uint32_t red_lo[kRotThreads / 64], red_hi[kRotThreads / 64];
    const int L = P.L, W = P.W, t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const uint32_t* ps = P.H.seq + (size_t)P.piv[b] * W;
    for (int x = t; x < L; x += kRotThreads) s[x] = ((ps[x >> 5] >> (31 - (x & 31))) & 1u) ? 1 : -1;
    // V bit j = digit of element j (LSB first), zero past the sequence
    for (int w = t; w < 40; w += kRotThreads) V[w] = w < W ? __builtin_bitreverse32(ps[w]) : 0u;
    if (t == 0) P.pw0[b] = ps[0];
    __syncthreads();
    // C_k = (L - k) - 2 (number of positions where s_i != s_{i+k}), by popcounts
    for (int k = 1 + t; k < L; k += kRotThreads) {
        const int q = k >> 5, r = k & 31, n = L - k;
        int dis = 0;
        for (int w = 0; w * 32 < n; ++w) {
            const uint32_t sh = __builtin_amdgcn_alignbit(V[w + q + 1], V[w + q], r);
            const int left = n - 32 * w;
            const uint32_t m = left >= 32 ? 0xffffffffu : ((1u << left) - 1u);
            dis += __popc((V[w] ^ sh) & m);
        }
        C0[k] = n - 2 * dis;
    }
    __syncthreads();
    for (int dir = 0; dir < 2; ++dir) {
        for (int k = 1 + t; k < L; k += kRotThreads) C[k] = C0[k];
        __syncthreads();
        for (int r = 1; r <= P.Tr; ++r) {
            // x_i (1-based) of the pivot rotated by r-1 in this direction is
            // s[(i - 1 + off) mod L]
            const int off = dir == 0 ? r - 1 : L - (r - 1);
            for (int k = 1 + t; k < L; k += kRotThreads) {
                if (dir == 0)
                    C[k] += s[off % L] * (s[(L + off - k) % L] - s[(k + off) % L]);
                else
                    C[k] += s[(L - 1 + off) % L] * (s[(k - 1 + off) % L] - s[(L - k - 1 + off) % L]);
            }
            __syncthreads();
            const int off2 = dir == 0 ? r : L - r;   // the rotation by r
            int e = 0;
            for (int k = 1 + t; k < L; k += kRotThreads) e += C[k] * C[k];
            unsigned long long h = 0;
            for (int i = t; i < L; i += kRotThreads)
                if (s[(i + off2) % L] > 0) h ^= zob(i);
            e = __ockl_wfred_add_i32(e);
            uint32_t lo = (uint32_t)h, hi = (uint32_t)(h >> 32);
            for (int o = 32; o > 0; o >>= 1) {
                lo ^= (uint32_t)__shfl_xor((int)lo, o, 64);
                hi ^= (uint32_t)__shfl_xor((int)hi, o, 64);
            }
            if (lane == 0) {
                red_e[wv] = e;
                red_lo[wv] = lo;
                red_hi[wv] = hi;
            }
            __syncthreads();
            if (t == 0) {
                int E = 0;
                uint32_t l2 = 0, h2 = 0;
                for (int q = 0; q < kRotThreads / 64; ++q) {
                    E += red_e[q];
                    l2 ^= red_lo[q];
                    h2 ^= red_hi[q];
                }
                const long long idx = b * P.R2 + dir * P.Tr + (r - 1);
                P.rkey[idx] = (((unsigned long long)h2 << 32) | l2) | 1ull;
                P.rE[idx] = E;
            }
            __syncthreads();
        }
    }
}

// The rotations of pivot b take their fixed Open positions.  One is DEAD when it
// equals an earlier rotation of the round (in (pivot, q) order), when it lies
// within one flip of a pivot of the round (it is then that pivot, CLOSED, or one
// of the round's single-flip neighbours, which come first), or when H holds it
// as OPEN or CLOSED; otherwise it is a new entry.  H is only read.
__global__ __launch_bounds__(kRotThreads) void k_rot_stage(Params P) {
    Ctl* c = P.ctl;
    if (c->stop) return;
    const long long b = blockIdx.x;
    const long long np = c->n_piv;
    if (b >= np) return;
    __shared__ uint32_t rw[2 * kMaxTr][32];
    __shared__ unsigned long long rk[2 * kMaxTr];
    __shared__ int dupq[2 * kMaxTr];
    __shared__ int s_cnt, s_min, s_max;
    const int t = threadIdx.x, L = P.L, W = P.W, R2 = P.R2;
    const uint32_t last_mask = (L & 31) ? ~0u << (32 - (L & 31)) : ~0u;
    const uint32_t* ps = P.H.seq + (size_t)P.piv[b] * W;
    for (int x = t; x < R2 * W; x += kRotThreads) rw[x / W][x % W] = rot_word(ps, L, W, rot_shift(P, x / W), x % W);
    if (t < R2) {
        rk[t] = P.rkey[b * R2 + t];
        dupq[t] = 0;
    }
    if (t == 0) {
        s_cnt = 0;
        s_min = INT32_MAX;
        s_max = 0;
    }
    __syncthreads();
    // earlier rotations with an equal key: compare the sequences
    for (long long u = t; u < (b + 1) * R2; u += kRotThreads) {
        const unsigned long long ku = P.rkey[u];
        for (int q = 0; q < R2; ++q) {
            if (u >= b * R2 + q || ku != rk[q]) continue;
            const uint32_t* pu = P.H.seq + (size_t)P.piv[u / R2] * W;
            const int su = rot_shift(P, (int)(u % R2));
            bool eq = true;
            for (int w = 0; w < W && eq; ++w) eq = rot_word(pu, L, W, su, w) == rw[q][w];
            if (eq) dupq[q] = 1;
        }
    }
    // within one flip of a pivot of the round (first words compared first)
    for (long long v = t; v < np; v += kRotThreads) {
        const uint32_t w0 = P.pw0[v];
        for (int q = 0; q < R2; ++q) {
            uint32_t x0 = rw[q][0] ^ w0;
            if (W == 1) x0 &= last_mask;
            if (__popc(x0) > 1) continue;
            const uint32_t* pv = P.H.seq + (size_t)P.piv[v] * W;
            int d = __popc(x0);
            for (int w = 1; w < W && d <= 1; ++w) {
                uint32_t x = rw[q][w] ^ pv[w];
                if (w == W - 1) x &= last_mask;
                d += __popc(x);
            }
            if (d <= 1) dupq[q] = 1;
        }
    }
    __syncthreads();
    if (t < R2) {
        const int q = t;
        const long long idx = b * R2 + q;
        const unsigned long long key = rk[q];
        bool take = !dupq[q];
        int tomb = -1;
        if (take) {
            const Table& H = P.H;
            const uint8_t tg = tag_of(key);
            uint64_t sl = key & H.mask;
            for (uint64_t probe = 0; probe <= H.mask; ++probe, sl = (sl + 1) & H.mask) {
                const uint8_t ts = H.tag[sl];
                if (ts == 0) break;
                if (ts != tg) continue;
                const SlotRec rc = H.rec[sl];   // key and state in one load
                if (rc.key != key) continue;
                // the slot's words kWordChunk at a time against the rotation's in LDS
                bool eq = true;
                for (int w0 = 0; w0 < W && eq; w0 += kWordChunk) {
                    uint32_t a[kWordChunk];
#pragma unroll
                    for (int w = 0; w < kWordChunk; ++w) a[w] = w0 + w < W ? H.seq[sl * W + w0 + w] : 0u;
#pragma unroll
                    for (int w = 0; w < kWordChunk; ++w)
                        if (w0 + w < W) eq &= a[w] == rw[q][w0 + w];
                }
                if (!eq) continue;
                if (rc.state == ST_EVICTED) tomb = (int)sl;
                else take = false;
                break;
            }
        }
        const int cur = c->which;
        const long long j = np * L + idx;
        const long long o = c->batch_begin + j;
        if (!take) {
            P.oE[cur][o] = DEAD;
        } else {
            const int32_t En = P.rE[idx];
            P.oE[cur][o] = En;
            P.oS[cur][o] = -1;
            P.oZ[cur][o] = key;
            P.ntomb[j] = tomb;
            atomicAdd(&s_cnt, 1);
            atomicMin(&s_min, En);
            atomicMax(&s_max, En);
        }
    }
    __syncthreads();
    if (t == 0) {
        P.bcnt[b] += s_cnt;
        if (s_min < P.bmin[b]) P.bmin[b] = s_min;
        if (s_max > P.bmax[b]) P.bmax[b] = s_max;
    }
}

__device__ void best_scan(const Params& P, int initial);


// best = smallest (z, sequence) among live entries in [batch_begin, n_tot) with
// E == batch_minE.
__device__ __forceinline__ bool entry_less(const Params& P, int cur, long long a, long long b) {
    const unsigned long long za = P.oZ[cur][a], zb = P.oZ[cur][b];
    if (za != zb) return za < zb;
    const int sa = P.oS[cur][a], sb = P.oS[cur][b];
    for (int w = 0; w < P.W; ++w) {
        const uint32_t x = entry_word(P, sa, a, w), y = entry_word(P, sb, b, w);
        if (x != y) return x < y;
    }
    return false;
}

__device__ void best_scan(const Params& P, int initial) {
    Ctl* c = P.ctl;
    __shared__ long long best[1024];
    const int cur = c->which;
    const long long lo = c->batch_begin;
    const int32_t target = c->batch_minE;
    long long mine = -1;
    for (long long i = lo + threadIdx.x; i < c->n_tot; i += blockDim.x) {
        if (P.oE[cur][i] != target) continue;
        if (mine < 0 || entry_less(P, cur, i, mine)) mine = i;
    }
    best[threadIdx.x] = mine;
    __syncthreads();
    for (int o = (int)blockDim.x >> 1; o > 0; o >>= 1) {
        if (threadIdx.x < (unsigned)o) {
            const long long x = best[threadIdx.x], y = best[threadIdx.x + o];
            if (x < 0 || (y >= 0 && entry_less(P, cur, y, x))) best[threadIdx.x] = y;
        }
        __syncthreads();
    }
    const long long b = best[0];
    if (b >= 0 && threadIdx.x < (unsigned)P.W)
        P.best_seq[threadIdx.x] = entry_word(P, P.oS[cur][b], b, threadIdx.x);
    if (threadIdx.x == 0 && b >= 0) {
        c->best_slot = 1;   // a best sequence has been recorded
        c->best_E = target;
        if (!initial) {
            c->best_round = (int32_t)c->rounds;
            c->u = 0;
        }
    }
}

__global__ __launch_bounds__(1024) void k_best(Params P, int initial) {
    Ctl* c = P.ctl;
    if (c->stop) return;
    if (!initial && !c->improved) return;
    best_scan(P, initial);
}

// Keep the flagged live entries (all live entries when no cut is needed) in the
// other buffer; the rest become EVICTED (or, new entries, are never written to
// H).  Each thread handles kItems entries per pass, one atomic per block pass.

__global__ __launch_bounds__(kSelThreads) void k_keep(Params P) {
    __shared__ Ctl cs;
    snap_ctl(cs, P.ctl);
    const Ctl* c = &cs;
    Ctl* cg = P.ctl;
    if (c->stop) return;
    // the classify pass and the tie select have read the histograms: empty them for
    // the next selection
    for (long long b = (long long)blockIdx.x * blockDim.x + threadIdx.x; b < kHistWords;
         b += (long long)gridDim.x * blockDim.x)
        P.ghist[b] = 0u;
    const int cur = c->which;
    const uint32_t zv = c->zv, zv2 = c->zv2;
    const bool cut = !c->sel_all;           // entries are evicted
    const bool dual = c->dual;
    const bool dual_all = c->dual_all;
    const Table& H = P.H;
    const long long n_tot = c->n_tot, bb = c->batch_begin;
    long long claims = 0;
    const long long stride = (long long)gridDim.x * blockDim.x * kKeepItems;
    for (long long base = (long long)blockIdx.x * blockDim.x * kKeepItems; base < n_tot; base += stride) {
        int slot[kKeepItems];
        bool keep[kKeepItems];
        int32_t ev[kKeepItems];
        uint32_t fv[kKeepItems];
        unsigned long long zk[kKeepItems];
        int tb[kKeepItems];
        int cnt = 0;
        // every load of the pass first (a new entry's tombstone slot too)
#pragma unroll
        for (int k = 0; k < kKeepItems; ++k) {
            const long long i = base + threadIdx.x + (long long)k * blockDim.x;
            const bool in = i < n_tot;
            ev[k] = in ? P.oE[cur][i] : DEAD;
            fv[k] = in ? P.flag[i] : 0u;
            slot[k] = in ? P.oS[cur][i] : -1;
            zk[k] = in ? P.oZ[cur][i] : 0ull;
            tb[k] = in && i >= bb ? P.ntomb[i - bb] : -1;
        }
#pragma unroll
        for (int k = 0; k < kKeepItems; ++k) {
            const long long i = base + threadIdx.x + (long long)k * blockDim.x;
            const uint32_t f = fv[k];
            keep[k] = ev[k] != DEAD && (!cut || (f & 1u) || ((f & 4u) && (uint32_t)(zk[k] >> 56) < zv));
            if (ev[k] == DEAD) {
                slot[k] = -1;
            } else if (slot[k] >= 0) {
                if (!keep[k]) H.rec[slot[k]].state = ST_EVICTED;
            } else if (keep[k]) {
                const long long j = i - bb;
                const unsigned long long key = zk[k];
                const int tomb = tb[k];
                if (tomb >= 0) {
                    slot[k] = tomb;
                    H.rec[slot[k]].state = ST_OPEN;
                } else {
                    uint64_t s2 = key & H.mask;
                    for (uint64_t probe = 0; probe <= H.mask; ++probe, s2 = (s2 + 1) & H.mask)
                        if (atomicCAS(&H.rec[s2].key, 0ull, key) == 0ull) {
                            slot[k] = (int)s2;
                            H.tag[s2] = tag_of(key);
                            break;
                        }
                    if (slot[k] < 0) {
                        atomicExch(&cg->error, 2);
                        keep[k] = false;
                    } else {
                        uint32_t* dst = H.seq + (size_t)slot[k] * H.W;
                        if (j < c->n_piv * P.L) {
                            // a flip of a pivot: its row loaded kWordChunk words at a
                            // time, then stored
                            const int ji = (int)j, pi = ji / P.L, fl = ji - pi * P.L;
                            const uint32_t* src = P.pseq + (size_t)pi * H.W;
                            const int fw = fl >> 5;
                            const uint32_t fm = 1u << (31 - (fl & 31));
                            for (int w0 = 0; w0 < H.W; w0 += kWordChunk) {
                                uint32_t wv[kWordChunk];
#pragma unroll
                                for (int w = 0; w < kWordChunk; ++w) wv[w] = w0 + w < H.W ? src[w0 + w] : 0u;
#pragma unroll
                                for (int w = 0; w < kWordChunk; ++w)
                                    if (w0 + w < H.W) dst[w0 + w] = wv[w] ^ (w0 + w == fw ? fm : 0u);
                            }
                        } else {
                            // a rotation of a pivot: its words computed a few at a time,
                            // every load of a chunk issued before its stores
                            const long long jr = j - c->n_piv * P.L;
                            const int pi = (int)(jr / P.R2), q = (int)(jr - (long long)pi * P.R2);
                            const uint32_t* src = P.pseq + (size_t)pi * H.W;
                            const int sh = rot_shift(P, q);
                            constexpr int kc = kWordChunk / 2;   // up to four loads a word
                            for (int w0 = 0; w0 < H.W; w0 += kc) {
                                uint32_t wv[kc];
#pragma unroll
                                for (int w = 0; w < kc; ++w)
                                    wv[w] = w0 + w < H.W ? rot_word(src, P.L, H.W, sh, w0 + w) : 0u;
#pragma unroll
                                for (int w = 0; w < kc; ++w)
                                    if (w0 + w < H.W) dst[w0 + w] = wv[w];
                            }
                        }
                        H.rec[slot[k]].E = ev[k];
                        H.rec[slot[k]].state = ST_OPEN;
                        ++claims;
                    }
                }
            }
            cnt += keep[k] ? 1 : 0;
        }
        // the next round's pivots: every survivor (dual_all) or those of flag bit 1.
        // At most B per round, so they take their list places per wavefront (one
        // atomic for each wavefront that holds some), not per workgroup.
        bool pv[kKeepItems];
        long long opk[kKeepItems];
        const int lane = threadIdx.x & 63;
        const uint64_t lt = lane ? (~0ull >> (64 - lane)) : 0ull;
#pragma unroll
        for (int k = 0; k < kKeepItems; ++k) {
            if (dual && keep[k] && !dual_all) {
                const uint32_t f = fv[k];
                pv[k] = (f & 2u) || ((f & 8u) && (uint32_t)(zk[k] >> 56) < zv2);
            } else {
                pv[k] = dual && keep[k];
            }
            const uint64_t pm = __ballot(pv[k]);
            unsigned long long pb = 0;
            if (pm && lane == __ffsll((unsigned long long)pm) - 1)
                pb = atomicAdd((unsigned long long*)&cg->n_pivpos, (unsigned long long)__popcll(pm));
            pb = __shfl(pb, __ffsll((unsigned long long)pm) - 1, 64);
            opk[k] = (long long)pb + __popcll(pm & lt);
        }
        long long o = block_append_n(&cg->survivors, cnt);
#pragma unroll
        for (int k = 0; k < kKeepItems; ++k) {
            if (!keep[k]) continue;
            const long long op = opk[k];
            P.oE[1 - cur][o] = ev[k];
            P.oS[1 - cur][o] = slot[k];
            P.oZ[1 - cur][o] = zk[k];
            if (pv[k]) {
                // a pivot of the next round: out of Open (CLOSED, DEAD in the list),
                // its slot and words copied for the expansion
                if (op < P.B) {
                    const int sl = slot[k];
                    P.pivn[op] = sl;
                    P.pivEn[op] = ev[k];
                    P.pivKn[op] = zk[k];
                    P.pivpos[op] = (int32_t)o;
                    if (P.take_pivots) {
                        P.oE[1 - cur][o] = DEAD;
                        H.rec[sl].state = ST_CLOSED;
                    }
                    // the words loaded together (W <= 32), then stored
                    for (int w0 = 0; w0 < H.W; w0 += 16) {
                        uint32_t wv[16];
#pragma unroll
                        for (int w = 0; w < 16; ++w)
                            wv[w] = w0 + w < H.W ? H.seq[(size_t)sl * H.W + w0 + w] : 0u;
#pragma unroll
                        for (int w = 0; w < 16; ++w)
                            if (w0 + w < H.W) P.pseqn[(size_t)op * H.W + w0 + w] = wv[w];
                    }
                }
            }
            ++o;
        }
    }
    // the workgroup's claims: a wave sum, then the waves' sums
    __shared__ int s_claims[kSelThreads / 64];
    const int wcl = __ockl_wfred_add_i32((int)claims);
    if ((threadIdx.x & 63) == 0) s_claims[threadIdx.x >> 6] = wcl;
    __syncthreads();
    if (threadIdx.x == 0) {
        int tot = 0;
        for (int k = 0; k < (int)(blockDim.x >> 6); ++k) tot += s_claims[k];
        P.kclaims[(size_t)(c->rounds % kCheck) * kKeepBlocks + blockIdx.x] = tot;
    }
}

__device__ void round_end(const Params& P, int count_round, Ctl* c) {
    if (c->stop) return;
    if (!c->sel_all) {   // the cut evicted entries
        // (the seeding cut admits the Q smallest candidates: no evictions)
        if (count_round) c->evictions += c->n_live - c->survivors;
        c->blo = c->emin;
        c->bhi = c->emin + (c->Dt << 2);   // survivors lie at or below the cut's energy
    } else {
        c->blo = c->emin < c->blo ? c->emin : c->blo;
        c->bhi = c->emax > c->bhi ? c->emax : c->bhi;
    }
    c->n_live = c->survivors;
    c->n_tot = c->survivors;
    c->which ^= 1;
    c->sel_enabled = 0;
    if (count_round) c->rounds += 1;
}

__global__ void k_round_end(Params P, int count_round) { round_end(P, count_round, P.ctl); }

// The end of a round and the start of the next in one launch (one wavefront): the
// control block is copied to LDS in one go, updated there by one thread and
// written back whole (no other kernel runs beside this one).
__global__ __launch_bounds__(64) void k_round_next(Params P) {
    __shared__ Ctl cs;
    snap_ctl(cs, P.ctl);
    if (threadIdx.x == 0) {
        round_end(P, 1, &cs);
        round_begin(P, P.pivn, &cs);
    }
    __syncthreads();
    constexpr int n = (int)(sizeof(Ctl) / 8);
    if (threadIdx.x < (unsigned)n)
        reinterpret_cast<unsigned long long*>(P.ctl)[threadIdx.x] =
            reinterpret_cast<const unsigned long long*>(&cs)[threadIdx.x];
}

__global__ void k_outputs(Params P, uint32_t* best_seq, int32_t* best_E, labs_step2_stats* st,
                          uint32_t* open_seqs, int32_t* open_E, long long open_cap, long long rebuilds) {
    Ctl* c = P.ctl;
    const int W = P.W;
    if (blockIdx.x == 0 && threadIdx.x < (unsigned)W && c->best_slot >= 0)
        best_seq[threadIdx.x] = P.best_seq[threadIdx.x];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        *best_E = c->best_E;
        st->expansions = c->expansions;
        st->pushes = c->pushes;
        st->dup_skips = c->dups;
        st->evictions = c->evictions;
        st->rounds = c->rounds;
        st->open_count = c->n_live;
        st->best_E = c->best_E;
        st->best_round = c->best_round;
        st->rebuilds = rebuilds;
    }
    if (!open_seqs && !open_E) return;
    const int cur = c->which;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < c->n_tot;
         i += (long long)gridDim.x * blockDim.x) {
        if (P.oE[cur][i] == DEAD || i >= open_cap) continue;
        const int s = P.oS[cur][i];
        if (open_E) open_E[i] = P.oE[cur][i];
        if (open_seqs)
            for (int w = 0; w < W; ++w) open_seqs[i * W + w] = P.H.seq[(size_t)s * W + w];
    }
}

// ---------------------------------------------------------------- table rebuild
// Re-insert the OPEN and CLOSED slots of `src` into the empty table `dst`
// (tombstones of evicted sequences are dropped) and record old -> new slots.
__global__ void k_rebuild(Table src, Table dst, uint32_t* remap, Ctl* c) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i <= src.mask;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t st = src.rec[i].state;
        if (src.rec[i].key == 0ull || (st != ST_OPEN && st != ST_CLOSED)) continue;
        const unsigned long long key = src.rec[i].key;
        uint64_t s = key & dst.mask;
        for (uint64_t probe = 0; probe <= dst.mask; ++probe) {
            if (atomicCAS(&dst.rec[s].key, 0ull, key) == 0ull) break;
            s = (s + 1) & dst.mask;
        }
        dst.tag[s] = tag_of(key);
        for (int w = 0; w < src.W; ++w) dst.seq[s * dst.W + w] = src.seq[i * src.W + w];
        dst.rec[s].E = src.rec[i].E;
        dst.rec[s].state = st;
        remap[i] = (uint32_t)s;
        atomicAdd((unsigned long long*)&c->claimed_new, 1ull);
    }
}

__global__ void k_remap(Params P, const uint32_t* remap) {
    Ctl* c = P.ctl;
    const int cur = c->which;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < c->n_tot;
         i += (long long)gridDim.x * blockDim.x)
        if (P.oE[cur][i] != DEAD) P.oS[cur][i] = (int32_t)remap[P.oS[cur][i]];
    // the coming round's pivots (CLOSED, DEAD in the list)
    for (long long b = (long long)blockIdx.x * blockDim.x + threadIdx.x; b < c->n_piv;
         b += (long long)gridDim.x * blockDim.x)
        P.piv[b] = (int32_t)remap[P.piv[b]];
}

__global__ void k_rebuild_fin(Ctl* c, const uint32_t* remap) {
    c->claimed = c->claimed_new;
    c->claimed_new = 0;
}

__global__ void k_init_ctl(Ctl* c) {
    if (threadIdx.x || blockIdx.x) return;
    Ctl z = {};
    z.best_E = INT32_MAX;
    z.best_slot = -1;
    z.best_round = -1;
    *c = z;
}

// After seeding: count the live entries and set up the capacity cut.
__global__ void k_seed_fin(Params P) {
    Ctl* c = P.ctl;
    c->n_live = c->n_tot;
    c->claimed = c->n_tot;
    cut_setup(P);
    c->emin = UINT32_MAX;
    c->emax = 0;
}

// Before the initial best: the whole (cut) Open list is the "batch".
// After the seeding: round 0's pivots (listed by the seeding cut) leave Open.
__global__ void k_take_pivots(Params P) {
    Ctl* c = P.ctl;
    const int cur = c->which;
    const long long n = c->n_pivpos < P.B ? c->n_pivpos : P.B;
    for (long long b = (long long)blockIdx.x * blockDim.x + threadIdx.x; b < n;
         b += (long long)gridDim.x * blockDim.x) {
        P.oE[cur][P.pivpos[b]] = DEAD;
        P.H.rec[P.piv[b]].state = ST_CLOSED;
    }
}

__global__ void k_seed_best_setup(Ctl* c) {
    c->batch_begin = 0;
    c->batch_minE = INT32_MAX;
    c->blo = UINT32_MAX;
    c->bhi = 0;
}

// Exact energy bounds of the live entries after seeding.
__global__ __launch_bounds__(kSelThreads) void k_live_bounds(Params P) {
    Ctl* c = P.ctl;
    const int cur = c->which;
    uint32_t mn = UINT32_MAX, mx = 0;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < c->n_tot;
         i += (long long)gridDim.x * blockDim.x) {
        const int32_t e = P.oE[cur][i];
        if (e == DEAD) continue;
        mn = (uint32_t)e < mn ? (uint32_t)e : mn;
        mx = (uint32_t)e > mx ? (uint32_t)e : mx;
    }
    mn = (uint32_t)__ockl_wfred_min_i32((int)(mn > (uint32_t)INT32_MAX ? (uint32_t)INT32_MAX : mn));
    mx = __ockl_wfred_max_u32(mx);
    if ((threadIdx.x & 63) == 0) {
        atomicMin(&c->blo, mn);
        atomicMax(&c->bhi, mx);
    }
}

// Minimum E over live entries into batch_minE (the initial best's energy).
__global__ __launch_bounds__(kSelThreads) void k_min_live(Params P) {
    Ctl* c = P.ctl;
    const int cur = c->which;
    int mn = INT32_MAX;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < c->n_tot;
         i += (long long)gridDim.x * blockDim.x)
        mn = min(mn, (int)P.oE[cur][i]);
    mn = __ockl_wfred_min_i32(mn);
    if ((threadIdx.x & 63) == 0 && mn != INT32_MAX) atomicMin(&c->batch_minE, mn);
}

uint64_t next_pow2(uint64_t x) {
    uint64_t p = 1;
    while (p < x) p <<= 1;
    return p;
}


struct S2Layout {
    uint64_t cap_ht;
    long long cap_o, cap_pend, cap_new;
    size_t total;
};

S2Layout s2_layout(const labs_step2_cfg& c, long long n_cand) {
    S2Layout lo;
    const int W = words_of(c.L);
    const long long base = (n_cand > c.pq_capacity ? n_cand : c.pq_capacity);
    const long long BL = (long long)c.batch * (c.L + 2 * c.T_r);   // products of one round
    lo.cap_o = base + BL + 1024;
    lo.cap_pend = (BL > n_cand ? BL : n_cand) + 1024;
    // live slots never exceed n_cand + X + Q + BL; the table is rebuilt when half
    // of it is claimed (claims: seeds, and new entries surviving their round's
    // cut), with kCheck rounds of claims as headroom.
    const long long live = n_cand + c.max_expansions + c.pq_capacity + BL;
    lo.cap_ht = next_pow2((uint64_t)(4 * (live + (long long)kCheck * BL) + 1024));
    lo.cap_new = BL + 1024;
    size_t t = 0;
    for (int tb = 0; tb < 2; ++tb) {
        t += align_up(sizeof(SlotRec) * lo.cap_ht, 256);                 // key, E, state
        t += align_up(lo.cap_ht, 256);                                   // tag
        t += align_up(sizeof(uint32_t) * lo.cap_ht * W, 256);
    }
    t += align_up(sizeof(uint32_t) * lo.cap_ht, 256);                  // remap
    t += align_up(sizeof(int32_t) * lo.cap_new, 256);                  // ntomb
    t += 3 * align_up(sizeof(int32_t) * c.batch, 256);                 // bcnt, bmin, bmax
    t += align_up(lo.cap_new + 4, 256);                                // repeat
    t += 2 * align_up(sizeof(uint32_t) * c.batch * words_of(c.L), 256);  // pseq, this round's and the next's
    t += align_up(sizeof(unsigned long long) * (2 * c.T_r * c.batch + 1), 256);   // rotation keys
    t += align_up(sizeof(int32_t) * (2 * c.T_r * c.batch + 1), 256);              // rotation energies
    t += align_up(sizeof(uint32_t) * c.batch, 256);                                // pivots' first words
    t += align_up(sizeof(Ctl), 256);
    t += 2 * align_up(sizeof(int32_t) * lo.cap_o, 256);                // oE
    t += 2 * align_up(sizeof(int32_t) * lo.cap_o, 256);                // oS
    t += 2 * align_up(sizeof(unsigned long long) * lo.cap_o, 256);     // oZ
    t += align_up(sizeof(uint32_t) * lo.cap_o, 256);                   // flag
    t += 2 * align_up(sizeof(int32_t) * lo.cap_o, 256);                // cand
    t += 2 * align_up(sizeof(unsigned long long) * lo.cap_o, 256);     // candz
    t += 2 * align_up(sizeof(int32_t) * lo.cap_o, 256);                // cand2
    t += 2 * align_up(sizeof(unsigned long long) * lo.cap_o, 256);     // candz2
    t += 2 * align_up(sizeof(int32_t) * c.batch, 256);                 // piv, this round's and the next's
    t += 2 * align_up(sizeof(int32_t) * c.batch, 256);                 // their energies
    t += 2 * align_up(sizeof(unsigned long long) * c.batch, 256);      // their keys
    t += align_up(sizeof(int32_t) * c.batch, 256);                     // pivpos
    t += align_up(sizeof(int32_t) * kClassifyBlocks, 256);             // best candidates
    t += align_up(sizeof(uint32_t) * kHistWords, 256);                 // select histograms
    t += align_up(sizeof(uint32_t) * 32, 256);                         // best sequence
    t += align_up(sizeof(int32_t) * kCheck * kKeepBlocks, 256);        // claims per cut workgroup
    t += 2 * align_up(sizeof(Pend) * lo.cap_pend, 256);                // pending, collisions
    lo.total = t + 4096;
    return lo;
}

}  // namespace

size_t step2_workspace_bytes(const labs_step2_cfg& c, long long n_cand) {
    return s2_layout(c, n_cand).total;
}

bool step2_fits(const labs_step2_cfg& c, long long n_cand) {
    return s2_layout(c, n_cand).cap_ht <= (1ull << 31);
}

// The host loop.  `tb`/`te` bracket every expansion launch (launch timing).
labs_status step2_run(const labs_step2_cfg& cfg, long long n_cand, const uint32_t* cand_seqs,
                      const labs_step2_out& out, void* ws, size_t ws_bytes, hipStream_t st,
                      labs_status (*tb)(void*, hipStream_t), labs_status (*te)(void*, hipStream_t),
                      void* tctx) {
    const S2Layout lo = s2_layout(cfg, n_cand);
    if (ws_bytes < lo.total) {
        set_error("workspace needs %zu bytes, got %zu", lo.total, ws_bytes);
        return LABS_E_NOMEM;
    }
    Carve cv(ws, ws_bytes);
    Params P{};
    P.L = cfg.L;
    P.W = words_of(cfg.L);
    P.B = cfg.batch;
    P.Q = cfg.pq_capacity;
    P.X = cfg.max_expansions;
    P.T_u = cfg.T_u;
    P.cap_o = lo.cap_o;
    P.cap_pend = lo.cap_pend;
    Table tabs[2];
    for (int tb2 = 0; tb2 < 2; ++tb2) {
        tabs[tb2].rec = cv.take<SlotRec>(lo.cap_ht);
        tabs[tb2].tag = cv.take<uint8_t>(lo.cap_ht);
        tabs[tb2].seq = cv.take<uint32_t>(lo.cap_ht * P.W);
        tabs[tb2].mask = lo.cap_ht - 1;
        tabs[tb2].W = P.W;
    }
    uint32_t* remap = cv.take<uint32_t>(lo.cap_ht);
    P.ntomb = cv.take<int32_t>(lo.cap_new);
    P.bcnt = cv.take<int32_t>(cfg.batch);
    P.bmin = cv.take<int32_t>(cfg.batch);
    P.bmax = cv.take<int32_t>(cfg.batch);
    P.repeat = cv.take<uint8_t>(lo.cap_new + 4);
    uint32_t* pseqb[2];
    for (int b = 0; b < 2; ++b) pseqb[b] = cv.take<uint32_t>((size_t)cfg.batch * P.W);
    P.Tr = cfg.T_r;
    P.R2 = 2 * cfg.T_r;
    P.rkey = cv.take<unsigned long long>((size_t)P.R2 * cfg.batch + 1);
    P.rE = cv.take<int32_t>((size_t)P.R2 * cfg.batch + 1);
    P.pw0 = cv.take<uint32_t>((size_t)cfg.batch);
    int tcur = 0;
    P.H = tabs[0];
    P.ctl = cv.take<Ctl>(1);
    for (int b = 0; b < 2; ++b) P.oE[b] = cv.take<int32_t>(lo.cap_o);
    for (int b = 0; b < 2; ++b) P.oS[b] = cv.take<int32_t>(lo.cap_o);
    for (int b = 0; b < 2; ++b) P.oZ[b] = cv.take<unsigned long long>(lo.cap_o);
    P.flag = cv.take<uint32_t>(lo.cap_o);
    for (int b = 0; b < 2; ++b) P.cand[b] = cv.take<int32_t>(lo.cap_o);
    for (int b = 0; b < 2; ++b) P.candz[b] = cv.take<unsigned long long>(lo.cap_o);
    for (int b = 0; b < 2; ++b) P.cand2[b] = cv.take<int32_t>(lo.cap_o);
    for (int b = 0; b < 2; ++b) P.candz2[b] = cv.take<unsigned long long>(lo.cap_o);
    P.pivpos = cv.take<int32_t>(cfg.batch);
    P.bestc = cv.take<int32_t>(kClassifyBlocks);
    int32_t* pivb[2];
    for (int b = 0; b < 2; ++b) pivb[b] = cv.take<int32_t>(cfg.batch);
    int32_t* pivEb[2];
    for (int b = 0; b < 2; ++b) pivEb[b] = cv.take<int32_t>(cfg.batch);
    unsigned long long* pivKb[2];
    for (int b = 0; b < 2; ++b) pivKb[b] = cv.take<unsigned long long>(cfg.batch);
    // round r expands the pivots of buffer r & 1; its cut writes those of round r + 1
    auto set_round = [&](long long r) {
        P.piv = pivb[r & 1];
        P.pivE = pivEb[r & 1];
        P.pivK = pivKb[r & 1];
        P.pseq = pseqb[r & 1];
        P.pivn = pivb[(r + 1) & 1];
        P.pivEn = pivEb[(r + 1) & 1];
        P.pivKn = pivKb[(r + 1) & 1];
        P.pseqn = pseqb[(r + 1) & 1];
    };
    set_round(-1);   // the seeding cut writes round 0's pivots
    P.take_pivots = 0;
    P.ghist = cv.take<uint32_t>((size_t)kHistWords);
    P.best_seq = cv.take<uint32_t>(32);
    P.kclaims = cv.take<int32_t>((size_t)kCheck * kKeepBlocks);
    P.pend = cv.take<Pend>(lo.cap_pend);
    P.slow = cv.take<Pend>(lo.cap_pend);
    P.cands = cand_seqs;
    if (!cv.ok()) return invalid("workspace layout overflow");

    LABS_HIP(hipMemsetAsync(P.H.rec, 0, sizeof(SlotRec) * lo.cap_ht, st));
    LABS_HIP(hipMemsetAsync(P.H.tag, 0, lo.cap_ht, st));
    LABS_HIP(hipMemsetAsync(P.best_seq, 0, sizeof(uint32_t) * 32, st));
    LABS_HIP(hipMemsetAsync(P.kclaims, 0, sizeof(int32_t) * kCheck * kKeepBlocks, st));
    LABS_HIP(hipMemsetAsync(P.ghist, 0, sizeof(uint32_t) * kHistWords, st));
    const dim3 gS(kGridBlocks), tS(kSelThreads);
    // Selection; rounds take their energy bounds from the control block instead
    // of a min/max pass.
    // dual: the round's cut, which may also select the next round's pivots
    // round: the round's counts come with the histogram pass, and the classify
    // launch's extra workgroup finds an improving round's best
    auto select = [&](bool minmax, bool round) {
        P.best_in_classify = round ? 1 : 0;
        if (round) {
            hipLaunchKernelGGL(k_mid_hist, dim3(kSelBlocks), tS, 0, st, P);
        } else {
            if (minmax) hipLaunchKernelGGL(k_sel_minmax, dim3(kSelBlocks), tS, 0, st, P);
            hipLaunchKernelGGL(k_sel_hist, dim3(kSelBlocks), tS, 0, st, P);
        }
        hipLaunchKernelGGL(k_sel_classify, dim3(kClassifyBlocks), tS, 0, st, P);
        hipLaunchKernelGGL(k_sel_keys, dim3(round ? 3 : 2), dim3(1024), 0, st, P);
    };

    // seeding: insert the candidates (exact dedupe), cut to Q, best = minimum
    hipLaunchKernelGGL(k_init_ctl, dim3(1), dim3(1), 0, st, P.ctl);
    hipLaunchKernelGGL(k_seed, dim3((unsigned)n_cand), dim3(64), 0, st, P, n_cand);
    hipLaunchKernelGGL(k_resolve, gS, tS, 0, st, P);
    hipLaunchKernelGGL(k_slow, dim3(1), dim3(1), 0, st, P);
    hipLaunchKernelGGL(k_seed_fin, dim3(1), dim3(1), 0, st, P);
    select(true, false);
    hipLaunchKernelGGL(k_keep, dim3(kKeepBlocks), tS, 0, st, P);
    hipLaunchKernelGGL(k_round_end, dim3(1), dim3(1), 0, st, P, 0);
    hipLaunchKernelGGL(k_seed_best_setup, dim3(1), dim3(1), 0, st, P.ctl);
    hipLaunchKernelGGL(k_min_live, gS, tS, 0, st, P);
    hipLaunchKernelGGL(k_live_bounds, gS, tS, 0, st, P);
    hipLaunchKernelGGL(k_best, dim3(1), dim3(1024), 0, st, P, 1);
    set_round(0);
    hipLaunchKernelGGL(k_take_pivots, dim3(4), dim3(256), 0, st, P);
    P.take_pivots = 1;
    LABS_LAUNCHED("step2 seeding");

    labs_status s;
    unsigned eth = 64;
    const expand_kernel_t ek = pick_expand(cfg.L, &eth);
    P.direct = ek == k_expand_direct ? 1 : 0;
    // A round: in-round repeats (the bit-sliced expansion finds its own),
    // expansion, counts / statistics / best, cut selection, the cut (which takes
    // the next round's pivots out of Open), then the end of the round together
    // with the start of the next.
    hipLaunchKernelGGL(k_round_begin, dim3(1), dim3(1), 0, st, P);
    // the control block's flags and the cut's claims as copied after every kCheck
    // rounds (pinned, two batches in turn); claimed = the block's count (set by the
    // seeding and by a rebuild) + the claims summed since
    struct ChkFlags {
        int32_t stop, error;
        long long claimed;
        int32_t claims[kCheck * kKeepBlocks];
    };
    struct ChkRes {
        hipStream_t st = nullptr;
        ChkFlags* h = nullptr;
        hipEvent_t ev[2] = {nullptr, nullptr};
        ~ChkRes() {
            // copies into h may still be queued when the search ends early
            if (h && hipStreamSynchronize(st) == hipSuccess) (void)hipHostFree(h);
            for (hipEvent_t e : ev)
                if (e) (void)hipEventDestroy(e);
        }
    } chk_res;
    chk_res.st = st;
    LABS_HIP(hipHostMalloc((void**)&chk_res.h, 2 * sizeof(ChkFlags), hipHostMallocDefault));
    for (int b = 0; b < 2; ++b) LABS_HIP(hipEventCreateWithFlags(&chk_res.ev[b], hipEventDisableTiming));
    ChkFlags* hflags = chk_res.h;
    hipEvent_t* chk = chk_res.ev;
    const long long BLr = (long long)cfg.batch * (cfg.L + 2 * cfg.T_r);   // claims of one round at most
    long long claimed_seen = n_cand;
    long long claims_acc = 0;
    long long n_rebuilds = 0;
    int inflight = -1;
    for (long long r = 0;; ++r) {
        set_round(r);
        if (P.direct) {
            hipLaunchKernelGGL(k_clear_repeats, gS, tS, 0, st, P);
            const unsigned nt = (unsigned)((cfg.batch + kRepTile - 1) / kRepTile);
            hipLaunchKernelGGL(k_repeats, dim3(nt, nt), dim3(256), 0, st, P);
        }
        if (tb && (s = tb(tctx, st)) != LABS_OK) return s;
        hipLaunchKernelGGL(ek, dim3((unsigned)cfg.batch), dim3(eth), 0, st, P);
        if (te && (s = te(tctx, st)) != LABS_OK) return s;
        if (P.Tr) {
            hipLaunchKernelGGL(k_rot_build, dim3((unsigned)cfg.batch), dim3(kRotThreads), 0, st, P);
            hipLaunchKernelGGL(k_rot_stage, dim3((unsigned)cfg.batch), dim3(kRotThreads), 0, st, P);
        }
        select(false, true);
        hipLaunchKernelGGL(k_keep, dim3(kKeepBlocks), tS, 0, st, P);
        hipLaunchKernelGGL(k_round_next, dim3(1), dim3(64), 0, st, P);
        LABS_LAUNCHED("step2 round");
        if ((r + 1) % kCheck == 0) {
            // This batch's flags are copied; the host reads the previous batch's,
            // so the stream always holds a batch of rounds ahead of the host.
            // Rounds enqueued after the stop return at once.  A rebuild decided on
            // flags a batch old would come later than one decided now, so when
            // the claims could reach half the table within the unread batches the
            // host reads this batch's flags at once instead.
            const int slot = (int)(((r + 1) / kCheck) & 1);
            LABS_HIP(hipMemcpyAsync(&hflags[slot].stop, &P.ctl->stop, 2 * sizeof(int32_t),
                                    hipMemcpyDeviceToHost, st));
            LABS_HIP(hipMemcpyAsync(&hflags[slot].claimed, &P.ctl->claimed, sizeof(long long),
                                    hipMemcpyDeviceToHost, st));
            LABS_HIP(hipMemcpyAsync(hflags[slot].claims, P.kclaims, sizeof(int32_t) * kCheck * kKeepBlocks,
                                    hipMemcpyDeviceToHost, st));
            LABS_HIP(hipEventRecord(chk[slot], st));
            const bool now = (uint64_t)(claimed_seen + 3LL * kCheck * BLr) * 2 >= lo.cap_ht;
            int look;
            if (now) {
                look = slot;
                inflight = -1;
            } else if (inflight >= 0) {
                look = inflight;
                inflight = slot;
            } else {
                inflight = slot;
                continue;
            }
            LABS_HIP(hipEventSynchronize(chk[look]));
            const ChkFlags& f = hflags[look];
            if (f.error) {
                set_error("second-step hash set failure (code %d)", f.error);
                return LABS_E_DEVICE;
            }
            if (f.stop) break;
            for (int k = 0; k < kCheck * kKeepBlocks; ++k) claims_acc += f.claims[k];
            const long long claimed = f.claimed + claims_acc;
            claimed_seen = claimed;
            if ((uint64_t)claimed * 2 >= lo.cap_ht) {
                inflight = -1;   // its claims were counted before the rebuild
                claims_acc = 0;  // the rebuild recounts the claimed slots
                Table& dst = tabs[1 - tcur];
                LABS_HIP(hipMemsetAsync(dst.rec, 0, sizeof(SlotRec) * lo.cap_ht, st));
                LABS_HIP(hipMemsetAsync(dst.tag, 0, lo.cap_ht, st));
                hipLaunchKernelGGL(k_rebuild, dim3(8192), dim3(256), 0, st, tabs[tcur], dst, remap, P.ctl);
                set_round(r + 1);   // the coming round's pivot slots are remapped too
                hipLaunchKernelGGL(k_remap, gS, tS, 0, st, P, remap);
                hipLaunchKernelGGL(k_rebuild_fin, dim3(1), dim3(1), 0, st, P.ctl, remap);
                LABS_LAUNCHED("step2 rebuild");
                tcur = 1 - tcur;
                P.H = tabs[tcur];
                ++n_rebuilds;
            }
        }
    }
    hipLaunchKernelGGL(k_outputs, gS, tS, 0, st, P, out.best_seq, out.best_E, out.stats, out.open_seqs,
                       out.open_E, (long long)out.open_capacity, n_rebuilds);
    LABS_LAUNCHED("step2 outputs");
    LABS_HIP(hipStreamSynchronize(st));
    return LABS_OK;
}

}  // namespace labsdev
