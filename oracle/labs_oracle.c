/*
 * labs_oracle.c -- plain, slow CPU reference for the LABS dual-step hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, includes or
 * calls this file; only the test-suite, the smoke check and the CPU-baseline leg
 * of the benchmark load it (through oracle/__init__.py).  It shares no code,
 * header, table or constant generator with the HIP path.
 *
 * Every function is written from the definitions in the paper
 * (Psenicnik, Mlinaric, Brest, Boskovic, "Dual-Step Optimization for Binary
 * Sequences with High Merit Factors", arXiv 2409.07222):
 *   - Sec. 1, the autocorrelation C_k and energy E definitions and Eq. (1), merit factor;
 *   - Sec. 1, Eq. (2), skew-symmetry; Eq. (3), restriction-class prefix layout;
 *   - Sec. 3, Algorithm 1 (first step) and the neighbourhood it searches, with a
 *     tabu tenure and with the Bloom filter the algorithm names;
 *   - Sec. 3, Algorithm 2 (second step) -- its queue bookkeeping lives in
 *     oracle/__init__.py, this file only provides the energies it needs.
 * No incremental formula is used anywhere: every energy change is computed as
 * E(flipped sequence) - E(sequence), each energy from the definition.
 *
 * Sequences are arrays of int8 holding +1 / -1; s[0] is s_1, s[L-1] is s_L.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Sec. 1: C_k(S) = sum_{i=1}^{L-k} s_i s_{i+k}.                              */
int64_t or_autocorr(int32_t L, const int8_t* s, int32_t k)
{
    int64_t c = 0;
    for (int32_t i = 1; i <= L - k; ++i)
        c += (int64_t)s[i - 1] * (int64_t)s[i + k - 1];
    return c;
}

/* Sec. 1: E(S) = sum_{k=1}^{L-1} C_k(S)^2.  C_out (nullable) receives C_1..C_{L-1}. */
int64_t or_energy(int32_t L, const int8_t* s, int64_t* C_out)
{
    int64_t e = 0;
    for (int32_t k = 1; k <= L - 1; ++k) {
        int64_t c = or_autocorr(L, s, k);
        if (C_out) C_out[k - 1] = c;
        e += c * c;
    }
    return e;
}

/* Batched form for tests: n sequences of length L stored back to back. */
void or_energy_batch(int32_t L, int64_t n, const int8_t* s, int64_t* E, int64_t* C)
{
    for (int64_t j = 0; j < n; ++j)
        E[j] = or_energy(L, s + j * L, C ? C + j * (int64_t)(L > 1 ? L - 1 : 0) : NULL);
}

/* ------------------------------------------------------------------------ */
/* Eq. (2): for L = 2k+1, s_{(k+1)+i} = (-1)^i s_{(k+1)-i}, i = 1..k.
 * Fills s_{k+2}..s_L from s_1..s_{k+1}. */
void or_skew_complete(int32_t L, int8_t* s)
{
    int32_t k = (L - 1) / 2;
    for (int32_t i = 1; i <= k; ++i) {
        int8_t v = s[(k + 1 - i) - 1];
        s[(k + 1 + i) - 1] = (i % 2 == 0) ? v : (int8_t)(-v);
    }
}

int32_t or_is_skew(int32_t L, const int8_t* s)
{
    if (L % 2 == 0) return 0;
    int32_t k = (L - 1) / 2;
    for (int32_t i = 1; i <= k; ++i) {
        int8_t v = s[(k + 1 - i) - 1];
        int8_t w = (i % 2 == 0) ? v : (int8_t)(-v);
        if (s[(k + 1 + i) - 1] != w) return 0;
    }
    return 1;
}

/* A neighbour in the first step (Sec. 3, the BEST_NEIGHBOUR description) stays
 * skew-symmetric: flipping a free position a <= k also flips the element Eq. (2)
 * ties to it, s_{L+1-a}; the centre a = k+1 is tied only to itself. */
void or_flip_skew(int32_t L, int8_t* s, int32_t a)
{
    int32_t b = L + 1 - a;
    s[a - 1] = (int8_t)(-s[a - 1]);
    if (b != a) s[b - 1] = (int8_t)(-s[b - 1]);
}

/* Energy change of one single flip at position i (1-based), Sec. 3 second step
 * neighbourhood: E(flip_i S) - E(S), both by definition. */
int64_t or_delta_single(int32_t L, const int8_t* s, int32_t i)
{
    int8_t* t = (int8_t*)malloc((size_t)L);
    memcpy(t, s, (size_t)L);
    int64_t e0 = or_energy(L, t, NULL);
    t[i - 1] = (int8_t)(-t[i - 1]);
    int64_t e1 = or_energy(L, t, NULL);
    free(t);
    return e1 - e0;
}

/* Energy change of one skew-preserving flip at position a: E(flip_skew_a S) - E(S). */
int64_t or_delta_skew(int32_t L, const int8_t* s, int32_t a)
{
    int8_t* t = (int8_t*)malloc((size_t)L);
    memcpy(t, s, (size_t)L);
    int64_t e0 = or_energy(L, t, NULL);
    or_flip_skew(L, t, a);
    int64_t e1 = or_energy(L, t, NULL);
    free(t);
    return e1 - e0;
}

/* All L single-flip changes of one sequence (second-step neighbourhood). */
void or_deltas_single(int32_t L, const int8_t* s, int64_t* out)
{
    for (int32_t i = 1; i <= L; ++i) out[i - 1] = or_delta_single(L, s, i);
}

/* The skew flips of the free positions a = p+1..k+1 (Eq. (3) layout). */
void or_deltas_skew(int32_t L, int32_t p, const int8_t* s, int64_t* out)
{
    int32_t k = (L - 1) / 2;
    for (int32_t a = p + 1; a <= k + 1; ++a) out[a - p - 1] = or_delta_skew(L, s, a);
}

/* ------------------------------------------------------------------------ */
/* SplitMix64 (G. Steele, D. Lea, C. Flood, "Fast splittable pseudorandom number
 * generators", OOPSLA 2014), written from its published definition: the state
 * advances by the golden-ratio increment and each output is the state passed
 * through the variant-13 finaliser.  The paper does not fix a generator; the
 * walker streams below are a reading of ours. */
static const uint64_t OR_GAMMA = 0x9E3779B97F4A7C15ull;

uint64_t or_mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

uint64_t or_splitmix64_next(uint64_t* state)
{
    *state += OR_GAMMA;
    return or_mix64(*state);
}

/* Walker stream key: depends only on (seed, L, walker id). */
uint64_t or_walker_key(uint64_t seed, int32_t L, int64_t walker)
{
    uint64_t lw = ((uint64_t)(uint32_t)L << 32) ^ (uint64_t)(walker + 1);
    return or_mix64(seed ^ or_mix64(lw));
}

/* INIT_PARTITIONED_SEQUENCE of Algorithm 1, with the restriction-class prefix of
 * Eq. (3) drawn from the seed (the paper's minimal-potential classes are not
 * reproduced).  The walker's SplitMix64 stream, started at its key, is read in
 * order: draw number i-1 decides s_i for i = 1..k+1 (+1 when its top bit is set;
 * when p >= 1 the first draw is discarded and s_1 = +1), draw number k+1 gives the
 * tabu tenure lo + (draw mod (hi-lo+1)).  The last k elements follow Eq. (2). */
void or_walker_init(uint64_t seed, int32_t L, int32_t p, int64_t walker,
                    int32_t tenure_lo, int32_t tenure_hi, int8_t* s, int32_t* tenure)
{
    int32_t k = (L - 1) / 2;
    uint64_t st = or_walker_key(seed, L, walker);
    for (int32_t i = 1; i <= k + 1; ++i) {
        uint64_t d = or_splitmix64_next(&st);
        s[i - 1] = (d >> 63) ? (int8_t)1 : (int8_t)-1;
    }
    if (p >= 1) s[0] = 1;
    or_skew_complete(L, s);
    uint64_t d = or_splitmix64_next(&st);
    uint64_t span = (uint64_t)(tenure_hi - tenure_lo + 1);
    *tenure = tenure_lo + (int32_t)(d % span);
}

/* ------------------------------------------------------------------------ */
/* One first-step walker (Algorithm 1 with a tabu tenure in place of the Bloom
 * filter).  For t = 1..steps:
 *   - evaluate every free skew neighbour a = p+1..k+1 (the whole neighbourhood,
 *     tabu or not), delta_a = E(flip_skew_a S) - E(S);
 *   - admissible: tabu_until[a] < t; none admissible -> the walk stops
 *     (the "i = -1" exit of Algorithm 1); the remaining trajectory is -1;
 *   - take the admissible a with the lowest (delta_a, a), uphill moves included;
 *   - flip it, e += delta, tabu_until[a] = t + tenure;
 *   - the sieve of Algorithm 1 with E_l = e_max + 1: emit the sequence when
 *     e <= e_max (e_max < 0 disables it).
 * best_* record the first step (t >= 0, t = 0 being the initial sequence) at
 * which the lowest energy of the walk was reached.
 * moves (nullable) receives the position flipped at each step (-1 after a stop).
 * emit_* (nullable) receive up to emit_cap emissions; the return value is the
 * total number of emissions (which may exceed emit_cap). */
int64_t or_walk_one(int32_t L, int32_t p, int32_t steps, int32_t tenure_lo, int32_t tenure_hi,
                    uint64_t seed, int64_t walker, int32_t e_max,
                    int32_t* traj, int32_t* moves, int8_t* final_s, int64_t* final_E,
                    int8_t* best_s, int64_t* best_E, int32_t* best_step,
                    int64_t emit_cap, int64_t* emit_E, int8_t* emit_s, int32_t* emit_t)
{
    int32_t k = (L - 1) / 2;
    int32_t nfree = k + 1 - p;
    int8_t* s = (int8_t*)malloc((size_t)L);
    int32_t* tabu_until = (int32_t*)calloc((size_t)nfree, sizeof(int32_t));
    int64_t* delta = (int64_t*)malloc((size_t)nfree * sizeof(int64_t));
    int32_t tenure = 0;
    int64_t n_emit = 0;

    or_walker_init(seed, L, p, walker, tenure_lo, tenure_hi, s, &tenure);
    int64_t e = or_energy(L, s, NULL);
    *best_E = e;
    *best_step = 0;
    memcpy(best_s, s, (size_t)L);

    int32_t t = 1;
    for (; t <= steps; ++t) {
        int64_t e_here = or_energy(L, s, NULL);
        for (int32_t a = p + 1; a <= k + 1; ++a) {
            or_flip_skew(L, s, a);
            delta[a - p - 1] = or_energy(L, s, NULL) - e_here;
            or_flip_skew(L, s, a);
        }
        int32_t best_a = -1;
        for (int32_t a = p + 1; a <= k + 1; ++a) {
            if (tabu_until[a - p - 1] >= t) continue;
            if (best_a < 0 || delta[a - p - 1] < delta[best_a - p - 1]) best_a = a;
        }
        if (best_a < 0) break;
        or_flip_skew(L, s, best_a);
        e += delta[best_a - p - 1];
        tabu_until[best_a - p - 1] = t + tenure;
        if (traj) traj[t - 1] = (int32_t)e;
        if (moves) moves[t - 1] = best_a;
        if (e < *best_E) {
            *best_E = e;
            *best_step = t;
            memcpy(best_s, s, (size_t)L);
        }
        if (e_max >= 0 && e <= e_max) {
            if (n_emit < emit_cap && emit_E) {
                emit_E[n_emit] = e;
                memcpy(emit_s + n_emit * L, s, (size_t)L);
                emit_t[n_emit] = t;
            }
            ++n_emit;
        }
    }
    for (; t <= steps; ++t) {
        if (traj) traj[t - 1] = -1;
        if (moves) moves[t - 1] = -1;
    }
    memcpy(final_s, s, (size_t)L);
    *final_E = e;
    free(s);
    free(tabu_until);
    free(delta);
    return n_emit;
}

/* ------------------------------------------------------------------------ */
/* Exhaustive enumeration over the skew-symmetric sequences whose first p
 * elements equal prefix[0..p-1]: the free elements s_{p+1}..s_{k+1} run over all
 * 2^(k+1-p) patterns (pattern bit j, LSB first, set -> s_{p+1+j} = +1).
 * E_out[pattern] receives every energy (nullable); returns the minimum. */
int64_t or_skew_exhaustive(int32_t L, int32_t p, const int8_t* prefix, int64_t* E_out)
{
    int32_t k = (L - 1) / 2;
    int32_t nfree = k + 1 - p;
    int8_t* s = (int8_t*)malloc((size_t)L);
    int64_t best = -1;
    uint64_t count = 1ull << nfree;
    for (uint64_t x = 0; x < count; ++x) {
        for (int32_t i = 0; i < p; ++i) s[i] = prefix[i];
        for (int32_t j = 0; j < nfree; ++j) s[p + j] = ((x >> j) & 1) ? 1 : -1;
        or_skew_complete(L, s);
        int64_t e = or_energy(L, s, NULL);
        if (E_out) E_out[x] = e;
        if (best < 0 || e < best) best = e;
    }
    free(s);
    return best;
}

/* Exhaustive minimum over all 2^L sequences (tiny L only). */
int64_t or_exhaustive_min(int32_t L, int64_t* count_out)
{
    int8_t* s = (int8_t*)malloc((size_t)L);
    int64_t best = -1, cnt = 0;
    for (uint64_t x = 0; x < (1ull << L); ++x) {
        for (int32_t i = 0; i < L; ++i) s[i] = ((x >> i) & 1) ? 1 : -1;
        int64_t e = or_energy(L, s, NULL);
        if (best < 0 || e < best) { best = e; cnt = 1; }
        else if (e == best) ++cnt;
    }
    free(s);
    if (count_out) *count_out = cnt;
    return best;
}

/* ------------------------------------------------------------------------ */
/* Bloom-filter self-avoidance (Sec. 3, Algorithm 1 with its Bloom filter,
 * Bloom 1970).  The paper fixes neither the hash nor the filter's size, so the
 * following are readings of ours:
 *   - a sequence is keyed by the 64-bit Zobrist hash (Zobrist 1970) of its first
 *     k+1 elements, which fix the rest under Eq. (2), with the table of the
 *     second step's keys:
 *       h(S) = XOR of Z_i over i = 1..k+1 with s_i = +1,
 *     Z_i = draw number i-1 of the SplitMix64 stream started at OR_ZOBRIST_STATE;
 *   - the filter holds m = 2^log2_bits bits; a key h sets / tests the bits
 *       (g1 + j*g2) mod m,  j = 0..n_hash-1,  g1 = low 32 bits of h,
 *       g2 = (high 32 bits of h) | 1
 *     (double hashing, Kirsch and Mitzenmacher 2006), arithmetic on 32 bits;
 *     a key is a member when all its bits are set. */
static const uint64_t OR_ZOBRIST_STATE = 0x6A09E667F3BCC909ull;

uint64_t or_zobrist_key(int32_t i)
{
    uint64_t st = OR_ZOBRIST_STATE;
    uint64_t z = 0;
    for (int32_t q = 1; q <= i; ++q) z = or_splitmix64_next(&st);
    return z;
}

uint64_t or_seq_hash(int32_t L, const int8_t* s)
{
    int32_t k = (L - 1) / 2;
    uint64_t st = OR_ZOBRIST_STATE;
    uint64_t h = 0;
    for (int32_t i = 1; i <= k + 1; ++i) {
        uint64_t z = or_splitmix64_next(&st);
        if (s[i - 1] > 0) h ^= z;
    }
    return h;
}

/* Bit index j of key h in a filter of 2^log2_bits bits. */
uint32_t or_bloom_index(uint64_t h, int32_t log2_bits, int32_t j)
{
    uint32_t g1 = (uint32_t)h;
    uint32_t g2 = (uint32_t)(h >> 32) | 1u;
    uint32_t v = g1 + (uint32_t)j * g2;
    return v & (uint32_t)((1ull << log2_bits) - 1ull);
}

/* bits: (2^log2_bits)/8 bytes, bit x at byte x/8, bit x%8. */
void or_bloom_insert(uint8_t* bits, int32_t log2_bits, int32_t n_hash, uint64_t h)
{
    for (int32_t j = 0; j < n_hash; ++j) {
        uint32_t x = or_bloom_index(h, log2_bits, j);
        bits[x >> 3] |= (uint8_t)(1u << (x & 7));
    }
}

int32_t or_bloom_member(const uint8_t* bits, int32_t log2_bits, int32_t n_hash, uint64_t h)
{
    for (int32_t j = 0; j < n_hash; ++j) {
        uint32_t x = or_bloom_index(h, log2_bits, j);
        if (!(bits[x >> 3] & (1u << (x & 7)))) return 0;
    }
    return 1;
}

/* One first-step walker of Algorithm 1 with the Bloom filter: the initial
 * sequence (or_walker_init; its tenure draw is unused) is inserted; for
 * t = 1..steps every free skew neighbour a = p+1..k+1 is evaluated, an
 * "unexplored" neighbour is one whose hash the filter does not hold, the walker
 * takes the unexplored a with the lowest (delta_a, a), uphill included, and
 * inserts the new sequence; with no unexplored neighbour the walk stops (its
 * remaining trajectory is -1).  Every hash is computed from the whole sequence
 * (no incremental update).  Sieve and outputs as in or_walk_one. */
int64_t or_walk_bloom_one(int32_t L, int32_t p, int32_t steps, int32_t log2_bits, int32_t n_hash,
                          uint64_t seed, int64_t walker, int32_t e_max,
                          int32_t* traj, int32_t* moves, int8_t* final_s, int64_t* final_E,
                          int8_t* best_s, int64_t* best_E, int32_t* best_step,
                          int64_t emit_cap, int64_t* emit_E, int8_t* emit_s, int32_t* emit_t)
{
    int32_t k = (L - 1) / 2;
    int32_t nfree = k + 1 - p;
    int8_t* s = (int8_t*)malloc((size_t)L);
    uint8_t* bits = (uint8_t*)calloc((size_t)1 << (log2_bits > 3 ? log2_bits - 3 : 0), 1);
    int64_t* delta = (int64_t*)malloc((size_t)nfree * sizeof(int64_t));
    int32_t* fresh = (int32_t*)malloc((size_t)nfree * sizeof(int32_t));
    int32_t unused_tenure = 0;
    int64_t n_emit = 0;

    or_walker_init(seed, L, p, walker, 0, 0, s, &unused_tenure);
    or_bloom_insert(bits, log2_bits, n_hash, or_seq_hash(L, s));
    int64_t e = or_energy(L, s, NULL);
    *best_E = e;
    *best_step = 0;
    memcpy(best_s, s, (size_t)L);

    int32_t t = 1;
    for (; t <= steps; ++t) {
        int64_t e_here = or_energy(L, s, NULL);
        for (int32_t a = p + 1; a <= k + 1; ++a) {
            or_flip_skew(L, s, a);
            delta[a - p - 1] = or_energy(L, s, NULL) - e_here;
            fresh[a - p - 1] = !or_bloom_member(bits, log2_bits, n_hash, or_seq_hash(L, s));
            or_flip_skew(L, s, a);
        }
        int32_t best_a = -1;
        for (int32_t a = p + 1; a <= k + 1; ++a) {
            if (!fresh[a - p - 1]) continue;
            if (best_a < 0 || delta[a - p - 1] < delta[best_a - p - 1]) best_a = a;
        }
        if (best_a < 0) break;
        or_flip_skew(L, s, best_a);
        or_bloom_insert(bits, log2_bits, n_hash, or_seq_hash(L, s));
        e += delta[best_a - p - 1];
        if (traj) traj[t - 1] = (int32_t)e;
        if (moves) moves[t - 1] = best_a;
        if (e < *best_E) {
            *best_E = e;
            *best_step = t;
            memcpy(best_s, s, (size_t)L);
        }
        if (e_max >= 0 && e <= e_max) {
            if (n_emit < emit_cap && emit_E) {
                emit_E[n_emit] = e;
                memcpy(emit_s + n_emit * L, s, (size_t)L);
                emit_t[n_emit] = t;
            }
            ++n_emit;
        }
    }
    for (; t <= steps; ++t) {
        if (traj) traj[t - 1] = -1;
        if (moves) moves[t - 1] = -1;
    }
    memcpy(final_s, s, (size_t)L);
    *final_E = e;
    free(s);
    free(bits);
    free(delta);
    free(fresh);
    return n_emit;
}
