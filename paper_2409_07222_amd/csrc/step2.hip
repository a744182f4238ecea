// Second step (Algorithm 2) as a device-resident, batch-synchronous best-first
// search.  Every round runs as a fixed sequence of kernels that read a control
// block in device memory; the host enqueues rounds and looks at the stop flag
// every few rounds.
//
// Data structures (all in the caller's workspace):
//  * a hash set H keyed by the exact sequence (open addressing, linear probing).
//    A slot holds a 64-bit Zobrist key (0 = empty), a state (0 = being written,
//    OPEN, CLOSED, EVICTED), E and the packed sequence.  Zobrist keys make the
//    neighbour key one XOR away from the pivot's (Alg. 2's HASH_FLIP).  H holds
//    Closed U Open U evicted; an EVICTED slot counts as absent and is re-opened
//    when its sequence is pushed again.
//  * the Open list: (E, slot) pairs, unordered, with dead entries (E = DEAD)
//    left by pops and evictions and compacted away when space runs short.
//  * an exact "T smallest in key order" selection: radix select on E in 11-bit
//    digits, then an MSD byte-wise radix select on the sequence among entries
//    tied at the threshold energy.
//
// Insertion is exact without sorting: a lane claims an empty slot with a 64-bit
// CAS of its key and then publishes the slot (data first, state last); a lane
// that meets its own key in a slot waits (bounded) for publication and compares
// sequences.  Claim-and-publish precedes the wait in program order, so a
// publisher in the same wavefront has always published before anyone waits.
#include "labs_internal.h"

#include <climits>

namespace labsdev {

namespace {

constexpr int32_t DEAD = INT32_MAX;
constexpr uint32_t ST_OPEN = 1, ST_CLOSED = 2, ST_EVICTED = 3;
constexpr uint64_t ZKEY = 0x6A09E667F3BCC909ull;   // Zobrist stream key
constexpr int kSelBits = 11;
constexpr int kSelBins = 1 << kSelBits;
constexpr int kMaxL = 1023;
constexpr int kPad = 1024;
constexpr int kSv = kMaxL + 2 * kPad + 2;
constexpr int kSpinLimit = 1 << 22;

struct Table {
    unsigned long long* hkey;
    uint32_t* state;
    int32_t* E;
    uint32_t* seq;
    uint64_t mask;
    int32_t W;
};

struct Ctl {
    // persistent
    long long n_tot, n_live;
    long long expansions, pushes, dups, evictions, rounds, u;
    int32_t best_E, best_slot, best_round, stop;
    int32_t error, which, pad0, pad1;
    // per round
    long long n_piv, batch_begin;
    int32_t batch_minE, improved, need_compact, pad2;
    long long compact_count;
    // selection
    long long T, c_lt, need;
    uint32_t emin, emax;
    int32_t sel_enabled, sel_all;
    int32_t hi_shift, lo_shift;
    uint32_t prefix, Dt;
    int32_t resolved, n_cand;
    int32_t Et, pad3;
    // table occupancy (claimed slots, tombstones included) and rebuild scratch
    long long claimed, claimed_new;
};

struct Params {
    int32_t L, W, B;
    long long Q, X, T_u;
    long long cap_o;
    Table H;
    Ctl* ctl;
    int32_t* oE[2];
    int32_t* oS[2];
    uint32_t* flag;     // [cap_o]
    int32_t* cand[2];   // [cap_o] each
    int32_t* piv;       // [B]
    uint32_t* ghist;    // [kSelBins]
    uint32_t* best_seq; // [W] copy of the best sequence
};

__device__ __forceinline__ uint64_t zob(int i) { return sm64_at(ZKEY, (uint64_t)i); }

__device__ __forceinline__ uint32_t ld_acq(const uint32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t ld_rlx(const uint32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned long long ld_rlx64(const unsigned long long* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Wave-aggregated append: returns this lane's index (valid only where `take`).
__device__ __forceinline__ long long wave_append(long long* counter, bool take) {
    const uint64_t m = __ballot(take);
    if (!m) return -1;
    const int lane = threadIdx.x & 63;
    const int leader = __ffsll((unsigned long long)m) - 1;
    long long base = 0;
    if (lane == leader) base = atomicAdd((unsigned long long*)counter, (unsigned long long)__popcll(m));
    base = __shfl(base, leader, 64);
    const uint64_t lt = lane ? (~0ull >> (64 - lane)) : 0ull;
    return base + __popcll(m & lt);
}

__device__ __forceinline__ int wave_min_i32(int v) { return __ockl_wfred_min_i32(v); }

// Key order between the sequences of two slots (words compared as unsigned).
__device__ __forceinline__ bool key_less(const Table& H, int a, int b) {
    for (int w = 0; w < H.W; ++w) {
        uint32_t x = H.seq[(size_t)a * H.W + w], y = H.seq[(size_t)b * H.W + w];
        if (x != y) return x < y;
    }
    return false;
}

enum { INS_DUP = 0, INS_PUSHED = 1, INS_FAIL = 2 };

// Insert the sequence `wrd` (W words) with energy E and key; returns the slot
// through *slot_out when pushed.  Called by every lane of a wavefront (lanes
// with active = false do nothing).  The probe loop runs until no lane of the
// wave is left probing, so no lane leaves it early: a lane that claims a slot
// publishes it in the same iteration, before any lane of the wave waits on a
// claimed-but-unpublished slot.  That rules out a wait cycle between waves.
__device__ int table_insert(const Table& H, const uint32_t* wrd, int32_t E, unsigned long long key,
                            int* slot_out, Ctl* ctl, bool active) {
    uint64_t s = key & H.mask;
    bool done = !active;
    int res = INS_DUP;
    uint64_t probes = 0;
    while (__ballot(!done)) {
        unsigned long long cur = 0;
        bool claimed = false;
        if (!done) {
            cur = ld_rlx64(&H.hkey[s]);
            if (cur == 0ull) {
                unsigned long long prev = atomicCAS(&H.hkey[s], 0ull, key);
                if (prev == 0ull) claimed = true;
                else cur = prev;
            }
        }
        if (claimed) {
            for (int w = 0; w < H.W; ++w) H.seq[s * H.W + w] = wrd[w];
            H.E[s] = E;
            __hip_atomic_store(&H.state[s], ST_OPEN, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            *slot_out = (int)s;
            res = INS_PUSHED;
            done = true;
        }
        {
            const uint64_t cm = __ballot(claimed);
            if (cm && (threadIdx.x & 63) == (unsigned)(__ffsll((unsigned long long)cm) - 1))
                atomicAdd((unsigned long long*)&ctl->claimed, (unsigned long long)__popcll(cm));
        }
        __builtin_amdgcn_wave_barrier();
        if (!done && cur == key) {
            uint32_t st = ld_acq(&H.state[s]);
            for (int it = 0; st == 0 && it < kSpinLimit; ++it) {
                __builtin_amdgcn_s_sleep(2);
                st = ld_acq(&H.state[s]);
            }
            if (st == 0) {
                atomicExch(&ctl->error, 1);
                res = INS_FAIL;
                done = true;
            } else {
                bool eq = true;
                for (int w = 0; w < H.W; ++w)
                    if (ld_rlx(&H.seq[s * H.W + w]) != wrd[w]) { eq = false; break; }
                if (eq) {
                    res = INS_DUP;
                    if (st == ST_EVICTED &&
                        atomicCAS(&H.state[s], ST_EVICTED, ST_OPEN) == ST_EVICTED) {
                        *slot_out = (int)s;
                        res = INS_PUSHED;
                    }
                    done = true;
                }
            }
        }
        if (!done) {
            s = (s + 1) & H.mask;
            if (++probes > H.mask) {
                atomicExch(&ctl->error, 2);
                res = INS_FAIL;
                done = true;
            }
        }
    }
    return res;
}

// Unpack W words into the zero-padded int8 array and compute C_1..C_{L-1}.
__device__ void load_seq_and_c(const uint32_t* words, int L, int8_t* sv, int32_t* Cl, int lane) {
    for (int i = lane; i < kSv; i += 64) sv[i] = 0;
    __syncthreads();
    for (int x = 1 + lane; x <= L; x += 64) sv[kPad + x] = packed_bit(words, x) ? 1 : -1;
    __syncthreads();
    for (int d = 1 + lane; d <= L - 1; d += 64) {
        int c = 0;
        for (int i = 1; i <= L - d; ++i) c += (int)sv[kPad + i] * (int)sv[kPad + i + d];
        Cl[d] = c;
    }
    __syncthreads();
}

__device__ unsigned long long zobrist_of(const int8_t* sv, int L, int lane) {
    unsigned long long h = 0;
    for (int x = 1 + lane; x <= L; x += 64)
        if (sv[kPad + x] > 0) h ^= zob(x - 1);
    for (int o = 32; o > 0; o >>= 1) h ^= __shfl_xor(h, o, 64);
    return h;
}

// ---------------------------------------------------------------- seeding
__global__ __launch_bounds__(64) void k_seed(Params P, const uint32_t* cand, long long n_cand) {
    __shared__ int8_t sv[kSv];
    __shared__ int32_t Cl[kMaxL + 1];
    __shared__ uint32_t wrd[32];
    const int lane = threadIdx.x;
    const long long j = blockIdx.x;
    const int L = P.L, W = P.W;
    if (lane < W) wrd[lane] = cand[j * W + lane];
    __syncthreads();
    load_seq_and_c(wrd, L, sv, Cl, lane);
    int e = 0;
    for (int d = 1 + lane; d <= L - 1; d += 64) e += Cl[d] * Cl[d];
    e = __ockl_wfred_add_i32(e);
    unsigned long long key = zobrist_of(sv, L, lane) | 1ull;
    int slot = -1;
    const int res = table_insert(P.H, wrd, e, key, &slot, P.ctl, lane == 0);
    const bool take = lane == 0 && res == INS_PUSHED;
    long long idx = wave_append(&P.ctl->n_tot, take);
    if (take) {
        P.oE[0][idx] = e;
        P.oS[0][idx] = slot;
        atomicAdd((unsigned long long*)&P.ctl->n_live, 1ull);
    }
}

// ---------------------------------------------------------------- round control
__global__ void k_round_begin(Params P) {
    Ctl* c = P.ctl;
    if (c->stop) return;
    if (c->n_live == 0 || c->expansions >= P.X || c->u >= P.T_u) {
        c->stop = 1;
        return;
    }
    long long T = P.X - c->expansions;
    if (T > P.B) T = P.B;
    c->T = T;
    c->sel_enabled = 1;
    c->n_piv = 0;
    c->batch_minE = INT32_MAX;
    c->improved = 0;
    c->need_compact = (c->n_tot + (long long)P.B * P.L > P.cap_o) ? 1 : 0;
    c->compact_count = 0;
}

// Move live entries to the other buffer when space runs short.
__global__ void k_compact(Params P) {
    Ctl* c = P.ctl;
    if (c->stop || !c->need_compact) return;
    const int src = c->which;
    const long long n = c->n_tot;
    for (long long base = (long long)blockIdx.x * blockDim.x; base < n;
         base += (long long)gridDim.x * blockDim.x) {
        const long long i = base + threadIdx.x;
        const bool live = i < n && P.oE[src][i] != DEAD;
        const long long o = wave_append(&c->compact_count, live);
        if (live) {
            P.oE[1 - src][o] = P.oE[src][i];
            P.oS[1 - src][o] = P.oS[src][i];
        }
    }
}

__global__ void k_compact_fin(Params P) {
    Ctl* c = P.ctl;
    if (c->stop || !c->need_compact) return;
    c->n_tot = c->compact_count;
    c->which ^= 1;
}

// ---------------------------------------------------------------- selection
// Selects the T smallest live Open entries in key order into flag[].
__global__ void k_sel_reset(Params P) {
    Ctl* c = P.ctl;
    if (c->stop || !c->sel_enabled) return;
    c->emin = UINT32_MAX;
    c->emax = 0;
    c->n_cand = 0;
    c->sel_all = c->T >= c->n_live ? 1 : 0;
}

__global__ void k_sel_minmax(Params P) {
    Ctl* c = P.ctl;
    if (c->stop || !c->sel_enabled) return;
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
        atomicMin(&c->emin, mn);
        atomicMax(&c->emax, mx);
    }
}

__global__ void k_sel_setup(Params P) {
    Ctl* c = P.ctl;
    if (c->stop || !c->sel_enabled) return;
    const uint32_t R = c->emax - c->emin;
    const int nbits = R ? 32 - __clz((int)R) : 0;
    c->hi_shift = nbits;
    c->lo_shift = nbits > kSelBits ? nbits - kSelBits : 0;
    c->prefix = 0;
    c->c_lt = 0;
    c->need = c->T;
    c->resolved = (nbits == 0) ? 1 : 0;
    c->Dt = 0;
}

__global__ __launch_bounds__(256) void k_sel_hist(Params P) {
    Ctl* c = P.ctl;
    if (c->stop || !c->sel_enabled || c->sel_all || c->resolved) return;
    __shared__ uint32_t h[kSelBins];
    for (int b = threadIdx.x; b < kSelBins; b += blockDim.x) h[b] = 0;
    __syncthreads();
    const int cur = c->which;
    const uint32_t emin = c->emin, prefix = c->prefix;
    const int hs = c->hi_shift, ls = c->lo_shift;
    const uint32_t dmask = (1u << (hs - ls)) - 1u;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < c->n_tot;
         i += (long long)gridDim.x * blockDim.x) {
        const int32_t e = P.oE[cur][i];
        if (e == DEAD) continue;
        const uint32_t D = (uint32_t)e - emin;
        if (hs < 32 && (D >> hs) != prefix) continue;
        atomicAdd(&h[(D >> ls) & dmask], 1u);
    }
    __syncthreads();
    for (int b = threadIdx.x; b < kSelBins; b += blockDim.x)
        if (h[b]) atomicAdd(&P.ghist[b], h[b]);
}

__global__ __launch_bounds__(1024) void k_sel_find(Params P) {
    Ctl* c = P.ctl;
    if (c->stop || !c->sel_enabled || c->sel_all || c->resolved) return;
    __shared__ uint32_t part[1024];
    // 2 bins per thread
    const int t = threadIdx.x;
    const uint32_t a = P.ghist[2 * t], b = P.ghist[2 * t + 1];
    part[t] = a + b;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
        uint32_t x = t >= o ? part[t - o] : 0;
        __syncthreads();
        part[t] += x;
        __syncthreads();
    }
    const long long need = c->need - c->c_lt;   // entries still to take at this level
    const long long before = (long long)part[t] - (a + b);
    int v = -1;
    long long below = 0;
    if (before < need && need <= before + a) {
        v = 2 * t;
        below = before;
    } else if (before + a < need && need <= before + a + b) {
        v = 2 * t + 1;
        below = before + a;
    }
    __syncthreads();
    if (v >= 0) {
        const int hs = c->hi_shift, ls = c->lo_shift;
        c->c_lt += below;
        c->prefix = (c->prefix << (hs - ls)) | (uint32_t)v;
        if (ls == 0) {
            c->resolved = 1;
            c->Dt = c->prefix;
        } else {
            c->hi_shift = ls;
            c->lo_shift = ls > kSelBits ? ls - kSelBits : 0;
        }
    }
    __syncthreads();
    P.ghist[2 * t] = 0;
    P.ghist[2 * t + 1] = 0;
}

__global__ void k_sel_classify(Params P) {
    Ctl* c = P.ctl;
    if (c->stop || !c->sel_enabled) return;
    const int cur = c->which;
    const bool all = c->sel_all;
    const uint32_t Et = c->emin + c->Dt;
    for (long long base = (long long)blockIdx.x * blockDim.x; base < c->n_tot;
         base += (long long)gridDim.x * blockDim.x) {
        const long long i = base + threadIdx.x;
        bool tie = false;
        if (i < c->n_tot) {
            const int32_t e = P.oE[cur][i];
            uint32_t f = 0;
            if (e != DEAD) {
                if (all || (uint32_t)e < Et) f = 1;
                else if ((uint32_t)e == Et) tie = true;
            }
            P.flag[i] = f;
        }
        const uint64_t m = __ballot(tie);
        if (m) {
            const int lane = threadIdx.x & 63;
            const int leader = __ffsll((unsigned long long)m) - 1;
            int base_idx = 0;
            if (lane == leader) base_idx = atomicAdd(&c->n_cand, __popcll(m));
            base_idx = __shfl(base_idx, leader, 64);
            const uint64_t lt = lane ? (~0ull >> (64 - lane)) : 0ull;
            if (tie) P.cand[0][base_idx + __popcll(m & lt)] = (int32_t)i;
        }
    }
}

// Among the tied candidates, flag the `need - c_lt` smallest by sequence.
__global__ __launch_bounds__(1024) void k_sel_keys(Params P) {
    Ctl* c = P.ctl;
    if (c->stop || !c->sel_enabled || c->sel_all) return;
    __shared__ uint32_t h[256];
    __shared__ int s_v, s_m2;
    __shared__ long long s_r;
    const int cur = c->which;
    const int t = threadIdx.x;
    int m = c->n_cand;
    long long r = c->need - c->c_lt;
    int src = 0;
    const int W = P.W;
    for (int pos = 0; pos < 4 * W && r > 0; ++pos) {
        if (r == m) break;
        const int w = pos >> 2, sh = 24 - 8 * (pos & 3);
        for (int b = t; b < 256; b += blockDim.x) h[b] = 0;
        if (t == 0) s_m2 = 0;
        __syncthreads();
        for (int q = t; q < m; q += blockDim.x) {
            const int slot = P.oS[cur][P.cand[src][q]];
            atomicAdd(&h[(P.H.seq[(size_t)slot * W + w] >> sh) & 255u], 1u);
        }
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
            const int idx = P.cand[src][q];
            const int slot = P.oS[cur][idx];
            const int dgt = (P.H.seq[(size_t)slot * W + w] >> sh) & 255u;
            if (dgt < v) P.flag[idx] = 1;
            else if (dgt == v) P.cand[1 - src][atomicAdd(&s_m2, 1)] = idx;
        }
        __syncthreads();
        m = s_m2;
        r = s_r;
        src = 1 - src;
        __syncthreads();
    }
    if (r > 0)
        for (int q = t; q < m; q += blockDim.x) P.flag[P.cand[src][q]] = 1;
}

// ---------------------------------------------------------------- pop / expand
__global__ void k_pop(Params P) {
    Ctl* c = P.ctl;
    if (c->stop) return;
    const int cur = c->which;
    for (long long base = (long long)blockIdx.x * blockDim.x; base < c->n_tot;
         base += (long long)gridDim.x * blockDim.x) {
        const long long i = base + threadIdx.x;
        const bool take = i < c->n_tot && P.flag[i] && P.oE[cur][i] != DEAD;
        const long long o = wave_append(&c->n_piv, take);
        if (take && o >= P.B) atomicExch(&c->error, 3);
        if (take && o < P.B) {
            const int slot = P.oS[cur][i];
            P.piv[o] = slot;
            P.oE[cur][i] = DEAD;
            P.H.state[slot] = ST_CLOSED;
        }
    }
}

__global__ void k_pop_fin(Params P) {
    Ctl* c = P.ctl;
    if (c->stop) return;
    c->expansions += c->n_piv;
    c->n_live -= c->n_piv;
    c->batch_begin = c->n_tot;
}

__global__ __launch_bounds__(64) void k_expand(Params P) {
    Ctl* c = P.ctl;
    if (c->stop || (long long)blockIdx.x >= c->n_piv) return;
    __shared__ int8_t sv[kSv];
    __shared__ int32_t Cl[kMaxL + 1];
    __shared__ uint32_t pk[32];
    const int lane = threadIdx.x;
    const int L = P.L, W = P.W;
    const int cur = c->which;
    const int ps = P.piv[blockIdx.x];
    const int32_t Ep = P.H.E[ps];
    if (lane < W) pk[lane] = P.H.seq[(size_t)ps * W + lane];
    __syncthreads();
    load_seq_and_c(pk, L, sv, Cl, lane);
    const unsigned long long hp = zobrist_of(sv, L, lane);
    uint32_t nb[32];
    for (int r0 = 0; r0 < L; r0 += 64) {
        const int i = 1 + r0 + lane;
        const bool valid = i <= L;
        int slot = -1;
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
            for (int w = 0; w < W; ++w) nb[w] = pk[w];
            nb[(i - 1) >> 5] ^= 1u << (31 - ((i - 1) & 31));
            key = (hp ^ zob(i - 1)) | 1ull;
        }
        const int res = table_insert(P.H, nb, En, key, &slot, c, valid);
        const bool take = res == INS_PUSHED;
        const long long o = wave_append(&c->n_tot, take);
        if (take && o >= P.cap_o) atomicExch(&c->error, 4);
        if (take && o < P.cap_o) {
            P.oE[cur][o] = En;
            P.oS[cur][o] = slot;
        }
        const int mn = wave_min_i32(take ? En : INT32_MAX);
        if (lane == 0 && mn != INT32_MAX) atomicMin(&c->batch_minE, mn);
    }
}

__global__ void k_expand_fin(Params P) {
    Ctl* c = P.ctl;
    if (c->stop) return;
    const long long n_new = c->n_tot - c->batch_begin;
    c->pushes += n_new;
    c->dups += c->n_piv * P.L - n_new;
    c->n_live += n_new;
    if (c->batch_minE < c->best_E) c->improved = 1;
    else c->u += c->n_piv;
}

// best = smallest key among live entries in [lo, n_tot) with E == target.
__global__ __launch_bounds__(1024) void k_best(Params P, int initial) {
    Ctl* c = P.ctl;
    if (c->stop) return;
    if (!initial && !c->improved) return;
    __shared__ int best[1024];
    const int cur = c->which;
    const long long lo = initial ? 0 : c->batch_begin;
    const int32_t target = initial ? (int32_t)c->emin : c->batch_minE;
    int mine = -1;
    for (long long i = lo + threadIdx.x; i < c->n_tot; i += blockDim.x) {
        if (P.oE[cur][i] != target) continue;
        const int s = P.oS[cur][i];
        if (mine < 0 || key_less(P.H, s, mine)) mine = s;
    }
    best[threadIdx.x] = mine;
    __syncthreads();
    for (int o = 512; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
            const int x = best[threadIdx.x], y = best[threadIdx.x + o];
            if (x < 0 || (y >= 0 && key_less(P.H, y, x))) best[threadIdx.x] = y;
        }
        __syncthreads();
    }
    if (best[0] >= 0 && threadIdx.x < (unsigned)P.W)
        P.best_seq[threadIdx.x] = P.H.seq[(size_t)best[0] * P.W + threadIdx.x];
    if (threadIdx.x == 0 && best[0] >= 0) {
        c->best_slot = best[0];
        c->best_E = target;
        if (!initial) {
            c->best_round = (int32_t)c->rounds;
            c->u = 0;
        }
    }
}

__global__ void k_evict_setup(Params P) {
    Ctl* c = P.ctl;
    if (c->stop) return;
    c->sel_enabled = c->n_live > P.Q ? 1 : 0;
    c->T = P.Q;
}

__global__ void k_evict(Params P) {
    Ctl* c = P.ctl;
    if (c->stop || !c->sel_enabled) return;
    const int cur = c->which;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < c->n_tot;
         i += (long long)gridDim.x * blockDim.x) {
        if (P.oE[cur][i] == DEAD || P.flag[i]) continue;
        P.H.state[P.oS[cur][i]] = ST_EVICTED;
        P.oE[cur][i] = DEAD;
    }
}

__global__ void k_evict_fin(Params P) {
    Ctl* c = P.ctl;
    if (c->stop || !c->sel_enabled) return;
    c->evictions += c->n_live - P.Q;
    c->n_live = P.Q;
    c->sel_enabled = 0;
}

__global__ void k_round_end(Params P) {
    Ctl* c = P.ctl;
    if (c->stop) return;
    c->rounds += 1;
}

__global__ void k_outputs(Params P, uint32_t* best_seq, int32_t* best_E, labs_step2_stats* st,
                          uint32_t* open_seqs, int32_t* open_E, long long open_cap) {
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
    }
    if (!open_seqs && !open_E) return;
    // live entries in list order; ranks via one block-serial prefix is too slow,
    // so emit with a counter (order is unspecified by the ABI)
    const int cur = c->which;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < c->n_tot;
         i += (long long)gridDim.x * blockDim.x) {
        if (P.oE[cur][i] == DEAD) continue;
        const long long o = (long long)atomicAdd((unsigned long long*)&c->compact_count, 1ull);
        if (o >= open_cap) continue;
        const int s = P.oS[cur][i];
        if (open_E) open_E[o] = P.oE[cur][i];
        if (open_seqs)
            for (int w = 0; w < W; ++w) open_seqs[o * W + w] = P.H.seq[(size_t)s * W + w];
    }
}

// ---------------------------------------------------------------- table rebuild
// Re-insert the OPEN and CLOSED slots of `src` into the empty table `dst`
// (tombstones of evicted sequences are dropped) and record old -> new slots.
__global__ void k_rebuild(Table src, Table dst, uint32_t* remap, Ctl* c) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i <= src.mask;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t st = src.state[i];
        if (src.hkey[i] == 0ull || (st != ST_OPEN && st != ST_CLOSED)) continue;
        const unsigned long long key = src.hkey[i];
        uint64_t s = key & dst.mask;
        for (uint64_t probe = 0; probe <= dst.mask; ++probe) {
            if (atomicCAS(&dst.hkey[s], 0ull, key) == 0ull) break;
            s = (s + 1) & dst.mask;
        }
        for (int w = 0; w < src.W; ++w) dst.seq[s * dst.W + w] = src.seq[i * src.W + w];
        dst.E[s] = src.E[i];
        dst.state[s] = st;
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
}

__global__ void k_rebuild_fin(Ctl* c, const uint32_t* remap) {
    if (c->best_slot >= 0) c->best_slot = (int32_t)remap[c->best_slot];
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

__global__ void k_prepare_outputs(Ctl* c) { c->compact_count = 0; }

// The initial best is the smallest live entry; k_sel_minmax provides its energy.
__global__ void k_initial_best_setup(Params P) { P.ctl->sel_enabled = 1; }

inline unsigned grid_for(long long n, int t, unsigned cap = 2048) {
    long long b = (n + t - 1) / t;
    if (b < 1) b = 1;
    return (unsigned)(b > cap ? cap : b);
}

uint64_t next_pow2(uint64_t x) {
    uint64_t p = 1;
    while (p < x) p <<= 1;
    return p;
}

constexpr int kCheck = 16;   // rounds between host looks at the control block

struct S2Layout {
    uint64_t cap_ht;
    long long cap_o;
    size_t total;
};

S2Layout s2_layout(const labs_step2_cfg& c, long long n_cand) {
    S2Layout lo;
    const int W = words_of(c.L);
    const long long base = (n_cand > c.pq_capacity ? n_cand : c.pq_capacity);
    const long long BL = (long long)c.batch * c.L;
    lo.cap_o = base + 2 * BL + 1024;
    // live slots never exceed n_cand + X + Q + BL; the table is rebuilt when half
    // of it is claimed, with kCheck rounds of claims as headroom.
    const long long live = n_cand + c.max_expansions + c.pq_capacity + BL;
    lo.cap_ht = next_pow2((uint64_t)(4 * (live + (long long)kCheck * BL) + 1024));
    size_t t = 0;
    for (int tb = 0; tb < 2; ++tb) {
        t += align_up(sizeof(unsigned long long) * lo.cap_ht, 256);
        t += align_up(sizeof(uint32_t) * lo.cap_ht, 256);
        t += align_up(sizeof(int32_t) * lo.cap_ht, 256);
        t += align_up(sizeof(uint32_t) * lo.cap_ht * W, 256);
    }
    t += align_up(sizeof(uint32_t) * lo.cap_ht, 256);     // remap
    t += align_up(sizeof(Ctl), 256);
    t += 2 * align_up(sizeof(int32_t) * lo.cap_o, 256);   // oE
    t += 2 * align_up(sizeof(int32_t) * lo.cap_o, 256);   // oS
    t += align_up(sizeof(uint32_t) * lo.cap_o, 256);      // flag
    t += 2 * align_up(sizeof(int32_t) * lo.cap_o, 256);   // cand
    t += align_up(sizeof(int32_t) * c.batch, 256);        // piv
    t += align_up(sizeof(uint32_t) * kSelBins, 256);      // ghist
    t += align_up(sizeof(uint32_t) * 32, 256);            // best sequence
    lo.total = t + 4096;
    return lo;
}

}  // namespace

size_t step2_workspace_bytes(const labs_step2_cfg& c, long long n_cand) {
    return s2_layout(c, n_cand).total;
}

// The host loop.  `timer_begin/end` bracket every expansion launch.
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
    Table tabs[2];
    for (int tb = 0; tb < 2; ++tb) {
        tabs[tb].hkey = cv.take<unsigned long long>(lo.cap_ht);
        tabs[tb].state = cv.take<uint32_t>(lo.cap_ht);
        tabs[tb].E = cv.take<int32_t>(lo.cap_ht);
        tabs[tb].seq = cv.take<uint32_t>(lo.cap_ht * P.W);
        tabs[tb].mask = lo.cap_ht - 1;
        tabs[tb].W = P.W;
    }
    uint32_t* remap = cv.take<uint32_t>(lo.cap_ht);
    int tcur = 0;
    P.H = tabs[0];
    P.ctl = cv.take<Ctl>(1);
    for (int b = 0; b < 2; ++b) P.oE[b] = cv.take<int32_t>(lo.cap_o);
    for (int b = 0; b < 2; ++b) P.oS[b] = cv.take<int32_t>(lo.cap_o);
    P.flag = cv.take<uint32_t>(lo.cap_o);
    for (int b = 0; b < 2; ++b) P.cand[b] = cv.take<int32_t>(lo.cap_o);
    P.piv = cv.take<int32_t>(cfg.batch);
    P.ghist = cv.take<uint32_t>(kSelBins);
    P.best_seq = cv.take<uint32_t>(32);
    if (!cv.ok()) return invalid("workspace layout overflow");

    LABS_HIP(hipMemsetAsync(P.H.hkey, 0, sizeof(unsigned long long) * lo.cap_ht, st));
    LABS_HIP(hipMemsetAsync(P.H.state, 0, sizeof(uint32_t) * lo.cap_ht, st));
    LABS_HIP(hipMemsetAsync(P.best_seq, 0, sizeof(uint32_t) * 32, st));
    LABS_HIP(hipMemsetAsync(P.ghist, 0, sizeof(uint32_t) * kSelBins, st));
    hipLaunchKernelGGL(k_init_ctl, dim3(1), dim3(1), 0, st, P.ctl);
    hipLaunchKernelGGL(k_seed, dim3((unsigned)n_cand), dim3(64), 0, st, P, cand_seqs, n_cand);
    LABS_LAUNCHED("step2 seed");

    const unsigned gsel = grid_for(lo.cap_o, 256);
    auto select = [&]() -> labs_status {
        hipLaunchKernelGGL(k_sel_reset, dim3(1), dim3(1), 0, st, P);
        hipLaunchKernelGGL(k_sel_minmax, dim3(gsel), dim3(256), 0, st, P);
        hipLaunchKernelGGL(k_sel_setup, dim3(1), dim3(1), 0, st, P);
        for (int lv = 0; lv < 3; ++lv) {
            hipLaunchKernelGGL(k_sel_hist, dim3(gsel), dim3(256), 0, st, P);
            hipLaunchKernelGGL(k_sel_find, dim3(1), dim3(1024), 0, st, P);
        }
        hipLaunchKernelGGL(k_sel_classify, dim3(gsel), dim3(256), 0, st, P);
        hipLaunchKernelGGL(k_sel_keys, dim3(1), dim3(1024), 0, st, P);
        LABS_LAUNCHED("step2 select");
        return LABS_OK;
    };
    labs_status s;
    // initial cut to Q and the initial best
    hipLaunchKernelGGL(k_evict_setup, dim3(1), dim3(1), 0, st, P);
    if ((s = select()) != LABS_OK) return s;
    hipLaunchKernelGGL(k_evict, dim3(gsel), dim3(256), 0, st, P);
    hipLaunchKernelGGL(k_evict_fin, dim3(1), dim3(1), 0, st, P);
    hipLaunchKernelGGL(k_initial_best_setup, dim3(1), dim3(1), 0, st, P);
    hipLaunchKernelGGL(k_sel_reset, dim3(1), dim3(1), 0, st, P);
    hipLaunchKernelGGL(k_sel_minmax, dim3(gsel), dim3(256), 0, st, P);
    hipLaunchKernelGGL(k_best, dim3(1), dim3(1024), 0, st, P, 1);
    LABS_LAUNCHED("step2 init");

    for (long long r = 0;; ++r) {
        hipLaunchKernelGGL(k_round_begin, dim3(1), dim3(1), 0, st, P);
        hipLaunchKernelGGL(k_compact, dim3(gsel), dim3(256), 0, st, P);
        hipLaunchKernelGGL(k_compact_fin, dim3(1), dim3(1), 0, st, P);
        if ((s = select()) != LABS_OK) return s;
        hipLaunchKernelGGL(k_pop, dim3(gsel), dim3(256), 0, st, P);
        hipLaunchKernelGGL(k_pop_fin, dim3(1), dim3(1), 0, st, P);
        if (tb && (s = tb(tctx, st)) != LABS_OK) return s;
        hipLaunchKernelGGL(k_expand, dim3((unsigned)cfg.batch), dim3(64), 0, st, P);
        if (te && (s = te(tctx, st)) != LABS_OK) return s;
        hipLaunchKernelGGL(k_expand_fin, dim3(1), dim3(1), 0, st, P);
        hipLaunchKernelGGL(k_best, dim3(1), dim3(1024), 0, st, P, 0);
        hipLaunchKernelGGL(k_evict_setup, dim3(1), dim3(1), 0, st, P);
        if ((s = select()) != LABS_OK) return s;
        hipLaunchKernelGGL(k_evict, dim3(gsel), dim3(256), 0, st, P);
        hipLaunchKernelGGL(k_evict_fin, dim3(1), dim3(1), 0, st, P);
        hipLaunchKernelGGL(k_round_end, dim3(1), dim3(1), 0, st, P);
        LABS_LAUNCHED("step2 round");
        if ((r + 1) % kCheck == 0) {
            int32_t flags[2];
            long long claimed = 0;
            LABS_HIP(hipMemcpyAsync(flags, &P.ctl->stop, sizeof(flags), hipMemcpyDeviceToHost, st));
            LABS_HIP(hipMemcpyAsync(&claimed, &P.ctl->claimed, sizeof(claimed), hipMemcpyDeviceToHost, st));
            LABS_HIP(hipStreamSynchronize(st));
            if (flags[1]) {
                set_error("second-step hash set failure (code %d)", flags[1]);
                return LABS_E_DEVICE;
            }
            if (flags[0]) break;
            if ((uint64_t)claimed * 2 >= lo.cap_ht) {
                Table& dst = tabs[1 - tcur];
                LABS_HIP(hipMemsetAsync(dst.hkey, 0, sizeof(unsigned long long) * lo.cap_ht, st));
                LABS_HIP(hipMemsetAsync(dst.state, 0, sizeof(uint32_t) * lo.cap_ht, st));
                hipLaunchKernelGGL(k_rebuild, dim3(grid_for((long long)lo.cap_ht, 256, 8192)), dim3(256), 0, st,
                                   tabs[tcur], dst, remap, P.ctl);
                hipLaunchKernelGGL(k_remap, dim3(gsel), dim3(256), 0, st, P, remap);
                hipLaunchKernelGGL(k_rebuild_fin, dim3(1), dim3(1), 0, st, P.ctl, remap);
                LABS_LAUNCHED("step2 rebuild");
                tcur = 1 - tcur;
                P.H = tabs[tcur];
            }
        }
    }
    hipLaunchKernelGGL(k_prepare_outputs, dim3(1), dim3(1), 0, st, P.ctl);
    hipLaunchKernelGGL(k_outputs, dim3(gsel), dim3(256), 0, st, P, out.best_seq, out.best_E, out.stats,
                       out.open_seqs, out.open_E, (long long)out.open_capacity);
    LABS_LAUNCHED("step2 outputs");
    LABS_HIP(hipStreamSynchronize(st));
    return LABS_OK;
}

}  // namespace labsdev
