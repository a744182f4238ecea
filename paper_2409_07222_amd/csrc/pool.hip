// Candidate pool (the sieve of Algorithm 1 feeding Algorithm 2) and top-k.
//
// Records live word-major in a RecBuf: key word 0 = E, words 1..W = packed
// sequence, word W+1 = walker id, word W+2 = step.  Ordering by all KW words
// (word 0 most significant) sorts by (E, sequence) and, within copies of one
// sequence, by (walker, step): the first record of each run of equal
// sequences is then the earliest offer.  The sort is an LSD radix sort over
// 8-bit digits of a permutation; digits that are equal in every record are
// found up front and skipped.
#include "labs_internal.h"

namespace labsdev {

namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
constexpr int kRounds = 32;                              // rounds of 64 items per wave
constexpr int kTile = kThreads * kRounds;                // 8192 items per block
constexpr int kMaxKeyWords = 40;                         // W + 3 <= 35 for L <= 1023

__global__ void k_iota(uint32_t* p, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = (uint32_t)i;
}

// OR over records of (word ^ word of record 0), per key word.
__global__ void k_varying(const uint32_t* rec, int64_t stride, int64_t n, int KW, uint32_t* var) {
    for (int q = 0; q < KW; ++q) {
        const uint32_t* w = rec + q * stride;
        const uint32_t w0 = w[0];
        uint32_t acc = 0;
        for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
             i += (int64_t)gridDim.x * blockDim.x)
            acc |= w[i] ^ w0;
        acc = __ockl_wfred_or_u32(acc);
        if ((threadIdx.x & 63) == 0 && acc) atomicOr(&var[q], acc);
    }
}

__device__ __forceinline__ int digit_of(const uint32_t* kw, const uint32_t* perm, int64_t i,
                                        int64_t n, int shift) {
    return i < n ? (int)((kw[perm[i]] >> shift) & 255u) : 256;
}

__global__ __launch_bounds__(kThreads) void k_rs_hist(const uint32_t* kw, const uint32_t* perm,
                                                      int64_t n, int shift, uint32_t* ghist,
                                                      int nblk) {
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kTile;
    for (int r = 0; r < kRounds; ++r) {
        int64_t i = base + (int64_t)r * kThreads + threadIdx.x;
        int d = digit_of(kw, perm, i, n, shift);
        if (d < 256) atomicAdd(&h[d], 1u);
    }
    __syncthreads();
    ghist[(int64_t)threadIdx.x * nblk + blockIdx.x] = h[threadIdx.x];
}

// Exclusive scan of M values in one block of 1024 threads.
__global__ __launch_bounds__(1024) void k_scan_excl(uint32_t* v, int64_t M) {
    __shared__ uint32_t part[1024];
    const int64_t per = (M + 1023) / 1024;
    const int64_t b = threadIdx.x * per;
    const int64_t e = min(b + per, M);
    uint32_t s = 0;
    for (int64_t i = b; i < e; ++i) s += v[i];
    part[threadIdx.x] = s;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
        uint32_t x = threadIdx.x >= o ? part[threadIdx.x - o] : 0;
        __syncthreads();
        part[threadIdx.x] += x;
        __syncthreads();
    }
    uint32_t run = part[threadIdx.x] - s;
    for (int64_t i = b; i < e; ++i) {
        uint32_t x = v[i];
        v[i] = run;
        run += x;
    }
}

// Stable scatter of one digit pass.  Wave w of block b owns items
// [b*kTile + w*64*kRounds, +64*kRounds), processed in rounds of 64 in order.
__global__ __launch_bounds__(kThreads) void k_rs_scatter(const uint32_t* kw, const uint32_t* perm_in,
                                                         uint32_t* perm_out, int64_t n, int shift,
                                                         const uint32_t* gofs, int nblk) {
    __shared__ uint32_t cnt[kWaves][256];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int d = threadIdx.x; d < kWaves * 256; d += kThreads) (&cnt[0][0])[d] = 0;
    __syncthreads();
    const int64_t wbase = (int64_t)blockIdx.x * kTile + (int64_t)wv * 64 * kRounds;
    for (int r = 0; r < kRounds; ++r) {
        int d = digit_of(kw, perm_in, wbase + r * 64 + lane, n, shift);
        if (d < 256) atomicAdd(&cnt[wv][d], 1u);
    }
    __syncthreads();
    {
        const int d = threadIdx.x;  // kThreads == 256 digits
        uint32_t run = gofs[(int64_t)d * nblk + blockIdx.x];
        for (int w = 0; w < kWaves; ++w) {
            uint32_t t = cnt[w][d];
            cnt[w][d] = run;
            run += t;
        }
    }
    __syncthreads();
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    for (int r = 0; r < kRounds; ++r) {
        const int64_t i = wbase + r * 64 + lane;
        const int d = digit_of(kw, perm_in, i, n, shift);
        const bool valid = d < 256;
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const uint64_t bal = __ballot((d >> b) & 1);
            peers &= ((d >> b) & 1) ? bal : ~bal;
        }
        uint32_t base = valid ? cnt[wv][d] : 0;
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        if (valid) {
            const uint32_t rank = (uint32_t)__popcll(peers & lt);
            perm_out[base + rank] = perm_in[i];
            if (rank == 0) cnt[wv][d] = base + (uint32_t)__popcll(peers);
        }
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    }
}

// first[i] = 1 when sorted record i starts a new sequence (words 1..W differ).
__global__ void k_unique_flags(const uint32_t* rec, int64_t stride, int W, const uint32_t* perm,
                               int64_t n, uint32_t* flag) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t f = 1;
    if (i > 0) {
        f = 0;
        const uint32_t a = perm[i], b = perm[i - 1];
        for (int q = 1; q <= W; ++q)
            if (rec[q * stride + a] != rec[q * stride + b]) { f = 1; break; }
    }
    flag[i] = f;
}

// Block-level pieces of a two-level exclusive scan over n values.
__global__ __launch_bounds__(1024) void k_block_sums(const uint32_t* v, int64_t n, uint32_t* sums) {
    __shared__ uint32_t s[1024];
    int64_t i = (int64_t)blockIdx.x * 1024 + threadIdx.x;
    s[threadIdx.x] = i < n ? v[i] : 0;
    __syncthreads();
    for (int o = 512; o > 0; o >>= 1) {
        if (threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) sums[blockIdx.x] = s[0];
}

__global__ __launch_bounds__(1024) void k_block_scan_apply(uint32_t* v, int64_t n,
                                                           const uint32_t* sums_excl, uint32_t* total) {
    __shared__ uint32_t s[1024];
    int64_t i = (int64_t)blockIdx.x * 1024 + threadIdx.x;
    uint32_t x = i < n ? v[i] : 0;
    s[threadIdx.x] = x;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
        uint32_t y = threadIdx.x >= o ? s[threadIdx.x - o] : 0;
        __syncthreads();
        s[threadIdx.x] += y;
        __syncthreads();
    }
    if (i < n) v[i] = sums_excl[blockIdx.x] + s[threadIdx.x] - x;
    if (i == n - 1) *total = sums_excl[blockIdx.x] + s[threadIdx.x];
}

// Write the first `cap` distinct sorted records into the output arrays.
__global__ void k_gather_unique(const uint32_t* rec, int64_t stride, int W, const uint32_t* perm,
                                const uint32_t* flag_raw, const uint32_t* pos, int64_t n, int64_t cap,
                                uint32_t* out_seqs, int32_t* out_E, int64_t* out_walker,
                                int32_t* out_step) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || !flag_raw[i]) return;
    const int64_t o = pos[i];
    if (o >= cap) return;
    const uint32_t a = perm[i];
    out_E[o] = (int32_t)rec[a];
    for (int q = 1; q <= W; ++q) out_seqs[o * W + (q - 1)] = rec[q * stride + a];
    if (out_walker) out_walker[o] = (int64_t)rec[(W + 1) * stride + a];
    if (out_step) out_step[o] = (int32_t)rec[(W + 2) * stride + a];
}

// dropped (when not null) grows by the distinct sequences beyond the capacity;
// with a cut set the set's inserts count them instead.
__global__ void k_finish_counts(const uint32_t* distinct, int64_t cap, int64_t* count,
                                int64_t* dropped, int64_t* out_n) {
    if (threadIdx.x || blockIdx.x) return;
    const int64_t D = *distinct;
    const int64_t keep = D < cap ? D : cap;
    if (count) *count = keep;
    if (dropped) *dropped += D - keep;
    if (out_n) *out_n = keep;
}

// ---------------------------------------------------------------- cut set
// Hash of record a's sequence words (a SplitMix64 finaliser chain), never 0.
__device__ __forceinline__ uint64_t rec_seq_hash(const uint32_t* rec, int64_t stride, int W, uint32_t a) {
    uint64_t h = 0x243F6A8885A308D3ull;
    for (int q = 1; q <= W; ++q) h = sm64_mix(h ^ ((uint64_t)rec[q * stride + a] << 16) ^ (uint64_t)q);
    return h | 1ull;
}

// Sorted record i is a candidate when it starts a run of equal sequences
// (flag[i] = 1) at a position beyond the capacity.  Candidates the set already
// holds (from an earlier compaction of the call) are cleared in flag; the set
// is not written here, so every comparison sees whole entries.
__global__ void k_cut_lookup(const uint32_t* rec, int64_t stride, int W, const uint32_t* perm,
                             uint32_t* flag, const uint32_t* pos, int64_t n, int64_t cap, CutSet cs) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || !flag[i]) return;
    if ((int64_t)pos[i] < cap) {
        flag[i] = 0;
        return;
    }
    if (cs.status[1] > (uint32_t)(cs.slots >> 1)) {
        // more than half full before this batch: the count cannot stay exact
        flag[i] = 0;
        atomicOr(&cs.status[0], 1u);
        return;
    }
    const uint32_t a = perm[i];
    const uint64_t key = rec_seq_hash(rec, stride, W, a);
    const uint64_t mask = (uint64_t)cs.slots - 1;
    uint64_t slot = key & mask;
    for (int64_t probe = 0; probe < cs.slots; ++probe, slot = (slot + 1) & mask) {
        const uint64_t k = cs.keys[slot];
        if (k == 0) return;                               // absent: stays a candidate
        if (k != key) continue;
        const uint32_t* w = cs.words + slot * (uint64_t)W;
        bool eq = true;
        for (int q = 0; q < W && eq; ++q) eq = w[q] == rec[(q + 1) * stride + a];
        if (eq) {
            flag[i] = 0;                                  // cut earlier in this call
            return;
        }
    }
}

// Inserts the remaining candidates.  They are distinct sequences that the set
// does not hold, so a claimed slot is never compared: an insert takes the first
// empty slot it wins.  Each insert adds one to *dropped.  The set was at most
// half full before the batch and a batch holds at most half its slots, so
// every insert finds a slot.
__global__ void k_cut_insert(const uint32_t* rec, int64_t stride, int W, const uint32_t* perm,
                             const uint32_t* flag, int64_t n, CutSet cs, int64_t* dropped) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool added = false;
    if (i < n && flag[i]) {
        const uint32_t a = perm[i];
        const uint64_t key = rec_seq_hash(rec, stride, W, a);
        const uint64_t mask = (uint64_t)cs.slots - 1;
        uint64_t slot = key & mask;
        for (int64_t probe = 0; probe < cs.slots; ++probe, slot = (slot + 1) & mask) {
            if (cs.keys[slot] != 0) continue;
            if (atomicCAS((unsigned long long*)&cs.keys[slot], 0ull, (unsigned long long)key) != 0ull)
                continue;
            uint32_t* w = cs.words + slot * (uint64_t)W;
            for (int q = 0; q < W; ++q) w[q] = rec[(q + 1) * stride + a];
            added = true;
            break;
        }
        if (!added) atomicOr(&cs.status[0], 1u);
    }
    const uint64_t b = __ballot(added);
    if ((threadIdx.x & 63) == 0 && b) {
        const int c = __popcll(b);
        atomicAdd((unsigned long long*)dropped, (unsigned long long)c);
        atomicAdd(&cs.status[1], (uint32_t)c);
    }
}

// Copy a pool's records into a RecBuf at offset `off`.
__global__ void k_pool_to_rec(const uint32_t* seqs, const int32_t* E, const int64_t* walker,
                              const int32_t* step, int64_t n, int W, uint32_t* rec, int64_t stride,
                              int64_t off) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    rec[off + i] = (uint32_t)E[i];
    for (int q = 1; q <= W; ++q) rec[q * stride + off + i] = seqs[i * W + (q - 1)];
    rec[(W + 1) * stride + off + i] = walker ? (uint32_t)walker[i] : 0u;
    rec[(W + 2) * stride + off + i] = step ? (uint32_t)step[i] : 0u;
}

inline unsigned blocks_for(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

}  // namespace

size_t sort_workspace_bytes(int64_t nmax, int32_t KW) {
    const int64_t nblk = (nmax + kTile - 1) / kTile;
    size_t b = 0;
    b += align_up(sizeof(uint32_t) * (size_t)nmax, 256) * 2;           // perm ping-pong
    b += align_up(sizeof(uint32_t) * 256 * (size_t)(nblk + 1), 256);  // histograms
    b += align_up(sizeof(uint32_t) * (size_t)KW, 256);                 // varying bits
    return b + 1024;
}

labs_status radix_sort_records(const RecBuf& rb, int64_t n, int32_t nkeys, void* ws, size_t ws_bytes,
                               uint32_t** perm_out, hipStream_t st) {
    if (rb.KW < 1 || rb.KW > kMaxKeyWords || nkeys > rb.KW) return invalid("record key words out of range");
    Carve cv(ws, ws_bytes);
    const int64_t nblk = (n + kTile - 1) / kTile;
    uint32_t* p0 = cv.take<uint32_t>((size_t)n);
    uint32_t* p1 = cv.take<uint32_t>((size_t)n);
    uint32_t* hist = cv.take<uint32_t>((size_t)256 * (nblk + 1));
    uint32_t* var = cv.take<uint32_t>((size_t)rb.KW);
    if (!cv.ok()) return invalid("sort workspace too small");
    *perm_out = p0;
    if (n <= 0) return LABS_OK;
    hipLaunchKernelGGL(k_iota, dim3(blocks_for(n, 256)), dim3(256), 0, st, p0, n);
    LABS_HIP(hipMemsetAsync(var, 0, sizeof(uint32_t) * rb.KW, st));
    hipLaunchKernelGGL(k_varying, dim3(blocks_for(n, 256) < 1024u ? blocks_for(n, 256) : 1024u), dim3(256), 0, st,
                       rb.rec, rb.stride, n, rb.KW, var);
    LABS_LAUNCHED("k_varying");
    uint32_t hv[kMaxKeyWords];   // host copy of the varying bits (no heap: used by the no-allocation top-k)
    LABS_HIP(hipMemcpyAsync(hv, var, sizeof(uint32_t) * rb.KW, hipMemcpyDeviceToHost, st));
    LABS_HIP(hipStreamSynchronize(st));
    uint32_t* in = p0;
    uint32_t* out = p1;
    for (int q = nkeys - 1; q >= 0; --q) {
        for (int byte = 0; byte < 4; ++byte) {
            const int shift = 8 * byte;
            if (((hv[q] >> shift) & 255u) == 0) continue;   // constant digit
            const uint32_t* kw = rb.rec + q * rb.stride;
            hipLaunchKernelGGL(k_rs_hist, dim3((unsigned)nblk), dim3(kThreads), 0, st, kw, in, n,
                               shift, hist, (int)nblk);
            hipLaunchKernelGGL(k_scan_excl, dim3(1), dim3(1024), 0, st, hist, (int64_t)256 * nblk);
            hipLaunchKernelGGL(k_rs_scatter, dim3((unsigned)nblk), dim3(kThreads), 0, st, kw, in, out,
                               n, shift, hist, (int)nblk);
            LABS_LAUNCHED("radix pass");
            uint32_t* t = in;
            in = out;
            out = t;
        }
    }
    *perm_out = in;
    return LABS_OK;
}

// ---------------------------------------------------------------- pool compaction
size_t compact_workspace_bytes(int64_t nmax, int32_t KW) {
    size_t b = sort_workspace_bytes(nmax, KW);
    b += align_up(sizeof(uint32_t) * (size_t)nmax, 256) * 2;  // flags, positions
    b += align_up(sizeof(uint32_t) * (size_t)(nmax / 1024 + 2), 256) * 2;
    b += 1024;
    return b;
}

int64_t cutset_slots(int64_t cap, int64_t staged) {
    int64_t s = 1 << 12;
    while (s < 2 * (cap + staged)) s <<= 1;
    return s;
}

size_t cutset_bytes(int64_t slots, int32_t W) {
    return align_up(sizeof(uint64_t) * (size_t)slots, 256) +
           align_up(sizeof(uint32_t) * (size_t)slots * (size_t)W, 256) + 256 + 256;
}

CutSet cutset_carve(Carve& cv, int64_t slots, int32_t W) {
    CutSet cs;
    cs.keys = cv.take<uint64_t>((size_t)slots);
    cs.words = cv.take<uint32_t>((size_t)slots * (size_t)W);
    cs.status = cv.take<uint32_t>(2);
    cs.slots = slots;
    return cs;
}

labs_status cutset_clear(const CutSet& cs, hipStream_t st) {
    LABS_HIP(hipMemsetAsync(cs.keys, 0, sizeof(uint64_t) * (size_t)cs.slots, st));
    LABS_HIP(hipMemsetAsync(cs.status, 0, sizeof(uint32_t) * 2, st));
    return LABS_OK;
}

labs_status compact_records(const RecBuf& rb, int32_t W, int64_t n, int64_t cap, uint32_t* out_seqs,
                            int32_t* out_E, int64_t* out_walker, int32_t* out_step, int64_t* count,
                            int64_t* dropped, int64_t* out_n, const CutSet* cut, void* ws,
                            size_t ws_bytes, hipStream_t st) {
    Carve cv(ws, ws_bytes);
    const size_t sort_bytes = sort_workspace_bytes(n > 0 ? n : 1, rb.KW);
    void* sort_ws = cv.take<char>(sort_bytes);
    uint32_t* flag = cv.take<uint32_t>((size_t)(n > 0 ? n : 1));
    uint32_t* pos = cv.take<uint32_t>((size_t)(n > 0 ? n : 1));
    const int64_t nb = (n + 1023) / 1024;
    uint32_t* sums = cv.take<uint32_t>((size_t)nb + 2);
    uint32_t* total = cv.take<uint32_t>(2);
    if (!cv.ok()) return invalid("compaction workspace too small");
    LABS_HIP(hipMemsetAsync(total, 0, sizeof(uint32_t) * 2, st));
    if (n > 0) {
        uint32_t* perm = nullptr;
        labs_status s = radix_sort_records(rb, n, rb.KW, sort_ws, sort_bytes, &perm, st);
        if (s != LABS_OK) return s;
        hipLaunchKernelGGL(k_unique_flags, dim3(blocks_for(n, 256)), dim3(256), 0, st, rb.rec, rb.stride,
                           W, perm, n, flag);
        LABS_HIP(hipMemcpyAsync(pos, flag, sizeof(uint32_t) * n, hipMemcpyDeviceToDevice, st));
        hipLaunchKernelGGL(k_block_sums, dim3((unsigned)nb), dim3(1024), 0, st, pos, n, sums);
        hipLaunchKernelGGL(k_scan_excl, dim3(1), dim3(1024), 0, st, sums, nb);
        hipLaunchKernelGGL(k_block_scan_apply, dim3((unsigned)nb), dim3(1024), 0, st, pos, n, sums, total);
        hipLaunchKernelGGL(k_gather_unique, dim3(blocks_for(n, 256)), dim3(256), 0, st, rb.rec, rb.stride,
                           W, perm, flag, pos, n, cap, out_seqs, out_E, out_walker, out_step);
        LABS_LAUNCHED("pool compaction");
        if (cut && dropped && n > cap) {
            hipLaunchKernelGGL(k_cut_lookup, dim3(blocks_for(n, 256)), dim3(256), 0, st, rb.rec, rb.stride,
                               W, perm, flag, pos, n, cap, *cut);
            hipLaunchKernelGGL(k_cut_insert, dim3(blocks_for(n, 256)), dim3(256), 0, st, rb.rec, rb.stride,
                               W, perm, flag, n, *cut, dropped);
            LABS_LAUNCHED("cut set");
        }
    }
    hipLaunchKernelGGL(k_finish_counts, dim3(1), dim3(64), 0, st, total, cap, count,
                       cut ? nullptr : dropped, out_n);
    LABS_LAUNCHED("k_finish_counts");
    return LABS_OK;
}

labs_status pool_to_rec(const labs_pool& pool, int64_t n, int32_t W, const RecBuf& rb, int64_t off,
                        hipStream_t st) {
    if (n <= 0) return LABS_OK;
    hipLaunchKernelGGL(k_pool_to_rec, dim3(blocks_for(n, 256)), dim3(256), 0, st, pool.seqs, pool.E,
                       pool.walker, pool.step, n, W, rb.rec, rb.stride, off);
    LABS_LAUNCHED("k_pool_to_rec");
    return LABS_OK;
}

}  // namespace labsdev
