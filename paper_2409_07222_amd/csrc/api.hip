// Host side of the C ABI (include/labs.h): validation, workspace layout and
// orchestration.  Every computation is enqueued on the caller's stream.
#include "labs_internal.h"

#include <climits>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

namespace labsdev {

namespace {
thread_local std::string g_err;
}

void set_error(const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
}
void clear_error() { g_err.clear(); }
labs_status invalid(const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return LABS_E_INVALID;
}
labs_status device_error(hipError_t e, const char* what) {
    set_error("%s: %s", what, hipGetErrorString(e));
    return LABS_E_DEVICE;
}
const char* last_error() { return g_err.c_str(); }

}  // namespace labsdev

using namespace labsdev;

namespace {

// ---------------------------------------------------------------- launch timing
struct TimingTable {
    std::mutex mu;
    bool on = false;
    std::map<std::string, std::pair<double, int64_t>> acc;
};
TimingTable& timing() {
    static TimingTable t;
    return t;
}

// Brackets launches with events on their stream; flush() waits and accumulates.
class LaunchTimer {
  public:
    explicit LaunchTimer(const char* name) : name_(name), on_(false) {
        std::lock_guard<std::mutex> g(timing().mu);
        on_ = timing().on;
    }
    ~LaunchTimer() {
        for (auto& e : ev_) {
            hipEventDestroy(e.first);
            hipEventDestroy(e.second);
        }
    }
    labs_status begin(hipStream_t st) {
        if (!on_) return LABS_OK;
        hipEvent_t a, b;
        LABS_HIP(hipEventCreate(&a));
        LABS_HIP(hipEventCreate(&b));
        ev_.push_back({a, b});
        LABS_HIP(hipEventRecord(a, st));
        return LABS_OK;
    }
    labs_status end(hipStream_t st) {
        if (!on_) return LABS_OK;
        LABS_HIP(hipEventRecord(ev_.back().second, st));
        return LABS_OK;
    }
    labs_status flush() {
        if (!on_ || ev_.empty()) return LABS_OK;
        LABS_HIP(hipEventSynchronize(ev_.back().second));
        double ms = 0;
        for (auto& e : ev_) {
            float x = 0;
            LABS_HIP(hipEventElapsedTime(&x, e.first, e.second));
            ms += x;
        }
        std::lock_guard<std::mutex> g(timing().mu);
        auto& slot = timing().acc[name_];
        slot.first += ms;
        slot.second += (int64_t)ev_.size();
        for (auto& e : ev_) {
            hipEventDestroy(e.first);
            hipEventDestroy(e.second);
        }
        ev_.clear();
        return LABS_OK;
    }

  private:
    std::string name_;
    bool on_;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_;
};

constexpr int kSegMax = 4096;    // walk steps per launch without a pool
constexpr int kSegPool0 = 256;   // first segment length with a pool

hipStream_t S(void* s) { return (hipStream_t)s; }

labs_status check_step1_cfg(const labs_step1_cfg& c) {
    if (c.L < 5 || c.L > 639 || (c.L & 1) == 0)
        return invalid("first-step L must be odd in [5, 639], got %d", c.L);
    const int k = (c.L - 1) / 2;
    if (c.p < 0 || c.p > k - 1) return invalid("p must be in [0, k-1] = [0, %d], got %d", k - 1, c.p);
    const int nf = k + 1 - c.p;
    if (c.steps < 0) return invalid("steps must be >= 0");
    if (c.tenure_lo < 0 || c.tenure_hi < c.tenure_lo || c.tenure_hi >= nf)
        return invalid("tenure range must satisfy 0 <= lo <= hi < %d (free positions)", nf);
    if (c.walker_begin < 0 || c.n_walkers < 1 || c.walker_begin + c.n_walkers > (int64_t)INT32_MAX)
        return invalid("walker range must be non-empty, non-negative and below 2^31");
    if (c.flags & ~LABS_POOL_WALKER_BEST) return invalid("unknown flags 0x%x", c.flags);
    if (c.reserved != 0) return invalid("reserved must be 0");
    if (!walk_shape_supported(c.L, c.p)) return invalid("no walker kernel for L=%d p=%d", c.L, c.p);
    return LABS_OK;
}

int64_t staging_cap(const labs_step1_cfg& c) {
    int64_t s = 64 * c.n_walkers;
    if (s < (1 << 16)) s = 1 << 16;
    if (s > (1 << 22)) s = 1 << 22;
    return s;
}

bool uses_pool(const labs_step1_cfg& c) {
    return c.e_max >= 0 || (c.flags & LABS_POOL_WALKER_BEST);
}

struct WalkLayout {
    size_t state_bytes = 0;   // one contiguous block, checkpointed as a unit
    size_t off_seq = 0, off_E = 0, off_ten = 0, off_halt = 0, off_tabu = 0, off_bE = 0, off_bT = 0,
           off_bS = 0, off_zh = 0, off_bloom = 0;
    int64_t S = 0, cap = 0;
    int32_t KW = 0;
    size_t total = 0;
};

// bloom: the Bloom walk's filters and keys join the state block (no tabu table).
WalkLayout walk_layout(const labs_step1_cfg& c, int64_t pool_cap, bool pool,
                       const labs_bloom* bloom = nullptr) {
    WalkLayout lo;
    const int64_t n = c.n_walkers;
    const int W = words_of(c.L);
    const int k = (c.L - 1) / 2;
    const int nf = k + 1 - c.p;
    size_t o = 0;
    auto put = [&](size_t bytes) {
        size_t at = o;
        o = align_up(o + bytes, 256);
        return at;
    };
    lo.off_seq = put(sizeof(uint32_t) * n * W);
    lo.off_E = put(sizeof(int32_t) * n);
    lo.off_ten = put(sizeof(int32_t) * n);
    lo.off_halt = put(sizeof(int32_t) * n);
    lo.off_tabu = put(bloom ? 0 : sizeof(int32_t) * n * nf);
    lo.off_bE = put(sizeof(int32_t) * n);
    lo.off_bT = put(sizeof(int32_t) * n);
    lo.off_bS = put(sizeof(uint32_t) * n * W);
    if (bloom) {
        lo.off_zh = put(sizeof(uint64_t) * n);
        lo.off_bloom = put((size_t)n << (bloom->log2_bits - 3));
    }
    lo.state_bytes = o;
    size_t total = o;
    if (pool) {
        lo.S = staging_cap(c);
        if (lo.S < n) lo.S = n;   // room for one offer per walker
        lo.cap = pool_cap;
        lo.KW = W + 3;
        total += o;                                                           // checkpoint
        total += align_up(sizeof(uint32_t) * lo.KW * (lo.S + lo.cap), 256);   // records
        total += 512;                                                         // counters
        total += compact_workspace_bytes(lo.S + lo.cap, lo.KW);
        total += cutset_bytes(cutset_slots(lo.cap, lo.S), W);
    }
    lo.total = total + 4096;
    return lo;
}

labs_status check_pool(const labs_pool* pl) {
    if (!pl) return invalid("a pool is required when e_max >= 0 or LABS_POOL_WALKER_BEST is set");
    if (pl->capacity < 1 || pl->capacity > (int64_t)INT32_MAX)
        return invalid("pool capacity must be in [1, 2^31)");
    if (!pl->seqs || !pl->E || !pl->count || !pl->dropped)
        return invalid("pool seqs, E, count and dropped must not be NULL");
    return LABS_OK;
}

labs_status check_bloom(const labs_step1_cfg& c, const labs_bloom* b) {
    if (!b) return invalid("bloom must not be NULL");
    if (b->log2_bits < 6 || b->log2_bits > 18)
        return invalid("Bloom filter bits must be 2^6..2^18 per walker, got 2^%d", b->log2_bits);
    if (b->n_hash < 1 || b->n_hash > 16) return invalid("n_hash must be in [1, 16], got %d", b->n_hash);
    if (b->reserved[0] || b->reserved[1]) return invalid("bloom reserved fields must be 0");
    if (c.tenure_lo != 0 || c.tenure_hi != 0) return invalid("a Bloom walk takes no tenure (lo = hi = 0)");
    if ((uint64_t)c.n_walkers << (b->log2_bits - 3) > (1ull << 40))
        return invalid("Bloom filters of %lld walkers exceed 1 TiB", (long long)c.n_walkers);
    return LABS_OK;
}

// Host scalars read back between segments.
struct HostPair {
    uint32_t st_count;
    int64_t pool_count;
};

}  // namespace

namespace labsdev {
labs_status validate_step1_cfg(const labs_step1_cfg& c) { return check_step1_cfg(c); }
}  // namespace labsdev

extern "C" {

int32_t labs_abi_version(void) { return LABS_ABI_VERSION; }

const char* labs_status_str(labs_status s) {
    switch (s) {
        case LABS_OK: return "ok";
        case LABS_E_INVALID: return "invalid argument";
        case LABS_E_DEVICE: return "device error";
        case LABS_E_NOMEM: return "workspace too small";
        case LABS_E_UNSUPPORTED: return "unsupported";
        default: return "unknown status";
    }
}

const char* labs_last_error(void) { return last_error(); }

int32_t labs_words(int32_t L) { return L <= 0 ? 0 : words_of(L); }

labs_status labs_realtime_hz(int64_t* hz) {
    clear_error();
    if (!hz) return invalid("hz must not be NULL");
    int dev = 0, khz = 0;
    LABS_HIP(hipGetDevice(&dev));
    LABS_HIP(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
    if (khz <= 0) return invalid("the device reports no real-time counter rate");
    *hz = (int64_t)khz * 1000;
    return LABS_OK;
}

labs_status labs_energy(int32_t L, int64_t n, const uint32_t* seqs, int32_t* E, int32_t* C,
                        void* stream) {
    clear_error();
    if (L < 1 || L > 1023) return invalid("L must be in [1, 1023], got %d", L);
    if (n < 0 || n > (int64_t)INT32_MAX) return invalid("n must be in [0, 2^31)");
    if (n > 0 && (!seqs || !E)) return invalid("seqs and E must not be NULL");
    return launch_energy(L, n, seqs, E, L > 1 ? C : nullptr, S(stream));
}

labs_status labs_flip_deltas(int32_t L, int32_t p, int32_t skew, int64_t n, const uint32_t* seqs,
                             int32_t* dE, void* stream) {
    clear_error();
    if (L < 1 || L > 1023) return invalid("L must be in [1, 1023], got %d", L);
    if (skew != 0 && skew != 1) return invalid("skew must be 0 or 1");
    if (skew) {
        if ((L & 1) == 0 || L < 3) return invalid("skew flips need odd L >= 3");
        const int k = (L - 1) / 2;
        if (p < 0 || p > k) return invalid("p must be in [0, k]");
    }
    if (n < 0 || n > (int64_t)INT32_MAX) return invalid("n must be in [0, 2^31)");
    if (n > 0 && (!seqs || !dE)) return invalid("seqs and dE must not be NULL");
    return launch_flip_deltas(L, p, skew, n, seqs, dE, S(stream));
}

static labs_status check_batch(const labs_step1_cfg* cfg, int32_t n_cfg) {
    if (n_cfg < 2 || n_cfg > 4096) return invalid("a batch holds 2..4096 configurations");
    for (int i = 0; i < n_cfg; ++i) {
        labs_status s = check_step1_cfg(cfg[i]);
        if (s != LABS_OK) return s;
        if (cfg[i].e_max >= 0 || cfg[i].flags) return invalid("batched walks take no pool (cfg %d)", i);
    }
    return LABS_OK;
}

labs_status labs_walk_step1_workspace(const labs_step1_cfg* cfg, int32_t n_cfg, int64_t pool_capacity,
                                      size_t* bytes) {
    clear_error();
    if (!cfg || !bytes) return invalid("cfg and bytes must not be NULL");
    if (n_cfg > 1) {
        labs_status sb = check_batch(cfg, n_cfg);
        if (sb != LABS_OK) return sb;
        *bytes = batch_workspace_bytes(cfg, n_cfg);
        return LABS_OK;
    }
    if (n_cfg != 1) return invalid("n_cfg must be >= 1");
    labs_status s = check_step1_cfg(cfg[0]);
    if (s != LABS_OK) return s;
    const bool pool = uses_pool(cfg[0]);
    if (pool && (pool_capacity < 1 || pool_capacity > (int64_t)INT32_MAX))
        return invalid("pool capacity must be in [1, 2^31)");
    *bytes = walk_layout(cfg[0], pool ? pool_capacity : 0, pool).total;
    return LABS_OK;
}

}  // extern "C"

namespace {

// One configuration in segmented launches (tabu tenure, or the Bloom filter when
// `bloom` is set).
labs_status walk_single(const labs_step1_cfg& c, const labs_bloom* bloom, labs_pool* pools,
                        const labs_step1_out& o, void* ws, size_t ws_bytes, hipStream_t st) {
    labs_status s = check_step1_cfg(c);
    if (s != LABS_OK) return s;
    if (bloom && (s = check_bloom(c, bloom)) != LABS_OK) return s;
    if (!o.final_seqs || !o.final_E) return invalid("final_seqs and final_E must not be NULL");
    const bool pool = uses_pool(c);
    labs_pool pl{};
    if (pool) {
        if ((s = check_pool(pools)) != LABS_OK) return s;
        pl = pools[0];
    }
    if (!ws) return invalid("workspace must not be NULL");
    const WalkLayout lo = walk_layout(c, pool ? pl.capacity : 0, pool, bloom);
    if (ws_bytes < lo.total) {
        set_error("workspace needs %zu bytes, got %zu", lo.total, ws_bytes);
        return LABS_E_NOMEM;
    }
    const int L = c.L, k = (L - 1) / 2, W = words_of(L);
    const int steps = c.steps ? c.steps : 4 * (L + 1);
    char* base = (char*)ws;
    WalkArgs A{};
    A.L = L;
    A.p = c.p;
    A.k = k;
    A.nf = k + 1 - c.p;
    A.W = W;
    A.steps_total = steps;
    A.n = c.n_walkers;
    A.walker_begin = c.walker_begin;
    A.seed = c.seed;
    A.tenure_lo = c.tenure_lo;
    A.tenure_hi = c.tenure_hi;
    A.seq = (uint32_t*)(base + lo.off_seq);
    A.E = (int32_t*)(base + lo.off_E);
    A.tenure = (int32_t*)(base + lo.off_ten);
    A.halted = (int32_t*)(base + lo.off_halt);
    A.tabu = (int32_t*)(base + lo.off_tabu);
    A.bestE = (int32_t*)(base + lo.off_bE);
    A.bestT = (int32_t*)(base + lo.off_bT);
    A.bestSeq = (uint32_t*)(base + lo.off_bS);
    A.traj = o.traj_E;
    A.e_max = c.e_max;
    if ((s = set_stamps(A, o)) != LABS_OK) return s;
    if (bloom) {
        A.tabu = nullptr;
        A.zh = (uint64_t*)(base + lo.off_zh);
        A.bloom = (uint32_t*)(base + lo.off_bloom);
        A.bloom_log2 = bloom->log2_bits;
        A.bloom_hashes = bloom->n_hash;
    }

    if ((s = launch_walker_init(A, st)) != LABS_OK) return s;
    if (bloom && (s = launch_bloom_init(A, st)) != LABS_OK) return s;
    LaunchTimer tw(bloom ? "walk_bloom" : "walk");
    auto walk = [&]() -> labs_status {
        labs_status r;
        if ((r = tw.begin(st)) != LABS_OK) return r;
        if ((r = launch_walk(A, st)) != LABS_OK) return r;
        return tw.end(st);
    };

    if (!pool) {
        for (int t = 0; t < steps; t += kSegMax) {
            A.t0 = t;
            A.t1 = t + kSegMax < steps ? t + kSegMax : steps;
            if ((s = walk()) != LABS_OK) return s;
        }
        A.t1 = steps;
        if ((s = launch_walk_outputs(A, o, st)) != LABS_OK) return s;
        return tw.flush();
    }

    // ---- pool mode: segments, compaction after each, exact retry on overflow
    Carve cv(base + lo.state_bytes, ws_bytes - lo.state_bytes);
    char* ckpt = cv.take<char>(lo.state_bytes);
    RecBuf rb;
    rb.KW = lo.KW;
    rb.stride = lo.S + lo.cap;
    rb.rec = cv.take<uint32_t>((size_t)rb.KW * rb.stride);
    uint32_t* st_count = cv.take<uint32_t>(16);
    const size_t cws_bytes = compact_workspace_bytes(lo.S + lo.cap, lo.KW);
    void* cws = cv.take<char>(cws_bytes);
    const CutSet cut = cutset_carve(cv, cutset_slots(lo.cap, lo.S), W);
    if (!cv.ok()) return invalid("workspace layout overflow");
    A.rec = rb.rec;
    A.rec_stride = rb.stride;
    A.st_count = st_count;
    A.st_cap = (uint32_t)lo.S;
    HostPair hp{};
    auto read_counts = [&]() -> labs_status {
        LABS_HIP(hipMemcpyAsync(&hp.st_count, st_count, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
        LABS_HIP(hipMemcpyAsync(&hp.pool_count, pl.count, sizeof(int64_t), hipMemcpyDeviceToHost, st));
        LABS_HIP(hipStreamSynchronize(st));
        return LABS_OK;
    };
    // initial compaction: normalise the pool's previous contents
    LABS_HIP(hipMemsetAsync(st_count, 0, 64, st));
    if ((s = cutset_clear(cut, st)) != LABS_OK) return s;
    if ((s = read_counts()) != LABS_OK) return s;
    if (hp.pool_count < 0 || hp.pool_count > pl.capacity) return invalid("pool count out of range");
    if ((s = pool_to_rec(pl, hp.pool_count, W, rb, 0, st)) != LABS_OK) return s;
    if ((s = compact_records(rb, W, hp.pool_count, pl.capacity, pl.seqs, pl.E, pl.walker, pl.step,
                             pl.count, pl.dropped, nullptr, &cut, cws, cws_bytes, st)) != LABS_OK)
        return s;

    int seg = kSegPool0;
    int t = 0;
    while (c.e_max >= 0 && t < steps) {
        const int len = seg < steps - t ? seg : steps - t;
        LABS_HIP(hipMemcpyAsync(ckpt, base, lo.state_bytes, hipMemcpyDeviceToDevice, st));
        LABS_HIP(hipMemsetAsync(st_count, 0, sizeof(uint32_t), st));
        A.t0 = t;
        A.t1 = t + len;
        if ((s = walk()) != LABS_OK) return s;
        if ((s = read_counts()) != LABS_OK) return s;
        if (hp.st_count > (uint32_t)lo.S) {
            // staging overflowed: restore and redo the segment in halves
            LABS_HIP(hipMemcpyAsync(base, ckpt, lo.state_bytes, hipMemcpyDeviceToDevice, st));
            if (len == 1) return invalid("staging too small for one step of offers");
            seg = len / 2;
            continue;
        }
        const int64_t nst = hp.st_count;
        if ((s = pool_to_rec(pl, hp.pool_count, W, rb, nst, st)) != LABS_OK) return s;
        if ((s = compact_records(rb, W, nst + hp.pool_count, pl.capacity, pl.seqs, pl.E, pl.walker,
                                 pl.step, pl.count, pl.dropped, nullptr, &cut, cws, cws_bytes,
                                 st)) != LABS_OK)
            return s;
        t += len;
        if ((int64_t)nst < lo.S / 8 && seg < kSegMax) seg *= 2;
    }
    if (c.e_max < 0) {
        for (int tt = 0; tt < steps; tt += kSegMax) {
            A.t0 = tt;
            A.t1 = tt + kSegMax < steps ? tt + kSegMax : steps;
            if ((s = walk()) != LABS_OK) return s;
        }
    }
    if (c.flags & LABS_POOL_WALKER_BEST) {
        LABS_HIP(hipMemsetAsync(st_count, 0, sizeof(uint32_t), st));
        if ((s = launch_offer_best(A, st)) != LABS_OK) return s;
        if ((s = read_counts()) != LABS_OK) return s;
        const int64_t nst = hp.st_count;
        if ((s = pool_to_rec(pl, hp.pool_count, W, rb, nst, st)) != LABS_OK) return s;
        if ((s = compact_records(rb, W, nst + hp.pool_count, pl.capacity, pl.seqs, pl.E, pl.walker,
                                 pl.step, pl.count, pl.dropped, nullptr, &cut, cws, cws_bytes,
                                 st)) != LABS_OK)
            return s;
    }
    A.t1 = steps;
    if ((s = launch_walk_outputs(A, o, st)) != LABS_OK) return s;
    uint32_t cut_status[2] = {0, 0};
    LABS_HIP(hipMemcpyAsync(cut_status, cut.status, sizeof cut_status, hipMemcpyDeviceToHost, st));
    LABS_HIP(hipStreamSynchronize(st));
    if (cut_status[0]) {
        set_error("more than %lld distinct sequences were cut from the pool in one call: the pool "
                  "is complete but its dropped count is not exact",
                  (long long)(cut.slots >> 1));
        return LABS_E_NOMEM;
    }
    return tw.flush();
}

}  // namespace

extern "C" {

labs_status labs_walk_step1(const labs_step1_cfg* cfg, int32_t n_cfg, const void* prop,
                            labs_pool* pools, labs_step1_out* outs, void* ws, size_t ws_bytes,
                            void* stream) {
    clear_error();
    if (!cfg || !outs) return invalid("cfg and outs must not be NULL");
    if (prop) return invalid("prop must be NULL for the plain walker");
    if (n_cfg > 1) {
        labs_status sb = check_batch(cfg, n_cfg);
        if (sb != LABS_OK) return sb;
        if (pools) return invalid("batched walks take no pool");
        for (int i = 0; i < n_cfg; ++i)
            if (!outs[i].final_seqs || !outs[i].final_E) return invalid("final_seqs and final_E must not be NULL");
        if (!ws) return invalid("workspace must not be NULL");
        LaunchTimer tb("walk_batched");
        if ((sb = tb.begin(S(stream))) != LABS_OK) return sb;
        if ((sb = batch_walk(cfg, n_cfg, outs, ws, ws_bytes, S(stream), nullptr, true)) != LABS_OK) return sb;
        if ((sb = tb.end(S(stream))) != LABS_OK) return sb;
        return tb.flush();
    }
    if (n_cfg != 1) return invalid("n_cfg must be >= 1");
    return walk_single(cfg[0], nullptr, pools, outs[0], ws, ws_bytes, S(stream));
}

labs_status labs_walk_step1_bloom_workspace(const labs_step1_cfg* cfg, const labs_bloom* bloom,
                                            int64_t pool_capacity, size_t* bytes) {
    clear_error();
    if (!cfg || !bytes) return invalid("cfg and bytes must not be NULL");
    labs_status s = check_step1_cfg(*cfg);
    if (s != LABS_OK) return s;
    if ((s = check_bloom(*cfg, bloom)) != LABS_OK) return s;
    const bool pool = uses_pool(*cfg);
    if (pool && (pool_capacity < 1 || pool_capacity > (int64_t)INT32_MAX))
        return invalid("pool capacity must be in [1, 2^31)");
    *bytes = walk_layout(*cfg, pool ? pool_capacity : 0, pool, bloom).total;
    return LABS_OK;
}

labs_status labs_walk_step1_bloom(const labs_step1_cfg* cfg, const labs_bloom* bloom, labs_pool* pool,
                                  labs_step1_out* out, void* ws, size_t ws_bytes, void* stream) {
    clear_error();
    if (!cfg || !out) return invalid("cfg and out must not be NULL");
    if (!bloom) return invalid("bloom must not be NULL");
    return walk_single(*cfg, bloom, pool, *out, ws, ws_bytes, S(stream));
}

static labs_status check_step2_cfg(const labs_step2_cfg& c, int64_t n_cand) {
    if (c.L < 2 || c.L > 1023) return invalid("second-step L must be in [2, 1023], got %d", c.L);
    if (c.batch < 1 || c.batch > (1 << 20)) return invalid("batch must be in [1, 2^20]");
    if (c.T_r < 0 || c.T_r > 32 || (c.T_r > 0 && 2 * c.T_r >= c.L))
        return invalid("T_r must be in [0, 32] with 2 T_r < L, got %d", c.T_r);
    if (c.reserved != 0) return invalid("reserved must be 0");
    if (c.pq_capacity < 1 || c.pq_capacity > (int64_t)1 << 28) return invalid("pq_capacity must be in [1, 2^28]");
    if (c.max_expansions < 0 || c.max_expansions > (int64_t)1 << 30)
        return invalid("max_expansions must be in [0, 2^30]");
    if (c.T_u < 1) return invalid("T_u must be >= 1");
    if (n_cand < 1 || n_cand > (int64_t)1 << 28) return invalid("n_cand must be in [1, 2^28]");
    if (!step2_fits(c, n_cand))
        return invalid("max_expansions + pq_capacity + batch*L too large: the hash set would exceed 2^31 slots");
    return LABS_OK;
}

labs_status labs_refine_step2_workspace(const labs_step2_cfg* cfg, int64_t n_cand, size_t* bytes) {
    clear_error();
    if (!cfg || !bytes) return invalid("cfg and bytes must not be NULL");
    labs_status s = check_step2_cfg(*cfg, n_cand);
    if (s != LABS_OK) return s;
    *bytes = step2_workspace_bytes(*cfg, n_cand);
    return LABS_OK;
}

static labs_status timer_begin_cb(void* t, hipStream_t st) { return ((LaunchTimer*)t)->begin(st); }
static labs_status timer_end_cb(void* t, hipStream_t st) { return ((LaunchTimer*)t)->end(st); }

labs_status labs_refine_step2(const labs_step2_cfg* cfg, int64_t n_cand, const uint32_t* cand_seqs,
                              const labs_step2_out* out, void* ws, size_t ws_bytes, void* stream) {
    clear_error();
    if (!cfg || !out) return invalid("cfg and out must not be NULL");
    labs_status s = check_step2_cfg(*cfg, n_cand);
    if (s != LABS_OK) return s;
    if (!cand_seqs) return invalid("cand_seqs must not be NULL");
    if (!out->best_seq || !out->best_E || !out->stats) return invalid("best_seq, best_E and stats must not be NULL");
    if (out->open_capacity < 0) return invalid("open_capacity must be >= 0");
    if (!ws) return invalid("workspace must not be NULL");
    LaunchTimer te("expand");
    s = step2_run(*cfg, n_cand, cand_seqs, *out, ws, ws_bytes, S(stream), timer_begin_cb, timer_end_cb, &te);
    if (s != LABS_OK) return s;
    return te.flush();
}

labs_status labs_autotune_step1(const int32_t* Ls, int32_t n_L, int32_t p, int32_t walkers, int32_t steps,
                                void* stream) {
    clear_error();
    if (!Ls || n_L < 1) return invalid("Ls must hold at least one length");
    for (int i = 0; i < n_L; ++i) {
        labs_step1_cfg c{};
        c.L = Ls[i];
        c.p = p;
        c.steps = steps;
        c.n_walkers = walkers;
        labs_status s = check_step1_cfg(c);
        if (s != LABS_OK) return s;
    }
    if (walkers < 1 || steps < 1) return invalid("walkers and steps must be >= 1");
    return autotune_step1(Ls, n_L, p, walkers, steps, S(stream));
}

labs_status labs_autotune_save(const char* path) {
    clear_error();
    if (!path) return invalid("path must not be NULL");
    return autotune_save(path);
}

labs_status labs_autotune_load(const char* path) {
    clear_error();
    if (!path) return invalid("path must not be NULL");
    return autotune_load(path);
}

labs_status labs_autotune_get(int32_t L, int32_t p, int32_t* rb, int32_t* waves_per_simd) {
    clear_error();
    if (!rb || !waves_per_simd) return invalid("outputs must not be NULL");
    labs_step1_cfg c{};
    c.L = L;
    c.p = p;
    c.n_walkers = 1;
    labs_status s = check_step1_cfg(c);
    if (s != LABS_OK) return s;
    int a = 0, b = 0;
    autotune_get(L, p, &a, &b);
    *rb = a;
    *waves_per_simd = b;
    return LABS_OK;
}

labs_status labs_timing_enable(int32_t on) {
    clear_error();
    std::lock_guard<std::mutex> g(timing().mu);
    timing().on = on != 0;
    return LABS_OK;
}

labs_status labs_timing_reset(void) {
    clear_error();
    std::lock_guard<std::mutex> g(timing().mu);
    timing().acc.clear();
    return LABS_OK;
}

labs_status labs_timing_read(const char* kernel, double* total_ms, int64_t* launches) {
    clear_error();
    if (!kernel || !total_ms || !launches) return invalid("arguments must not be NULL");
    std::lock_guard<std::mutex> g(timing().mu);
    auto it = timing().acc.find(kernel);
    *total_ms = it == timing().acc.end() ? 0.0 : it->second.first;
    *launches = it == timing().acc.end() ? 0 : it->second.second;
    return LABS_OK;
}

labs_status labs_legendre_pairs(int32_t L, const labs_legendre_sweep* sweep, int32_t* n_out, int32_t* o_out,
                                int64_t capacity, int64_t* count) {
    clear_error();
    const labs_legendre_sweep def{0, 900, 1800, 2600};
    return legendre_pairs(L, sweep ? *sweep : def, n_out, o_out, capacity, count);
}

labs_status labs_legendre_build_workspace(int64_t n_pairs, size_t* bytes) {
    clear_error();
    if (!bytes) return invalid("bytes must not be NULL");
    if (n_pairs < 0) return invalid("n_pairs must be >= 0");
    *bytes = legendre_workspace_bytes(n_pairs);
    return LABS_OK;
}

labs_status labs_legendre_build(int32_t L, int64_t n_pairs, const int32_t* n, const int32_t* o,
                                uint32_t* seqs, int32_t* E, void* ws, size_t ws_bytes, void* stream) {
    clear_error();
    return legendre_build(L, n_pairs, n, o, seqs, E, ws, ws_bytes, S(stream));
}

labs_status labs_length_operators(int32_t L, int64_t n, const uint32_t* seqs, uint32_t* minus, int32_t* E_minus,
                                  uint32_t* plus, int32_t* E_plus, void* stream) {
    clear_error();
    return length_operators(L, n, seqs, minus, E_minus, plus, E_plus, S(stream));
}

labs_status labs_pool_topk_workspace(int64_t capacity, int32_t L, size_t* bytes) {
    clear_error();
    if (!bytes) return invalid("bytes must not be NULL");
    if (capacity < 0 || capacity > (int64_t)INT32_MAX) return invalid("capacity out of range");
    if (L < 1 || L > 1023) return invalid("L must be in [1, 1023]");
    const int32_t KW = words_of(L) + 3;
    const int64_t n = capacity > 0 ? capacity : 1;
    *bytes = align_up(sizeof(uint32_t) * KW * n, 256) + compact_workspace_bytes(n, KW) + 4096;
    return LABS_OK;
}

labs_status labs_pool_topk(const labs_pool* pool, int32_t L, int32_t k, uint32_t* out_seqs, int32_t* out_E,
                           int64_t* out_n, void* ws, size_t ws_bytes, void* stream) {
    clear_error();
    if (!pool || !pool->count) return invalid("pool and pool->count must not be NULL");
    if (L < 1 || L > 1023) return invalid("L must be in [1, 1023]");
    if (k < 1) return invalid("k must be >= 1");
    if (!out_seqs || !out_E || !out_n) return invalid("outputs must not be NULL");
    if (pool->capacity < 0 || pool->capacity > (int64_t)INT32_MAX) return invalid("capacity out of range");
    size_t need = 0;
    labs_status s = labs_pool_topk_workspace(pool->capacity, L, &need);
    if (s != LABS_OK) return s;
    if (!ws || ws_bytes < need) {
        set_error("workspace needs %zu bytes, got %zu", need, ws_bytes);
        return LABS_E_NOMEM;
    }
    hipStream_t st = S(stream);
    int64_t n = 0;
    LABS_HIP(hipMemcpyAsync(&n, pool->count, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    LABS_HIP(hipStreamSynchronize(st));
    if (n < 0 || n > pool->capacity) return invalid("pool count %lld out of range", (long long)n);
    if (n > 0 && (!pool->seqs || !pool->E)) return invalid("pool seqs and E must not be NULL");
    const int32_t W = words_of(L);
    Carve cv(ws, ws_bytes);
    RecBuf rb;
    rb.KW = W + 3;
    rb.stride = n > 0 ? n : 1;
    rb.rec = cv.take<uint32_t>((size_t)rb.KW * rb.stride);
    const size_t cws_bytes = compact_workspace_bytes(rb.stride, rb.KW);
    void* cws = cv.take<char>(cws_bytes);
    if (!cv.ok()) return invalid("workspace layout overflow");
    if ((s = pool_to_rec(*pool, n, W, rb, 0, st)) != LABS_OK) return s;
    return compact_records(rb, W, n, k, out_seqs, out_E, nullptr, nullptr, nullptr, nullptr, out_n, nullptr,
                           cws, cws_bytes, st);
}

}  // extern "C"
