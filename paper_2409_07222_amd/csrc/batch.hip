// Batched first step over uneven lengths: one hipGraph-captured launch in which
// persistent walker kernels (one per shape class) drain a queue of
// (configuration, walker) items, longest lengths first; plus the autotuner that
// picks each shape class's tile (slots scanned per pass, resident waves per SIMD).
#include "walk_impl.h"

#include <algorithm>
#include <climits>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

namespace labsdev {

namespace {

struct Tile {
    int RB;        // slots per pass
    int waves;     // resident waves per SIMD requested for persistent launches
    double ms;     // measured time of the winning trial (0 when untuned)
};

std::mutex g_mu;
std::map<std::pair<int, int>, Tile> g_tiles;   // (NW, R) -> tile

struct Shape {
    int NW, R;
};

Shape shape_of(int L, int p) {
    const int k = (L - 1) / 2;
    Shape s;
    s.NW = (k + 31) / 32;
    s.R = (k + 1 - p + 63) / 64;
    WalkKernels wk;
    if (walk_kernels_lookup(s.NW, s.R, s.R, &wk)) s.R = wk.R;   // instantiated R
    return s;
}

// The untuned slot tile of a shape: all R slot groups in one pass, unless that
// kernel keeps at most three waves per SIMD resident and the half tile keeps more
// (the half tile ballots the planes twice per step, which the extra wave more than
// pays for there: L = 409, p = 12, three against four waves: 1.30 -> 1.34e11
// flip-evals/s; where both keep three, at L = 451, 501 and 527, or the full tile
// keeps four, at L = 387, the full tile is faster).
std::map<std::pair<int, int>, int> g_default_rb;   // guarded by g_mu

int default_rb(const Shape& s) {
    const int half = (s.R + 1) / 2;
    if (half == s.R) return s.R;
    WalkKernels full, hk;
    if (!walk_kernels_lookup(s.NW, s.R, s.R, &full) || !walk_kernels_lookup(s.NW, s.R, half, &hk) ||
        full.RB != s.R || hk.RB != half)
        return s.R;
    int bf = 0, bh = 0;   // resident one-wave workgroups per CU (four SIMDs)
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&bf, (const void*)full.plain, 64, 0) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&bh, (const void*)hk.plain, 64, 0) != hipSuccess)
        return s.R;
    return (bf <= 12 && bh > bf) ? half : s.R;
}

Tile tile_for(const Shape& s) {
    std::lock_guard<std::mutex> g(g_mu);
    auto it = g_tiles.find({s.NW, s.R});
    if (it != g_tiles.end()) return it->second;
    auto d = g_default_rb.find({s.NW, s.R});
    if (d == g_default_rb.end()) d = g_default_rb.emplace(std::make_pair(s.NW, s.R), default_rb(s)).first;
    return Tile{d->second, 2, 0.0};
}

int cu_count() {
    static int n = 0;
    if (!n) {
        int dev = 0;
        hipGetDevice(&dev);
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0)
            n = 256;
    }
    return n;
}

__global__ void k_zero_u32(unsigned* p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

__global__ void k_walk_outputs_cfg(const WalkArgs* args, int c, uint32_t* final_seqs, int32_t* final_E,
                                   uint32_t* best_seqs, int32_t* best_E, int32_t* best_step,
                                   int64_t* flip_evals) {
    const WalkArgs A = args[c];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int W = A.W;
    if (i < A.n * W) {
        if (final_seqs) final_seqs[i] = A.seq[i];
        if (best_seqs) best_seqs[i] = A.bestSeq[i];
    }
    if (i < A.n) {
        if (final_E) final_E[i] = A.E[i];
        if (best_E) best_E[i] = A.bestE[i];
        if (best_step) best_step[i] = A.bestT[i];
    }
    if (flip_evals) {
        int64_t v = 0;
        if (i < A.n) {
            const int h = A.halted[i];
            v = (int64_t)(h ? h - 1 : A.t1) * A.nf;
        }
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        if ((threadIdx.x & 63) == 0 && v) atomicAdd((unsigned long long*)flip_evals, (unsigned long long)v);
    }
}

// ------------------------------------------------------------------ layout
struct CfgLayout {
    size_t off_seq, off_E, off_ten, off_halt, off_tabu, off_bE, off_bT, off_bS;
};

size_t state_bytes(const labs_step1_cfg& c, CfgLayout* lo, size_t base) {
    const int64_t n = c.n_walkers;
    const int W = words_of(c.L);
    const int k = (c.L - 1) / 2;
    const int nf = k + 1 - c.p;
    size_t o = base;
    auto put = [&](size_t bytes) {
        size_t at = o;
        o = align_up(o + bytes, 256);
        return at;
    };
    CfgLayout l;
    l.off_seq = put(sizeof(uint32_t) * n * W);
    l.off_E = put(sizeof(int32_t) * n);
    l.off_ten = put(sizeof(int32_t) * n);
    l.off_halt = put(sizeof(int32_t) * n);
    l.off_tabu = put(sizeof(int32_t) * n * nf);
    l.off_bE = put(sizeof(int32_t) * n);
    l.off_bT = put(sizeof(int32_t) * n);
    l.off_bS = put(sizeof(uint32_t) * n * W);
    if (lo) *lo = l;
    return o;
}

struct BatchLayout {
    std::vector<CfgLayout> cfg;
    size_t off_args, off_items, off_heads, total;
    int64_t n_items;
};

BatchLayout batch_layout(const labs_step1_cfg* c, int n) {
    BatchLayout b;
    size_t o = 0;
    b.n_items = 0;
    b.cfg.resize(n);
    for (int i = 0; i < n; ++i) {
        o = state_bytes(c[i], &b.cfg[i], o);
        b.n_items += c[i].n_walkers;
    }
    b.off_args = o;
    o = align_up(o + sizeof(WalkArgs) * n, 256);
    b.off_items = o;
    o = align_up(o + sizeof(int2) * b.n_items, 256);
    b.off_heads = o;
    o = align_up(o + sizeof(unsigned) * 64, 256);
    b.total = o + 4096;
    return b;
}

// ------------------------------------------------------------------ plans and graphs
struct ClassRun {
    walkimpl::walk_persistent_t kern;
    int offset, count;
    unsigned grid;
};

struct Plan {
    WalkArgs* args_h = nullptr;   // pinned
    int2* items_h = nullptr;      // pinned
    int n_cfg = 0;
    int64_t n_items = 0;
    std::vector<ClassRun> classes;
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
};

std::mutex g_plan_mu;
std::map<std::string, Plan*> g_plans;

// A private stream used only to record graphs (capture executes nothing, and the
// caller's stream may be the legacy default stream, which cannot be captured).
hipStream_t capture_stream() {
    static hipStream_t cs = nullptr;
    if (!cs && hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) cs = nullptr;
    return cs;
}

std::string plan_key(const labs_step1_cfg* c, int n, const labs_step1_out* o, const void* ws, size_t wsb,
                     const std::vector<Tile>& tiles) {
    std::string k;
    k.append((const char*)c, sizeof(labs_step1_cfg) * n);
    k.append((const char*)o, sizeof(labs_step1_out) * n);
    k.append((const char*)&ws, sizeof(ws));
    k.append((const char*)&wsb, sizeof(wsb));
    for (const Tile& t : tiles) {
        k.append((const char*)&t.RB, sizeof(int));
        k.append((const char*)&t.waves, sizeof(int));
    }
    return k;
}

void free_plan(Plan* p) {
    if (!p) return;
    if (p->exec) hipGraphExecDestroy(p->exec);
    if (p->graph) hipGraphDestroy(p->graph);
    if (p->args_h) hipHostFree(p->args_h);
    if (p->items_h) hipHostFree(p->items_h);
    delete p;
}

// Builds the items (longest work first) and per-class persistent launches.
labs_status build_plan(const labs_step1_cfg* c, int n, const labs_step1_out* outs, void* ws,
                       const BatchLayout& bl, const Tile* tile_override, Plan* P) {
    char* base = (char*)ws;
    P->n_cfg = n;
    P->n_items = bl.n_items;
    LABS_HIP(hipHostMalloc((void**)&P->args_h, sizeof(WalkArgs) * n, hipHostMallocDefault));
    LABS_HIP(hipHostMalloc((void**)&P->items_h, sizeof(int2) * (bl.n_items ? bl.n_items : 1),
                           hipHostMallocDefault));
    std::map<std::pair<int, int>, std::vector<int>> byshape;
    for (int i = 0; i < n; ++i) {
        const labs_step1_cfg& ci = c[i];
        const int L = ci.L, k = (L - 1) / 2;
        WalkArgs& A = P->args_h[i];
        std::memset(&A, 0, sizeof(A));
        A.L = L;
        A.p = ci.p;
        A.k = k;
        A.nf = k + 1 - ci.p;
        A.W = words_of(L);
        A.steps_total = ci.steps ? ci.steps : 4 * (L + 1);
        A.t0 = 0;
        A.t1 = A.steps_total;
        A.n = ci.n_walkers;
        A.walker_begin = ci.walker_begin;
        A.seed = ci.seed;
        A.tenure_lo = ci.tenure_lo;
        A.tenure_hi = ci.tenure_hi;
        const CfgLayout& l = bl.cfg[i];
        A.seq = (uint32_t*)(base + l.off_seq);
        A.E = (int32_t*)(base + l.off_E);
        A.tenure = (int32_t*)(base + l.off_ten);
        A.halted = (int32_t*)(base + l.off_halt);
        A.tabu = (int32_t*)(base + l.off_tabu);
        A.bestE = (int32_t*)(base + l.off_bE);
        A.bestT = (int32_t*)(base + l.off_bT);
        A.bestSeq = (uint32_t*)(base + l.off_bS);
        A.traj = outs[i].traj_E;
        A.e_max = -1;
        if (labs_status st_ = set_stamps(A, outs[i])) return st_;
        const Shape sh = shape_of(L, ci.p);
        byshape[{sh.NW, sh.R}].push_back(i);
    }
    // classes in order of decreasing per-walker cost; inside a class, longest L first
    std::vector<std::pair<double, std::pair<int, int>>> order;
    for (auto& kv : byshape) {
        double cost = 0;
        for (int i : kv.second) {
            const double w = (double)P->args_h[i].steps_total * P->args_h[i].nf * (kv.first.first + 1);
            cost = std::max(cost, w);
        }
        order.push_back({-cost, kv.first});
    }
    std::sort(order.begin(), order.end());
    int64_t at = 0;
    const int cus = cu_count();
    for (auto& oc : order) {
        std::vector<int>& cl = byshape[oc.second];
        std::sort(cl.begin(), cl.end(), [&](int a, int b) {
            const double wa = (double)P->args_h[a].steps_total * P->args_h[a].nf;
            const double wb = (double)P->args_h[b].steps_total * P->args_h[b].nf;
            return wa > wb;
        });
        const Shape sh{oc.second.first, oc.second.second};
        const Tile t = tile_override ? *tile_override : tile_for(sh);
        WalkKernels wk;
        if (!walk_kernels_lookup(sh.NW, sh.R, t.RB, &wk)) return invalid("no walker kernel for shape");
        ClassRun run;
        run.kern = wk.persistent;
        run.offset = (int)at;
        int64_t cnt = 0;
        for (int i : cl)
            for (int64_t j = 0; j < c[i].n_walkers; ++j) {
                P->items_h[at + cnt] = make_int2(i, (int)j);
                ++cnt;
            }
        run.count = (int)cnt;
        const int64_t want = (int64_t)cus * 4 * (t.waves > 0 ? t.waves : 2);
        run.grid = (unsigned)std::min<int64_t>(want, cnt > 0 ? cnt : 1);
        P->classes.push_back(run);
        at += cnt;
    }
    return LABS_OK;
}

labs_status enqueue_plan(const Plan* P, const labs_step1_out* outs, char* base, const BatchLayout& bl,
                         hipStream_t st) {
    WalkArgs* args_d = (WalkArgs*)(base + bl.off_args);
    int2* items_d = (int2*)(base + bl.off_items);
    unsigned* heads = (unsigned*)(base + bl.off_heads);
    LABS_HIP(hipMemcpyAsync(args_d, P->args_h, sizeof(WalkArgs) * P->n_cfg, hipMemcpyHostToDevice, st));
    LABS_HIP(hipMemcpyAsync(items_d, P->items_h, sizeof(int2) * P->n_items, hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, st, heads, 64);
    labs_status s = launch_walker_init_items(args_d, items_d, (int)P->n_items, st);
    if (s != LABS_OK) return s;
    for (size_t q = 0; q < P->classes.size() && q < 64; ++q) {
        const ClassRun& r = P->classes[q];
        hipLaunchKernelGGL(r.kern, dim3(r.grid), dim3(64), 0, st, (const WalkArgs*)args_d,
                           (const int2*)(items_d + r.offset), r.count, heads + q);
    }
    for (int i = 0; i < P->n_cfg; ++i) {
        const WalkArgs& A = P->args_h[i];
        const int64_t total = A.n * A.W > A.n ? A.n * A.W : A.n;
        hipLaunchKernelGGL(k_walk_outputs_cfg, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st,
                           (const WalkArgs*)args_d, i, outs[i].final_seqs, outs[i].final_E,
                           outs[i].best_seqs, outs[i].best_E, outs[i].best_step, outs[i].flip_evals);
    }
    LABS_LAUNCHED("batched walk");
    return LABS_OK;
}

}  // namespace

int walk_tile_rb(int L, int p, int R) {
    const Shape sh = shape_of(L, p);
    if (sh.R != R) return R;
    return tile_for(sh).RB;
}

size_t batch_workspace_bytes(const labs_step1_cfg* c, int n) { return batch_layout(c, n).total; }

labs_status batch_walk(const labs_step1_cfg* c, int n, const labs_step1_out* outs, void* ws, size_t wsb,
                       hipStream_t st, const void* tile_override_ptr, bool use_graph) {
    const BatchLayout bl = batch_layout(c, n);
    if (wsb < bl.total) {
        set_error("workspace needs %zu bytes, got %zu", bl.total, wsb);
        return LABS_E_NOMEM;
    }
    if (bl.n_items > INT32_MAX) return invalid("too many walkers in one batch");
    const Tile* ovr = (const Tile*)tile_override_ptr;
    std::vector<Tile> tiles;
    for (int i = 0; i < n; ++i) tiles.push_back(ovr ? *ovr : tile_for(shape_of(c[i].L, c[i].p)));
    labs_status s;
    if (!use_graph) {
        Plan P;
        s = build_plan(c, n, outs, ws, bl, ovr, &P);
        if (s == LABS_OK) s = enqueue_plan(&P, outs, (char*)ws, bl, st);
        // pinned buffers must outlive the copies
        if (s == LABS_OK) LABS_HIP(hipStreamSynchronize(st));
        if (P.args_h) hipHostFree(P.args_h);
        if (P.items_h) hipHostFree(P.items_h);
        P.args_h = nullptr;
        P.items_h = nullptr;
        return s;
    }
    const std::string key = plan_key(c, n, outs, ws, wsb, tiles);
    std::lock_guard<std::mutex> g(g_plan_mu);
    auto it = g_plans.find(key);
    Plan* P = nullptr;
    if (it != g_plans.end()) {
        P = it->second;
    } else {
        P = new Plan();
        s = build_plan(c, n, outs, ws, bl, ovr, P);
        if (s != LABS_OK) {
            free_plan(P);
            return s;
        }
        hipStream_t cs = capture_stream();
        if (!cs) {
            free_plan(P);
            return invalid("cannot create the graph capture stream");
        }
        hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) {
            free_plan(P);
            return device_error(e, "hipStreamBeginCapture");
        }
        s = enqueue_plan(P, outs, (char*)ws, bl, cs);
        hipGraph_t graph = nullptr;
        e = hipStreamEndCapture(cs, &graph);
        if (s != LABS_OK || e != hipSuccess) {
            if (graph) hipGraphDestroy(graph);
            free_plan(P);
            return s != LABS_OK ? s : device_error(e, "hipStreamEndCapture");
        }
        P->graph = graph;
        e = hipGraphInstantiate(&P->exec, graph, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            free_plan(P);
            return device_error(e, "hipGraphInstantiate");
        }
        if (g_plans.size() >= 16) {
            free_plan(g_plans.begin()->second);
            g_plans.erase(g_plans.begin());
        }
        g_plans[key] = P;
    }
    LABS_HIP(hipGraphLaunch(P->exec, st));
    return LABS_OK;
}

// ------------------------------------------------------------------ autotuner
labs_status autotune_step1(const int32_t* Ls, int n_L, int p, int walkers, int steps, hipStream_t st) {
    std::map<std::pair<int, int>, int> rep;   // shape -> largest L
    for (int i = 0; i < n_L; ++i) {
        const Shape sh = shape_of(Ls[i], p);
        auto& v = rep[{sh.NW, sh.R}];
        v = std::max(v, (int)Ls[i]);
    }
    for (auto& kv : rep) {
        const int L = kv.second;
        const Shape sh{kv.first.first, kv.first.second};
        labs_step1_cfg c{};
        c.L = L;
        c.p = p;
        c.steps = steps;
        c.tenure_lo = L / 10;
        c.tenure_hi = L / 5;
        const int nf = (L - 1) / 2 + 1 - p;
        if (c.tenure_hi >= nf) c.tenure_hi = nf - 1;
        if (c.tenure_lo > c.tenure_hi) c.tenure_lo = c.tenure_hi;
        c.e_max = -1;
        c.n_walkers = walkers;
        c.seed = 12345;
        const BatchLayout bl = batch_layout(&c, 1);
        const int W = words_of(L);
        void* ws = nullptr;
        void* fin = nullptr;
        LABS_HIP(hipMalloc(&ws, bl.total));
        hipError_t e = hipMalloc(&fin, (size_t)walkers * (W + 1) * 4);
        if (e != hipSuccess) {
            hipFree(ws);
            return device_error(e, "hipMalloc");
        }
        labs_step1_out o{};
        o.final_seqs = (uint32_t*)fin;
        o.final_E = (int32_t*)fin + (size_t)walkers * W;
        std::vector<int> rbs = {sh.R};
        if ((sh.R + 1) / 2 != sh.R) rbs.push_back((sh.R + 1) / 2);
        Tile best{sh.R, 2, 1e30};
        hipEvent_t a, b;
        hipEventCreate(&a);
        hipEventCreate(&b);
        labs_status s = LABS_OK;
        for (int rb : rbs)
            for (int waves : {1, 2, 3, 4, 8}) {
                Tile t{rb, waves, 0};
                s = batch_walk(&c, 1, &o, ws, bl.total, st, &t, false);   // warm-up
                if (s != LABS_OK) break;
                hipEventRecord(a, st);
                s = batch_walk(&c, 1, &o, ws, bl.total, st, &t, false);
                hipEventRecord(b, st);
                if (s != LABS_OK) break;
                hipEventSynchronize(b);
                float ms = 0;
                hipEventElapsedTime(&ms, a, b);
                if (ms < best.ms) best = Tile{rb, waves, ms};
            }
        hipEventDestroy(a);
        hipEventDestroy(b);
        hipFree(ws);
        hipFree(fin);
        if (s != LABS_OK) return s;
        std::lock_guard<std::mutex> g(g_mu);
        g_tiles[kv.first] = best;
    }
    return LABS_OK;
}

labs_status autotune_save(const char* path) {
    std::lock_guard<std::mutex> g(g_mu);
    FILE* f = fopen(path, "w");
    if (!f) return invalid("cannot write %s", path);
    fprintf(f, "{\"walker_tiles\": [");
    bool first = true;
    for (auto& kv : g_tiles) {
        fprintf(f, "%s\n  {\"NW\": %d, \"R\": %d, \"RB\": %d, \"waves_per_simd\": %d, \"trial_ms\": %.4f}",
                first ? "" : ",", kv.first.first, kv.first.second, kv.second.RB, kv.second.waves, kv.second.ms);
        first = false;
    }
    fprintf(f, "\n]}\n");
    fclose(f);
    return LABS_OK;
}

labs_status autotune_load(const char* path) {
    FILE* f = fopen(path, "r");
    if (!f) return invalid("cannot read %s", path);
    std::string txt;
    char buf[4096];
    size_t n;
    while ((n = fread(buf, 1, sizeof buf, f)) > 0) txt.append(buf, n);
    fclose(f);
    std::map<std::pair<int, int>, Tile> tiles;
    size_t pos = 0;
    while ((pos = txt.find("{\"NW\"", pos)) != std::string::npos) {
        int nw, r, rb, waves;
        double ms = 0;
        if (sscanf(txt.c_str() + pos, "{\"NW\": %d, \"R\": %d, \"RB\": %d, \"waves_per_simd\": %d, \"trial_ms\": %lf",
                   &nw, &r, &rb, &waves, &ms) < 4)
            return invalid("malformed tile table %s", path);
        WalkKernels wk;
        if (!walk_kernels_lookup(nw, r, rb, &wk) || wk.RB != rb || waves < 1 || waves > 8)
            return invalid("tile table %s names an unsupported tile", path);
        tiles[{nw, r}] = Tile{rb, waves, ms};
        ++pos;
    }
    std::lock_guard<std::mutex> g(g_mu);
    for (auto& kv : tiles) g_tiles[kv.first] = kv.second;
    return LABS_OK;
}

labs_status autotune_get(int L, int p, int* rb, int* waves) {
    const Shape sh = shape_of(L, p);
    const Tile t = tile_for(sh);
    *rb = t.RB;
    *waves = t.waves;
    return LABS_OK;
}

}  // namespace labsdev
