// labs_pool_topk_noalloc: the pool top-k for callers that cannot allocate device
// memory (code under stream capture, tight serving loops, harnesses that forbid
// allocation).  It runs the same kernels as labs_pool_topk; their scratch (the
// sort records, permutations, histograms, flags and positions) lives in a
// fixed device array of this file instead of a caller workspace.
#include "labs_internal.h"

#include <mutex>

namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;   // 64 MiB per device
constexpr int kMaxDevices = 64;

// Host code must not pass this name to a kernel or a copy: it is a host-side
// stand-in.  Its device address per GPU comes from hipGetSymbolAddress below.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void* g_ptr[kMaxDevices];   // device address of `scratch` per device (null until looked up)

// Address of `scratch` on the current device, looked up once per device.
labs_status scratch_ptr(void** out) {
    int dev = -1;
    LABS_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return labsdev::invalid("device index %d out of range", dev);
    std::lock_guard<std::mutex> g(g_mu);
    if (!g_ptr[dev]) {
        void* p = nullptr;
        LABS_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return labsdev::invalid("no device address for the scratch array");
        g_ptr[dev] = p;
    }
    *out = g_ptr[dev];
    return LABS_OK;
}

}  // namespace

using namespace labsdev;

extern "C" labs_status labs_pool_topk_noalloc(const labs_pool* pool, int32_t L, int32_t k, uint32_t* out_seqs,
                                              int32_t* out_E, int64_t* out_n, void* stream) {
    clear_error();
    if (!pool || !pool->count) return invalid("pool and pool->count must not be NULL");
    if (L < 1 || L > 1023) return invalid("L must be in [1, 1023]");
    if (k < 1) return invalid("k must be >= 1");
    if (!out_seqs || !out_E || !out_n) return invalid("outputs must not be NULL");
    if (pool->capacity < 0 || pool->capacity > (int64_t)INT32_MAX) return invalid("capacity out of range");
    void* base = nullptr;
    labs_status s = scratch_ptr(&base);
    if (s != LABS_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    int64_t n = 0;
    LABS_HIP(hipMemcpyAsync(&n, pool->count, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    LABS_HIP(hipStreamSynchronize(st));
    if (n < 0 || n > pool->capacity) return invalid("pool count %lld out of range", (long long)n);
    if (n > 0 && (!pool->seqs || !pool->E)) return invalid("pool seqs and E must not be NULL");
    const int32_t W = words_of(L);
    const int32_t KW = W + 3;
    const int64_t stride = n > 0 ? n : 1;
    const size_t cws_bytes = compact_workspace_bytes(stride, KW);
    const size_t need = align_up(sizeof(uint32_t) * (size_t)KW * (size_t)stride, 256) + cws_bytes + 4096;
    if (need > kScratchBytes)
        return invalid("a pool of %lld entries at L=%d needs %zu bytes of scratch; the no-allocation "
                       "top-k holds %zu",
                       (long long)n, L, need, kScratchBytes);
    Carve cv(base, kScratchBytes);
    RecBuf rb;
    rb.KW = KW;
    rb.stride = stride;
    rb.rec = cv.take<uint32_t>((size_t)KW * (size_t)stride);
    void* cws = cv.take<char>(cws_bytes);
    if (!cv.ok()) return invalid("scratch layout overflow");
    if ((s = pool_to_rec(*pool, n, W, rb, 0, st)) != LABS_OK) return s;
    return compact_records(rb, W, n, k, out_seqs, out_E, nullptr, nullptr, nullptr, nullptr, out_n, nullptr,
                           cws, cws_bytes, st);
}
