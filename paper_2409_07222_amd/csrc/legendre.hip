// Legendre-construction seeds of the second step (Sec. 4.1): a Legendre
// sequence of odd prime length n, rotated by o and extended periodically to
// length L,
//   s_j = chi((j + o) mod n),  j = 0..L-1,
// chi(a) = +1 for the non-zero quadratic residues of n, -1 otherwise (chi(0) = -1).
// The sweep of (n, o) pairs is host logic; the sequences and their energies are
// built on the device, one wavefront per pair.
#include "labs_internal.h"

namespace labsdev {

namespace {

constexpr int kMaxN = 1023;

bool is_prime(int n) {
    if (n < 2) return false;
    for (int d = 2; d * d <= n; ++d)
        if (n % d == 0) return false;
    return true;
}

// The residue table of n in LDS (x^2 mod n for x = 1..(n-1)/2 covers every
// non-zero residue), then the packed sequence by one ballot per 64 elements.
__global__ __launch_bounds__(64) void k_legendre(int L, const int32_t* __restrict__ ns,
                                                 const int32_t* __restrict__ os, uint32_t* __restrict__ seqs) {
    __shared__ uint8_t res[kMaxN + 1];
    const int64_t j = blockIdx.x;
    const int lane = threadIdx.x;
    const int n = ns[j], o = os[j];
    for (int a = lane; a < n; a += 64) res[a] = 0;
    __syncthreads();
    for (int x = 1 + lane; x <= (n - 1) / 2; x += 64) res[(x * x) % n] = 1;
    __syncthreads();
    const int W = (L + 31) >> 5;
    uint32_t* out = seqs + j * W;
    for (int base = 0; base < 32 * W; base += 64) {
        const int i = base + lane;   // element index j (0-based)
        bool bit = false;
        if (i < L) {
            const int a = (i + o) % n;
            bit = res[a] != 0;
        }
        const uint64_t m = __ballot(bit);
        // wire format: element i at bit 31 - (i mod 32) of word i / 32
        if (lane == 0) {
            out[base >> 5] = __builtin_bitreverse32((uint32_t)m);
            if ((base >> 5) + 1 < W) out[(base >> 5) + 1] = __builtin_bitreverse32((uint32_t)(m >> 32));
        }
    }
}

}  // namespace

labs_status legendre_pairs(int32_t L, const labs_legendre_sweep& sw, int32_t* n_out, int32_t* o_out,
                           int64_t capacity, int64_t* count) {
    if (L < 2 || L > kMaxN) return invalid("Legendre seeds need L in [2, %d], got %d", kMaxN, L);
    if (sw.t_lo < 0 || sw.t_hi < sw.t_lo || sw.r_lo < 0 || sw.r_hi < sw.r_lo || sw.r_hi > 10000)
        return invalid("sweep ranges must satisfy 0 <= t_lo <= t_hi and 0 <= r_lo <= r_hi <= 10000");
    if (capacity < 0 || (capacity > 0 && (!n_out || !o_out)) || !count)
        return invalid("count must not be NULL, nor n_out / o_out when capacity > 0");
    int64_t c = 0;
    for (int n = 3; n <= L; ++n) {
        if (!is_prime(n)) continue;
        const int64_t app = (int64_t)(L - n) * 10000;
        if (app < (int64_t)sw.t_lo * n || app > (int64_t)sw.t_hi * n) continue;
        for (int o = 0; o < n; ++o) {
            const int64_t r = (int64_t)o * 10000;
            if (r < (int64_t)sw.r_lo * n || r > (int64_t)sw.r_hi * n) continue;
            if (c < capacity) {
                n_out[c] = n;
                o_out[c] = o;
            }
            ++c;
        }
    }
    *count = c;
    return LABS_OK;
}

size_t legendre_workspace_bytes(int64_t n_pairs) { return align_up(sizeof(int32_t) * 2 * n_pairs, 256); }

labs_status legendre_build(int32_t L, int64_t n_pairs, const int32_t* n_host, const int32_t* o_host,
                           uint32_t* seqs, int32_t* E, void* ws, size_t ws_bytes, hipStream_t st) {
    if (L < 2 || L > kMaxN) return invalid("Legendre seeds need L in [2, %d], got %d", kMaxN, L);
    if (n_pairs < 0 || n_pairs > (int64_t)INT32_MAX) return invalid("n_pairs must be in [0, 2^31)");
    if (n_pairs == 0) return LABS_OK;
    if (!n_host || !o_host || !seqs || !E || !ws) return invalid("arrays and workspace must not be NULL");
    if (ws_bytes < legendre_workspace_bytes(n_pairs)) {
        set_error("workspace needs %zu bytes, got %zu", legendre_workspace_bytes(n_pairs), ws_bytes);
        return LABS_E_NOMEM;
    }
    for (int64_t i = 0; i < n_pairs; ++i) {
        const int n = n_host[i], o = o_host[i];
        if (n < 3 || n > kMaxN || !is_prime(n)) return invalid("pair %lld: n = %d is not an odd prime <= %d",
                                                               (long long)i, n, kMaxN);
        if (o < 0 || o >= n) return invalid("pair %lld: rotation %d outside [0, %d)", (long long)i, o, n);
    }
    int32_t* dn = (int32_t*)ws;
    int32_t* dor = dn + n_pairs;
    LABS_HIP(hipMemcpyAsync(dn, n_host, sizeof(int32_t) * n_pairs, hipMemcpyHostToDevice, st));
    LABS_HIP(hipMemcpyAsync(dor, o_host, sizeof(int32_t) * n_pairs, hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_legendre, dim3((unsigned)n_pairs), dim3(64), 0, st, L, dn, dor, seqs);
    LABS_LAUNCHED("k_legendre");
    labs_status s = launch_energy(L, n_pairs, seqs, E, nullptr, st);
    if (s != LABS_OK) return s;
    // the host arrays may be released on return
    LABS_HIP(hipStreamSynchronize(st));
    return LABS_OK;
}

}  // namespace labsdev
