// The end operators of Sec. 3 that carry the search to even lengths (and back):
// from each sequence of length L, the two of length L-1 without its first or its
// last element, and the four of length L+1 with +1 or -1 before its first or
// after its last element.  One wavefront per input sequence builds the six
// packed results; their energies follow from the energy kernel.
#include "labs_internal.h"

namespace labsdev {

namespace {

constexpr int kMaxL = 1023;

// Bit i (0-based element index, wire format: bit 31 - (i mod 32) of word i/32).
__device__ __forceinline__ uint32_t bit_at(const uint32_t* w, int i) { return (w[i >> 5] >> (31 - (i & 31))) & 1u; }

// out element i = in element i + shift (shift = +1: drop the first element; -1: a
// new first element `first`), for i < Lout; `last` (when >= 0) is element Lout-1.
__device__ __forceinline__ void shifted(const uint32_t* in, int shift, int Lout, int first, int last,
                                        uint32_t* out, int lane) {
    const int Wo = (Lout + 31) >> 5;
    for (int base = 0; base < 32 * Wo; base += 64) {
        const int i = base + lane;
        uint32_t b = 0;
        if (i < Lout) {
            const int src = i + shift;
            if (i == Lout - 1 && last >= 0) b = (uint32_t)last;
            else if (src < 0) b = (uint32_t)first;
            else b = bit_at(in, src);
        }
        const uint64_t m = __ballot(b != 0);
        if (lane == 0) {
            out[base >> 5] = __builtin_bitreverse32((uint32_t)m);
            if ((base >> 5) + 1 < Wo) out[(base >> 5) + 1] = __builtin_bitreverse32((uint32_t)(m >> 32));
        }
    }
}

__global__ __launch_bounds__(64) void k_operators(int L, const uint32_t* __restrict__ seqs,
                                                  uint32_t* __restrict__ minus, uint32_t* __restrict__ plus) {
    const int64_t j = blockIdx.x;
    const int lane = threadIdx.x;
    const int W = (L + 31) >> 5, Wm = (L - 1 + 31) >> 5, Wp = (L + 1 + 31) >> 5;
    const uint32_t* in = seqs + j * W;
    if (minus) {
        shifted(in, 1, L - 1, 0, -1, minus + (2 * j) * Wm, lane);        // without the first
        shifted(in, 0, L - 1, 0, -1, minus + (2 * j + 1) * Wm, lane);    // without the last
    }
    shifted(in, -1, L + 1, 1, -1, plus + (4 * j) * Wp, lane);            // +1 first
    shifted(in, -1, L + 1, 0, -1, plus + (4 * j + 1) * Wp, lane);        // -1 first
    shifted(in, 0, L + 1, 0, 1, plus + (4 * j + 2) * Wp, lane);          // +1 last
    shifted(in, 0, L + 1, 0, 0, plus + (4 * j + 3) * Wp, lane);          // -1 last
}

}  // namespace

labs_status length_operators(int32_t L, int64_t n, const uint32_t* seqs, uint32_t* minus, int32_t* E_minus,
                             uint32_t* plus, int32_t* E_plus, hipStream_t st) {
    if (L < 1 || L > kMaxL - 1) return invalid("length operators need L in [1, %d], got %d", kMaxL - 1, L);
    if (n < 0 || n > (int64_t)INT32_MAX / 4) return invalid("n must be in [0, 2^29)");
    if (n == 0) return LABS_OK;
    if (!seqs || !plus || !E_plus) return invalid("seqs, plus and E_plus must not be NULL");
    const bool want_minus = L >= 2;
    if (want_minus && (!minus || !E_minus)) return invalid("minus and E_minus must not be NULL for L >= 2");
    hipLaunchKernelGGL(k_operators, dim3((unsigned)n), dim3(64), 0, st, L, seqs, want_minus ? minus : nullptr,
                       plus);
    LABS_LAUNCHED("k_operators");
    labs_status s;
    if (want_minus && (s = launch_energy(L - 1, 2 * n, minus, E_minus, nullptr, st)) != LABS_OK) return s;
    return launch_energy(L + 1, 4 * n, plus, E_plus, nullptr, st);
}

}  // namespace labsdev
