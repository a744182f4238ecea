// Energies and exact neighbour energy changes (Sec. 1 definitions; the
// neighbourhoods of Algorithm 1 and Algorithm 2).
//
// One wavefront per sequence.  The sequence is unpacked into a zero-padded
// int8 array in LDS, so s_x reads as 0 outside 1..L and range tests vanish.
#include "labs_internal.h"

namespace labsdev {

namespace {

constexpr int kMaxL = 1023;
constexpr int kPad = 1024;                 // s_x for x in [1-kPad, L+kPad] is addressable
constexpr int kSv = kMaxL + 2 * kPad + 2;

__device__ __forceinline__ void unpack_to_lds(const uint32_t* w, int L, int8_t* sv, int lane) {
    for (int i = lane; i < kSv; i += 64) sv[i] = 0;
    __syncthreads();
    for (int x = 1 + lane; x <= L; x += 64) sv[kPad + x] = packed_bit(w, x) ? 1 : -1;
    __syncthreads();
}

// C_d = sum_{i=1}^{L-d} s_i s_{i+d}
__device__ __forceinline__ int autocorr_lds(const int8_t* sv, int L, int d) {
    int c = 0;
    for (int i = 1; i <= L - d; ++i) c += (int)sv[kPad + i] * (int)sv[kPad + i + d];
    return c;
}

__global__ __launch_bounds__(64) void k_energy(int L, int64_t n, const uint32_t* __restrict__ seqs,
                                               int32_t* __restrict__ E, int32_t* __restrict__ C) {
    __shared__ int8_t sv[kSv];
    const int64_t j = blockIdx.x;
    const int lane = threadIdx.x;
    const int W = (L + 31) >> 5;
    unpack_to_lds(seqs + j * W, L, sv, lane);
    int e = 0;
    for (int d = 1 + lane; d <= L - 1; d += 64) {
        int c = autocorr_lds(sv, L, d);
        if (C) C[j * (L - 1) + (d - 1)] = c;
        e += c * c;
    }
    e = __ockl_wfred_add_i32(e);
    if (lane == 0) E[j] = e;
}

// dE for flipping the set {a, b} (b == a: a single flip), exact for any S:
//   dC_d = -2 s_a t_{a,d} - 2 s_b t_{b,d} + 4 s_a s_b [d == |b-a|],  t_{x,d} = s_{x+d} + s_{x-d}
//   dE   = sum_d dC_d (2 C_d + dC_d)
__device__ __forceinline__ int pair_delta(const int8_t* sv, const int* Cl, int L, int a, int b) {
    const int sa = sv[kPad + a];
    int acc = 0;
    if (a == b) {
        for (int d = 1; d <= L - 1; ++d) {
            int t = sv[kPad + a + d] + sv[kPad + a - d];
            int dc = -2 * sa * t;
            acc += dc * (2 * Cl[d] + dc);
        }
    } else {
        const int sb = sv[kPad + b];
        const int gap = b > a ? b - a : a - b;
        for (int d = 1; d <= L - 1; ++d) {
            int ta = sv[kPad + a + d] + sv[kPad + a - d];
            int tb = sv[kPad + b + d] + sv[kPad + b - d];
            int dc = -2 * sa * ta - 2 * sb * tb + (d == gap ? 4 * sa * sb : 0);
            acc += dc * (2 * Cl[d] + dc);
        }
    }
    return acc;
}

__global__ __launch_bounds__(64) void k_flip_deltas(int L, int p, int skew, int64_t n,
                                                    const uint32_t* __restrict__ seqs,
                                                    int32_t* __restrict__ dE) {
    __shared__ int8_t sv[kSv];
    __shared__ int Cl[kMaxL + 1];
    const int64_t j = blockIdx.x;
    const int lane = threadIdx.x;
    const int W = (L + 31) >> 5;
    unpack_to_lds(seqs + j * W, L, sv, lane);
    for (int d = 1 + lane; d <= L - 1; d += 64) Cl[d] = autocorr_lds(sv, L, d);
    __syncthreads();
    if (!skew) {
        for (int i = 1 + lane; i <= L; i += 64) dE[j * L + (i - 1)] = pair_delta(sv, Cl, L, i, i);
    } else {
        const int k = (L - 1) / 2;
        const int nf = k + 1 - p;
        for (int a = p + 1 + lane; a <= k + 1; a += 64)
            dE[j * nf + (a - p - 1)] = pair_delta(sv, Cl, L, a, L + 1 - a);
    }
}

}  // namespace

labs_status launch_energy(int32_t L, int64_t n, const uint32_t* seqs, int32_t* E, int32_t* C,
                          hipStream_t st) {
    if (n == 0) return LABS_OK;
    hipLaunchKernelGGL(k_energy, dim3((unsigned)n), dim3(64), 0, st, L, n, seqs, E, C);
    LABS_LAUNCHED("k_energy");
    return LABS_OK;
}

labs_status launch_flip_deltas(int32_t L, int32_t p, int32_t skew, int64_t n,
                               const uint32_t* seqs, int32_t* dE, hipStream_t st) {
    if (n == 0) return LABS_OK;
    hipLaunchKernelGGL(k_flip_deltas, dim3((unsigned)n), dim3(64), 0, st, L, p, skew, n, seqs, dE);
    LABS_LAUNCHED("k_flip_deltas");
    return LABS_OK;
}

}  // namespace labsdev
