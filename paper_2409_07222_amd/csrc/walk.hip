// First step (Algorithm 1, with a tabu tenure or with its Bloom filter): walker
// init and the walk.
//
// One wavefront runs one walker.  Notation: L = 2k+1, even lags d = 2m,
// m = 1..K with K = k (odd-lag C vanish for skew sequences, Sec. 1).  Free
// positions a = p+1..k+1 (Eq. (3)); lane l owns a = p+1+l+64r, r = 0..R-1.
//
// Energy change of the skew flip of a (partner b = L+1-a, partner lag
// mp = (b-a)/2 = k+1-a).  Flipping a and b changes C_{2m} by -4 s_a u_m with
//   u_m = s_{a+2m}[a+2m <= L, a+2m != b] + s_{a-2m}[a-2m >= 1]
// (for even lags the partner's contribution equals a's by Eq. (2), and the
// s_a s_b product inside C_{b-a} is unchanged), so
//   dE_a = sum_m (2 C dC + dC^2) = -8 s_a G_a + 16 Q_a,
//   G_a  = sum_m C_{2m} u_m,   Q_a = sum_m u_m^2.
// The centre a = k+1 flips alone: dC_{2m} = -4 s_a s_{a-2m}.
//
// G_a is evaluated bit-sliced.  Forward/backward windows F_a, B_a hold, at bit
// m-1, the 0/1 digit of s_{a+2m} / s_{a-2m} (0 outside 1..L).  Every C_{2m} is
// odd (L - 2m terms of +-1), so with C'_m = (C_{2m} - 1)/2 and the two's-complement
// bit planes P_j of (C'_m)_m,
//   sum_m C_{2m} F_a(m) = 2 sum_j w_j popcount(P_j & F_a) + popcount(F_a),
//   w_j = 2^j (sign plane -2^j),
// and since s = 2*digit - 1 on valid lags,
//   G_a = 2 (H_f + H_b) - PC[Mf] - PC[Mb] - C_{2mp} s_b,   PC = prefix sums of C_{2m},
//   Q_a = Mf - 1 + 3 Mb - 4 popcount((F ^ B) & [m <= Mb]) - 2 [mp <= Mb] s_b s_{a-2mp},
// with Mf = (L-a)/2 and Mb = (a-1)/2 the valid forward/backward lag counts.
// The planes are built per step with one ballot per (plane, 64 lags); the
// number of planes is the bit length of max |C'_m| plus the sign, read off the
// current table each step, so the scan is exact for every state.
//
// Windows come from per-parity bit vectors of the sequence: V_pi bit j is the
// digit of position 2j+2-pi (pi = x & 1, j = (x-1)>>1), VR_pi its reversal over
// N = 32*NV bits; F_a = V_pi >> (j_a + 1), B_a = VR_pi >> (N - j_a), read with
// funnel shifts.  Backward windows never need more than NQ = ceil(NW/2) words
// because Mb <= k/2.
#include "walk_impl.h"

#include <climits>

namespace labsdev {



namespace {

}  // namespace

using namespace walkimpl;

namespace {

__device__ void walker_init_body(const WalkArgs& A, int64_t j, Lds<10>& S) {
    constexpr int NW = 10;
    const int lane = threadIdx.x;
    const int64_t w = A.walker_begin + j;
    const int L = A.L, k = A.k, p = A.p;
    const uint64_t key = walker_key(A.seed, L, w);
    if (A.start_ticks && lane == 0) atomicMin(A.start_ticks, __builtin_amdgcn_s_memrealtime());
    // s_i for i = 1..k+1 from stream outputs i-1; s_1 = +1 when p >= 1; Eq. (2) for the rest
    for (int i = lane; i < Lds<NW>::SV; i += 64) S.sv[i] = 0;
    __syncthreads();
    constexpr int PADL = Lds<NW>::PADL;
    for (int i = 1 + lane; i <= k + 1; i += 64) {
        uint64_t d = sm64_at(key, (uint64_t)(i - 1));
        int s = (d >> 63) ? 1 : -1;
        if (i == 1 && p >= 1) s = 1;
        S.sv[PADL + i] = (int8_t)s;
        if (i <= k) {
            int ii = k + 1 - i;               // s_{k+1+ii} = (-1)^ii s_{k+1-ii}
            S.sv[PADL + k + 1 + ii] = (int8_t)((ii & 1) ? -s : s);
        }
    }
    __syncthreads();
    // pack
    const int W = A.W;
    for (int base = 0; base < 32 * W; base += 64) {
        int x = base + lane + 1;
        bool bit = x <= L && S.sv[PADL + x] > 0;
        uint64_t m = __ballot(bit);
        // lane 0..31 bits map to MSB-first positions: bit (31 - (x-1)%32)
        if (lane == 0) {
            uint32_t lo = (uint32_t)m, hi = (uint32_t)(m >> 32);
            S.pk[base >> 5] = __builtin_bitreverse32(lo);
            if ((base >> 5) + 1 < W) S.pk[(base >> 5) + 1] = __builtin_bitreverse32(hi);
        }
    }
    __syncthreads();
    // energy from even lags (odd lags vanish under Eq. (2))
    int e = 0;
    for (int m = 1 + lane; m <= k; m += 64) {
        int d = 2 * m, c = 0;
        for (int i = 1; i <= L - d; ++i) c += (int)S.sv[PADL + i] * (int)S.sv[PADL + i + d];
        e += c * c;
    }
    e = __ockl_wfred_add_i32(e);
    const uint64_t span = (uint64_t)(A.tenure_hi - A.tenure_lo + 1);
    const int ten = A.tenure_lo + (int)(sm64_at(key, (uint64_t)(k + 1)) % span);
    if (lane < W) {
        A.seq[j * W + lane] = S.pk[lane];
        A.bestSeq[j * W + lane] = S.pk[lane];
    }
    if (A.tabu)   // null for Bloom-filter walks
        for (int i = lane; i < A.nf; i += 64) A.tabu[j * A.nf + i] = 0;
    if (lane == 0) {
        A.E[j] = e;
        A.tenure[j] = ten;
        A.halted[j] = 0;
        A.bestE[j] = e;
        A.bestT[j] = 0;
    }
    if (A.n_levels > 0 && e <= pending_level(A)) stamp_levels(A, e, lane);
}

__global__ __launch_bounds__(64) void k_walker_init(WalkArgs A) {
    __shared__ Lds<10> S;
    walker_init_body(A, blockIdx.x, S);
}

// Init for a batch of (configuration, walker) items.
__global__ __launch_bounds__(64) void k_walker_init_items(const WalkArgs* args, const int2* items) {
    __shared__ Lds<10> S;
    const int2 it = items[blockIdx.x];
    const WalkArgs A = args[it.x];
    walker_init_body(A, (int64_t)it.y, S);
}

// Bloom-filter walks: the key of each walker's initial sequence (Zobrist XOR over
// the +1 elements among s_1..s_{k+1}), and its filter holding only that key.
__global__ __launch_bounds__(64) void k_bloom_init(WalkArgs A) {
    const int lane = threadIdx.x;
    const int64_t j = blockIdx.x;
    const uint32_t* s = A.seq + j * A.W;
    uint64_t h = 0;
    for (int i = 1 + lane; i <= A.k + 1; i += 64)
        if (packed_bit(s, i)) h ^= zobrist_at(i - 1);
    uint32_t lo = (uint32_t)h, hi = (uint32_t)(h >> 32);
    for (int o = 32; o > 0; o >>= 1) {
        lo ^= (uint32_t)__shfl_xor((int)lo, o, 64);
        hi ^= (uint32_t)__shfl_xor((int)hi, o, 64);
    }
    h = ((uint64_t)hi << 32) | lo;
    const int nbw = 1 << (A.bloom_log2 - 5);
    const uint32_t mask = (1u << A.bloom_log2) - 1u;
    const uint32_t g2 = hi | 1u;
    uint32_t* f = A.bloom + j * (int64_t)nbw;
    for (int w = lane; w < nbw; w += 64) {
        uint32_t v = 0, x = lo;
        for (int q = 0; q < A.bloom_hashes; ++q) {
            const uint32_t b = x & mask;
            if ((int)(b >> 5) == w) v |= 1u << (b & 31);
            x += g2;
        }
        f[w] = v;
    }
    if (lane == 0) A.zh[j] = h;
}

// Offer every walker's best sequence to the staging buffer.
__global__ __launch_bounds__(64) void k_offer_best(WalkArgs A) {
    const int lane = threadIdx.x;
    const int64_t j = blockIdx.x;
    const int W = A.W;
    const int bE = A.bestE[j];
    uint32_t slot = 0;
    if (lane == 0) slot = atomicAdd(A.st_count, 1u);
    slot = __shfl(slot, 0, 64);
    if (slot < A.st_cap && lane < W + 3) {
        uint32_t v;
        if (lane == 0) v = (uint32_t)bE;
        else if (lane <= W) v = A.bestSeq[j * W + lane - 1];
        else if (lane == W + 1) v = (uint32_t)(A.walker_begin + j);
        else v = (uint32_t)A.bestT[j];
        A.rec[(int64_t)lane * A.rec_stride + slot] = v;
    }
}

__global__ void k_walk_outputs(WalkArgs A, uint32_t* final_seqs, int32_t* final_E,
                               uint32_t* best_seqs, int32_t* best_E, int32_t* best_step,
                               int64_t* flip_evals) {
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
            const int taken = h ? h - 1 : A.t1;
            v = (int64_t)taken * A.nf;
        }
        // wave sum then one atomic per wave
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        if ((threadIdx.x & 63) == 0 && v) atomicAdd((unsigned long long*)flip_evals, (unsigned long long)v);
    }
}

}  // namespace

bool walk_kernels_lookup(int NW, int R, int RB, WalkKernels* out) {
    if (NW >= 1 && NW <= 4) return walk_kernels_a(NW, R, RB, out);
    if (NW >= 5 && NW <= 7) return walk_kernels_b(NW, R, RB, out);
    if (NW >= 8 && NW <= 10) return walk_kernels_c(NW, R, RB, out);
    return false;
}

bool walk_shape_supported(int L, int p) {
    const int k = (L - 1) / 2;
    const int NW = (k + 31) / 32;
    const int R = (k + 1 - p + 63) / 64;
    WalkKernels wk;
    return walk_kernels_lookup(NW, R, R, &wk);
}

labs_status launch_walker_init_items(const WalkArgs* args, const int2* items, int n_items, hipStream_t st) {
    if (n_items <= 0) return LABS_OK;
    hipLaunchKernelGGL(k_walker_init_items, dim3((unsigned)n_items), dim3(64), 0, st, args, items);
    LABS_LAUNCHED("k_walker_init_items");
    return LABS_OK;
}

labs_status launch_walker_init(const WalkArgs& A, hipStream_t st) {
    hipLaunchKernelGGL(k_walker_init, dim3((unsigned)A.n), dim3(64), 0, st, A);
    LABS_LAUNCHED("k_walker_init");
    return LABS_OK;
}

labs_status launch_bloom_init(const WalkArgs& A, hipStream_t st) {
    hipLaunchKernelGGL(k_bloom_init, dim3((unsigned)A.n), dim3(64), 0, st, A);
    LABS_LAUNCHED("k_bloom_init");
    return LABS_OK;
}

labs_status launch_walk(const WalkArgs& A, hipStream_t st) {
    const int NW = (A.k + 31) / 32;
    const int R = (A.nf + 63) / 64;
    WalkKernels wk;
    if (!walk_kernels_lookup(NW, R, walk_tile_rb(A.L, A.p, R), &wk))
        return invalid("no walker kernel for L=%d p=%d", A.L, A.p);
    if (A.bloom) {
        const size_t lds = sizeof(uint32_t) << (A.bloom_log2 - 5);
        hipLaunchKernelGGL(wk.bloom, dim3((unsigned)A.n), dim3(64), lds, st, A);
        LABS_LAUNCHED("k_walk_bloom");
        return LABS_OK;
    }
    hipLaunchKernelGGL(wk.plain, dim3((unsigned)A.n), dim3(64), 0, st, A);
    LABS_LAUNCHED("k_walk");
    return LABS_OK;
}

labs_status launch_offer_best(const WalkArgs& A, hipStream_t st) {
    hipLaunchKernelGGL(k_offer_best, dim3((unsigned)A.n), dim3(64), 0, st, A);
    LABS_LAUNCHED("k_offer_best");
    return LABS_OK;
}

labs_status launch_walk_outputs(const WalkArgs& A, const labs_step1_out& o, hipStream_t st) {
    const int64_t total = A.n * A.W > A.n ? A.n * A.W : A.n;
    const unsigned blocks = (unsigned)((total + 255) / 256);
    hipLaunchKernelGGL(k_walk_outputs, dim3(blocks), dim3(256), 0, st, A, o.final_seqs, o.final_E,
                       o.best_seqs, o.best_E, o.best_step, o.flip_evals);
    LABS_LAUNCHED("k_walk_outputs");
    return LABS_OK;
}

}  // namespace labsdev
