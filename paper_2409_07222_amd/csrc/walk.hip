// First step (Algorithm 1 with a tabu tenure): walker init and the walk.
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
// m-1, the 0/1 digit of s_{a+2m} / s_{a-2m} (0 outside 1..L).  With the
// two's-complement bit planes P_j of the vector (C_{2m})_m,
//   sum_m C_{2m} F_a(m) = sum_j w_j popcount(P_j & F_a),  w_j = 2^j (sign plane -2^j),
// and since s = 2*digit - 1 on valid lags,
//   G_a = 2 (H_f + H_b) - PC[Mf] - PC[Mb] - C_{2mp} s_b,   PC = prefix sums of C_{2m},
//   Q_a = Mf - 1 + 3 Mb - 4 popcount((F ^ B) & [m <= Mb]) - 2 [mp <= Mb] s_b s_{a-2mp},
// with Mf = (L-a)/2 and Mb = (a-1)/2 the valid forward/backward lag counts.
// The planes are built per step with one ballot per (plane, 64 lags); the
// number of planes is the bit length of max |C_{2m}| plus the sign, read off
// the current table each step, so the scan is exact for every state.
//
// Windows come from per-parity bit vectors of the sequence: V_pi bit j is the
// digit of position 2j+2-pi (pi = x & 1, j = (x-1)>>1), VR_pi its reversal over
// N = 32*NV bits; F_a = V_pi >> (j_a + 1), B_a = VR_pi >> (N - j_a), read with
// funnel shifts.  Backward windows never need more than NQ = ceil(NW/2) words
// because Mb <= k/2.
#include "labs_internal.h"

#include <climits>

namespace labsdev {



namespace {

template <int NW>
struct Lds {
    static constexpr int K = 32 * NW;          // max even-lag count
    static constexpr int PADL = 2 * K;         // sv index of position x is PADL + x
    static constexpr int SV = 5 * K + 8;
    static constexpr int VW = 2 * NW + 4;
    int8_t sv[SV];
    uint32_t V[2][VW];
    uint32_t VR[2][VW];
    int32_t Cev[K + 1];
    int32_t PC[K + 1];
    uint32_t pk[32];
    uint32_t pkbest[32];
};

__device__ __forceinline__ int wave_incl_scan(int v, int lane) {
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        int u = __shfl_up(v, o, 64);
        if (lane >= o) v += u;
    }
    return v;
}

// Fill sv, V, VR from the packed sequence held in S.pk.
template <int NW>
__device__ void build_from_packed(Lds<NW>& S, int L, int k, int lane) {
    constexpr int PADL = Lds<NW>::PADL;
    for (int i = lane; i < Lds<NW>::SV; i += 64) S.sv[i] = 0;
    for (int i = lane; i < 2 * Lds<NW>::VW; i += 64) {
        (&S.V[0][0])[i] = 0;
        (&S.VR[0][0])[i] = 0;
    }
    __syncthreads();
    for (int x = 1 + lane; x <= L; x += 64) S.sv[PADL + x] = packed_bit(S.pk, x) ? 1 : -1;
    __syncthreads();
    const int NV = (k + 1 + 31) >> 5;  // words holding j = 0..k
    const int N = 32 * NV;
    for (int pi = 0; pi < 2; ++pi) {
        for (int base = 0; base < N; base += 64) {
            int j = base + lane;
            int x = 2 * j + 2 - pi;
            bool bit = (x >= 1 && x <= L) && S.sv[PADL + x] > 0;
            uint64_t m = __ballot(bit);
            // reversed: VR bit i = V bit N-1-i
            int jr = N - 1 - j;
            int xr = 2 * jr + 2 - pi;
            bool bitr = (jr >= 0 && xr >= 1 && xr <= L) && S.sv[PADL + xr] > 0;
            uint64_t mr = __ballot(bitr);
            if (lane == 0) {
                S.V[pi][base >> 5] = (uint32_t)m;
                if ((base >> 5) + 1 < Lds<NW>::VW) S.V[pi][(base >> 5) + 1] = (uint32_t)(m >> 32);
                S.VR[pi][base >> 5] = (uint32_t)mr;
                if ((base >> 5) + 1 < Lds<NW>::VW) S.VR[pi][(base >> 5) + 1] = (uint32_t)(mr >> 32);
            }
        }
    }
    __syncthreads();
}

// C_{2m} for this lane's lags m = 64q + lane + 1 (0 beyond K), from sv.
template <int NW>
__device__ void compute_cev(const Lds<NW>& S, int L, int K, int lane, int32_t* C) {
    constexpr int NQ = (NW + 1) / 2;
    constexpr int PADL = Lds<NW>::PADL;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        int m = 64 * q + lane + 1;
        int c = 0;
        if (m <= K) {
            int d = 2 * m;
            for (int i = 1; i <= L - d; ++i) c += (int)S.sv[PADL + i] * (int)S.sv[PADL + i + d];
        }
        C[q] = c;
    }
}

template <int NW>
__device__ void store_tables(Lds<NW>& S, int K, int lane, const int32_t* C) {
    constexpr int NQ = (NW + 1) / 2;
    int carry = 0;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        int m = 64 * q + lane + 1;
        int v = (m <= K) ? C[q] : 0;
        int s = wave_incl_scan(v, lane);
        if (m <= K) {
            S.Cev[m] = C[q];
            S.PC[m] = carry + s;
        }
        carry += __shfl(s, 63, 64);
    }
    if (lane == 0) {
        S.Cev[0] = 0;
        S.PC[0] = 0;
    }
}

template <int NW, int R>
__device__ __forceinline__ void build_windows(const Lds<NW>& S, int p, int k, int lane,
                                              uint32_t (&F)[R][NW],
                                              uint32_t (&B)[R][(NW + 1) / 2]) {
    constexpr int NQ = (NW + 1) / 2;
    const int NV = (k + 1 + 31) >> 5;
    const int N = 32 * NV;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        int a = p + 1 + lane + 64 * r;
        if (a > k + 1) a = k + 1;
        const int pi = a & 1;
        const int ja = (a - 1) >> 1;
        const int sf = ja + 1, qf = sf >> 5, hf = sf & 31;
        const int sb = N - ja, qb = sb >> 5, hb = sb & 31;
        const uint32_t* Vp = S.V[pi];
        const uint32_t* VRp = S.VR[pi];
#pragma unroll
        for (int w = 0; w < NW; ++w)
            F[r][w] = __builtin_amdgcn_alignbit(Vp[qf + w + 1], Vp[qf + w], hf);
#pragma unroll
        for (int w = 0; w < NQ; ++w)
            B[r][w] = __builtin_amdgcn_alignbit(VRp[qb + w + 1], VRp[qb + w], hb);
    }
}

__global__ __launch_bounds__(64) void k_walker_init(WalkArgs A) {
    constexpr int NW = 10;
    __shared__ Lds<NW> S;
    const int lane = threadIdx.x;
    const int64_t j = blockIdx.x;
    const int64_t w = A.walker_begin + j;
    const int L = A.L, k = A.k, p = A.p;
    const uint64_t key = walker_key(A.seed, L, w);
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
    for (int i = lane; i < A.nf; i += 64) A.tabu[j * A.nf + i] = 0;
    if (lane == 0) {
        A.E[j] = e;
        A.tenure[j] = ten;
        A.halted[j] = 0;
        A.bestE[j] = e;
        A.bestT[j] = 0;
    }
}

template <int NW, int R>
__global__ __launch_bounds__(64) void k_walk(WalkArgs A) {
    constexpr int NQ = (NW + 1) / 2;
    constexpr int PADL = Lds<NW>::PADL;
    __shared__ Lds<NW> S;
    const int lane = threadIdx.x;
    const int64_t j = blockIdx.x;
    const int L = A.L, k = A.k, p = A.p, K = A.k, W = A.W, nf = A.nf;
    const int t0 = A.t0, t1 = A.t1;

    int halted = A.halted[j];
    if (halted) {
        if (A.traj)
            for (int t = t0 + 1 + lane; t <= t1; t += 64)
                A.traj[j * A.steps_total + (t - 1)] = -1;
        return;
    }
    if (lane < W) {
        S.pk[lane] = A.seq[j * W + lane];
        S.pkbest[lane] = A.bestSeq[j * W + lane];
    }
    __syncthreads();
    build_from_packed<NW>(S, L, k, lane);
    int32_t C[NQ];
    compute_cev<NW>(S, L, K, lane, C);
    store_tables<NW>(S, K, lane, C);
    int32_t tabu[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        int i = lane + 64 * r;
        tabu[r] = (i < nf) ? A.tabu[j * nf + i] : INT_MAX;
    }
    int E = A.E[j];
    int bestE = A.bestE[j];
    int bestT = A.bestT[j];
    const int tenure = A.tenure[j];
    const bool sieve = A.e_max >= 0;
    int thr = A.e_max;
    if (sieve && A.thr) thr = min(thr, *A.thr);
    const int64_t wid = A.walker_begin + j;
    __syncthreads();

    uint32_t F[R][NW], B[R][NQ];
    build_windows<NW, R>(S, p, k, lane, F, B);
    // masks of lags m <= Mb for the backward-overlap count
    uint32_t QM[R][NQ];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        int a = p + 1 + lane + 64 * r;
        if (a > k + 1) a = k + 1;
        const int Mb = (a - 1) >> 1;
#pragma unroll
        for (int w = 0; w < NQ; ++w) {
            int c = Mb - 32 * w;
            QM[r][w] = c >= 32 ? 0xffffffffu : (c <= 0 ? 0u : ((1u << c) - 1u));
        }
    }

    for (int t = t0 + 1; t <= t1; ++t) {
        // ---- number of bit planes for the current C table
        uint32_t orv = 0;
#pragma unroll
        for (int q = 0; q < NQ; ++q) orv |= (uint32_t)(C[q] ^ (C[q] >> 31));
        orv = __ockl_wfred_or_u32(orv);
        const int nb = (32 - __clz((int)orv)) + 1;

        // ---- H = H_f + H_b, bit-sliced
        int32_t H[R];
#pragma unroll
        for (int r = 0; r < R; ++r) H[r] = 0;
        for (int jp = 0; jp < nb; ++jp) {
            uint32_t acc[R];
#pragma unroll
            for (int r = 0; r < R; ++r) acc[r] = 0;
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                const uint64_t bal = __ballot((C[q] >> jp) & 1);
                const uint32_t lo = (uint32_t)bal, hi = (uint32_t)(bal >> 32);
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    acc[r] += __popc(lo & F[r][2 * q]);
                    if (2 * q + 1 < NW) acc[r] += __popc(hi & F[r][2 * q + 1]);
                    if (2 * q < NQ) acc[r] += __popc(lo & B[r][2 * q]);
                    if (2 * q + 1 < NQ) acc[r] += __popc(hi & B[r][2 * q + 1]);
                }
            }
            const int wgt = (jp == nb - 1) ? -(1 << jp) : (1 << jp);
#pragma unroll
            for (int r = 0; r < R; ++r) H[r] += wgt * (int)acc[r];
        }

        // ---- exact dE per slot
        int dlt[R];
        bool adm[R];
        int dmin = INT_MAX;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int a0 = p + 1 + lane + 64 * r;
            const bool valid = a0 <= k + 1;
            const int a = valid ? a0 : k + 1;
            const int Mf = (L - a) >> 1, Mb = (a - 1) >> 1;
            const int sa = S.sv[PADL + a];
            int d;
            if (a == k + 1) {
                d = -8 * sa * (H[r] - S.PC[Mb]) + 16 * Mb;
            } else {
                const int mp = k + 1 - a;
                const int sbv = S.sv[PADL + L + 1 - a];
                int X = 0;
#pragma unroll
                for (int w = 0; w < NQ; ++w) X += __popc((F[r][w] ^ B[r][w]) & QM[r][w]);
                const int G = 2 * H[r] - S.PC[Mf] - S.PC[Mb] - S.Cev[mp] * sbv;
                const int corr = (mp <= Mb) ? 2 * sbv * S.sv[PADL + a - 2 * mp] : 0;
                const int Q = Mf - 1 + 3 * Mb - 4 * X - corr;
                d = -8 * sa * G + 16 * Q;
            }
            dlt[r] = d;
            adm[r] = valid && tabu[r] < t;
            if (adm[r]) dmin = min(dmin, d);
        }
        const int g = __ockl_wfred_min_i32(dmin);
        if (g == INT_MAX) {
            halted = t;
            break;
        }
        int astar = -1;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const uint64_t m = __ballot(adm[r] && dlt[r] == g);
            if (astar < 0 && m) astar = p + 1 + 64 * r + (__ffsll((unsigned long long)m) - 1);
        }
        // ---- apply: C update from the old sequence
        const int as = astar, bs = L + 1 - astar;
        const bool cen = (as == k + 1);
        const int s_as = S.sv[PADL + as];
        const int s_bs = S.sv[PADL + bs];
        const int mps = k + 1 - as;
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const int m = 64 * q + lane + 1;
            if (m <= K) {
                int u;
                if (cen) u = S.sv[PADL + as - 2 * m];
                else u = S.sv[PADL + as + 2 * m] + S.sv[PADL + as - 2 * m] - (m == mps ? s_bs : 0);
                C[q] += -4 * s_as * u;
            }
        }
        E += g;
#pragma unroll
        for (int r = 0; r < R; ++r)
            if (p + 1 + lane + 64 * r == as) tabu[r] = t + tenure;
        __syncthreads();
        store_tables<NW>(S, K, lane, C);
        if (lane == 0 || (lane == 1 && !cen)) {
            const int x = lane == 0 ? as : bs;
            S.sv[PADL + x] = (int8_t)(-S.sv[PADL + x]);
            const int pi = x & 1, jj = (x - 1) >> 1;
            const int NV = (k + 1 + 31) >> 5;
            const int ir = 32 * NV - 1 - jj;
            atomicXor(&S.V[pi][jj >> 5], 1u << (jj & 31));
            atomicXor(&S.VR[pi][ir >> 5], 1u << (ir & 31));
            atomicXor(&S.pk[(x - 1) >> 5], 1u << (31 - ((x - 1) & 31)));
        }
        __syncthreads();
        if (E < bestE) {
            bestE = E;
            bestT = t;
            if (lane < W) S.pkbest[lane] = S.pk[lane];
        }
        if (A.traj && lane == 0) A.traj[j * A.steps_total + (t - 1)] = E;
        if (sieve && E <= thr) {
            uint32_t slot = 0;
            if (lane == 0) slot = atomicAdd(A.st_count, 1u);
            slot = __shfl(slot, 0, 64);
            if (slot < A.st_cap && lane < W + 3) {
                uint32_t v;
                if (lane == 0) v = (uint32_t)E;
                else if (lane <= W) v = S.pk[lane - 1];
                else if (lane == W + 1) v = (uint32_t)wid;
                else v = (uint32_t)t;
                A.rec[(int64_t)lane * A.rec_stride + slot] = v;
            }
        }
        build_windows<NW, R>(S, p, k, lane, F, B);
    }
    __syncthreads();
    if (halted && A.traj)
        for (int t = halted + lane; t <= t1; t += 64) A.traj[j * A.steps_total + (t - 1)] = -1;
    if (lane < W) {
        A.seq[j * W + lane] = S.pk[lane];
        A.bestSeq[j * W + lane] = S.pkbest[lane];
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        int i = lane + 64 * r;
        if (i < nf) A.tabu[j * nf + i] = tabu[r];
    }
    if (lane == 0) {
        A.E[j] = E;
        A.bestE[j] = bestE;
        A.bestT[j] = bestT;
        A.halted[j] = halted;
    }
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

typedef void (*walk_kernel_t)(WalkArgs);

template <int NW, int R>
walk_kernel_t pick() {
    return k_walk<NW, R>;
}

// R in {ceil(NW/2), ceil(NW/2)+1}
template <int NW>
walk_kernel_t pick_r(int R) {
    constexpr int R0 = (NW + 1) / 2;
    if (R <= R0) return pick<NW, R0>();
    if (R == R0 + 1) return pick<NW, R0 + 1>();
    return nullptr;
}

walk_kernel_t select_walk_kernel(int NW, int R) {
    switch (NW) {
        case 1: return pick_r<1>(R);
        case 2: return pick_r<2>(R);
        case 3: return pick_r<3>(R);
        case 4: return pick_r<4>(R);
        case 5: return pick_r<5>(R);
        case 6: return pick_r<6>(R);
        case 7: return pick_r<7>(R);
        case 8: return pick_r<8>(R);
        case 9: return pick_r<9>(R);
        case 10: return pick_r<10>(R);
        default: return nullptr;
    }
}

}  // namespace

bool walk_shape_supported(int L, int p) {
    const int k = (L - 1) / 2;
    const int NW = (k + 31) / 32;
    const int R = (k + 1 - p + 63) / 64;
    return NW >= 1 && NW <= 10 && select_walk_kernel(NW, R) != nullptr;
}

labs_status launch_walker_init(const WalkArgs& A, hipStream_t st) {
    hipLaunchKernelGGL(k_walker_init, dim3((unsigned)A.n), dim3(64), 0, st, A);
    LABS_LAUNCHED("k_walker_init");
    return LABS_OK;
}

labs_status launch_walk(const WalkArgs& A, hipStream_t st) {
    const int NW = (A.k + 31) / 32;
    const int R = (A.nf + 63) / 64;
    walk_kernel_t kern = select_walk_kernel(NW, R);
    if (!kern) return invalid("no walker kernel for L=%d p=%d", A.L, A.p);
    hipLaunchKernelGGL(kern, dim3((unsigned)A.n), dim3(64), 0, st, A);
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
