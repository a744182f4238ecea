// Templates of the first-step walker (shared by the instantiation units).
// See walk.hip for the method and the notation.
#pragma once
#include "labs_internal.h"

#include <climits>

namespace labsdev {
namespace walkimpl {

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

// Inclusive prefix sum over the wavefront (the device library's scan: DPP row
// shifts and broadcasts, no LDS permutes).
__device__ __forceinline__ int wave_incl_scan(int v, int lane) {
    (void)lane;
    return __ockl_wfscan_add_i32(v, true);
}

// Fill sv, V, VR from the packed sequence held in S.pk.
template <int NW>
__device__ inline void build_from_packed(Lds<NW>& S, int L, int k, int lane) {
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
__device__ inline void compute_cev(const Lds<NW>& S, int L, int K, int lane, int32_t* C) {
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
__device__ inline void store_tables(Lds<NW>& S, int K, int lane, const int32_t* C) {
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

// bfull: the last backward word holds a lag (k/2 > 32(NQ-1)); when it does not
// (k = 64(NQ-1)+1 with NW odd), that word is zero for every slot and is skipped.
// g0: slot group of F[0].  Slot group g holds positions a >= 1 + 64 g, whose forward
// windows reach at most (L - a)/2 <= k - 32 g lags: forward words w >= NW - g are zero
// (the loops are unrolled, so those words and every popcount of them fold away).
template <int NW, int R>
__device__ __forceinline__ void build_windows(const Lds<NW>& S, int p, int k, int lane, bool bfull, int g0,
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
            F[r][w] = w < NW - (g0 + r) ? __builtin_amdgcn_alignbit(Vp[qf + w + 1], Vp[qf + w], hf) : 0u;
#pragma unroll
        for (int w = 0; w < NQ - 1; ++w)
            B[r][w] = __builtin_amdgcn_alignbit(VRp[qb + w + 1], VRp[qb + w], hb);
        B[r][NQ - 1] = bfull ? __builtin_amdgcn_alignbit(VRp[qb + NQ], VRp[qb + NQ - 1], hb) : 0u;
    }
}

// One walker (walker index j of configuration A) for steps t0+1..t1.  Slots are
// scanned in groups of RB (R = RB: one pass with every window resident; smaller
// RB: fewer window registers, the bit planes re-ballotted once per group).
// BL: self-avoidance by the walker's Bloom filter (copied into `bl` in LDS for
// the segment) instead of the tabu tenure.
template <int NW, int R, int RB, bool BL>
__device__ __forceinline__ void walk_body(const WalkArgs& A, int64_t j, Lds<NW>& S, uint32_t* bl) {
    constexpr int NQ = (NW + 1) / 2;
    constexpr int PADL = Lds<NW>::PADL;
    constexpr int NG = (R + RB - 1) / RB;
    const int lane = threadIdx.x & 63;
    const int L = A.L, k = A.k, p = A.p, K = A.k, W = A.W, nf = A.nf;
    const int t0 = A.t0, t1 = A.t1;

    __syncthreads();
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
    int32_t Ch[NQ];   // (C_{2m} - 1)/2 on valid lags, 0 beyond; kept beside C
#pragma unroll
    for (int q = 0; q < NQ; ++q) Ch[q] = (64 * q + lane + 1 <= K) ? (C[q] - 1) >> 1 : 0;
    // +1 digits at even (ones0) and odd (ones1) positions, kept through the walk: a
    // slot's windows F_a and B_a cover every other position of a's parity, so
    // together they hold (ones of a's parity) - [s_a = +1] set bits
    int ones0, ones1;
    {
        int c0 = 0, c1 = 0;
        for (int x = 1 + lane; x <= L; x += 64)
            if (S.sv[PADL + x] > 0) {
                if (x & 1) ++c1;
                else ++c0;
            }
        ones0 = __ockl_wfred_add_i32(c0);
        ones1 = __ockl_wfred_add_i32(c1);
    }
    int32_t tabu[R];
    uint64_t zr[R];        // Bloom: Zobrist entry of each slot's position
    uint64_t hk = 0;       // Bloom: key of the current sequence
    int last_a = -1;       // Bloom: position flipped by the previous step of this segment
    uint32_t* gbl = nullptr;
    const int nbw = BL ? 1 << (A.bloom_log2 - 5) : 0;
    const uint32_t bmask = BL ? (1u << A.bloom_log2) - 1u : 0u;
    const int nh = BL ? A.bloom_hashes : 0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        int i = lane + 64 * r;
        if constexpr (BL) {
            tabu[r] = 0;
            zr[r] = zobrist_at(p + (i < nf ? i : nf - 1));
        } else {
            tabu[r] = (i < nf) ? A.tabu[j * nf + i] : INT_MAX;
            zr[r] = 0;
        }
    }
    if constexpr (BL) {
        gbl = A.bloom + j * (int64_t)nbw;
        for (int i = lane; i < nbw; i += 64) bl[i] = gbl[i];
        hk = A.zh[j];
    }
    int E = A.E[j];
    int bestE = A.bestE[j];
    int bestT = A.bestT[j];
    const int tenure = A.tenure[j];
    const bool sieve = A.e_max >= 0;
    const int thr = A.e_max;
    const int64_t wid = A.walker_begin + j;
    const bool bfull = (NW & 1) == 0 || (k >> 1) > 32 * (NQ - 1);   // always, for even NW
    int pend = pending_level(A);          // first-hit stamps: largest level energy above E
    __syncthreads();

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
        // ---- bit planes of v = C' + bias, C' = (C - 1)/2: for odd L every even-lag
        // C_{2m} is odd (a sum of L - 2m terms of +-1), so sum_m C F = 2 sum_m C' F +
        // popcount(F); bias = -min C' makes every v >= 0, so the planes need only the
        // bits of max C' - min C' (no sign plane), and sum_m C' F = sum_m v F - bias
        // popcount(F).  Lags beyond k hold C' = 0 and meet zero window bits.
        int lmin = Ch[0], lmax = Ch[0];
#pragma unroll
        for (int q = 1; q < NQ; ++q) {
            lmin = min(lmin, Ch[q]);
            lmax = max(lmax, Ch[q]);
        }
        const int cmin = __ockl_wfred_min_i32(lmin);
        const int cmax = __ockl_wfred_max_i32(lmax);
        const int bias = -cmin;
        const uint32_t vmax = (uint32_t)(cmax - cmin);
        const int nb = vmax ? 32 - __clz((int)vmax) : 0;
        uint32_t Vq[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) Vq[q] = (uint32_t)(Ch[q] + bias);

        // ---- H = H_f + H_b, bit-sliced, then the exact dE, RB slots at a time
        int dlt[R];
        bool adm[R];
        int dmin = INT_MAX;
#pragma unroll
        for (int gi = 0; gi < NG; ++gi) {
            uint32_t F[RB][NW], B[RB][NQ];
            build_windows<NW, RB>(S, p + 64 * RB * gi, k, lane, bfull, RB * gi, F, B);
            int32_t H[RB];
#pragma unroll
            for (int r = 0; r < RB; ++r) H[r] = 0;
            for (int jp = 0; jp < nb; ++jp) {
                uint32_t acc[RB];
#pragma unroll
                for (int r = 0; r < RB; ++r) acc[r] = 0;
#pragma unroll
                for (int q = 0; q < NQ; ++q) {
                    const uint64_t bal = __ballot((Vq[q] >> jp) & 1u);
                    const uint32_t lo = (uint32_t)bal, hi = (uint32_t)(bal >> 32);
#pragma unroll
                    for (int r = 0; r < RB; ++r) {
                        // forward words beyond the group's reach are zero (see build_windows)
                        const int g = RB * gi + r;
                        if (2 * q < NW - g) acc[r] = bcnt_add(lo & F[r][2 * q], acc[r]);
                        if (2 * q + 1 < NW - g) acc[r] = bcnt_add(hi & F[r][2 * q + 1], acc[r]);
                        if (2 * q < NQ - 1) acc[r] = bcnt_add(lo & B[r][2 * q], acc[r]);
                        if (2 * q + 1 < NQ - 1) acc[r] = bcnt_add(hi & B[r][2 * q + 1], acc[r]);
                    }
                    if ((2 * q == NQ - 1 || 2 * q + 1 == NQ - 1) && bfull) {
                        const uint32_t hl = (2 * q == NQ - 1) ? lo : hi;
#pragma unroll
                        for (int r = 0; r < RB; ++r) acc[r] = bcnt_add(hl & B[r][NQ - 1], acc[r]);
                    }
                }
#pragma unroll
                for (int r = 0; r < RB; ++r) H[r] += (int)(acc[r] << jp);
            }
#pragma unroll
            for (int r = 0; r < RB; ++r) {
                int a = p + 1 + lane + 64 * (gi * RB + r);
                if (a > k + 1) a = k + 1;
                const int pf = ((a & 1) ? ones1 : ones0) - (S.sv[PADL + a] > 0 ? 1 : 0);
                H[r] = 2 * (H[r] - bias * pf) + pf;
            }
#pragma unroll
            for (int rr = 0; rr < RB; ++rr) {
                const int r = gi * RB + rr;
                if (r >= R) break;
                const int a0 = p + 1 + lane + 64 * r;
                const bool valid = a0 <= k + 1;
                const int a = valid ? a0 : k + 1;
                const int Mf = (L - a) >> 1, Mb = (a - 1) >> 1;
                const int sa = S.sv[PADL + a];
                int d;
                if (a == k + 1) {
                    d = -8 * sa * (H[rr] - S.PC[Mb]) + 16 * Mb;
                } else {
                    const int mp = k + 1 - a;
                    const int sbv = S.sv[PADL + L + 1 - a];
                    int X = 0;
#pragma unroll
                    for (int w = 0; w < NQ - 1; ++w) X += __popc((F[rr][w] ^ B[rr][w]) & QM[r][w]);
                    if (bfull) X += __popc((F[rr][NQ - 1] ^ B[rr][NQ - 1]) & QM[r][NQ - 1]);
                    const int G = 2 * H[rr] - S.PC[Mf] - S.PC[Mb] - S.Cev[mp] * sbv;
                    const int corr = (mp <= Mb) ? 2 * sbv * S.sv[PADL + a - 2 * mp] : 0;
                    const int Q = Mf - 1 + 3 * Mb - 4 * X - corr;
                    d = -8 * sa * G + 16 * Q;
                }
                dlt[r] = d;
                // Bloom: undoing the last move returns to a sequence the filter holds
                // (no false negatives), so that slot is out without a probe; the
                // others are tested below, best candidate first
                if constexpr (BL) adm[r] = valid && a0 != last_a;
                else adm[r] = valid && tabu[r] < t;
                if (adm[r]) dmin = min(dmin, d);
            }
        }
        int g = INT_MAX, astar = -1;
        uint64_t hnext = 0;
        for (;;) {
            g = __ockl_wfred_min_i32(dmin);
            if (g == INT_MAX) break;
            astar = -1;
            int owner = 0, rsel = 0;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const uint64_t m = __ballot(adm[r] && dlt[r] == g);
                if (astar < 0 && m) {
                    owner = __ffsll((unsigned long long)m) - 1;
                    rsel = r;
                    astar = p + 1 + 64 * r + owner;
                }
            }
            if constexpr (!BL) {
                break;
            } else {
                // Bloom: the lowest (dE, a) not in the filter.  Test the current
                // best candidate (probe q on lane q); a member is excluded and the
                // next best taken, so each pass removes one slot and the loop ends.
                uint64_t z = 0;
#pragma unroll
                for (int r = 0; r < R; ++r)
                    if (r == rsel) z = zr[r];
                const uint32_t zlo = __builtin_amdgcn_readlane((uint32_t)z, owner);
                const uint32_t zhi = __builtin_amdgcn_readlane((uint32_t)(z >> 32), owner);
                const uint64_t key = hk ^ (((uint64_t)zhi << 32) | zlo);
                bool set = true;
                if (lane < nh) {
                    const uint32_t b =
                        ((uint32_t)key + (uint32_t)lane * ((uint32_t)(key >> 32) | 1u)) & bmask;
                    set = (bl[b >> 5] >> (b & 31)) & 1u;
                }
                if (__ballot(!set)) {
                    hnext = key;
                    break;
                }
                dmin = INT_MAX;
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    if (p + 1 + lane + 64 * r == astar) adm[r] = false;
                    if (adm[r]) dmin = min(dmin, dlt[r]);
                }
            }
        }
        if (g == INT_MAX) {
            halted = t;
            break;
        }
        // ---- apply: C update from the old sequence
        const int as = astar, bs = L + 1 - astar;
        const bool cen = (as == k + 1);
        const int s_as = S.sv[PADL + as];
        const int s_bs = S.sv[PADL + bs];
        const int mps = k + 1 - as;
        {
            const int dn = -s_as - (cen ? 0 : s_bs);   // as and bs share a parity (L + 1 is even)
            if (as & 1) ones1 += dn;
            else ones0 += dn;
        }
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const int m = 64 * q + lane + 1;
            if (m <= K) {
                int u;
                if (cen) u = S.sv[PADL + as - 2 * m];
                else u = S.sv[PADL + as + 2 * m] + S.sv[PADL + as - 2 * m] - (m == mps ? s_bs : 0);
                C[q] += -4 * s_as * u;
                Ch[q] += -2 * s_as * u;
            }
        }
        E += g;
        if constexpr (!BL) {
#pragma unroll
            for (int r = 0; r < R; ++r)
                if (p + 1 + lane + 64 * r == as) tabu[r] = t + tenure;
        }
        __syncthreads();
        if constexpr (BL) {
            // insert the new sequence's key; read by the next step after the barrier below
            hk = hnext;
            last_a = as;
            if (lane < nh) {
                const uint32_t b = ((uint32_t)hk + (uint32_t)lane * ((uint32_t)(hk >> 32) | 1u)) & bmask;
                atomicOr(&bl[b >> 5], 1u << (b & 31));
            }
        }
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
        if (E <= pend) pend = stamp_levels(A, E, lane);
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
    }
    __syncthreads();
    if (halted && A.traj)
        for (int t = halted + lane; t <= t1; t += 64) A.traj[j * A.steps_total + (t - 1)] = -1;
    if (lane < W) {
        A.seq[j * W + lane] = S.pk[lane];
        A.bestSeq[j * W + lane] = S.pkbest[lane];
    }
    if constexpr (BL) {
        for (int i = lane; i < nbw; i += 64) gbl[i] = bl[i];
        if (lane == 0) A.zh[j] = hk;
    } else {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            int i = lane + 64 * r;
            if (i < nf) A.tabu[j * nf + i] = tabu[r];
        }
    }
    if (lane == 0) {
        A.E[j] = E;
        A.bestE[j] = bestE;
        A.bestT[j] = bestT;
        A.halted[j] = halted;
    }
}


// Waves per SIMD the compiler is held to for a plain walk kernel, where a kernel
// left free lands a few VGPRs above an occupancy step and runs faster held below it
// despite a few spilled registers (flip-evals/s, 8,000 steps):
//   (9, 4, 4) 184 -> 168 VGPRs, three waves: L = 527, p = 16: 1.24 -> 1.32e11
//   (7, 3, 3) 137 -> 128 VGPRs, four waves:  L = 387, p = 12: 1.51 -> 1.66e11
//   (7, 4, 2) 139 -> 128 VGPRs, four waves:  L = 409, p = 12: 1.23 -> 1.34e11
template <int NW, int R, int RB>
struct WalkWaves {
    static constexpr int value = (NW == 9 && R == 4 && RB == 4)                            ? 3
                                 : (NW == 7 && ((R == 3 && RB == 3) || (R == 4 && RB == 2))) ? 4
                                                                                             : 1;
};

template <int NW, int R, int RB>
__global__ __launch_bounds__(64, (WalkWaves<NW, R, RB>::value)) void k_walk(WalkArgs A) {
    __shared__ Lds<NW> S;
    walk_body<NW, R, RB, false>(A, blockIdx.x, S, nullptr);
}

// Bloom-filter form: the walker's filter (2^bloom_log2 bits) in dynamic LDS.
template <int NW, int R, int RB>
__global__ __launch_bounds__(64) void k_walk_bloom(WalkArgs A) {
    __shared__ Lds<NW> S;
    extern __shared__ uint32_t bloom_words[];
    walk_body<NW, R, RB, true>(A, blockIdx.x, S, bloom_words);
}

// Persistent form: each wavefront takes (configuration, walker) items from a
// queue until it is empty, so every wavefront exits.
template <int NW, int R, int RB>
__global__ __launch_bounds__(64) void k_walk_persistent(const WalkArgs* __restrict__ args, const int2* items,
                                                        int n_items, unsigned* head) {
    __shared__ Lds<NW> S;
    for (;;) {
        unsigned it = 0;
        if (threadIdx.x == 0) it = atomicAdd(head, 1u);
        // a wave-uniform item (readfirstlane, not a shuffle), so the item and its
        // configuration's arguments load into scalar registers as a plain launch's do
        it = __builtin_amdgcn_readfirstlane(it);
        if (it >= (unsigned)n_items) break;
        const int2 w = items[it];
        // by reference: the fields load on demand, as from a plain launch's arguments
        const WalkArgs& A = args[__builtin_amdgcn_readfirstlane(w.x)];
        walk_body<NW, R, RB, false>(A, (int64_t)w.y, S, nullptr);
    }
}

typedef void (*walk_kernel_t)(WalkArgs);
typedef void (*walk_persistent_t)(const WalkArgs*, const int2*, int, unsigned*);

}  // namespace walkimpl

// Kernel lookup across the instantiation units: plain and persistent forms for
// (NW, R, RB); R is rounded up to an instantiated value, RB to R or ceil(R/2).
struct WalkKernels {
    walkimpl::walk_kernel_t plain;
    walkimpl::walk_kernel_t bloom;
    walkimpl::walk_persistent_t persistent;
    int R, RB;
};
bool walk_kernels_lookup(int NW, int R, int RB, WalkKernels* out);
bool walk_kernels_a(int NW, int R, int RB, WalkKernels* out);   // NW 1..4
bool walk_kernels_b(int NW, int R, int RB, WalkKernels* out);   // NW 5..7
bool walk_kernels_c(int NW, int R, int RB, WalkKernels* out);   // NW 8..10

}  // namespace labsdev
