// Learned flip proposal: a 2-hidden-layer GELU MLP over walker states, trained
// and evaluated with bfloat16 MFMA products (FP32 accumulation) on gfx950.
//
// The network is not part of the paper's method; it only reorders which skew
// flips (Eq. (2) partners flipped together) get their exact energy change
// computed.  Layout of the parameter blob and every buffer is described in
// include/labs.h next to labs_mlp_layout_of.
#include "labs_internal.h"

#include <cmath>

namespace labsdev {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// ------------------------------------------------------------------ scalars
__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// GELU, tanh form (Hendrycks and Gimpel 2016), and its derivative.
__device__ __forceinline__ float gelu_f(float x) {
    const float u = 0.7978845608028654f * (x + 0.044715f * x * x * x);
    return 0.5f * x * (1.0f + tanhf(u));
}
__device__ __forceinline__ float gelu_grad_f(float x) {
    const float u = 0.7978845608028654f * (x + 0.044715f * x * x * x);
    const float t = tanhf(u);
    const float du = 0.7978845608028654f * (1.0f + 3.0f * 0.044715f * x * x);
    return 0.5f * (1.0f + t) + 0.5f * x * (1.0f - t * t) * du;
}

// ------------------------------------------------------------------ GEMM
// C[m][n] = sum_k A(m,k) B(k,n) over bf16 operands with FP32 accumulation.
//   A(m,k) = A[m*lda + k] when A_K (K contiguous), else A[k*lda + m]
//   B(k,n) = B[n*ldb + k] when B_K (K contiguous), else B[k*ldb + n]
// Leading dimensions are multiples of 8 elements and bases 16-byte aligned
// (checked on the host), so 8-element chunks load as one 16-byte access.
// Tile 64x64x32, four waves each owning a 32x32 quarter as 2x2 MFMA 16x16x32
// blocks.  Operand fragments (gfx950 v_mfma_f32_16x16x32_bf16): lane l feeds
// row l%16 of A and column l%16 of B with k = 8*(l/16) .. 8*(l/16)+7; the
// result holds column l%16, rows 4*(l/16) .. 4*(l/16)+3.
enum EpiKind { EPI_F32 = 0, EPI_BIAS_F32 = 1, EPI_BIAS_GELU = 2, EPI_DGELU = 3 };

struct Epi {
    int kind;
    float* out_f;        // fp32 output (EPI_F32, EPI_BIAS_F32, EPI_DGELU), row stride ldf
    int64_t ldf;
    uint16_t* out_b;     // bf16 output (EPI_BIAS_GELU, EPI_DGELU), row stride ldb
    int64_t ldb;
    const float* bias;   // [N] (EPI_BIAS_*)
    float* pre;          // EPI_BIAS_GELU: pre-activation out (nullable); EPI_DGELU: read
    int64_t ldp;
    int64_t zstride;     // split-K: FP32 output offset per split
};

constexpr int GT = 64, GK = 32, GPAD = 8;

// One thread's share of a 64-row x 32-k operand slice (8 bf16 values).
// K-contiguous operand: row t/4, k chunk 8*(t%4); row-contiguous operand
// (element (r, k) at k*ld + r): k row t/8, rows 8*(t%8) .. +7.  Reads past
// `rows` or `K` give zeros.
template <bool A_K>
__device__ __forceinline__ uint4 fetch64(const uint16_t* __restrict__ P, int64_t ld, int rows, int K, int r0,
                                         int k0) {
    const int t = threadIdx.x;
    uint4 v = make_uint4(0, 0, 0, 0);
    if (A_K) {
        const int gr = r0 + (t >> 2), gk = k0 + (t & 3) * 8;
        if (gr < rows) {
            const uint16_t* src = P + (int64_t)gr * ld + gk;
            if (gk + 8 <= K) {
                v = *(const uint4*)src;
            } else {
                uint16_t e[8];
                for (int j = 0; j < 8; ++j) e[j] = (gk + j < K) ? src[j] : (uint16_t)0;
                v.x = e[0] | ((uint32_t)e[1] << 16);
                v.y = e[2] | ((uint32_t)e[3] << 16);
                v.z = e[4] | ((uint32_t)e[5] << 16);
                v.w = e[6] | ((uint32_t)e[7] << 16);
            }
        }
    } else {
        const int gk = k0 + (t >> 3), gr = r0 + (t & 7) * 8;
        if (gk < K) {
            const uint16_t* src = P + (int64_t)gk * ld + gr;
            if (gr + 8 <= rows) {
                v = *(const uint4*)src;
            } else {
                uint16_t e[8];
                for (int j = 0; j < 8; ++j) e[j] = (gr + j < rows) ? src[j] : (uint16_t)0;
                v.x = e[0] | ((uint32_t)e[1] << 16);
                v.y = e[2] | ((uint32_t)e[3] << 16);
                v.z = e[4] | ((uint32_t)e[5] << 16);
                v.w = e[6] | ((uint32_t)e[7] << 16);
            }
        }
    }
    return v;
}

// Stores a fetched share into the [row][k] LDS tile (transposing row-contiguous data).
template <bool A_K>
__device__ __forceinline__ void put64(uint16_t (*S)[GK + GPAD], uint4 v) {
    const int t = threadIdx.x;
    if (A_K) {
        *(uint4*)&S[t >> 2][(t & 3) * 8] = v;
    } else {
        const int kr = t >> 3, rc = (t & 7) * 8;
        const uint32_t w[4] = {v.x, v.y, v.z, v.w};
        for (int j = 0; j < 4; ++j) {
            S[rc + 2 * j][kr] = (uint16_t)(w[j] & 0xFFFF);
            S[rc + 2 * j + 1][kr] = (uint16_t)(w[j] >> 16);
        }
    }
}

__device__ __forceinline__ void epilogue(const Epi& epi, int m, int n, float v);

// 64x64x32 tiles, four waves each owning a 32x32 quarter as 2x2 MFMA blocks;
// the next K slice is fetched into registers while the current one is
// multiplied (double-buffered LDS, one barrier per K step).  blockIdx.z selects
// a K range of `kchunk` for split-K products; the epilogue's FP32 output then
// advances by epi.zstride per split.
template <bool A_K, bool B_K>
__global__ __launch_bounds__(256) void k_gemm(int M, int N, int K, int kchunk, const uint16_t* __restrict__ A,
                                              int64_t lda, const uint16_t* __restrict__ B, int64_t ldb,
                                              Epi epi) {
    __shared__ __attribute__((aligned(16))) uint16_t As[2][GT][GK + GPAD];
    __shared__ __attribute__((aligned(16))) uint16_t Bs[2][GT][GK + GPAD];
    const int m0 = blockIdx.y * GT, n0 = blockIdx.x * GT;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    const int fr = lane & 15, fk = (lane >> 4) * 8;
    const int klo = blockIdx.z * kchunk;
    const int khi = (klo + kchunk < K) ? klo + kchunk : K;
    if (epi.out_f) epi.out_f += (int64_t)blockIdx.z * epi.zstride;

    f32x4 acc[2][2];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

    if (klo < khi) {
        uint4 ra = fetch64<A_K>(A, lda, M, khi, m0, klo);
        uint4 rb = fetch64<B_K>(B, ldb, N, khi, n0, klo);
        put64<A_K>(As[0], ra);
        put64<B_K>(Bs[0], rb);
        __syncthreads();
        int cur = 0;
        for (int k0 = klo; k0 < khi; k0 += GK) {
            const bool more = k0 + GK < khi;
            if (more) {
                ra = fetch64<A_K>(A, lda, M, khi, m0, k0 + GK);
                rb = fetch64<B_K>(B, ldb, N, khi, n0, k0 + GK);
            }
            bf16x8 a[2], b[2];
            for (int i = 0; i < 2; ++i) a[i] = *(const bf16x8*)&As[cur][wm + 16 * i + fr][fk];
            for (int j = 0; j < 2; ++j) b[j] = *(const bf16x8*)&Bs[cur][wn + 16 * j + fr][fk];
            for (int i = 0; i < 2; ++i)
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
            if (more) {
                put64<A_K>(As[cur ^ 1], ra);
                put64<B_K>(Bs[cur ^ 1], rb);
            }
            __syncthreads();
            cur ^= 1;
        }
    }

    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) {
            const int n = n0 + wn + 16 * j + fr;
            if (n >= N) continue;
            for (int r = 0; r < 4; ++r) {
                const int m = m0 + wm + 16 * i + (lane >> 4) * 4 + r;
                if (m < M) epilogue(epi, m, n, acc[i][j][r]);
            }
        }
}

// Sum of `splits` FP32 partial products [splits][M][N] into out (row stride ldo),
// in split order.
__global__ __launch_bounds__(256) void k_sum_splits(int M, int N, int splits, const float* __restrict__ part,
                                                    float* __restrict__ out, int64_t ldo) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= (int64_t)M * N) return;
    float s = 0.f;
    for (int z = 0; z < splits; ++z) s += part[(int64_t)z * M * N + i];
    out[(i / N) * ldo + (i % N)] = s;
}

// Forward products (both operands K-contiguous) on 128x128x32 tiles: each of
// the four waves owns a 64x64 quarter as 4x4 MFMA blocks; LDS is double
// buffered and the next K slice is fetched into registers while the current
// one is multiplied, so one barrier per K step suffices.
constexpr int BT = 128;

__device__ __forceinline__ void fetch_rows(uint4 (&r)[2], const uint16_t* __restrict__ P, int64_t ld, int rows,
                                           int K, int r0, int k0) {
    const int t = threadIdx.x;
    #pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int rr = (t >> 2) + 64 * h, kc = (t & 3) * 8;
        const int gr = r0 + rr, gk = k0 + kc;
        uint4 v = make_uint4(0, 0, 0, 0);
        if (gr < rows) {
            const uint16_t* src = P + (int64_t)gr * ld + gk;
            if (gk + 8 <= K) {
                v = *(const uint4*)src;
            } else {
                uint16_t e[8];
                for (int j = 0; j < 8; ++j) e[j] = (gk + j < K) ? src[j] : (uint16_t)0;
                v.x = e[0] | ((uint32_t)e[1] << 16);
                v.y = e[2] | ((uint32_t)e[3] << 16);
                v.z = e[4] | ((uint32_t)e[5] << 16);
                v.w = e[6] | ((uint32_t)e[7] << 16);
            }
        }
        r[h] = v;
    }
}

__device__ __forceinline__ void put_rows(uint16_t (*S)[GK + GPAD], const uint4 (&r)[2]) {
    const int t = threadIdx.x;
    #pragma unroll
    for (int h = 0; h < 2; ++h) *(uint4*)&S[(t >> 2) + 64 * h][(t & 3) * 8] = r[h];
}

__device__ __forceinline__ void epilogue(const Epi& epi, int m, int n, float v) {
    switch (epi.kind) {
        case EPI_F32: epi.out_f[(int64_t)m * epi.ldf + n] = v; break;
        case EPI_BIAS_F32: epi.out_f[(int64_t)m * epi.ldf + n] = v + epi.bias[n]; break;
        case EPI_BIAS_GELU: {
            const float a = v + epi.bias[n];
            if (epi.pre) epi.pre[(int64_t)m * epi.ldp + n] = a;
            epi.out_b[(int64_t)m * epi.ldb + n] = f2bf(gelu_f(a));
            break;
        }
        default: {
            const float d = v * gelu_grad_f(epi.pre[(int64_t)m * epi.ldp + n]);
            epi.out_f[(int64_t)m * epi.ldf + n] = d;
            epi.out_b[(int64_t)m * epi.ldb + n] = f2bf(d);
            break;
        }
    }
}

__global__ __launch_bounds__(256) void k_gemm_nt128(int M, int N, int K, const uint16_t* __restrict__ A,
                                                    int64_t lda, const uint16_t* __restrict__ B, int64_t ldb,
                                                    Epi epi) {
    __shared__ __attribute__((aligned(16))) uint16_t As[2][BT][GK + GPAD];
    __shared__ __attribute__((aligned(16))) uint16_t Bs[2][BT][GK + GPAD];
    const int m0 = blockIdx.y * BT, n0 = blockIdx.x * BT;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;
    const int fr = lane & 15, fk = (lane >> 4) * 8;

    f32x4 acc[4][4];
    #pragma unroll
    for (int i = 0; i < 4; ++i)
        #pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

    uint4 ra[2], rb[2];
    fetch_rows(ra, A, lda, M, K, m0, 0);
    fetch_rows(rb, B, ldb, N, K, n0, 0);
    put_rows(As[0], ra);
    put_rows(Bs[0], rb);
    __syncthreads();
    int cur = 0;
    for (int k0 = 0; k0 < K; k0 += GK) {
        const bool more = k0 + GK < K;
        if (more) {
            fetch_rows(ra, A, lda, M, K, m0, k0 + GK);
            fetch_rows(rb, B, ldb, N, K, n0, k0 + GK);
        }
        bf16x8 a[4], b[4];
        #pragma unroll
        for (int i = 0; i < 4; ++i) a[i] = *(const bf16x8*)&As[cur][wm + 16 * i + fr][fk];
        #pragma unroll
        for (int j = 0; j < 4; ++j) b[j] = *(const bf16x8*)&Bs[cur][wn + 16 * j + fr][fk];
        #pragma unroll
        for (int i = 0; i < 4; ++i)
            #pragma unroll
            for (int j = 0; j < 4; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
        if (more) {
            put_rows(As[cur ^ 1], ra);
            put_rows(Bs[cur ^ 1], rb);
        }
        __syncthreads();
        cur ^= 1;
    }

    #pragma unroll

    for (int i = 0; i < 4; ++i)
        #pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int n = n0 + wn + 16 * j + fr;
            if (n >= N) continue;
            #pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int m = m0 + wm + 16 * i + (lane >> 4) * 4 + r;
                if (m < M) epilogue(epi, m, n, acc[i][j][r]);
            }
        }
}

static bool al16(const void* p) { return ((uintptr_t)p & 15) == 0; }

constexpr int kMaxSplits = 16;

// C = A B with the epilogue `epi`.  128x128 tiles when the grid still holds two
// workgroups per CU, else 64x64 tiles; plain FP32 products over a long K whose
// grid is small (weight gradients: K is the batch) are split over K into
// `split_ws` (kMaxSplits * M * N floats) and summed in split order.
labs_status gemm(bool a_k, bool b_k, int M, int N, int K, const uint16_t* A, int64_t lda,
                 const uint16_t* B, int64_t ldb, const Epi& epi, hipStream_t st, float* split_ws = nullptr) {
    if (M <= 0 || N <= 0) return LABS_OK;
    if ((lda & 7) || (ldb & 7) || !al16(A) || !al16(B))
        return invalid("internal: GEMM operands must be 16-byte aligned with strides of 8 elements");
    const long long t128 = (long long)((M + BT - 1) / BT) * ((N + BT - 1) / BT);
    if (a_k && b_k && t128 >= 512) {
        dim3 g2((N + BT - 1) / BT, (M + BT - 1) / BT);
        hipLaunchKernelGGL(k_gemm_nt128, g2, dim3(256), 0, st, M, N, K, A, lda, B, ldb, epi);
        LABS_LAUNCHED("k_gemm_nt128");
        return LABS_OK;
    }
    const long long tiles = (long long)((M + GT - 1) / GT) * ((N + GT - 1) / GT);
    int splits = 1, kchunk = (K + GK - 1) / GK * GK;
    Epi e = epi;
    if (epi.kind == EPI_F32 && split_ws && tiles < 512 && K >= 2 * 256) {
        splits = (int)((512 + tiles - 1) / tiles);
        if (splits > kMaxSplits) splits = kMaxSplits;
        if (splits > K / 256) splits = K / 256;
        kchunk = ((K + splits - 1) / splits + GK - 1) / GK * GK;
        splits = (K + kchunk - 1) / kchunk;
        e.out_f = split_ws;
        e.ldf = N;
        e.zstride = (int64_t)M * N;
    }
    dim3 grid((N + GT - 1) / GT, (M + GT - 1) / GT, splits);
    if (a_k && b_k)
        hipLaunchKernelGGL((k_gemm<true, true>), grid, dim3(256), 0, st, M, N, K, kchunk, A, lda, B, ldb, e);
    else if (a_k && !b_k)
        hipLaunchKernelGGL((k_gemm<true, false>), grid, dim3(256), 0, st, M, N, K, kchunk, A, lda, B, ldb, e);
    else if (!a_k && !b_k)
        hipLaunchKernelGGL((k_gemm<false, false>), grid, dim3(256), 0, st, M, N, K, kchunk, A, lda, B, ldb, e);
    else
        hipLaunchKernelGGL((k_gemm<false, true>), grid, dim3(256), 0, st, M, N, K, kchunk, A, lda, B, ldb, e);
    LABS_LAUNCHED("k_gemm");
    if (splits > 1) {
        const int64_t total = (int64_t)M * N;
        hipLaunchKernelGGL(k_sum_splits, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, M, N, splits,
                           split_ws, epi.out_f, epi.ldf);
        LABS_LAUNCHED("k_sum_splits");
    }
    return LABS_OK;
}

// ------------------------------------------------------------------ features
// x = (s_1..s_L as +1/-1, C_{2m}/(L-2m) for m = 1..k, zeros to ld_in), bf16.
// C_j = (L-j) - 2 * popcount(b XOR (b << j)) over the L-j overlapping bits of
// the packed string b (bit set for +1).  One wave per sequence.
__global__ __launch_bounds__(256) void k_features(int L, int W, int64_t n, const uint32_t* __restrict__ seqs,
                                                  uint16_t* __restrict__ X, int ld_in) {
    __shared__ uint32_t sw[4][33];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t r = (int64_t)blockIdx.x * 4 + wv;
    const bool live = r < n;
    if (live && lane < W) sw[wv][lane] = seqs[r * W + lane];
    if (lane == 0) sw[wv][W] = 0;
    __syncthreads();
    if (!live) return;
    const uint32_t* u = sw[wv];
    uint16_t* x = X + r * ld_in;
    const int k = (L - 1) / 2;
    for (int i = lane; i < ld_in; i += 64) {
        uint16_t v = 0;
        if (i < L) {
            v = ((u[i >> 5] >> (31 - (i & 31))) & 1) ? (uint16_t)0x3F80 : (uint16_t)0xBF80;
        } else if (i < L + k) {
            const int m = i - L + 1, j = 2 * m, len = L - j;
            const int q = j >> 5, sh = j & 31;
            int pc = 0;
            for (int w = 0; w * 32 < len; ++w) {
                const uint32_t hi = u[w + q];
                const uint32_t lo = (w + q + 1 < W) ? u[w + q + 1] : 0u;
                const uint32_t sft = sh ? ((hi << sh) | (lo >> (32 - sh))) : hi;
                uint32_t d = u[w] ^ sft;
                const int rem = len - w * 32;
                if (rem < 32) d &= ~(0xFFFFFFFFu >> rem);
                pc += __popc(d);
            }
            const int c = len - 2 * pc;
            v = f2bf((float)c / (float)len);
        }
        x[i] = v;
    }
}

// ------------------------------------------------------------------ cross-entropy
// One wave per row: softmax over the admissible logits (mask bit j set, or j the
// label), loss = logsumexp - z_label; dz = (softmax - onehot) / n on admissible
// entries, 0 elsewhere (pads included).
__device__ __forceinline__ float wave_max_f(float v) {
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
    return v;
}
__device__ __forceinline__ float wave_sum_f(float v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

__global__ __launch_bounds__(256) void k_masked_ce(int64_t n, int d_out, int ld_out, int MW,
                                                   const float* __restrict__ z, const uint32_t* __restrict__ mask,
                                                   const int32_t* __restrict__ labels, float* __restrict__ dzf,
                                                   uint16_t* __restrict__ dzb, float* __restrict__ rowloss) {
    const int lane = threadIdx.x & 63;
    const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (r >= n) return;
    const float* zr = z + r * ld_out;
    const uint32_t* mr = mask + r * MW;
    const int lab = labels[r];
    constexpr int PER = 16;   // d_out <= 1024
    float zv[PER];
    bool ok[PER];
    float mx = -INFINITY;
    for (int c = 0; c < PER; ++c) {
        const int j = lane + 64 * c;
        ok[c] = j < d_out && (j == lab || ((mr[j >> 5] >> (j & 31)) & 1));
        zv[c] = ok[c] ? zr[j] : -INFINITY;
        mx = fmaxf(mx, zv[c]);
    }
    mx = wave_max_f(mx);
    float se = 0.f;
    for (int c = 0; c < PER; ++c) {
        zv[c] = ok[c] ? expf(zv[c] - mx) : 0.f;
        se += zv[c];
    }
    se = wave_sum_f(se);
    const float inv_n = 1.0f / (float)n;
    for (int c = 0; c < PER; ++c) {
        const int j = lane + 64 * c;
        if (j >= ld_out) break;
        float d = 0.f;
        if (ok[c]) d = (zv[c] / se - (j == lab ? 1.f : 0.f)) * inv_n;
        dzf[r * ld_out + j] = d;
        dzb[r * ld_out + j] = f2bf(d);
    }
    if (lane == 0) rowloss[r] = logf(se) + mx - ((lab >= 0 && lab < d_out) ? zr[lab] : 0.f);
}

// Mean of n values by one block, fixed summation order.
__global__ __launch_bounds__(256) void k_mean(int64_t n, const float* __restrict__ v, float* __restrict__ out) {
    __shared__ float part[256];
    float s = 0.f;
    const int64_t per = (n + 255) / 256;
    const int64_t b = threadIdx.x * per, e = (b + per < n) ? b + per : n;
    for (int64_t i = b; i < e; ++i) s += v[i];
    part[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = n > 0 ? part[0] / (float)n : 0.f;
}

// Column sums of an fp32 [rows x cols] matrix (row stride ld) in two passes:
// partial sums over row chunks, then a fixed-order sum of the partials.
constexpr int kColChunks = 64;
__global__ __launch_bounds__(256) void k_colsum_part(int64_t rows, int cols, int64_t ld, const float* __restrict__ D,
                                                     float* __restrict__ part) {
    __shared__ float red[4][64];
    const int c = blockIdx.x * 64 + (threadIdx.x & 63), g = threadIdx.x >> 6;
    const int64_t per = (rows + kColChunks - 1) / kColChunks;
    const int64_t rb = blockIdx.y * per, re = (rb + per < rows) ? rb + per : rows;
    float s = 0.f;
    if (c < cols)
        for (int64_t r = rb + g; r < re; r += 4) s += D[r * ld + c];
    red[g][threadIdx.x & 63] = s;
    __syncthreads();
    if (g == 0 && c < cols)
        part[(int64_t)blockIdx.y * cols + c] = red[0][threadIdx.x] + red[1][threadIdx.x] + red[2][threadIdx.x] +
                                                red[3][threadIdx.x];
}
__global__ __launch_bounds__(256) void k_colsum_final(int cols, const float* __restrict__ part, float* __restrict__ out) {
    const int c = blockIdx.x * 256 + threadIdx.x;
    if (c >= cols) return;
    float s = 0.f;
    for (int q = 0; q < kColChunks; ++q) s += part[(int64_t)q * cols + c];
    out[c] = s;
}

__global__ __launch_bounds__(256) void k_fill_f32(int64_t n, float* __restrict__ p, float v) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) p[i] = v;
}

// ------------------------------------------------------------------ Adam
// Kingma and Ba (2015), FP32 masters; every operation rounded separately
// (contraction into FMAs is switched off) so that a float32 host computation
// in the same order matches bit for bit.
__global__ __launch_bounds__(256) void k_adam(int64_t n, float* __restrict__ P, uint16_t* __restrict__ Pb,
                                              const float* __restrict__ G, float* __restrict__ M, float* __restrict__ V,
                                              float b1, float omb1, float b2, float omb2, float bc1, float bc2,
                                              float lr, float eps) {
#pragma clang fp contract(off)
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const float g = G[i];
        const float m = b1 * M[i] + omb1 * g;
        const float v = b2 * V[i] + (omb2 * g) * g;
        M[i] = m;
        V[i] = v;
        const float mh = m / bc1, vh = v / bc2;
        const float p = P[i] - (lr * mh) / (sqrtf(vh) + eps);   // sqrtf and '/' are correctly rounded
        P[i] = p;
        Pb[i] = f2bf(p);
    }
}

__global__ __launch_bounds__(256) void k_cast_bf16(int64_t n, const float* __restrict__ P, uint16_t* __restrict__ Pb) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) Pb[i] = f2bf(P[i]);
}

// ------------------------------------------------------------------ host side
static int grid_for(int64_t n) {
    int64_t g = (n + 255) / 256;
    if (g > 4096) g = 4096;
    return (int)(g < 1 ? 1 : g);
}

bool mlp_layout(int L, int hidden, labs_mlp_layout* o) {
    if (L < 5 || L > 1023 || (L & 1) == 0 || hidden < 64 || hidden > 1024 || (hidden & 63)) return false;
    const int k = (L - 1) / 2;
    o->L = L;
    o->k = k;
    o->d_in = L + k;
    o->d_out = k + 1;
    o->hidden = hidden;
    o->ld_in = (o->d_in + 63) / 64 * 64;
    o->ld_out = (o->d_out + 63) / 64 * 64;
    o->mask_words = (o->d_out + 31) / 32;
    int64_t off = 0;
    auto take = [&](int64_t cnt) { int64_t r = off; off += (cnt + 63) / 64 * 64; return r; };
    o->off_W1 = take((int64_t)hidden * o->ld_in);
    o->off_b1 = take(hidden);
    o->off_W2 = take((int64_t)hidden * hidden);
    o->off_b2 = take(hidden);
    o->off_W3 = take((int64_t)o->ld_out * hidden);
    o->off_b3 = take(o->ld_out);
    o->n_params = off;
    return true;
}

labs_status launch_features(int L, int64_t n, const uint32_t* seqs, uint16_t* X, int ld_in, hipStream_t st) {
    if (n <= 0) return LABS_OK;
    hipLaunchKernelGGL(k_features, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, st, L, words_of(L), n, seqs, X,
                       ld_in);
    LABS_LAUNCHED("k_features");
    return LABS_OK;
}

size_t mlp_forward_ws(const labs_mlp_layout& y, int64_t n) {
    return 2 * align_up((size_t)n * y.hidden * 2, 256) + 256;
}

labs_status mlp_forward(const labs_mlp_layout& y, const float* P, const uint16_t* Pb, int64_t n, const uint16_t* X,
                        float* logits, void* ws, size_t wsb, hipStream_t st) {
    if (n <= 0) return LABS_OK;
    Carve cv(ws, wsb);
    uint16_t* h1 = cv.take<uint16_t>((size_t)n * y.hidden);
    uint16_t* h2 = cv.take<uint16_t>((size_t)n * y.hidden);
    if (!cv.ok() || !h1) return LABS_E_NOMEM;
    Epi e{};
    e.kind = EPI_BIAS_GELU;
    e.out_b = h1;
    e.ldb = y.hidden;
    e.bias = P + y.off_b1;
    labs_status s = gemm(true, true, (int)n, y.hidden, y.d_in, X, y.ld_in, Pb + y.off_W1, y.ld_in, e, st);
    if (s) return s;
    e.out_b = h2;
    e.bias = P + y.off_b2;
    s = gemm(true, true, (int)n, y.hidden, y.hidden, h1, y.hidden, Pb + y.off_W2, y.hidden, e, st);
    if (s) return s;
    Epi z{};
    z.kind = EPI_BIAS_F32;
    z.out_f = logits;
    z.ldf = y.ld_out;
    z.bias = P + y.off_b3;
    return gemm(true, true, (int)n, y.d_out, y.hidden, h2, y.hidden, Pb + y.off_W3, y.hidden, z, st);
}

size_t mlp_grads_ws(const labs_mlp_layout& y, int64_t n) {
    const size_t H = (size_t)n * y.hidden, O = (size_t)n * y.ld_out;
    size_t b = 0;
    auto add = [&](size_t bytes) { b += align_up(bytes, 256); };
    add(H * 4); add(H * 2); add(H * 4); add(H * 2);   // a1 h1 a2 h2
    add(O * 4); add(O * 4); add(O * 2);               // z dz_f dz_b
    add(H * 4); add(H * 2); add(H * 4); add(H * 2);   // da2_f da2_b da1_f da1_b
    add((size_t)n * 4);                               // row losses
    add((size_t)kColChunks * (y.hidden > y.ld_out ? y.hidden : y.ld_out) * 4);
    add((size_t)kMaxSplits * y.hidden * (y.ld_in > y.hidden ? y.ld_in : y.hidden) * 4);   // split-K partials
    return b + 256;
}

static labs_status colsum(int64_t rows, int cols, int64_t ld, const float* D, float* part, float* out,
                          hipStream_t st) {
    hipLaunchKernelGGL(k_colsum_part, dim3((cols + 63) / 64, kColChunks), dim3(256), 0, st, rows, cols, ld, D, part);
    LABS_LAUNCHED("k_colsum_part");
    hipLaunchKernelGGL(k_colsum_final, dim3((cols + 255) / 256), dim3(256), 0, st, cols, part, out);
    LABS_LAUNCHED("k_colsum_final");
    return LABS_OK;
}

labs_status mlp_grads(const labs_mlp_layout& y, const float* P, const uint16_t* Pb, int64_t n, const uint16_t* X,
                      const uint32_t* mask, const int32_t* labels, float* G, float* loss, void* ws, size_t wsb,
                      hipStream_t st) {
    Carve cv(ws, wsb);
    const size_t H = (size_t)n * y.hidden, O = (size_t)n * y.ld_out;
    float* a1 = cv.take<float>(H);
    uint16_t* h1 = cv.take<uint16_t>(H);
    float* a2 = cv.take<float>(H);
    uint16_t* h2 = cv.take<uint16_t>(H);
    float* z = cv.take<float>(O);
    float* dzf = cv.take<float>(O);
    uint16_t* dzb = cv.take<uint16_t>(O);
    float* d2f = cv.take<float>(H);
    uint16_t* d2b = cv.take<uint16_t>(H);
    float* d1f = cv.take<float>(H);
    uint16_t* d1b = cv.take<uint16_t>(H);
    float* rl = cv.take<float>((size_t)n);
    float* part = cv.take<float>((size_t)kColChunks * (y.hidden > y.ld_out ? y.hidden : y.ld_out));
    float* splitw = cv.take<float>((size_t)kMaxSplits * y.hidden * (y.ld_in > y.hidden ? y.ld_in : y.hidden));
    if (!cv.ok() || !splitw) return LABS_E_NOMEM;

    hipLaunchKernelGGL(k_fill_f32, dim3(grid_for(y.n_params)), dim3(256), 0, st, y.n_params, G, 0.f);
    LABS_LAUNCHED("k_fill_f32");
    if (n <= 0) {
        hipLaunchKernelGGL(k_fill_f32, dim3(1), dim3(256), 0, st, (int64_t)1, loss, 0.f);
        LABS_LAUNCHED("k_fill_f32");
        return LABS_OK;
    }
    const int Hd = y.hidden;
    // forward, keeping pre-activations
    Epi e{};
    e.kind = EPI_BIAS_GELU;
    e.out_b = h1; e.ldb = Hd; e.bias = P + y.off_b1; e.pre = a1; e.ldp = Hd;
    labs_status s = gemm(true, true, (int)n, Hd, y.d_in, X, y.ld_in, Pb + y.off_W1, y.ld_in, e, st);
    if (s) return s;
    e.out_b = h2; e.bias = P + y.off_b2; e.pre = a2;
    if ((s = gemm(true, true, (int)n, Hd, Hd, h1, Hd, Pb + y.off_W2, Hd, e, st))) return s;
    Epi zf{};
    zf.kind = EPI_BIAS_F32; zf.out_f = z; zf.ldf = y.ld_out; zf.bias = P + y.off_b3;
    if ((s = gemm(true, true, (int)n, y.d_out, Hd, h2, Hd, Pb + y.off_W3, Hd, zf, st))) return s;
    // loss and dz
    hipLaunchKernelGGL(k_masked_ce, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, st, n, y.d_out, y.ld_out,
                       y.mask_words, z, mask, labels, dzf, dzb, rl);
    LABS_LAUNCHED("k_masked_ce");
    hipLaunchKernelGGL(k_mean, dim3(1), dim3(256), 0, st, n, rl, loss);
    LABS_LAUNCHED("k_mean");
    // layer 3: dW3 = dz^T h2, db3 = colsum dz, dh2 = dz W3 -> da2 = dh2 * gelu'(a2)
    Epi g{};
    g.kind = EPI_F32; g.out_f = G + y.off_W3; g.ldf = Hd;
    if ((s = gemm(false, false, y.d_out, Hd, (int)n, dzb, y.ld_out, h2, Hd, g, st, splitw))) return s;
    if ((s = colsum(n, y.d_out, y.ld_out, dzf, part, G + y.off_b3, st))) return s;
    Epi d{};
    d.kind = EPI_DGELU; d.out_f = d2f; d.ldf = Hd; d.out_b = d2b; d.ldb = Hd; d.pre = a2; d.ldp = Hd;
    if ((s = gemm(true, false, (int)n, Hd, y.d_out, dzb, y.ld_out, Pb + y.off_W3, Hd, d, st))) return s;
    // layer 2
    g.out_f = G + y.off_W2; g.ldf = Hd;
    if ((s = gemm(false, false, Hd, Hd, (int)n, d2b, Hd, h1, Hd, g, st, splitw))) return s;
    if ((s = colsum(n, Hd, Hd, d2f, part, G + y.off_b2, st))) return s;
    d.out_f = d1f; d.out_b = d1b; d.pre = a1;
    if ((s = gemm(true, false, (int)n, Hd, Hd, d2b, Hd, Pb + y.off_W2, Hd, d, st))) return s;
    // layer 1
    g.out_f = G + y.off_W1; g.ldf = y.ld_in;
    if ((s = gemm(false, false, Hd, y.d_in, (int)n, d1b, Hd, X, y.ld_in, g, st, splitw))) return s;
    return colsum(n, Hd, Hd, d1f, part, G + y.off_b1, st);
}

labs_status mlp_adam(const labs_mlp_layout& y, float* P, uint16_t* Pb, const float* G, float* M, float* V, int t,
                     double lr, double b1, double b2, double eps, hipStream_t st) {
    const float bc1 = (float)(1.0 - std::pow(b1, (double)t));
    const float bc2 = (float)(1.0 - std::pow(b2, (double)t));
    hipLaunchKernelGGL(k_adam, dim3(grid_for(y.n_params)), dim3(256), 0, st, y.n_params, P, Pb, G, M, V, (float)b1,
                       (float)(1.0 - b1), (float)b2, (float)(1.0 - b2), bc1, bc2, (float)lr, (float)eps);
    LABS_LAUNCHED("k_adam");
    return LABS_OK;
}

labs_status mlp_cast(const labs_mlp_layout& y, const float* P, uint16_t* Pb, hipStream_t st) {
    hipLaunchKernelGGL(k_cast_bf16, dim3(grid_for(y.n_params)), dim3(256), 0, st, y.n_params, P, Pb);
    LABS_LAUNCHED("k_cast_bf16");
    return LABS_OK;
}

}  // namespace labsdev
