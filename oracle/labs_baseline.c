/*
 * labs_baseline.c -- CPU baseline of the first step: the tabu walker of
 * Sec. 3, Algorithm 1, with its linear-time neighbour evaluation, one walker per
 * OpenMP thread.
 *
 * TEST AND BENCHMARK INFRASTRUCTURE ONLY: the benchmark times it on the host
 * cores as the CPU baseline, and a CPU test checks its trajectories against the
 * definitional oracle (labs_oracle.c).  It shares no code with the HIP path or
 * with labs_oracle.c.
 *
 * Method (Psenicnik, Mlinaric, Brest, Boskovic, arXiv 2409.07222):
 *   Sec. 1       C_k(S) = sum_{i=1}^{L-k} s_i s_{i+k}, E = sum_k C_k^2.
 *   Eq. (2)      skew-symmetry for L = 2k+1: s_{k+1+i} = (-1)^i s_{k+1-i}; every
 *                odd-lag C vanishes, and flipping a free element together with
 *                its Eq. (2) partner keeps the sequence skew-symmetric.
 *   Eq. (3)      free elements s_{p+1}..s_{k+1} after a prefix of p.
 *   Sec. 3       the walker keeps its C table and evaluates each neighbour in
 *                time linear in L: flipping the set {a, b} (b = L+1-a, or a
 *                alone at the centre) changes lag d by
 *                  dC_d = -2 s_a t_{a,d} - 2 s_b t_{b,d} + 4 s_a s_b [d = b-a],
 *                  t_{x,d} = s_{x+d} [x+d <= L] + s_{x-d} [x-d >= 1]
 *                (the last term restores the product s_a s_b, whose two
 *                factors both flip), and dE = sum_d dC_d (2 C_d + dC_d); only
 *                even d contribute.  The taken move applies dC to the table.
 * Walker readings (the same as the library's and the oracle's): SplitMix64
 * (Steele, Lea, Flood 2014) stream per (seed, L, walker); draw i-1 sets s_i for
 * i = 1..k+1 (+1 when its top bit is set; s_1 = +1 when p >= 1), draw k+1 the
 * tenure lo + draw mod (hi-lo+1); at step t every free a is evaluated, the
 * admissible ones (tabu_until[a] < t) compete on (dE, a), the least is taken even
 * uphill and becomes tabu until t + tenure; no admissible move stops the walk.
 *
 * Plain C99 + OpenMP; built -O3 -march=native -fopenmp for the host it runs on.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static uint64_t bl_mix(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* One walker; traj (nullable) gets E after each step, -1 after a stop.
 * Returns the number of steps taken. */
static int32_t bl_walk_one(int32_t L, int32_t p, int32_t steps, int32_t lo, int32_t hi, uint64_t seed,
                           int64_t w, int32_t* traj, int32_t* final_E, int32_t* best_E)
{
    const int32_t k = (L - 1) / 2;
    const int32_t nf = k + 1 - p;
    /* s[1..L] with zero padding on both sides so that t_{x,d} needs no bounds test */
    int8_t* buf = (int8_t*)calloc((size_t)(3 * L + 2), 1);
    int8_t* s = buf + L;
    int32_t* C = (int32_t*)calloc((size_t)(L + 1), sizeof(int32_t));
    int32_t* dC = (int32_t*)malloc((size_t)(L + 1) * sizeof(int32_t));
    int32_t* tabu = (int32_t*)calloc((size_t)(nf + 1), sizeof(int32_t));

    uint64_t st = bl_mix(seed ^ bl_mix(((uint64_t)(uint32_t)L << 32) ^ (uint64_t)(w + 1)));
    for (int32_t i = 1; i <= k + 1; ++i) {
        st += 0x9E3779B97F4A7C15ull;
        s[i] = (bl_mix(st) >> 63) ? 1 : -1;
    }
    if (p >= 1) s[1] = 1;
    for (int32_t i = 1; i <= k; ++i) s[k + 1 + i] = (i & 1) ? (int8_t)-s[k + 1 - i] : s[k + 1 - i];
    st += 0x9E3779B97F4A7C15ull;
    const int32_t tenure = lo + (int32_t)(bl_mix(st) % (uint64_t)(hi - lo + 1));

    int32_t E = 0;
    for (int32_t d = 2; d <= L - 1; d += 2) {
        int32_t c = 0;
        for (int32_t i = 1; i + d <= L; ++i) c += s[i] * s[i + d];
        C[d] = c;
        E += c * c;
    }
    int32_t bE = E;
    int32_t t = 1;
    for (; t <= steps; ++t) {
        int32_t best_a = -1, best_d = 0;
        for (int32_t a = p + 1; a <= k + 1; ++a) {
            const int32_t b = L + 1 - a;
            const int32_t sa = s[a], sb = s[b];
            int32_t de = 0;
            if (a == b) {
                for (int32_t d = 2; d <= L - 1; d += 2) {
                    const int32_t g = -2 * sa * (s[a + d] + s[a - d]);
                    de += g * (2 * C[d] + g);
                }
            } else {
                for (int32_t d = 2; d <= L - 1; d += 2) {
                    int32_t g = -2 * sa * (s[a + d] + s[a - d]) - 2 * sb * (s[b + d] + s[b - d]);
                    if (d == b - a) g += 4 * sa * sb;
                    de += g * (2 * C[d] + g);
                }
            }
            if (tabu[a - p] >= t) continue;
            if (best_a < 0 || de < best_d) {
                best_a = a;
                best_d = de;
            }
        }
        if (best_a < 0) break;
        {
            const int32_t a = best_a, b = L + 1 - a;
            const int32_t sa = s[a], sb = s[b];
            for (int32_t d = 2; d <= L - 1; d += 2) {
                int32_t g;
                if (a == b) g = -2 * sa * (s[a + d] + s[a - d]);
                else {
                    g = -2 * sa * (s[a + d] + s[a - d]) - 2 * sb * (s[b + d] + s[b - d]);
                    if (d == b - a) g += 4 * sa * sb;
                }
                dC[d] = g;
            }
            for (int32_t d = 2; d <= L - 1; d += 2) C[d] += dC[d];
            s[a] = (int8_t)-sa;
            if (b != a) s[b] = (int8_t)-sb;
        }
        E += best_d;
        tabu[best_a - p] = t + tenure;
        if (E < bE) bE = E;
        if (traj) traj[t - 1] = E;
    }
    const int32_t taken = t - 1;
    if (traj)
        for (; t <= steps; ++t) traj[t - 1] = -1;
    *final_E = E;
    *best_E = bE;
    free(buf);
    free(C);
    free(dC);
    free(tabu);
    return taken;
}

/* n walkers with ids walker_begin..walker_begin+n-1 on `threads` OpenMP threads
 * (<= 0: the runtime's default).  traj [n*steps] (nullable), final_E [n],
 * best_E [n]; *flip_evals = sum over walkers of steps taken x free positions.
 * Returns the number of threads that ran. */
int32_t bl_walk(int32_t L, int32_t p, int32_t steps, int32_t lo, int32_t hi, uint64_t seed,
                int64_t walker_begin, int64_t n, int32_t threads, int32_t* traj, int32_t* final_E,
                int32_t* best_E, int64_t* flip_evals)
{
    const int32_t nf = (L - 1) / 2 + 1 - p;
    int64_t evals = 0;
    int32_t used = 1;
#ifdef _OPENMP
    if (threads > 0) omp_set_num_threads(threads);
#pragma omp parallel reduction(+ : evals)
    {
#pragma omp single
        used = omp_get_num_threads();
#pragma omp for schedule(dynamic, 1)
        for (int64_t j = 0; j < n; ++j) {
            const int32_t taken = bl_walk_one(L, p, steps, lo, hi, seed, walker_begin + j,
                                              traj ? traj + j * (int64_t)steps : NULL, &final_E[j], &best_E[j]);
            evals += (int64_t)taken * nf;
        }
    }
#else
    (void)threads;
    for (int64_t j = 0; j < n; ++j) {
        const int32_t taken = bl_walk_one(L, p, steps, lo, hi, seed, walker_begin + j,
                                          traj ? traj + j * (int64_t)steps : NULL, &final_E[j], &best_E[j]);
        evals += (int64_t)taken * nf;
    }
#endif
    *flip_evals = evals;
    return used;
}
