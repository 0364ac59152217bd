/*
 * walsh_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously correct CPU implementation of what the S-box
 * Walsh-spectrum / nonlinearity path computes.  Only the test-suite, the
 * smoke check and the benchmark's CPU-baseline leg may load this library;
 * the product path (the HIP library) never links, calls or imports it, and
 * this file shares no code with it.
 *
 * Conventions (the readings of the paper that every routine below follows):
 *   - An n x m S-box is a table S[0 .. 2^n) of values < 2^m (bits at or
 *     above m are ignored).  Component function for output mask b is
 *     x -> parity(b & S[x])  (Section 3, Eq. 2: a linear combination of the
 *     coordinate functions f_i = bit i of S(x)).
 *   - Walsh spectrum (Section 3, Eq. 1, exponent read as <u,x> + <v,S(x)>):
 *        W(a, b) = sum_x (-1)^( parity(a & x) XOR parity(b & S[x]) ),
 *     for a in [0, 2^n), b in [0, 2^m).
 *   - Nonlinearity (Section 3, Eq. 3, with the all-zero output mask left
 *     out, as in Algorithms 1-3 which only carry the 2^m - 1 nonzero
 *     columns):
 *        NL = 2^(n-1) - (1/2) max_{b != 0, a} |W(a, b)|.
 *     Every W is congruent to 2^n mod 2, so the halving is exact.
 *   - Polarity truth table sign: bit 0 -> +1, bit 1 -> -1.
 *   - Fast transform (Algorithm 1 / Algorithm 3): radix-2 butterflies on
 *     index pairs (i, i + h) with (i & h) == 0, h = 1, 2, 4, ..., in natural
 *     (Sylvester) order, so output index == a.
 *   - Per-mask maximum |W| and per-mask nl value (the "var" array of
 *     Algorithms 2, 3 and 5), then the minimum over masks (Algorithm 6),
 *     starting from 2^(n-1) rather than the paper's fixed sentinel.
 *
 * Layouts of a stored spectrum:
 *   ORACLE_B_MAJOR (1): W[b * 2^n + a]  (the transposed matrix of Section 5.1)
 *   ORACLE_A_MAJOR (2): W[a * 2^m + b]  (the matrix of Algorithm 1)
 *
 * Every entry point returns 0 on success and -1 on an invalid argument.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_B_MAJOR 1
#define ORACLE_A_MAJOR 2

/* parity of the set bits of v, by clearing the lowest set bit until none is left */
static int parity32(uint32_t v) {
    int p = 0;
    while (v) {
        v &= v - 1u;
        p ^= 1;
    }
    return p;
}

static int valid_nm(int n, int m) {
    return n >= 1 && n <= 24 && m >= 1 && m <= 24;
}

/* Component function of mask b as a polarity column: f[x] = (-1)^parity(b & S[x]). */
static void polarity_column(const uint32_t* S, int n, uint32_t b, int32_t* f) {
    const uint32_t N = 1u << n;
    for (uint32_t x = 0; x < N; ++x) f[x] = parity32(b & S[x]) ? -1 : 1;
}

/* In-place fast Walsh-Hadamard transform of length 2^n (Algorithm 1 on one column). */
static void fwht_inplace(int32_t* f, int n) {
    const uint32_t N = 1u << n;
    for (uint32_t h = 1; h < N; h <<= 1) {
        for (uint32_t i = 0; i < N; i += 2 * h) {
            for (uint32_t j = i; j < i + h; ++j) {
                const int32_t u = f[j];
                const int32_t v = f[j + h];
                f[j] = u + v;
                f[j + h] = u - v;
            }
        }
    }
}

static int32_t max_abs(const int32_t* f, uint32_t N) {
    int32_t best = 0;
    for (uint32_t i = 0; i < N; ++i) {
        const int32_t a = f[i] < 0 ? -f[i] : f[i];
        if (a > best) best = a;
    }
    return best;
}

/*
 * One Walsh column: col[a] = W(a, b) for a in [0, 2^n).  Any b (also 0).
 */
int oracle_walsh_column(const uint32_t* S, int n, int m, uint32_t b, int32_t* col) {
    if (!S || !col || !valid_nm(n, m) || (m < 32 && b >= (1u << m))) return -1;
    polarity_column(S, n, b, col);
    fwht_inplace(col, n);
    return 0;
}

/*
 * One coefficient straight from the definition (Eq. 1), O(2^n).
 */
int32_t oracle_walsh_entry(const uint32_t* S, int n, uint32_t a, uint32_t b) {
    const uint32_t N = 1u << n;
    int32_t sum = 0;
    for (uint32_t x = 0; x < N; ++x) sum += (parity32(a & x) ^ parity32(b & S[x])) ? -1 : 1;
    return sum;
}

/*
 * Fused path (Algorithm 3 + Algorithm 6): for every nonzero mask b,
 * transform its column, keep only max_a |W(a,b)|; then NL is the minimum
 * of (2^n - max) / 2 over b.  maxabs (2^m entries, may be NULL) receives
 * the per-mask maximum, with maxabs[0] = 2^n (row b = 0 is 2^n at a = 0).
 * nthreads <= 1 runs serially; larger values split the masks into
 * contiguous blocks, one per OpenMP thread (the split of Algorithm 5).
 */
int oracle_walsh_nl(const uint32_t* S, int n, int m, int32_t* maxabs, int32_t* nl, int nthreads) {
    if (!S || !nl || !valid_nm(n, m)) return -1;
    const uint32_t N = 1u << n;
    const int64_t M = (int64_t)1 << m;
    int32_t best = (int32_t)(N >> 1);
    int failed = 0;
    if (maxabs) maxabs[0] = (int32_t)N;
    if (nthreads < 1) nthreads = 1;
#pragma omp parallel num_threads(nthreads) reduction(min : best) reduction(| : failed)
    {
        int32_t* f = (int32_t*)malloc(sizeof(int32_t) * N);
        if (!f) {
            failed = 1;
        } else {
#pragma omp for schedule(static)
            for (int64_t b = 1; b < M; ++b) {
                polarity_column(S, n, (uint32_t)b, f);
                fwht_inplace(f, n);
                const int32_t mx = max_abs(f, N);
                if (maxabs) maxabs[b] = mx;
                const int32_t nlb = ((int32_t)N - mx) >> 1;
                if (nlb < best) best = nlb;
            }
            free(f);
        }
    }
    if (failed) return -1;
    *nl = best;
    return 0;
}

/*
 * Same fused path restricted to the masks listed in bs[0..count) (all
 * nonzero); maxabs_out[i] receives max_a |W(a, bs[i])|.  Used to time or
 * check a bounded sample of a large S-box.
 */
int oracle_walsh_maxabs_masks(const uint32_t* S, int n, int m, const uint32_t* bs, int64_t count,
                              int32_t* maxabs_out, int nthreads) {
    if (!S || !bs || !maxabs_out || !valid_nm(n, m) || count < 0) return -1;
    const uint32_t N = 1u << n;
    int failed = 0;
    if (nthreads < 1) nthreads = 1;
#pragma omp parallel num_threads(nthreads) reduction(| : failed)
    {
        int32_t* f = (int32_t*)malloc(sizeof(int32_t) * N);
        if (!f) {
            failed = 1;
        } else {
#pragma omp for schedule(static)
            for (int64_t i = 0; i < count; ++i) {
                polarity_column(S, n, bs[i], f);
                fwht_inplace(f, n);
                maxabs_out[i] = max_abs(f, N);
            }
            free(f);
        }
    }
    return failed ? -1 : 0;
}

/*
 * Full spectrum (all 2^(n+m) coefficients, row b = 0 included) in the
 * requested layout.  W must hold 2^(n+m) int32.  nthreads <= 1 runs
 * serially; larger values split the masks into contiguous blocks, one per
 * thread (the partition of Algorithms 4 and 5), each thread transforming
 * its own columns with a buffer of its own.
 */
int oracle_spectrum_threads(const uint32_t* S, int n, int m, int layout, int32_t* W, int nthreads) {
    if (!S || !W || !valid_nm(n, m) || n + m > 32) return -1;
    if (layout != ORACLE_B_MAJOR && layout != ORACLE_A_MAJOR) return -1;
    const uint32_t N = 1u << n;
    const uint32_t M = 1u << m;
    int failed = 0;
    if (nthreads < 1) nthreads = 1;
#pragma omp parallel num_threads(nthreads) reduction(| : failed)
    {
        int32_t* f = (int32_t*)malloc(sizeof(int32_t) * N);
        if (!f) {
            failed = 1;
        } else {
#pragma omp for schedule(static)
            for (int64_t bb = 0; bb < (int64_t)M; ++bb) {
                const uint32_t b = (uint32_t)bb;
                polarity_column(S, n, b, f);
                fwht_inplace(f, n);
                for (uint32_t a = 0; a < N; ++a) {
                    if (layout == ORACLE_B_MAJOR)
                        W[(size_t)b * N + a] = f[a];
                    else
                        W[(size_t)a * M + b] = f[a];
                }
            }
            free(f);
        }
    }
    return failed ? -1 : 0;
}

int oracle_spectrum(const uint32_t* S, int n, int m, int layout, int32_t* W) {
    return oracle_spectrum_threads(S, n, m, layout, W, 1);
}

/*
 * Unfused path (Algorithm 2, then Algorithm 6): re-scan a stored spectrum
 * for the per-mask maximum and the nonlinearity.  maxabs may be NULL.
 * nthreads as for oracle_spectrum_threads (each thread scans a contiguous
 * block of masks).
 */
int oracle_nl_from_spectrum_threads(const int32_t* W, int n, int m, int layout, int32_t* maxabs, int32_t* nl,
                                    int nthreads) {
    if (!W || !nl || !valid_nm(n, m) || n + m > 32) return -1;
    if (layout != ORACLE_B_MAJOR && layout != ORACLE_A_MAJOR) return -1;
    const uint32_t N = 1u << n;
    const uint32_t M = 1u << m;
    int32_t best = (int32_t)(N >> 1);
    if (nthreads < 1) nthreads = 1;
#pragma omp parallel for num_threads(nthreads) schedule(static) reduction(min : best)
    for (int64_t bb = 0; bb < (int64_t)M; ++bb) {
        const uint32_t b = (uint32_t)bb;
        int32_t mx = 0;
        for (uint32_t a = 0; a < N; ++a) {
            const int32_t w = layout == ORACLE_B_MAJOR ? W[(size_t)b * N + a] : W[(size_t)a * M + b];
            const int32_t aw = w < 0 ? -w : w;
            if (aw > mx) mx = aw;
        }
        if (maxabs) maxabs[b] = mx;
        if (b == 0) continue;
        const int32_t nlb = ((int32_t)N - mx) >> 1;
        if (nlb < best) best = nlb;
    }
    *nl = best;
    return 0;
}

int oracle_nl_from_spectrum(const int32_t* W, int n, int m, int layout, int32_t* maxabs, int32_t* nl) {
    return oracle_nl_from_spectrum_threads(W, n, m, layout, maxabs, nl, 1);
}

/*
 * Further criteria of the component functions, the future work named in the
 * paper's conclusion (Section 7), each from its textbook definition:
 *   balancedness:        W(0, b) == 0 (the component b.S takes 0 and 1 equally often);
 *   correlation immunity: order t if W(a, b) == 0 for every a with 1 <= wt(a) <= t;
 *                         resiliency order = that t when also balanced, else -1;
 *   autocorrelation:     r_b(d) = sum_x (-1)^(f_b(x) XOR f_b(x XOR d));
 *   absolute indicator:  max over d != 0 of |r_b(d)|;
 *   propagation order:   k if r_b(d) == 0 for every d with 1 <= wt(d) <= k.
 * Aggregates take the worst case over nonzero masks b.  Per-mask outputs
 * (each may be NULL, 2^m entries, entry 0 left as 0):
 *   w0[b]     = W(0, b)
 *   minwt[b]  = min wt(a) over a != 0 with W(a, b) != 0   (n + 1 if none)
 *   acmax[b]  = max_{d != 0} |r_b(d)|
 *   pcwt[b]   = min wt(d) over d != 0 with r_b(d) != 0   (n + 1 if none)
 * summary[0..5] = {NL, #unbalanced masks, CI order, resiliency order,
 *                  absolute indicator, propagation order}.
 * The autocorrelation is summed directly from its definition (O(4^n) per mask).
 */
static int weight32(uint32_t v) {
    int w = 0;
    while (v) {
        v &= v - 1u;
        ++w;
    }
    return w;
}

int oracle_criteria(const uint32_t* S, int n, int m, int32_t* w0, int32_t* minwt, int32_t* acmax,
                    int32_t* pcwt, int32_t* summary, int nthreads) {
    if (!S || !summary || !valid_nm(n, m) || n > 16) return -1;
    const uint32_t N = 1u << n;
    const int64_t M = (int64_t)1 << m;
    int32_t nl = (int32_t)(N >> 1), unbal = 0, ciw = n + 1, ac = 0, pcw = n + 1;
    int failed = 0;
    if (nthreads < 1) nthreads = 1;
    if (w0) w0[0] = 0;
    if (minwt) minwt[0] = 0;
    if (acmax) acmax[0] = 0;
    if (pcwt) pcwt[0] = 0;
#pragma omp parallel num_threads(nthreads) reduction(min : nl, ciw, pcw) reduction(max : ac) \
    reduction(+ : unbal) reduction(| : failed)
    {
        int32_t* f = (int32_t*)malloc(sizeof(int32_t) * N);
        int8_t* g = (int8_t*)malloc(N);
        if (!f || !g) {
            failed = 1;
        } else {
#pragma omp for schedule(dynamic, 1)
            for (int64_t b = 1; b < M; ++b) {
                for (uint32_t x = 0; x < N; ++x) g[x] = (int8_t)parity32((uint32_t)b & S[x]);
                polarity_column(S, n, (uint32_t)b, f);
                fwht_inplace(f, n);
                const int32_t mx = max_abs(f, N);
                int mw = n + 1;
                for (uint32_t a = 1; a < N; ++a)
                    if (f[a] != 0 && weight32(a) < mw) mw = weight32(a);
                int32_t amax = 0;
                int pw = n + 1;
                for (uint32_t d = 1; d < N; ++d) {
                    int32_t r = 0;
                    for (uint32_t x = 0; x < N; ++x) r += (g[x] ^ g[x ^ d]) ? -1 : 1;
                    const int32_t ar = r < 0 ? -r : r;
                    if (ar > amax) amax = ar;
                    if (r != 0 && weight32(d) < pw) pw = weight32(d);
                }
                if (w0) w0[b] = f[0];
                if (minwt) minwt[b] = mw;
                if (acmax) acmax[b] = amax;
                if (pcwt) pcwt[b] = pw;
                const int32_t nlb = ((int32_t)N - mx) >> 1;
                if (nlb < nl) nl = nlb;
                if (f[0] != 0) unbal += 1;
                if (mw < ciw) ciw = mw;
                if (amax > ac) ac = amax;
                if (pw < pcw) pcw = pw;
            }
        }
        free(f);
        free(g);
    }
    if (failed) return -1;
    summary[0] = nl;
    summary[1] = unbal;
    summary[2] = ciw - 1;
    summary[3] = unbal == 0 ? ciw - 1 : -1;
    summary[4] = ac;
    summary[5] = pcw - 1;
    return 0;
}

/* Autocorrelation column r_b(d) for all d, from the definition. */
int oracle_autocorrelation(const uint32_t* S, int n, int m, uint32_t b, int32_t* r) {
    if (!S || !r || !valid_nm(n, m) || n > 16) return -1;
    const uint32_t N = 1u << n;
    for (uint32_t d = 0; d < N; ++d) {
        int32_t acc = 0;
        for (uint32_t x = 0; x < N; ++x) acc += (parity32(b & S[x]) ^ parity32(b & S[x ^ d])) ? -1 : 1;
        r[d] = acc;
    }
    return 0;
}

/*
 * Histogram of |W| over the nonzero masks: the distribution of the entries
 * of the Walsh matrix of Section 3, Eq. 1 (equivalently of the linear
 * approximation table W/2), columns b = 1 .. 2^m - 1 as in Eq. 3:
 *   hist[k] = #{(a, b) : b != 0, |W(a, b)| = 2k},   k = 0 .. 2^(n-1).
 * One transform per mask as in Algorithm 1, then a count; threads split the
 * masks and their private counts are added at the end.
 */
int oracle_walsh_histogram(const uint32_t* S, int n, int m, uint64_t* hist, int nthreads) {
    if (!S || !hist || !valid_nm(n, m) || n > 20) return -1;
    const uint32_t N = 1u << n;
    const uint32_t NB = (N >> 1) + 1u;
    const int64_t M = (int64_t)1 << m;
    int failed = 0;
    if (nthreads < 1) nthreads = 1;
    memset(hist, 0, sizeof(uint64_t) * NB);
#pragma omp parallel num_threads(nthreads) reduction(| : failed)
    {
        int32_t* f = (int32_t*)malloc(sizeof(int32_t) * N);
        uint64_t* h = (uint64_t*)calloc(NB, sizeof(uint64_t));
        if (!f || !h) {
            failed = 1;
        } else {
#pragma omp for schedule(dynamic, 1)
            for (int64_t b = 1; b < M; ++b) {
                polarity_column(S, n, (uint32_t)b, f);
                fwht_inplace(f, n);
                for (uint32_t a = 0; a < N; ++a) {
                    const int32_t w = f[a] < 0 ? -f[a] : f[a];
                    h[(uint32_t)w >> 1] += 1;
                }
            }
#pragma omp critical
            for (uint32_t k = 0; k < NB; ++k) hist[k] += h[k];
        }
        free(f);
        free(h);
    }
    return failed ? -1 : 0;
}

/* r_b(e_i) = sum_x (-1)^parity(b & (S[x] ^ S[x ^ e_i])), from the definition. */
static int32_t unit_autocorrelation(const uint32_t* S, int n, uint32_t mmask, int i, uint32_t b) {
    const uint32_t N = 1u << n;
    int32_t acc = 0;
    for (uint32_t x = 0; x < N; ++x) acc += parity32(b & (S[x] ^ S[x ^ (1u << i)]) & mmask) ? -1 : 1;
    return acc;
}

/*
 * Avalanche and bit independence (criteria named as future work in
 * Section 7), from the autocorrelation of the components at the unit input
 * differences e_i = 2^i:
 *   r[i * 2^m + b] = sum_x (-1)^parity(b & (S[x] ^ S[x ^ e_i])),  i < n, b < 2^m,
 * summed from its definition (all of it when r is given; otherwise only the
 * entries the summary needs).  Flipping input bit i flips the component of
 * mask b with probability (1 - r / 2^n) / 2.  summary[0..2]:
 *   [0] max_{i, j} |r_{e_j}(e_i)|: strict avalanche of each output bit
 *       (0 when every output bit flips with probability exactly 1/2);
 *   [1] max_{i, j < k} |r_{e_j ^ e_k}(e_i)|: the same for the XOR of two output
 *       bits, the avalanche half of bit independence (-1 if m < 2);
 *   [2] min_{j < k} NL(x -> bit j of S(x) XOR bit k of S(x)), each from its own
 *       transform (Eq. 3 for one mask): the nonlinearity half of bit
 *       independence (-1 if m < 2).
 */
int oracle_avalanche(const uint32_t* S, int n, int m, int32_t* r, int32_t* summary, int nthreads) {
    if (!S || !summary || !valid_nm(n, m) || n > 16 || m > 16) return -1;
    const uint32_t N = 1u << n;
    const uint32_t M = 1u << m;
    const uint32_t mmask = M - 1u;
    if (nthreads < 1) nthreads = 1;
    if (r) {
#pragma omp parallel for num_threads(nthreads) schedule(dynamic, 1) collapse(2)
        for (int i = 0; i < n; ++i)
            for (int64_t b = 0; b < (int64_t)M; ++b)
                r[(size_t)i * M + (uint32_t)b] = unit_autocorrelation(S, n, mmask, i, (uint32_t)b);
    }
    int32_t sac = 0, bic = m >= 2 ? 0 : -1, bicnl = m >= 2 ? (int32_t)(N >> 1) : -1;
#pragma omp parallel for num_threads(nthreads) schedule(dynamic, 1) reduction(max : sac, bic)
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < m; ++j) {
            const uint32_t bj = 1u << j;
            const int32_t v = r ? r[(size_t)i * M + bj] : unit_autocorrelation(S, n, mmask, i, bj);
            if ((v < 0 ? -v : v) > sac) sac = v < 0 ? -v : v;
            for (int k = j + 1; k < m; ++k) {
                const uint32_t bjk = bj | (1u << k);
                const int32_t u = r ? r[(size_t)i * M + bjk] : unit_autocorrelation(S, n, mmask, i, bjk);
                if ((u < 0 ? -u : u) > bic) bic = u < 0 ? -u : u;
            }
        }
    if (m >= 2) {
        int32_t* f = (int32_t*)malloc(sizeof(int32_t) * N);
        if (!f) return -1;
        for (int j = 0; j < m; ++j)
            for (int k = j + 1; k < m; ++k) {
                polarity_column(S, n, (1u << j) | (1u << k), f);
                fwht_inplace(f, n);
                const int32_t nlb = ((int32_t)N - max_abs(f, N)) >> 1;
                if (nlb < bicnl) bicnl = nlb;
            }
        free(f);
    }
    summary[0] = sac;
    summary[1] = bic;
    summary[2] = bicnl;
    return 0;
}

/* r[i * count + j] = r_{bs[j]}(e_i) for i < n, from the definition (a sample of masks). */
int oracle_unit_autocorrelation_masks(const uint32_t* S, int n, int m, const uint32_t* bs, int64_t count,
                                      int32_t* r, int nthreads) {
    if (!S || !bs || !r || !valid_nm(n, m) || n > 20 || count < 0) return -1;
    const uint32_t mmask = (m >= 32) ? 0xffffffffu : ((1u << m) - 1u);
    if (nthreads < 1) nthreads = 1;
#pragma omp parallel for num_threads(nthreads) schedule(dynamic, 1) collapse(2)
    for (int i = 0; i < n; ++i)
        for (int64_t j = 0; j < count; ++j) r[(size_t)i * count + j] = unit_autocorrelation(S, n, mmask, i, bs[j]);
    return 0;
}
