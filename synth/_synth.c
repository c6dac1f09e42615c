/*
 * _synth.c -- multi-threaded kernels of the seeded input generators in
 * gen.py: the inverse-CDF lookup of the Zipf index sampler, exact removal of
 * repeated coordinate tuples (first occurrence kept, in draw order), and the
 * values of the planted low-rank tensor at given coordinates.
 *
 * Data synthesis only: nothing here belongs to the SGD sweep. The random
 * numbers are drawn by numpy (gen.py) and passed in, so the output depends
 * only on them, never on the thread count.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

/* out[i] = label[min(#{k : cdf[k] <= u[i]}, I - 1)]: numpy's
 * searchsorted(cdf, u, side="right") through a guide table. guide[b] counts
 * the cdf entries <= b / K; a lookup starts one bucket early (so rounding of
 * u * K can only make it start too low) and walks forward. */
int syn_zipf_lookup(const double *cdf, int64_t I, const int32_t *label,
                    const double *u, int64_t n, int32_t *out)
{
    const int64_t K = 2 * I;
    int64_t *guide = malloc(sizeof(int64_t) * (size_t)(K + 1));
    if (!guide) return -1;
    int64_t k = 0;
    for (int64_t b = 0; b <= K; ++b) {
        const double edge = (double)b / (double)K;
        while (k < I && cdf[k] <= edge) ++k;
        guide[b] = k;
    }
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        const double x = u[i];
        int64_t b = (int64_t)(x * (double)K) - 1;
        if (b < 0) b = 0;
        if (b > K) b = K;
        int64_t j = guide[b];
        while (j < I && cdf[j] <= x) ++j;
        if (j > I - 1) j = I - 1;
        out[i] = label[j];
    }
    free(guide);
    return 0;
}

static inline uint64_t mix64(uint64_t z)
{
    /* SplitMix64 finaliser (Steele, Lea and Flood, 2014) */
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

static inline int same_tuple(int N, const int32_t *idx, int64_t n, int64_t a,
                             int64_t b)
{
    for (int m = 0; m < N; ++m)
        if (idx[(int64_t)m * n + a] != idx[(int64_t)m * n + b]) return 0;
    return 1;
}

/* keep[i] = 1 if tuple i (idx is structure-of-arrays, N x n) does not occur
 * among tuples 0..i-1, else 0. The tuples are partitioned into buckets by a
 * hash (stable, so each bucket lists its tuples in increasing i), then every
 * bucket is scanned in order with an open-addressing table that compares the
 * full tuples. Exact for any key space. n < 2^32. */
int syn_first_distinct(int N, const int32_t *idx, int64_t n, uint8_t *keep)
{
    const int bbits = 14;
    const int64_t nb = (int64_t)1 << bbits;
    uint64_t *h = malloc(sizeof(uint64_t) * (size_t)(n ? n : 1));
    uint32_t *arr = malloc(sizeof(uint32_t) * (size_t)(n ? n : 1));
    const int T = omp_get_max_threads();
    int64_t *cnt = calloc((size_t)(T * nb), sizeof(int64_t));
    int64_t *start = malloc(sizeof(int64_t) * (size_t)(nb + 1));
    if (!h || !arr || !cnt || !start) {
        free(h); free(arr); free(cnt); free(start);
        return -1;
    }
#pragma omp parallel num_threads(T)
    {
        const int t = omp_get_thread_num();
        const int64_t lo = n * t / T, hi = n * (t + 1) / T;
        int64_t *c = cnt + (int64_t)t * nb;
        for (int64_t i = lo; i < hi; ++i) {
            uint64_t z = 0x9e3779b97f4a7c15ull;
            for (int m = 0; m < N; ++m)
                z = mix64(z ^ (uint32_t)idx[(int64_t)m * n + i]);
            h[i] = z;
            c[z >> (64 - bbits)]++;
        }
#pragma omp barrier
#pragma omp single
        {
            /* offsets ordered by (bucket, thread): thread chunks are in
             * increasing i, so each bucket stays in draw order */
            int64_t off = 0;
            for (int64_t b = 0; b < nb; ++b) {
                start[b] = off;
                for (int tt = 0; tt < T; ++tt) {
                    const int64_t v = cnt[(int64_t)tt * nb + b];
                    cnt[(int64_t)tt * nb + b] = off;
                    off += v;
                }
            }
            start[nb] = off;
        }
        for (int64_t i = lo; i < hi; ++i)
            arr[c[h[i] >> (64 - bbits)]++] = (uint32_t)i;
    }
    int64_t maxb = 0;
    for (int64_t b = 0; b < nb; ++b)
        if (start[b + 1] - start[b] > maxb) maxb = start[b + 1] - start[b];
    int64_t cap = 16;
    while (cap < 2 * maxb) cap <<= 1;
    int err = 0;
#pragma omp parallel num_threads(T)
    {
        uint32_t *tab = malloc(sizeof(uint32_t) * (size_t)cap);
        if (!tab) {
#pragma omp atomic write
            err = 1;
        }
#pragma omp for schedule(dynamic, 16)
        for (int64_t b = 0; b < nb; ++b) {
            if (!tab) continue;
            const int64_t cb = start[b + 1] - start[b];
            int64_t tc = 16;
            while (tc < 2 * cb) tc <<= 1;
            memset(tab, 0xff, sizeof(uint32_t) * (size_t)tc);
            for (int64_t e = start[b]; e < start[b + 1]; ++e) {
                const uint32_t i = arr[e];
                int64_t slot = (int64_t)(h[i] & (uint64_t)(tc - 1));
                uint8_t k = 1;
                for (;;) {
                    const uint32_t j = tab[slot];
                    if (j == 0xffffffffu) {
                        tab[slot] = i;
                        break;
                    }
                    if (h[j] == h[i] && same_tuple(N, idx, n, j, i)) {
                        k = 0;
                        break;
                    }
                    slot = (slot + 1) & (tc - 1);
                }
                keep[i] = k;
            }
        }
        free(tab);
    }
    free(h);
    free(arr);
    free(cnt);
    free(start);
    return err ? -1 : 0;
}

/* out[s] = scale * sum_r prod_n U[n][idx[n][s] * R + r], products in mode
 * order and the sum in r order (the planted tensor's value at each
 * coordinate; U[n] = P^(n) Q^(n) of the planted model, I_n x R). */
void syn_planted(int N, int R, const double *const *U, const int32_t *idx,
                 int64_t nnz, double scale, double *out)
{
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < nnz; ++s) {
        double acc = 0.0;
        for (int r = 0; r < R; ++r) {
            double p = 1.0;
            for (int n = 0; n < N; ++n)
                p *= U[n][(int64_t)idx[(int64_t)n * nnz + s] * R + r];
            acc += p;
        }
        out[s] = acc * scale;
    }
}
