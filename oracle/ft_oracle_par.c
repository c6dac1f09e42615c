/*
 * ft_oracle_par.c -- the oracle of ft_oracle.c plus forms of its loops that
 * spread independent samples over host threads (OpenMP), for timing the
 * oracle on all cores. liboracle.so is built from this file.
 *
 * TEST INFRASTRUCTURE, like ft_oracle.c: only the test suite, the smoke
 * check and the benchmark's CPU-baseline leg may load it.
 */
#include "ft_oracle.c"

#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* The same loops spread over host threads (OpenMP), for timing the oracle   */
/* on all cores. The per-sample arithmetic is the serial code's, unchanged.  */
/* ------------------------------------------------------------------------ */

/*
 * orc_factor_minibatch with the per-sample work (c, d, residual and the
 * row gradients r * B d) computed in parallel into per-sample buffers; the
 * buffers are then added into G in sample order by one thread, with the
 * regulariser term added exactly as the serial loop does, so every result is
 * bitwise the serial one's.
 */
double orc_factor_minibatch_par(int N, const int64_t *dims, const int32_t *J,
                                int32_t R, double *const *A, double *const *B,
                                int64_t m, const int32_t *idx,
                                const double *vals, double lrA, double lamA,
                                int row_mean, int apply, double *const *G_out,
                                int64_t *const *cnt_out)
{
    int64_t sumJ = 0, off[ORC_MAX_ORDER];
    for (int n = 0; n < N; ++n) {
        off[n] = sumJ;
        sumJ += J[n];
    }
    double *gbuf = malloc(sizeof(double) * (size_t)(m * sumJ));
    double *rbuf = malloc(sizeof(double) * (size_t)m);
#pragma omp parallel
    {
        double *c = malloc(sizeof(double) * N * R);
        double *d = malloc(sizeof(double) * N * R);
        int64_t rows[ORC_MAX_ORDER];
#pragma omp for schedule(static)
        for (int64_t s = 0; s < m; ++s) {
            sample_rows(N, m, idx, s, rows);
            sample_c(N, J, R, A, B, rows, c);
            sample_d(N, R, c, d);
            double r = sample_xhat(N, R, c) - vals[s];
            rbuf[s] = r;
            for (int n = 0; n < N; ++n)
                for (int32_t j = 0; j < J[n]; ++j) {
                    double bd = 0.0;
                    for (int32_t q = 0; q < R; ++q)
                        bd += B[n][(int64_t)j * R + q] * d[n * R + q];
                    gbuf[s * sumJ + off[n] + j] = r * bd;
                }
        }
        free(c);
        free(d);
    }
    double *G[ORC_MAX_ORDER];
    int64_t *cnt[ORC_MAX_ORDER];
    for (int n = 0; n < N; ++n) {
        G[n] = calloc((size_t)(dims[n] * J[n]), sizeof(double));
        cnt[n] = calloc((size_t)dims[n], sizeof(int64_t));
    }
    double loss = 0.0;
    for (int64_t s = 0; s < m; ++s) {
        loss += 0.5 * rbuf[s] * rbuf[s];
        for (int n = 0; n < N; ++n) {
            const int64_t row = idx[(int64_t)n * m + s];
            const double *a = A[n] + row * (int64_t)J[n];
            double *gr = G[n] + row * (int64_t)J[n];
            for (int32_t j = 0; j < J[n]; ++j)
                gr[j] += gbuf[s * sumJ + off[n] + j] + lamA * a[j];
            cnt[n][row] += 1;
        }
    }
    free(gbuf);
    free(rbuf);
    for (int n = 0; n < N; ++n) {
        if (G_out && G_out[n])
            memcpy(G_out[n], G[n], sizeof(double) * dims[n] * J[n]);
        if (cnt_out && cnt_out[n])
            memcpy(cnt_out[n], cnt[n], sizeof(int64_t) * dims[n]);
        if (apply) {
            for (int64_t i = 0; i < dims[n]; ++i) {
                if (cnt[n][i] == 0) continue;
                double scale = row_mean ? 1.0 / (double)cnt[n][i] : 1.0;
                double *a = A[n] + i * (int64_t)J[n];
                const double *gr = G[n] + i * (int64_t)J[n];
                for (int32_t j = 0; j < J[n]; ++j)
                    a[j] -= lrA * (gr[j] * scale);
            }
        }
        free(G[n]);
        free(cnt[n]);
    }
    return loss;
}

/* orc_factor_epoch over orc_factor_minibatch_par (bitwise the same). */
void orc_factor_epoch_par(int N, const int64_t *dims, const int32_t *J,
                          int32_t R, double *const *A, double *const *B,
                          int64_t nnz, const int32_t *idx, const double *vals,
                          const int64_t *perm, int64_t M, double lrA,
                          double lamA, int row_mean, double *mb_loss)
{
    int32_t *bidx = malloc(sizeof(int32_t) * N * (size_t)M);
    double *bvals = malloc(sizeof(double) * (size_t)M);
    int64_t b = 0;
    for (int64_t first = 0; first < nnz; first += M, ++b) {
        int64_t m = (nnz - first < M) ? nnz - first : M;
        gather_batch(N, nnz, idx, vals, perm, first, m, bidx, bvals);
        double l = orc_factor_minibatch_par(N, dims, J, R, A, B, m, bidx,
                                            bvals, lrA, lamA, row_mean, 1,
                                            NULL, NULL);
        if (mb_loss) mb_loss[b] = l;
    }
    free(bidx);
    free(bvals);
}

#define ORC_PAR_CHUNK 4096

/* Threads of the *_par functions (n < 1: all); returns the count in force. */
int orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
    else omp_set_num_threads(omp_get_num_procs());
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}

/*
 * orc_core_grad with the samples cut into consecutive chunks of
 * ORC_PAR_CHUNK: each chunk's sum (the serial loop over its samples) is
 * formed by one thread, and the chunk sums are added in chunk order. The
 * result does not depend on the thread count; it differs from the serial
 * sum only in the order of the additions.
 */
double orc_core_grad_par(int N, const int32_t *J, int32_t R, double *const *A,
                         double *const *B, int64_t nnz, const int32_t *idx,
                         const double *vals, double *const *Grad)
{
    int64_t per = 0;
    for (int n = 0; n < N; ++n) per += (int64_t)J[n] * R;
    const int64_t nch = (nnz + ORC_PAR_CHUNK - 1) / ORC_PAR_CHUNK;
    double *part = calloc((size_t)(nch * per + 1), sizeof(double));
    double *lpart = calloc((size_t)(nch + 1), sizeof(double));
#pragma omp parallel
    {
        double *c = malloc(sizeof(double) * N * R);
        double *d = malloc(sizeof(double) * N * R);
        int64_t rows[ORC_MAX_ORDER];
#pragma omp for schedule(dynamic, 1)
        for (int64_t ch = 0; ch < nch; ++ch) {
            double *g = part + ch * per;
            const int64_t s1 = (ch + 1) * ORC_PAR_CHUNK < nnz
                                   ? (ch + 1) * ORC_PAR_CHUNK : nnz;
            double loss = 0.0;
            for (int64_t s = ch * ORC_PAR_CHUNK; s < s1; ++s) {
                sample_rows(N, nnz, idx, s, rows);
                sample_c(N, J, R, A, B, rows, c);
                sample_d(N, R, c, d);
                double r = sample_xhat(N, R, c) - vals[s];
                loss += 0.5 * r * r;
                int64_t o = 0;
                for (int n = 0; n < N; ++n) {
                    const double *a = A[n] + rows[n] * (int64_t)J[n];
                    for (int32_t j = 0; j < J[n]; ++j)
                        for (int32_t q = 0; q < R; ++q)
                            g[o + (int64_t)j * R + q] += r * a[j] * d[n * R + q];
                    o += (int64_t)J[n] * R;
                }
            }
            lpart[ch] = loss;
        }
        free(c);
        free(d);
    }
    for (int n = 0; n < N; ++n)
        memset(Grad[n], 0, sizeof(double) * J[n] * (size_t)R);
    double loss = 0.0;
    for (int64_t ch = 0; ch < nch; ++ch) {
        int64_t o = 0;
        for (int n = 0; n < N; ++n) {
            for (int64_t e = 0; e < (int64_t)J[n] * R; ++e)
                Grad[n][e] += part[ch * per + o + e];
            o += (int64_t)J[n] * R;
        }
        loss += lpart[ch];
    }
    free(part);
    free(lpart);
    return loss;
}

/* Algorithm 5's core epoch over orc_core_grad_par. */
double orc_core_epoch_par(int N, const int32_t *J, int32_t R, double *const *A,
                          double *const *B, int64_t nnz, const int32_t *idx,
                          const double *vals, double lrB, double lamB)
{
    double *Grad[ORC_MAX_ORDER];
    for (int n = 0; n < N; ++n)
        Grad[n] = malloc(sizeof(double) * J[n] * (size_t)R);
    double loss = orc_core_grad_par(N, J, R, A, B, nnz, idx, vals, Grad);
    for (int n = 0; n < N; ++n) {
        for (int64_t e = 0; e < (int64_t)J[n] * R; ++e)
            B[n][e] -= lrB * (Grad[n][e] / (double)nnz + lamB * B[n][e]);
        free(Grad[n]);
    }
    return loss;
}

/* orc_residual_stats with chunk sums added in chunk order (as above). */
void orc_residual_stats_par(int N, const int32_t *J, int32_t R,
                            double *const *A, double *const *B, int64_t nnz,
                            const int32_t *idx, const double *vals,
                            double *sse, double *sae)
{
    const int64_t nch = (nnz + ORC_PAR_CHUNK - 1) / ORC_PAR_CHUNK;
    double *p2 = calloc((size_t)(nch + 1), sizeof(double));
    double *p1 = calloc((size_t)(nch + 1), sizeof(double));
#pragma omp parallel
    {
        double *c = malloc(sizeof(double) * N * R);
        int64_t rows[ORC_MAX_ORDER];
#pragma omp for schedule(dynamic, 1)
        for (int64_t ch = 0; ch < nch; ++ch) {
            const int64_t s1 = (ch + 1) * ORC_PAR_CHUNK < nnz
                                   ? (ch + 1) * ORC_PAR_CHUNK : nnz;
            double s2 = 0.0, s1a = 0.0;
            for (int64_t s = ch * ORC_PAR_CHUNK; s < s1; ++s) {
                sample_rows(N, nnz, idx, s, rows);
                sample_c(N, J, R, A, B, rows, c);
                double r = sample_xhat(N, R, c) - vals[s];
                s2 += r * r;
                s1a += fabs(r);
            }
            p2[ch] = s2;
            p1[ch] = s1a;
        }
        free(c);
    }
    double t2 = 0.0, t1 = 0.0;
    for (int64_t ch = 0; ch < nch; ++ch) {
        t2 += p2[ch];
        t1 += p1[ch];
    }
    free(p2);
    free(p1);
    *sse = t2;
    *sae = t1;
}
