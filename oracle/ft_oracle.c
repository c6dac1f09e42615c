/*
 * ft_oracle.c -- plain FP64 CPU oracle for sparse FastTucker SGD as defined by
 * FastTuckerPlus (Li et al., "cuFastTuckerPlus: A Stochastic Parallel Sparse
 * FastTucker Decomposition Using GPU Tensor Cores", arXiv 2404.10087).
 *
 * TEST INFRASTRUCTURE. This file is the checker, not the product: only the
 * test suite, the smoke check and the CPU-baseline leg of the benchmark may
 * load it. It shares no code, header, table or helper with the HIP library.
 *
 * Everything is scalar double-precision loops in the paper's order and
 * notation; nothing is blocked, fused or reordered. Conventions:
 *   N        tensor order (1..ORC_MAX_ORDER)
 *   dims[n]  I_n,   J[n] the rank J_n of mode n,   R the Kruskal rank
 *   A[n]     factor matrix A^(n), row-major I_n x J_n   (a^(n)_{i,:} = A[n]+i*J[n])
 *   B[n]     core matrix  B^(n), row-major J_n x R
 *   idx      nonzero coordinates, structure-of-arrays: idx[n*nnz + s] = i_n of
 *            nonzero s (0-based)
 *   vals     nonzero values x_s
 * Residual convention: r_s = xhat_s - x_s (the quantity the GPU algorithms of
 * Section 4.5 name X-hat after subtracting X); the data loss of one sample is
 * r_s^2 / 2, whose gradients are exactly the update directions of Eq. (12)
 * and Eq. (13) (Eqs. (8)/(9) drop the factor 2 of the squared norm).
 *
 * Every function validates nothing: the Python wrapper checks shapes.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_MAX_ORDER 10

/* ------------------------------------------------------------------------ */
/* Per-sample quantities (Eq. (3) and the definition of d^(n) after Eq. (9)) */
/* ------------------------------------------------------------------------ */

/* c^(n)_r = a^(n)_{i_n,:} . b^(n)_{:,r}   for every mode n and r  (Eq. (3)). */
static void sample_c(int N, const int32_t *J, int32_t R, double *const *A,
                     double *const *B, const int64_t *rows, double *c /* N*R */)
{
    for (int n = 0; n < N; ++n) {
        const double *a = A[n] + rows[n] * (int64_t)J[n];
        for (int32_t r = 0; r < R; ++r) {
            double acc = 0.0;
            for (int32_t j = 0; j < J[n]; ++j)
                acc += a[j] * B[n][(int64_t)j * R + r];
            c[n * R + r] = acc;
        }
    }
}

/* d^(n)_r = prod_{k != n} c^(k)_r, a plain product in increasing k; the empty
 * product (N = 1) is 1 (definition following Eq. (9)). */
static void sample_d(int N, int32_t R, const double *c, double *d /* N*R */)
{
    for (int n = 0; n < N; ++n)
        for (int32_t r = 0; r < R; ++r) {
            double p = 1.0;
            for (int k = 0; k < N; ++k)
                if (k != n) p *= c[k * R + r];
            d[n * R + r] = p;
        }
}

/* xhat = sum_r prod_n c^(n)_r   (last line of Eq. (3)). */
static double sample_xhat(int N, int32_t R, const double *c)
{
    double x = 0.0;
    for (int32_t r = 0; r < R; ++r) {
        double p = 1.0;
        for (int n = 0; n < N; ++n) p *= c[n * R + r];
        x += p;
    }
    return x;
}

static void sample_rows(int N, int64_t nnz, const int32_t *idx, int64_t s,
                        int64_t *rows)
{
    for (int n = 0; n < N; ++n) rows[n] = idx[(int64_t)n * nnz + s];
}

/* ------------------------------------------------------------------------ */
/* Prediction and residual statistics                                        */
/* ------------------------------------------------------------------------ */

/* Eq. (3) for every nonzero. */
void orc_predict(int N, const int32_t *J, int32_t R, double *const *A,
                 double *const *B, int64_t nnz, const int32_t *idx,
                 double *xhat)
{
    double *c = malloc(sizeof(double) * N * R);
    int64_t rows[ORC_MAX_ORDER];
    for (int64_t s = 0; s < nnz; ++s) {
        sample_rows(N, nnz, idx, s, rows);
        sample_c(N, J, R, A, B, rows, c);
        xhat[s] = sample_xhat(N, R, c);
    }
    free(c);
}

/* sum_s (x_s - xhat_s)^2 and sum_s |x_s - xhat_s| over a set; the root of the
 * first over |set| is the test RMSE of Section 5.2, the second over |set| the
 * MAE. */
void orc_residual_stats(int N, const int32_t *J, int32_t R, double *const *A,
                        double *const *B, int64_t nnz, const int32_t *idx,
                        const double *vals, double *sse, double *sae)
{
    double *c = malloc(sizeof(double) * N * R);
    int64_t rows[ORC_MAX_ORDER];
    double s2 = 0.0, s1 = 0.0;
    for (int64_t s = 0; s < nnz; ++s) {
        sample_rows(N, nnz, idx, s, rows);
        sample_c(N, J, R, A, B, rows, c);
        double r = sample_xhat(N, R, c) - vals[s];
        s2 += r * r;
        s1 += fabs(r);
    }
    free(c);
    *sse = s2;
    *sae = s1;
}

/* Objective of Eq. (4) with the regularisers summed over all modes:
 * sum (x - xhat)^2 + lamA sum_n ||A^(n)||_F^2 + lamB sum_n ||B^(n)||_F^2. */
double orc_loss(int N, const int64_t *dims, const int32_t *J, int32_t R,
                double *const *A, double *const *B, int64_t nnz,
                const int32_t *idx, const double *vals, double lamA,
                double lamB)
{
    double sse, sae;
    orc_residual_stats(N, J, R, A, B, nnz, idx, vals, &sse, &sae);
    double na = 0.0, nb = 0.0;
    for (int n = 0; n < N; ++n) {
        for (int64_t e = 0; e < dims[n] * (int64_t)J[n]; ++e)
            na += A[n][e] * A[n][e];
        for (int64_t e = 0; e < (int64_t)J[n] * R; ++e)
            nb += B[n][e] * B[n][e];
    }
    return sse + lamA * na + lamB * nb;
}

/* ------------------------------------------------------------------------ */
/* Factor phase: Algorithm 3 (first inner loop) with update rule Eq. (12)    */
/* ------------------------------------------------------------------------ */

/*
 * One minibatch Psi of m samples (coordinates idx with stride m, values
 * vals). All reads use the parameters as they stand when the minibatch
 * starts, and the modes are independent within a sample (the remark after
 * Eq. (13)). For every sample s in order and every mode n the row gradient
 *     g = r_s * (B^(n) d^(n)_s)          (Eq. (8), residual r = xhat - x)
 * plus lamA * a^(n)_{i_n} is added to G^(n)[i_n] and the occurrence count
 * k^(n)[i_n] is incremented. Then each touched row takes
 *     a <- a - lrA * G            (row_mean = 0: gradient of the minibatch loss)
 *     a <- a - lrA * G / k        (row_mean = 1: mean of the per-sample steps)
 * when apply != 0. Returns sum_s r_s^2 / 2.
 *
 * If G_out[n] / cnt_out[n] are given (dense I_n x J_n and I_n arrays), they
 * receive G^(n) and k^(n) (zero for untouched rows).
 */
double orc_factor_minibatch(int N, const int64_t *dims, const int32_t *J,
                            int32_t R, double *const *A, double *const *B,
                            int64_t m, const int32_t *idx, const double *vals,
                            double lrA, double lamA, int row_mean, int apply,
                            double *const *G_out, int64_t *const *cnt_out)
{
    double *G[ORC_MAX_ORDER];
    int64_t *cnt[ORC_MAX_ORDER];
    for (int n = 0; n < N; ++n) {
        G[n] = calloc((size_t)(dims[n] * J[n]), sizeof(double));
        cnt[n] = calloc((size_t)dims[n], sizeof(int64_t));
    }
    double *c = malloc(sizeof(double) * N * R);
    double *d = malloc(sizeof(double) * N * R);
    int64_t rows[ORC_MAX_ORDER];
    double loss = 0.0;

    for (int64_t s = 0; s < m; ++s) {
        sample_rows(N, m, idx, s, rows);
        sample_c(N, J, R, A, B, rows, c);
        sample_d(N, R, c, d);
        double r = sample_xhat(N, R, c) - vals[s];
        loss += 0.5 * r * r;
        for (int n = 0; n < N; ++n) {
            const double *a = A[n] + rows[n] * (int64_t)J[n];
            double *gr = G[n] + rows[n] * (int64_t)J[n];
            for (int32_t j = 0; j < J[n]; ++j) {
                double bd = 0.0;
                for (int32_t q = 0; q < R; ++q)
                    bd += B[n][(int64_t)j * R + q] * d[n * R + q];
                gr[j] += r * bd + lamA * a[j];
            }
            cnt[n][rows[n]] += 1;
        }
    }

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
    free(c);
    free(d);
    return loss;
}

/* Gather the coordinates and values of perm[first .. first+m) into contiguous
 * SoA buffers (the sample set Psi of Section 3.2). */
static void gather_batch(int N, int64_t nnz, const int32_t *idx,
                         const double *vals, const int64_t *perm, int64_t first,
                         int64_t m, int32_t *bidx, double *bvals)
{
    for (int64_t s = 0; s < m; ++s) {
        int64_t src = perm ? perm[first + s] : first + s;
        for (int n = 0; n < N; ++n)
            bidx[(int64_t)n * m + s] = idx[(int64_t)n * nnz + src];
        bvals[s] = vals[src];
    }
}

/*
 * One factor epoch: the training set is visited in the order perm (a
 * permutation of 0..nnz-1), split into consecutive minibatches of M samples,
 * the last one possibly shorter (sampling without replacement). mb_loss, if
 * given, receives sum r^2/2 of each minibatch (ceil(nnz/M) entries).
 */
void orc_factor_epoch(int N, const int64_t *dims, const int32_t *J, int32_t R,
                      double *const *A, double *const *B, int64_t nnz,
                      const int32_t *idx, const double *vals,
                      const int64_t *perm, int64_t M, double lrA, double lamA,
                      int row_mean, double *mb_loss)
{
    int32_t *bidx = malloc(sizeof(int32_t) * N * (size_t)M);
    double *bvals = malloc(sizeof(double) * (size_t)M);
    int64_t b = 0;
    for (int64_t first = 0; first < nnz; first += M, ++b) {
        int64_t m = (nnz - first < M) ? nnz - first : M;
        gather_batch(N, nnz, idx, vals, perm, first, m, bidx, bvals);
        double l = orc_factor_minibatch(N, dims, J, R, A, B, m, bidx, bvals,
                                        lrA, lamA, row_mean, 1, NULL, NULL);
        if (mb_loss) mb_loss[b] = l;
    }
    free(bidx);
    free(bvals);
}

/* ------------------------------------------------------------------------ */
/* Core phase: Algorithm 5 (gradient accumulation, then one update)          */
/* ------------------------------------------------------------------------ */

/*
 * Grad^(n) = sum_s r_s * a^(n)_{i_n}^T d^(n)_s   (J_n x R, Eq. (9) without the
 * regulariser), with A and B held fixed. Grad[n] is overwritten. Returns
 * sum_s r_s^2 / 2.
 */
double orc_core_grad(int N, const int32_t *J, int32_t R, double *const *A,
                     double *const *B, int64_t nnz, const int32_t *idx,
                     const double *vals, double *const *Grad)
{
    for (int n = 0; n < N; ++n)
        memset(Grad[n], 0, sizeof(double) * J[n] * (size_t)R);
    double *c = malloc(sizeof(double) * N * R);
    double *d = malloc(sizeof(double) * N * R);
    int64_t rows[ORC_MAX_ORDER];
    double loss = 0.0;
    for (int64_t s = 0; s < nnz; ++s) {
        sample_rows(N, nnz, idx, s, rows);
        sample_c(N, J, R, A, B, rows, c);
        sample_d(N, R, c, d);
        double r = sample_xhat(N, R, c) - vals[s];
        loss += 0.5 * r * r;
        for (int n = 0; n < N; ++n) {
            const double *a = A[n] + rows[n] * (int64_t)J[n];
            for (int32_t j = 0; j < J[n]; ++j)
                for (int32_t q = 0; q < R; ++q)
                    Grad[n][(int64_t)j * R + q] += r * a[j] * d[n * R + q];
        }
    }
    free(c);
    free(d);
    return loss;
}

/*
 * One core epoch. per_minibatch = 0 (Algorithm 5): accumulate Grad over the
 * whole training set, then, for all modes at once,
 *     B^(n) <- B^(n) - lrB * (Grad^(n) / nnz + lamB * B^(n)).
 * per_minibatch = 1 (Algorithm 3's second loop read with the minibatch mean of
 * Eq. (5)): the same step after every minibatch of M samples in the order
 * perm, with Grad over that minibatch and its size in place of nnz.
 * Returns sum r^2/2 over the training set, each sample's residual taken with
 * the parameters in force when it was visited.
 */
double orc_core_epoch(int N, const int64_t *dims, const int32_t *J, int32_t R,
                      double *const *A, double *const *B, int64_t nnz,
                      const int32_t *idx, const double *vals,
                      const int64_t *perm, int64_t M, double lrB, double lamB,
                      int per_minibatch)
{
    (void)dims;
    double *Grad[ORC_MAX_ORDER];
    for (int n = 0; n < N; ++n)
        Grad[n] = malloc(sizeof(double) * J[n] * (size_t)R);
    double loss = 0.0;
    if (!per_minibatch) {
        loss = orc_core_grad(N, J, R, A, B, nnz, idx, vals, Grad);
        for (int n = 0; n < N; ++n)
            for (int64_t e = 0; e < (int64_t)J[n] * R; ++e)
                B[n][e] -= lrB * (Grad[n][e] / (double)nnz + lamB * B[n][e]);
    } else {
        int32_t *bidx = malloc(sizeof(int32_t) * N * (size_t)M);
        double *bvals = malloc(sizeof(double) * (size_t)M);
        for (int64_t first = 0; first < nnz; first += M) {
            int64_t m = (nnz - first < M) ? nnz - first : M;
            gather_batch(N, nnz, idx, vals, perm, first, m, bidx, bvals);
            loss += orc_core_grad(N, J, R, A, B, m, bidx, bvals, Grad);
            for (int n = 0; n < N; ++n)
                for (int64_t e = 0; e < (int64_t)J[n] * R; ++e)
                    B[n][e] -= lrB * (Grad[n][e] / (double)m + lamB * B[n][e]);
        }
        free(bidx);
        free(bvals);
    }
    for (int n = 0; n < N; ++n) free(Grad[n]);
    return loss;
}
