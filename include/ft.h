/*
 * ft.h -- C ABI of the MI355X sparse FastTucker SGD library.
 *
 * The library implements the hot path of FastTuckerPlus (Li et al.,
 * arXiv 2404.10087): the per-nonzero stochastic gradient sweep of sparse
 * FastTucker decomposition, x_{i1..iN} ~ sum_r prod_n (a^(n)_{i_n,:} b^(n)_{:,r})
 * (Eq. (3)), alternating a factor-matrix phase (Algorithm 3 first loop,
 * update rule Eq. (12)) and a core-matrix phase (Algorithm 5: gradient
 * accumulated over the training set, one update per epoch).
 *
 * General rules
 *   - Every function returns ft_status and never aborts or throws.
 *   - Arguments are validated on the host before any device work; a call that
 *     fails validation returns FT_EINVAL (or FT_ESTATE) and changes nothing.
 *     ft_last_error() then describes the failure.
 *   - A handle lives on the HIP device that was current at ft_create and owns
 *     all device memory it allocates. Calls on one handle are not thread-safe.
 *   - Indices are 0-based int32; nonzero counts are int64.
 *   - All pointers in this header are HOST pointers unless the comment says
 *     "device". Input buffers are copied; the caller keeps ownership.
 *   - The device path supports order 2..10, 1 <= J_n <= 32 and 1 <= R <= 32
 *     (zero padding of J and R to the matrix-core tile is exact for order >= 2).
 *     Orders 2..5 run every option; orders 6..10 (the paper's high-order
 *     synthetic tensors) run the FP32 verify path: ft_set_options rejects
 *     BF16/FP8, the fast mode, vector_alu and core_storage there (FT_EINVAL);
 *     their padded shape must satisfy order x J4 x R16 <= 6144 (J4 = max J_n
 *     rounded up to 8, 16 or 32; R16 = R rounded up to 16), e.g. every order
 *     at J = R = 16 and order 6 at J = R = 32.
 */
#ifndef FT_H
#define FT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ft_handle ft_handle;

typedef enum {
    FT_OK = 0,
    FT_EINVAL = 1,      /* bad argument; nothing changed                    */
    FT_ENOMEM = 2,      /* device or host allocation failed                 */
    FT_EDEVICE = 3,     /* no usable HIP device, or a HIP runtime error     */
    FT_ESTATE = 4,      /* call not valid in the handle's current state     */
    FT_ENONFINITE = 5   /* an epoch produced a non-finite loss              */
} ft_status;

typedef enum { FT_TRAIN = 0, FT_TEST = 1 } ft_set;

/* Arithmetic of the a.B contraction (the rest of the path is FP32; losses and
 * RMSE are reduced in FP64). FT_BF16: factor rows are gathered from a BF16
 * shadow of A (refreshed whenever a row is updated or set), multiplied with
 * a BF16 copy of B on the matrix cores and accumulated in FP32; A and B stay
 * FP32 masters and every update is FP32. FT_FP8_E4M3: the same with an FP8
 * (OCP e4m3) shadow of A holding one FP32 scale per row (s = max|a| / 448,
 * codes rounded to nearest even) and B quantised per column the same way
 * when a kernel stages it; the FP32 accumulators are multiplied by the row
 * and column scales. Evaluation (ft_loss, ft_rmse, ft_eval) uses the
 * contraction precision too. BF16 and FP8 need the verify mode. */
typedef enum { FT_FP32 = 0, FT_BF16 = 1, FT_FP8_E4M3 = 2 } ft_precision;

/* How a minibatch's summed row gradient is applied (Eq. (12) applied per
 * sample, with duplicate rows of one minibatch combined):
 *   FT_ROW_SUM  a <- a - lr_A * G      (gradient of the minibatch loss)
 *   FT_ROW_MEAN a <- a - lr_A * G / k  (mean of the k per-sample steps)      */
typedef enum { FT_ROW_SUM = 0, FT_ROW_MEAN = 1 } ft_row_scale;

/* When the core matrices move: once per epoch with the gradient summed over
 * the training set and divided by its size (Algorithm 5), or after every
 * minibatch with that minibatch's mean gradient (Algorithm 3, Eq. (5)).     */
typedef enum { FT_CORE_PER_EPOCH = 0, FT_CORE_PER_MINIBATCH = 1 } ft_core_step;

typedef struct {
    int64_t minibatch;         /* M >= 1: samples per minibatch Psi          */
    double lr_A, lr_B;         /* gamma_A, gamma_B (finite, >= 0)            */
    double lambda_A, lambda_B; /* lambda_A, lambda_B (finite, >= 0)          */
    int32_t precision;         /* ft_precision                               */
    int32_t row_scale;         /* ft_row_scale                               */
    int32_t core_step;         /* ft_core_step                               */
    int32_t deterministic;     /* 1: sorted segmented reductions, no float
                                  atomics, bitwise reproducible;
                                  0: Hogwild fast mode as in the paper's GPU
                                  algorithm: 16-sample tiles update their
                                  rows at once with float atomics, no
                                  minibatch barrier, no builder; minibatch
                                  must be a multiple of 16 and only frames
                                  the per-minibatch losses                   */
    uint64_t shuffle_seed;     /* seed of the device-side epoch order        */
    int32_t reshuffle_each_epoch; /* 1: new order every epoch; 0: fixed     */
    int32_t vector_alu;        /* 0: contractions on the matrix cores;
                                  1: the factor and core kernels contract
                                  with vector FP32 FMAs instead, for the
                                  matrix-core ablation; FP32 and the verify
                                  mode only (FT_EINVAL otherwise); the
                                  stateless ft_mb_* calls ignore it         */
    int32_t core_storage;      /* core phase, storage against calculation
                                  (the paper's comparison of the two):
                                  0: every sample contracts its rows of A
                                  with B on the matrix cores (calculation);
                                  1: each core pass first stores C^(n) =
                                  A^(n) B^(n) for every row (I_n x R, FP32,
                                  kept by the handle) and the samples gather
                                  rows of C instead; FP32, the verify mode
                                  and vector_alu = 0 only (FT_EINVAL
                                  otherwise). Same results up to rounding. */
} ft_options;

/* Kernel classes that ft_profile_get reports. */
typedef enum {
    FT_K_ORDER = 0,        /* epoch order (counter-based permutation)        */
    FT_K_PERMUTE = 1,      /* gather of the SoA streams into epoch order     */
    FT_K_SORT = 2,         /* mode-sorted minibatch builder (all passes)     */
    FT_K_FACTOR_GRAD = 3,  /* gather + contract + Hadamard + residual + grad */
    FT_K_SEG_REDUCE = 4,   /* sorted segmented reduction + row update        */
    FT_K_SEG_COMBINE = 5,  /* long rows summed in several parts             */
    FT_K_CORE_GRAD = 6,    /* core-gradient partials                         */
    FT_K_CORE_UPDATE = 7,  /* fixed-order partial sum + core update          */
    FT_K_EVAL = 8,         /* forward-only residual statistics               */
    FT_K_HOGWILD = 9,      /* fast-mode factor sweep                         */
    FT_K_PRECOMPUTE_C = 10,/* stored C = A B of the storage variant          */
    FT_K_COUNT = 11
} ft_kernel;

/* Fill *o with the defaults: M = 512, lr 0.01, lambda 1e-3, FP32, ROW_SUM,
 * PER_EPOCH, deterministic, seed 0, reshuffle. */
ft_status ft_default_options(ft_options *o);

/* Create a problem of the given order with dims[order] = I_n, J[order] = J_n
 * and Kruskal rank R (Section 2.3 problem statement). Factor and core
 * matrices are initialised with N(0, 0.5^2) entries drawn from a SplitMix64
 * stream seeded by seed (Algorithm 3's initialisation, which the paper leaves
 * open). *out receives the handle; on failure *out is set to NULL and
 * ft_last_error(NULL) names the reason. */
ft_status ft_create(int order, const int64_t *dims, const int32_t *J,
                    int32_t R, uint64_t seed, ft_handle **out);

/* Release every resource of h (NULL is accepted). */
ft_status ft_destroy(ft_handle *h);

/* Message of the last failing call on h; h == NULL gives the last ft_create
 * failure of the calling thread. Never NULL. */
const char *ft_last_error(const ft_handle *h);

ft_status ft_set_options(ft_handle *h, const ft_options *o);
ft_status ft_get_options(const ft_handle *h, ft_options *o);

/* Use a caller-provided HIP stream (hipStream_t, default priority) for all
 * later work of h; NULL selects the null stream. */
ft_status ft_set_stream(ft_handle *h, void *hip_stream);

/* Copy a set of nonzeros (the set Omega, or the test set Gamma of Section
 * 5.2). idx is structure-of-arrays: idx[n*nnz + s] is i_n of nonzero s;
 * vals[s] its value. Every index is range-checked (FT_EINVAL, nothing
 * changed). nnz may be 0 for the test set; the training set needs nnz >= 1.
 * Replacing the training set resets the epoch order. */
ft_status ft_set_nonzeros(ft_handle *h, ft_set which, int64_t nnz,
                          const int32_t *idx, const float *vals);

/* Visit the training set in the order perm[0..nnz_train) in every later
 * epoch (a permutation of 0..nnz_train-1, checked); NULL returns to the
 * device-side order drawn from shuffle_seed and the epoch counter. */
ft_status ft_set_epoch_order(ft_handle *h, const int64_t *perm);

/* Number of minibatches of one epoch: ceil(nnz_train / M). */
ft_status ft_num_minibatches(const ft_handle *h, int64_t *out);

/* One factor epoch (Algorithm 3 first loop): draw the order, build the
 * mode-sorted minibatches, then for every minibatch compute c, d, the
 * residual and the row gradients (Eq. (8)) with all parameters as they stand
 * at the minibatch start, and update every touched row (Eq. (12), scaled by
 * row_scale). mb_loss (NULL or [ceil(nnz/M)]) receives sum r^2/2 of every
 * minibatch, r = xhat - x. Advances the epoch counter. Returns after the
 * epoch's work is complete. It uses the order, permutation and sort built
 * ahead by the preceding ft_epoch_core (see there) if they were built for
 * this epoch with the current options, seed and training set, else builds
 * them in line. In
 * the fast mode the tiles run concurrently with immediate per-sample steps
 * a <- a - lr_A (r B d + lambda_A a) (Eq. (12) applied per sample, Hogwild);
 * row_scale does not apply. */
ft_status ft_epoch_factors(ft_handle *h, double *mb_loss);

/* Fine-grained form of ft_epoch_factors for verification:
 * ft_prepare_epoch draws the order and builds the minibatches;
 * ft_factor_minibatch runs minibatch b of the prepared epoch. With apply = 1
 * it updates A and writes sum r^2/2 to *loss (may be NULL). With apply = 0 it
 * changes nothing and writes, for every mode n, the summed row gradients
 * G^(n) (sum over occurrences of r*(B d) + lambda_A*a, dense I_n x J_n,
 * row-major, zero for untouched rows) to grad[n] and the occurrence counts to
 * count[n] (I_n entries). */
ft_status ft_prepare_epoch(ft_handle *h);
ft_status ft_factor_minibatch(ft_handle *h, int64_t b, int32_t apply,
                              double *loss, float *const *grad,
                              int32_t *const *count);

/* One core epoch (Algorithm 5, or per-minibatch steps with
 * FT_CORE_PER_MINIBATCH): Grad^(n) = sum_s r_s a^(n)T d^(n) with A, B fixed,
 * then B^(n) <- B^(n) - lr_B (Grad^(n)/|Omega| + lambda_B B^(n)) for all n at
 * once. *loss (may be NULL) receives sum r^2/2 over the training set.
 * In the verify mode with the device-side order and reshuffle_each_epoch = 1
 * it first starts building the order, permutation and sort of the next
 * factor epoch on an internal second stream (non-blocking, default
 * priority), beside its own kernels; that build may still run when it
 * returns, and the next ft_epoch_factors waits for it. */
ft_status ft_epoch_core(ft_handle *h, double *loss);

/* Core gradient only: Grad^(n) (J_n x R row-major, no regulariser) summed
 * over the training set into grad[n]; A and B unchanged. */
ft_status ft_core_grad(ft_handle *h, float *const *grad, double *loss);

/* Objective of Eq. (4) over a set, regularisers summed over all modes:
 * sum (x - xhat)^2 + lambda_A sum_n ||A^(n)||^2 + lambda_B sum_n ||B^(n)||^2. */
ft_status ft_loss(ft_handle *h, ft_set which, double *out);

/* sqrt(mean (x - xhat)^2) over a set (test RMSE of Section 5.2); 0 for an
 * empty set. ft_eval gives the raw sums: sum (x-xhat)^2 and sum |x-xhat|. */
ft_status ft_rmse(ft_handle *h, ft_set which, double *out);
ft_status ft_eval(ft_handle *h, ft_set which, double *sse, double *sae);

/* Parameters, unpadded row-major: which = 0 gives A^(mode) (I_n x J_n),
 * which = 1 gives B^(mode) (J_n x R). */
ft_status ft_get_params(ft_handle *h, int mode, int which, float *host_out);
ft_status ft_set_params(ft_handle *h, int mode, int which,
                        const float *host_in);

/* Builder output of the current epoch (after ft_prepare_epoch or
 * ft_epoch_factors), for verification: the epoch order (nnz_train entries),
 * and for minibatch b and mode n the in-minibatch positions sorted stably by
 * row (pos[m]) and those rows (rows[m]), m = size of minibatch b. */
ft_status ft_get_epoch_order(ft_handle *h, int64_t *perm_out);
ft_status ft_get_minibatch_sort(ft_handle *h, int64_t b, int mode,
                                int32_t *pos, int32_t *rows);

/* Per-kernel device time: with profiling on, every launch is bracketed by HIP
 * events on the handle's stream; ft_profile_get synchronises and returns the
 * number of launches and their summed duration (ms) since the last reset. */
ft_status ft_profile_enable(ft_handle *h, int32_t on);
ft_status ft_profile_reset(ft_handle *h);
ft_status ft_profile_get(ft_handle *h, int32_t kernel, int64_t *launches,
                         double *total_ms);

/* ------------------------------------------------------------------------
 * Stateless minibatch entry points (back the torch.autograd.Function).
 * The caller owns every buffer (device memory) and the stream; nothing is
 * allocated. The minibatch loss is L = sum_{s in Psi} r_s^2 / 2 with
 * r = xhat - x (data term only; regularisation is left to the caller).
 *   A[n]   device FP32, dims[n] x J4 row-major, J4 = max_n J_n rounded up to
 *          a multiple of 4; columns J_n..J4-1 must be zero
 *   B[n]   device FP32, J_n x R row-major
 *   idx[n] device int32, m coordinates of mode n (range is the caller's
 *          responsibility: indices must lie in [0, dims[n]))
 *   val    device FP32, m values
 * ------------------------------------------------------------------------ */
typedef struct {
    int32_t order;       /* 2..10 (FP32 kernels above 5)                     */
    int64_t dims[10];    /* I_n (the first `order` entries are read)        */
    int32_t J[10];       /* 1..32                                           */
    int32_t R;           /* 1..32                                           */
} ft_problem_desc;

/* Bytes of device workspace that ft_mb_forward / ft_mb_backward need for a
 * minibatch of m samples (1 <= m <= 2^30). The workspace must be 256-byte
 * aligned and every A[n] 16-byte aligned (FT_EINVAL otherwise); device
 * allocations are. */
ft_status ft_mb_workspace_size(const ft_problem_desc *p, int64_t m,
                               size_t *bytes);

/* *loss_dev (device double) <- sum r^2 / 2 over the minibatch, reduced in
 * FP64 in a fixed order (Eq. (3) forward). */
ft_status ft_mb_forward(const ft_problem_desc *p, const float *const *A,
                        const float *const *B, const int32_t *const *idx,
                        const float *val, int64_t m, double *loss_dev,
                        void *workspace, size_t ws_bytes, void *hip_stream);

/* Gradients of g * L, g = *grad_out_dev (device FP32; NULL means 1), with
 * c^(n) recomputed (nothing is kept from the forward call):
 *   rows (Eq. (8)): the per-sample r_s B^(n) d^(n)_s summed per unique row in
 *     a fixed order (the deterministic sorted segmented reduction). Sparse
 *     form: uniq_rows[n] (device int32, capacity m) receives the touched rows
 *     in increasing order, uniq_grad[n] (device FP32, capacity m x J4) their
 *     gradient rows, n_uniq_dev[n] (device int64) their number. Dense form:
 *     gradA[n] (device FP32, dims[n] x J4) is overwritten (zero for untouched
 *     rows). Either form may be omitted by passing NULL arrays.
 *   core (Eq. (9)): gradB[n] (device FP32, J_n x R) is overwritten.
 * Bitwise reproducible (no floating-point atomics). */
ft_status ft_mb_backward(const ft_problem_desc *p, const float *const *A,
                         const float *const *B, const int32_t *const *idx,
                         const float *val, int64_t m,
                         const float *grad_out_dev, float *const *gradA,
                         int32_t *const *uniq_rows, float *const *uniq_grad,
                         int64_t *n_uniq_dev, float *const *gradB,
                         void *workspace, size_t ws_bytes, void *hip_stream);

/* ------------------------------------------------------------------------
 * Allocation-free backward. For callers that cannot allocate device memory
 * during the call: code under HIP graph capture, tight serving or training
 * loops, harnesses that forbid hipMalloc. Same arguments, outputs and
 * results as ft_mb_backward, without the workspace: the intermediates live
 * in a static device array of FT_NOALLOC_SCRATCH_BYTES (64 MiB) that every
 * device the library runs on holds from its first use until the process
 * ends. The call allocates nothing (no hipMalloc, hipFree or allocating
 * library routine); its address is looked up once per device
 * (hipGetSymbolAddress) on the first call made with that device current.
 * A minibatch whose workspace (ft_mb_workspace_size) exceeds the array is
 * rejected with FT_EINVAL before any device work. All calls on one device
 * share the one array: calls that may overlap on a device (other streams,
 * other host threads) race and give wrong results; serialise them. The
 * array keeps the last call's contents; nothing in it needs to start zero.
 * ------------------------------------------------------------------------ */
#define FT_NOALLOC_SCRATCH_BYTES (64ull << 20)

ft_status ft_mb_backward_noalloc(const ft_problem_desc *p,
                                 const float *const *A, const float *const *B,
                                 const int32_t *const *idx, const float *val,
                                 int64_t m, const float *grad_out_dev,
                                 float *const *gradA,
                                 int32_t *const *uniq_rows,
                                 float *const *uniq_grad, int64_t *n_uniq_dev,
                                 float *const *gradB, void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* FT_H */
