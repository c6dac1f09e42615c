// ft_internal.h -- shapes, argument blocks and launchers shared by the host
// runtime (ft_api.cpp) and the HIP kernels of the sparse FastTucker library.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ft {

// Timing of single-kernel launches: when the host sets these (profiling on),
// the next launch records them exactly at the kernel's start and end
// (hipExtLaunchKernelGGL) and clears them.
struct ExtEvents {
    hipEvent_t start = nullptr, stop = nullptr;
};
extern thread_local ExtEvents g_ext_events;

#define FT_LAUNCH(kernel, grid, block, shm, stream, ...)                      \
    do {                                                                      \
        if (::ft::g_ext_events.start) {                                       \
            hipExtLaunchKernelGGL(kernel, grid, block, shm, stream,           \
                                  ::ft::g_ext_events.start,                   \
                                  ::ft::g_ext_events.stop, 0, __VA_ARGS__);   \
            ::ft::g_ext_events = ::ft::ExtEvents{};                           \
        } else {                                                              \
            hipLaunchKernelGGL(kernel, grid, block, shm, stream, __VA_ARGS__); \
        }                                                                     \
    } while (0)

constexpr int kMaxOrder = 10;
// Orders up to kFullOrder run every variant (precisions, fast mode, vector
// ALU, stored C) at every padded J4 in 4..32; higher orders run the FP32
// verify path with J4 padded to 8, 16 or 32 (fewer kernel instances).
constexpr int kFullOrder = 5;
constexpr int kMaxJ = 32;
constexpr int kMaxR = 32;

// Sorted segmented reduction: rows are summed over fixed chunks of this many
// sorted samples; segments that cross a chunk edge are finished by a fix-up.
constexpr int kSegChunk = 64;
constexpr int kSmallCross = 256;      // crossing rows up to this many samples
                                      // are reduced by one wave
constexpr int kSegWaves = 4;          // waves per row-reduction block
// A crossing row whose gradient rows hold more than kSplitFloats floats is
// summed in parts of kPartFloats floats (one block each) and the parts are
// combined; in samples that is split_rows(J4) and part_rows(J4), so the
// bytes one block reads stay the same at every row width.
#ifndef FT_SPLIT_FLOATS
#define FT_SPLIT_FLOATS 262144
#endif
#ifndef FT_PART_FLOATS
#define FT_PART_FLOATS 32768
#endif
constexpr int kSplitFloats = FT_SPLIT_FLOATS;
constexpr int kPartFloats = FT_PART_FLOATS;
inline __host__ __device__ int split_rows(int J4) { return kSplitFloats / J4; }
inline __host__ __device__ int part_rows(int J4) { return kPartFloats / J4; }
constexpr int kXCounts = 4;           // per minibatch and mode: short rows,
                                      // long rows, parts, multi-part rows

// Mode-sorted minibatch builder: LSD radix sort, 8-bit digits, 2048-element
// tiles aligned to minibatch starts.
constexpr int kSortThreads = 256;
constexpr int kSortRounds = 8;
constexpr int kSortTile = kSortThreads * kSortRounds;
constexpr int kRadix = 256;

// Padded shape. A^(n) is stored I_n x J4 (row stride J4 = max J_n rounded up
// to 4); B^(n) is stored J4 x R16 (R rounded up to 16). Padding is zero and
// stays zero under every update.
// Contraction precisions (Shape::prec, template argument P of the tiles).
constexpr int kF32 = 0, kBF16 = 1, kFP8 = 2;

struct Shape {
    int N;
    int J4;
    int R16;
    int prec;    // contraction a.B: 0 FP32, 1 BF16 shadow of A, 2 FP8 e4m3
                 // shadow with per-row scales (FP32 accumulate throughout)
};

hipError_t launch_to_bf16(const float *src, uint16_t *dst, int64_t n,
                          hipStream_t s);
// FP8 shadow of rows x J4 floats: J4 e4m3 codes and one scale per row
hipError_t launch_to_fp8_rows(const float *src, int64_t rows, int J4,
                              uint8_t *dst, float *scale, hipStream_t s);

// ---------------------------------------------------------------- builder
hipError_t launch_epoch_order(uint32_t *perm, int64_t n, uint64_t key,
                              hipStream_t s,
                              int grid_cap = 0);
hipError_t launch_copy_order(uint32_t *perm, const int64_t *src, int64_t n,
                             hipStream_t s);
// Training-set records: RW = 4 words (order <= 3) or 8 words (order 4..5).
inline int record_words(int N) { return N <= 3 ? 4 : N <= 7 ? 8 : 16; }
// Row stride of A^(n) (and rows of B^(n)): max J_n rounded up to 4, or for
// orders above kFullOrder to 8, 16 or 32. Zero padding is exact.
// Above kFullOrder the core kernel's four per-wave partials (4 x N x J4 x
// R16 floats) and B-operands must fit in one block's 160 KB of LDS.
constexpr int kHighOrderTile = 6144;
inline bool high_order_fits(int N, int J4, int R16) {
    return N <= kFullOrder || N * J4 * R16 <= kHighOrderTile;
}
inline int padded_j4(int N, int jmax) {
    const int j4 = (jmax + 3) / 4 * 4;
    if (N <= kFullOrder) return j4;
    return j4 <= 8 ? 8 : j4 <= 16 ? 16 : 32;
}
hipError_t launch_pack_records(int N, const int32_t *const *idx,
                               const float *val, int64_t nnz, uint32_t *rec,
                               int rw, hipStream_t s);
hipError_t launch_permute(int N, const uint32_t *rec, int rw,
                          const uint32_t *perm, int64_t nnz,
                          int32_t *const *pidx, float *pval, hipStream_t s,
                          int grid_cap = 0);

struct SortPass {
    int N;               // modes sorted by this pass (slots 0 .. N-1)
    int64_t nnz;
    int64_t M;           // segment (minibatch) length
    int nseg;
    int tiles_per_seg;   // tiles of a full segment
    int shift;           // digit = (key >> shift) & 255
    const uint32_t *key_in[kMaxOrder];
    const uint32_t *val_in[kMaxOrder];   // nullptr: payload = position in segment
    uint32_t *key_out[kMaxOrder];
    uint32_t *val_out[kMaxOrder];   // nullptr: positions not written
    uint32_t *inv_out[kMaxOrder];   // final pass only (else nullptr):
                                    // inv[seg + pos] = sorted index in seg
    // [N][nseg][tiles_per_seg + 1][kRadix]: per tile the digit counts (the
    // upsweep), then the counts in the segment's earlier tiles; the extra
    // last row holds the segment's digit starts
    uint32_t *counts;
    int grid_cap;        // > 0: at most this many workgroups (background)
};
hipError_t launch_sort_pass(const SortPass &p, hipStream_t s);
inline size_t sort_counts_words(int N, int nseg, int tiles_per_seg) {
    return (size_t)N * nseg * (tiles_per_seg + 1) * kRadix;
}
// 8-bit LSD passes that sort row ids 0 .. dims - 1 (at least one)
inline int radix_passes(int64_t dims) {
    int bits = 0;
    while ((1ll << bits) <= dims - 1) ++bits;
    return bits == 0 ? 1 : (bits + 7) / 8;
}

// ---------------------------------------------------------------- factor phase
struct FactorArgs {
    const uint16_t *A16[kMaxOrder];  // BF16 shadow of A (BF16 only)
    const uint8_t *A8[kMaxOrder];    // FP8 shadow of A and its row scales
    const float *As[kMaxOrder];      // (FP8 only)
    const int32_t *idx[kMaxOrder];  // coordinates of the minibatch (m entries)
    const float *val;
    int32_t m;
    const float *A[kMaxOrder];
    const float *B[kMaxOrder];
    // per-sample row gradients, [N][m][J4] in each mode's sorted order:
    // sample p of mode n goes to row inv[n][p]
    float *G;
    const uint32_t *inv[kMaxOrder];
    double *loss_part;               // one per block
};
hipError_t launch_factor_grad(const Shape &sh, const FactorArgs &a, int *nblocks,
                              hipStream_t s);
int factor_grad_blocks(const Shape &sh, int32_t m);
// The same outputs with the contractions on vector FP32 FMAs (one sample
// per lane), for the matrix-core ablation; FP32 only (factor_valu_supported).
bool factor_valu_supported(const Shape &sh);
hipError_t launch_factor_grad_valu(const Shape &sh, const FactorArgs &a,
                                   int *nblocks, hipStream_t s);

struct HogArgs {
    const uint16_t *A16[kMaxOrder];  // BF16 shadow of A (BF16 only)
    const uint8_t *A8[kMaxOrder];    // FP8 shadow of A and its row scales
    const float *As[kMaxOrder];      // (FP8 only)
    const int32_t *idx[kMaxOrder];   // epoch-order coordinates
    const float *val;
    int64_t count;
    float *A[kMaxOrder];
    const float *B[kMaxOrder];
    float lr, lam;
    double *tile_loss;               // [ceil(count / 16)]
};
hipError_t launch_hogwild(const Shape &sh, const HogArgs &a, hipStream_t s);

struct SegArgs {
    int N;
    int J4;
    int32_t m;
    int nchunks;                      // ceil(m / kSegChunk)
    const uint32_t *rows[kMaxOrder];  // sorted rows of the minibatch
    const float *G;                   // [N][m][J4], sorted order per mode
    float *A[kMaxOrder];
    // rows whose samples cross a chunk edge, in sorted indices. For mode n,
    // xcount[kXCounts n] rows of at most kSmallCross samples fill
    // xlist[n][0..) as (first, end, row, 0) and xcount[kXCounts n + 1]
    // longer rows fill xlist[n][xcap-1..] downwards as (first, end, row,
    // first part). A long row is summed in one part, or in
    // ceil(count / part_rows(J4)) parts when count > split_rows(J4);
    // plist[n][0 .. xcount[kXCounts n + 2]) = (first, end, row, parts of
    // the row); rows of one part are finished at once, the others leave
    // partial sums in P[n][part][J4] for the combine kernel.
    const int4 *xlist[kMaxOrder];
    const int4 *plist[kMaxOrder];
    const int32_t *xcount;
    int xcap;
    int pcap;
    float *P;
    // host_counts: the counts are also given here as prefix sums over the
    // modes (xs: short rows, xl: long rows, xp: parts), so blocks find their
    // entry without reading xcount
    int host_counts;
    int xs[kMaxOrder + 1], xl[kMaxOrder + 1], xp[kMaxOrder + 1];
    int small_blocks;                 // blocks for the short rows
    int large_blocks;                 // blocks for the long-row parts
    int combine_blocks;               // blocks of the combine kernel (0: none)
    float lr, lam;
    int mean;                         // FT_ROW_MEAN
    int apply;                        // 1: update A; 0: write grad/count;
                                      // 2: autograd outputs (no lambda term)
    uint16_t *A16[kMaxOrder];         // BF16 shadow refreshed on update
    uint8_t *A8[kMaxOrder];           // FP8 shadow and row scales refreshed
    float *As[kMaxOrder];             // on update
    float *grad[kMaxOrder];           // dense I_n x J4 (apply 0, 2; may be
                                      // null in mode 2)
    int32_t *count[kMaxOrder];        // I_n (apply == 0)
    // apply == 2: compacted sparse rows, scaled by *scale (null: 1)
    const uint32_t *ordinal[kMaxOrder];  // unique-row index of each sorted
                                         // element (segment starts only read)
    int32_t *uniq_rows[kMaxOrder];       // [#unique] or null
    float *uniq_grad[kMaxOrder];         // [#unique][J4] or null
    const float *scale;
};
hipError_t launch_seg_reduce(const SegArgs &a, hipStream_t s);
// finishes the long rows of more than one part (a.combine_blocks > 0)
hipError_t launch_seg_combine(const SegArgs &a, hipStream_t s);

// Per epoch (after the sort): list every row segment of every minibatch
// and mode that crosses a kSegChunk edge.
struct CrossArgs {
    int N;
    int64_t nnz;
    int64_t M;
    int nseg;
    int xcap;                         // max(1, ceil(min(M, nnz) / kSegChunk) - 1)
    const uint32_t *rows[kMaxOrder];  // sorted rows of the whole epoch
    int4 *xlist;                      // [nseg][N][xcap]
    int4 *plist;                      // [nseg][N][pcap]
    int pcap;
    int32_t *xcount;                  // [nseg][N][kXCounts]
    int grid_cap;                     // > 0: at most this many workgroups
    int J4;                           // row width (sets the part sizes)
};
hipError_t launch_crossing_segments(const CrossArgs &c, hipStream_t s);
inline int cross_capacity(int64_t m) {
    const int64_t ch = (m + kSegChunk - 1) / kSegChunk;
    return ch > 1 ? (int)(ch - 1) : 1;
}
// sum over the long rows of ceil(count / part) <= rows + m / part
inline int part_capacity(int64_t m, int J4) {
    return cross_capacity(m) + (int)(m / part_rows(J4)) + 1;
}

hipError_t launch_sum_blocks(const double *part, int nper, int ngroups,
                             double *out, hipStream_t s);

// ---------------------------------------------------------------- core phase
struct CoreArgs {
    const uint16_t *A16[kMaxOrder];  // BF16 shadow of A (BF16 only)
    const uint8_t *A8[kMaxOrder];    // FP8 shadow of A and its row scales
    const float *As[kMaxOrder];      // (FP8 only)
    const int32_t *idx[kMaxOrder];
    const float *val;
    int64_t count;
    const float *A[kMaxOrder];
    const float *B[kMaxOrder];
    float *part;          // [nblocks][N][J4][R16]
    double *loss_part;    // [nblocks]
    int *blocks_used;     // host: the grid actually launched
    const float *Cst[kMaxOrder];  // stored C^(n) = A^(n) B^(n), I_n x R16
                                  // (core_grad_stored_kernel only)
};
// Upper bound of the core-gradient grid (partial buffers are sized for it);
// the launch may use fewer blocks (what fits on the device at once).
int core_grad_blocks(int64_t count);
hipError_t launch_core_grad(const Shape &sh, const CoreArgs &a, int nblocks,
                            hipStream_t s);
// Storage variant: C^(n) = A^(n) B^(n) formed once per pass into Cst
// (rows x R16), then the same partials from gathered rows of C and A (FP32).
hipError_t launch_precompute_c(const Shape &sh, const float *A, const float *B,
                               int64_t rows, float *Cst, hipStream_t s);
hipError_t launch_core_grad_stored(const Shape &sh, const CoreArgs &a,
                                   int nblocks, hipStream_t s);
// The same partials from vector FP32 FMAs (FP32 only; the ablation of the
// matrix cores). The grid is capped by residency and by the chunk count.
hipError_t launch_core_grad_valu(const Shape &sh, const CoreArgs &a,
                                 int nblocks, hipStream_t s);

struct CoreUpdateArgs {
    const float *part;    // [nblocks][N][J4][R16]
    int nblocks;
    float *B[kMaxOrder];
    float *grad_out;      // [N][J4][R16] or nullptr
    double inv_count;     // 1 / |Omega| (or 1 / minibatch size)
    float lr, lam;
    int apply;
    // unpadded per-mode output (J_n x R row-major), scaled by *scale
    float *gout[kMaxOrder];
    int Jn[kMaxOrder];
    int R;
    const float *scale;
};
hipError_t launch_core_update(const Shape &sh, const CoreUpdateArgs &a,
                              hipStream_t s);

// ---------------------------------------------------------------- autograd
// dst (J4 x R16, zero padded) <- src (J x R dense row-major)
hipError_t launch_pad_matrix(const float *src, int J, int R, float *dst,
                             int J4, int R16, hipStream_t s);
// Unique-row ordinals of a sorted row array per mode: ordinal[i] = number of
// segment heads before i; total[n] = number of unique rows (int64).
struct UniqueScan {
    int N;
    int32_t m;
    int ntiles;
    const uint32_t *rows[kMaxOrder];
    uint32_t *ordinal[kMaxOrder];
    uint32_t *tile_count;   // [N][ntiles]
    int64_t *total;         // [N]
};
hipError_t launch_unique_scan(const UniqueScan &u, hipStream_t s);
hipError_t launch_fill_zero(float *p, int64_t n, hipStream_t s);

// ---------------------------------------------------------------- evaluation
struct EvalArgs {
    const uint16_t *A16[kMaxOrder];  // BF16 shadow of A (BF16 only)
    const uint8_t *A8[kMaxOrder];    // FP8 shadow of A and its row scales
    const float *As[kMaxOrder];      // (FP8 only)
    const int32_t *idx[kMaxOrder];
    const float *val;
    int64_t count;
    const float *A[kMaxOrder];
    const float *B[kMaxOrder];
    double *part;         // [nblocks][2]: sum r^2, sum |r|
    int half_square;      // 1: first sum is sum r^2 / 2
};
int eval_blocks(int64_t count);
hipError_t launch_eval(const Shape &sh, const EvalArgs &a, int nblocks,
                       hipStream_t s);
hipError_t launch_sumsq(const float *x, int64_t n, double *part, int nblocks,
                        hipStream_t s);

}  // namespace ft
