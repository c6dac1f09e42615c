// k_factor.hip -- factor phase of FastTuckerPlus on CDNA4 (Algorithm 3 first
// loop, update rule Eq. (12) in the matrix form of Eq. (14)).
//
// factor_grad_kernel: one wave per 16-sample tile. For every sample s and
// mode n it gathers the row a^(n)_{i_n}, forms C^(n)T = B^(n)T A_Psi^(n)T on the
// matrix cores (samples along the lane's column, r along the accumulator
// rows), the leave-one-out products D^(n) = prod_{k != n} C^(k) (prefix and
// suffix products, in registers), xhat = C^(1) . D^(1) (sum over r by lane
// shuffles), r = xhat - x, and the row gradient
//     g^(n)_s = r_s * B^(n) d^(n)_s            (Eq. (8)),
// again on the matrix cores as G^T = B^(n) (r (*) D^(n))^T, which lands in the
// natural "sample-column" layout so it is stored as float4 rows with no
// transpose. All reads use A and B as they stand at the minibatch start.
//
// seg_reduce_kernel / seg_fixup_kernel: the deterministic row reduction.
// The builder has sorted every minibatch's samples by row (ties in minibatch
// order). Each group of lanes (one lane per column j) walks a fixed chunk of
// kSegChunk sorted samples in order, summing g per row; rows whose samples
// all lie in the chunk are finished there, the partial sums of rows that
// cross a chunk edge are finished by the fix-up kernel in chunk order. A
// finished row takes
//     G = sum_s g_s + k * lambda_A * a,   a <- a - lr_A * G   (or G / k)
// No floating-point atomics are used, so results are bitwise reproducible.
#include "ft_internal.h"
#include "mfma_tile.h"

namespace ft {

constexpr int kFactorThreads = 256;
constexpr int kFactorMaxBlocks = 2048;

int factor_grad_blocks(int32_t m) {
    int ntiles = (m + 15) / 16;
    int blocks = (ntiles + 3) / 4;
    if (blocks > kFactorMaxBlocks) blocks = kFactorMaxBlocks;
    return blocks < 1 ? 1 : blocks;
}

// Per-wave state and arithmetic of one 16-sample tile (shared by the
// deterministic and the Hogwild factor kernels).
template <int N, int KQ, int RB, bool BF>
struct FactorTile {
    static constexpr int J4 = 4 * KQ;
    static constexpr int R16 = 16 * RB;
    static constexpr int JB = (KQ + 3) / 4;   // 16-row output blocks of J4
    int q, c;
    // A-operands: B^(n)T for the contraction over j (FP32 or BF16 packs),
    // B^(n) for the one over r (FP32)
    ColFrag<KQ, BF> bf[N][RB];
    float bb[N][JB][RB][4];
    floatx4 D[N][RB];

    __device__ __forceinline__ void load_B(const float *const *Bm) {
        const int lane = threadIdx.x & 63;
        q = lane >> 4;
        c = lane & 15;
#pragma unroll
        for (int n = 0; n < N; ++n) {
            const float *B = Bm[n];
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) bf[n][rb].load(B, R16, q, 16 * rb + c);
#pragma unroll
            for (int jb = 0; jb < JB; ++jb) {
                const int j = 16 * jb + c;
#pragma unroll
                for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                    for (int v = 0; v < 4; ++v)
                        bb[n][jb][rb][v] =
                            j < J4 ? B[j * R16 + 16 * rb + 4 * q + v] : 0.f;
            }
        }
    }

    // Sample ps (this lane's column): gather its rows, C^(n)T on the matrix
    // cores, D^(n) by prefix/suffix products; returns xhat (all four lanes of
    // the column hold it).
    __device__ __forceinline__ float forward(const int32_t *const *idx,
                                             const float *const *A,
                                             const uint16_t *const *A16,
                                             int64_t ps, int *rows) {
        RowFrag<KQ, BF> arow[N];
#pragma unroll
        for (int n = 0; n < N; ++n) {
            rows[n] = idx[n][ps];
            arow[n].load(A[n], A16[n], (int64_t)rows[n] * J4 + KQ * q);
        }
        floatx4 C[N][RB];
#pragma unroll
        for (int n = 0; n < N; ++n)
#pragma unroll
            for (int rb = 0; rb < RB; ++rb)
                C[n][rb] = contract(bf[n][rb], arow[n],
                                    floatx4{0.f, 0.f, 0.f, 0.f});
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
            floatx4 pre = {1.f, 1.f, 1.f, 1.f};
#pragma unroll
            for (int n = 0; n < N; ++n) {
                D[n][rb] = pre;
                pre *= C[n][rb];
            }
            floatx4 suf = {1.f, 1.f, 1.f, 1.f};
#pragma unroll
            for (int n = N - 1; n >= 0; --n) {
                D[n][rb] *= suf;
                suf *= C[n][rb];
            }
        }
        float xh = 0.f;
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int v = 0; v < 4; ++v) xh += C[0][rb][v] * D[0][rb][v];
        return sum_quads(xh);
    }

    // Rows 16 jb + 4q .. +3 of g^(n) = r * B^(n) d^(n) for this lane's sample.
    __device__ __forceinline__ floatx4 grad(int n, int jb, float r) const {
        floatx4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int v = 0; v < 4; ++v)
                acc = mfma_16x16x4(bb[n][jb][rb][v], r * D[n][rb][v], acc);
        return acc;
    }
};

template <int N, int KQ, int RB, bool BF>
__global__ __launch_bounds__(kFactorThreads) void factor_grad_kernel(
    FactorArgs a, int ntiles) {
    using T = FactorTile<N, KQ, RB, BF>;
    T tl;
    tl.load_B(a.B);
    double loss = 0.0;
    const int nwaves = gridDim.x * (kFactorThreads / 64);
    for (int tile = blockIdx.x * (kFactorThreads / 64) + (threadIdx.x >> 6);
         tile < ntiles; tile += nwaves) {
        const int p = tile * 16 + tl.c;
        const bool valid = p < a.m;
        const int ps = valid ? p : a.m - 1;
        int rows[N];
        const float xh = tl.forward(a.idx, a.A, a.A16, ps, rows);
        const float r = valid ? xh - a.val[ps] : 0.f;
        if (valid && tl.q == 0) loss += 0.5 * (double)r * (double)r;
#pragma unroll
        for (int n = 0; n < N; ++n) {
            float *Gn = a.G + ((int64_t)n * a.m + p) * T::J4;
#pragma unroll
            for (int jb = 0; jb < T::JB; ++jb) {
                const floatx4 g = tl.grad(n, jb, r);
                const int j0 = 16 * jb + 4 * tl.q;
                if (valid && j0 < T::J4)
                    *reinterpret_cast<floatx4 *>(Gn + j0) = g;
            }
        }
    }
    const double tot = block_sum_256(loss);
    if (threadIdx.x == 0) a.loss_part[blockIdx.x] = tot;
}

// Hogwild fast mode (the paper's execution model, Algorithm 4): persistent
// waves sweep all 16-sample tiles of the epoch order with no minibatch
// barrier; each tile reads its rows, forms g, and applies
// a <- a - lr_A (g + lambda_A a) at once with hardware float atomics, so
// concurrent tiles race on shared rows by design. One FP64 loss per tile.
template <int N, int KQ, int RB>
__global__ __launch_bounds__(kFactorThreads) void hogwild_kernel(HogArgs a) {
    using T = FactorTile<N, KQ, RB, false>;
    T tl;
    tl.load_B(a.B);
    const int64_t ntiles = (a.count + 15) / 16;
    const int64_t nwaves = (int64_t)gridDim.x * (kFactorThreads / 64);
    for (int64_t tile = (int64_t)blockIdx.x * (kFactorThreads / 64) +
                        (threadIdx.x >> 6);
         tile < ntiles; tile += nwaves) {
        const int64_t p = tile * 16 + tl.c;
        const bool valid = p < a.count;
        const int64_t ps = valid ? p : a.count - 1;
        int rows[N];
        const float xh = tl.forward(a.idx, a.A, a.A16, ps, rows);
        const float r = valid ? xh - a.val[ps] : 0.f;
        double tl_loss = (valid && tl.q == 0) ? 0.5 * (double)r * (double)r : 0.0;
        tl_loss = wave_sum(tl_loss);
        if ((threadIdx.x & 63) == 0) a.tile_loss[tile] = tl_loss;
#pragma unroll
        for (int n = 0; n < N; ++n) {
#pragma unroll
            for (int jb = 0; jb < T::JB; ++jb) {
                const floatx4 g = tl.grad(n, jb, r);
                const int j0 = 16 * jb + 4 * tl.q;
                if (valid && j0 < T::J4) {
                    float *ap = a.A[n] + (int64_t)rows[n] * T::J4 + j0;
#pragma unroll
                    for (int v = 0; v < 4; ++v)
                        unsafeAtomicAdd(ap + v, -a.lr * (g[v] + a.lam * ap[v]));
                }
            }
        }
    }
}

template <int N, int KQ, int RB, bool BF>
static hipError_t launch_fg(const FactorArgs &a, int blocks, hipStream_t s) {
    const int ntiles = (a.m + 15) / 16;
    hipLaunchKernelGGL((factor_grad_kernel<N, KQ, RB, BF>), dim3(blocks),
                       dim3(kFactorThreads), 0, s, a, ntiles);
    return hipGetLastError();
}

template <int N, int KQ>
static hipError_t launch_fg_r(const Shape &sh, const FactorArgs &a, int blocks,
                              hipStream_t s) {
    if (sh.bf16)
        return sh.R16 == 16 ? launch_fg<N, KQ, 1, true>(a, blocks, s)
                            : launch_fg<N, KQ, 2, true>(a, blocks, s);
    return sh.R16 == 16 ? launch_fg<N, KQ, 1, false>(a, blocks, s)
                        : launch_fg<N, KQ, 2, false>(a, blocks, s);
}

template <int N>
static hipError_t launch_fg_j(const Shape &sh, const FactorArgs &a, int blocks,
                              hipStream_t s) {
    switch (sh.J4) {
    case 4: return launch_fg_r<N, 1>(sh, a, blocks, s);
    case 8: return launch_fg_r<N, 2>(sh, a, blocks, s);
    case 12: return launch_fg_r<N, 3>(sh, a, blocks, s);
    case 16: return launch_fg_r<N, 4>(sh, a, blocks, s);
    case 20: return launch_fg_r<N, 5>(sh, a, blocks, s);
    case 24: return launch_fg_r<N, 6>(sh, a, blocks, s);
    case 28: return launch_fg_r<N, 7>(sh, a, blocks, s);
    case 32: return launch_fg_r<N, 8>(sh, a, blocks, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_factor_grad(const Shape &sh, const FactorArgs &a, int *nblocks,
                              hipStream_t s) {
    const int blocks = factor_grad_blocks(a.m);
    *nblocks = blocks;
    switch (sh.N) {
    case 2: return launch_fg_j<2>(sh, a, blocks, s);
    case 3: return launch_fg_j<3>(sh, a, blocks, s);
    case 4: return launch_fg_j<4>(sh, a, blocks, s);
    case 5: return launch_fg_j<5>(sh, a, blocks, s);
    }
    return hipErrorInvalidValue;
}

template <int N, int KQ, int RB>
static hipError_t launch_hw(const HogArgs &a, int blocks, hipStream_t s) {
    hipLaunchKernelGGL((hogwild_kernel<N, KQ, RB>), dim3(blocks),
                       dim3(kFactorThreads), 0, s, a);
    return hipGetLastError();
}

template <int N, int KQ>
static hipError_t launch_hw_r(const Shape &sh, const HogArgs &a, int blocks,
                              hipStream_t s) {
    return sh.R16 == 16 ? launch_hw<N, KQ, 1>(a, blocks, s)
                        : launch_hw<N, KQ, 2>(a, blocks, s);
}

template <int N>
static hipError_t launch_hw_j(const Shape &sh, const HogArgs &a, int blocks,
                              hipStream_t s) {
    switch (sh.J4) {
    case 4: return launch_hw_r<N, 1>(sh, a, blocks, s);
    case 8: return launch_hw_r<N, 2>(sh, a, blocks, s);
    case 12: return launch_hw_r<N, 3>(sh, a, blocks, s);
    case 16: return launch_hw_r<N, 4>(sh, a, blocks, s);
    case 20: return launch_hw_r<N, 5>(sh, a, blocks, s);
    case 24: return launch_hw_r<N, 6>(sh, a, blocks, s);
    case 28: return launch_hw_r<N, 7>(sh, a, blocks, s);
    case 32: return launch_hw_r<N, 8>(sh, a, blocks, s);
    }
    return hipErrorInvalidValue;
}

int hogwild_blocks(int64_t count) {
    int64_t ntiles = (count + 15) / 16;
    int64_t blocks = (ntiles + 3) / 4;
    if (blocks > kFactorMaxBlocks) blocks = kFactorMaxBlocks;
    return blocks < 1 ? 1 : (int)blocks;
}

hipError_t launch_hogwild(const Shape &sh, const HogArgs &a, hipStream_t s) {
    const int blocks = hogwild_blocks(a.count);
    switch (sh.N) {
    case 2: return launch_hw_j<2>(sh, a, blocks, s);
    case 3: return launch_hw_j<3>(sh, a, blocks, s);
    case 4: return launch_hw_j<4>(sh, a, blocks, s);
    case 5: return launch_hw_j<5>(sh, a, blocks, s);
    }
    return hipErrorInvalidValue;
}

// ------------------------------------------------------------ row reduction
__device__ __forceinline__ void finish_row(const SegArgs &a, int n, int j,
                                           bool col, uint32_t row, float sum,
                                           int cnt, int start) {
    if (!col) return;
    if (a.apply == 2) {
        // autograd: gradient of the data term only, times grad_out
        const float g = sum * (a.scale ? *a.scale : 1.f);
        if (a.grad[n]) a.grad[n][(int64_t)row * a.J4 + j] = g;
        if (a.uniq_grad[n]) {
            const uint32_t ord = a.ordinal[n][start];
            a.uniq_grad[n][(int64_t)ord * a.J4 + j] = g;
            if (j == 0 && a.uniq_rows[n]) a.uniq_rows[n][ord] = (int32_t)row;
        }
        return;
    }
    float *ap = a.A[n] + (int64_t)row * a.J4 + j;
    const float av = *ap;
    float g = sum + (float)cnt * a.lam * av;
    if (a.apply) {
        if (a.mean) g /= (float)cnt;
        const float nv = av - a.lr * g;
        *ap = nv;
        if (a.A16[n]) a.A16[n][(int64_t)row * a.J4 + j] = f2bf(nv);
    } else {
        a.grad[n][(int64_t)row * a.J4 + j] = g;
        if (j == 0) a.count[n][row] = cnt;
    }
}

template <int LP>
__global__ __launch_bounds__(256) void seg_reduce_kernel(SegArgs a) {
    const int g = blockIdx.x * (256 / LP) + threadIdx.x / LP;
    const int j = threadIdx.x % LP;
    if (g >= a.N * a.nchunks) return;
    const int n = g / a.nchunks, c = g % a.nchunks;
    const int i0 = c * kSegChunk;
    const int i1 = min(i0 + kSegChunk, a.m);
    const uint32_t *rows = a.rows[n];
    const uint32_t *pos = a.pos[n];
    const float *G = a.G + (int64_t)n * a.m * a.J4;
    const bool col = j < a.J4;
    const uint32_t first_row = rows[i0];
    const bool starts_before = i0 > 0 && rows[i0 - 1] == first_row;
    const bool continues_after = i1 < a.m && rows[i1] == rows[i1 - 1];
    float *first = a.first + ((int64_t)n * a.nchunks + c) * a.J4 + j;
    float *last = a.last + ((int64_t)n * a.nchunks + c) * a.J4 + j;

    float acc = 0.f;
    int cnt = 0;
    int start = i0;
    uint32_t cur = first_row;
    bool is_first = true;
    for (int base = i0; base < i1; base += 8) {
        uint32_t rr[8];
        float gg[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int i = base + u;
            rr[u] = i < i1 ? rows[i] : cur;
            gg[u] = (i < i1 && col) ? G[(int64_t)pos[i] * a.J4 + j] : 0.f;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            if (base + u >= i1) break;
            if (rr[u] != cur) {
                // close the fragment of row `cur`; it cannot continue past the
                // chunk, so it is finished here unless it started before
                if (is_first && starts_before) {
                    if (col) *first = acc;
                } else {
                    finish_row(a, n, j, col, cur, acc, cnt, start);
                }
                acc = 0.f;
                cnt = 0;
                start = base + u;
                cur = rr[u];
                is_first = false;
            }
            acc += gg[u];
            ++cnt;
        }
    }
    const bool span_before = is_first && starts_before;
    if (!span_before && !continues_after) {
        finish_row(a, n, j, col, cur, acc, cnt, start);
    } else if (col) {
        if (is_first) *first = acc;
        *last = acc;
    }
}

__global__ __launch_bounds__(256) void seg_fixup_kernel(SegArgs a, int LP) {
    const int g = blockIdx.x * (256 / LP) + threadIdx.x / LP;
    const int j = threadIdx.x % LP;
    if (g >= a.N * a.nchunks) return;
    const int n = g / a.nchunks, c = g % a.nchunks;
    const int i0 = c * kSegChunk;
    if (i0 == 0) return;
    const uint32_t *rows = a.rows[n];
    const uint32_t row = rows[i0];
    if (rows[i0 - 1] != row) return;              // segment starts in c
    const int i1 = min(i0 + kSegChunk, a.m);
    if (i1 < a.m && rows[i1 - 1] == row && rows[i1] == row)
        return;                                   // segment ends after c
    int lo = 0, hi = i0;                          // first sorted index of row
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (rows[mid] < row) lo = mid + 1; else hi = mid;
    }
    const int start = lo;
    int end = i0;
    while (end < i1 && rows[end] == row) ++end;
    const bool col = j < a.J4;
    if (!col) return;
    const int c0 = start / kSegChunk;
    const float *first = a.first + (int64_t)n * a.nchunks * a.J4 + j;
    const float *last = a.last + (int64_t)n * a.nchunks * a.J4 + j;
    float acc = last[(int64_t)c0 * a.J4];
    for (int cc = c0 + 1; cc <= c; ++cc) acc += first[(int64_t)cc * a.J4];
    finish_row(a, n, j, col, row, acc, end - start, start);
}

static int lanes_per_group(int J4) {
    int lp = 4;
    while (lp < J4) lp <<= 1;
    return lp;
}

hipError_t launch_seg_reduce(const SegArgs &a, hipStream_t s) {
    const int lp = lanes_per_group(a.J4);
    const int groups = a.N * a.nchunks;
    const int blocks = (groups + 256 / lp - 1) / (256 / lp);
    switch (lp) {
    case 4: hipLaunchKernelGGL(seg_reduce_kernel<4>, dim3(blocks), dim3(256), 0, s, a); break;
    case 8: hipLaunchKernelGGL(seg_reduce_kernel<8>, dim3(blocks), dim3(256), 0, s, a); break;
    case 16: hipLaunchKernelGGL(seg_reduce_kernel<16>, dim3(blocks), dim3(256), 0, s, a); break;
    case 32: hipLaunchKernelGGL(seg_reduce_kernel<32>, dim3(blocks), dim3(256), 0, s, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_seg_fixup(const SegArgs &a, hipStream_t s) {
    const int lp = lanes_per_group(a.J4);
    const int groups = a.N * a.nchunks;
    const int blocks = (groups + 256 / lp - 1) / (256 / lp);
    hipLaunchKernelGGL(seg_fixup_kernel, dim3(blocks), dim3(256), 0, s, a, lp);
    return hipGetLastError();
}

// ------------------------------------------------------------ block sums
// out[g] = sum of part[g*nper .. g*nper + nper) in a fixed order.
__global__ __launch_bounds__(256) void sum_blocks_kernel(const double *part,
                                                         int nper,
                                                         double *out) {
    const double *p = part + (int64_t)blockIdx.x * nper;
    double acc = 0.0;
    for (int i = threadIdx.x; i < nper; i += 256) acc += p[i];
    const double t = block_sum_256(acc);
    if (threadIdx.x == 0) out[blockIdx.x] = t;
}

hipError_t launch_sum_blocks(const double *part, int nper, int ngroups,
                             double *out, hipStream_t s) {
    if (ngroups <= 0) return hipSuccess;
    hipLaunchKernelGGL(sum_blocks_kernel, dim3(ngroups), dim3(256), 0, s, part,
                       nper, out);
    return hipGetLastError();
}

}  // namespace ft
