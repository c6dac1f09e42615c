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
// transpose, at the sample's slot in the mode's sorted order (from the
// builder), so the row reduction reads each row's gradients contiguously.
// All reads use A and B as they stand at the minibatch start.
//
// seg_reduce_kernel: the deterministic row reduction. The builder has sorted
// every minibatch's samples by row (ties in minibatch order) and listed the
// rows whose samples cross a chunk edge. A wave takes a fixed chunk of
// kSegChunk sorted samples, one per lane, and sums each row's gradients by a
// segmented scan across its lanes; every listed crossing row gets a block of
// its own. A finished row takes
//     G = sum_s g_s + k * lambda_A * a,   a <- a - lr_A * G   (or G / k)
// No floating-point atomics are used, so results are bitwise reproducible.
#include "ft_internal.h"
#include "mfma_tile.h"

namespace ft {

constexpr int kFactorThreads = 256;
#ifndef FT_FACTOR_MAX_BLOCKS
#define FT_FACTOR_MAX_BLOCKS 2048
#endif
constexpr int kFactorMaxBlocks = FT_FACTOR_MAX_BLOCKS;
// Grid cap for shapes whose B operands live in LDS (large N J R): each block
// first stages B and builds the operand words (tens of KB of LDS writes), so
// fewer blocks that loop over more tiles spend less of their time on it.
#ifndef FT_FACTOR_LDS_CAP
#define FT_FACTOR_LDS_CAP 2048
#endif
constexpr int kFactorLdsCap = FT_FACTOR_LDS_CAP;
constexpr int kFactorTilesPerWave = 1;

// Operand words per lane of the factor tile (FactorTile::OPW), from the
// padded shape: the A-operand fragments of B^T (FP32: KQ words; BF16: two
// per four entries; FP8: two per eight entries plus the scale, 8-byte
// aligned) for every mode and column block, and the FP32 B fragments.
constexpr int factor_operand_words(int N, int J4, int R16, int prec) {
    const int KQ = J4 / 4, RB = R16 / 16, JB = (KQ + 3) / 4;
    const int cfw = prec == kBF16 ? 2 * ((KQ + 3) / 4)
                    : prec == kFP8 ? 2 * ((KQ + 7) / 8) + 2
                                   : KQ;
    return N * RB * cfw + N * JB * RB * 4;
}
static int factor_operand_words(const Shape &sh) {
    return factor_operand_words(sh.N, sh.J4, sh.R16, sh.prec);
}

int factor_grad_blocks(const Shape &sh, int32_t m) {
    int ntiles = (m + 15) / 16;
    int blocks = (ntiles + 4 * kFactorTilesPerWave - 1) /
                 (4 * kFactorTilesPerWave);
    const int cap = factor_operand_words(sh) > 48 ? kFactorLdsCap
                                                  : kFactorMaxBlocks;
    if (blocks > cap) blocks = cap;
    return blocks < 1 ? 1 : blocks;
}

// Per-wave state and arithmetic of one 16-sample tile (shared by the
// deterministic and the Hogwild factor kernels).
template <int N, int KQ, int RB, int P>
struct FactorTile {
    static constexpr int J4 = 4 * KQ;
    static constexpr int R16 = 16 * RB;
    static constexpr int JB = (KQ + 3) / 4;   // 16-row output blocks of J4
    // Operand words per lane: the A-operands B^(n)T of the contraction over
    // j (FP32, BF16 or FP8 packs) and B^(n) of the one over r (FP32). They
    // are the same in every wave; small sets stay in registers, large ones
    // (J = R = 32 and order 4-5: up to 160 words) are kept in LDS, one copy
    // per block laid out [word][lane], and read when a step needs them, so
    // the registers go to waves in flight instead.
    static constexpr int CFW = sizeof(ColFrag<KQ, P>) / 4;
    static constexpr int OPW = N * RB * CFW + N * JB * RB * 4;
    static constexpr bool kLdsOps = OPW > 48;
    static_assert(OPW == factor_operand_words(N, J4, R16, P),
                  "the grid cap's operand count must match the tile's");
    int q, c, lane;
    ColFrag<KQ, P> bf[N][RB];
    float bb[N][JB][RB][4];
    const uint32_t *ops;             // LDS operand words (kLdsOps)
    floatx4 D[N][RB];

    // Operands from B (global memory, or the LDS copy the Hogwild kernel
    // stages). With kLdsOps wave 0 writes them to ops_lds and the caller
    // synchronises the block before the first tile.
    __device__ __forceinline__ void load_B(const float *const *Bm,
                                           uint32_t *ops_lds) {
        lane = threadIdx.x & 63;
        q = lane >> 4;
        c = lane & 15;
        ops = ops_lds;
        if constexpr (kLdsOps) {
            if (threadIdx.x >= 64) return;
        }
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
        if constexpr (kLdsOps) {
#pragma unroll
            for (int n = 0; n < N; ++n)
#pragma unroll
                for (int rb = 0; rb < RB; ++rb) {
                    uint32_t w[CFW];
                    __builtin_memcpy(w, &bf[n][rb], sizeof(w));
#pragma unroll
                    for (int i = 0; i < CFW; ++i)
                        ops_lds[((n * RB + rb) * CFW + i) * 64 + lane] = w[i];
                }
#pragma unroll
            for (int n = 0; n < N; ++n)
#pragma unroll
                for (int jb = 0; jb < JB; ++jb)
#pragma unroll
                    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                        for (int v = 0; v < 4; ++v)
                            ops_lds[(N * RB * CFW +
                                     ((n * JB + jb) * RB + rb) * 4 + v) * 64 +
                                    lane] = __float_as_uint(bb[n][jb][rb][v]);
        }
    }

    // The lane index is passed through an empty asm statement at every use,
    // so the compiler cannot hoist the LDS reads out of the tile loop (which
    // would bring the operands back into registers).
    __device__ __forceinline__ int opaque_lane() const {
        int l = lane;
        asm volatile("" : "+v"(l));
        return l;
    }

    __device__ __forceinline__ ColFrag<KQ, P> bfrag(int n, int rb) const {
        if constexpr (kLdsOps) {
            const uint32_t *o = ops + opaque_lane();
            uint32_t w[CFW];
#pragma unroll
            for (int i = 0; i < CFW; ++i)
                w[i] = o[((n * RB + rb) * CFW + i) * 64];
            ColFrag<KQ, P> f;
            __builtin_memcpy(&f, w, sizeof(w));
            return f;
        } else {
            return bf[n][rb];
        }
    }

    __device__ __forceinline__ float bbv(int n, int jb, int rb, int v) const {
        if constexpr (kLdsOps)
            return __uint_as_float(
                ops[(N * RB * CFW + ((n * JB + jb) * RB + rb) * 4 + v) * 64 +
                    opaque_lane()]);
        else
            return bb[n][jb][rb][v];
    }

    // Gather the rows of sample ps (this lane's column).
    template <class Args>
    __device__ __forceinline__ void gather(const Args &a, int64_t ps,
                                           int *rows,
                                           RowFrag<KQ, P> *arow) const {
#pragma unroll
        for (int n = 0; n < N; ++n) {
            rows[n] = a.idx[n][ps];
            arow[n].load(RowSrc{a.A[n], a.A16[n], a.A8[n], a.As[n]}, rows[n],
                         J4, q);
        }
    }

    // C^(n)T on the matrix cores, D^(n) by prefix/suffix products; returns
    // xhat of this lane's sample (all four lanes of the column hold it).
    template <class Args>
    __device__ __forceinline__ float forward(const Args &a, int64_t ps,
                                             int *rows) {
        RowFrag<KQ, P> arow[N];
        gather(a, ps, rows, arow);
        return contract_rows(arow);
    }

    __device__ __forceinline__ float contract_rows(
        const RowFrag<KQ, P> *arow) {
        floatx4 C[N][RB];
#pragma unroll
        for (int n = 0; n < N; ++n)
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) {
                const ColFrag<KQ, P> x = bfrag(n, rb);
                C[n][rb] = contract(x, arow[n], floatx4{0.f, 0.f, 0.f, 0.f});
                if constexpr (P == kFP8)
                    C[n][rb] = fp8_scale_ct(C[n][rb], x.s, arow[n].s, q);
            }
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
                acc = mfma_16x16x4(bbv(n, jb, rb, v), r * D[n][rb][v], acc);
        return acc;
    }
};

// The block copies B^(1..N) into LDS once (float4 loads) and every wave
// takes its two operand layouts from there.
template <int N, int E>
__device__ __forceinline__ void stage_B(const float *const *B, float *sB,
                                        const float **sBm) {
#pragma unroll
    for (int n = 0; n < N; ++n) {
        const float4 *src = reinterpret_cast<const float4 *>(B[n]);
        float4 *dst = reinterpret_cast<float4 *>(sB + n * E);
        for (int i = threadIdx.x; i < E / 4; i += kFactorThreads)
            dst[i] = src[i];
        sBm[n] = sB + n * E;
    }
    __syncthreads();
}

// Each wave sweeps its tiles (one or two per wave at the large shapes) and
// gathers each tile's rows when it starts it; the hardware hides the gather
// latency with the other waves. Holding the next tile's rows in registers
// (a software prefetch) and staging B in LDS before building the operands
// both cost registers or LDS that kept a wave per SIMD out, and measured
// slower at order 4-5, J = R = 32 (without them, per minibatch: order 5 BF16
// 98 -> 79 us, order 4 FP32 96 -> 82 us) and no faster elsewhere.
// Waves per SIMD the register allocator is asked to reach. Without a hint
// it reserves accumulator registers apart and lands one wave lower on most
// shapes; two is reached by every shape without spilling or scratch
// (checked per instantiation at build time). Asking for three where it
// fits (order 4, J = R = 32) made the kernel faster but slowed the builder
// running beside it, and the epoch with it. Order 10 at J = 16, R = 32 needs
// one wave per SIMD to stay in registers.
constexpr int factor_waves(int N, int KQ, int RB, int) {
    return N > kFullOrder && N * KQ * RB >= 80 ? 1 : 2;
}


template <int N, int KQ, int RB, int P>
__global__ __launch_bounds__(kFactorThreads)
__attribute__((amdgpu_waves_per_eu(factor_waves(N, KQ, RB, P)))) void
factor_grad_kernel(
    FactorArgs a, int ntiles) {
    using T = FactorTile<N, KQ, RB, P>;
    __shared__ uint32_t sOps[T::kLdsOps ? T::OPW * 64 : 1];
    T tl;
    tl.q = (threadIdx.x & 63) >> 4;
    tl.c = threadIdx.x & 15;
    double loss = 0.0;
    const int nwaves = gridDim.x * (kFactorThreads / 64);
    int tile = blockIdx.x * (kFactorThreads / 64) + (threadIdx.x >> 6);
    int rows[N];
    RowFrag<KQ, P> arow[N];
    float x = 0.f;
    // the first tile's gathers are issued before the B operands are built,
    // so their latency overlaps that and its barrier
    if (tile < ntiles) {
        const int p = tile * 16 + tl.c;
        const int ps = p < a.m ? p : a.m - 1;
        tl.gather(a, ps, rows, arow);
        x = a.val[ps];
    }
    tl.load_B(a.B, sOps);
    if constexpr (T::kLdsOps) __syncthreads();
    for (bool first = true; tile < ntiles; tile += nwaves, first = false) {
        const int p = tile * 16 + tl.c;
        const bool valid = p < a.m;
        const int ps = valid ? p : a.m - 1;
        if (!first) {
            tl.gather(a, ps, rows, arow);
            x = a.val[ps];
        }
        // sorted slots, read at a clamped index rather than under a branch:
        // a branch around each load made it wait before the next one
        uint32_t inv[N];
#pragma unroll
        for (int n = 0; n < N; ++n) inv[n] = a.inv[n][ps];
        const float xh = tl.contract_rows(arow);
        const float r = valid ? xh - x : 0.f;
        if (valid && tl.q == 0) loss += 0.5 * (double)r * (double)r;
#pragma unroll
        for (int n = 0; n < N; ++n) {
            float *Gn = a.G + ((int64_t)n * a.m + inv[n]) * T::J4;
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
// concurrent tiles race on shared rows by design. Samples of one tile that
// share a row are summed first (lane shuffles) and the row takes one step
// a <- a - lr_A (sum g + k lambda_A a): the tile is a Jacobi step of 16
// samples, and a hot row takes one atomic per tile instead of one per
// sample. One FP64 loss per tile.
template <int N, int KQ, int RB>
__global__ __launch_bounds__(kFactorThreads) void hogwild_kernel(HogArgs a) {
    using T = FactorTile<N, KQ, RB, kF32>;
    __shared__ float sB[N * T::J4 * T::R16];
    __shared__ uint32_t sOps[T::kLdsOps ? T::OPW * 64 : 1];
    const float *sBm[N];
    stage_B<N, T::J4 * T::R16>(a.B, sB, sBm);
    T tl;
    tl.load_B(sBm, sOps);
    if constexpr (T::kLdsOps) __syncthreads();
    const int64_t ntiles = (a.count + 15) / 16;
    const int64_t nwaves = (int64_t)gridDim.x * (kFactorThreads / 64);
    for (int64_t tile = (int64_t)blockIdx.x * (kFactorThreads / 64) +
                        (threadIdx.x >> 6);
         tile < ntiles; tile += nwaves) {
        const int64_t p = tile * 16 + tl.c;
        const bool valid = p < a.count;
        const int64_t ps = valid ? p : a.count - 1;
        int rows[N];
        const float xh = tl.forward(a, ps, rows);
        const float r = valid ? xh - a.val[ps] : 0.f;
        double tl_loss = (valid && tl.q == 0) ? 0.5 * (double)r * (double)r : 0.0;
        tl_loss = wave_sum(tl_loss);
        if ((threadIdx.x & 63) == 0) a.tile_loss[tile] = tl_loss;
#pragma unroll
        for (int n = 0; n < N; ++n) {
            // the tile's samples on this lane's row (bit k: sample k; lane k
            // holds sample k); padding lanes match nothing
            const int myrow = valid ? rows[n] : -1 - tl.c;
            uint32_t peers = 0;
#pragma unroll
            for (int k = 0; k < 16; ++k)
                peers |= (__shfl(myrow, k) == myrow ? 1u : 0u) << k;
            const bool leader = (peers & ((1u << tl.c) - 1u)) == 0u;
            const int cnt = __popc(peers);
            const bool dup = __ballot(cnt > 1) != 0ull;   // wave-uniform
#pragma unroll
            for (int jb = 0; jb < T::JB; ++jb) {
                floatx4 g = tl.grad(n, jb, r);
                if (dup) {
                    // one step per row and tile: the sum of its samples'
                    // gradients, applied by the first of them
                    floatx4 sum = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                    for (int k = 0; k < 16; ++k) {
                        floatx4 gk;
#pragma unroll
                        for (int v = 0; v < 4; ++v)
                            gk[v] = __shfl(g[v], 16 * tl.q + k);
                        if ((peers >> k) & 1u) sum += gk;
                    }
                    g = sum;
                }
                const int j0 = 16 * jb + 4 * tl.q;
                // the row's current entries, read by every lane from an
                // in-bounds address before the branch (a read inside it
                // would be waited for there, once per store)
                float *ap = a.A[n] + (int64_t)rows[n] * T::J4 +
                            (j0 < T::J4 ? j0 : T::J4 - 4);
                const float4 av = *reinterpret_cast<const float4 *>(ap);
                if (valid && leader && j0 < T::J4) {
                    const float k = (float)cnt * a.lam;
                    unsafeAtomicAdd(ap + 0, -a.lr * (g[0] + k * av.x));
                    unsafeAtomicAdd(ap + 1, -a.lr * (g[1] + k * av.y));
                    unsafeAtomicAdd(ap + 2, -a.lr * (g[2] + k * av.z));
                    unsafeAtomicAdd(ap + 3, -a.lr * (g[3] + k * av.w));
                }
            }
        }
    }
}

// ------------------------------------------------- vector-ALU factor kernel
// The factor kernel's arithmetic with vector FP32 FMAs instead of the matrix
// cores (for the ablation): one sample per lane; B^(1..N) staged in LDS and
// read by every lane at the same address (broadcast). Per sample
//     c^(n)_r = sum_j a^(n)_j B^(n)[j][r]           (all modes, in registers)
//     d^(n)_r = prod_{m != n} c^(m)_r,   xhat = sum_r c^(1)_r d^(1)_r,
//     g^(n)_j = (xhat - x) sum_r B^(n)[j][r] d^(n)_r,
// with the factor rows streamed four elements at a time, and each gradient
// row written to the sample's sorted slot like the matrix-core kernel.
template <int N, int J4, int R16>
__global__ __launch_bounds__(256) void factor_grad_valu_kernel(FactorArgs a) {
    __shared__ float sB[N * J4 * R16];
    const float *sBm[N];
    stage_B<N, J4 * R16>(a.B, sB, sBm);
    const int p = blockIdx.x * 256 + threadIdx.x;
    const bool valid = p < a.m;
    const int ps = valid ? p : a.m - 1;
    float C[N][R16];
#pragma unroll
    for (int n = 0; n < N; ++n) {
        const float4 *ar =
            reinterpret_cast<const float4 *>(a.A[n] + (int64_t)a.idx[n][ps] * J4);
#pragma unroll
        for (int r = 0; r < R16; ++r) C[n][r] = 0.f;
        // the row loop stays rolled so that the mode and rank loops unroll
        // fully and C stays in registers
#pragma unroll 1
        for (int jq = 0; jq < J4 / 4; ++jq) {
            const float4 v = ar[jq];
            const float av[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int e = 0; e < 4; ++e)
#pragma unroll
                for (int r = 0; r < R16; ++r)
                    C[n][r] = fmaf(av[e], sBm[n][(4 * jq + e) * R16 + r], C[n][r]);
        }
    }
    float xh = 0.f;
#pragma unroll
    for (int r = 0; r < R16; ++r) {
        float prod = C[0][r];
#pragma unroll
        for (int n = 1; n < N; ++n) prod *= C[n][r];
        xh += prod;
    }
    const float res = valid ? xh - a.val[ps] : 0.f;
    const double loss = valid ? 0.5 * (double)res * (double)res : 0.0;
    if (valid) {
#pragma unroll
        for (int n = 0; n < N; ++n) {
            float d[R16];
#pragma unroll
            for (int r = 0; r < R16; ++r) {
                float prod = 1.f;
#pragma unroll
                for (int m = 0; m < N; ++m)
                    if (m != n) prod *= C[m][r];
                d[r] = prod;
            }
            float4 *gr = reinterpret_cast<float4 *>(
                a.G + ((int64_t)n * a.m + a.inv[n][p]) * J4);
#pragma unroll 1
            for (int jq = 0; jq < J4 / 4; ++jq) {
                float g[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    float acc = 0.f;
#pragma unroll
                    for (int r = 0; r < R16; ++r)
                        acc = fmaf(sBm[n][(4 * jq + e) * R16 + r], d[r], acc);
                    g[e] = res * acc;
                }
                gr[jq] = make_float4(g[0], g[1], g[2], g[3]);
            }
        }
    }
    const double tot = block_sum_256(loss);
    if (threadIdx.x == 0) a.loss_part[blockIdx.x] = tot;
}

bool factor_valu_supported(const Shape &sh) {
    return sh.prec == kF32 && sh.N >= 2 && sh.N <= 5 && sh.J4 <= 32 &&
           sh.R16 <= 32;
}

template <int N, int J4>
static hipError_t launch_fgv_r(const Shape &sh, const FactorArgs &a, int blocks,
                               hipStream_t s) {
    if (sh.R16 == 16)
        FT_LAUNCH((factor_grad_valu_kernel<N, J4, 16>), dim3(blocks), dim3(256),
                  0, s, a);
    else if (sh.R16 == 32)
        FT_LAUNCH((factor_grad_valu_kernel<N, J4, 32>), dim3(blocks), dim3(256),
                  0, s, a);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

template <int N>
static hipError_t launch_fgv_j(const Shape &sh, const FactorArgs &a, int blocks,
                               hipStream_t s) {
    switch (sh.J4) {
    case 4: return launch_fgv_r<N, 4>(sh, a, blocks, s);
    case 8: return launch_fgv_r<N, 8>(sh, a, blocks, s);
    case 12: return launch_fgv_r<N, 12>(sh, a, blocks, s);
    case 16: return launch_fgv_r<N, 16>(sh, a, blocks, s);
    case 20: return launch_fgv_r<N, 20>(sh, a, blocks, s);
    case 24: return launch_fgv_r<N, 24>(sh, a, blocks, s);
    case 28: return launch_fgv_r<N, 28>(sh, a, blocks, s);
    case 32: return launch_fgv_r<N, 32>(sh, a, blocks, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_factor_grad_valu(const Shape &sh, const FactorArgs &a,
                                   int *nblocks, hipStream_t s) {
    if (!factor_valu_supported(sh)) return hipErrorInvalidValue;
    const int blocks = (a.m + 255) / 256;
    *nblocks = blocks;
    switch (sh.N) {
    case 2: return launch_fgv_j<2>(sh, a, blocks, s);
    case 3: return launch_fgv_j<3>(sh, a, blocks, s);
    case 4: return launch_fgv_j<4>(sh, a, blocks, s);
    case 5: return launch_fgv_j<5>(sh, a, blocks, s);
    }
    return hipErrorInvalidValue;
}

template <int N, int KQ, int RB, int P>
static hipError_t launch_fg(const FactorArgs &a, int blocks, hipStream_t s) {
    const int ntiles = (a.m + 15) / 16;
    FT_LAUNCH((factor_grad_kernel<N, KQ, RB, P>), dim3(blocks),
                       dim3(kFactorThreads), 0, s, a, ntiles);
    return hipGetLastError();
}

template <int N, int KQ, int P>
static hipError_t launch_fg_p(const Shape &sh, const FactorArgs &a, int blocks,
                              hipStream_t s) {
    return sh.R16 == 16 ? launch_fg<N, KQ, 1, P>(a, blocks, s)
                        : launch_fg<N, KQ, 2, P>(a, blocks, s);
}

template <int N, int KQ>
static hipError_t launch_fg_r(const Shape &sh, const FactorArgs &a, int blocks,
                              hipStream_t s) {
    if constexpr (N > kFullOrder) {  // FP32 only above the full orders
        return sh.prec == kF32 ? launch_fg_p<N, KQ, kF32>(sh, a, blocks, s)
                               : hipErrorInvalidValue;
    } else {
        switch (sh.prec) {
        case kF32: return launch_fg_p<N, KQ, kF32>(sh, a, blocks, s);
        case kBF16: return launch_fg_p<N, KQ, kBF16>(sh, a, blocks, s);
        case kFP8: return launch_fg_p<N, KQ, kFP8>(sh, a, blocks, s);
        }
        return hipErrorInvalidValue;
    }
}

template <int N>
static hipError_t launch_fg_j(const Shape &sh, const FactorArgs &a, int blocks,
                              hipStream_t s) {
    if constexpr (N > kFullOrder) {   // J4 padded to 8, 16 or 32
        switch (sh.J4) {
        case 8: return launch_fg_r<N, 2>(sh, a, blocks, s);
        case 16: return launch_fg_r<N, 4>(sh, a, blocks, s);
        case 32: return launch_fg_r<N, 8>(sh, a, blocks, s);
        }
        return hipErrorInvalidValue;
    } else {
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
}

hipError_t launch_factor_grad(const Shape &sh, const FactorArgs &a, int *nblocks,
                              hipStream_t s) {
    const int blocks = factor_grad_blocks(sh, a.m);
    *nblocks = blocks;
    switch (sh.N) {
    case 2: return launch_fg_j<2>(sh, a, blocks, s);
    case 3: return launch_fg_j<3>(sh, a, blocks, s);
    case 4: return launch_fg_j<4>(sh, a, blocks, s);
    case 5: return launch_fg_j<5>(sh, a, blocks, s);
    case 6: return launch_fg_j<6>(sh, a, blocks, s);
    case 7: return launch_fg_j<7>(sh, a, blocks, s);
    case 8: return launch_fg_j<8>(sh, a, blocks, s);
    case 9: return launch_fg_j<9>(sh, a, blocks, s);
    case 10: return launch_fg_j<10>(sh, a, blocks, s);
    }
    return hipErrorInvalidValue;
}

template <int N, int KQ, int RB>
static hipError_t launch_hw(const HogArgs &a, int blocks, hipStream_t s) {
    FT_LAUNCH((hogwild_kernel<N, KQ, RB>), dim3(blocks),
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
// Finish one row of mode n whose summed per-sample gradient g[0..J4) over
// cnt occurrences is complete; start is the sorted index of its first
// occurrence and av the row's current value (unused for autograd output).
// Writes the whole row (one lane).
template <int J4>
__device__ __forceinline__ void finish_row_av(const SegArgs &a, int n,
                                              uint32_t row, const float (&g)[J4],
                                              int cnt, int start,
                                              const float (&av)[J4]) {
    const int64_t off = (int64_t)row * J4;
    if (a.apply == 2) {
        // autograd: gradient of the data term only, times grad_out
        const float sc = a.scale ? *a.scale : 1.f;
        float o[J4];
#pragma unroll
        for (int j = 0; j < J4; ++j) o[j] = g[j] * sc;
        if (a.grad[n]) store_row<J4>(a.grad[n] + off, o);
        if (a.uniq_grad[n]) {
            const uint32_t ord = a.ordinal[n][start];
            store_row<J4>(a.uniq_grad[n] + (int64_t)ord * J4, o);
            if (a.uniq_rows[n]) a.uniq_rows[n][ord] = (int32_t)row;
        }
        return;
    }
    float o[J4];
#pragma unroll
    for (int j = 0; j < J4; ++j) o[j] = g[j] + (float)cnt * a.lam * av[j];
    if (a.apply) {
        const float inv = a.mean ? 1.f / (float)cnt : 1.f;
#pragma unroll
        for (int j = 0; j < J4; ++j) o[j] = av[j] - a.lr * (a.mean ? o[j] * inv : o[j]);
        store_row<J4>(a.A[n] + off, o);
        if (a.A16[n]) {
#pragma unroll
            for (int j = 0; j < J4; ++j) a.A16[n][off + j] = f2bf(o[j]);
        }
        if (a.A8[n]) quantize_row_fp8<J4>(o, a.A8[n] + off, a.As[n] + row);
    } else {
        store_row<J4>(a.grad[n] + off, o);
        a.count[n][row] = cnt;
    }
}

template <int J4>
__device__ __forceinline__ void load_av(const SegArgs &a, int n, uint32_t row,
                                        float (&av)[J4]) {
    if (a.apply != 2) {
        load_row_part<J4>(a.A[n] + (int64_t)row * J4, av);
    } else {
#pragma unroll
        for (int j = 0; j < J4; ++j) av[j] = 0.f;
    }
}

template <int J4>
__device__ __forceinline__ void finish_row(const SegArgs &a, int n,
                                           uint32_t row, const float (&g)[J4],
                                           int cnt, int start) {
    float av[J4];
    load_av<J4>(a, n, row, av);
    finish_row_av<J4>(a, n, row, g, cnt, start, av);
}

// One launch, three kinds of blocks (kSegWaves waves each), longest work
// first so that it starts at once:
//  * long crossing rows (blocks [0, large_blocks)): one block per row of
//    more than kSmallCross samples, or, for a row of more than
//    split_rows(J4), one block per part of part_rows(J4) samples; a row of
//    one part is finished
//    at once, the others leave part sums for seg_combine_kernel;
//  * chunks (the next chunk_blocks): one wave per chunk of 64 sorted
//    samples of one mode; lane l holds sample i0 + l with its whole gradient
//    row. A segmented inclusive scan across the lanes (seg_scan_dpp: DPP
//    shifts within 16-lane rows, then row broadcasts; a lane adds only
//    values of its own segment) leaves every row's sum in the lane of its
//    last sample, which finishes the row -- unless the row's samples cross a
//    chunk edge. The finishing lanes fetch their rows of A together with the
//    gradient rows;
//  * short crossing rows (the rest): one wave per row of at most kSmallCross
//    samples, kSegWaves per block, from the front of the list.
// A crossing row's threads sum its (contiguous) gradient rows with a fixed
// stride, seg_unroll rows loaded before they are added; a fixed butterfly
// adds a wave and wave 0 adds a block's wave sums in order.
// No block depends on another and every addition order is fixed by the
// data, so results are reproducible.
constexpr int kSegThreads = 64 * kSegWaves;

// rows loaded per thread before they are added
constexpr int seg_unroll(int J4) { return J4 <= 16 ? 4 : 2; }

// Sum of the gradient rows [se.x, se.y) of mode n (contiguous in the sorted
// order), thread t of a group of `stride` taking rows t, t + stride, ...,
// then a fixed butterfly over the 64 lanes of the wave.
template <int J4>
__device__ __forceinline__ void sum_rows_strided(const SegArgs &a, int n,
                                                 int4 se, int t, int stride,
                                                 float (&acc)[J4]) {
    constexpr int U = seg_unroll(J4);
#pragma unroll
    for (int q = 0; q < J4; ++q) acc[q] = 0.f;
    const float *G = a.G + (int64_t)n * a.m * J4;
    for (int i = se.x + t; i < se.y; i += stride * U) {
        float g[U][J4];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int iu = i + u * stride;
            if (iu < se.y) {
                load_row_part<J4>(G + (int64_t)iu * J4, g[u]);
            } else {
#pragma unroll
                for (int q = 0; q < J4; ++q) g[u][q] = 0.f;
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int q = 0; q < J4; ++q) acc[q] += g[u][q];
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1)
#pragma unroll
        for (int q = 0; q < J4; ++q) acc[q] += __shfl_xor(acc[q], d);
}

// The same sum with coalesced loads, for row widths that divide 64 lanes
// into whole rows (J4 = 4, 8, 16, 32): the count rows at `rows` are read as
// one flat run of float4s, thread t taking float4s t, t + stride, ..., all of
// them in column quad t mod (J4 / 4); a fixed butterfly adds the lanes of
// each column quad (log2(64 / (J4 / 4)) steps on four floats instead of six
// steps on J4), and every lane then takes the whole row by J4 shuffles.
template <int J4>
__device__ __forceinline__ void sum_rows_coalesced(const float *rows,
                                                   int count, int t,
                                                   int stride,
                                                   float (&acc)[J4]) {
    constexpr int Q = J4 / 4;
    constexpr int U = 16;
    const float4 *G4 = reinterpret_cast<const float4 *>(rows);
    const int total = count * Q;
    float4 s = make_float4(0.f, 0.f, 0.f, 0.f);
    for (int i = t; i < total; i += stride * U) {
        float4 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int k = i + u * stride;
            v[u] = k < total ? G4[k] : make_float4(0.f, 0.f, 0.f, 0.f);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            s.x += v[u].x;
            s.y += v[u].y;
            s.z += v[u].z;
            s.w += v[u].w;
        }
    }
#pragma unroll
    for (int d = 32; d >= Q; d >>= 1) {
        s.x += __shfl_xor(s.x, d);
        s.y += __shfl_xor(s.y, d);
        s.z += __shfl_xor(s.z, d);
        s.w += __shfl_xor(s.w, d);
    }
#pragma unroll
    for (int c = 0; c < Q; ++c) {
        acc[4 * c] = __shfl(s.x, c);
        acc[4 * c + 1] = __shfl(s.y, c);
        acc[4 * c + 2] = __shfl(s.z, c);
        acc[4 * c + 3] = __shfl(s.w, c);
    }
}

template <int J4>
__device__ __forceinline__ void sum_rows(const SegArgs &a, int n, int4 se,
                                         int t, int stride, float (&acc)[J4]) {
    if constexpr ((J4 & (J4 - 1)) == 0)
        sum_rows_coalesced<J4>(a.G + ((int64_t)n * a.m + se.x) * J4,
                               se.y - se.x, t, stride, acc);
    else
        sum_rows_strided<J4>(a, n, se, t, stride, acc);
}

// Entry k of one class (cls 0: short rows, 1: long rows, 2: long-row
// parts) over the modes in order: returns the mode (N if k is past the last
// entry) and leaves the index within that mode's class in k.
__device__ __forceinline__ int find_mode(const SegArgs &a, int cls, int &k) {
    if (a.host_counts) {
        const int *pre = cls == 0 ? a.xs : (cls == 1 ? a.xl : a.xp);
        int n = 0;
        while (n < a.N && k >= pre[n + 1]) ++n;
        if (n < a.N) k -= pre[n];
        return n;
    }
    int n = 0;
    while (n < a.N && k >= a.xcount[kXCounts * n + cls])
        k -= a.xcount[kXCounts * n++ + cls];
    return n;
}

// Fixed-order sum of the block's wave sums (in red[w][0..J4)): lane q < J4
// of wave 0 returns entry q, and g of every lane gets the whole row.
template <int J4>
__device__ __forceinline__ float sum_waves(float (*red)[J4 + 1], int lane,
                                           float (&g)[J4]) {
    float v = 0.f;
    if (lane < J4)
        for (int ww = 0; ww < kSegWaves; ++ww) v += red[ww][lane];
#pragma unroll
    for (int q = 0; q < J4; ++q) g[q] = __shfl(v, q);
    return v;
}

// Data-parallel-primitive moves between lanes (no LDS): row_shr:d gives
// lane l the value of lane l - d of its 16-lane row (0 where there is none);
// row_bcast:15 gives rows 1 and 3 the value of the last lane of the row
// before; row_bcast:31 gives rows 2 and 3 the value of lane 31.
template <int CTRL, int ROWS>
__device__ __forceinline__ float dpp_take(float x) {
    return __int_as_float(__builtin_amdgcn_update_dpp(
        0, __float_as_int(x), CTRL, ROWS, 0xf, false));
}

// Inclusive segmented scan of the J4 values of every lane in lane order,
// s being the first lane of the lane's segment: afterwards lane l holds the
// sum over lanes s .. l. Hillis-Steele within each 16-lane row (shifts 1, 2,
// 4, 8), then the rows are joined in order: row 1 takes row 0's last lane
// and row 3 row 2's (row_bcast:15), then rows 2-3 take lane 31, which by
// then covers rows 0-1 (row_bcast:31); a lane adds only inside its segment.
// Every move is a DPP operand of the add, where shuffles through LDS cost a
// crossbar round trip per value and step.
template <int J4>
__device__ __forceinline__ void seg_scan_dpp(float (&g)[J4], int lane,
                                             int s) {
    const int in_row = lane & 15, row0 = lane & ~15;
    const bool t1 = in_row >= 1 && lane - 1 >= s;
    const bool t2 = in_row >= 2 && lane - 2 >= s;
    const bool t4 = in_row >= 4 && lane - 4 >= s;
    const bool t8 = in_row >= 8 && lane - 8 >= s;
    const bool t15 = (lane & 16) && s < row0;
    const bool t31 = lane >= 32 && s < 32;
    // one value at a time through all six steps (the step masks are
    // shared), so no value waits in a register for the others
#pragma unroll
    for (int q = 0; q < J4; ++q) {
        float x = g[q], t;
        t = dpp_take<0x111, 0xf>(x);
        if (t1) x += t;
        t = dpp_take<0x112, 0xf>(x);
        if (t2) x += t;
        t = dpp_take<0x114, 0xf>(x);
        if (t4) x += t;
        t = dpp_take<0x118, 0xf>(x);
        if (t8) x += t;
        t = dpp_take<0x142, 0xa>(x);
        if (t15) x += t;
        t = dpp_take<0x143, 0xc>(x);
        if (t31) x += t;
        g[q] = x;
    }
}

template <int KQ>
__global__ __launch_bounds__(kSegThreads) void seg_reduce_kernel(
    SegArgs a, int chunk_blocks) {
    constexpr int J4 = 4 * KQ;
    __shared__ float red[kSegWaves][J4 + 1];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    int j = blockIdx.x;
    if (j < a.large_blocks) {
        const int n = find_mode(a, 2, j);     // long-row part j (block-uniform)
        if (n == a.N) return;
        const int4 pt = a.plist[n][j];        // (first, end, row, parts)
        float acc[J4];
        sum_rows<J4>(a, n, pt, t, kSegThreads, acc);
        if (lane == 0)
#pragma unroll
            for (int q = 0; q < J4; ++q) red[w][q] = acc[q];
        __syncthreads();
        if (w == 0) {
            float g[J4];
            const float v = sum_waves<J4>(red, lane, g);
            if (pt.w == 1) {                  // the whole row: finish it
                if (lane == 0)
                    finish_row<J4>(a, n, (uint32_t)pt.z, g, pt.y - pt.x, pt.x);
            } else if (lane < J4) {           // one part: leave its sum
                a.P[((int64_t)n * a.pcap + j) * J4 + lane] = v;
            }
        }
        return;
    }
    j -= a.large_blocks;
    if (j >= chunk_blocks) {
        int k = (j - chunk_blocks) * kSegWaves + w;   // short row k
        const int n = find_mode(a, 0, k);
        if (n == a.N) return;                         // wave-uniform
        const int4 se = a.xlist[n][k];
        float acc[J4];
        sum_rows<J4>(a, n, se, lane, 64, acc);
        if (lane == 0)
            finish_row<J4>(a, n, (uint32_t)se.z, acc, se.y - se.x, se.x);
        return;
    }
    const int gw = j * kSegWaves + w;
    if (gw >= a.N * a.nchunks) return;           // uniform per wave
    const int n = gw / a.nchunks, c = gw % a.nchunks;
    const int i0 = c * kSegChunk, i = i0 + lane;
    const int i1 = min(i0 + kSegChunk, a.m);
    const bool valid = i < i1;
    const uint32_t *rows = a.rows[n];
    // every load below is issued unconditionally from a clamped or dummy
    // address and its value selected afterwards: a load under a branch is
    // waited for inside the branch, which serialised the chunk's round trips
    const uint32_t row_v = rows[min(i, i1 - 1)];
    const uint32_t before_v = rows[max(i0 - 1, 0)];
    const uint32_t after_v = rows[min(i1, a.m - 1)];
    const uint32_t row = valid ? row_v : 0xffffffffu;
    const uint32_t before_chunk = i0 > 0 ? before_v : 0xffffffffu;
    const uint32_t after_chunk = i1 < a.m ? after_v : 0xffffffffu;
    const uint32_t below = __shfl_up(row, 1);
    const uint32_t above = __shfl_down(row, 1);
    const uint32_t last_row = __shfl(row, i1 - 1 - i0);
    const bool head = lane == 0 || row != below;
    // first lane of my segment: the highest head at or below my lane
    const uint64_t heads = __ballot(head) & ((2ull << lane) - 1ull);
    const int s = 63 - __clzll(heads);
    const bool last_in_chunk = i == i1 - 1;
    const bool tail = valid && (last_in_chunk || above != row);
    // the chunk's first segment may continue from the previous chunk and
    // its last one into the next: such rows are finished by their own
    // waves, so their gradient rows are not loaded here
    const bool in_crossing = (s == 0 && before_chunk == row) ||
                             (row == last_row && after_chunk == row);
    const bool finish = tail && !in_crossing;
    const bool take = valid && !in_crossing;
    // lanes that take nothing read the chunk's first gradient row (one
    // line for all of them) and the first row of A
    float g[J4];
    load_row_part<J4>(a.G + ((int64_t)n * a.m + (take ? i : i0)) * J4, g);
#pragma unroll
    for (int q = 0; q < J4; ++q) g[q] = take ? g[q] : 0.f;
    float av[J4];
    if (a.apply != 2) {
        load_row_part<J4>(a.A[n] + (int64_t)(finish ? row : 0u) * J4, av);
    } else {
#pragma unroll
        for (int j = 0; j < J4; ++j) av[j] = 0.f;
    }
    seg_scan_dpp<J4>(g, lane, s);
    if (finish) finish_row_av<J4>(a, n, row, g, lane - s + 1, i0 + s, av);
}

template <int KQ>
static hipError_t launch_seg_kq(const SegArgs &a, hipStream_t s) {
    const int chunk_blocks = (a.N * a.nchunks + kSegWaves - 1) / kSegWaves;
    const int blocks = a.large_blocks + chunk_blocks + a.small_blocks;
    FT_LAUNCH(seg_reduce_kernel<KQ>, dim3(blocks), dim3(kSegThreads), 0, s, a,
              chunk_blocks);
    return hipGetLastError();
}

// Long rows of more than one part: one wave per long row (rows of one part
// were finished by the reduction kernel and are skipped); lane l adds the
// row's part sums l, l + 64, ... and a fixed butterfly adds the lanes.
template <int KQ>
__global__ __launch_bounds__(kSegThreads) void seg_combine_kernel(SegArgs a) {
    constexpr int J4 = 4 * KQ;
    const int lane = threadIdx.x & 63;
    int k = blockIdx.x * kSegWaves + (threadIdx.x >> 6);
    const int n = find_mode(a, 1, k);
    if (n == a.N) return;                            // wave-uniform
    const int4 e = a.xlist[n][a.xcap - 1 - k];       // (first, end, row, p0)
    const int cnt = e.y - e.x;
    if (cnt <= split_rows(J4)) return;               // finished in one part
    const int parts = (cnt + part_rows(J4) - 1) / part_rows(J4);
    float acc[J4];
    const float *P = a.P + ((int64_t)n * a.pcap + e.w) * J4;
    if constexpr ((J4 & (J4 - 1)) == 0) {
        sum_rows_coalesced<J4>(P, parts, lane, 64, acc);
    } else {
#pragma unroll
        for (int q = 0; q < J4; ++q) acc[q] = 0.f;
        for (int i = lane; i < parts; i += 64) {
            float g[J4];
            load_row_part<J4>(P + (int64_t)i * J4, g);
#pragma unroll
            for (int q = 0; q < J4; ++q) acc[q] += g[q];
        }
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1)
#pragma unroll
            for (int q = 0; q < J4; ++q) acc[q] += __shfl_xor(acc[q], d);
    }
    if (lane == 0) finish_row<J4>(a, n, (uint32_t)e.z, acc, e.y - e.x, e.x);
}

template <int KQ>
static hipError_t launch_comb_kq(const SegArgs &a, hipStream_t s) {
    FT_LAUNCH(seg_combine_kernel<KQ>, dim3(a.combine_blocks), dim3(kSegThreads),
              0, s, a);
    return hipGetLastError();
}

hipError_t launch_seg_combine(const SegArgs &a, hipStream_t s) {
    if (a.combine_blocks <= 0) return hipSuccess;
    switch (a.J4) {
    case 4: return launch_comb_kq<1>(a, s);
    case 8: return launch_comb_kq<2>(a, s);
    case 12: return launch_comb_kq<3>(a, s);
    case 16: return launch_comb_kq<4>(a, s);
    case 20: return launch_comb_kq<5>(a, s);
    case 24: return launch_comb_kq<6>(a, s);
    case 28: return launch_comb_kq<7>(a, s);
    case 32: return launch_comb_kq<8>(a, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_seg_reduce(const SegArgs &a, hipStream_t s) {
    switch (a.J4) {
    case 4: return launch_seg_kq<1>(a, s);
    case 8: return launch_seg_kq<2>(a, s);
    case 12: return launch_seg_kq<3>(a, s);
    case 16: return launch_seg_kq<4>(a, s);
    case 20: return launch_seg_kq<5>(a, s);
    case 24: return launch_seg_kq<6>(a, s);
    case 28: return launch_seg_kq<7>(a, s);
    case 32: return launch_seg_kq<8>(a, s);
    }
    return hipErrorInvalidValue;
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
