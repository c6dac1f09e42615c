// k_core.hip -- core phase of FastTuckerPlus (Algorithm 5; Eq. (13) in the
// matrix form of Eq. (15)).
//
// core_grad_kernel: one wave per 16-sample tile, A and B fixed. C^(n) =
// A_Psi^(n) B^(n) is formed on the matrix cores in the "sample-row" layout
// (lane column = r), D^(n) by prefix/suffix products, xhat by a 16-lane
// reduction, and the core gradient
//     Grad^(n) += E^(n)T D^(n),   E^(n) = r (*) A_Psi^(n)
// by a second matrix-core product whose contraction runs over the 16 samples
// of the tile. Every wave keeps its Grad^(n) in accumulator registers across
// all of its tiles (the register accumulation of Algorithm 5); a block sums its
// four waves in a fixed order and writes one partial per block.
//
// core_update_kernel: sums the block partials in a fixed order (no atomics:
// 32 strided slices, then the slices in order) and applies B^(n) <- B^(n) - lr_B (Grad^(n) / count + lambda_B B^(n)).
#include "ft_internal.h"
#include "mfma_tile.h"

namespace ft {

constexpr int kCoreMaxBlocks = 1024;

int core_grad_blocks(int64_t count) {
    int64_t ntiles = (count + 15) / 16;
    int64_t blocks = (ntiles + 3) / 4;
    if (blocks > kCoreMaxBlocks) blocks = kCoreMaxBlocks;
    return blocks < 1 ? 1 : (int)blocks;
}

// Per-tile inputs, loaded one tile ahead of the arithmetic.
template <int N, int KQ, int P>
struct CoreTileIn {
    RowFrag<KQ, P> arow[N];   // A[s = c][KQ q .. KQ q + KQ - 1]
    float x[4];                // values of samples 4q + v
};

template <int N, int KQ, int P>
__device__ __forceinline__ void load_core_tile(const CoreArgs &a, int64_t tile,
                                               int q, int c,
                                               CoreTileIn<N, KQ, P> &in) {
    constexpr int J4 = 4 * KQ;
    const int64_t base = tile * 16;
    const int64_t last = a.count - 1;
    const int64_t ps = base + c <= last ? base + c : last;
#pragma unroll
    for (int n = 0; n < N; ++n) {
        const int row = a.idx[n][ps];
        in.arow[n].load(RowSrc{a.A[n], a.A16[n], a.A8[n], a.As[n]}, row, J4,
                        q);
    }
    const int64_t s0 = base + 4 * q;
    if (s0 + 3 <= last) {
        const float4 xv = *reinterpret_cast<const float4 *>(a.val + s0);
        in.x[0] = xv.x;
        in.x[1] = xv.y;
        in.x[2] = xv.z;
        in.x[3] = xv.w;
    } else {
#pragma unroll
        for (int v = 0; v < 4; ++v) in.x[v] = s0 + v <= last ? a.val[s0 + v] : 0.f;
    }
}

// Waves per SIMD the register allocator is held to: four where the tile fits
// in 128 registers without spilling (checked per shape at build time), else
// the compiler's choice.
constexpr int core_waves(int N, int KQ, int RB, int P) {
    if (N > kFullOrder)   // high orders: one wave per SIMD keeps the tile
        return 1;         // in registers (orders 9-10 at J = R = 32 spill)
    if (N * RB * KQ > 32)   // B-operands in LDS: two waves fit, except
        return (P == kF32 && N == 5 && KQ * RB >= 14) ? 1 : 2;  // (spills)
    if (P == kFP8)   // the scale shuffles need a few more registers
        return (KQ * RB <= 4 && RB == 1 && (N <= 3 || (N == 4 && KQ <= 2)))
                   ? 4
                   : 1;
    return (KQ * RB <= 4 &&
            (N <= 3 || (RB == 1 && (N == 4 ? KQ <= 3 : KQ <= 1))))
               ? 4
               : 1;
}

template <int N, int KQ, int RB, int P>
__global__ __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu(core_waves(N, KQ, RB, P)))) void
core_grad_kernel(CoreArgs a, int64_t ntiles) {
    constexpr int J4 = 4 * KQ;
    constexpr int R16 = 16 * RB;
    constexpr int JB = (KQ + 3) / 4;
    constexpr int TP = J4 + 1;       // padded row of the per-wave transpose
    // [4 waves][N][J4][R16] partials at the end; during the sweep each wave
    // uses [N][16][TP] of it to transpose its tile's factor rows
    extern __shared__ float lds[];
    const int lane = threadIdx.x & 63, q = lane >> 4, c = lane & 15;
    const int wave = threadIdx.x >> 6;
    constexpr int WAVE_LDS = (N * J4 * R16 > N * 16 * TP) ? N * J4 * R16
                                                          : N * 16 * TP;
    float *tr = lds + wave * WAVE_LDS;

    // B-operands B[k = KQ*q + t][r = 16 rb + c]: the same in every wave.
    // Large sets (order 4-5 at J = R = 32) live in LDS, one copy per block
    // laid out [word][lane], written by wave 0 and read at each use (the
    // lane index goes through an empty asm statement once per tile so the
    // reads are not hoisted back into registers but are scheduled freely
    // within the tile); small sets stay in registers.
    constexpr int CFW = sizeof(ColFrag<KQ, P>) / 4;
    constexpr bool kLdsOps = N * RB * CFW > 32;
    __shared__ uint32_t sOps[kLdsOps ? N * RB * CFW * 64 : 1];
    ColFrag<KQ, P> bop[N][RB];
    if (!kLdsOps || wave == 0) {
#pragma unroll
        for (int n = 0; n < N; ++n)
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) {
                bop[n][rb].load(a.B[n], R16, q, 16 * rb + c);
                if constexpr (kLdsOps) {
                    uint32_t w[CFW];
                    __builtin_memcpy(w, &bop[n][rb], sizeof(w));
#pragma unroll
                    for (int i = 0; i < CFW; ++i)
                        sOps[((n * RB + rb) * CFW + i) * 64 + lane] = w[i];
                }
            }
    }
    if constexpr (kLdsOps) __syncthreads();
    int lane_o = lane;
    auto operand = [&](int n, int rb) -> ColFrag<KQ, P> {
        if constexpr (kLdsOps) {
            const int l = lane_o;
            uint32_t w[CFW];
#pragma unroll
            for (int i = 0; i < CFW; ++i)
                w[i] = sOps[((n * RB + rb) * CFW + i) * 64 + l];
            ColFrag<KQ, P> f;
            __builtin_memcpy(&f, w, sizeof(w));
            return f;
        } else {
            return bop[n][rb];
        }
    };

    floatx4 grad[N][JB][RB];
#pragma unroll
    for (int n = 0; n < N; ++n)
#pragma unroll
        for (int jb = 0; jb < JB; ++jb)
#pragma unroll
            for (int rb = 0; rb < RB; ++rb)
                grad[n][jb][rb] = floatx4{0.f, 0.f, 0.f, 0.f};

    double loss = 0.0;
    const int64_t nwaves = (int64_t)gridDim.x * 4;
    const int64_t last = a.count - 1;
    int64_t tile = (int64_t)blockIdx.x * 4 + wave;
    CoreTileIn<N, KQ, P> nxt;
    if (tile < ntiles) load_core_tile<N, KQ, P>(a, tile, q, c, nxt);
    for (; tile < ntiles; tile += nwaves) {
        lane_o = lane;
        asm volatile("" : "+v"(lane_o));
        const CoreTileIn<N, KQ, P> cur = nxt;
        if (tile + nwaves < ntiles)
            load_core_tile<N, KQ, P>(a, tile + nwaves, q, c, nxt);
        const int64_t base = tile * 16;

        floatx4 C[N][RB];   // C[s = 4q + v][r = 16 rb + c]
#pragma unroll
        for (int n = 0; n < N; ++n)
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) {
                const ColFrag<KQ, P> bo = operand(n, rb);
                C[n][rb] = contract(cur.arow[n], bo,
                                    floatx4{0.f, 0.f, 0.f, 0.f});
                if constexpr (P == kFP8)
                    C[n][rb] = fp8_scale_c(C[n][rb], bo.s,
                                           cur.arow[n].s, q);
            }
        floatx4 D[N][RB];
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
        float r[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            float xh = 0.f;
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) xh += C[0][rb][v] * D[0][rb][v];
            xh = sum_row16(xh);
            const bool ok = base + 4 * q + v <= last;
            r[v] = ok ? xh - cur.x[v] : 0.f;
            if (c == 0 && ok) loss += 0.5 * (double)r[v] * (double)r[v];
        }
        // transpose the tile's rows through LDS: lane (c, q) needs
        // A[s = 4q + v][j = 16 jb + c] for the contraction over samples
        wave_lds_sync();
#pragma unroll
        for (int n = 0; n < N; ++n)
#pragma unroll
            for (int t = 0; t < KQ; ++t)
                tr[(n * 16 + c) * TP + KQ * q + t] = cur.arow[n].value(t);
        wave_lds_sync();
#pragma unroll
        for (int n = 0; n < N; ++n) {
#pragma unroll
            for (int jb = 0; jb < JB; ++jb) {
                const int j = 16 * jb + c;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const float av =
                        j < J4 ? tr[(n * 16 + 4 * q + v) * TP + j] : 0.f;
                    const float e = r[v] * av;
#pragma unroll
                    for (int rb = 0; rb < RB; ++rb)
                        grad[n][jb][rb] =
                            mfma_16x16x4(e, D[n][rb][v], grad[n][jb][rb]);
                }
            }
        }
    }
    wave_lds_sync();
    __syncthreads();

    // grad[n][jb][rb][v] holds Grad^(n)[j = 16 jb + 4q + v][r = 16 rb + c]
    float *mine = lds + wave * (N * J4 * R16);
#pragma unroll
    for (int n = 0; n < N; ++n)
#pragma unroll
        for (int jb = 0; jb < JB; ++jb)
#pragma unroll
            for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int j = 16 * jb + 4 * q + v;
                    if (j < J4)
                        mine[(n * J4 + j) * R16 + 16 * rb + c] =
                            grad[n][jb][rb][v];
                }
    __syncthreads();
    constexpr int E = N * J4 * R16;
    float *out = a.part + (int64_t)blockIdx.x * E;
    for (int e = threadIdx.x; e < E; e += 256)
        out[e] = ((lds[e] + lds[E + e]) + lds[2 * E + e]) + lds[3 * E + e];
    const double tot = block_sum_256(loss);
    if (threadIdx.x == 0) a.loss_part[blockIdx.x] = tot;
}

// Persistent grid: as many blocks as fit on the device at once (never more
// than one per four tiles); the tile-to-wave assignment, and with it the
// summation order, depends only on this number.
static int resident_blocks(const void *kernel, size_t lds) {
    static int ncu = 0;
    if (ncu == 0) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount,
                                  dev) != hipSuccess || ncu < 1)
            ncu = 256;
    }
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, 256,
                                                     lds) != hipSuccess ||
        per_cu < 1)
        per_cu = 1;
    return ncu * per_cu;
}

template <int N, int KQ, int RB, int P>
static hipError_t launch_cg(const CoreArgs &a, int blocks, hipStream_t s) {
    const int64_t ntiles = (a.count + 15) / 16;
    const int part = N * (4 * KQ) * (16 * RB);
    const int trans = N * 16 * (4 * KQ + 1);
    const size_t lds = sizeof(float) * 4 * (part > trans ? part : trans);
    const int fit = resident_blocks(
        reinterpret_cast<const void *>(&core_grad_kernel<N, KQ, RB, P>), lds);
    if (blocks > fit) blocks = fit;
    *a.blocks_used = blocks;
    FT_LAUNCH((core_grad_kernel<N, KQ, RB, P>), dim3(blocks),
                       dim3(256), lds, s, a, ntiles);
    return hipGetLastError();
}

template <int N, int KQ, int P>
static hipError_t launch_cg_p(const Shape &sh, const CoreArgs &a, int blocks,
                              hipStream_t s) {
    return sh.R16 == 16 ? launch_cg<N, KQ, 1, P>(a, blocks, s)
                        : launch_cg<N, KQ, 2, P>(a, blocks, s);
}

template <int N, int KQ>
static hipError_t launch_cg_r(const Shape &sh, const CoreArgs &a, int blocks,
                              hipStream_t s) {
    if constexpr (N > kFullOrder) {  // FP32 only above the full orders
        return sh.prec == kF32 ? launch_cg_p<N, KQ, kF32>(sh, a, blocks, s)
                               : hipErrorInvalidValue;
    } else {
        switch (sh.prec) {
        case kF32: return launch_cg_p<N, KQ, kF32>(sh, a, blocks, s);
        case kBF16: return launch_cg_p<N, KQ, kBF16>(sh, a, blocks, s);
        case kFP8: return launch_cg_p<N, KQ, kFP8>(sh, a, blocks, s);
        }
        return hipErrorInvalidValue;
    }
}

template <int N>
static hipError_t launch_cg_j(const Shape &sh, const CoreArgs &a, int blocks,
                              hipStream_t s) {
    if constexpr (N > kFullOrder) {   // J4 padded to 8, 16 or 32
        switch (sh.J4) {
        case 8: return launch_cg_r<N, 2>(sh, a, blocks, s);
        case 16: return launch_cg_r<N, 4>(sh, a, blocks, s);
        case 32: return launch_cg_r<N, 8>(sh, a, blocks, s);
        }
        return hipErrorInvalidValue;
    } else {
        switch (sh.J4) {
        case 4: return launch_cg_r<N, 1>(sh, a, blocks, s);
        case 8: return launch_cg_r<N, 2>(sh, a, blocks, s);
        case 12: return launch_cg_r<N, 3>(sh, a, blocks, s);
        case 16: return launch_cg_r<N, 4>(sh, a, blocks, s);
        case 20: return launch_cg_r<N, 5>(sh, a, blocks, s);
        case 24: return launch_cg_r<N, 6>(sh, a, blocks, s);
        case 28: return launch_cg_r<N, 7>(sh, a, blocks, s);
        case 32: return launch_cg_r<N, 8>(sh, a, blocks, s);
        }
        return hipErrorInvalidValue;
    }
}

hipError_t launch_core_grad(const Shape &sh, const CoreArgs &a, int nblocks,
                            hipStream_t s) {
    if (nblocks > kCoreMaxBlocks) nblocks = kCoreMaxBlocks;
    switch (sh.N) {
    case 2: return launch_cg_j<2>(sh, a, nblocks, s);
    case 3: return launch_cg_j<3>(sh, a, nblocks, s);
    case 4: return launch_cg_j<4>(sh, a, nblocks, s);
    case 5: return launch_cg_j<5>(sh, a, nblocks, s);
    case 6: return launch_cg_j<6>(sh, a, nblocks, s);
    case 7: return launch_cg_j<7>(sh, a, nblocks, s);
    case 8: return launch_cg_j<8>(sh, a, nblocks, s);
    case 9: return launch_cg_j<9>(sh, a, nblocks, s);
    case 10: return launch_cg_j<10>(sh, a, nblocks, s);
    }
    return hipErrorInvalidValue;
}

// ------------------------------------------------- stored-C core kernel
// The storage variant of the core phase (the paper's storage-against-
// calculation comparison): with A and B fixed for the whole pass, every row's
// C^(n)_i = a^(n)_i B^(n) is formed once (precompute_c_kernel) and the core
// kernel gathers the R-wide rows of C instead of contracting the J-wide rows
// of A with B; it still gathers the rows of A for E^(n) = r (*) A_Psi^(n).
// FP32 only. The tile, transpose and accumulation are those of
// core_grad_kernel, so the two give the same partials up to the rounding of
// C (the stored C is the same FP32 product, summed in order over j).

// C^(n) (rows x R16, row-major) <- A^(n) (rows x J4) B^(n) (J4 x R16): one
// thread per four consecutive entries of a row, B staged in LDS.
template <int J4, int R16>
__global__ __launch_bounds__(256) void precompute_c_kernel(const float *A,
                                                           const float *B,
                                                           int64_t rows,
                                                           float *Cst) {
    __shared__ float sB[J4 * R16];
    for (int e = threadIdx.x; e < J4 * R16; e += 256) sB[e] = B[e];
    __syncthreads();
    constexpr int QR = R16 / 4;
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t row = t / QR;
    const int rq = (int)(t % QR);
    if (row >= rows) return;
    const float4 *a4 = reinterpret_cast<const float4 *>(A + row * J4);
    float acc[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int jq = 0; jq < J4 / 4; ++jq) {
        const float4 av = a4[jq];
        const float aj[4] = {av.x, av.y, av.z, av.w};
#pragma unroll
        for (int e = 0; e < 4; ++e)
#pragma unroll
            for (int k = 0; k < 4; ++k)
                acc[k] = fmaf(aj[e], sB[(4 * jq + e) * R16 + 4 * rq + k],
                              acc[k]);
    }
    reinterpret_cast<float4 *>(Cst + row * R16)[rq] =
        make_float4(acc[0], acc[1], acc[2], acc[3]);
}

template <int N, int KQ, int RB>
struct StoredTileIn {
    RowFrag<KQ, kF32> arow[N];   // A[s = c][KQ q .. KQ q + KQ - 1]
    floatx4 C[N][RB];            // C[s = 4q + v][r = 16 rb + c]
    float x[4];                  // values of samples 4q + v
};

template <int N, int KQ, int RB>
__device__ __forceinline__ void load_stored_tile(const CoreArgs &a,
                                                 int64_t tile, int q, int c,
                                                 StoredTileIn<N, KQ, RB> &in) {
    constexpr int J4 = 4 * KQ;
    constexpr int R16 = 16 * RB;
    const int64_t base = tile * 16;
    const int64_t last = a.count - 1;
    const int64_t ps = base + c <= last ? base + c : last;
#pragma unroll
    for (int n = 0; n < N; ++n) {
        const int row = a.idx[n][ps];
        in.arow[n].load(RowSrc{a.A[n], nullptr, nullptr, nullptr}, row, J4, q);
        // rows of samples 4q + v come from the lanes that loaded them
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int rv = __shfl(row, 4 * q + v, 64);
            const float *cr = a.Cst[n] + (int64_t)rv * R16 + c;
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) in.C[n][rb][v] = cr[16 * rb];
        }
    }
    const int64_t s0 = base + 4 * q;
#pragma unroll
    for (int v = 0; v < 4; ++v) in.x[v] = s0 + v <= last ? a.val[s0 + v] : 0.f;
}

template <int N, int KQ, int RB>
__global__ __launch_bounds__(256) void core_grad_stored_kernel(
    CoreArgs a, int64_t ntiles) {
    constexpr int J4 = 4 * KQ;
    constexpr int R16 = 16 * RB;
    constexpr int JB = (KQ + 3) / 4;
    constexpr int TP = J4 + 1;
    extern __shared__ float lds[];
    const int lane = threadIdx.x & 63, q = lane >> 4, c = lane & 15;
    const int wave = threadIdx.x >> 6;
    constexpr int WAVE_LDS = (N * J4 * R16 > N * 16 * TP) ? N * J4 * R16
                                                          : N * 16 * TP;
    float *tr = lds + wave * WAVE_LDS;
    floatx4 grad[N][JB][RB];
#pragma unroll
    for (int n = 0; n < N; ++n)
#pragma unroll
        for (int jb = 0; jb < JB; ++jb)
#pragma unroll
            for (int rb = 0; rb < RB; ++rb)
                grad[n][jb][rb] = floatx4{0.f, 0.f, 0.f, 0.f};
    double loss = 0.0;
    const int64_t nwaves = (int64_t)gridDim.x * 4;
    const int64_t last = a.count - 1;
    int64_t tile = (int64_t)blockIdx.x * 4 + wave;
    StoredTileIn<N, KQ, RB> nxt;
    if (tile < ntiles) load_stored_tile<N, KQ, RB>(a, tile, q, c, nxt);
    for (; tile < ntiles; tile += nwaves) {
        const StoredTileIn<N, KQ, RB> cur = nxt;
        if (tile + nwaves < ntiles)
            load_stored_tile<N, KQ, RB>(a, tile + nwaves, q, c, nxt);
        const int64_t base = tile * 16;
        floatx4 D[N][RB];
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
            floatx4 pre = {1.f, 1.f, 1.f, 1.f};
#pragma unroll
            for (int n = 0; n < N; ++n) {
                D[n][rb] = pre;
                pre *= cur.C[n][rb];
            }
            floatx4 suf = {1.f, 1.f, 1.f, 1.f};
#pragma unroll
            for (int n = N - 1; n >= 0; --n) {
                D[n][rb] *= suf;
                suf *= cur.C[n][rb];
            }
        }
        float r[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            float xh = 0.f;
#pragma unroll
            for (int rb = 0; rb < RB; ++rb)
                xh += cur.C[0][rb][v] * D[0][rb][v];
            xh = sum_row16(xh);
            const bool ok = base + 4 * q + v <= last;
            r[v] = ok ? xh - cur.x[v] : 0.f;
            if (c == 0 && ok) loss += 0.5 * (double)r[v] * (double)r[v];
        }
        wave_lds_sync();
#pragma unroll
        for (int n = 0; n < N; ++n)
#pragma unroll
            for (int t = 0; t < KQ; ++t)
                tr[(n * 16 + c) * TP + KQ * q + t] = cur.arow[n].value(t);
        wave_lds_sync();
#pragma unroll
        for (int n = 0; n < N; ++n) {
#pragma unroll
            for (int jb = 0; jb < JB; ++jb) {
                const int j = 16 * jb + c;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const float av =
                        j < J4 ? tr[(n * 16 + 4 * q + v) * TP + j] : 0.f;
                    const float e = r[v] * av;
#pragma unroll
                    for (int rb = 0; rb < RB; ++rb)
                        grad[n][jb][rb] =
                            mfma_16x16x4(e, D[n][rb][v], grad[n][jb][rb]);
                }
            }
        }
    }
    wave_lds_sync();
    __syncthreads();
    float *mine = lds + wave * (N * J4 * R16);
#pragma unroll
    for (int n = 0; n < N; ++n)
#pragma unroll
        for (int jb = 0; jb < JB; ++jb)
#pragma unroll
            for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int j = 16 * jb + 4 * q + v;
                    if (j < J4)
                        mine[(n * J4 + j) * R16 + 16 * rb + c] =
                            grad[n][jb][rb][v];
                }
    __syncthreads();
    constexpr int E = N * J4 * R16;
    float *out = a.part + (int64_t)blockIdx.x * E;
    for (int e = threadIdx.x; e < E; e += 256)
        out[e] = ((lds[e] + lds[E + e]) + lds[2 * E + e]) + lds[3 * E + e];
    const double tot = block_sum_256(loss);
    if (threadIdx.x == 0) a.loss_part[blockIdx.x] = tot;
}

template <int J4, int R16>
static hipError_t launch_pc(const float *A, const float *B, int64_t rows,
                            float *Cst, hipStream_t s) {
    const int64_t threads = rows * (R16 / 4);
    const int64_t blocks = (threads + 255) / 256;
    FT_LAUNCH((precompute_c_kernel<J4, R16>), dim3((unsigned)blocks),
              dim3(256), 0, s, A, B, rows, Cst);
    return hipGetLastError();
}

template <int J4>
static hipError_t launch_pc_r(int R16, const float *A, const float *B,
                              int64_t rows, float *Cst, hipStream_t s) {
    return R16 == 16 ? launch_pc<J4, 16>(A, B, rows, Cst, s)
                     : launch_pc<J4, 32>(A, B, rows, Cst, s);
}

hipError_t launch_precompute_c(const Shape &sh, const float *A, const float *B,
                               int64_t rows, float *Cst, hipStream_t s) {
    if (rows < 1) return hipSuccess;
    switch (sh.J4) {
    case 4: return launch_pc_r<4>(sh.R16, A, B, rows, Cst, s);
    case 8: return launch_pc_r<8>(sh.R16, A, B, rows, Cst, s);
    case 12: return launch_pc_r<12>(sh.R16, A, B, rows, Cst, s);
    case 16: return launch_pc_r<16>(sh.R16, A, B, rows, Cst, s);
    case 20: return launch_pc_r<20>(sh.R16, A, B, rows, Cst, s);
    case 24: return launch_pc_r<24>(sh.R16, A, B, rows, Cst, s);
    case 28: return launch_pc_r<28>(sh.R16, A, B, rows, Cst, s);
    case 32: return launch_pc_r<32>(sh.R16, A, B, rows, Cst, s);
    }
    return hipErrorInvalidValue;
}

template <int N, int KQ, int RB>
static hipError_t launch_cgs(const CoreArgs &a, int blocks, hipStream_t s) {
    const int64_t ntiles = (a.count + 15) / 16;
    const int part = N * (4 * KQ) * (16 * RB);
    const int trans = N * 16 * (4 * KQ + 1);
    const size_t lds = sizeof(float) * 4 * (part > trans ? part : trans);
    const int fit = resident_blocks(
        reinterpret_cast<const void *>(&core_grad_stored_kernel<N, KQ, RB>),
        lds);
    if (blocks > fit) blocks = fit;
    *a.blocks_used = blocks;
    FT_LAUNCH((core_grad_stored_kernel<N, KQ, RB>), dim3(blocks), dim3(256),
              lds, s, a, ntiles);
    return hipGetLastError();
}

template <int N, int KQ>
static hipError_t launch_cgs_r(const Shape &sh, const CoreArgs &a, int blocks,
                               hipStream_t s) {
    return sh.R16 == 16 ? launch_cgs<N, KQ, 1>(a, blocks, s)
                        : launch_cgs<N, KQ, 2>(a, blocks, s);
}

template <int N>
static hipError_t launch_cgs_j(const Shape &sh, const CoreArgs &a, int blocks,
                               hipStream_t s) {
    switch (sh.J4) {
    case 4: return launch_cgs_r<N, 1>(sh, a, blocks, s);
    case 8: return launch_cgs_r<N, 2>(sh, a, blocks, s);
    case 12: return launch_cgs_r<N, 3>(sh, a, blocks, s);
    case 16: return launch_cgs_r<N, 4>(sh, a, blocks, s);
    case 20: return launch_cgs_r<N, 5>(sh, a, blocks, s);
    case 24: return launch_cgs_r<N, 6>(sh, a, blocks, s);
    case 28: return launch_cgs_r<N, 7>(sh, a, blocks, s);
    case 32: return launch_cgs_r<N, 8>(sh, a, blocks, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_core_grad_stored(const Shape &sh, const CoreArgs &a,
                                   int nblocks, hipStream_t s) {
    if (sh.prec != kF32) return hipErrorInvalidValue;
    if (nblocks > kCoreMaxBlocks) nblocks = kCoreMaxBlocks;
    switch (sh.N) {
    case 2: return launch_cgs_j<2>(sh, a, nblocks, s);
    case 3: return launch_cgs_j<3>(sh, a, nblocks, s);
    case 4: return launch_cgs_j<4>(sh, a, nblocks, s);
    case 5: return launch_cgs_j<5>(sh, a, nblocks, s);
    }
    return hipErrorInvalidValue;
}

// ------------------------------------------------- vector-ALU core kernel
// The core kernel's arithmetic with vector FP32 FMAs instead of the matrix
// cores (for the ablation). A persistent block sweeps chunks of S samples:
//   1. TPS = 256 / S threads per sample split the rank range (r = sub + TPS k)
//      and form their part of c^(n)_r = sum_j a^(n)_j B^(n)[j][r] (B staged in
//      LDS); xhat is summed across the sample's threads by shuffles; each
//      thread writes its d^(n)_r and a share of e^(n)_j = (xhat - x) a^(n)_j
//      to LDS.
//   2. Grad^(n) += e^(n)T d^(n) as register-blocked 4 x 4 outer products:
//      thread u owns tile u mod T of the T = N (J4/4)(R16/4) tiles and the
//      samples s = g, g + G, ... of the chunk, g = u / T (G = 256 / T groups
//      when the tiles are fewer than the threads).
// At the end each block sums its groups in increasing g and writes one
// partial [N][J4][R16] in the layout of the matrix-core kernel, so the same
// fixed-order update kernel finishes the step.
template <int N, int J4, int R16>
struct CoreValu {
    static constexpr int S =
        N * (J4 + R16) * 64 * 4 <= 32768 ? 64 : 32;   // samples per chunk
    static constexpr int TPS = 256 / S;                 // threads per sample
    static constexpr int RK = R16 / TPS;                // ranks per thread
    static constexpr int T = N * (J4 / 4) * (R16 / 4);  // 4 x 4 tiles
    static constexpr int G = T < 256 ? 256 / T : 1;     // sample groups
    static constexpr int PAIRS = T * G;
    static constexpr int PP = (PAIRS + 255) / 256;      // pairs per thread
    static constexpr int WORK = S * N * (J4 + R16) > PAIRS * 16
                                    ? S * N * (J4 + R16)
                                    : PAIRS * 16;
};

template <int N, int J4, int R16>
__global__ __launch_bounds__(256) void core_grad_valu_kernel(CoreArgs a,
                                                             int64_t nchunks) {
    using V = CoreValu<N, J4, R16>;
    constexpr int S = V::S, TPS = V::TPS, RK = V::RK, T = V::T, G = V::G;
    constexpr int TJ = J4 / 4, TR = R16 / 4;
    __shared__ float4 sB4[N * J4 * R16 / 4];
    __shared__ float4 work4[V::WORK / 4];
    float *sB = reinterpret_cast<float *>(sB4);
    float *sE = reinterpret_cast<float *>(work4);   // [S][N][J4]
    float *sD = sE + S * N * J4;                    // [S][N][R16]
    for (int e = threadIdx.x; e < N * J4 * R16; e += 256)
        sB[e] = a.B[e / (J4 * R16)][e % (J4 * R16)];
    __syncthreads();

    const int s = threadIdx.x / TPS, sub = threadIdx.x % TPS;
    float acc[V::PP][4][4];
#pragma unroll
    for (int pp = 0; pp < V::PP; ++pp)
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int k = 0; k < 4; ++k) acc[pp][i][k] = 0.f;
    double loss = 0.0;

    for (int64_t chunk = blockIdx.x; chunk < nchunks; chunk += gridDim.x) {
        const int64_t p = chunk * S + s;
        const bool valid = p < a.count;
        const int64_t ps = valid ? p : a.count - 1;
        int rows[N];
        float C[N][RK];
#pragma unroll
        for (int n = 0; n < N; ++n) {
            rows[n] = a.idx[n][ps];
            const float4 *ar =
                reinterpret_cast<const float4 *>(a.A[n] + (int64_t)rows[n] * J4);
            const float *bn = sB + n * J4 * R16 + sub;
#pragma unroll
            for (int k = 0; k < RK; ++k) C[n][k] = 0.f;
#pragma unroll 1
            for (int jq = 0; jq < J4 / 4; ++jq) {
                const float4 v = ar[jq];
                const float av[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
                for (int e = 0; e < 4; ++e)
#pragma unroll
                    for (int k = 0; k < RK; ++k)
                        C[n][k] = fmaf(av[e], bn[(4 * jq + e) * R16 + TPS * k],
                                       C[n][k]);
            }
        }
        float xh = 0.f;
#pragma unroll
        for (int k = 0; k < RK; ++k) {
            float prod = C[0][k];
#pragma unroll
            for (int n = 1; n < N; ++n) prod *= C[n][k];
            xh += prod;
        }
#pragma unroll
        for (int o = 1; o < TPS; o <<= 1) xh += __shfl_xor(xh, o);
        const float res = valid ? xh - a.val[ps] : 0.f;
        if (valid && sub == 0) loss += 0.5 * (double)res * (double)res;
#pragma unroll
        for (int n = 0; n < N; ++n) {
#pragma unroll
            for (int k = 0; k < RK; ++k) {
                float prod = 1.f;
#pragma unroll
                for (int m = 0; m < N; ++m)
                    if (m != n) prod *= C[m][k];
                sD[(s * N + n) * R16 + sub + TPS * k] = prod;
            }
            const float *ar = a.A[n] + (int64_t)rows[n] * J4;
            for (int j = sub; j < J4; j += TPS)
                sE[(s * N + n) * J4 + j] = res * ar[j];
        }
        __syncthreads();
#pragma unroll
        for (int pp = 0; pp < V::PP; ++pp) {
            const int u = threadIdx.x + 256 * pp;
            if (u < V::PAIRS) {
                const int tile = u % T, g = u / T;
                const int n = tile / (TJ * TR), jt = (tile / TR) % TJ,
                          rt = tile % TR;
                for (int s2 = g; s2 < S; s2 += G) {
                    const float4 e4 = *reinterpret_cast<const float4 *>(
                        sE + (s2 * N + n) * J4 + 4 * jt);
                    const float4 d4 = *reinterpret_cast<const float4 *>(
                        sD + (s2 * N + n) * R16 + 4 * rt);
                    const float ev[4] = {e4.x, e4.y, e4.z, e4.w};
                    const float dv[4] = {d4.x, d4.y, d4.z, d4.w};
#pragma unroll
                    for (int i = 0; i < 4; ++i)
#pragma unroll
                        for (int k = 0; k < 4; ++k)
                            acc[pp][i][k] = fmaf(ev[i], dv[k], acc[pp][i][k]);
                }
            }
        }
        __syncthreads();
    }

    float *red = reinterpret_cast<float *>(work4);   // [G][T][16]
#pragma unroll
    for (int pp = 0; pp < V::PP; ++pp) {
        const int u = threadIdx.x + 256 * pp;
        if (u < V::PAIRS)
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int k = 0; k < 4; ++k) red[u * 16 + 4 * i + k] = acc[pp][i][k];
    }
    __syncthreads();
    float *out = a.part + (int64_t)blockIdx.x * (N * J4 * R16);
    for (int e = threadIdx.x; e < N * J4 * R16; e += 256) {
        const int n = e / (J4 * R16), j = (e / R16) % J4, r = e % R16;
        const int tile = (n * TJ + j / 4) * TR + r / 4;
        const int inner = 4 * (j % 4) + r % 4;
        float sum = 0.f;
        for (int g = 0; g < G; ++g) sum += red[(g * T + tile) * 16 + inner];
        out[e] = sum;
    }
    const double tot = block_sum_256(loss);
    if (threadIdx.x == 0) a.loss_part[blockIdx.x] = tot;
}

template <int N, int J4, int R16>
static hipError_t launch_cgv(const CoreArgs &a, int blocks, hipStream_t s) {
    using V = CoreValu<N, J4, R16>;
    const int64_t nchunks = (a.count + V::S - 1) / V::S;
    const int fit = resident_blocks(
        reinterpret_cast<const void *>(&core_grad_valu_kernel<N, J4, R16>), 0);
    if (blocks > fit) blocks = fit;
    if (blocks > nchunks) blocks = (int)nchunks;
    if (blocks < 1) blocks = 1;
    *a.blocks_used = blocks;
    FT_LAUNCH((core_grad_valu_kernel<N, J4, R16>), dim3(blocks), dim3(256), 0,
              s, a, nchunks);
    return hipGetLastError();
}

template <int N, int J4>
static hipError_t launch_cgv_r(const Shape &sh, const CoreArgs &a, int blocks,
                               hipStream_t s) {
    if (sh.R16 == 16) return launch_cgv<N, J4, 16>(a, blocks, s);
    if (sh.R16 == 32) return launch_cgv<N, J4, 32>(a, blocks, s);
    return hipErrorInvalidValue;
}

template <int N>
static hipError_t launch_cgv_j(const Shape &sh, const CoreArgs &a, int blocks,
                               hipStream_t s) {
    switch (sh.J4) {
    case 4: return launch_cgv_r<N, 4>(sh, a, blocks, s);
    case 8: return launch_cgv_r<N, 8>(sh, a, blocks, s);
    case 12: return launch_cgv_r<N, 12>(sh, a, blocks, s);
    case 16: return launch_cgv_r<N, 16>(sh, a, blocks, s);
    case 20: return launch_cgv_r<N, 20>(sh, a, blocks, s);
    case 24: return launch_cgv_r<N, 24>(sh, a, blocks, s);
    case 28: return launch_cgv_r<N, 28>(sh, a, blocks, s);
    case 32: return launch_cgv_r<N, 32>(sh, a, blocks, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_core_grad_valu(const Shape &sh, const CoreArgs &a,
                                 int nblocks, hipStream_t s) {
    if (sh.prec != kF32) return hipErrorInvalidValue;
    if (nblocks > kCoreMaxBlocks) nblocks = kCoreMaxBlocks;
    switch (sh.N) {
    case 2: return launch_cgv_j<2>(sh, a, nblocks, s);
    case 3: return launch_cgv_j<3>(sh, a, nblocks, s);
    case 4: return launch_cgv_j<4>(sh, a, nblocks, s);
    case 5: return launch_cgv_j<5>(sh, a, nblocks, s);
    }
    return hipErrorInvalidValue;
}

// 64 consecutive elements per block; four slices of the partials each summed
// in increasing block order, then the slices in order.
// One block per 32 consecutive elements of [N][J4][R16]; thread (slice sl,
// element el) sums partials sl, sl + 32, ... (eight loads in flight), and
// thread sl = 0 adds the 32 slice sums in order.
constexpr int kUpdElems = 32, kUpdSlices = 32;

__global__ __launch_bounds__(kUpdElems * kUpdSlices) void core_update_kernel(
    CoreUpdateArgs a, int E, int J4, int R16) {
    __shared__ float part[kUpdSlices][kUpdElems + 1];
    const int el = threadIdx.x % kUpdElems, sl = threadIdx.x / kUpdElems;
    const int e = blockIdx.x * kUpdElems + el;
    float acc = 0.f;
    if (e < E) {
        int b = sl;
        for (; b + 7 * kUpdSlices < a.nblocks; b += 8 * kUpdSlices) {
            float v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u)
                v[u] = a.part[(int64_t)(b + u * kUpdSlices) * E + e];
#pragma unroll
            for (int u = 0; u < 8; ++u) acc += v[u];
        }
        for (; b < a.nblocks; b += kUpdSlices) acc += a.part[(int64_t)b * E + e];
    }
    part[sl][el] = acc;
    __syncthreads();
    if (sl == 0 && e < E) {
        float g = 0.f;
        for (int k = 0; k < kUpdSlices; ++k) g += part[k][el];
        if (a.grad_out) a.grad_out[e] = g;
        const int n = e / (J4 * R16);
        const int j = (e / R16) % J4, r = e % R16;
        if (a.gout[n] && j < a.Jn[n] && r < a.R)
            a.gout[n][j * a.R + r] = g * (a.scale ? *a.scale : 1.f);
        if (a.apply) {
            float *bp = a.B[n] + (e - n * J4 * R16);
            const float bv = *bp;
            *bp = bv - a.lr * (float)((double)g * a.inv_count + (double)a.lam * bv);
        }
    }
}

hipError_t launch_core_update(const Shape &sh, const CoreUpdateArgs &a,
                              hipStream_t s) {
    const int E = sh.N * sh.J4 * sh.R16;
    FT_LAUNCH(core_update_kernel, dim3((E + kUpdElems - 1) / kUpdElems),
              dim3(kUpdElems * kUpdSlices), 0, s, a, E, sh.J4, sh.R16);
    return hipGetLastError();
}

}  // namespace ft
