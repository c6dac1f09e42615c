// k_eval.hip -- forward-only residual statistics (test RMSE/MAE of Section
// 5.2 and the data term of Eq. (4)) and squared Frobenius norms of the
// parameters (the regularisers of Eq. (4)). Residuals are formed in FP32 and
// reduced in FP64 in a fixed order.
#include "ft_internal.h"
#include "mfma_tile.h"

namespace ft {

constexpr int kEvalMaxBlocks = 1024;

int eval_blocks(int64_t count) {
    int64_t ntiles = (count + 15) / 16;
    int64_t blocks = (ntiles + 3) / 4;
    if (blocks > kEvalMaxBlocks) blocks = kEvalMaxBlocks;
    return blocks < 1 ? 1 : (int)blocks;
}

template <int N, int KQ, int RB, bool BF>
__global__ __launch_bounds__(256) void eval_kernel(EvalArgs a, int64_t ntiles) {
    constexpr int J4 = 4 * KQ;
    constexpr int R16 = 16 * RB;
    const int lane = threadIdx.x & 63, q = lane >> 4, c = lane & 15;
    ColFrag<KQ, BF> bf[N][RB];
#pragma unroll
    for (int n = 0; n < N; ++n)
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
            bf[n][rb].load(a.B[n], R16, q, 16 * rb + c);
    double sse = 0.0, sae = 0.0;
    const int64_t nwaves = (int64_t)gridDim.x * 4;
    for (int64_t tile = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
         tile < ntiles; tile += nwaves) {
        const int64_t p = tile * 16 + c;
        const bool valid = p < a.count;
        const int64_t ps = valid ? p : a.count - 1;
        RowFrag<KQ, BF> arow[N];
#pragma unroll
        for (int n = 0; n < N; ++n) {
            const int row = a.idx[n][ps];
            arow[n].load(a.A[n], a.A16[n], (int64_t)row * J4 + KQ * q);
        }
        float xh = 0.f;
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
            floatx4 prod = {1.f, 1.f, 1.f, 1.f};
#pragma unroll
            for (int n = 0; n < N; ++n) {
                prod *= contract(bf[n][rb], arow[n],
                                 floatx4{0.f, 0.f, 0.f, 0.f});
            }
            xh += (prod[0] + prod[1]) + (prod[2] + prod[3]);
        }
        xh = sum_quads(xh);
        if (valid && q == 0) {
            const double r = (double)(xh - a.val[ps]);
            sse += a.half_square ? 0.5 * r * r : r * r;
            sae += fabs(r);
        }
    }
    const double t1 = block_sum_256(sse);
    const double t2 = block_sum_256(sae);
    if (threadIdx.x == 0) {
        a.part[blockIdx.x] = t1;
        a.part[gridDim.x + blockIdx.x] = t2;
    }
}

template <int N, int KQ, int RB, bool BF>
static hipError_t launch_ev(const EvalArgs &a, int blocks, hipStream_t s) {
    const int64_t ntiles = (a.count + 15) / 16;
    FT_LAUNCH((eval_kernel<N, KQ, RB, BF>), dim3(blocks), dim3(256), 0,
                       s, a, ntiles);
    return hipGetLastError();
}

template <int N, int KQ>
static hipError_t launch_ev_r(const Shape &sh, const EvalArgs &a, int blocks,
                              hipStream_t s) {
    if (sh.bf16)
        return sh.R16 == 16 ? launch_ev<N, KQ, 1, true>(a, blocks, s)
                            : launch_ev<N, KQ, 2, true>(a, blocks, s);
    return sh.R16 == 16 ? launch_ev<N, KQ, 1, false>(a, blocks, s)
                        : launch_ev<N, KQ, 2, false>(a, blocks, s);
}

template <int N>
static hipError_t launch_ev_j(const Shape &sh, const EvalArgs &a, int blocks,
                              hipStream_t s) {
    switch (sh.J4) {
    case 4: return launch_ev_r<N, 1>(sh, a, blocks, s);
    case 8: return launch_ev_r<N, 2>(sh, a, blocks, s);
    case 12: return launch_ev_r<N, 3>(sh, a, blocks, s);
    case 16: return launch_ev_r<N, 4>(sh, a, blocks, s);
    case 20: return launch_ev_r<N, 5>(sh, a, blocks, s);
    case 24: return launch_ev_r<N, 6>(sh, a, blocks, s);
    case 28: return launch_ev_r<N, 7>(sh, a, blocks, s);
    case 32: return launch_ev_r<N, 8>(sh, a, blocks, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_eval(const Shape &sh, const EvalArgs &a, int nblocks,
                       hipStream_t s) {
    switch (sh.N) {
    case 2: return launch_ev_j<2>(sh, a, nblocks, s);
    case 3: return launch_ev_j<3>(sh, a, nblocks, s);
    case 4: return launch_ev_j<4>(sh, a, nblocks, s);
    case 5: return launch_ev_j<5>(sh, a, nblocks, s);
    }
    return hipErrorInvalidValue;
}

__global__ __launch_bounds__(256) void sumsq_kernel(const float *x, int64_t n,
                                                    double *part) {
    double acc = 0.0;
    const int64_t stride = (int64_t)gridDim.x * 256;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride)
        acc += (double)x[i] * (double)x[i];
    const double t = block_sum_256(acc);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

__global__ void to_bf16_kernel(const float *src, uint16_t *dst, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += stride)
        dst[i] = f2bf(src[i]);
}

hipError_t launch_to_bf16(const float *src, uint16_t *dst, int64_t n,
                          hipStream_t s) {
    int64_t blocks = (n + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    if (blocks < 1) return hipSuccess;
    hipLaunchKernelGGL(to_bf16_kernel, dim3((int)blocks), dim3(256), 0, s, src,
                       dst, n);
    return hipGetLastError();
}

hipError_t launch_sumsq(const float *x, int64_t n, double *part, int nblocks,
                        hipStream_t s) {
    hipLaunchKernelGGL(sumsq_kernel, dim3(nblocks), dim3(256), 0, s, x, n,
                       part);
    return hipGetLastError();
}

}  // namespace ft
