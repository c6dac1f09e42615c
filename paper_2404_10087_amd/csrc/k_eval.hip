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

template <int N, int KQ, int RB, int P>
__global__ __launch_bounds__(256) void eval_kernel(EvalArgs a, int64_t ntiles) {
    constexpr int J4 = 4 * KQ;
    constexpr int R16 = 16 * RB;
    const int lane = threadIdx.x & 63, q = lane >> 4, c = lane & 15;
    ColFrag<KQ, P> bf[N][RB];
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
        RowFrag<KQ, P> arow[N];
#pragma unroll
        for (int n = 0; n < N; ++n) {
            const int row = a.idx[n][ps];
            arow[n].load(RowSrc{a.A[n], a.A16[n], a.A8[n], a.As[n]}, row, J4,
                         q);
        }
        float xh = 0.f;
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
            floatx4 prod = {1.f, 1.f, 1.f, 1.f};
#pragma unroll
            for (int n = 0; n < N; ++n) {
                floatx4 C = contract(bf[n][rb], arow[n],
                                     floatx4{0.f, 0.f, 0.f, 0.f});
                if constexpr (P == kFP8)
                    C = fp8_scale_ct(C, bf[n][rb].s, arow[n].s, q);
                prod *= C;
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

template <int N, int KQ, int RB, int P>
static hipError_t launch_ev(const EvalArgs &a, int blocks, hipStream_t s) {
    const int64_t ntiles = (a.count + 15) / 16;
    FT_LAUNCH((eval_kernel<N, KQ, RB, P>), dim3(blocks), dim3(256), 0,
                       s, a, ntiles);
    return hipGetLastError();
}

template <int N, int KQ, int P>
static hipError_t launch_ev_p(const Shape &sh, const EvalArgs &a, int blocks,
                              hipStream_t s) {
    return sh.R16 == 16 ? launch_ev<N, KQ, 1, P>(a, blocks, s)
                        : launch_ev<N, KQ, 2, P>(a, blocks, s);
}

template <int N, int KQ>
static hipError_t launch_ev_r(const Shape &sh, const EvalArgs &a, int blocks,
                              hipStream_t s) {
    if constexpr (N > kFullOrder) {  // FP32 only above the full orders
        return sh.prec == kF32 ? launch_ev_p<N, KQ, kF32>(sh, a, blocks, s)
                               : hipErrorInvalidValue;
    } else {
        switch (sh.prec) {
        case kF32: return launch_ev_p<N, KQ, kF32>(sh, a, blocks, s);
        case kBF16: return launch_ev_p<N, KQ, kBF16>(sh, a, blocks, s);
        case kFP8: return launch_ev_p<N, KQ, kFP8>(sh, a, blocks, s);
        }
        return hipErrorInvalidValue;
    }
}

template <int N>
static hipError_t launch_ev_j(const Shape &sh, const EvalArgs &a, int blocks,
                              hipStream_t s) {
    if constexpr (N > kFullOrder) {   // J4 padded to 8, 16 or 32
        switch (sh.J4) {
        case 8: return launch_ev_r<N, 2>(sh, a, blocks, s);
        case 16: return launch_ev_r<N, 4>(sh, a, blocks, s);
        case 32: return launch_ev_r<N, 8>(sh, a, blocks, s);
        }
        return hipErrorInvalidValue;
    } else {
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
}

hipError_t launch_eval(const Shape &sh, const EvalArgs &a, int nblocks,
                       hipStream_t s) {
    switch (sh.N) {
    case 2: return launch_ev_j<2>(sh, a, nblocks, s);
    case 3: return launch_ev_j<3>(sh, a, nblocks, s);
    case 4: return launch_ev_j<4>(sh, a, nblocks, s);
    case 5: return launch_ev_j<5>(sh, a, nblocks, s);
    case 6: return launch_ev_j<6>(sh, a, nblocks, s);
    case 7: return launch_ev_j<7>(sh, a, nblocks, s);
    case 8: return launch_ev_j<8>(sh, a, nblocks, s);
    case 9: return launch_ev_j<9>(sh, a, nblocks, s);
    case 10: return launch_ev_j<10>(sh, a, nblocks, s);
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

// One thread per row: J4 e4m3 codes and the row's scale (the same
// quantisation as a factor-row update).
template <int J4>
__global__ void to_fp8_rows_kernel(const float *src, int64_t rows,
                                   uint8_t *dst, float *scale) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < rows;
         r += stride) {
        float x[J4];
        load_row_part<J4>(src + r * J4, x);
        quantize_row_fp8<J4>(x, dst + r * J4, scale + r);
    }
}

hipError_t launch_to_fp8_rows(const float *src, int64_t rows, int J4,
                              uint8_t *dst, float *scale, hipStream_t s) {
    int64_t blocks = (rows + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    if (blocks < 1) return hipSuccess;
    const dim3 g((int)blocks), b(256);
    switch (J4) {
    case 4: hipLaunchKernelGGL(to_fp8_rows_kernel<4>, g, b, 0, s, src, rows, dst, scale); break;
    case 8: hipLaunchKernelGGL(to_fp8_rows_kernel<8>, g, b, 0, s, src, rows, dst, scale); break;
    case 12: hipLaunchKernelGGL(to_fp8_rows_kernel<12>, g, b, 0, s, src, rows, dst, scale); break;
    case 16: hipLaunchKernelGGL(to_fp8_rows_kernel<16>, g, b, 0, s, src, rows, dst, scale); break;
    case 20: hipLaunchKernelGGL(to_fp8_rows_kernel<20>, g, b, 0, s, src, rows, dst, scale); break;
    case 24: hipLaunchKernelGGL(to_fp8_rows_kernel<24>, g, b, 0, s, src, rows, dst, scale); break;
    case 28: hipLaunchKernelGGL(to_fp8_rows_kernel<28>, g, b, 0, s, src, rows, dst, scale); break;
    case 32: hipLaunchKernelGGL(to_fp8_rows_kernel<32>, g, b, 0, s, src, rows, dst, scale); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
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
