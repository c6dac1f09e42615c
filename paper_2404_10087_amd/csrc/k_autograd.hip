// k_autograd.hip -- helpers of the stateless minibatch entry points that back
// the torch.autograd.Function: zero-padding of caller-owned core matrices
// into the tile layout, and the unique-row ordinals that compact the sorted
// row reduction into a sparse (row, gradient) list.
#include "ft_internal.h"

namespace ft {

__global__ void pad_matrix_kernel(const float *src, int J, int R, float *dst,
                                  int J4, int R16) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= J4 * R16) return;
    const int j = e / R16, r = e % R16;
    dst[e] = (j < J && r < R) ? src[j * R + r] : 0.f;
}

hipError_t launch_pad_matrix(const float *src, int J, int R, float *dst,
                             int J4, int R16, hipStream_t s) {
    const int E = J4 * R16;
    hipLaunchKernelGGL(pad_matrix_kernel, dim3((E + 255) / 256), dim3(256), 0,
                       s, src, J, R, dst, J4, R16);
    return hipGetLastError();
}

__global__ void fill_zero_kernel(float *p, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += stride)
        p[i] = 0.f;
}

// A kernel, not hipMemsetAsync, so that callers may capture it in a graph.
hipError_t launch_fill_zero(float *p, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(fill_zero_kernel, dim3((int)blocks), dim3(256), 0, s, p,
                       n);
    return hipGetLastError();
}

constexpr int kScanItems = 8;
constexpr int kScanTile = 256 * kScanItems;

__device__ __forceinline__ uint32_t is_head(const uint32_t *rows, int32_t i) {
    return (i == 0 || rows[i] != rows[i - 1]) ? 1u : 0u;
}

// Exclusive scan of one value per thread over a 256-thread block (fixed
// Hillis-Steele order); returns the block total through *total.
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v,
                                                         uint32_t *total) {
    __shared__ uint32_t s[256];
    const int t = threadIdx.x;
    s[t] = v;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        const uint32_t x = t >= off ? s[t - off] : 0u;
        __syncthreads();
        s[t] += x;
        __syncthreads();
    }
    const uint32_t incl = s[t];
    *total = s[255];
    __syncthreads();
    return incl - v;
}

// grid (ntiles, N)
__global__ __launch_bounds__(256) void unique_count_kernel(UniqueScan u) {
    const int tile = blockIdx.x, n = blockIdx.y;
    const int32_t base = tile * kScanTile + threadIdx.x * kScanItems;
    uint32_t c = 0;
    for (int k = 0; k < kScanItems; ++k)
        if (base + k < u.m) c += is_head(u.rows[n], base + k);
    uint32_t total;
    block_exclusive_scan(c, &total);
    if (threadIdx.x == 0) u.tile_count[(int64_t)n * u.ntiles + tile] = total;
}

// grid (N): exclusive scan of the tile counts, 256 at a time with a carry
__global__ __launch_bounds__(256) void unique_offsets_kernel(UniqueScan u) {
    const int n = blockIdx.x;
    uint32_t *tc = u.tile_count + (int64_t)n * u.ntiles;
    uint32_t carry = 0;
    for (int b = 0; b < u.ntiles; b += 256) {
        const int t = b + threadIdx.x;
        const uint32_t v = t < u.ntiles ? tc[t] : 0u;
        uint32_t total;
        const uint32_t ex = block_exclusive_scan(v, &total);
        if (t < u.ntiles) tc[t] = carry + ex;
        carry += total;
    }
    if (threadIdx.x == 0) u.total[n] = (int64_t)carry;
}

// grid (ntiles, N)
__global__ __launch_bounds__(256) void unique_ordinal_kernel(UniqueScan u) {
    const int tile = blockIdx.x, n = blockIdx.y;
    const int32_t base = tile * kScanTile + threadIdx.x * kScanItems;
    uint32_t h[kScanItems];
    uint32_t c = 0;
    for (int k = 0; k < kScanItems; ++k) {
        h[k] = base + k < u.m ? is_head(u.rows[n], base + k) : 0u;
        c += h[k];
    }
    uint32_t total;
    uint32_t run = block_exclusive_scan(c, &total) +
                   u.tile_count[(int64_t)n * u.ntiles + tile];
    for (int k = 0; k < kScanItems; ++k) {
        if (base + k < u.m) u.ordinal[n][base + k] = run;
        run += h[k];
    }
}

hipError_t launch_unique_scan(const UniqueScan &u, hipStream_t s) {
    dim3 g(u.ntiles, u.N);
    hipLaunchKernelGGL(unique_count_kernel, g, dim3(256), 0, s, u);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(unique_offsets_kernel, dim3(u.N), dim3(256), 0, s, u);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(unique_ordinal_kernel, g, dim3(256), 0, s, u);
    return hipGetLastError();
}

}  // namespace ft
