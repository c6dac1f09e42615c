// mfma_tile.h -- 16-sample tiles on the CDNA matrix cores.
//
// v_mfma_f32_16x16x4_f32 multiplies a 16x4 A-operand by a 4x16 B-operand into
// a 16x16 FP32 accumulator. In a wave of 64 lanes, lane l supplies
//     A[i = l % 16][k = l / 16]   and   B[k = l / 16][j = l % 16]
// and holds the result rows i = 4*(l / 16) + v (v = 0..3) of column j = l % 16.
//
// Contraction over K = 4*KQ is split into KQ steps. The K index that step t
// gives lane quad q = l / 16 is k = KQ*q + t, so every lane reads KQ
// *consecutive* entries of one factor row with a single vector load. Any
// permutation of K applied to both operands leaves the product unchanged.
#pragma once

#include <hip/hip_runtime.h>

namespace ft {

typedef float floatx4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ floatx4 mfma_16x16x4(float a, float b, floatx4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Load KQ consecutive floats (16-byte aligned when KQ is a multiple of 4).
template <int KQ>
__device__ __forceinline__ void load_row_part(const float *p, float (&out)[KQ]) {
    if constexpr (KQ % 4 == 0) {
#pragma unroll
        for (int t = 0; t < KQ; t += 4) {
            float4 v = *reinterpret_cast<const float4 *>(p + t);
            out[t] = v.x;
            out[t + 1] = v.y;
            out[t + 2] = v.z;
            out[t + 3] = v.w;
        }
    } else if constexpr (KQ == 2) {
        float2 v = *reinterpret_cast<const float2 *>(p);
        out[0] = v.x;
        out[1] = v.y;
    } else {
#pragma unroll
        for (int t = 0; t < KQ; ++t) out[t] = p[t];
    }
}

// Sum over the four lanes that share l % 16 (lanes l, l^16, l^32, l^48).
__device__ __forceinline__ float sum_quads(float x) {
    x += __shfl_xor(x, 16);
    x += __shfl_xor(x, 32);
    return x;
}

// Sum over the sixteen lanes that share l / 16.
__device__ __forceinline__ float sum_row16(float x) {
    x += __shfl_xor(x, 1);
    x += __shfl_xor(x, 2);
    x += __shfl_xor(x, 4);
    x += __shfl_xor(x, 8);
    return x;
}

__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o);
    return x;
}

// Fixed-order block reduction of one double per thread (blockDim.x = 256):
// wave sums, then waves 0..3 in order. Returns the total in thread 0.
__device__ __forceinline__ double block_sum_256(double x) {
    __shared__ double ws[4];
    x = wave_sum(x);
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = x;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0) t = ((ws[0] + ws[1]) + ws[2]) + ws[3];
    __syncthreads();
    return t;
}

}  // namespace ft
