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
typedef short shortx4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ floatx4 mfma_16x16x4(float a, float b, floatx4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// BF16 inputs, FP32 accumulation: 16x16 output, K = 16 split as 4 bf16 per
// lane over the four lane quads (same row/column roles as above).
__device__ __forceinline__ floatx4 mfma_16x16x16_bf16(shortx4 a, shortx4 b,
                                                      floatx4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// FP32 -> BF16 with round-to-nearest-even (finite inputs), and back.
__device__ __forceinline__ uint16_t f2bf(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) {
    return __uint_as_float((uint32_t)h << 16);
}

// One lane's share of a factor row for the contraction over j: KQ
// consecutive entries starting at KQ*q (q = lane / 16). FP32 keeps them as
// floats (one 16x16x4 step each); BF16 packs them four to a 16x16x16 step,
// zero-filling the last pack.
template <int KQ, bool BF>
struct RowFrag;

template <int KQ>
struct RowFrag<KQ, false> {
    static constexpr int STEPS = KQ;
    float v[KQ];
    __device__ __forceinline__ void load(const float *A, const uint16_t *,
                                         int64_t off) {
        load_row(A + off);
    }
    __device__ __forceinline__ void load_row(const float *p);
    __device__ __forceinline__ float value(int t) const { return v[t]; }
};

template <int KQ>
struct RowFrag<KQ, true> {
    static constexpr int STEPS = (KQ + 3) / 4;
    shortx4 v[STEPS];
    __device__ __forceinline__ void load(const float *, const uint16_t *A16,
                                         int64_t off) {
        const uint16_t *p = A16 + off;
        if constexpr (KQ % 4 == 0) {
#pragma unroll
            for (int u = 0; u < STEPS; ++u)
                v[u] = *reinterpret_cast<const shortx4 *>(p + 4 * u);
        } else {
#pragma unroll
            for (int u = 0; u < STEPS; ++u)
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    v[u][e] = 4 * u + e < KQ ? (short)p[4 * u + e] : (short)0;
        }
    }
    __device__ __forceinline__ float value(int t) const {
        return bf2f((uint16_t)v[t / 4][t % 4]);
    }
};

// The matching share of a core matrix column block: entry (t) is
// B[KQ*q + t][col], packed like RowFrag.
template <int KQ, bool BF>
struct ColFrag;

template <int KQ>
struct ColFrag<KQ, false> {
    float v[KQ];
    __device__ __forceinline__ void load(const float *B, int R16, int q,
                                         int col) {
#pragma unroll
        for (int t = 0; t < KQ; ++t) v[t] = B[(KQ * q + t) * R16 + col];
    }
};

template <int KQ>
struct ColFrag<KQ, true> {
    static constexpr int STEPS = (KQ + 3) / 4;
    shortx4 v[STEPS];
    __device__ __forceinline__ void load(const float *B, int R16, int q,
                                         int col) {
#pragma unroll
        for (int u = 0; u < STEPS; ++u)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int t = 4 * u + e;
                v[u][e] = t < KQ ? (short)f2bf(B[(KQ * q + t) * R16 + col])
                                 : (short)0;
            }
    }
};

// acc += X Y over the K shares of one lane (X is the A-operand, Y the
// B-operand of the matrix-core step).
template <int KQ>
__device__ __forceinline__ floatx4 contract(const ColFrag<KQ, false> &x,
                                            const RowFrag<KQ, false> &y,
                                            floatx4 acc) {
#pragma unroll
    for (int t = 0; t < KQ; ++t) acc = mfma_16x16x4(x.v[t], y.v[t], acc);
    return acc;
}
template <int KQ>
__device__ __forceinline__ floatx4 contract(const ColFrag<KQ, true> &x,
                                            const RowFrag<KQ, true> &y,
                                            floatx4 acc) {
#pragma unroll
    for (int u = 0; u < (KQ + 3) / 4; ++u)
        acc = mfma_16x16x16_bf16(x.v[u], y.v[u], acc);
    return acc;
}
template <int KQ>
__device__ __forceinline__ floatx4 contract(const RowFrag<KQ, false> &x,
                                            const ColFrag<KQ, false> &y,
                                            floatx4 acc) {
#pragma unroll
    for (int t = 0; t < KQ; ++t) acc = mfma_16x16x4(x.v[t], y.v[t], acc);
    return acc;
}
template <int KQ>
__device__ __forceinline__ floatx4 contract(const RowFrag<KQ, true> &x,
                                            const ColFrag<KQ, true> &y,
                                            floatx4 acc) {
#pragma unroll
    for (int u = 0; u < (KQ + 3) / 4; ++u)
        acc = mfma_16x16x16_bf16(x.v[u], y.v[u], acc);
    return acc;
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

// Store N consecutive floats (16-byte aligned when N is a multiple of 4).
template <int NF>
__device__ __forceinline__ void store_row(float *p, const float (&v)[NF]) {
    if constexpr (NF % 4 == 0) {
#pragma unroll
        for (int t = 0; t < NF; t += 4)
            *reinterpret_cast<float4 *>(p + t) =
                make_float4(v[t], v[t + 1], v[t + 2], v[t + 3]);
    } else {
#pragma unroll
        for (int t = 0; t < NF; ++t) p[t] = v[t];
    }
}

template <int KQ>
__device__ __forceinline__ void RowFrag<KQ, false>::load_row(const float *p) {
    load_row_part<KQ>(p, v);
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

// Order the LDS traffic of one wave (its lanes exchange data through LDS
// without a workgroup barrier).
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
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
