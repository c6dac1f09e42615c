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

#include "ft_internal.h"

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

// FP8 (OCP e4m3) inputs, FP32 accumulation: 16x16 output, K = 32 split as 8
// bytes per lane over the four lane quads: lane l gives A[l % 16][8(l / 16)
// + e] and B[8(l / 16) + e][l % 16], e = 0..7 (byte e of the 64-bit operand).
__device__ __forceinline__ floatx4 mfma_16x16x32_fp8(long a, long b, floatx4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(a, b, c, 0, 0, 0);
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

// FP8 e4m3 quantisation with one FP32 scale per vector: s = max|x| / 448
// (448 is the largest e4m3 value), q = e4m3(x * (448 / max|x|)) rounded to
// nearest even by the hardware conversion, clamped to +-448 first; x is
// represented as s * q. An all-zero vector gets s = 0 and zero codes. A
// vector holding a NaN or an infinity gets a NaN scale (fmaxf would drop a
// NaN and the clamp would turn it into a finite code), so non-finite
// parameters stay visible in the losses computed from the shadow.
constexpr float kFP8Max = 448.f;
__device__ __forceinline__ uint32_t fp8x4(float a, float b, float c, float d) {
    const uint32_t w = __builtin_amdgcn_cvt_pk_fp8_f32(a, b, 0u, false);
    return __builtin_amdgcn_cvt_pk_fp8_f32(c, d, w, true);
}
__device__ __forceinline__ float fp8_prescale(float maxabs) {
    return maxabs > 0.f ? kFP8Max / maxabs : 0.f;
}
__device__ __forceinline__ float fp8_clamp(float x) {
    return fminf(fmaxf(x, -kFP8Max), kFP8Max);
}
__device__ __forceinline__ float fp8_byte(uint64_t w, int e) {
    const uint32_t h = (uint32_t)(w >> (32 * (e / 4)));
    switch (e & 3) {
    case 0: return __builtin_amdgcn_cvt_f32_fp8(h, 0);
    case 1: return __builtin_amdgcn_cvt_f32_fp8(h, 1);
    case 2: return __builtin_amdgcn_cvt_f32_fp8(h, 2);
    default: return __builtin_amdgcn_cvt_f32_fp8(h, 3);
    }
}

// Quantise one row of J4 floats (J4 a multiple of 4) to J4 e4m3 bytes and
// its scale.
template <int J4>
__device__ __forceinline__ void quantize_row_fp8(const float (&x)[J4],
                                                 uint8_t *dst, float *sdst) {
    float m = 0.f, nf = 0.f;
#pragma unroll
    for (int j = 0; j < J4; ++j) {
        m = fmaxf(m, fabsf(x[j]));
        nf += x[j] * 0.f;   // NaN if x[j] is NaN or infinite
    }
    const float inv = fp8_prescale(m);
    uint32_t *d = reinterpret_cast<uint32_t *>(dst);
#pragma unroll
    for (int j = 0; j < J4; j += 4)
        d[j / 4] = fp8x4(fp8_clamp(x[j] * inv), fp8_clamp(x[j + 1] * inv),
                         fp8_clamp(x[j + 2] * inv), fp8_clamp(x[j + 3] * inv));
    *sdst = m / kFP8Max + nf;
}

// Where a tile reads factor rows from: the FP32 master and the BF16 or FP8
// (+ per-row scale) shadow of the contraction precision.
struct RowSrc {
    const float *A;
    const uint16_t *A16;
    const uint8_t *A8;
    const float *As;
};

// One lane's share of a factor row for the contraction over j: KQ
// consecutive entries starting at KQ*q (q = lane / 16). FP32 keeps them as
// floats (one 16x16x4 step each); BF16 packs them four to a 16x16x16 step
// and FP8 eight to a 16x16x32 step, zero-filling the last pack. FP8 also
// keeps the row's scale.
template <int KQ, int P>
struct RowFrag;

template <int KQ>
struct RowFrag<KQ, kF32> {
    static constexpr int STEPS = KQ;
    float v[KQ];
    __device__ __forceinline__ void load(const RowSrc &src, int64_t row,
                                         int J4, int q) {
        load_row(src.A + row * J4 + KQ * q);
    }
    __device__ __forceinline__ void load_row(const float *p);
    __device__ __forceinline__ float value(int t) const { return v[t]; }
};

template <int KQ>
struct RowFrag<KQ, kBF16> {
    static constexpr int STEPS = (KQ + 3) / 4;
    shortx4 v[STEPS];
    __device__ __forceinline__ void load(const RowSrc &src, int64_t row,
                                         int J4, int q) {
        const uint16_t *p = src.A16 + row * J4 + KQ * q;
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

template <int KQ>
struct RowFrag<KQ, kFP8> {
    static constexpr int STEPS = (KQ + 7) / 8;
    long v[STEPS];
    float s;
    __device__ __forceinline__ void load(const RowSrc &src, int64_t row,
                                         int J4, int q) {
        const uint8_t *p = src.A8 + row * J4 + KQ * q;
        s = src.As[row];
        if constexpr (KQ == 8) {
            v[0] = *reinterpret_cast<const long *>(p);
        } else if constexpr (KQ == 4) {
            v[0] = (long)*reinterpret_cast<const uint32_t *>(p);
        } else {
            uint64_t w = 0;
#pragma unroll
            for (int t = 0; t < KQ; ++t) w |= (uint64_t)p[t] << (8 * t);
            v[0] = (long)w;
        }
    }
    __device__ __forceinline__ float value(int t) const {
        return s * fp8_byte((uint64_t)v[t / 8], t % 8);
    }
};

// The matching share of a core matrix column block: entry (t) is
// B[KQ*q + t][col], packed like RowFrag. FP8 quantises the whole column
// (all J4 entries, gathered over the four lane quads) with one scale.
template <int KQ, int P>
struct ColFrag;

template <int KQ>
struct ColFrag<KQ, kF32> {
    float v[KQ];
    __device__ __forceinline__ void load(const float *B, int R16, int q,
                                         int col) {
#pragma unroll
        for (int t = 0; t < KQ; ++t) v[t] = B[(KQ * q + t) * R16 + col];
    }
};

template <int KQ>
struct ColFrag<KQ, kBF16> {
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

template <int KQ>
struct ColFrag<KQ, kFP8> {
    static constexpr int STEPS = (KQ + 7) / 8;
    long v[STEPS];
    float s;
    __device__ __forceinline__ void load(const float *B, int R16, int q,
                                         int col) {
        float x[KQ];
        float m = 0.f, nf = 0.f;
#pragma unroll
        for (int t = 0; t < KQ; ++t) {
            x[t] = B[(KQ * q + t) * R16 + col];
            m = fmaxf(m, fabsf(x[t]));
            nf += x[t] * 0.f;   // NaN if x[t] is NaN or infinite
        }
        m = fmaxf(m, __shfl_xor(m, 16));
        m = fmaxf(m, __shfl_xor(m, 32));
        nf += __shfl_xor(nf, 16);
        nf += __shfl_xor(nf, 32);
        const float inv = fp8_prescale(m);
        uint64_t w = 0;
#pragma unroll
        for (int t = 0; t < KQ; t += 4) {
            const float x0 = fp8_clamp(x[t] * inv);
            const float x1 = t + 1 < KQ ? fp8_clamp(x[t + 1] * inv) : 0.f;
            const float x2 = t + 2 < KQ ? fp8_clamp(x[t + 2] * inv) : 0.f;
            const float x3 = t + 3 < KQ ? fp8_clamp(x[t + 3] * inv) : 0.f;
            w |= (uint64_t)fp8x4(x0, x1, x2, x3) << (8 * t);
        }
        v[0] = (long)w;
        s = m / kFP8Max + nf;
    }
};

// acc += X Y over the K shares of one lane (X is the A-operand, Y the
// B-operand of the matrix-core step). For FP8 the caller applies the
// scales (fp8_scale_ct / fp8_scale_c).
template <int KQ>
__device__ __forceinline__ floatx4 contract(const ColFrag<KQ, kF32> &x,
                                            const RowFrag<KQ, kF32> &y,
                                            floatx4 acc) {
#pragma unroll
    for (int t = 0; t < KQ; ++t) acc = mfma_16x16x4(x.v[t], y.v[t], acc);
    return acc;
}
template <int KQ>
__device__ __forceinline__ floatx4 contract(const ColFrag<KQ, kBF16> &x,
                                            const RowFrag<KQ, kBF16> &y,
                                            floatx4 acc) {
#pragma unroll
    for (int u = 0; u < (KQ + 3) / 4; ++u)
        acc = mfma_16x16x16_bf16(x.v[u], y.v[u], acc);
    return acc;
}
template <int KQ>
__device__ __forceinline__ floatx4 contract(const ColFrag<KQ, kFP8> &x,
                                            const RowFrag<KQ, kFP8> &y,
                                            floatx4 acc) {
#pragma unroll
    for (int u = 0; u < (KQ + 7) / 8; ++u)
        acc = mfma_16x16x32_fp8(x.v[u], y.v[u], acc);
    return acc;
}
template <int KQ>
__device__ __forceinline__ floatx4 contract(const RowFrag<KQ, kF32> &x,
                                            const ColFrag<KQ, kF32> &y,
                                            floatx4 acc) {
#pragma unroll
    for (int t = 0; t < KQ; ++t) acc = mfma_16x16x4(x.v[t], y.v[t], acc);
    return acc;
}
template <int KQ>
__device__ __forceinline__ floatx4 contract(const RowFrag<KQ, kBF16> &x,
                                            const ColFrag<KQ, kBF16> &y,
                                            floatx4 acc) {
#pragma unroll
    for (int u = 0; u < (KQ + 3) / 4; ++u)
        acc = mfma_16x16x16_bf16(x.v[u], y.v[u], acc);
    return acc;
}
template <int KQ>
__device__ __forceinline__ floatx4 contract(const RowFrag<KQ, kFP8> &x,
                                            const ColFrag<KQ, kFP8> &y,
                                            floatx4 acc) {
#pragma unroll
    for (int u = 0; u < (KQ + 7) / 8; ++u)
        acc = mfma_16x16x32_fp8(x.v[u], y.v[u], acc);
    return acc;
}

// Scales of an FP8 product. C^T form (rows r = 4q + v of a column block,
// column = this lane's sample): column scale of r from lane 4q + v, row
// scale of the lane's own sample. C form (rows = samples 4q + v, column =
// this lane's r): the lane's own column scale, sample scales from lanes
// 4q + v.
__device__ __forceinline__ floatx4 fp8_scale_ct(floatx4 acc, float col_s,
                                                float row_s, int q) {
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[v] *= __shfl(col_s, 4 * q + v) * row_s;
    return acc;
}
__device__ __forceinline__ floatx4 fp8_scale_c(floatx4 acc, float col_s,
                                               float row_s, int q) {
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[v] *= col_s * __shfl(row_s, 4 * q + v);
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
__device__ __forceinline__ void RowFrag<KQ, kF32>::load_row(const float *p) {
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
