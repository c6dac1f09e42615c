// k_builder.hip -- epoch order, stream permutation and the mode-sorted
// minibatch builder.
//
// Algorithm 3 draws every sample set Psi at random from the whole of Omega
// (Section 3.2, Table 3); one epoch is read as one pass without replacement:
// a permutation of the training set cut into consecutive minibatches of M.
// The factor-phase reduction needs, for every minibatch and mode, the samples
// grouped by row in a fixed order; the builder sorts each minibatch's row
// keys stably (ties keep minibatch order) with an LSD radix sort whose tiles
// never straddle a minibatch.
#include <algorithm>

#include "ft_internal.h"

namespace ft {

// ------------------------------------------------------------------ order
// Counter-based permutation of [0, n): a 4-round balanced Feistel network on
// 2h bits (Luby-Rackoff) whose round function is the SplitMix64 finaliser
// (Steele, Lea & Flood, 2014), restricted to [0, n) by cycle walking (Black &
// Rogaway, 2002). Round keys are consecutive SplitMix64 outputs from `key`.
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

struct Feistel {
    uint64_t k[4];
    int h;
    uint64_t mask;
};

__global__ void epoch_order_kernel(uint32_t *perm, int64_t n, Feistel f) {
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n;
         p += stride) {
        uint64_t x = (uint64_t)p;
        do {
            uint64_t L = x >> f.h, R = x & f.mask;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                uint64_t t = L ^ (mix64(R ^ f.k[i]) & f.mask);
                L = R;
                R = t;
            }
            x = (L << f.h) | R;
        } while (x >= (uint64_t)n);
        perm[p] = (uint32_t)x;
    }
}

static uint64_t host_mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

hipError_t launch_epoch_order(uint32_t *perm, int64_t n, uint64_t key,
                              hipStream_t s) {
    Feistel f;
    uint64_t st = key;
    for (int i = 0; i < 4; ++i) {
        st += 0x9e3779b97f4a7c15ull;
        f.k[i] = host_mix64(st);
    }
    int bits = 2;
    while ((1ll << bits) < n) ++bits;
    if (bits & 1) ++bits;
    f.h = bits / 2;
    f.mask = (1ull << f.h) - 1;
    int blocks = (int)((n + 255) / 256);
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(epoch_order_kernel, dim3(blocks), dim3(256), 0, s, perm,
                       n, f);
    return hipGetLastError();
}

__global__ void copy_order_kernel(uint32_t *perm, const int64_t *src,
                                  int64_t n) {
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n;
         p += stride)
        perm[p] = (uint32_t)src[p];
}

hipError_t launch_copy_order(uint32_t *perm, const int64_t *src, int64_t n,
                             hipStream_t s) {
    int blocks = (int)((n + 255) / 256);
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(copy_order_kernel, dim3(blocks), dim3(256), 0, s, perm,
                       src, n);
    return hipGetLastError();
}

// ------------------------------------------------------------------ permute
// The training set is also kept as records (i_1..i_N, x) of RW 32-bit words
// (RW = 4 for order <= 3, 8 otherwise), so the random gather of one sample is
// one 16- or 32-byte load: pidx[n][p] = rec[perm[p]].i_n, pval[p] = .x.
hipError_t launch_pack_records(int N, const int32_t *const *idx,
                               const float *val, int64_t nnz, uint32_t *rec,
                               int rw, hipStream_t s);

struct PackArgs {
    const int32_t *idx[kMaxOrder];
    const float *val;
    int64_t nnz;
    int N;
    uint32_t *rec;
};

template <int RW>
__global__ void pack_records_kernel(PackArgs a) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < a.nnz;
         s += stride) {
        uint32_t w[RW];
#pragma unroll
        for (int k = 0; k < RW; ++k) w[k] = 0u;
        for (int n = 0; n < a.N; ++n) w[n] = (uint32_t)a.idx[n][s];
        w[RW - 1] = __float_as_uint(a.val[s]);
        uint4 *dst = reinterpret_cast<uint4 *>(a.rec + s * RW);
#pragma unroll
        for (int k = 0; k < RW; k += 4)
            dst[k / 4] = make_uint4(w[k], w[k + 1], w[k + 2], w[k + 3]);
    }
}

hipError_t launch_pack_records(int N, const int32_t *const *idx,
                               const float *val, int64_t nnz, uint32_t *rec,
                               int rw, hipStream_t s) {
    PackArgs a{};
    for (int n = 0; n < N; ++n) a.idx[n] = idx[n];
    a.val = val;
    a.nnz = nnz;
    a.N = N;
    a.rec = rec;
    int blocks = (int)std::min<int64_t>((nnz + 255) / 256, 8192);
    if (rw == 4)
        hipLaunchKernelGGL(pack_records_kernel<4>, dim3(blocks), dim3(256), 0,
                           s, a);
    else
        hipLaunchKernelGGL(pack_records_kernel<8>, dim3(blocks), dim3(256), 0,
                           s, a);
    return hipGetLastError();
}

struct PermuteArgs {
    const uint32_t *rec;
    int32_t *pidx[kMaxOrder];
    float *pval;
    const uint32_t *perm;
    int64_t nnz;
    int N;
};

template <int RW>
__global__ void permute_kernel(PermuteArgs a) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < a.nnz;
         p += stride) {
        const uint4 *src =
            reinterpret_cast<const uint4 *>(a.rec + (int64_t)a.perm[p] * RW);
        uint32_t w[RW];
#pragma unroll
        for (int k = 0; k < RW; k += 4) {
            const uint4 v = src[k / 4];
            w[k] = v.x;
            w[k + 1] = v.y;
            w[k + 2] = v.z;
            w[k + 3] = v.w;
        }
#pragma unroll
        for (int n = 0; n < kMaxOrder; ++n)
            if (n < a.N) a.pidx[n][p] = (int32_t)w[n];
        a.pval[p] = __uint_as_float(w[RW - 1]);
    }
}

hipError_t launch_permute(int N, const uint32_t *rec, int rw,
                          const uint32_t *perm, int64_t nnz,
                          int32_t *const *pidx, float *pval, hipStream_t s) {
    PermuteArgs a{};
    for (int n = 0; n < N; ++n) a.pidx[n] = pidx[n];
    a.rec = rec;
    a.pval = pval;
    a.perm = perm;
    a.nnz = nnz;
    a.N = N;
    int blocks = (int)std::min<int64_t>((nnz + 255) / 256, 8192);
    if (rw == 4)
        hipLaunchKernelGGL(permute_kernel<4>, dim3(blocks), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL(permute_kernel<8>, dim3(blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

// ------------------------------------------------------------------ sort
// Tile t of mode n covers elements [b*M + tb*kSortTile, ...) of segment b.
struct TileInfo {
    int64_t seg_start;
    int seg_len;
    int tile_off;     // offset of the tile inside its segment
    int tile_len;     // 0 for a tile past the end of a short last segment
    int tiles_in_seg;
};

__device__ __forceinline__ TileInfo tile_info(const SortPass &p, int b,
                                              int tb) {
    TileInfo t;
    t.seg_start = (int64_t)b * p.M;
    int64_t rem = p.nnz - t.seg_start;
    t.seg_len = (int)(rem < p.M ? rem : p.M);
    t.tiles_in_seg = (t.seg_len + kSortTile - 1) / kSortTile;
    t.tile_off = tb * kSortTile;
    int left = t.seg_len - t.tile_off;
    t.tile_len = left <= 0 ? 0 : (left < kSortTile ? left : kSortTile);
    return t;
}

__device__ __forceinline__ uint32_t *counts_at(const SortPass &p, int n, int b,
                                               int d) {
    return p.counts +
           (((int64_t)n * p.nseg + b) * kRadix + d) * p.tiles_per_seg;
}

// grid: (tiles_per_seg, nseg, N)
__global__ __launch_bounds__(kSortThreads) void sort_upsweep_kernel(SortPass p) {
    const int tb = blockIdx.x, b = blockIdx.y, n = blockIdx.z;
    TileInfo t = tile_info(p, b, tb);
    if (t.tile_len == 0) return;
    __shared__ uint32_t hist[kRadix];
    hist[threadIdx.x] = 0;
    __syncthreads();
    const uint32_t *keys = p.key_in[n] + t.seg_start + t.tile_off;
    for (int i = threadIdx.x; i < t.tile_len; i += kSortThreads)
        atomicAdd(&hist[(keys[i] >> p.shift) & (kRadix - 1)], 1u);
    __syncthreads();
    counts_at(p, n, b, threadIdx.x)[tb] = hist[threadIdx.x];
}

// grid: (nseg, N). Exclusive scan of a segment's counts in (digit, tile)
// order: the start of every (digit, tile) run in the sorted segment.
__global__ __launch_bounds__(kSortThreads) void sort_scan_kernel(SortPass p) {
    const int b = blockIdx.x, n = blockIdx.y, d = threadIdx.x;
    TileInfo t = tile_info(p, b, 0);
    uint32_t *c = counts_at(p, n, b, d);
    uint32_t total = 0;
    for (int tb = 0; tb < t.tiles_in_seg; ++tb) total += c[tb];
    __shared__ uint32_t s[kRadix];
    s[d] = total;
    __syncthreads();
    // Hillis-Steele inclusive scan over the 256 digit totals
    for (int off = 1; off < kRadix; off <<= 1) {
        uint32_t v = d >= off ? s[d - off] : 0u;
        __syncthreads();
        s[d] += v;
        __syncthreads();
    }
    uint32_t run = s[d] - total;
    for (int tb = 0; tb < t.tiles_in_seg; ++tb) {
        uint32_t k = c[tb];
        c[tb] = run;
        run += k;
    }
}

// grid: (tiles_per_seg, nseg, N). Stable scatter, staged in LDS: the tile is
// first ordered by digit locally (the rank of an element among equal digits
// is the number of equal digits before it in the tile, taken round by round
// -- 256 consecutive elements per round -- from wave match masks and per-wave
// counts), then written out so that consecutive threads store consecutive
// positions of one digit's run.
__global__ __launch_bounds__(kSortThreads) void sort_downsweep_kernel(
    SortPass p) {
    const int tb = blockIdx.x, b = blockIdx.y, n = blockIdx.z;
    TileInfo t = tile_info(p, b, tb);
    if (t.tile_len == 0) return;
    __shared__ uint32_t base[kRadix];     // global start of digit d (this tile)
    __shared__ uint32_t lstart[kRadix];   // local start of digit d
    __shared__ uint32_t run[kRadix];      // digit d elements placed so far
    __shared__ uint32_t wcnt[kSortThreads / 64][kRadix];
    __shared__ uint32_t skey[kSortTile];
    __shared__ uint32_t sval[kSortTile];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const uint32_t *keys = p.key_in[n] + t.seg_start + t.tile_off;
    const uint32_t *vals =
        p.val_in[n] ? p.val_in[n] + t.seg_start + t.tile_off : nullptr;
    uint32_t *kout = p.key_out[n] + t.seg_start;
    uint32_t *vout = p.val_out[n] + t.seg_start;

    uint32_t key[kSortRounds], val[kSortRounds];
    base[tid] = counts_at(p, n, b, tid)[tb];
    run[tid] = 0;
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kSortRounds; ++r) {
        const int i = r * kSortThreads + tid;
        const bool valid = i < t.tile_len;
        key[r] = valid ? keys[i] : 0u;
        val[r] = valid ? (vals ? vals[i] : (uint32_t)(t.tile_off + i)) : 0u;
        if (valid) atomicAdd(&run[(key[r] >> p.shift) & (kRadix - 1)], 1u);
    }
    __syncthreads();
    // exclusive scan of the tile histogram (Hillis-Steele over 256 digits)
    const uint32_t cnt = run[tid];
    lstart[tid] = cnt;
    __syncthreads();
    for (int off = 1; off < kRadix; off <<= 1) {
        const uint32_t v = tid >= off ? lstart[tid - off] : 0u;
        __syncthreads();
        lstart[tid] += v;
        __syncthreads();
    }
    lstart[tid] -= cnt;
    run[tid] = 0;
    __syncthreads();

#pragma unroll
    for (int r = 0; r < kSortRounds; ++r) {
        const int i = r * kSortThreads + tid;
        const bool valid = i < t.tile_len;
        const uint32_t dig = (key[r] >> p.shift) & (kRadix - 1);
        for (int w = 0; w < kSortThreads / 64; ++w) wcnt[w][tid] = 0;
        __syncthreads();
        uint64_t peers = __ballot(valid);
        if (!valid) peers = ~peers;
#pragma unroll
        for (int bit = 0; bit < 8; ++bit) {
            const uint64_t bb = __ballot((dig >> bit) & 1u);
            peers &= ((dig >> bit) & 1u) ? bb : ~bb;
        }
        const uint32_t rank = __popcll(peers & lt);
        if (valid && rank == 0) wcnt[wave][dig] = __popcll(peers);
        __syncthreads();
        if (valid) {
            uint32_t before = 0;
            for (int w = 0; w < wave; ++w) before += wcnt[w][dig];
            const uint32_t dst = lstart[dig] + run[dig] + before + rank;
            skey[dst] = key[r];
            sval[dst] = val[r];
        }
        __syncthreads();
        uint32_t add = 0;
        for (int w = 0; w < kSortThreads / 64; ++w) add += wcnt[w][tid];
        run[tid] += add;
        __syncthreads();
    }
    for (int k = tid; k < t.tile_len; k += kSortThreads) {
        const uint32_t kk = skey[k];
        const uint32_t d = (kk >> p.shift) & (kRadix - 1);
        const uint32_t dst = base[d] + (uint32_t)k - lstart[d];
        kout[dst] = kk;
        vout[dst] = sval[k];
    }
}

// ------------------------------------------------------------------ crossings
// One thread per chunk edge q = k * kSegChunk (k >= 1) of every minibatch and
// mode: if the row at q also occupies q - 1 and q is the first edge its
// segment crosses, record (first, end) of the segment. The list order is
// arbitrary; every entry is reduced independently.
__global__ void crossing_segments_kernel(CrossArgs c) {
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t per_seg = (int64_t)c.N * c.xcap;
    if (tid >= (int64_t)c.nseg * per_seg) return;
    const int b = (int)(tid / per_seg);
    const int n = (int)((tid % per_seg) / c.xcap);
    const int k = (int)(tid % c.xcap) + 1;
    const int64_t off = (int64_t)b * c.M;
    const int64_t rem = c.nnz - off;
    const int m = (int)(rem < c.M ? rem : c.M);
    const int q = k * kSegChunk;
    if (q >= m) return;
    const uint32_t *r = c.rows[n] + off;
    const uint32_t row = r[q];
    if (r[q - 1] != row) return;
    int lo = 0, hi = q;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (r[mid] < row) lo = mid + 1; else hi = mid;
    }
    const int first = lo;
    if ((first / kSegChunk + 1) * kSegChunk != q) return;
    lo = q;
    hi = m;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (r[mid] <= row) lo = mid + 1; else hi = mid;
    }
    const int slot = atomicAdd(&c.xcount[b * c.N + n], 1);
    c.xlist[((int64_t)b * c.N + n) * c.xcap + slot] = make_int2(first, lo);
}

hipError_t launch_crossing_segments(const CrossArgs &c, hipStream_t s) {
    const int64_t counts = (int64_t)c.nseg * c.N;
    hipError_t e = launch_fill_zero(reinterpret_cast<float *>(c.xcount),
                                    counts, s);
    if (e != hipSuccess) return e;
    const int64_t threads = counts * c.xcap;
    hipLaunchKernelGGL(crossing_segments_kernel,
                       dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s,
                       c);
    return hipGetLastError();
}

hipError_t launch_sort_pass(const SortPass &p, hipStream_t s) {
    dim3 g3(p.tiles_per_seg, p.nseg, p.N);
    hipLaunchKernelGGL(sort_upsweep_kernel, g3, dim3(kSortThreads), 0, s, p);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(sort_scan_kernel, dim3(p.nseg, p.N), dim3(kSortThreads),
                       0, s, p);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(sort_downsweep_kernel, g3, dim3(kSortThreads), 0, s, p);
    return hipGetLastError();
}

}  // namespace ft
