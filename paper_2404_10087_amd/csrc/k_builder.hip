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
// Counter-based permutation of [0, n): a 4-round Feistel network on the
// mixed-radix domain Z_a x Z_b with a = ceil(sqrt n), b = ceil(n / a)
// (Black & Rogaway, 2002, generalised Feistel): x = L b + R; a round maps
// (L in Z_p, R in Z_q) to (R, (L + F_i(R)) mod p), so the halves swap moduli
// and after four rounds the pair is back in Z_a x Z_b. F_i(R) is the
// MurmurHash3 32-bit finaliser (Appleby) of R ^ k_i, scaled into [0, p) by a
// 32x32 -> 64-bit product. Values in [n, ab) are cycle-walked; since
// ab - n < a the walk almost never runs, so the lanes of a wave stay
// converged. Round keys are the high halves of consecutive SplitMix64
// outputs (Steele, Lea & Flood, 2014) from `key`. All arithmetic is 32-bit.
__device__ __forceinline__ uint32_t fmix32(uint32_t h) {
    h ^= h >> 16;
    h *= 0x85ebca6bu;
    h ^= h >> 13;
    h *= 0xc2b2ae35u;
    h ^= h >> 16;
    return h;
}

struct Feistel {
    uint32_t k[4];
    uint32_t a, b;
};

__device__ __forceinline__ uint32_t feistel_enc(uint32_t x, const Feistel &f) {
    uint32_t L = x / f.b, R = x - L * f.b;
    uint32_t p = f.a, q = f.b;            // L in Z_p, R in Z_q
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const uint32_t fr = __umulhi(fmix32(R ^ f.k[i]), p);
        uint32_t t = L + fr;
        if (t >= p) t -= p;
        L = R;
        R = t;
        const uint32_t s = p;
        p = q;
        q = s;
    }
    return L * f.b + R;
}

__global__ void epoch_order_kernel(uint32_t *perm, uint32_t n, Feistel f) {
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t p = blockIdx.x * blockDim.x + threadIdx.x; p < n;
         p += stride) {
        uint32_t x = feistel_enc(p, f);
        while (x >= n) x = feistel_enc(x, f);
        perm[p] = x;
    }
}

static uint64_t host_mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

hipError_t launch_epoch_order(uint32_t *perm, int64_t n, uint64_t key,
                              hipStream_t s, int grid_cap) {
    if (n < 1 || n > 0x7fffffffll) return hipErrorInvalidValue;
    Feistel f;
    uint64_t st = key;
    for (int i = 0; i < 4; ++i) {
        st += 0x9e3779b97f4a7c15ull;
        f.k[i] = (uint32_t)(host_mix64(st) >> 32);
    }
    uint64_t a = 1;
    while (a * a < (uint64_t)n) ++a;
    f.a = (uint32_t)a;
    f.b = (uint32_t)((n + a - 1) / a);
    int blocks = (int)((n + 255) / 256);
    if (blocks > 8192) blocks = 8192;
    if (grid_cap > 0 && blocks > grid_cap) blocks = grid_cap;
    hipLaunchKernelGGL(epoch_order_kernel, dim3(blocks), dim3(256), 0, s, perm,
                       (uint32_t)n, f);
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
// (RW = 4 for order <= 3, 8 up to order 7, 16 above), so the random gather of
// one sample is one 16-, 32- or 64-byte load: pidx[n][p] = rec[perm[p]].i_n,
// pval[p] = .x.
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
    else if (rw == 8)
        hipLaunchKernelGGL(pack_records_kernel<8>, dim3(blocks), dim3(256), 0,
                           s, a);
    else
        hipLaunchKernelGGL(pack_records_kernel<16>, dim3(blocks), dim3(256),
                           0, s, a);
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
        constexpr int NW = RW - 1 < kMaxOrder ? RW - 1 : kMaxOrder;
#pragma unroll
        for (int n = 0; n < NW; ++n)
            if (n < a.N) a.pidx[n][p] = (int32_t)w[n];
        a.pval[p] = __uint_as_float(w[RW - 1]);
    }
}

hipError_t launch_permute(int N, const uint32_t *rec, int rw,
                          const uint32_t *perm, int64_t nnz,
                          int32_t *const *pidx, float *pval, hipStream_t s,
                          int grid_cap) {
    PermuteArgs a{};
    for (int n = 0; n < N; ++n) a.pidx[n] = pidx[n];
    a.rec = rec;
    a.pval = pval;
    a.perm = perm;
    a.nnz = nnz;
    a.N = N;
    int blocks = (int)std::min<int64_t>((nnz + 255) / 256, 8192);
    if (grid_cap > 0 && blocks > grid_cap) blocks = grid_cap;
    if (rw == 4)
        hipLaunchKernelGGL(permute_kernel<4>, dim3(blocks), dim3(256), 0, s, a);
    else if (rw == 8)
        hipLaunchKernelGGL(permute_kernel<8>, dim3(blocks), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL(permute_kernel<16>, dim3(blocks), dim3(256), 0, s,
                           a);
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

// XCD-aware tile mapping: workgroups are dealt to the 8 XCDs round-robin by
// their linear id, so linear id L runs on XCD L % 8. All tiles of one
// (mode, minibatch) segment are given ids with the same residue, so a
// segment's scattered output (digit runs, and in the final pass the inverse
// positions) is assembled in one L2 before it is written back. Returns false
// for the surplus ids of the last group.
constexpr int kXcds = 8;

__device__ __forceinline__ bool sort_tile_of(const SortPass &p, int L, int &tb,
                                             int &b, int &n) {
    const int slot = L / kXcds;
    const int sn = (slot / p.tiles_per_seg) * kXcds + L % kXcds;
    if (sn >= p.nseg * p.N) return false;
    tb = slot % p.tiles_per_seg;
    n = sn / p.nseg;
    b = sn % p.nseg;
    return true;
}

__host__ __device__ inline int sort_grid(const SortPass &p) {
    const int groups = (p.nseg * p.N + kXcds - 1) / kXcds;
    return groups * kXcds * p.tiles_per_seg;
}

// counts of tile tb of segment b, mode n: kRadix consecutive words (tb =
// tiles_per_seg: the segment's digit starts)
__device__ __forceinline__ uint32_t *counts_at(const SortPass &p, int n, int b,
                                               int tb) {
    return p.counts +
           (((int64_t)n * p.nseg + b) * (p.tiles_per_seg + 1) + tb) * kRadix;
}

// Digit histogram of tile id L (sort_tile_of); every wave counts into its
// own LDS histogram so hot rows contend only within a wave.
__device__ __forceinline__ void upsweep_tile(const SortPass &p, int L) {
    int tb, b, n;
    if (!sort_tile_of(p, L, tb, b, n)) return;
    TileInfo t = tile_info(p, b, tb);
    if (t.tile_len == 0) return;
    constexpr int W = kSortThreads / 64;
    __shared__ uint32_t hist[W][kRadix];
    for (int w = 0; w < W; ++w) hist[w][threadIdx.x] = 0;
    __syncthreads();
    const uint32_t *keys = p.key_in[n] + t.seg_start + t.tile_off;
    uint32_t *mine = hist[threadIdx.x >> 6];
    uint32_t k[kSortRounds];
#pragma unroll
    for (int r = 0; r < kSortRounds; ++r) {
        const int i = r * kSortThreads + threadIdx.x;
        k[r] = i < t.tile_len ? keys[i] : 0u;
    }
#pragma unroll
    for (int r = 0; r < kSortRounds; ++r)
        if (r * kSortThreads + (int)threadIdx.x < t.tile_len)
            atomicAdd(&mine[(k[r] >> p.shift) & (kRadix - 1)], 1u);
    __syncthreads();
    uint32_t c = 0;
    for (int w = 0; w < W; ++w) c += hist[w][threadIdx.x];
    counts_at(p, n, b, tb)[threadIdx.x] = c;
}

// Tile ids blockIdx.x, blockIdx.x + gridDim.x, ... (gridDim.x a multiple of
// kXcds keeps every id on its block's XCD).
__global__ __launch_bounds__(kSortThreads) void sort_upsweep_kernel(SortPass p) {
    const int total = sort_grid(p);
    for (int L = blockIdx.x; L < total; L += gridDim.x) {
        upsweep_tile(p, L);
        __syncthreads();
    }
}

// Offsets of every (mode, segment) of the pass, one block each: thread d
// replaces the upsweep's count of digit d in every tile by the count in the
// tiles before it (an exclusive scan over the tiles, eight loads in flight),
// and the segment's totals are scanned over the digits into its digit
// starts. The downsweep then reads two words per digit instead of a column
// of counts per tile.
__global__ __launch_bounds__(kSortThreads) void sort_scan_kernel(SortPass p) {
    __shared__ uint32_t sc[kRadix];
    const int tid = threadIdx.x;
    for (int sb = blockIdx.x; sb < p.N * p.nseg; sb += gridDim.x) {
        const int n = sb / p.nseg, b = sb % p.nseg;
        const TileInfo t = tile_info(p, b, 0);
        uint32_t *c = counts_at(p, n, b, 0) + tid;
        uint32_t run = 0;
        int k = 0;
        for (; k + 8 <= t.tiles_in_seg; k += 8) {
            uint32_t v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = c[(int64_t)(k + u) * kRadix];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                c[(int64_t)(k + u) * kRadix] = run;
                run += v[u];
            }
        }
        for (; k < t.tiles_in_seg; ++k) {
            const uint32_t v = c[(int64_t)k * kRadix];
            c[(int64_t)k * kRadix] = run;
            run += v;
        }
        sc[tid] = run;
        __syncthreads();
        for (int off = 1; off < kRadix; off <<= 1) {
            const uint32_t v = tid >= off ? sc[tid - off] : 0u;
            __syncthreads();
            sc[tid] += v;
            __syncthreads();
        }
        counts_at(p, n, b, p.tiles_per_seg)[tid] = sc[tid] - run;
        __syncthreads();
    }
}

// Stable scatter of tile id L (sort_tile_of), staged in LDS. The global
// start of digit d for this tile is the segment's start of d plus the count
// of d in the tiles before this one (both from the scan kernel). The tile
// is then ordered by digit
// locally (the rank of an element among equal digits
// is the number of equal digits before it in the tile, taken round by round
// -- 256 consecutive elements per round -- from wave match masks and per-wave
// counts), then written out so that consecutive threads store consecutive
// positions of one digit's run. The final pass also records, for every
// in-minibatch position, its sorted index (the factor kernel writes each
// sample's gradient rows straight to their sorted slots).
__device__ __forceinline__ void downsweep_tile(const SortPass &p, int L) {
    int tb, b, n;
    if (!sort_tile_of(p, L, tb, b, n)) return;
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
    uint32_t *vout = p.val_out[n] ? p.val_out[n] + t.seg_start : nullptr;

    uint32_t key[kSortRounds], val[kSortRounds];
    base[tid] = counts_at(p, n, b, p.tiles_per_seg)[tid] +
                counts_at(p, n, b, tb)[tid];
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
    uint32_t *inv = p.inv_out[n] ? p.inv_out[n] + t.seg_start : nullptr;
    for (int k = tid; k < t.tile_len; k += kSortThreads) {
        const uint32_t kk = skey[k];
        const uint32_t d = (kk >> p.shift) & (kRadix - 1);
        const uint32_t dst = base[d] + (uint32_t)k - lstart[d];
        kout[dst] = kk;
        if (vout) vout[dst] = sval[k];
        if (inv) inv[sval[k]] = dst;
    }
}

__global__ __launch_bounds__(kSortThreads) void sort_downsweep_kernel(
    SortPass p) {
    const int total = sort_grid(p);
    for (int L = blockIdx.x; L < total; L += gridDim.x) {
        downsweep_tile(p, L);
        __syncthreads();
    }
}

// ------------------------------------------------------------------ crossings
// One block per minibatch and mode, one thread per chunk edge q = k kSegChunk
// (k = 1 .. xcap, in rounds of kCrossThreads edges). A thread whose edge is
// the first one its row crosses (the row occupies q - 1 and q but not
// q - kSegChunk - 1) finds the row's first sample in the chunk before q and
// its end by a galloping search, and lists (first, end, row). Rows of at
// most kSmallCross samples are listed from the front of the minibatch's
// list, longer ones from the back together with their first part, and every
// long row is cut into parts of part_rows(J4) samples listed in plist. Each
// class is in edge order: slots and part offsets come from block scans
// (wave ballots and shuffle scans, then wave totals in LDS), so no atomics
// and the lists are the same on every run.
// 256 threads: the list is built beside the core kernel, whose blocks leave
// room for four-wave workgroups but not for sixteen-wave ones
constexpr int kCrossThreads = 256;

__device__ __forceinline__ void crossing_one(const CrossArgs &c, int b,
                                             int n) {
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    constexpr int W = kCrossThreads / 64;
    __shared__ int wtot[4][W];
    const int64_t off = (int64_t)b * c.M;
    const int64_t rem = c.nnz - off;
    const int m = (int)(rem < c.M ? rem : c.M);
    const uint32_t *r = c.rows[n] + off;
    int4 *list = c.xlist + ((int64_t)b * c.N + n) * c.xcap;
    int4 *plist = c.plist + ((int64_t)b * c.N + n) * c.pcap;
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    int nsmall = 0, nlarge = 0, nparts = 0, nmulti = 0;
    for (int k0 = 1; k0 <= c.xcap; k0 += kCrossThreads) {
        const int k = k0 + t;
        const int q = k * kSegChunk;
        bool flag = false;
        int first = 0, end = 0;
        uint32_t row = 0;
        if (k <= c.xcap && q < m) {
            row = r[q];
            flag = r[q - 1] == row &&
                   !(q > kSegChunk && r[q - kSegChunk - 1] == row);
            if (flag) {
                int lo = q - kSegChunk, hi = q;
                while (lo < hi) {
                    const int mid = (lo + hi) >> 1;
                    if (r[mid] < row) lo = mid + 1; else hi = mid;
                }
                first = lo;
                int step = kSegChunk, probe = q;
                while (probe + step < m && r[probe + step] == row) {
                    probe += step;
                    step <<= 1;
                }
                lo = probe + 1;
                hi = probe + step < m ? probe + step : m;
                while (lo < hi) {
                    const int mid = (lo + hi) >> 1;
                    if (r[mid] == row) lo = mid + 1; else hi = mid;
                }
                end = lo;
            }
        }
        const bool small = flag && end - first <= kSmallCross;
        const bool large = flag && !small;
        const int cnt = end - first;
        const int prows = part_rows(c.J4);
        const int parts = !large ? 0
                          : (cnt > split_rows(c.J4) ? (cnt + prows - 1) / prows
                                                    : 1);
        // inclusive scan of the part counts over the wave
        int pincl = parts;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const int y = __shfl_up(pincl, d);
            if (lane >= d) pincl += y;
        }
        const uint64_t bs = __ballot(small), bl = __ballot(large);
        const uint64_t bm = __ballot(parts > 1);
        if (lane == 63) wtot[2][w] = pincl;
        if (lane == 0) {
            wtot[0][w] = __popcll(bs);
            wtot[1][w] = __popcll(bl);
            wtot[3][w] = __popcll(bm);
        }
        __syncthreads();
        int ps = nsmall, pl = nlarge, pp = nparts;
        for (int v = 0; v < w; ++v) {
            ps += wtot[0][v];
            pl += wtot[1][v];
            pp += wtot[2][v];
        }
        if (small) list[ps + __popcll(bs & lt)] = make_int4(first, end, (int)row, 0);
        if (large) {
            const int p0 = pp + pincl - parts;
            list[c.xcap - 1 - (pl + __popcll(bl & lt))] =
                make_int4(first, end, (int)row, p0);
            const int span = parts == 1 ? cnt : prows;   // whole row
            for (int j = 0; j < parts; ++j) {
                const int f = first + j * span;
                const int e = f + span < end ? f + span : end;
                plist[p0 + j] = make_int4(f, e, (int)row, parts);
            }
        }
        for (int v = 0; v < W; ++v) {
            nsmall += wtot[0][v];
            nlarge += wtot[1][v];
            nparts += wtot[2][v];
            nmulti += wtot[3][v];
        }
        __syncthreads();
    }
    if (t == 0) {
        int32_t *xc = c.xcount + (int64_t)(b * c.N + n) * kXCounts;
        xc[0] = nsmall;
        xc[1] = nlarge;
        xc[2] = nparts;
        xc[3] = nmulti;
    }
}

// (minibatch, mode) pairs blockIdx.x, blockIdx.x + gridDim.x, ...
__global__ __launch_bounds__(kCrossThreads) void crossing_segments_kernel(
    CrossArgs c) {
    for (int id = blockIdx.x; id < c.nseg * c.N; id += gridDim.x) {
        crossing_one(c, id / c.N, id % c.N);
        __syncthreads();
    }
}

hipError_t launch_crossing_segments(const CrossArgs &c, hipStream_t s) {
    int blocks = c.nseg * c.N;
    if (c.grid_cap > 0 && blocks > c.grid_cap) blocks = c.grid_cap;
    hipLaunchKernelGGL(crossing_segments_kernel, dim3(blocks),
                       dim3(kCrossThreads), 0, s, c);
    return hipGetLastError();
}

hipError_t launch_sort_pass(const SortPass &p, hipStream_t s) {
    int grid = sort_grid(p);
    if (p.grid_cap > 0 && grid > p.grid_cap)
        grid = (p.grid_cap + kXcds - 1) / kXcds * kXcds;
    dim3 g3(grid);
    hipLaunchKernelGGL(sort_upsweep_kernel, g3, dim3(kSortThreads), 0, s, p);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    int sgrid = p.N * p.nseg;
    if (p.grid_cap > 0 && sgrid > p.grid_cap) sgrid = p.grid_cap;
    hipLaunchKernelGGL(sort_scan_kernel, dim3(sgrid), dim3(kSortThreads), 0, s,
                       p);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(sort_downsweep_kernel, g3, dim3(kSortThreads), 0, s, p);
    return hipGetLastError();
}

}  // namespace ft
