// ft_api.cpp -- host runtime of the sparse FastTucker library: argument
// validation, device memory, the epoch schedule and the C ABI of ft.h.
//
// Every entry point validates its arguments before touching the device, so
// the boundary behaves the same on a host without a GPU (FT_EINVAL for bad
// arguments, FT_EDEVICE when a valid call needs a device that is absent).
#include "../../include/ft.h"
#include "ft_internal.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

using namespace ft;

namespace ft {
thread_local ExtEvents g_ext_events;
}

namespace {
thread_local std::string g_create_error = "no error";

struct Pending {
    int kind;
    hipEvent_t a, b;
};
}  // namespace

// Everything the builder makes for one epoch order.
struct EpochBufs {
    uint32_t *perm = nullptr;
    int32_t *pidx[kMaxOrder] = {};
    float *pval = nullptr;
    uint32_t *sk[2][kMaxOrder] = {};
    uint32_t *sv[2][kMaxOrder] = {};
    uint32_t *inv[kMaxOrder] = {};    // sorted index of every position
    uint32_t *counts = nullptr;
    size_t counts_cap = 0;
    int sort_final[kMaxOrder] = {};   // ping-pong set holding each mode's
                                      // sorted rows
    int4 *xlist = nullptr;            // crossing rows per minibatch and mode
    size_t xlist_cap = 0;
    int4 *plist = nullptr;            // their parts of kPartRows samples
    size_t plist_cap = 0;
    int32_t *xcount = nullptr;        // kXCounts per minibatch and mode
    size_t xcount_cap = 0;
    int xcap = 1;
    int pcap = 1;
    int32_t *xcount_host = nullptr;   // pinned copy of xcount
    size_t xcount_host_cap = 0;
    hipEvent_t ready = nullptr;       // recorded after the last builder step
    bool pending = false;             // xcount_host not yet waited for
    // what the set holds (valid: built for this epoch, M, seed, training set)
    bool valid = false;
    uint64_t epoch = 0, seed = 0, gen = 0;
    int64_t M = 0;
};

struct ft_handle {
    int device = 0;
    hipStream_t stream = nullptr;
    int N = 0;
    int64_t dims[kMaxOrder] = {};
    int32_t J[kMaxOrder] = {};
    int32_t R = 0;
    Shape sh{};
    ft_options opt{};
    std::string err = "no error";

    float *A[kMaxOrder] = {};
    float *B[kMaxOrder] = {};
    uint16_t *A16[kMaxOrder] = {};   // BF16 shadow (precision FT_BF16)
    uint8_t *A8[kMaxOrder] = {};     // FP8 shadow and per-row scales
    float *As[kMaxOrder] = {};       // (precision FT_FP8_E4M3)

    int64_t nnz[2] = {0, 0};
    int32_t *idx[2][kMaxOrder] = {};
    float *val[2] = {};

    // epoch state: two builder buffer sets, the current epoch's and the
    // next one's (built ahead on bstream)
    uint64_t epoch = 0;
    bool use_user_perm = false;
    uint32_t *user_perm = nullptr;
    uint32_t *rec = nullptr;          // training records (record_words(N) words)
    uint64_t train_gen = 0;           // bumped by every new training set
    EpochBufs eb[2];
    int cur = 0;
    hipStream_t bstream = nullptr;    // builder-ahead stream (default priority)
    bool prepared = false;
    int64_t prepared_M = 0;

    // factor-phase scratch
    float *G = nullptr;
    size_t G_cap = 0;
    float *P = nullptr;               // part sums of long rows
    size_t P_cap = 0;
    double *mb_part = nullptr;
    size_t mb_part_cap = 0;
    double *mb_loss = nullptr;
    size_t mb_loss_cap = 0;
    double *tile_loss = nullptr;
    size_t tile_loss_cap = 0;

    // core-phase / evaluation scratch
    float *Cst[kMaxOrder] = {};       // stored C^(n) (core_storage)
    float *core_part = nullptr;
    size_t core_part_cap = 0;
    double *dpart = nullptr;
    size_t dpart_cap = 0;
    double *scal = nullptr;   // 64 doubles

    // profiling
    bool prof = false;
    std::vector<Pending> pending;
    std::vector<hipEvent_t> pool;
    int64_t launches[FT_K_COUNT] = {};
    double ms[FT_K_COUNT] = {};
};

// ------------------------------------------------------------------ helpers
static ft_status fail(ft_handle *h, ft_status code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (h) h->err = buf; else g_create_error = buf;
    return code;
}

#define HIPCHK(h, expr)                                                      \
    do {                                                                     \
        hipError_t e_ = (expr);                                              \
        if (e_ != hipSuccess)                                                \
            return fail((h),                                                 \
                        e_ == hipErrorOutOfMemory ? FT_ENOMEM : FT_EDEVICE,  \
                        "%s failed: %s", #expr, hipGetErrorString(e_));      \
    } while (0)

#define CHECK_HANDLE(h)                                                      \
    do {                                                                     \
        if (!(h)) return fail(nullptr, FT_EINVAL, "handle is NULL");         \
    } while (0)

template <typename T>
static hipError_t ensure(T **p, size_t *cap, size_t count) {
    if (count <= *cap && *p) return hipSuccess;
    if (*p) (void)hipFree(*p);
    *p = nullptr;
    *cap = 0;
    hipError_t e = hipMalloc((void **)p, sizeof(T) * (count ? count : 1));
    if (e == hipSuccess) *cap = count;
    return e;
}

static void dfree(void *p) {
    if (p) (void)hipFree(p);
}

static ft_status alloc_epoch_bufs(ft_handle *h, EpochBufs &E);

static void free_epoch_bufs(EpochBufs &E) {
    dfree(E.perm);
    dfree(E.pval);
    for (int n = 0; n < kMaxOrder; ++n) {
        dfree(E.pidx[n]);
        dfree(E.inv[n]);
        for (int s = 0; s < 2; ++s) {
            dfree(E.sk[s][n]);
            dfree(E.sv[s][n]);
        }
    }
    dfree(E.counts);
    dfree(E.xlist);
    dfree(E.plist);
    dfree(E.xcount);
    if (E.xcount_host) (void)hipHostFree(E.xcount_host);
    if (E.ready) (void)hipEventDestroy(E.ready);
    E = EpochBufs{};
}

static int64_t nminibatches(const ft_handle *h) {
    return (h->nnz[FT_TRAIN] + h->opt.minibatch - 1) / h->opt.minibatch;
}

static hipEvent_t pool_event(ft_handle *h) {
    hipEvent_t e = nullptr;
    if (h->pool.empty()) {
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
    } else {
        e = h->pool.back();
        h->pool.pop_back();
    }
    return e;
}

// Bracketing form (several kernels in one class): markers on the stream.
static void prof_begin(ft_handle *h, int kind, hipStream_t s) {
    if (!h->prof) return;
    hipEvent_t a = pool_event(h);
    if (!a) return;
    (void)hipEventRecord(a, s);
    h->pending.push_back({kind, a, nullptr});
}

static void prof_end(ft_handle *h, hipStream_t s) {
    if (!h->prof || h->pending.empty() || h->pending.back().b) return;
    hipEvent_t b = pool_event(h);
    if (!b) return;
    (void)hipEventRecord(b, s);
    h->pending.back().b = b;
}

// Single-kernel form: the launch itself records the two events.
static void prof_ext(ft_handle *h, int kind) {
    g_ext_events = ExtEvents{};
    if (!h->prof) return;
    hipEvent_t a = pool_event(h), b = pool_event(h);
    if (!a || !b) return;
    h->pending.push_back({kind, a, b});
    g_ext_events.start = a;
    g_ext_events.stop = b;
}

static ft_status prof_collect(ft_handle *h) {
    if (h->pending.empty()) return FT_OK;
    HIPCHK(h, hipStreamSynchronize(h->stream));
    if (h->bstream) HIPCHK(h, hipStreamSynchronize(h->bstream));
    for (auto &p : h->pending) {
        if (p.b) {
            float t = 0.f;
            if (hipEventElapsedTime(&t, p.a, p.b) == hipSuccess) {
                h->launches[p.kind] += 1;
                h->ms[p.kind] += t;
            }
            h->pool.push_back(p.b);
        }
        h->pool.push_back(p.a);
    }
    h->pending.clear();
    return FT_OK;
}

struct Launch {
    ft_handle *h;
    hipStream_t s;
    Launch(ft_handle *hh, int kind) : h(hh), s(hh->stream) { prof_begin(h, kind, s); }
    Launch(ft_handle *hh, int kind, hipStream_t ss) : h(hh), s(ss) {
        prof_begin(h, kind, s);
    }
    ~Launch() { prof_end(h, s); }
};

struct LaunchExt {
    LaunchExt(ft_handle *h, int kind) { prof_ext(h, kind); }
    ~LaunchExt() { g_ext_events = ExtEvents{}; }
};

// SplitMix64 (Steele, Lea & Flood, 2014) and the Box-Muller transform for the
// seeded initial parameters.
static uint64_t splitmix64(uint64_t &s) {
    uint64_t z = (s += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

static double normal01(uint64_t &s) {
    const double u1 = 1.0 - (double)(splitmix64(s) >> 11) * 0x1.0p-53;
    const double u2 = (double)(splitmix64(s) >> 11) * 0x1.0p-53;
    return std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2);
}

static ft_status upload_padded(ft_handle *h, float *dst, const float *src,
                               int64_t rows, int cols, int ld) {
    HIPCHK(h, hipMemcpy2DAsync(dst, sizeof(float) * ld, src,
                               sizeof(float) * cols, sizeof(float) * cols, rows,
                               hipMemcpyHostToDevice, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    return FT_OK;
}

static ft_status download_padded(ft_handle *h, float *dst, const float *src,
                                 int64_t rows, int cols, int ld) {
    HIPCHK(h, hipMemcpy2DAsync(dst, sizeof(float) * cols, src,
                               sizeof(float) * ld, sizeof(float) * cols, rows,
                               hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    return FT_OK;
}

static void release(ft_handle *h) {
    for (int n = 0; n < kMaxOrder; ++n) {
        dfree(h->A[n]);
        dfree(h->B[n]);
        dfree(h->A16[n]);
        dfree(h->A8[n]);
        dfree(h->As[n]);
        dfree(h->Cst[n]);

        for (int s = 0; s < 2; ++s) dfree(h->idx[s][n]);
    }
    if (h->bstream) (void)hipStreamSynchronize(h->bstream);
    for (auto &E : h->eb) free_epoch_bufs(E);
    if (h->bstream) (void)hipStreamDestroy(h->bstream);
    dfree(h->val[0]);
    dfree(h->val[1]);
    dfree(h->user_perm);
    dfree(h->rec);
    dfree(h->G);
    dfree(h->P);
    dfree(h->mb_part);
    dfree(h->mb_loss);
    dfree(h->tile_loss);
    dfree(h->core_part);
    dfree(h->dpart);
    dfree(h->scal);
    for (auto &p : h->pending) {
        if (p.a) (void)hipEventDestroy(p.a);
        if (p.b) (void)hipEventDestroy(p.b);
    }
    for (auto e : h->pool) (void)hipEventDestroy(e);
}

// ------------------------------------------------------------------ options
extern "C" ft_status ft_default_options(ft_options *o) {
    if (!o) return fail(nullptr, FT_EINVAL, "options pointer is NULL");
    std::memset(o, 0, sizeof *o);
    o->minibatch = 512;
    o->lr_A = o->lr_B = 0.01;
    o->lambda_A = o->lambda_B = 1e-3;
    o->precision = FT_FP32;
    o->row_scale = FT_ROW_SUM;
    o->core_step = FT_CORE_PER_EPOCH;
    o->deterministic = 1;
    o->shuffle_seed = 0;
    o->reshuffle_each_epoch = 1;
    o->vector_alu = 0;
    o->core_storage = 0;
    return FT_OK;
}

extern "C" const char *ft_last_error(const ft_handle *h) {
    return h ? h->err.c_str() : g_create_error.c_str();
}

static ft_status check_options(ft_handle *h, const ft_options *o) {
    if (!o) return fail(h, FT_EINVAL, "options pointer is NULL");
    if (o->minibatch < 1 || o->minibatch > (1ll << 30))
        return fail(h, FT_EINVAL, "minibatch must be in [1, 2^30], got %lld",
                    (long long)o->minibatch);
    const double v[4] = {o->lr_A, o->lr_B, o->lambda_A, o->lambda_B};
    for (double x : v)
        if (!std::isfinite(x) || x < 0)
            return fail(h, FT_EINVAL,
                        "learning rates and lambdas must be finite and >= 0");
    if (o->precision != FT_FP32 && o->precision != FT_BF16 &&
        o->precision != FT_FP8_E4M3)
        return fail(h, FT_EINVAL,
                    "precision must be FT_FP32, FT_BF16 or FT_FP8_E4M3, got %d",
                    o->precision);
    if (o->precision != FT_FP32 && o->deterministic == 0)
        return fail(h, FT_EINVAL,
                    "the BF16 and FP8 contractions are available in verify "
                    "mode only");
    if (o->row_scale != FT_ROW_SUM && o->row_scale != FT_ROW_MEAN)
        return fail(h, FT_EINVAL, "row_scale must be FT_ROW_SUM or FT_ROW_MEAN");
    if (o->core_step != FT_CORE_PER_EPOCH &&
        o->core_step != FT_CORE_PER_MINIBATCH)
        return fail(h, FT_EINVAL, "core_step must be PER_EPOCH or PER_MINIBATCH");
    if (o->deterministic != 0 && o->deterministic != 1)
        return fail(h, FT_EINVAL, "deterministic must be 0 or 1");
    if (o->deterministic == 0 && o->minibatch % 16 != 0)
        return fail(h, FT_EINVAL,
                    "the Hogwild fast mode needs a minibatch that is a "
                    "multiple of the 16-sample tile, got %lld",
                    (long long)o->minibatch);
    if (o->reshuffle_each_epoch != 0 && o->reshuffle_each_epoch != 1)
        return fail(h, FT_EINVAL, "reshuffle_each_epoch must be 0 or 1");
    if (o->vector_alu != 0 && o->vector_alu != 1)
        return fail(h, FT_EINVAL, "vector_alu must be 0 or 1");
    Shape vsh = h->sh;                  // the shape at the requested precision
    vsh.prec = kF32;
    if (o->vector_alu &&
        (o->precision != FT_FP32 || !o->deterministic ||
         !factor_valu_supported(vsh)))
        return fail(h, FT_EINVAL,
                    "vector_alu needs FP32 and the verify mode");
    if (o->core_storage != 0 && o->core_storage != 1)
        return fail(h, FT_EINVAL, "core_storage must be 0 or 1");
    if (h->N > kFullOrder &&
        (o->precision != FT_FP32 || !o->deterministic || o->vector_alu ||
         o->core_storage))
        return fail(h, FT_EINVAL,
                    "orders above %d run the FP32 verify path only (no "
                    "BF16/FP8, fast mode, vector_alu or core_storage)",
                    kFullOrder);
    if (o->core_storage &&
        (o->precision != FT_FP32 || !o->deterministic || o->vector_alu))
        return fail(h, FT_EINVAL,
                    "core_storage needs FP32, the verify mode and "
                    "vector_alu = 0");
    return FT_OK;
}

// Refresh the low-precision shadow of A^(n) (BF16, or FP8 codes and row
// scales) from the FP32 master.
static ft_status refresh_shadow(ft_handle *h, int n) {
    const int64_t count = h->dims[n] * h->sh.J4;
    if (h->sh.prec == kBF16) {
        if (!h->A16[n])
            HIPCHK(h, hipMalloc(&h->A16[n], sizeof(uint16_t) * count));
        HIPCHK(h, launch_to_bf16(h->A[n], h->A16[n], count, h->stream));
    } else if (h->sh.prec == kFP8) {
        if (!h->A8[n]) HIPCHK(h, hipMalloc(&h->A8[n], count));
        if (!h->As[n])
            HIPCHK(h, hipMalloc(&h->As[n], sizeof(float) * h->dims[n]));
        HIPCHK(h, launch_to_fp8_rows(h->A[n], h->dims[n], h->sh.J4, h->A8[n],
                                     h->As[n], h->stream));
    } else {
        return FT_OK;
    }
    HIPCHK(h, hipStreamSynchronize(h->stream));
    return FT_OK;
}

extern "C" ft_status ft_set_options(ft_handle *h, const ft_options *o) {
    CHECK_HANDLE(h);
    ft_status st = check_options(h, o);
    if (st != FT_OK) return st;
    const int prec = o->precision == FT_BF16       ? kBF16
                     : o->precision == FT_FP8_E4M3 ? kFP8
                                                   : kF32;
    if (prec != h->sh.prec) {
        const int old = h->sh.prec;
        h->sh.prec = prec;
        for (int n = 0; n < h->N; ++n) {
            st = refresh_shadow(h, n);
            if (st != FT_OK) {
                h->sh.prec = old;
                return st;
            }
        }
    }
    if (o->minibatch != h->opt.minibatch ||
        o->shuffle_seed != h->opt.shuffle_seed ||
        o->reshuffle_each_epoch != h->opt.reshuffle_each_epoch)
        h->prepared = false;
    h->opt = *o;
    return FT_OK;
}

extern "C" ft_status ft_get_options(const ft_handle *h, ft_options *o) {
    if (!h) return fail(nullptr, FT_EINVAL, "handle is NULL");
    if (!o) return FT_EINVAL;
    *o = h->opt;
    return FT_OK;
}

extern "C" ft_status ft_set_stream(ft_handle *h, void *hip_stream) {
    CHECK_HANDLE(h);
    h->stream = (hipStream_t)hip_stream;
    return FT_OK;
}

// ------------------------------------------------------------------ create
extern "C" ft_status ft_create(int order, const int64_t *dims,
                               const int32_t *J, int32_t R, uint64_t seed,
                               ft_handle **out) {
    if (!out) return fail(nullptr, FT_EINVAL, "out pointer is NULL");
    *out = nullptr;
    if (order < 2 || order > kMaxOrder)
        return fail(nullptr, FT_EINVAL,
                    "order must be in [2, %d] on the device path, got %d",
                    kMaxOrder, order);
    if (!dims || !J) return fail(nullptr, FT_EINVAL, "dims or J is NULL");
    for (int n = 0; n < order; ++n) {
        if (dims[n] < 1 || dims[n] > 0x7fffffffll)
            return fail(nullptr, FT_EINVAL, "dims[%d] = %lld out of [1, 2^31)",
                        n, (long long)dims[n]);
        if (J[n] < 1 || J[n] > kMaxJ)
            return fail(nullptr, FT_EINVAL, "J[%d] = %d out of [1, %d]", n,
                        J[n], kMaxJ);
    }
    if (R < 1 || R > kMaxR)
        return fail(nullptr, FT_EINVAL, "R = %d out of [1, %d]", R, kMaxR);
    {
        int jmax = 0;
        for (int n = 0; n < order; ++n) jmax = std::max(jmax, (int)J[n]);
        if (!high_order_fits(order, padded_j4(order, jmax), (R + 15) / 16 * 16))
            return fail(nullptr, FT_EINVAL,
                        "order %d with J4 = %d and R16 = %d exceeds the core "
                        "kernel's LDS (order x J4 x R16 <= %d above order %d)",
                        order, padded_j4(order, jmax), (R + 15) / 16 * 16,
                        kHighOrderTile, kFullOrder);
    }

    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1)
        return fail(nullptr, FT_EDEVICE, "no HIP device is available");

    ft_handle *h = new (std::nothrow) ft_handle();
    if (!h) return fail(nullptr, FT_ENOMEM, "out of host memory");
    if (hipGetDevice(&h->device) != hipSuccess) {
        delete h;
        return fail(nullptr, FT_EDEVICE, "hipGetDevice failed");
    }
    h->N = order;
    int jmax = 0;
    for (int n = 0; n < order; ++n) {
        h->dims[n] = dims[n];
        h->J[n] = J[n];
        if (J[n] > jmax) jmax = J[n];
    }
    h->R = R;
    h->sh.N = order;
    h->sh.J4 = padded_j4(order, jmax);
    h->sh.R16 = (R + 15) / 16 * 16;
    ft_default_options(&h->opt);

    ft_status st = FT_OK;
    std::vector<float> hostbuf;
    uint64_t rng = seed;
    for (int n = 0; n < order && st == FT_OK; ++n) {
        size_t capA = 0, capB = 0;
        hipError_t e = ensure(&h->A[n], &capA, (size_t)dims[n] * h->sh.J4);
        if (e == hipSuccess)
            e = ensure(&h->B[n], &capB, (size_t)h->sh.J4 * h->sh.R16);
        if (e == hipSuccess)
            e = hipMemset(h->A[n], 0, sizeof(float) * dims[n] * h->sh.J4);
        if (e == hipSuccess)
            e = hipMemset(h->B[n], 0, sizeof(float) * h->sh.J4 * h->sh.R16);
        if (e != hipSuccess) {
            st = fail(nullptr, e == hipErrorOutOfMemory ? FT_ENOMEM : FT_EDEVICE,
                      "allocation of parameters failed: %s",
                      hipGetErrorString(e));
            break;
        }
        hostbuf.assign((size_t)dims[n] * J[n], 0.f);
        for (auto &x : hostbuf) x = (float)(0.5 * normal01(rng));
        st = upload_padded(h, h->A[n], hostbuf.data(), dims[n], J[n], h->sh.J4);
        if (st != FT_OK) break;
        hostbuf.assign((size_t)J[n] * R, 0.f);
        for (auto &x : hostbuf) x = (float)(0.5 * normal01(rng));
        st = upload_padded(h, h->B[n], hostbuf.data(), J[n], R, h->sh.R16);
    }
    if (st == FT_OK) {
        size_t cap = 0;
        hipError_t e = ensure(&h->scal, &cap, 64);
        if (e != hipSuccess)
            st = fail(nullptr, FT_ENOMEM, "allocation failed: %s",
                      hipGetErrorString(e));
    }
    if (st != FT_OK) {
        if (h->err != "no error") g_create_error = h->err;
        release(h);
        delete h;
        return st;
    }
    *out = h;
    return FT_OK;
}

extern "C" ft_status ft_destroy(ft_handle *h) {
    if (!h) return FT_OK;
    (void)hipStreamSynchronize(h->stream);
    if (h->bstream) (void)hipStreamSynchronize(h->bstream);
    release(h);
    delete h;
    return FT_OK;
}

// ------------------------------------------------------------------ data
extern "C" ft_status ft_set_nonzeros(ft_handle *h, ft_set which, int64_t nnz,
                                     const int32_t *idx, const float *vals) {
    CHECK_HANDLE(h);
    if (which != FT_TRAIN && which != FT_TEST)
        return fail(h, FT_EINVAL, "which must be FT_TRAIN or FT_TEST");
    if (nnz < 0 || nnz > 0x7fffffffll)
        return fail(h, FT_EINVAL, "nnz = %lld out of [0, 2^31)", (long long)nnz);
    if (which == FT_TRAIN && nnz < 1)
        return fail(h, FT_EINVAL, "the training set needs at least 1 nonzero");
    if (nnz > 0 && (!idx || !vals))
        return fail(h, FT_EINVAL, "idx or vals is NULL");
    for (int n = 0; n < h->N; ++n) {
        const int32_t *row = idx + (size_t)n * nnz;
        const int64_t I = h->dims[n];
        for (int64_t s = 0; s < nnz; ++s)
            if (row[s] < 0 || row[s] >= I)
                return fail(h, FT_EINVAL,
                            "index %d of nonzero %lld in mode %d is out of "
                            "[0, %lld)",
                            row[s], (long long)s, n, (long long)I);
    }
    for (int64_t s = 0; s < nnz; ++s)
        if (!std::isfinite(vals[s]))
            return fail(h, FT_EINVAL, "value of nonzero %lld is not finite",
                        (long long)s);

    HIPCHK(h, hipStreamSynchronize(h->stream));
    if (h->bstream) HIPCHK(h, hipStreamSynchronize(h->bstream));
    for (int n = 0; n < h->N; ++n) {
        dfree(h->idx[which][n]);
        h->idx[which][n] = nullptr;
    }
    dfree(h->val[which]);
    h->val[which] = nullptr;
    h->nnz[which] = 0;
    if (nnz > 0) {
        for (int n = 0; n < h->N; ++n) {
            HIPCHK(h, hipMalloc(&h->idx[which][n], sizeof(int32_t) * nnz));
            HIPCHK(h, hipMemcpy(h->idx[which][n], idx + (size_t)n * nnz,
                                sizeof(int32_t) * nnz, hipMemcpyHostToDevice));
        }
        HIPCHK(h, hipMalloc(&h->val[which], sizeof(float) * nnz));
        HIPCHK(h, hipMemcpy(h->val[which], vals, sizeof(float) * nnz,
                            hipMemcpyHostToDevice));
    }
    h->nnz[which] = nnz;
    if (which == FT_TRAIN) {
        h->use_user_perm = false;
        h->prepared = false;
        h->epoch = 0;
        h->train_gen += 1;
        dfree(h->user_perm);
        h->user_perm = nullptr;
        for (auto &E : h->eb) free_epoch_bufs(E);
        h->cur = 0;
        dfree(h->rec);
        h->rec = nullptr;
        const int rw = record_words(h->N);
        HIPCHK(h, hipMalloc(&h->rec, sizeof(uint32_t) * rw * nnz));
        HIPCHK(h, launch_pack_records(h->N, h->idx[FT_TRAIN], h->val[FT_TRAIN],
                                      nnz, h->rec, rw, h->stream));
        HIPCHK(h, hipStreamSynchronize(h->stream));
        ft_status st = alloc_epoch_bufs(h, h->eb[0]);
        if (st != FT_OK) return st;
    }
    return FT_OK;
}

extern "C" ft_status ft_set_epoch_order(ft_handle *h, const int64_t *perm) {
    CHECK_HANDLE(h);
    const int64_t nnz = h->nnz[FT_TRAIN];
    if (nnz < 1) return fail(h, FT_ESTATE, "no training set");
    if (!perm) {
        h->use_user_perm = false;
        h->prepared = false;
        return FT_OK;
    }
    std::vector<uint8_t> seen((size_t)nnz, 0);
    std::vector<uint32_t> p32((size_t)nnz);
    for (int64_t i = 0; i < nnz; ++i) {
        const int64_t v = perm[i];
        if (v < 0 || v >= nnz || seen[(size_t)v])
            return fail(h, FT_EINVAL,
                        "perm is not a permutation of [0, %lld) (entry %lld)",
                        (long long)nnz, (long long)i);
        seen[(size_t)v] = 1;
        p32[(size_t)i] = (uint32_t)v;
    }
    if (!h->user_perm) HIPCHK(h, hipMalloc(&h->user_perm, sizeof(uint32_t) * nnz));
    HIPCHK(h, hipMemcpy(h->user_perm, p32.data(), sizeof(uint32_t) * nnz,
                        hipMemcpyHostToDevice));
    h->use_user_perm = true;
    h->prepared = false;
    return FT_OK;
}

extern "C" ft_status ft_num_minibatches(const ft_handle *h, int64_t *out) {
    if (!h) return fail(nullptr, FT_EINVAL, "handle is NULL");
    if (!out) return FT_EINVAL;
    *out = h->nnz[FT_TRAIN] > 0 ? nminibatches(h) : 0;
    return FT_OK;
}

// ------------------------------------------------------------------ builder
// The builder writes one buffer set E for the order of epoch `epoch` on
// stream s; nothing it reads or writes is touched by the parameters, so the
// next epoch's set can be built while the current epoch trains.
static ft_status alloc_epoch_bufs(ft_handle *h, EpochBufs &E) {
    const int64_t nnz = h->nnz[FT_TRAIN];
    HIPCHK(h, hipMalloc(&E.perm, sizeof(uint32_t) * nnz));
    HIPCHK(h, hipMalloc(&E.pval, sizeof(float) * nnz));
    for (int n = 0; n < h->N; ++n) {
        HIPCHK(h, hipMalloc(&E.pidx[n], sizeof(int32_t) * nnz));
        HIPCHK(h, hipMalloc(&E.inv[n], sizeof(uint32_t) * nnz));
        for (int s = 0; s < 2; ++s) {
            HIPCHK(h, hipMalloc(&E.sk[s][n], sizeof(uint32_t) * nnz));
            HIPCHK(h, hipMalloc(&E.sv[s][n], sizeof(uint32_t) * nnz));
        }
    }
    HIPCHK(h, hipEventCreateWithFlags(&E.ready, hipEventDisableTiming));
    return FT_OK;
}

static ft_status draw_order(ft_handle *h, EpochBufs &E, uint64_t epoch,
                            uint64_t salt, hipStream_t s) {
    const int64_t nnz = h->nnz[FT_TRAIN];
    Launch L(h, FT_K_ORDER, s);
    if (h->use_user_perm) {
        HIPCHK(h, hipMemcpyAsync(E.perm, h->user_perm, sizeof(uint32_t) * nnz,
                                 hipMemcpyDeviceToDevice, s));
    } else {
        const uint64_t e = h->opt.reshuffle_each_epoch ? epoch : 0;
        const uint64_t key = h->opt.shuffle_seed ^
                             (0x9e3779b97f4a7c15ull * (2 * e + 1 + 2 * salt));
        HIPCHK(h, launch_epoch_order(E.perm, nnz, key, s));
    }
    return FT_OK;
}

static ft_status permute_streams(ft_handle *h, EpochBufs &E, hipStream_t s) {
    Launch L(h, FT_K_PERMUTE, s);
    HIPCHK(h, launch_permute(h->N, h->rec, record_words(h->N), E.perm,
                             h->nnz[FT_TRAIN], E.pidx, E.pval, s));
    return FT_OK;
}

static ft_status build_minibatches(ft_handle *h, EpochBufs &E,
                                   hipStream_t s) {
    const int64_t nnz = h->nnz[FT_TRAIN];
    const int64_t M = h->opt.minibatch;
    const int nseg = (int)nminibatches(h);
    const int tps = (int)((std::min<int64_t>(M, nnz) + kSortTile - 1) / kSortTile);
    const size_t nx = (size_t)nseg * h->N * kXCounts;
    HIPCHK(h, ensure(&E.counts, &E.counts_cap,
                     sort_counts_words(h->N, nseg, tps)));
    const int xcap = cross_capacity(std::min<int64_t>(M, nnz));
    const int pcap = part_capacity(std::min<int64_t>(M, nnz), h->sh.J4);
    HIPCHK(h, ensure(&E.xlist, &E.xlist_cap, (size_t)nseg * h->N * xcap));
    HIPCHK(h, ensure(&E.plist, &E.plist_cap, (size_t)nseg * h->N * pcap));
    HIPCHK(h, ensure(&E.xcount, &E.xcount_cap, nx));
    if (E.xcount_host_cap < nx) {
        if (E.xcount_host) HIPCHK(h, hipHostFree(E.xcount_host));
        E.xcount_host = nullptr;
        E.xcount_host_cap = 0;
        HIPCHK(h, hipHostMalloc((void **)&E.xcount_host, sizeof(int32_t) * nx,
                                hipHostMallocDefault));
        E.xcount_host_cap = nx;
    }
    Launch L(h, FT_K_SORT, s);
    SortPass p{};
    p.N = h->N;
    p.nnz = nnz;
    p.M = M;
    p.nseg = nseg;
    p.tiles_per_seg = tps;
    p.counts = E.counts;
    // each mode takes as many 8-bit passes as its own row ids need; a pass
    // sorts the modes that still have digits left (packed into slots)
    int passes[kMaxOrder], cur[kMaxOrder] = {}, max_passes = 1;
    for (int n = 0; n < h->N; ++n) {
        passes[n] = radix_passes(h->dims[n]);
        max_passes = std::max(max_passes, passes[n]);
    }
    for (int pass = 0; pass < max_passes; ++pass) {
        p.shift = 8 * pass;
        p.N = 0;
        for (int n = 0; n < h->N; ++n) {
            if (pass >= passes[n]) continue;
            const int k = p.N++;
            const int out = pass == 0 ? 0 : cur[n] ^ 1;
            const bool last = pass == passes[n] - 1;
            p.key_in[k] = pass == 0 ? reinterpret_cast<const uint32_t *>(E.pidx[n])
                                    : E.sk[cur[n]][n];
            p.val_in[k] = pass == 0 ? nullptr : E.sv[cur[n]][n];
            p.key_out[k] = E.sk[out][n];
            // the last pass keeps the sorted rows and the inverse; the
            // sorted positions themselves are not needed downstream
            p.val_out[k] = last ? nullptr : E.sv[out][n];
            p.inv_out[k] = last ? E.inv[n] : nullptr;
            cur[n] = out;
        }
        HIPCHK(h, launch_sort_pass(p, s));
    }
    for (int n = 0; n < h->N; ++n) E.sort_final[n] = cur[n];
    CrossArgs cx{};
    cx.N = h->N;
    cx.nnz = nnz;
    cx.M = M;
    cx.nseg = nseg;
    cx.xcap = xcap;
    for (int n = 0; n < h->N; ++n) cx.rows[n] = E.sk[cur[n]][n];
    cx.xlist = E.xlist;
    cx.plist = E.plist;
    cx.pcap = pcap;
    cx.xcount = E.xcount;
    cx.J4 = h->sh.J4;
    E.xcap = xcap;
    E.pcap = pcap;
    HIPCHK(h, launch_crossing_segments(cx, s));
    // the crossing-row counts size the reduction grids: one read-back per
    // epoch (waited for before the first minibatch) instead of a worst-case
    // grid per minibatch
    HIPCHK(h, hipMemcpyAsync(E.xcount_host, E.xcount, sizeof(int32_t) * nx,
                             hipMemcpyDeviceToHost, s));
    HIPCHK(h, hipEventRecord(E.ready, s));
    E.pending = true;
    return FT_OK;
}

static ft_status build_epoch(ft_handle *h, EpochBufs &E, uint64_t epoch,
                             hipStream_t s) {
    E.valid = false;
    ft_status st = draw_order(h, E, epoch, 0, s);
    if (st == FT_OK) st = permute_streams(h, E, s);
    if (st == FT_OK) st = build_minibatches(h, E, s);
    if (st != FT_OK) return st;
    E.valid = true;
    E.epoch = epoch;
    E.M = h->opt.minibatch;
    E.seed = h->opt.shuffle_seed;
    E.gen = h->train_gen;
    return FT_OK;
}

// Host wait for a set's crossing-row counts.
static ft_status counts_ready(ft_handle *h, EpochBufs &E) {
    if (E.pending) {
        HIPCHK(h, hipEventSynchronize(E.ready));
        E.pending = false;
    }
    return FT_OK;
}

static ft_status prepare(ft_handle *h) {
    if (h->nnz[FT_TRAIN] < 1) return fail(h, FT_ESTATE, "no training set");
    EpochBufs &E = h->eb[h->cur];
    ft_status st = build_epoch(h, E, h->epoch, h->stream);
    if (st == FT_OK) st = counts_ready(h, E);
    if (st != FT_OK) return st;
    h->prepared = true;
    h->prepared_M = h->opt.minibatch;
    return FT_OK;
}

// Make the current epoch's builder output current: the set built ahead if
// it matches, else build it now.
static ft_status acquire_epoch(ft_handle *h) {
    EpochBufs &A = h->eb[h->cur ^ 1];
    if (A.valid && A.epoch == h->epoch && A.M == h->opt.minibatch &&
        A.seed == h->opt.shuffle_seed && A.gen == h->train_gen &&
        !h->use_user_perm && h->opt.reshuffle_each_epoch) {
        HIPCHK(h, hipStreamWaitEvent(h->stream, A.ready, 0));
        ft_status st = counts_ready(h, A);
        if (st != FT_OK) return st;
        h->cur ^= 1;
        h->prepared = true;
        h->prepared_M = h->opt.minibatch;
        return FT_OK;
    }
    return prepare(h);
}

// Build the set of factor epoch `ep` on the builder stream (it only reads
// the training records; the set it overwrites belonged to a finished epoch,
// and every epoch call returns synchronised). It is started when a core
// phase begins: the core kernels are bound by the matrix cores and leave
// room beside them, while the minibatch kernels of a factor phase are
// latency-bound and lose far more to a builder running beside them (at
// order 5, J = R = 32, 200M nonzeros: epoch 215 ms with the builder beside
// the factor phase on a small grid, 200 ms building serially before it,
// 180 ms beside the core phase on a full grid).
static ft_status build_ahead(ft_handle *h, uint64_t ep) {
    if (!h->opt.reshuffle_each_epoch || h->use_user_perm) return FT_OK;
    if (!h->bstream)
        HIPCHK(h, hipStreamCreateWithFlags(&h->bstream, hipStreamNonBlocking));
    EpochBufs &A = h->eb[h->cur ^ 1];
    if (A.valid && A.epoch == ep && A.M == h->opt.minibatch &&
        A.seed == h->opt.shuffle_seed && A.gen == h->train_gen)
        return FT_OK;                    // built (or being built) already
    if (!A.perm) {
        ft_status st = alloc_epoch_bufs(h, A);
        if (st != FT_OK) return st;
    }
    ft_status st = counts_ready(h, A);   // an unused earlier build of A
    if (st != FT_OK) return st;
    return build_epoch(h, A, ep, h->bstream);
}

extern "C" ft_status ft_prepare_epoch(ft_handle *h) {
    CHECK_HANDLE(h);
    return prepare(h);
}

// ------------------------------------------------------------------ factor
static ft_status run_minibatch(ft_handle *h, int64_t b, int apply,
                               double *loss_part, float *const *grad,
                               int32_t *const *count) {
    const int64_t M = h->opt.minibatch;
    const int64_t off = b * M;
    const int32_t m = (int32_t)std::min<int64_t>(M, h->nnz[FT_TRAIN] - off);
    const EpochBufs &E = h->eb[h->cur];
    FactorArgs fa{};
    for (int n = 0; n < h->N; ++n) {
        fa.idx[n] = E.pidx[n] + off;
        fa.A[n] = h->A[n];
        fa.A16[n] = h->sh.prec == kBF16 ? h->A16[n] : nullptr;
        fa.A8[n] = h->sh.prec == kFP8 ? h->A8[n] : nullptr;
        fa.As[n] = h->sh.prec == kFP8 ? h->As[n] : nullptr;
        fa.B[n] = h->B[n];
    }
    fa.val = E.pval + off;
    fa.m = m;
    fa.G = h->G;
    for (int n = 0; n < h->N; ++n) fa.inv[n] = E.inv[n] + off;
    fa.loss_part = loss_part;
    int nb = 0;
    {
        LaunchExt L(h, FT_K_FACTOR_GRAD);
        if (h->opt.vector_alu)
            HIPCHK(h, launch_factor_grad_valu(h->sh, fa, &nb, h->stream));
        else
            HIPCHK(h, launch_factor_grad(h->sh, fa, &nb, h->stream));
    }
    SegArgs sa{};
    sa.N = h->N;
    sa.J4 = h->sh.J4;
    sa.m = m;
    sa.nchunks = (m + kSegChunk - 1) / kSegChunk;
    for (int n = 0; n < h->N; ++n) {
        sa.rows[n] = E.sk[E.sort_final[n]][n] + off;
        sa.A[n] = h->A[n];
        sa.A16[n] = h->sh.prec == kBF16 ? h->A16[n] : nullptr;
        sa.A8[n] = h->sh.prec == kFP8 ? h->A8[n] : nullptr;
        sa.As[n] = h->sh.prec == kFP8 ? h->As[n] : nullptr;
        sa.xlist[n] = E.xlist + ((size_t)b * h->N + n) * E.xcap;
        sa.plist[n] = E.plist + ((size_t)b * h->N + n) * E.pcap;
        sa.grad[n] = grad ? grad[n] : nullptr;
        sa.count[n] = count ? count[n] : nullptr;
    }
    sa.G = h->G;
    sa.xcount = E.xcount + (size_t)b * h->N * kXCounts;
    sa.xcap = E.xcap;
    sa.pcap = E.pcap;
    sa.P = h->P;
    sa.host_counts = 1;
    sa.xs[0] = sa.xl[0] = sa.xp[0] = 0;
    int nmulti = 0;
    for (int n = 0; n < h->N; ++n) {
        const int32_t *xc = E.xcount_host + (b * h->N + n) * kXCounts;
        sa.xs[n + 1] = sa.xs[n] + xc[0];
        sa.xl[n + 1] = sa.xl[n] + xc[1];
        sa.xp[n + 1] = sa.xp[n] + xc[2];
        nmulti += xc[3];
    }
    sa.small_blocks = (sa.xs[h->N] + kSegWaves - 1) / kSegWaves;
    sa.large_blocks = sa.xp[h->N];
    sa.combine_blocks =
        nmulti > 0 ? (sa.xl[h->N] + kSegWaves - 1) / kSegWaves : 0;
    sa.lr = (float)h->opt.lr_A;
    sa.lam = (float)h->opt.lambda_A;
    sa.mean = h->opt.row_scale == FT_ROW_MEAN;
    sa.apply = apply;
    {
        LaunchExt L(h, FT_K_SEG_REDUCE);
        HIPCHK(h, launch_seg_reduce(sa, h->stream));
    }
    if (sa.combine_blocks > 0) {
        LaunchExt L(h, FT_K_SEG_COMBINE);
        HIPCHK(h, launch_seg_combine(sa, h->stream));
    }
    return FT_OK;
}

static ft_status alloc_factor(ft_handle *h, int64_t nmb, int nper) {
    const int64_t M = std::min<int64_t>(h->opt.minibatch, h->nnz[FT_TRAIN]);
    const int64_t nch = (M + kSegChunk - 1) / kSegChunk;
    (void)nch;
    HIPCHK(h, ensure(&h->G, &h->G_cap, (size_t)h->N * M * h->sh.J4));
    HIPCHK(h, ensure(&h->P, &h->P_cap,
                     (size_t)h->N * part_capacity(M, h->sh.J4) * h->sh.J4));
    HIPCHK(h, ensure(&h->mb_part, &h->mb_part_cap, (size_t)nmb * nper));
    HIPCHK(h, ensure(&h->mb_loss, &h->mb_loss_cap, (size_t)nmb));
    return FT_OK;
}

// Hogwild fast mode: order + permutation, then one persistent sweep over all
// tiles with immediate atomic row updates (no builder, no minibatch barrier).
static ft_status epoch_factors_fast(ft_handle *h, std::vector<double> &losses) {
    const int64_t nnz = h->nnz[FT_TRAIN];
    EpochBufs &E = h->eb[h->cur];
    E.valid = false;
    ft_status st = draw_order(h, E, h->epoch, 0, h->stream);
    if (st == FT_OK) st = permute_streams(h, E, h->stream);
    if (st != FT_OK) return st;
    h->prepared = false;
    const int64_t nmb = nminibatches(h);
    const int64_t tpm = h->opt.minibatch / 16;
    HIPCHK(h, ensure(&h->tile_loss, &h->tile_loss_cap, (size_t)(nmb * tpm)));
    HIPCHK(h, ensure(&h->mb_loss, &h->mb_loss_cap, (size_t)nmb));
    HIPCHK(h, hipMemsetAsync(h->tile_loss, 0, sizeof(double) * nmb * tpm,
                             h->stream));
    HogArgs ha{};
    for (int n = 0; n < h->N; ++n) {
        ha.idx[n] = E.pidx[n];
        ha.A[n] = h->A[n];
        ha.B[n] = h->B[n];
    }
    ha.val = E.pval;
    ha.count = nnz;
    ha.lr = (float)h->opt.lr_A;
    ha.lam = (float)h->opt.lambda_A;
    ha.tile_loss = h->tile_loss;
    {
        LaunchExt L(h, FT_K_HOGWILD);
        HIPCHK(h, launch_hogwild(h->sh, ha, h->stream));
    }
    HIPCHK(h, launch_sum_blocks(h->tile_loss, (int)tpm, (int)nmb, h->mb_loss,
                                h->stream));
    losses.resize((size_t)nmb);
    HIPCHK(h, hipMemcpyAsync(losses.data(), h->mb_loss, sizeof(double) * nmb,
                             hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    return FT_OK;
}

extern "C" ft_status ft_epoch_factors(ft_handle *h, double *mb_loss) {
    CHECK_HANDLE(h);
    if (h->nnz[FT_TRAIN] < 1) return fail(h, FT_ESTATE, "no training set");
    if (!h->opt.deterministic) {
        std::vector<double> losses;
        ft_status st = epoch_factors_fast(h, losses);
        if (st != FT_OK) return st;
        h->epoch += 1;
        if (mb_loss)
            std::memcpy(mb_loss, losses.data(), sizeof(double) * losses.size());
        for (double l : losses)
            if (!std::isfinite(l))
                return fail(h, FT_ENONFINITE, "a minibatch loss is not finite");
        return FT_OK;
    }
    const bool reuse = h->prepared && !h->opt.reshuffle_each_epoch &&
                       h->prepared_M == h->opt.minibatch;
    if (!reuse) {
        ft_status st = acquire_epoch(h);
        if (st != FT_OK) return st;
    }
    const int64_t nmb = nminibatches(h);
    const int nper = factor_grad_blocks(
        h->sh, (int32_t)std::min<int64_t>(h->opt.minibatch, h->nnz[FT_TRAIN]));
    ft_status st = alloc_factor(h, nmb, nper);
    if (st != FT_OK) return st;
    HIPCHK(h, hipMemsetAsync(h->mb_part, 0, sizeof(double) * nmb * nper,
                             h->stream));
    for (int64_t b = 0; b < nmb; ++b) {
        st = run_minibatch(h, b, 1, h->mb_part + b * nper, nullptr, nullptr);
        if (st != FT_OK) return st;
    }
    HIPCHK(h, launch_sum_blocks(h->mb_part, nper, (int)nmb, h->mb_loss,
                                h->stream));
    std::vector<double> losses((size_t)nmb);
    HIPCHK(h, hipMemcpyAsync(losses.data(), h->mb_loss, sizeof(double) * nmb,
                             hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    h->epoch += 1;
    if (mb_loss) std::memcpy(mb_loss, losses.data(), sizeof(double) * nmb);
    for (double l : losses)
        if (!std::isfinite(l))
            return fail(h, FT_ENONFINITE, "a minibatch loss is not finite");
    return FT_OK;
}

extern "C" ft_status ft_factor_minibatch(ft_handle *h, int64_t b,
                                         int32_t apply, double *loss,
                                         float *const *grad,
                                         int32_t *const *count) {
    CHECK_HANDLE(h);
    if (!h->prepared || h->prepared_M != h->opt.minibatch)
        return fail(h, FT_ESTATE, "no prepared epoch (call ft_prepare_epoch)");
    const int64_t nmb = nminibatches(h);
    if (b < 0 || b >= nmb)
        return fail(h, FT_EINVAL, "minibatch %lld out of [0, %lld)",
                    (long long)b, (long long)nmb);
    if (apply != 0 && apply != 1)
        return fail(h, FT_EINVAL, "apply must be 0 or 1");
    if (!apply && (!grad || !count))
        return fail(h, FT_EINVAL, "apply = 0 needs grad and count buffers");
    if (!apply)
        for (int n = 0; n < h->N; ++n)
            if (!grad[n] || !count[n])
                return fail(h, FT_EINVAL, "grad[%d] or count[%d] is NULL", n, n);
    const int nper = factor_grad_blocks(
        h->sh, (int32_t)std::min<int64_t>(h->opt.minibatch, h->nnz[FT_TRAIN]));
    ft_status st = alloc_factor(h, nmb, nper);
    if (st != FT_OK) return st;
    float *dgrad[kMaxOrder] = {};
    int32_t *dcount[kMaxOrder] = {};
    struct Guard {
        float **g;
        int32_t **c;
        ~Guard() {
            for (int n = 0; n < kMaxOrder; ++n) {
                dfree(g[n]);
                dfree(c[n]);
            }
        }
    } guard{dgrad, dcount};
    if (!apply) {
        for (int n = 0; n < h->N; ++n) {
            HIPCHK(h, hipMalloc(&dgrad[n], sizeof(float) * h->dims[n] * h->sh.J4));
            HIPCHK(h, hipMalloc(&dcount[n], sizeof(int32_t) * h->dims[n]));
            HIPCHK(h, hipMemsetAsync(dgrad[n], 0,
                                     sizeof(float) * h->dims[n] * h->sh.J4,
                                     h->stream));
            HIPCHK(h, hipMemsetAsync(dcount[n], 0, sizeof(int32_t) * h->dims[n],
                                     h->stream));
        }
    }
    HIPCHK(h, hipMemsetAsync(h->mb_part, 0, sizeof(double) * nper, h->stream));
    st = run_minibatch(h, b, apply, h->mb_part, apply ? nullptr : dgrad,
                       apply ? nullptr : dcount);
    if (st != FT_OK) return st;
    HIPCHK(h, launch_sum_blocks(h->mb_part, nper, 1, h->scal, h->stream));
    double l = 0.0;
    HIPCHK(h, hipMemcpyAsync(&l, h->scal, sizeof(double), hipMemcpyDeviceToHost,
                             h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    if (loss) *loss = l;
    if (!apply) {
        for (int n = 0; n < h->N; ++n) {
            st = download_padded(h, grad[n], dgrad[n], h->dims[n], h->J[n],
                                 h->sh.J4);
            if (st != FT_OK) return st;
            HIPCHK(h, hipMemcpy(count[n], dcount[n],
                                sizeof(int32_t) * h->dims[n],
                                hipMemcpyDeviceToHost));
        }
    }
    return FT_OK;
}

// ------------------------------------------------------------------ core
static ft_status core_pass(ft_handle *h, const int32_t *const *idx,
                           const float *val, int64_t count, int apply,
                           float *grad_out, double *loss_dev) {
    const int nb = core_grad_blocks(count);
    const size_t E = (size_t)h->N * h->sh.J4 * h->sh.R16;
    HIPCHK(h, ensure(&h->core_part, &h->core_part_cap, (size_t)nb * E));
    HIPCHK(h, ensure(&h->dpart, &h->dpart_cap, (size_t)2 * kMaxOrder * 1024 + 4096));
    CoreArgs ca{};
    for (int n = 0; n < h->N; ++n) {
        ca.idx[n] = idx[n];
        ca.A[n] = h->A[n];
        ca.A16[n] = h->sh.prec == kBF16 ? h->A16[n] : nullptr;
        ca.A8[n] = h->sh.prec == kFP8 ? h->A8[n] : nullptr;
        ca.As[n] = h->sh.prec == kFP8 ? h->As[n] : nullptr;
        ca.B[n] = h->B[n];
    }
    ca.val = val;
    ca.count = count;
    ca.part = h->core_part;
    ca.loss_part = h->dpart;
    int used = nb;
    ca.blocks_used = &used;
    if (h->opt.core_storage) {
        // A and B are fixed for the pass: store every row's C = a B once
        for (int n = 0; n < h->N; ++n) {
            if (!h->Cst[n])
                HIPCHK(h, hipMalloc(&h->Cst[n], sizeof(float) * h->dims[n] *
                                                    h->sh.R16));
            LaunchExt L(h, FT_K_PRECOMPUTE_C);
            HIPCHK(h, launch_precompute_c(h->sh, h->A[n], h->B[n], h->dims[n],
                                          h->Cst[n], h->stream));
            ca.Cst[n] = h->Cst[n];
        }
    }
    {
        LaunchExt L(h, FT_K_CORE_GRAD);
        if (h->opt.vector_alu)
            HIPCHK(h, launch_core_grad_valu(h->sh, ca, nb, h->stream));
        else if (h->opt.core_storage)
            HIPCHK(h, launch_core_grad_stored(h->sh, ca, nb, h->stream));
        else
            HIPCHK(h, launch_core_grad(h->sh, ca, nb, h->stream));
    }
    CoreUpdateArgs ua{};
    ua.part = h->core_part;
    ua.nblocks = used;
    for (int n = 0; n < h->N; ++n) ua.B[n] = h->B[n];
    ua.grad_out = grad_out;
    ua.inv_count = 1.0 / (double)count;
    ua.lr = (float)h->opt.lr_B;
    ua.lam = (float)h->opt.lambda_B;
    ua.apply = apply;
    {
        LaunchExt L(h, FT_K_CORE_UPDATE);
        HIPCHK(h, launch_core_update(h->sh, ua, h->stream));
    }
    HIPCHK(h, launch_sum_blocks(h->dpart, used, 1, loss_dev, h->stream));
    return FT_OK;
}

extern "C" ft_status ft_epoch_core(ft_handle *h, double *loss) {
    CHECK_HANDLE(h);
    const int64_t nnz = h->nnz[FT_TRAIN];
    if (nnz < 1) return fail(h, FT_ESTATE, "no training set");
    double l = 0.0;
    // the next factor epoch's order, permutation and sort run beside this
    // core phase
    if (h->opt.deterministic) {
        ft_status st = build_ahead(h, h->epoch);
        if (st != FT_OK) return st;
    }
    if (h->opt.core_step == FT_CORE_PER_EPOCH) {
        ft_status st = core_pass(h, h->idx[FT_TRAIN], h->val[FT_TRAIN], nnz, 1,
                                 nullptr, h->scal);
        if (st != FT_OK) return st;
        HIPCHK(h, hipMemcpyAsync(&l, h->scal, sizeof(double),
                                 hipMemcpyDeviceToHost, h->stream));
    } else {
        EpochBufs &E = h->eb[h->cur];
        E.valid = false;
        ft_status st = draw_order(h, E, h->epoch, 1, h->stream);
        if (st == FT_OK) st = permute_streams(h, E, h->stream);
        if (st != FT_OK) return st;
        h->prepared = false;   // the permuted streams now hold this order
        const int64_t M = h->opt.minibatch;
        const int64_t nmb = nminibatches(h);
        HIPCHK(h, ensure(&h->mb_loss, &h->mb_loss_cap, (size_t)nmb));
        for (int64_t b = 0; b < nmb; ++b) {
            const int64_t off = b * M;
            const int64_t m = std::min<int64_t>(M, nnz - off);
            const int32_t *pi[kMaxOrder] = {};
            for (int n = 0; n < h->N; ++n) pi[n] = E.pidx[n] + off;
            st = core_pass(h, pi, E.pval + off, m, 1, nullptr, h->mb_loss + b);
            if (st != FT_OK) return st;
        }
        HIPCHK(h, launch_sum_blocks(h->mb_loss, (int)nmb, 1, h->scal, h->stream));
        HIPCHK(h, hipMemcpyAsync(&l, h->scal, sizeof(double),
                                 hipMemcpyDeviceToHost, h->stream));
    }
    HIPCHK(h, hipStreamSynchronize(h->stream));
    if (loss) *loss = l;
    if (!std::isfinite(l))
        return fail(h, FT_ENONFINITE, "the core-phase loss is not finite");
    return FT_OK;
}

extern "C" ft_status ft_core_grad(ft_handle *h, float *const *grad,
                                  double *loss) {
    CHECK_HANDLE(h);
    if (!grad) return fail(h, FT_EINVAL, "grad is NULL");
    for (int n = 0; n < h->N; ++n)
        if (!grad[n]) return fail(h, FT_EINVAL, "grad[%d] is NULL", n);
    const int64_t nnz = h->nnz[FT_TRAIN];
    if (nnz < 1) return fail(h, FT_ESTATE, "no training set");
    const size_t E = (size_t)h->N * h->sh.J4 * h->sh.R16;
    float *dg = nullptr;
    HIPCHK(h, hipMalloc(&dg, sizeof(float) * E));
    ft_status st = core_pass(h, h->idx[FT_TRAIN], h->val[FT_TRAIN], nnz, 0, dg,
                             h->scal);
    double l = 0.0;
    if (st == FT_OK) {
        hipError_t e = hipMemcpyAsync(&l, h->scal, sizeof(double),
                                      hipMemcpyDeviceToHost, h->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
        if (e != hipSuccess) st = fail(h, FT_EDEVICE, "copy failed");
    }
    for (int n = 0; n < h->N && st == FT_OK; ++n)
        st = download_padded(h, grad[n], dg + (size_t)n * h->sh.J4 * h->sh.R16,
                             h->J[n], h->R, h->sh.R16);
    dfree(dg);
    if (st == FT_OK && loss) *loss = l;
    return st;
}

// ------------------------------------------------------------------ evaluation
extern "C" ft_status ft_eval(ft_handle *h, ft_set which, double *sse,
                             double *sae) {
    CHECK_HANDLE(h);
    if (which != FT_TRAIN && which != FT_TEST)
        return fail(h, FT_EINVAL, "which must be FT_TRAIN or FT_TEST");
    const int64_t count = h->nnz[which];
    double out[2] = {0.0, 0.0};
    if (count > 0) {
        const int nb = eval_blocks(count);
        HIPCHK(h, ensure(&h->dpart, &h->dpart_cap, (size_t)2 * kMaxOrder * 1024 + 4096));
        EvalArgs ea{};
        for (int n = 0; n < h->N; ++n) {
            ea.idx[n] = h->idx[which][n];
            ea.A[n] = h->A[n];
            ea.A16[n] = h->sh.prec == kBF16 ? h->A16[n] : nullptr;
            ea.A8[n] = h->sh.prec == kFP8 ? h->A8[n] : nullptr;
            ea.As[n] = h->sh.prec == kFP8 ? h->As[n] : nullptr;
            ea.B[n] = h->B[n];
        }
        ea.val = h->val[which];
        ea.count = count;
        ea.part = h->dpart;
        {
            LaunchExt L(h, FT_K_EVAL);
            HIPCHK(h, launch_eval(h->sh, ea, nb, h->stream));
        }
        HIPCHK(h, launch_sum_blocks(h->dpart, nb, 2, h->scal, h->stream));
        HIPCHK(h, hipMemcpyAsync(out, h->scal, sizeof out, hipMemcpyDeviceToHost,
                                 h->stream));
        HIPCHK(h, hipStreamSynchronize(h->stream));
    }
    if (sse) *sse = out[0];
    if (sae) *sae = out[1];
    return FT_OK;
}

extern "C" ft_status ft_rmse(ft_handle *h, ft_set which, double *out) {
    CHECK_HANDLE(h);
    if (!out) return fail(h, FT_EINVAL, "out is NULL");
    double sse = 0.0;
    ft_status st = ft_eval(h, which, &sse, nullptr);
    if (st != FT_OK) return st;
    const int64_t count = h->nnz[which];
    *out = count > 0 ? std::sqrt(sse / (double)count) : 0.0;
    return FT_OK;
}

extern "C" ft_status ft_loss(ft_handle *h, ft_set which, double *out) {
    CHECK_HANDLE(h);
    if (!out) return fail(h, FT_EINVAL, "out is NULL");
    double sse = 0.0;
    ft_status st = ft_eval(h, which, &sse, nullptr);
    if (st != FT_OK) return st;
    const int nb = 256;
    HIPCHK(h, ensure(&h->dpart, &h->dpart_cap, (size_t)2 * kMaxOrder * 1024 + 4096));
    for (int n = 0; n < h->N; ++n) {
        HIPCHK(h, launch_sumsq(h->A[n], h->dims[n] * h->sh.J4,
                               h->dpart + (size_t)(2 * n) * nb, nb, h->stream));
        HIPCHK(h, launch_sumsq(h->B[n], (int64_t)h->sh.J4 * h->sh.R16,
                               h->dpart + (size_t)(2 * n + 1) * nb, nb,
                               h->stream));
    }
    HIPCHK(h, launch_sum_blocks(h->dpart, nb, 2 * h->N, h->scal, h->stream));
    double norms[2 * kMaxOrder] = {};
    HIPCHK(h, hipMemcpyAsync(norms, h->scal, sizeof(double) * 2 * h->N,
                             hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    double na = 0.0, nbsum = 0.0;
    for (int n = 0; n < h->N; ++n) {
        na += norms[2 * n];
        nbsum += norms[2 * n + 1];
    }
    *out = sse + h->opt.lambda_A * na + h->opt.lambda_B * nbsum;
    return FT_OK;
}

// ------------------------------------------------------------------ params
extern "C" ft_status ft_get_params(ft_handle *h, int mode, int which,
                                   float *host_out) {
    CHECK_HANDLE(h);
    if (mode < 0 || mode >= h->N || (which != 0 && which != 1) || !host_out)
        return fail(h, FT_EINVAL, "bad mode/which/out");
    if (which == 0)
        return download_padded(h, host_out, h->A[mode], h->dims[mode],
                               h->J[mode], h->sh.J4);
    return download_padded(h, host_out, h->B[mode], h->J[mode], h->R,
                           h->sh.R16);
}

extern "C" ft_status ft_set_params(ft_handle *h, int mode, int which,
                                   const float *host_in) {
    CHECK_HANDLE(h);
    if (mode < 0 || mode >= h->N || (which != 0 && which != 1) || !host_in)
        return fail(h, FT_EINVAL, "bad mode/which/in");
    if (which == 0) {
        ft_status st = upload_padded(h, h->A[mode], host_in, h->dims[mode],
                                     h->J[mode], h->sh.J4);
        return st == FT_OK ? refresh_shadow(h, mode) : st;
    }
    return upload_padded(h, h->B[mode], host_in, h->J[mode], h->R, h->sh.R16);
}

// ------------------------------------------------------------------ builder output
extern "C" ft_status ft_get_epoch_order(ft_handle *h, int64_t *perm_out) {
    CHECK_HANDLE(h);
    if (!perm_out) return fail(h, FT_EINVAL, "perm_out is NULL");
    if (!h->prepared) return fail(h, FT_ESTATE, "no prepared epoch");
    const int64_t nnz = h->nnz[FT_TRAIN];
    std::vector<uint32_t> p((size_t)nnz);
    HIPCHK(h, hipMemcpyAsync(p.data(), h->eb[h->cur].perm, sizeof(uint32_t) * nnz,
                             hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    for (int64_t i = 0; i < nnz; ++i) perm_out[i] = p[(size_t)i];
    return FT_OK;
}

extern "C" ft_status ft_get_minibatch_sort(ft_handle *h, int64_t b, int mode,
                                           int32_t *pos, int32_t *rows) {
    CHECK_HANDLE(h);
    if (!h->prepared) return fail(h, FT_ESTATE, "no prepared epoch");
    const int64_t nmb = nminibatches(h);
    if (b < 0 || b >= nmb || mode < 0 || mode >= h->N || !pos || !rows)
        return fail(h, FT_EINVAL, "bad minibatch/mode/buffers");
    const int64_t off = b * h->opt.minibatch;
    const int64_t m = std::min<int64_t>(h->opt.minibatch, h->nnz[FT_TRAIN] - off);
    // the builder keeps, per position, its sorted index; invert it here
    std::vector<uint32_t> inv((size_t)m);
    const EpochBufs &E = h->eb[h->cur];
    HIPCHK(h, hipMemcpyAsync(inv.data(), E.inv[mode] + off,
                             sizeof(uint32_t) * m, hipMemcpyDeviceToHost,
                             h->stream));
    HIPCHK(h, hipMemcpyAsync(rows, E.sk[E.sort_final[mode]][mode] + off,
                             sizeof(int32_t) * m, hipMemcpyDeviceToHost,
                             h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    for (int64_t p = 0; p < m; ++p) {
        if (inv[p] >= (uint64_t)m)
            return fail(h, FT_EDEVICE, "inverse sort index out of range");
        pos[inv[p]] = (int32_t)p;
    }
    return FT_OK;
}

// ------------------------------------------------------------------ profiling
extern "C" ft_status ft_profile_enable(ft_handle *h, int32_t on) {
    CHECK_HANDLE(h);
    h->prof = on != 0;
    return FT_OK;
}

extern "C" ft_status ft_profile_reset(ft_handle *h) {
    CHECK_HANDLE(h);
    ft_status st = prof_collect(h);
    for (int k = 0; k < FT_K_COUNT; ++k) {
        h->launches[k] = 0;
        h->ms[k] = 0.0;
    }
    return st;
}

extern "C" ft_status ft_profile_get(ft_handle *h, int32_t kernel,
                                    int64_t *launches, double *total_ms) {
    CHECK_HANDLE(h);
    if (kernel < 0 || kernel >= FT_K_COUNT || !launches || !total_ms)
        return fail(h, FT_EINVAL, "bad kernel id or output");
    ft_status st = prof_collect(h);
    if (st != FT_OK) return st;
    *launches = h->launches[kernel];
    *total_ms = h->ms[kernel];
    return FT_OK;
}

// ------------------------------------------------------------------ stateless
namespace {
struct MbLayout {
    size_t bpad, G, P, sk0, sk1, sv0, sv1, inv, counts, xlist, plist, xcount,
        ordinal,
        tile_count, total, core_part, dpart, bytes;
    int xcap, pcap;
    int tps, nch, ntiles_scan, nb_core, nb_fact, nb_eval;
    Shape sh;
};

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

ft_status check_desc(const ft_problem_desc *p, int64_t m) {
    if (!p) return fail(nullptr, FT_EINVAL, "problem descriptor is NULL");
    if (p->order < 2 || p->order > kMaxOrder)
        return fail(nullptr, FT_EINVAL, "order must be in [2, %d], got %d",
                    kMaxOrder, p->order);
    for (int n = 0; n < p->order; ++n) {
        if (p->dims[n] < 1 || p->dims[n] > 0x7fffffffll)
            return fail(nullptr, FT_EINVAL, "dims[%d] out of [1, 2^31)", n);
        if (p->J[n] < 1 || p->J[n] > kMaxJ)
            return fail(nullptr, FT_EINVAL, "J[%d] out of [1, %d]", n, kMaxJ);
    }
    if (p->R < 1 || p->R > kMaxR)
        return fail(nullptr, FT_EINVAL, "R out of [1, %d]", kMaxR);
    {
        int jmax = 0;
        for (int n = 0; n < p->order; ++n) jmax = std::max(jmax, (int)p->J[n]);
        if (!high_order_fits(p->order, padded_j4(p->order, jmax),
                             (p->R + 15) / 16 * 16))
            return fail(nullptr, FT_EINVAL,
                        "order %d: order x J4 x R16 exceeds %d", p->order,
                        kHighOrderTile);
    }
    if (m < 1 || m > (1ll << 30))
        return fail(nullptr, FT_EINVAL, "m must be in [1, 2^30], got %lld",
                    (long long)m);
    return FT_OK;
}

MbLayout mb_layout(const ft_problem_desc *p, int64_t m) {
    MbLayout L{};
    int jmax = 0;
    for (int n = 0; n < p->order; ++n) jmax = std::max(jmax, (int)p->J[n]);
    L.sh.N = p->order;
    L.sh.J4 = padded_j4(p->order, jmax);
    L.sh.R16 = (p->R + 15) / 16 * 16;
    const size_t N = (size_t)p->order, J4 = L.sh.J4, R16 = L.sh.R16;
    L.tps = (int)((m + kSortTile - 1) / kSortTile);
    L.nch = (int)((m + kSegChunk - 1) / kSegChunk);
    L.ntiles_scan = (int)((m + 2047) / 2048);
    L.nb_core = core_grad_blocks(m);
    L.nb_fact = factor_grad_blocks(L.sh, (int32_t)m);
    L.nb_eval = eval_blocks(m);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += align256(bytes);
        return o;
    };
    L.bpad = take(sizeof(float) * N * J4 * R16);
    L.G = take(sizeof(float) * N * m * J4);
    L.sk0 = take(sizeof(uint32_t) * N * m);
    L.sk1 = take(sizeof(uint32_t) * N * m);
    L.sv0 = take(sizeof(uint32_t) * N * m);
    L.sv1 = take(sizeof(uint32_t) * N * m);
    L.inv = take(sizeof(uint32_t) * N * m);
    L.counts = take(sizeof(uint32_t) * sort_counts_words((int)N, 1, L.tps));
    L.xcap = cross_capacity(m);
    L.xlist = take(sizeof(int4) * N * L.xcap);
    L.pcap = part_capacity(m, L.sh.J4);
    L.plist = take(sizeof(int4) * N * L.pcap);
    L.P = take(sizeof(float) * N * L.pcap * J4);
    L.xcount = take(sizeof(int32_t) * N * kXCounts);
    L.ordinal = take(sizeof(uint32_t) * N * m);
    L.tile_count = take(sizeof(uint32_t) * N * L.ntiles_scan);
    L.total = take(sizeof(int64_t) * N);
    L.core_part = take(sizeof(float) * L.nb_core * N * J4 * R16);
    L.dpart = take(sizeof(double) *
                   std::max<size_t>(2 * L.nb_eval,
                                    std::max(L.nb_fact, L.nb_core)) + 64);
    L.bytes = off;
    return L;
}

template <typename T>
T *at(void *ws, size_t off) {
    return reinterpret_cast<T *>(static_cast<char *>(ws) + off);
}

#define HIPCHK0(expr) HIPCHK(nullptr, expr)

ft_status pad_cores(const ft_problem_desc *p, const MbLayout &L,
                    const float *const *B, void *ws, hipStream_t s,
                    const float **Bp) {
    for (int n = 0; n < p->order; ++n) {
        float *dst = at<float>(ws, L.bpad) + (size_t)n * L.sh.J4 * L.sh.R16;
        HIPCHK0(launch_pad_matrix(B[n], p->J[n], p->R, dst, L.sh.J4, L.sh.R16,
                                  s));
        Bp[n] = dst;
    }
    return FT_OK;
}
}  // namespace

extern "C" ft_status ft_mb_workspace_size(const ft_problem_desc *p, int64_t m,
                                          size_t *bytes) {
    ft_status st = check_desc(p, m);
    if (st != FT_OK) return st;
    if (!bytes) return fail(nullptr, FT_EINVAL, "bytes is NULL");
    *bytes = mb_layout(p, m).bytes;
    return FT_OK;
}

static ft_status check_mb_inputs(const ft_problem_desc *p,
                                 const float *const *A, const float *const *B,
                                 const int32_t *const *idx, const float *val,
                                 int64_t m) {
    ft_status st = check_desc(p, m);
    if (st != FT_OK) return st;
    if (!A || !B || !idx || !val)
        return fail(nullptr, FT_EINVAL, "A, B, idx or val is NULL");
    for (int n = 0; n < p->order; ++n) {
        if (!A[n] || !B[n] || !idx[n])
            return fail(nullptr, FT_EINVAL, "A[%d], B[%d] or idx[%d] is NULL",
                        n, n, n);
        if (reinterpret_cast<uintptr_t>(A[n]) % 16)
            return fail(nullptr, FT_EINVAL, "A[%d] is not 16-byte aligned", n);
    }
    return FT_OK;
}

static ft_status check_mb_args(const ft_problem_desc *p, const float *const *A,
                               const float *const *B, const int32_t *const *idx,
                               const float *val, int64_t m, void *ws,
                               size_t ws_bytes) {
    ft_status st = check_mb_inputs(p, A, B, idx, val, m);
    if (st != FT_OK) return st;
    if (!ws) return fail(nullptr, FT_EINVAL, "workspace is NULL");
    if (reinterpret_cast<uintptr_t>(ws) % 256)
        return fail(nullptr, FT_EINVAL, "workspace is not 256-byte aligned");
    const size_t need = mb_layout(p, m).bytes;
    if (ws_bytes < need)
        return fail(nullptr, FT_EINVAL, "workspace of %zu bytes < %zu needed",
                    ws_bytes, need);
    return FT_OK;
}

extern "C" ft_status ft_mb_forward(const ft_problem_desc *p,
                                   const float *const *A, const float *const *B,
                                   const int32_t *const *idx, const float *val,
                                   int64_t m, double *loss_dev, void *workspace,
                                   size_t ws_bytes, void *hip_stream) {
    ft_status st = check_mb_args(p, A, B, idx, val, m, workspace, ws_bytes);
    if (st != FT_OK) return st;
    if (!loss_dev) return fail(nullptr, FT_EINVAL, "loss_dev is NULL");
    hipStream_t s = (hipStream_t)hip_stream;
    const MbLayout L = mb_layout(p, m);
    const float *Bp[kMaxOrder] = {};
    st = pad_cores(p, L, B, workspace, s, Bp);
    if (st != FT_OK) return st;
    EvalArgs ea{};
    for (int n = 0; n < p->order; ++n) {
        ea.idx[n] = idx[n];
        ea.A[n] = A[n];
        ea.B[n] = Bp[n];
    }
    ea.val = val;
    ea.count = m;
    ea.part = at<double>(workspace, L.dpart);
    ea.half_square = 1;
    HIPCHK0(launch_eval(L.sh, ea, L.nb_eval, s));
    HIPCHK0(launch_sum_blocks(ea.part, L.nb_eval, 1, loss_dev, s));
    return FT_OK;
}

static ft_status check_backward_outputs(const ft_problem_desc *p,
                                        float *const *gradA,
                                        int32_t *const *uniq_rows,
                                        float *const *uniq_grad,
                                        int64_t *n_uniq_dev,
                                        float *const *gradB) {
    if (!gradB) return fail(nullptr, FT_EINVAL, "gradB is NULL");
    const bool sparse = uniq_rows && uniq_grad && n_uniq_dev;
    if ((uniq_rows || uniq_grad || n_uniq_dev) && !sparse)
        return fail(nullptr, FT_EINVAL,
                    "the sparse form needs uniq_rows, uniq_grad and n_uniq_dev");
    for (int n = 0; n < p->order; ++n) {
        if (!gradB[n]) return fail(nullptr, FT_EINVAL, "gradB[%d] is NULL", n);
        if (gradA && !gradA[n])
            return fail(nullptr, FT_EINVAL, "gradA[%d] is NULL", n);
        if (sparse && (!uniq_rows[n] || !uniq_grad[n]))
            return fail(nullptr, FT_EINVAL, "uniq_rows/grad[%d] is NULL", n);
    }
    return FT_OK;
}

// The backward kernels of one minibatch on the stream s, with every
// intermediate in the workspace ws (mb_layout(p, m).bytes, 256-byte
// aligned). Arguments are already validated.
static ft_status mb_backward_run(
    const ft_problem_desc *p, const float *const *A, const float *const *B,
    const int32_t *const *idx, const float *val, int64_t m,
    const float *grad_out_dev, float *const *gradA, int32_t *const *uniq_rows,
    float *const *uniq_grad, int64_t *n_uniq_dev, float *const *gradB,
    void *workspace, hipStream_t s) {
    const bool sparse = uniq_rows && uniq_grad && n_uniq_dev;
    ft_status st = FT_OK;
    const MbLayout L = mb_layout(p, m);
    const int N = p->order;
    const float *Bp[kMaxOrder] = {};
    st = pad_cores(p, L, B, workspace, s, Bp);
    if (st != FT_OK) return st;

    // per-sample row gradients (c, d recomputed)
    FactorArgs fa{};
    for (int n = 0; n < N; ++n) {
        fa.idx[n] = idx[n];
        fa.A[n] = A[n];
        fa.B[n] = Bp[n];
    }
    fa.val = val;
    fa.m = (int32_t)m;
    fa.G = at<float>(workspace, L.G);
    fa.loss_part = at<double>(workspace, L.dpart);
    uint32_t *inv = at<uint32_t>(workspace, L.inv);
    for (int n = 0; n < N; ++n) fa.inv[n] = inv + (size_t)n * m;

    // sort the minibatch's rows per mode (one segment); the last pass also
    // gives the sorted slot of every sample, where its gradients go
    SortPass sp{};
    sp.N = N;
    sp.nnz = m;
    sp.M = m;
    sp.nseg = 1;
    sp.tiles_per_seg = L.tps;
    sp.counts = at<uint32_t>(workspace, L.counts);
    uint32_t *sk[2] = {at<uint32_t>(workspace, L.sk0),
                       at<uint32_t>(workspace, L.sk1)};
    uint32_t *sv[2] = {at<uint32_t>(workspace, L.sv0),
                       at<uint32_t>(workspace, L.sv1)};
    int passes[kMaxOrder], cur[kMaxOrder] = {}, max_passes = 1;
    for (int n = 0; n < N; ++n) {
        passes[n] = radix_passes(p->dims[n]);
        max_passes = std::max(max_passes, passes[n]);
    }
    for (int pass = 0; pass < max_passes; ++pass) {
        sp.shift = 8 * pass;
        sp.N = 0;
        for (int n = 0; n < N; ++n) {
            if (pass >= passes[n]) continue;
            const int k = sp.N++;
            const int out = pass == 0 ? 0 : cur[n] ^ 1;
            const bool last = pass == passes[n] - 1;
            sp.key_in[k] = pass == 0 ? reinterpret_cast<const uint32_t *>(idx[n])
                                     : sk[cur[n]] + (size_t)n * m;
            sp.val_in[k] = pass == 0 ? nullptr : sv[cur[n]] + (size_t)n * m;
            sp.key_out[k] = sk[out] + (size_t)n * m;
            sp.val_out[k] = last ? nullptr : sv[out] + (size_t)n * m;
            sp.inv_out[k] = last ? inv + (size_t)n * m : nullptr;
            cur[n] = out;
        }
        HIPCHK0(launch_sort_pass(sp, s));
    }
    int nb = 0;
    HIPCHK0(launch_factor_grad(L.sh, fa, &nb, s));

    SegArgs sa{};
    sa.N = N;
    sa.J4 = L.sh.J4;
    sa.m = (int32_t)m;
    sa.nchunks = L.nch;
    sa.G = fa.G;
    sa.apply = 2;
    sa.scale = grad_out_dev;
    {
        CrossArgs cx{};
        cx.J4 = L.sh.J4;
        cx.N = N;
        cx.nnz = m;
        cx.M = m;
        cx.nseg = 1;
        cx.xcap = L.xcap;
        for (int n = 0; n < N; ++n) cx.rows[n] = sk[cur[n]] + (size_t)n * m;
        cx.xlist = at<int4>(workspace, L.xlist);
        cx.plist = at<int4>(workspace, L.plist);
        cx.pcap = L.pcap;
        cx.xcount = at<int32_t>(workspace, L.xcount);
        HIPCHK0(launch_crossing_segments(cx, s));
        sa.xcount = cx.xcount;
        sa.xcap = L.xcap;
        // worst case (surplus blocks exit): every crossing row short, every
        // part slot used, every long row in several parts
        sa.pcap = L.pcap;
        sa.P = at<float>(workspace, L.P);
        sa.small_blocks = (N * L.xcap + kSegWaves - 1) / kSegWaves;
        sa.large_blocks = N * L.pcap;
        sa.combine_blocks = (N * (int)(m / (kSmallCross + 1)) + kSegWaves - 1) /
                            kSegWaves;
        for (int n = 0; n < N; ++n) {
            sa.xlist[n] = cx.xlist + (size_t)n * L.xcap;
            sa.plist[n] = cx.plist + (size_t)n * L.pcap;
        }
    }
    for (int n = 0; n < N; ++n) {
        sa.rows[n] = sk[cur[n]] + (size_t)n * m;
        sa.A[n] = const_cast<float *>(A[n]);
        sa.grad[n] = gradA ? gradA[n] : nullptr;
        if (gradA)
            HIPCHK0(launch_fill_zero(gradA[n], p->dims[n] * L.sh.J4, s));
    }
    if (sparse) {
        UniqueScan u{};
        u.N = N;
        u.m = (int32_t)m;
        u.ntiles = L.ntiles_scan;
        u.tile_count = at<uint32_t>(workspace, L.tile_count);
        u.total = n_uniq_dev;
        for (int n = 0; n < N; ++n) {
            u.rows[n] = sa.rows[n];
            u.ordinal[n] = at<uint32_t>(workspace, L.ordinal) + (size_t)n * m;
            sa.ordinal[n] = u.ordinal[n];
            sa.uniq_rows[n] = uniq_rows[n];
            sa.uniq_grad[n] = uniq_grad[n];
        }
        HIPCHK0(launch_unique_scan(u, s));
    }
    HIPCHK0(launch_seg_reduce(sa, s));
    HIPCHK0(launch_seg_combine(sa, s));

    // core gradients over the minibatch
    CoreArgs ca{};
    for (int n = 0; n < N; ++n) {
        ca.idx[n] = idx[n];
        ca.A[n] = A[n];
        ca.B[n] = Bp[n];
    }
    ca.val = val;
    ca.count = m;
    ca.part = at<float>(workspace, L.core_part);
    ca.loss_part = at<double>(workspace, L.dpart);
    int used = L.nb_core;
    ca.blocks_used = &used;
    HIPCHK0(launch_core_grad(L.sh, ca, L.nb_core, s));
    CoreUpdateArgs ua{};
    ua.part = ca.part;
    ua.nblocks = used;
    ua.apply = 0;
    ua.R = p->R;
    ua.scale = grad_out_dev;
    for (int n = 0; n < N; ++n) {
        ua.gout[n] = gradB[n];
        ua.Jn[n] = p->J[n];
    }
    HIPCHK0(launch_core_update(L.sh, ua, s));
    return FT_OK;
}

extern "C" ft_status ft_mb_backward(
    const ft_problem_desc *p, const float *const *A, const float *const *B,
    const int32_t *const *idx, const float *val, int64_t m,
    const float *grad_out_dev, float *const *gradA, int32_t *const *uniq_rows,
    float *const *uniq_grad, int64_t *n_uniq_dev, float *const *gradB,
    void *workspace, size_t ws_bytes, void *hip_stream) {
    ft_status st = check_mb_args(p, A, B, idx, val, m, workspace, ws_bytes);
    if (st != FT_OK) return st;
    st = check_backward_outputs(p, gradA, uniq_rows, uniq_grad, n_uniq_dev,
                                gradB);
    if (st != FT_OK) return st;
    return mb_backward_run(p, A, B, idx, val, m, grad_out_dev, gradA,
                           uniq_rows, uniq_grad, n_uniq_dev, gradB, workspace,
                           (hipStream_t)hip_stream);
}

// ------------------------------------------------- allocation-free backward
// Workspace of ft_mb_backward_noalloc: one array per device, resident from
// the library's first use on that device until the process ends. In host
// code the array's name is not a device address; its address on the current
// device comes from hipGetSymbolAddress, taken once per device and kept in
// g_scratch_dev.
static __device__ __align__(256) unsigned char scratch[FT_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_dev[kScratchDevices] = {};
}  // namespace

static ft_status scratch_on_current_device(void **out) {
    int dev = -1;
    HIPCHK0(hipGetDevice(&dev));
    if (dev < 0 || dev >= kScratchDevices)
        return fail(nullptr, FT_EDEVICE, "device %d beyond the %d supported",
                    dev, kScratchDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(nullptr, FT_EDEVICE,
                        "hipGetSymbolAddress(scratch) on device %d: %s", dev,
                        hipGetErrorString(e));
        g_scratch_dev[dev] = ptr;
    }
    *out = g_scratch_dev[dev];
    return FT_OK;
}

extern "C" ft_status ft_mb_backward_noalloc(
    const ft_problem_desc *p, const float *const *A, const float *const *B,
    const int32_t *const *idx, const float *val, int64_t m,
    const float *grad_out_dev, float *const *gradA, int32_t *const *uniq_rows,
    float *const *uniq_grad, int64_t *n_uniq_dev, float *const *gradB,
    void *hip_stream) {
    ft_status st = check_mb_inputs(p, A, B, idx, val, m);
    if (st != FT_OK) return st;
    st = check_backward_outputs(p, gradA, uniq_rows, uniq_grad, n_uniq_dev,
                                gradB);
    if (st != FT_OK) return st;
    const size_t need = mb_layout(p, m).bytes;
    if (need > (size_t)FT_NOALLOC_SCRATCH_BYTES)
        return fail(nullptr, FT_EINVAL,
                    "minibatch needs %zu bytes of workspace, more than the "
                    "%zu of the static scratch (use ft_mb_backward)",
                    need, (size_t)FT_NOALLOC_SCRATCH_BYTES);
    void *ws = nullptr;
    st = scratch_on_current_device(&ws);
    if (st != FT_OK) return st;
    return mb_backward_run(p, A, B, idx, val, m, grad_out_dev, gradA,
                           uniq_rows, uniq_grad, n_uniq_dev, gradB, ws,
                           (hipStream_t)hip_stream);
}
