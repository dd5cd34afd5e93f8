// kmeans_api.hip -- host runtime behind include/kmeans.h: contexts, argument
// validation, device workspace, the iteration loop (hipGraph replays with one
// status read-back per batch of iterations) and result read-back.
#include "ctx.h"
#include "wide.h"

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <map>
#include <string>
#include <tuple>
#include <vector>

using km::State;

using km::fail;
using km::check_device_ptr;
using km::ensure_hist;
using km::ensure_events;

namespace {
thread_local std::string g_create_error;
}  // namespace

int km::fail(kmeans_ctx* c, int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c) c->err = buf;
    else g_create_error = buf;
    return code;
}

int km::check_device_ptr(kmeans_ctx* c, const void* p, const char* what) {
    if (!p) return fail(c, KM_EINVAL, "%s is NULL", what);
    hipPointerAttribute_t a;
    if (hipPointerGetAttributes(&a, p) != hipSuccess) {
        (void)hipGetLastError();
        return fail(c, KM_EINVAL, "%s is not a HIP device pointer", what);
    }
    if (a.type != hipMemoryTypeDevice && a.type != hipMemoryTypeManaged)
        return fail(c, KM_EINVAL, "%s must be device memory", what);
    return KM_OK;
}

int km::ensure_hist(kmeans_ctx* c, int cap) {
    if (cap <= c->hist_cap) return KM_OK;
    int n = c->hist_cap ? c->hist_cap : 256;
    while (n < cap) n *= 2;
    double* dv = nullptr;
    double* hv = nullptr;
    if (hipMalloc(&dv, sizeof(double) * 3 * (size_t)n) != hipSuccess)
        return fail(c, KM_ENOMEM, "hipMalloc of the history (%d entries) failed", n);
    if (hipHostMalloc(&hv, sizeof(double) * 3 * (size_t)n, 0) != hipSuccess) {
        (void)hipFree(dv);
        return fail(c, KM_ENOMEM, "hipHostMalloc of the history failed");
    }
    if (c->hist) {
        (void)hipStreamSynchronize(c->stream);
        (void)hipFree(c->hist);
        (void)hipHostFree(c->hist_h);
    }
    c->hist = dv;
    c->hist_h = hv;
    c->hist_cap = n;
    return KM_OK;
}

int km::ensure_events(kmeans_ctx* c, size_t n) {
    while (c->ev.size() < n) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return fail(c, KM_EHIP, "hipEventCreate failed");
        c->ev.push_back(e);
    }
    return KM_OK;
}

int km::range_error(kmeans_ctx* c) {
    return fail(c, KM_EUNSUPPORTED,
                "max|x| >= 2^28: the fixed-point cluster sums (|x| 2^F < 2^44) would not "
                "guarantee the centres to 1e-5 of a cluster near the origin; scale the data");
}

bool km::wide_shape(const kmeans_ctx* c, int d, int K) {
    return c->wide != 0 || (d != 2 && d != 3) || K > km::KMAX;
}

int km::validate(kmeans_ctx* c, int64_t N, int64_t ld, int32_t d, int32_t K, double tol,
             int32_t max_iter) {
    if (N < 1 || N > 2147483647LL) return fail(c, KM_EINVAL, "N=%lld out of [1, 2^31-1]", (long long)N);
    if (ld < N) return fail(c, KM_EINVAL, "ld=%lld < N=%lld", (long long)ld, (long long)N);
    if (d < 1) return fail(c, KM_EINVAL, "d=%d < 1", d);
    if (d > km::WD_MAX) return fail(c, KM_EUNSUPPORTED, "d=%d > %d", d, km::WD_MAX);
    if (K < 1) return fail(c, KM_EINVAL, "K=%d < 1", K);
    if (K > km::WK_MAX) return fail(c, KM_EUNSUPPORTED, "K=%d > %d", K, km::WK_MAX);
    if (K > N) return fail(c, KM_EINVAL, "K=%d > N=%lld", K, (long long)N);
    if (!(tol >= 0.0) || !isfinite(tol)) return fail(c, KM_EINVAL, "tol must be finite and >= 0");
    if (max_iter < 1) return fail(c, KM_EINVAL, "max_iter=%d < 1", max_iter);
    return KM_OK;
}

int km::check_centres(kmeans_ctx* c, const double* m, int K, int d, const char* what) {
    if (!m) return fail(c, KM_EINVAL, "%s is NULL", what);
    for (int i = 0; i < K * d; ++i)
        if (!isfinite(m[i])) return fail(c, KM_EINVAL, "%s[%d] is not finite", what, i);
    return KM_OK;
}

bool km::vec_ok(const float* X, int64_t ld) {
    return (reinterpret_cast<uintptr_t>(X) & 15u) == 0 && (ld & 3) == 0;
}

// Grid of the per-update kernels: about one block per 8192 points, at least
// 2 and at most 16 per compute unit, and never more blocks than groups of 4
// points per thread.  Each block has a fixed cost per update (staging the
// centre tables, clearing its accumulators, its partial and its share of the
// reduction), so blocks with few points lose: measured per update at K = 16,
// N = 4e6: 512 blocks 37.2 us, 3907 blocks 46.9 us; N = 1e7: 1024 blocks
// 52.9 us, 4096 blocks 64.7 us; at N = 2e8, K = 64 the 16 per unit cap
// (4096 blocks) is best.  Whatever the cap (KM_OPT_BLOCKS included), the grid
// is at least min_blocks(N), so that no block adds more than
// FXP_BLOCK_POINTS points into its int64 sums.
int64_t km::min_blocks(int64_t N) {
    const int64_t groups = (N + 3) / 4;
    const int64_t per_block = km::FXP_BLOCK_POINTS / 4;  // groups of 4 points
    return (groups + per_block - 1) / per_block;
}

int km::grid_blocks(int n_cu, int blocks_opt, int64_t N) {
    const int64_t groups = (N + 3) / 4;
    const int64_t need = (groups + km::BLOCK - 1) / km::BLOCK;
    int64_t cap;
    if (blocks_opt > 0) {
        cap = blocks_opt;
    } else {
        const int64_t lo = (int64_t)n_cu * 2, hi = (int64_t)n_cu * 16;
        const int64_t want = (N + 8191) / 8192;
        cap = want < lo ? lo : (want > hi ? hi : want);
    }
    if (cap > km::MAX_BLOCKS) cap = km::MAX_BLOCKS;
    int64_t g = need < cap ? need : cap;
    const int64_t lo = min_blocks(N);  // <= MAX_BLOCKS for N < 2^31
    if (g < lo) g = lo;
    return (int)(g < 1 ? 1 : g);
}

// Fill a host copy of the state for a problem and its centres.
void km::stage_state(State* h, const FitBufs& b, const float* X, int64_t N, int64_t ld, int d,
                     int K, const double* mu, double tol, int max_iter) {
    memset(h, 0, km::kUploadBytes);
    h->X = X;
    h->N = N;
    h->ld = ld;
    h->d = d;
    h->K = K;
    h->tol = tol;
    h->max_iter = max_iter;
    h->hist_cap = b.hist_cap;
    h->jpart = b.jpart;
    h->part = b.part;
    h->gpart = b.gpart;
    h->gjpart = b.gjpart;
    h->gticket = b.gticket;
    h->E_hist = b.hist;
    h->J_hist = b.hist + b.hist_cap;
    h->C_hist = b.chist;
    h->track = nullptr;
    h->E = INFINITY;
    h->minus_inf = -INFINITY;
    for (int k = 0; k < K; ++k) {
        float m[3] = {0.f, 0.f, 0.f};
        for (int j = 0; j < d; ++j) {
            h->mu64[k * d + j] = mu[k * d + j];
            m[j] = (float)mu[k * d + j];  // round to nearest even
        }
        h->mu32[k] = make_float4(m[0], m[1], m[2], 0.f);
    }
}

namespace {

using km::validate;
using km::check_centres;
using km::vec_ok;
using km::min_blocks;

int grid_for(kmeans_ctx* c, int64_t N) { return km::grid_blocks(c->n_cu, c->blocks, N); }

void stage(kmeans_ctx* c, const float* X, int64_t N, int64_t ld, int d, int K,
           const double* mu, double tol, int max_iter) {
    const km::FitBufs b{c->jpart, c->part,  c->gpart, c->gjpart, c->gticket,
                        c->hist,  reinterpret_cast<int64_t*>(c->hist + 2 * (size_t)c->hist_cap),
                        c->hist_cap};
    km::stage_state(c->st_h, b, X, N, ld, d, K, mu, tol, max_iter);
}

int get_graph(kmeans_ctx* c, int d, bool vec, int keys, bool track, int grid, int unroll,
              hipGraphExec_t* out) {
    km::GraphKey key{d, vec ? 1 : 0, keys, track ? 1 : 0, grid, unroll};
    auto it = c->graphs.find(key);
    if (it != c->graphs.end()) {
        *out = it->second;
        return KM_OK;
    }
    hipGraph_t g = nullptr;
    KM_HIP(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
    for (int i = 0; i < unroll; ++i) {
        hipError_t e = km::launch_iter(c->st, d, vec, keys, track, grid, c->cap_stream);
        if (e != hipSuccess) {
            hipGraph_t junk = nullptr;
            (void)hipStreamEndCapture(c->cap_stream, &junk);
            if (junk) (void)hipGraphDestroy(junk);
            return fail(c, KM_EHIP, "capture of the iteration kernel failed: %s", hipGetErrorString(e));
        }
    }
    KM_HIP(c, hipStreamEndCapture(c->cap_stream, &g));
    hipGraphExec_t ex = nullptr;
    hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return fail(c, KM_EHIP, "hipGraphInstantiate failed: %s", hipGetErrorString(e));
    c->graphs[key] = ex;
    *out = ex;
    return KM_OK;
}

int run_iterations(kmeans_ctx* c, int d, bool vec, int keys, bool track, int grid, int n_iter) {
    if (c->use_graph) {
        hipGraphExec_t ex;
        int rc = get_graph(c, d, vec, keys, track, grid, n_iter, &ex);
        if (rc) return rc;
        KM_HIP(c, hipGraphLaunch(ex, c->stream));
    } else {
        for (int i = 0; i < n_iter; ++i)
            KM_HIP(c, km::launch_iter(c->st, d, vec, keys, track, grid, c->stream));
    }
    return KM_OK;
}

// Scan variant for K centres (scan_keys): the matrix-core keys take the 3 d
// FMAs per centre off the VALU, leaving it the argmin tracking (five
// instructions per quad of centres) and a fixed per-point cost (operands,
// merge, re-keying the winning quad); at N = 2e8, K = 64 1203 vs 1547 us per
// update on one box.  The VALU scan stays faster for small K.
// Persistent fit: only when selected (KM_OPT_PERSIST = 2).  With the grid
// of grid_for, the launch per update is as fast or faster at every size
// measured (K = 16, per update: N = 1e6 22.3 vs 26.0 us, 4e6 37.3 vs 41.0 us,
// 1e7 58.8 vs 60.1 us, 1.6e7 82.6 vs 83.1 us, 4e7 181 vs 184 us): both are
// bound by the same chain of device-wide round trips of the reduction, and
// the persistent fit adds a grid-wide wait per update.
bool use_persist(kmeans_ctx* c, int64_t N, int keys) {
    (void)N;
    return keys == 0 && c->persist == 2 && !c->track;
}

int scan_keys(kmeans_ctx* c, int K) {
    if (c->keys == 1) return 0;
    if (c->keys == 2) return K > 32 ? 2 : 1;
    return km::auto_keys(K);
}

}  // namespace

// The matrix-core scan where it was measured faster (N = 5e7, d = 3, per
// update: K = 24 264 vs 273 us VALU vs matrix cores, 32 285 vs 275, 40 334
// vs 345, 48 366 vs 347, 64 444 vs 363): its cost per point hardly depends
// on K within a tile of 32 centres, the VALU scan's grows with K.
int km::auto_keys(int K) {
    if ((K > 24 && K <= 32) || K > 44) return K > 32 ? 2 : 1;
    return 0;
}

int km::auto_unroll(int64_t N, int max_iter) {
    int u = N >= (1 << 24) ? 10 : (N >= (1 << 20) ? 16 : 32);
    return u < max_iter ? u : max_iter;
}

extern "C" {

int kmeans_abi_version(void) { return KMEANS_ABI_VERSION; }

const char* kmeans_status_string(int s) {
    switch (s) {
        case KM_OK: return "KM_OK";
        case KM_EINVAL: return "KM_EINVAL";
        case KM_ENODEV: return "KM_ENODEV";
        case KM_EHIP: return "KM_EHIP";
        case KM_ENOMEM: return "KM_ENOMEM";
        case KM_EUNSUPPORTED: return "KM_EUNSUPPORTED";
        default: return "KM_UNKNOWN";
    }
}

int kmeans_validate(int64_t N, int64_t ld, int32_t d, int32_t K, double tol, int32_t max_iter) {
    kmeans_ctx tmp;
    return validate(&tmp, N, ld, d, K, tol, max_iter);
}

const char* kmeans_last_error(const kmeans_ctx* ctx) {
    return ctx ? ctx->err.c_str() : g_create_error.c_str();
}

int kmeans_create(kmeans_ctx** out, int device, void* hip_stream, uint32_t flags) {
    if (!out) return fail(nullptr, KM_EINVAL, "out is NULL");
    *out = nullptr;
    if (flags != 0) return fail(nullptr, KM_EINVAL, "flags must be 0");
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess || n < 1) {
        (void)hipGetLastError();
        return fail(nullptr, KM_ENODEV, "no HIP device available (%s)", hipGetErrorString(e));
    }
    if (device < 0 || device >= n) return fail(nullptr, KM_ENODEV, "device %d out of range [0, %d)", device, n);
    if (hipSetDevice(device) != hipSuccess) return fail(nullptr, KM_ENODEV, "hipSetDevice(%d) failed", device);
    kmeans_ctx* c = new kmeans_ctx();
    c->device = device;
    c->stream = (hipStream_t)hip_stream;
    int rc = KM_OK;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess && prop.multiProcessorCount > 0)
        c->n_cu = prop.multiProcessorCount;
    if (hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking) != hipSuccess) {
        rc = fail(nullptr, KM_EHIP, "stream/event creation failed");
    } else if (hipMalloc(&c->st, sizeof(State)) != hipSuccess ||
               hipMalloc(&c->jpart, sizeof(double) * km::MAX_BLOCKS) != hipSuccess ||
               hipMalloc(&c->part, sizeof(unsigned long long) * km::PART * km::MAX_BLOCKS) != hipSuccess ||
               hipMalloc(&c->gpart, sizeof(unsigned long long) * 2 * km::PART * km::MAX_GROUPS) != hipSuccess ||
               hipMalloc(&c->gjpart, sizeof(double) * km::MAX_GROUPS) != hipSuccess ||
               hipMalloc(&c->gticket, sizeof(uint32_t) * km::MAX_GROUPS) != hipSuccess) {
        rc = fail(nullptr, KM_ENOMEM, "hipMalloc of the workspace failed");
    } else if (hipMemset(c->gticket, 0, sizeof(uint32_t) * km::MAX_GROUPS) != hipSuccess ||
               hipDeviceSynchronize() != hipSuccess) {
        rc = fail(nullptr, KM_EHIP, "clearing the workspace failed");
    } else if (hipHostMalloc(&c->st_h, sizeof(State), 0) != hipSuccess) {
        rc = fail(nullptr, KM_ENOMEM, "hipHostMalloc of the staging buffer failed");
    } else if (ensure_hist(c, 256) != KM_OK) {
        rc = fail(nullptr, KM_ENOMEM, "%s", c->err.c_str());
    }
    if (rc != KM_OK) {
        kmeans_destroy(c);
        return rc;
    }
    *out = c;
    return KM_OK;
}

void kmeans_destroy(kmeans_ctx* c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    for (auto& kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
    if (c->st) (void)hipFree(c->st);
    if (c->jpart) (void)hipFree(c->jpart);
    if (c->part) (void)hipFree(c->part);
    if (c->gpart) (void)hipFree(c->gpart);
    if (c->gjpart) (void)hipFree(c->gjpart);
    if (c->gticket) (void)hipFree(c->gticket);
    if (c->hist) (void)hipFree(c->hist);
    if (c->st_h) (void)hipHostFree(c->st_h);
    if (c->hist_h) (void)hipHostFree(c->hist_h);
    for (auto& e : c->ev) (void)hipEventDestroy(e);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    if (c->bws) km::batched_ws_free(c->bws);
    if (c->nws) km::net_ws_free(c->nws);
    if (c->sws) km::seed_ws_free(c->sws);
    if (c->wws) km::wide_ws_free(c->wws);
    delete c;
}

int kmeans_set_option(kmeans_ctx* c, int32_t option, int64_t value) {
    if (!c) return KM_EINVAL;
    switch (option) {
        case KM_OPT_GRAPH:
            if (value != 0 && value != 1) return fail(c, KM_EINVAL, "KM_OPT_GRAPH takes 0 or 1");
            c->use_graph = (int)value;
            return KM_OK;
        case KM_OPT_UNROLL:
            if (value < 0 || value > 1024) return fail(c, KM_EINVAL, "KM_OPT_UNROLL out of [0, 1024]");
            c->unroll = (int)value;
            return KM_OK;
        case KM_OPT_BLOCKS:
            if (value < 0 || value > km::MAX_BLOCKS) return fail(c, KM_EINVAL, "KM_OPT_BLOCKS out of [0, %d]", km::MAX_BLOCKS);
            c->blocks = (int)value;
            return KM_OK;
        case KM_OPT_TIMING:
            if (value != 0 && value != 1) return fail(c, KM_EINVAL, "KM_OPT_TIMING takes 0 or 1");
            c->timing = (int)value;
            return KM_OK;
        case KM_OPT_KEYS:
            if (value < 0 || value > 2) return fail(c, KM_EINVAL, "KM_OPT_KEYS takes 0, 1 or 2");
            c->keys = (int)value;
            return KM_OK;
        case KM_OPT_PERSIST:
            if (value < 0 || value > 2) return fail(c, KM_EINVAL, "KM_OPT_PERSIST takes 0, 1 or 2");
            c->persist = (int)value;
            return KM_OK;
        case KM_OPT_WIDE:
            if (value != 0 && value != 1) return fail(c, KM_EINVAL, "KM_OPT_WIDE takes 0 or 1");
            c->wide = (int)value;
            return KM_OK;
        case KM_OPT_TRACK:
            if (value != 0 && value != 1) return fail(c, KM_EINVAL, "KM_OPT_TRACK takes 0 or 1");
            c->track = (int)value;
            return KM_OK;
        default:
            return fail(c, KM_EINVAL, "unknown option %d", option);
    }
}

int kmeans_assign(kmeans_ctx* c, const float* X, int64_t N, int64_t ld, int32_t d, int32_t K,
                  const double* centroids, int32_t* labels, double* objective) {
    if (!c) return KM_EINVAL;
    c->err.clear();
    int rc = validate(c, N, ld, d, K, 0.0, 1);
    if (!rc) rc = check_device_ptr(c, X, "X");
    if (!rc && labels) rc = check_device_ptr(c, labels, "labels");
    if (!rc) rc = check_centres(c, centroids, K, d, "centroids");
    if (rc) return rc;
    KM_HIP(c, hipSetDevice(c->device));
    if (km::wide_shape(c, d, K)) return km::wide_assign(c, X, N, ld, d, K, centroids, labels, objective);
    const bool vec = vec_ok(X, ld);
    const int grid = grid_for(c, N);
    stage(c, X, N, ld, d, K, centroids, 0.0, 1);
    KM_HIP(c, hipMemcpyAsync(c->st, c->st_h, km::kUploadBytes, hipMemcpyHostToDevice, c->stream));
    KM_HIP(c, km::launch_scan(c->st, d, vec, grid, c->stream));
    KM_HIP(c, km::launch_label(c->st, labels, d, vec, scan_keys(c, K), grid, c->stream));
    KM_HIP(c, hipMemcpyAsync(reinterpret_cast<char*>(c->st_h) + km::kProgressOffset,
                             reinterpret_cast<char*>(c->st) + km::kProgressOffset,
                             km::kProgressBytes, hipMemcpyDeviceToHost, c->stream));
    KM_HIP(c, hipStreamSynchronize(c->stream));
    if (c->st_h->flags & km::FLAG_NONFINITE) return fail(c, KM_EINVAL, "X holds a NaN or an infinity");
    if (objective) *objective = c->st_h->J;
    return KM_OK;
}

int kmeans_fit(kmeans_ctx* c, const float* X, int64_t N, int64_t ld, int32_t d, int32_t K,
               const double* init, double tol, int32_t max_iter, double* centroids_out,
               int32_t* labels_out, km_result* res) {
    if (!c) return KM_EINVAL;
    c->err.clear();
    int rc = validate(c, N, ld, d, K, tol, max_iter);
    if (!rc) rc = check_device_ptr(c, X, "X");
    if (!rc && labels_out) rc = check_device_ptr(c, labels_out, "labels_out");
    if (!rc) rc = check_centres(c, init, K, d, "init");
    if (!rc && !centroids_out) rc = fail(c, KM_EINVAL, "centroids_out is NULL");
    if (!rc && c->track && !labels_out)
        rc = fail(c, KM_EINVAL, "KM_OPT_TRACK needs labels_out (the tracked labels live there)");
    if (rc) return rc;
    KM_HIP(c, hipSetDevice(c->device));
    c->last_track = c->track;
    if (km::wide_shape(c, d, K))
        return km::wide_fit(c, X, N, ld, d, K, init, tol, max_iter, centroids_out, labels_out, res);
    rc = ensure_hist(c, max_iter);
    if (rc) return rc;
    const bool vec = vec_ok(X, ld);
    const int grid = grid_for(c, N);
    const int U = c->unroll > 0 ? (c->unroll < max_iter ? c->unroll : max_iter) : km::auto_unroll(N, max_iter);

    const bool track = c->track != 0;
    stage(c, X, N, ld, d, K, init, tol, max_iter);
    if (track) {
        // no label before the first update: every point counts as changed
        c->st_h->track = labels_out;
        KM_HIP(c, hipMemsetAsync(labels_out, 0xff, sizeof(int32_t) * (size_t)N, c->stream));
    }
    KM_HIP(c, hipMemcpyAsync(c->st, c->st_h, km::kUploadBytes, hipMemcpyHostToDevice, c->stream));
    KM_HIP(c, km::launch_scan(c->st, d, vec, grid, c->stream));

    c->iter_ms = 0.0;
    c->iter_kernels = 0;
    int launched = 0, batches = 0;
    State* h = c->st_h;
    const int keys = scan_keys(c, K);

    // Small N: the whole fit in one cooperative launch (lloyd_persist), which
    // saves a kernel launch and its cache maintenance per update.
    bool persisted = false;
    if (use_persist(c, N, keys)) {
        int& per_cu = c->persist_bpc[d == 3][vec ? 1 : 0];
        if (per_cu == 0) per_cu = km::persist_max_blocks_per_cu(d, vec);
        const int cap = c->n_cu * per_cu;
        const int pgrid = grid < cap ? grid : cap;
        if (pgrid >= 1 && pgrid >= min_blocks(N)) {
            if (c->timing) {
                rc = ensure_events(c, 2);
                if (rc) return rc;
                KM_HIP(c, hipEventRecord(c->ev[0], c->stream));
            }
            if (km::launch_persist(c->st, d, vec, pgrid, c->stream) == hipSuccess) {
                persisted = true;
                batches = 1;
                if (c->timing) KM_HIP(c, hipEventRecord(c->ev[1], c->stream));
            } else {
                (void)hipGetLastError();  // not co-resident: use the per-update launches
            }
        }
    }

    // Batches of U iterations; the device decides when to stop (kernels after
    // convergence return at once), the host reads the progress block once per
    // batch.  With tol == 0 the count is known and there is no read-back.
    while (!persisted && launched < max_iter) {
        const int n = (max_iter - launched) < U ? (max_iter - launched) : U;
        if (c->timing) {
            rc = ensure_events(c, 2 * (batches + 1));
            if (rc) return rc;
            KM_HIP(c, hipEventRecord(c->ev[2 * batches], c->stream));
        }
        rc = run_iterations(c, d, vec, keys, track, grid, n);
        if (rc) return rc;
        if (c->timing) KM_HIP(c, hipEventRecord(c->ev[2 * batches + 1], c->stream));
        launched += n;
        batches += 1;
        if ((tol > 0.0 || track) && launched < max_iter) {
            KM_HIP(c, hipMemcpyAsync(reinterpret_cast<char*>(h) + km::kProgressOffset,
                                     reinterpret_cast<char*>(c->st) + km::kProgressOffset,
                                     km::kProgressBytes, hipMemcpyDeviceToHost, c->stream));
            KM_HIP(c, hipStreamSynchronize(c->stream));
            if (h->done) break;
        }
    }
    KM_HIP(c, km::launch_label(c->st, labels_out, d, vec, keys, grid, c->stream));
    KM_HIP(c, hipMemcpyAsync(reinterpret_cast<char*>(h) + km::kProgressOffset,
                             reinterpret_cast<char*>(c->st) + km::kProgressOffset,
                             km::kUploadBytes - km::kProgressOffset, hipMemcpyDeviceToHost,
                             c->stream));
    // the E / J history of every update that may have run (T <= that count),
    // read with the results: one synchronisation per fit instead of two
    {
        const int ran = persisted ? max_iter : launched;
        const int nc = ran < c->hist_cap ? ran : c->hist_cap;
        if (nc > 0) {
            KM_HIP(c, hipMemcpyAsync(c->hist_h, c->hist, sizeof(double) * (size_t)nc,
                                     hipMemcpyDeviceToHost, c->stream));
            KM_HIP(c, hipMemcpyAsync(c->hist_h + c->hist_cap, c->hist + c->hist_cap,
                                     sizeof(double) * (size_t)nc, hipMemcpyDeviceToHost,
                                     c->stream));
            if (track)
                KM_HIP(c, hipMemcpyAsync(c->hist_h + 2 * c->hist_cap, c->hist + 2 * c->hist_cap,
                                         sizeof(double) * (size_t)nc, hipMemcpyDeviceToHost,
                                         c->stream));
        }
    }
    KM_HIP(c, hipStreamSynchronize(c->stream));
    if (h->flags & km::FLAG_TIMEOUT)
        return fail(c, KM_EHIP, "persistent fit: a block's wait for an update timed out");
    const int T = h->t;
    c->last_T = T;
    if (c->timing) {
        for (int b = 0; b < batches; ++b) {
            float ms = 0.f;
            KM_HIP(c, hipEventElapsedTime(&ms, c->ev[2 * b], c->ev[2 * b + 1]));
            c->iter_ms += ms;
        }
        c->iter_kernels = persisted ? T : launched;
    }
    if (h->flags & km::FLAG_NONFINITE) return fail(c, KM_EINVAL, "X holds a NaN or an infinity");
    if (h->flags & km::FLAG_RANGE) return km::range_error(c);
    memcpy(centroids_out, h->mu64, sizeof(double) * (size_t)K * d);
    if (res) {
        res->iters = T;
        res->converged = (h->E < tol || (track && h->changed == 0)) ? 1 : 0;
        res->E = h->E;
        res->shift_l2 = sqrt(h->E);
        res->objective = h->J;
        res->empty_events = h->empty_events;
    }
    return KM_OK;
}

int kmeans_get_changes(kmeans_ctx* c, int64_t* changed, int32_t cap) {
    if (!c || cap < 0) return KM_EINVAL;
    if (!c->last_track) return fail(c, KM_EINVAL, "the last fit did not track its indicators");
    int n = c->last_T < cap ? c->last_T : cap;
    if (n > c->hist_cap) n = c->hist_cap;
    if (changed) memcpy(changed, c->hist_h + 2 * c->hist_cap, sizeof(int64_t) * (size_t)n);
    return n;
}

int kmeans_get_history(kmeans_ctx* c, double* E, double* J, int32_t cap) {
    if (!c || cap < 0) return KM_EINVAL;
    int n = c->last_T < cap ? c->last_T : cap;
    if (n > c->hist_cap) n = c->hist_cap;
    if (E) memcpy(E, c->hist_h, sizeof(double) * (size_t)n);
    if (J) memcpy(J, c->hist_h + c->hist_cap, sizeof(double) * (size_t)n);
    return n;
}

int kmeans_get_timing(kmeans_ctx* c, double* iter_ms, int64_t* iter_kernels) {
    if (!c) return KM_EINVAL;
    if (iter_ms) *iter_ms = c->iter_ms;
    if (iter_kernels) *iter_kernels = c->iter_kernels;
    return KM_OK;
}

}  // extern "C"
