// wide_api.hip -- host side of the general-shape fit (wide.h): workspace,
// staging of the state and centres, the update loop as hipGraph replays of
// (wide_update, wide_reduce) with one progress read-back per batch, the final
// labels and the read-back of the results.  kmeans_fit and kmeans_assign call
// it, after validating their arguments, for d not in {2, 3}, for K > 64, and
// for every shape when KM_OPT_WIDE is set.
#include "ctx.h"
#include "wide.h"

#include <math.h>
#include <string.h>

#include <map>
#include <tuple>
#include <utility>

namespace km {

struct WideWS {
    WState* st = nullptr;      // device state
    WState* st_h = nullptr;    // pinned staging of the state
    double* mu_h = nullptr;    // pinned: K*d float64, then K*stride float32
    double* mu64 = nullptr;
    float* mu32 = nullptr;
    unsigned long long* part = nullptr;
    unsigned long long* tot = nullptr;
    double* jpart = nullptr;
    float* hh = nullptr;       // key constants, WK_MAX + 4 floats
    float* amax = nullptr;     // bound coefficients, WD_MAX + 1 floats
    size_t part_cap = 0;       // int64 slots of part
    // (d, K, track, matrix-core keys, grid, unroll)
    std::map<std::tuple<int, int, int, int, int, int>, hipGraphExec_t> graphs;
    std::map<std::tuple<int, int, int>, int> bpc;  // (d, K, matrix-core keys) -> blocks per CU
};

void wide_ws_free(WideWS* w) {
    if (!w) return;
    for (auto& kv : w->graphs) (void)hipGraphExecDestroy(kv.second);
    if (w->st) (void)hipFree(w->st);
    if (w->st_h) (void)hipHostFree(w->st_h);
    if (w->mu_h) (void)hipHostFree(w->mu_h);
    if (w->mu64) (void)hipFree(w->mu64);
    if (w->mu32) (void)hipFree(w->mu32);
    if (w->part) (void)hipFree(w->part);
    if (w->tot) (void)hipFree(w->tot);
    if (w->jpart) (void)hipFree(w->jpart);
    if (w->hh) (void)hipFree(w->hh);
    if (w->amax) (void)hipFree(w->amax);
    delete w;
}

namespace {

constexpr size_t kMu64Max = (size_t)WK_MAX * WD_MAX;  // float64 centres
constexpr size_t kMu32Max = (size_t)(WK_MAX + 2) * WD_MAX;  // float32 centres (stride <=
                                                            // WD_MAX, whole triples)
constexpr size_t kTotMax = (size_t)WK_MAX * (WD_MAX + 1);

int ensure_ws(kmeans_ctx* c) {
    if (c->wws) return KM_OK;
    WideWS* w = new WideWS();
    if (hipMalloc(&w->st, sizeof(WState)) != hipSuccess ||
        hipHostMalloc(&w->st_h, sizeof(WState), 0) != hipSuccess ||
        hipHostMalloc(&w->mu_h, sizeof(double) * kMu64Max + sizeof(float) * kMu32Max, 0) != hipSuccess ||
        hipMalloc(&w->mu64, sizeof(double) * kMu64Max) != hipSuccess ||
        hipMalloc(&w->mu32, sizeof(float) * kMu32Max) != hipSuccess ||
        hipMalloc(&w->tot, sizeof(unsigned long long) * 2 * kTotMax) != hipSuccess ||
        hipMalloc(&w->jpart, sizeof(double) * WMAX_GRID) != hipSuccess ||
        hipMalloc(&w->hh, sizeof(float) * (WK_MAX + 4)) != hipSuccess ||
        hipMalloc(&w->amax, sizeof(float) * (WD_MAX + 1)) != hipSuccess) {
        wide_ws_free(w);
        return fail(c, KM_ENOMEM, "allocation of the general-shape workspace failed");
    }
    c->wws = w;
    return KM_OK;
}

int ensure_part(kmeans_ctx* c, size_t n) {
    WideWS* w = c->wws;
    if (n <= w->part_cap) return KM_OK;
    size_t m = w->part_cap ? w->part_cap : ((size_t)1 << 16);
    while (m < n) m *= 2;
    unsigned long long* p = nullptr;
    if (hipMalloc(&p, sizeof(unsigned long long) * m) != hipSuccess)
        return fail(c, KM_ENOMEM, "hipMalloc of the partial sums (%zu slots) failed", m);
    if (w->part) {
        (void)hipStreamSynchronize(c->stream);
        (void)hipFree(w->part);
    }
    w->part = p;
    w->part_cap = m;
    return KM_OK;
}

int points_per_lane(int d) { return wide_width(d) <= 16 ? 4 : 2; }

// Grid of wide_update: the resident blocks of the device (or KM_OPT_BLOCKS),
// but never fewer than one block per FXP_BLOCK_POINTS points: a block takes
// ceil(groups / (grid WBLOCK)) groups of P points per thread, at most
// FXP_BLOCK_POINTS / (WBLOCK P) of them (N < 2^31 needs at most 4096 blocks).
// Whether the scan takes the matrix-core keys (KM_OPT_KEYS: 0 automatic --
// widths 8 to 16 with K >= 64 whose operands fit in LDS --, 1 never, 2
// wherever they fit).
bool use_mfma(const kmeans_ctx* c, int d, int K) {
    if (c->keys == 1 || !wide_mfma_fits(d, K)) return false;
    return c->keys == 2 || K >= 64;
}

int update_grid(kmeans_ctx* c, int d, int K, int64_t N, bool mfma) {
    int& b = c->wws->bpc[std::make_tuple(d, K, mfma ? 1 : 0)];
    if (b == 0) {
        b = wide_blocks_per_cu(d, K, mfma);
        // widths of 12 and more: at most 2 blocks per compute unit.  At d =
        // 16 the registers and LDS admit 3, which was measured slower (N =
        // 1e7, K = 256, per update: 512 blocks 1287 us, 768 blocks 1540 us,
        // 1024 blocks 1367 us; tiled, K = 2048, N = 2e6: 512 blocks 3522 us,
        // 768 blocks 4781 us).
        if (wide_width(d) >= 12 && b > 2) b = 2;
    }
    const int P = points_per_lane(d);
    const int64_t groups = (N + P - 1) / P;
    const int64_t need = (groups + WBLOCK - 1) / WBLOCK;
    int64_t cap = c->blocks > 0 ? c->blocks : (int64_t)c->n_cu * (b > 0 ? b : 1);
    if (cap > WMAX_GRID) cap = WMAX_GRID;
    int64_t g = need < cap ? need : cap;
    const int64_t per_block = FXP_BLOCK_POINTS / P;  // groups of one block
    const int64_t lo = (groups + per_block - 1) / per_block;
    if (g < lo) g = lo;
    return g < 1 ? 1 : (int)g;
}

int scan_grid(kmeans_ctx* c, int64_t N) {
    const int64_t need = (N + WBLOCK - 1) / WBLOCK;
    const int64_t cap = (int64_t)c->n_cu * 4;
    return (int)(need < cap ? (need < 1 ? 1 : need) : cap);
}

// Host staging of the state and centres, then the upload (one copy of the
// state, one of the centres) on the context's stream.  track: the labels of
// indicator tracking, or null.
int stage_upload(kmeans_ctx* c, const float* X, int64_t N, int64_t ld, int d, int K,
                 const double* mu, double tol, int max_iter, int grid, int32_t* track) {
    WideWS* w = c->wws;
    const int DS = wide_stride(wide_width(d));
    const int nacc = K * (d + 1);
    int rc = ensure_part(c, (size_t)grid * nacc);
    if (rc) return rc;
    // the previous call's work on this stream may still read the staging buffers
    KM_HIP(c, hipStreamSynchronize(c->stream));
    WState* h = w->st_h;
    memset(h, 0, sizeof(WState));
    h->X = X;
    h->N = N;
    h->ld = ld;
    h->d = d;
    h->K = K;
    h->tol = tol;
    h->max_iter = max_iter;
    h->hist_cap = c->hist_cap;
    h->grid = grid;
    h->vec = ((reinterpret_cast<uintptr_t>(X) & 15u) == 0 && (ld & 3) == 0) ? 1 : 0;
    h->mu64 = w->mu64;
    h->mu32 = w->mu32;
    h->part = w->part;
    h->tot = w->tot;
    h->jpart = w->jpart;
    h->hh = w->hh;
    h->amax = w->amax;
    h->plus_inf = INFINITY;
    h->E_hist = c->hist;
    h->J_hist = c->hist + c->hist_cap;
    h->C_hist = reinterpret_cast<int64_t*>(c->hist + 2 * (size_t)c->hist_cap);
    h->track = track;
    h->E = INFINITY;
    double* m64 = w->mu_h;
    float* m32 = reinterpret_cast<float*>(w->mu_h + (size_t)K * d);
    const int kp = wide_kpad(K);  // zero rows up to a whole triple
    for (int k = 0; k < kp; ++k) {
        for (int j = 0; j < DS; ++j) m32[(size_t)k * DS + j] = 0.0f;
        for (int j = 0; j < d && k < K; ++j) {
            m64[(size_t)k * d + j] = mu[(size_t)k * d + j];
            m32[(size_t)k * DS + j] = (float)mu[(size_t)k * d + j];  // round to nearest even
        }
    }
    KM_HIP(c, hipMemcpyAsync(w->st, h, kWUploadBytes, hipMemcpyHostToDevice, c->stream));
    KM_HIP(c, hipMemcpyAsync(w->mu64, m64, sizeof(double) * (size_t)K * d, hipMemcpyHostToDevice,
                             c->stream));
    KM_HIP(c, hipMemcpyAsync(w->mu32, m32, sizeof(float) * (size_t)kp * DS, hipMemcpyHostToDevice,
                             c->stream));
    return KM_OK;
}

int launch_one_update(kmeans_ctx* c, int d, int K, bool track, bool mfma, int grid,
                      hipStream_t s) {
    hipError_t e = launch_wide_update(c->wws->st, d, K, track, mfma, grid, s);
    if (e == hipSuccess) e = launch_wide_reduce(c->wws->st, d, K, grid, s);
    if (e != hipSuccess) return fail(c, KM_EHIP, "launch of a general-shape update failed: %s", hipGetErrorString(e));
    return KM_OK;
}

int get_graph(kmeans_ctx* c, int d, int K, bool track, bool mfma, int grid, int unroll,
              hipGraphExec_t* out) {
    WideWS* w = c->wws;
    const auto key = std::make_tuple(d, K, track ? 1 : 0, mfma ? 1 : 0, grid, unroll);
    auto it = w->graphs.find(key);
    if (it != w->graphs.end()) {
        *out = it->second;
        return KM_OK;
    }
    KM_HIP(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
    for (int i = 0; i < unroll; ++i) {
        hipError_t e = launch_wide_update(w->st, d, K, track, mfma, grid, c->cap_stream);
        if (e == hipSuccess) e = launch_wide_reduce(w->st, d, K, grid, c->cap_stream);
        if (e != hipSuccess) {
            hipGraph_t junk = nullptr;
            (void)hipStreamEndCapture(c->cap_stream, &junk);
            if (junk) (void)hipGraphDestroy(junk);
            return fail(c, KM_EHIP, "capture of the general-shape update failed: %s", hipGetErrorString(e));
        }
    }
    hipGraph_t g = nullptr;
    KM_HIP(c, hipStreamEndCapture(c->cap_stream, &g));
    hipGraphExec_t ex = nullptr;
    hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return fail(c, KM_EHIP, "hipGraphInstantiate failed: %s", hipGetErrorString(e));
    w->graphs[key] = ex;
    *out = ex;
    return KM_OK;
}

int read_progress(kmeans_ctx* c, size_t bytes) {
    WideWS* w = c->wws;
    KM_HIP(c, hipMemcpyAsync(reinterpret_cast<char*>(w->st_h) + kWProgressOffset,
                             reinterpret_cast<char*>(w->st) + kWProgressOffset, bytes,
                             hipMemcpyDeviceToHost, c->stream));
    KM_HIP(c, hipStreamSynchronize(c->stream));
    return KM_OK;
}

}  // namespace

int wide_fit(kmeans_ctx* c, const float* X, int64_t N, int64_t ld, int d, int K,
             const double* init, double tol, int max_iter, double* centroids_out,
             int32_t* labels_out, km_result* res) {
    int rc = ensure_ws(c);
    if (!rc) rc = ensure_hist(c, max_iter);
    if (rc) return rc;
    WideWS* w = c->wws;
    const bool mfma = use_mfma(c, d, K);
    const int grid = update_grid(c, d, K, N, mfma);
    const bool track = c->track != 0;
    rc = stage_upload(c, X, N, ld, d, K, init, tol, max_iter, grid, track ? labels_out : nullptr);
    if (rc) return rc;
    // no label before the first update: every point counts as changed
    if (track)
        KM_HIP(c, hipMemsetAsync(labels_out, 0xff, sizeof(int32_t) * (size_t)N, c->stream));
    KM_HIP(c, launch_wide_scan(w->st, scan_grid(c, N), c->stream));

    int U = c->unroll > 0 ? c->unroll : (N >= (1 << 24) ? 10 : (N >= (1 << 20) ? 16 : 32));
    if (U > max_iter) U = max_iter;
    c->iter_ms = 0.0;
    c->iter_kernels = 0;
    int launched = 0, batches = 0;
    while (launched < max_iter) {
        const int n = (max_iter - launched) < U ? (max_iter - launched) : U;
        if (c->timing) {
            rc = ensure_events(c, 2 * (size_t)(batches + 1));
            if (rc) return rc;
            KM_HIP(c, hipEventRecord(c->ev[2 * batches], c->stream));
        }
        if (c->use_graph) {
            hipGraphExec_t ex;
            rc = get_graph(c, d, K, track, mfma, grid, n, &ex);
            if (rc) return rc;
            KM_HIP(c, hipGraphLaunch(ex, c->stream));
        } else {
            for (int i = 0; i < n && !rc; ++i)
                rc = launch_one_update(c, d, K, track, mfma, grid, c->stream);
            if (rc) return rc;
        }
        if (c->timing) KM_HIP(c, hipEventRecord(c->ev[2 * batches + 1], c->stream));
        launched += n;
        batches += 1;
        if ((tol > 0.0 || track) && launched < max_iter) {
            rc = read_progress(c, kWProgressBytes);
            if (rc) return rc;
            if (w->st_h->done) break;
        }
    }
    KM_HIP(c, launch_wide_label(w->st, labels_out, d, K, mfma, grid, c->stream));
    double* m64 = w->mu_h;
    KM_HIP(c, hipMemcpyAsync(m64, w->mu64, sizeof(double) * (size_t)K * d, hipMemcpyDeviceToHost,
                             c->stream));
    // the E / J history of every update that ran (T <= launched), read with
    // the results: one synchronisation instead of two
    {
        const int nc = launched < c->hist_cap ? launched : c->hist_cap;
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
    rc = read_progress(c, kWProgressBytes);
    if (rc) return rc;
    const WState* h = w->st_h;
    const int T = h->t;
    c->last_T = T;
    if (c->timing) {
        for (int b = 0; b < batches; ++b) {
            float ms = 0.f;
            KM_HIP(c, hipEventElapsedTime(&ms, c->ev[2 * b], c->ev[2 * b + 1]));
            c->iter_ms += ms;
        }
        c->iter_kernels = launched;
    }
    if (h->flags & FLAG_NONFINITE) return fail(c, KM_EINVAL, "X holds a NaN or an infinity");
    if (h->flags & FLAG_RANGE) return range_error(c);
    memcpy(centroids_out, m64, sizeof(double) * (size_t)K * d);
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

int wide_assign(kmeans_ctx* c, const float* X, int64_t N, int64_t ld, int d, int K,
                const double* centroids, int32_t* labels, double* objective) {
    int rc = ensure_ws(c);
    if (rc) return rc;
    WideWS* w = c->wws;
    const bool mfma = use_mfma(c, d, K);
    const int grid = update_grid(c, d, K, N, mfma);
    rc = stage_upload(c, X, N, ld, d, K, centroids, 0.0, 1, grid, nullptr);
    if (rc) return rc;
    KM_HIP(c, launch_wide_scan(w->st, scan_grid(c, N), c->stream));
    KM_HIP(c, launch_wide_label(w->st, labels, d, K, mfma, grid, c->stream));
    rc = read_progress(c, kWProgressBytes);
    if (rc) return rc;
    if (w->st_h->flags & FLAG_NONFINITE) return fail(c, KM_EINVAL, "X holds a NaN or an infinity");
    if (objective) *objective = w->st_h->J;
    return KM_OK;
}

}  // namespace km
