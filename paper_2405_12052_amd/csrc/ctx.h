// ctx.h -- the context object behind the opaque kmeans_ctx of include/kmeans.h
// and helpers shared by the host-side sources of libkmeans_mi355x.so.
#pragma once

#include "../../include/kmeans.h"
#include "km_internal.h"

#include <map>
#include <string>
#include <tuple>
#include <vector>

namespace km {

struct GraphKey {
    int d, vec, keys, track, grid, unroll;
    bool operator<(const GraphKey& o) const {
        return std::tie(d, vec, keys, track, grid, unroll) <
               std::tie(o.d, o.vec, o.keys, o.track, o.grid, o.unroll);
    }
};

struct BatchedWS;                    // workspace of kmeans_fit_batched (batched_api.hip)
void batched_ws_free(BatchedWS* w);
struct NetWS;                        // workspace of the learned initialiser (initnet_api.hip)
void net_ws_free(NetWS* w);
struct SeedWS;                       // workspace of k-means++ seeding (seeding.hip)
void seed_ws_free(SeedWS* w);
struct WideWS;                       // workspace of the general-shape fit (wide_api.hip)
void wide_ws_free(WideWS* w);

}  // namespace km

struct kmeans_ctx {
    int device = 0;
    hipStream_t stream = nullptr;      // caller's stream: all work goes here
    hipStream_t cap_stream = nullptr;  // private stream used only for capture
    int n_cu = 256;
    km::State* st = nullptr;           // device state
    km::State* st_h = nullptr;         // pinned host staging of the state
    double* jpart = nullptr;           // [MAX_BLOCKS]
    unsigned long long* part = nullptr;   // [MAX_BLOCKS][PART]
    unsigned long long* gpart = nullptr;  // [MAX_GROUPS][PART]
    double* gjpart = nullptr;          // [MAX_GROUPS]
    uint32_t* gticket = nullptr;       // [MAX_GROUPS]
    double* hist = nullptr;            // [3 * hist_cap]: E, J, then the changed-label
                                       // counts (int64) of indicator tracking
    int hist_cap = 0;
    double* hist_h = nullptr;          // pinned copy of the history
    std::string err;
    // options
    int use_graph = 1;
    int unroll = 0;
    int blocks = 0;
    int timing = 0;
    int keys = 0;                      // KM_OPT_KEYS
    int persist = 0;                   // KM_OPT_PERSIST
    int track = 0;                     // KM_OPT_TRACK
    int last_track = 0;                // the last fit tracked its indicators
    int persist_bpc[2][2] = {{0, 0}, {0, 0}};  // resident blocks per CU of lloyd_persist [d==3][vec]
    // graph cache
    std::map<km::GraphKey, hipGraphExec_t> graphs;
    // timing of the last fit: one event pair per batch of iterations
    std::vector<hipEvent_t> ev;
    double iter_ms = 0.0;
    int64_t iter_kernels = 0;
    int last_T = 0;
    // batched fits
    km::BatchedWS* bws = nullptr;
    km_schedule sched = {0, 0, 0.0, 0, 0};  // zeros: automatic
    // learned initialiser
    km::NetWS* nws = nullptr;
    // k-means++ seeding
    km::SeedWS* sws = nullptr;
    // general-shape fit
    km::WideWS* wws = nullptr;
    int wide = 0;                      // KM_OPT_WIDE
};

namespace km {
// Record an error message on c (or, with c == NULL, for kmeans_create) and
// return `code`.
int fail(kmeans_ctx* c, int code, const char* fmt, ...) __attribute__((format(printf, 3, 4)));
int check_device_ptr(kmeans_ctx* c, const void* p, const char* what);
// Device history of E, J and the changed-label counts with room for cap
// updates (kmeans_api.hip).
int ensure_hist(kmeans_ctx* c, int cap);
// At least n timing events in c->ev (kmeans_api.hip).
int ensure_events(kmeans_ctx* c, size_t n);
// Records the error of a fit whose data exceed the range of the fixed-point
// cluster sums (FLAG_RANGE) and returns KM_EUNSUPPORTED (kmeans_api.hip).
int range_error(kmeans_ctx* c);
// True when (d, K) takes the general-shape fit: d not in {2, 3}, K > KMAX,
// or KM_OPT_WIDE set (kmeans_api.hip).
bool wide_shape(const kmeans_ctx* c, int d, int K);
// Argument checks of a fit or reassignment (kmeans_api.hip); with c == NULL
// the message goes where kmeans_last_error(NULL) reads it.
int validate(kmeans_ctx* c, int64_t N, int64_t ld, int32_t d, int32_t K, double tol,
             int32_t max_iter);
int check_centres(kmeans_ctx* c, const double* m, int K, int d, const char* what);
// Rows 16-byte aligned with ld % 4 == 0: the 128-bit load path.
bool vec_ok(const float* X, int64_t ld);
// Fewest blocks that keep every block at or below FXP_BLOCK_POINTS points.
int64_t min_blocks(int64_t N);
// Grid of the per-update kernels for N points on n_cu compute units
// (blocks_opt: KM_OPT_BLOCKS, 0 = automatic).
int grid_blocks(int n_cu, int blocks_opt, int64_t N);
// Scan variant of KM_OPT_KEYS = 0 (automatic) for K centres: 0 the VALU
// keys, 1 or 2 matrix-core tiles of 32 centres.
int auto_keys(int K);
// Updates per graph replay when KM_OPT_UNROLL is automatic.
int auto_unroll(int64_t N, int max_iter);
// Device buffers a fit's state points to.
struct FitBufs {
    double* jpart;
    unsigned long long* part;
    unsigned long long* gpart;
    double* gjpart;
    uint32_t* gticket;
    double* hist;   // [hist_cap] E, then [hist_cap] J
    int64_t* chist; // [hist_cap] changed-label counts, or null (no tracking)
    int hist_cap;
};
// Host copy of the state of a fit (or reassignment) of the given problem.
void stage_state(State* h, const FitBufs& b, const float* X, int64_t N, int64_t ld, int d,
                 int K, const double* mu, double tol, int max_iter);
// The general-shape fit and reassignment (wide_api.hip); same contract as
// kmeans_fit / kmeans_assign after argument validation.
int wide_fit(kmeans_ctx* c, const float* X, int64_t N, int64_t ld, int d, int K,
             const double* init, double tol, int max_iter, double* centroids_out,
             int32_t* labels_out, km_result* res);
int wide_assign(kmeans_ctx* c, const float* X, int64_t N, int64_t ld, int d, int K,
                const double* centroids, int32_t* labels, double* objective);
}  // namespace km

#define KM_HIP(ctx, call)                                                                   \
    do {                                                                                    \
        hipError_t e_ = (call);                                                             \
        if (e_ != hipSuccess)                                                               \
            return km::fail(ctx, KM_EHIP, "%s failed: %s", #call, hipGetErrorString(e_));  \
    } while (0)
