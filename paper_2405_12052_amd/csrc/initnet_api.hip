// initnet_api.hip -- host side of the learned initialiser: argument checks,
// the workspace, and the launch sequences of inference (gather + normalise +
// forward + head), of a gradient evaluation and of a training step (forward,
// head with matching and loss, backward, fixed-order reduction, Adam).
#include "ctx.h"
#include "initnet.h"

#include <math.h>
#include <string.h>

#include <vector>

using km::fail;
namespace net = km::net;

namespace km {
struct NetWS {
    int capB = 0, capP = 0;
    float* pool = nullptr;
    int32_t* argmax = nullptr;
    float* part = nullptr;
    float* pred = nullptr;     // [3 * KMAXN]: one instance (inference)
    double* loss = nullptr;
    int32_t* match = nullptr;
    float *dy = nullptr, *dybf = nullptr, *dz = nullptr, *dzbf = nullptr, *zbf = nullptr;
    float *dpool = nullptr, *poolbf = nullptr;
    float* gpts = nullptr;     // gathered, normalised sample [capP][3]
    double* stats = nullptr;   // mean0..2, s
    int32_t* idx = nullptr;
    double* loss_h = nullptr;  // pinned [capB]
    double* stats_h = nullptr; // pinned [4]
    float* pred_h = nullptr;   // pinned [3 * KMAXN]
};

void net_ws_free(NetWS* w) {
    if (!w) return;
    void* dev[] = {w->pool, w->argmax, w->part, w->pred, w->loss, w->match, w->dy, w->dybf,
                   w->dz, w->dzbf, w->zbf, w->dpool, w->poolbf, w->gpts, w->stats, w->idx};
    for (void* p : dev)
        if (p) (void)hipFree(p);
    void* host[] = {w->loss_h, w->stats_h, w->pred_h};
    for (void* p : host)
        if (p) (void)hipHostFree(p);
    delete w;
}
}  // namespace km

namespace {

template <typename T>
bool dalloc(T** p, size_t n) {
    if (*p) (void)hipFree(*p);
    *p = nullptr;
    return hipMalloc(reinterpret_cast<void**>(p), sizeof(T) * (n ? n : 1)) == hipSuccess;
}

int ensure_net(kmeans_ctx* c, int B, int P) {
    (void)hipSetDevice(c->device);
    if (!c->nws) {
        c->nws = new km::NetWS();
        km::NetWS* w = c->nws;
        if (hipHostMalloc(&w->stats_h, sizeof(double) * 4, 0) != hipSuccess ||
            hipHostMalloc(&w->pred_h, sizeof(float) * 3 * net::KMAXN, 0) != hipSuccess ||
            !dalloc(&w->stats, 4) || !dalloc(&w->pred, 3 * net::KMAXN))
            return fail(c, KM_ENOMEM, "allocation of the network workspace failed");
    }
    km::NetWS* w = c->nws;
    if (B > w->capB) {
        (void)hipStreamSynchronize(c->stream);
        const size_t b = (size_t)B;
        bool ok = dalloc(&w->pool, b * 2 * net::NH) && dalloc(&w->argmax, b * net::NH) &&
                  dalloc(&w->part, b * 4 * net::PT_SIZE) && dalloc(&w->loss, b) &&
                  dalloc(&w->match, b * net::KMAXN) && dalloc(&w->dy, b * 3 * net::KMAXN) &&
                  dalloc(&w->dybf, b * 3 * net::KMAXN) && dalloc(&w->dz, b * net::NZ) &&
                  dalloc(&w->dzbf, b * net::NZ) && dalloc(&w->zbf, b * net::NZ) &&
                  dalloc(&w->dpool, b * 2 * net::NH) && dalloc(&w->poolbf, b * 2 * net::NH);
        if (ok) {
            if (w->loss_h) (void)hipHostFree(w->loss_h);
            w->loss_h = nullptr;
            ok = hipHostMalloc(&w->loss_h, sizeof(double) * b, 0) == hipSuccess;
        }
        if (!ok) {
            w->capB = 0;
            return fail(c, KM_ENOMEM, "allocation of the network workspace (B=%d) failed", B);
        }
        w->capB = B;
    }
    if (P > w->capP) {
        (void)hipStreamSynchronize(c->stream);
        if (!dalloc(&w->gpts, (size_t)P * 3) || !dalloc(&w->idx, (size_t)P)) {
            w->capP = 0;
            return fail(c, KM_ENOMEM, "allocation of the sample buffer (P=%d) failed", P);
        }
        w->capP = P;
    }
    return KM_OK;
}

net::HeadOut head_out(km::NetWS* w) {
    net::HeadOut h;
    h.loss = w->loss;
    h.match = w->match;
    h.dy = w->dy;
    h.dybf = w->dybf;
    h.dz = w->dz;
    h.dzbf = w->dzbf;
    h.zbf = w->zbf;
    h.dpool = w->dpool;
    h.poolbf = w->poolbf;
    return h;
}

int check_shape(kmeans_ctx* c, int B, int P, int K) {
    if (B < 1 || B > 4096) return fail(c, KM_EINVAL, "B=%d out of [1, 4096]", B);
    if (P < 32 || P > 65536 || P % 32) return fail(c, KM_EINVAL, "P=%d: a multiple of 32 in [32, 65536]", P);
    if (K < 1 || K > net::KMAXN) return fail(c, KM_EUNSUPPORTED, "K=%d out of [1, %d]", K, net::KMAXN);
    return KM_OK;
}

int check_dev(kmeans_ctx* c, const void* p, const char* what) {
    return km::check_device_ptr(c, p, what);
}

// Forward + head (+ matching, loss, backward with targets); leaves the
// per-instance outputs in the workspace.
int run_net(kmeans_ctx* c, const float* pts, const float* targets, int B, int P, int K,
            const float* params, float* pred) {
    km::NetWS* w = c->nws;
    KM_HIP(c, net::launch_points_fwd(pts, B, P, params, w->pool, w->argmax, c->stream));
    KM_HIP(c, net::launch_head(w->pool, B, K, params, targets, pred, head_out(w), c->stream));
    if (targets)
        KM_HIP(c, net::launch_points_bwd(pts, B, P, params, w->dpool, w->argmax, w->part, c->stream));
    return KM_OK;
}

int read_loss(kmeans_ctx* c, int B, double* loss_out) {
    km::NetWS* w = c->nws;
    KM_HIP(c, hipMemcpyAsync(w->loss_h, w->loss, sizeof(double) * B, hipMemcpyDeviceToHost, c->stream));
    KM_HIP(c, hipStreamSynchronize(c->stream));
    double L = 0.0;
    for (int b = 0; b < B; ++b) L += w->loss_h[b];
    *loss_out = L;
    return KM_OK;
}

}  // namespace

extern "C" {

int32_t kmeans_initnet_param_count(int32_t K) {
    if (K < 1 || K > net::KMAXN) return -1;
    return net::param_count(K);
}

int kmeans_initnet_forward(kmeans_ctx* c, const float* pts, int32_t B, int32_t P, int32_t K,
                           const float* params, float* pred_out, float* pool_out) {
    if (!c) return KM_EINVAL;
    c->err.clear();
    int rc = check_shape(c, B, P, K);
    if (!rc) rc = check_dev(c, pts, "pts");
    if (!rc) rc = check_dev(c, params, "params");
    if (!rc) rc = check_dev(c, pred_out, "pred_out");
    if (!rc && pool_out) rc = check_dev(c, pool_out, "pool_out");
    if (rc) return rc;
    KM_HIP(c, hipSetDevice(c->device));
    rc = ensure_net(c, B, P);
    if (rc) return rc;
    rc = run_net(c, pts, nullptr, B, P, K, params, pred_out);
    if (rc) return rc;
    if (pool_out)
        KM_HIP(c, hipMemcpyAsync(pool_out, c->nws->pool, sizeof(float) * B * 2 * net::NH,
                                 hipMemcpyDeviceToDevice, c->stream));
    KM_HIP(c, hipStreamSynchronize(c->stream));
    return KM_OK;
}

int kmeans_initnet_grad(kmeans_ctx* c, const float* pts, const float* targets, int32_t B,
                        int32_t P, int32_t K, const float* params, float* grad_out,
                        double* loss_out, int32_t* match_out) {
    if (!c) return KM_EINVAL;
    c->err.clear();
    int rc = check_shape(c, B, P, K);
    if (!rc) rc = check_dev(c, pts, "pts");
    if (!rc) rc = check_dev(c, targets, "targets");
    if (!rc) rc = check_dev(c, params, "params");
    if (!rc) rc = check_dev(c, grad_out, "grad_out");
    if (!rc && match_out) rc = check_dev(c, match_out, "match_out");
    if (rc) return rc;
    KM_HIP(c, hipSetDevice(c->device));
    rc = ensure_net(c, B, P);
    if (rc) return rc;
    km::NetWS* w = c->nws;
    // no predictions are stored here (the workspace's pred holds one instance)
    rc = run_net(c, pts, targets, B, P, K, params, nullptr);
    if (rc) return rc;
    net::AdamArgs a{};
    KM_HIP(c, net::launch_reduce(B, K, w->part, head_out(w), grad_out, nullptr, nullptr, nullptr,
                                 a, c->stream));
    if (match_out)
        KM_HIP(c, hipMemcpyAsync(match_out, w->match, sizeof(int32_t) * B * K,
                                 hipMemcpyDeviceToDevice, c->stream));
    if (loss_out) return read_loss(c, B, loss_out);
    KM_HIP(c, hipStreamSynchronize(c->stream));
    return KM_OK;
}

int kmeans_initnet_train_step(kmeans_ctx* c, const float* pts, const float* targets, int32_t B,
                              int32_t P, int32_t K, float* params, float* adam_m, float* adam_v,
                              float lr, int32_t step, double* loss_out) {
    if (!c) return KM_EINVAL;
    c->err.clear();
    int rc = check_shape(c, B, P, K);
    if (!rc && (!(lr > 0.0f) || !isfinite(lr))) rc = fail(c, KM_EINVAL, "lr must be finite and > 0");
    if (!rc && step < 1) rc = fail(c, KM_EINVAL, "step=%d < 1", step);
    if (!rc) rc = check_dev(c, pts, "pts");
    if (!rc) rc = check_dev(c, targets, "targets");
    if (!rc) rc = check_dev(c, params, "params");
    if (!rc) rc = check_dev(c, adam_m, "adam_m");
    if (!rc) rc = check_dev(c, adam_v, "adam_v");
    if (rc) return rc;
    KM_HIP(c, hipSetDevice(c->device));
    rc = ensure_net(c, B, P);
    if (rc) return rc;
    km::NetWS* w = c->nws;
    rc = run_net(c, pts, targets, B, P, K, params, nullptr);
    if (rc) return rc;
    net::AdamArgs a;
    a.lr = lr;
    a.beta1 = 0.9f;
    a.beta2 = 0.999f;
    a.eps = 1e-8f;
    a.bc1 = (float)(1.0 - pow(0.9, step));
    a.bc2 = (float)(1.0 - pow(0.999, step));
    KM_HIP(c, net::launch_reduce(B, K, w->part, head_out(w), nullptr, params, adam_m, adam_v, a,
                                 c->stream));
    if (loss_out) return read_loss(c, B, loss_out);
    return KM_OK;
}

int kmeans_init_learned(kmeans_ctx* c, const float* X, int64_t N, int64_t ld, int32_t K,
                        const int32_t* idx, int32_t P, const float* params,
                        double* centroids_out) {
    if (!c) return KM_EINVAL;
    c->err.clear();
    int rc = check_shape(c, 1, P, K);
    if (!rc && P > net::GATHER_MAX) rc = fail(c, KM_EINVAL, "P=%d > %d", P, net::GATHER_MAX);
    if (!rc && (N < 1 || ld < N)) rc = fail(c, KM_EINVAL, "N=%lld, ld=%lld", (long long)N, (long long)ld);
    if (!rc && !centroids_out) rc = fail(c, KM_EINVAL, "centroids_out is NULL");
    if (!rc) rc = check_dev(c, X, "X");
    if (!rc) rc = check_dev(c, idx, "idx");
    if (!rc) rc = check_dev(c, params, "params");
    if (rc) return rc;
    KM_HIP(c, hipSetDevice(c->device));
    // the sample's per-point layers run as S equal slices in parallel blocks
    // (S the largest of 16, 8, 4, 2, 1 with P/S a multiple of 32), pooled
    // together by the inference head
    int S = 16;
    while (S > 1 && P % (32 * S)) S /= 2;
    rc = ensure_net(c, S, P);
    if (rc) return rc;
    km::NetWS* w = c->nws;
    KM_HIP(c, net::launch_gather(X, ld, N, idx, P, w->gpts, w->stats, c->stream));
    KM_HIP(c, net::launch_points_fwd(w->gpts, S, P / S, params, w->pool, nullptr, c->stream));
    KM_HIP(c, net::launch_infer_head(w->pool, S, K, params, w->zbf, w->pred, c->stream));
    KM_HIP(c, hipMemcpyAsync(w->pred_h, w->pred, sizeof(float) * 3 * K, hipMemcpyDeviceToHost, c->stream));
    KM_HIP(c, hipMemcpyAsync(w->stats_h, w->stats, sizeof(double) * 4, hipMemcpyDeviceToHost, c->stream));
    KM_HIP(c, hipStreamSynchronize(c->stream));
    for (int k = 0; k < K; ++k)
        for (int q = 0; q < 3; ++q) {
            const double v = (double)w->pred_h[3 * k + q] * w->stats_h[3] + w->stats_h[q];
            if (!isfinite(v)) return fail(c, KM_EINVAL, "the network produced a non-finite centre");
            centroids_out[3 * k + q] = v;
        }
    return KM_OK;
}

}  // extern "C"
