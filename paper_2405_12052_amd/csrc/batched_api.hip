// batched_api.hip -- host side of kmeans_fit_batched and its autotuner:
// validation, the device workspace, the split of the instances into the
// team-processed (large) and single-block (small) lists, largest first, the
// persistent launch (captured in a hipGraph when the runtime accepts a
// cooperative kernel in a capture), result read-back, and the schedule search
// with its JSON cache.
#include "ctx.h"
#include "batched_copy.h"

#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <numeric>
#include <string>
#include <vector>

using km::BatchState;
using km::BInst;
using km::BOut;
using km::BTeam;
using km::fail;

namespace km {

struct BatchedWS {
    int cap_inst = 0;          // capacity of the per-instance arrays
    size_t cap_init = 0;       // capacity of the initial-centre pool (doubles)
    int cap_blocks = 0;        // capacity of the team partials (blocks)
    BatchState* bs = nullptr;  // device
    BatchState* bs_h = nullptr;
    BInst* inst = nullptr;     // device [cap_inst]
    BInst* inst_h = nullptr;
    int32_t* order = nullptr;  // device [cap_inst]: big list then small list
    int32_t* order_h = nullptr;
    double* init = nullptr;    // device pool
    double* init_h = nullptr;
    uint32_t* absmax = nullptr;
    BOut* out = nullptr;       // device [cap_inst * BK_RMAX]
    BOut* out_h = nullptr;
    int32_t* best = nullptr;
    int32_t* best_h = nullptr;
    double* best_mu = nullptr;
    double* best_mu_h = nullptr;
    unsigned long long* tpart = nullptr;
    unsigned long long* fold = nullptr;
    double* tjpart = nullptr;
    BTeam* teams = nullptr;
    int32_t* error_h = nullptr;  // pinned copy of BatchState::error
    // restart groups: labels of the work items after an instance's first
    // (device), and the table of the copies of kept restarts' labels
    int32_t* tmp_labels = nullptr;
    size_t cap_tmp = 0;            // int32 entries of tmp_labels
    BCopy* copies = nullptr;       // device [cap_inst]
    BCopy* copies_h = nullptr;     // pinned [cap_inst]
    // graph of {scan, fit} for the current (grid, team size, n_inst) key
    hipGraphExec_t graph = nullptr;
    int g_grid = -1, g_S = -1, g_n = -1;
    bool coop_capture_ok = true;
    float last_ms = 0.f;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
};

void batched_ws_free(BatchedWS* w) {
    if (!w) return;
    if (w->graph) (void)hipGraphExecDestroy(w->graph);
    void* dev[] = {w->bs, w->inst, w->order, w->init, w->absmax, w->out, w->best, w->best_mu,
                   w->tpart, w->fold, w->tjpart, w->teams, w->tmp_labels, w->copies};
    for (void* p : dev)
        if (p) (void)hipFree(p);
    void* host[] = {w->bs_h, w->inst_h, w->order_h, w->init_h, w->out_h, w->best_h,
                    w->best_mu_h, w->error_h, w->copies_h};
    for (void* p : host)
        if (p) (void)hipHostFree(p);
    if (w->ev0) (void)hipEventDestroy(w->ev0);
    if (w->ev1) (void)hipEventDestroy(w->ev1);
    delete w;
}

}  // namespace km

namespace {

template <typename T>
int dev_alloc(kmeans_ctx* c, T** p, size_t n) {
    if (*p) (void)hipFree(*p);
    *p = nullptr;
    if (hipMalloc(reinterpret_cast<void**>(p), sizeof(T) * (n ? n : 1)) != hipSuccess)
        return fail(c, KM_ENOMEM, "hipMalloc of %zu bytes for the batched workspace failed",
                    sizeof(T) * n);
    return KM_OK;
}

template <typename T>
int host_alloc(kmeans_ctx* c, T** p, size_t n) {
    if (*p) (void)hipHostFree(*p);
    *p = nullptr;
    if (hipHostMalloc(reinterpret_cast<void**>(p), sizeof(T) * (n ? n : 1), 0) != hipSuccess)
        return fail(c, KM_ENOMEM, "hipHostMalloc for the batched workspace failed");
    return KM_OK;
}

void drop_graph(km::BatchedWS* w) {
    if (w->graph) (void)hipGraphExecDestroy(w->graph);
    w->graph = nullptr;
    w->g_grid = w->g_S = w->g_n = -1;
}

int ensure_ws(kmeans_ctx* c, int n_inst, size_t n_init, int blocks, size_t n_tmp) {
    (void)hipSetDevice(c->device);
    if (!c->bws) {
        c->bws = new km::BatchedWS();
        int rc = 0;
        if (!rc) rc = dev_alloc(c, &c->bws->bs, 1);
        if (!rc) rc = host_alloc(c, &c->bws->bs_h, 1);
        if (!rc) rc = host_alloc(c, &c->bws->error_h, 1);
        if (!rc && (hipEventCreate(&c->bws->ev0) != hipSuccess ||
                    hipEventCreate(&c->bws->ev1) != hipSuccess))
            rc = fail(c, KM_EHIP, "hipEventCreate failed");
        if (rc) return rc;
    }
    km::BatchedWS* w = c->bws;
    if (n_inst > w->cap_inst || w->cap_inst == 0) {
        (void)hipStreamSynchronize(c->stream);
        drop_graph(w);
        const int n = std::max(n_inst, 64);
        int rc = 0;
        if (!rc) rc = dev_alloc(c, &w->inst, n);
        if (!rc) rc = host_alloc(c, &w->inst_h, n);
        if (!rc) rc = dev_alloc(c, &w->order, n);
        if (!rc) rc = host_alloc(c, &w->order_h, n);
        if (!rc) rc = dev_alloc(c, &w->absmax, n);
        if (!rc) rc = dev_alloc(c, &w->out, (size_t)n * km::BK_RMAX);
        if (!rc) rc = host_alloc(c, &w->out_h, (size_t)n * km::BK_RMAX);
        if (!rc) rc = dev_alloc(c, &w->best, n);
        if (!rc) rc = host_alloc(c, &w->best_h, n);
        if (!rc) rc = dev_alloc(c, &w->best_mu, (size_t)n * km::BK_KMAX * km::DMAX);
        if (!rc) rc = host_alloc(c, &w->best_mu_h, (size_t)n * km::BK_KMAX * km::DMAX);
        if (!rc) rc = dev_alloc(c, &w->copies, n);
        if (!rc) rc = host_alloc(c, &w->copies_h, n);
        if (rc) {
            w->cap_inst = 0;
            return rc;
        }
        w->cap_inst = n;
    }
    if (n_init > w->cap_init) {
        (void)hipStreamSynchronize(c->stream);
        drop_graph(w);
        const size_t n = std::max(n_init, (size_t)4096);
        int rc = dev_alloc(c, &w->init, n);
        if (!rc) rc = host_alloc(c, &w->init_h, n);
        if (rc) {
            w->cap_init = 0;
            return rc;
        }
        w->cap_init = n;
    }
    if (n_tmp > w->cap_tmp) {
        (void)hipStreamSynchronize(c->stream);
        const size_t n = std::max(n_tmp, (size_t)1 << 20);
        int rc = dev_alloc(c, &w->tmp_labels, n);
        if (rc) {
            w->cap_tmp = 0;
            return rc;
        }
        w->cap_tmp = n;
    }
    if (blocks > w->cap_blocks) {
        (void)hipStreamSynchronize(c->stream);
        drop_graph(w);
        int rc = dev_alloc(c, &w->tpart, (size_t)2 * blocks * km::BK_PART * 2);
        if (!rc) rc = dev_alloc(c, &w->fold, (size_t)blocks * km::BK_PART * 2);
        if (!rc) rc = dev_alloc(c, &w->tjpart, (size_t)2 * blocks * km::BK_RMAX);
        if (!rc) rc = dev_alloc(c, &w->teams, (size_t)blocks);
        if (rc) {
            w->cap_blocks = 0;
            return rc;
        }
        w->cap_blocks = blocks;
    }
    return KM_OK;
}

int validate_instance(kmeans_ctx* c, int i, const km_instance& in) {
    if (in.N < 1 || in.N > km::BK_NMAX)
        return fail(c, KM_EINVAL, "instance %d: N=%lld out of [1, 2^27]", i, (long long)in.N);
    if (in.ld < in.N) return fail(c, KM_EINVAL, "instance %d: ld < N", i);
    if (in.d != 2 && in.d != 3) return fail(c, KM_EUNSUPPORTED, "instance %d: d=%d", i, in.d);
    if (in.K < 1 || in.K > in.N) return fail(c, KM_EINVAL, "instance %d: K=%d out of [1, N]", i, in.K);
    if (in.K > km::BK_KMAX) return fail(c, KM_EUNSUPPORTED, "instance %d: K=%d > %d", i, in.K, km::BK_KMAX);
    if (in.n_restarts < 1 || in.n_restarts > km::BK_RMAX)
        return fail(c, KM_EUNSUPPORTED, "instance %d: n_restarts=%d out of [1, %d]", i,
                    in.n_restarts, km::BK_RMAX);
    if (!in.init || !in.centroids_out) return fail(c, KM_EINVAL, "instance %d: NULL init or output", i);
    const int n = in.n_restarts * in.K * in.d;
    for (int q = 0; q < n; ++q)
        if (!isfinite(in.init[q])) return fail(c, KM_EINVAL, "instance %d: init[%d] not finite", i, q);
    int rc = km::check_device_ptr(c, in.X, "X");
    if (!rc && in.labels_out) rc = km::check_device_ptr(c, in.labels_out, "labels_out");
    if (rc) return fail(c, rc, "instance %d: %s", i, c->err.c_str());
    return KM_OK;
}

// Resolve a schedule (zeros = automatic) for a batch on this context.
km_schedule resolve(kmeans_ctx* c, const km_schedule& s, const std::vector<double>& work) {
    km_schedule r = s;
    if (r.team_size <= 0) r.team_size = 8;
    if (r.team_size > km::BK_TEAM_MAX) r.team_size = km::BK_TEAM_MAX;
    if (r.blocks_per_cu <= 0) r.blocks_per_cu = 3;
    if (r.mfma_min_k <= 0) r.mfma_min_k = KM_BATCHED_MFMA_MIN_K;
    if (r.big_work <= 0.0) {
        // default: instances above the 30th percentile of work go to teams.
        // Single blocks take the rest once the teams' list is empty; a
        // higher threshold leaves large instances to single blocks at the
        // end of the launch, where they run alone (measured on the 4096-
        // instance workload: teams of 8 for the top 70 % 1.26 s per call,
        // for the top 30 % 1.51 s).
        std::vector<double> w = work;
        std::sort(w.begin(), w.end());
        r.big_work = w.empty() ? 1.0 : w[(size_t)(0.30 * (double)(w.size() - 1))];
        if (r.big_work < 1.0) r.big_work = 1.0;
    }
    (void)c;
    return r;
}

// One work item of a batched call: restarts [r0, r0 + nr) of instance inst.
struct Item {
    int inst, r0, nr;
};

// The work items of a batch under restart groups of g (0: all of an
// instance's restarts in one item), instance by instance, restarts in order.
std::vector<Item> work_items(int32_t n_inst, const km_instance* inst, int g) {
    std::vector<Item> items;
    for (int i = 0; i < n_inst; ++i) {
        const int R = inst[i].n_restarts;
        const int G = g > 0 ? g : R;
        for (int r0 = 0; r0 < R; r0 += G) items.push_back({i, r0, std::min(G, R - r0)});
    }
    return items;
}

int run_batched(kmeans_ctx* c, int32_t n_inst, km_instance* inst, double tol, int32_t max_iter,
                const km_schedule& sched_in, float* ms_out) {
    if (!c) return KM_EINVAL;
    if (n_inst < 1) return fail(c, KM_EINVAL, "n_inst=%d < 1", n_inst);
    if (!inst) return fail(c, KM_EINVAL, "inst is NULL");
    if (!(tol >= 0.0) || !isfinite(tol)) return fail(c, KM_EINVAL, "tol must be finite and >= 0");
    if (max_iter < 1) return fail(c, KM_EINVAL, "max_iter=%d < 1", max_iter);
    if (sched_in.restart_group < 0 || sched_in.restart_group > km::BK_RMAX)
        return fail(c, KM_EINVAL, "restart_group out of [0, %d]", km::BK_RMAX);
    size_t n_init = 0;
    std::vector<size_t> init_off(n_inst);
    for (int i = 0; i < n_inst; ++i) {
        int rc = validate_instance(c, i, inst[i]);
        if (rc) return rc;
        init_off[i] = n_init;
        n_init += (size_t)inst[i].n_restarts * inst[i].K * inst[i].d;
    }
    // the work items: every restart group of every instance is scheduled as
    // an instance of its own by the kernel (same X, its own restarts)
    const std::vector<Item> items = work_items(n_inst, inst, sched_in.restart_group);
    const int n_items = (int)items.size();
    std::vector<double> work(n_items);
    size_t n_tmp = 0;
    std::vector<size_t> tmp_off(n_items, 0);
    for (int j = 0; j < n_items; ++j) {
        const km_instance& in = inst[items[j].inst];
        work[j] = (double)in.N * in.K * items[j].nr;
        if (items[j].r0 > 0 && in.labels_out) {
            tmp_off[j] = n_tmp;
            n_tmp += (size_t)in.N;
        }
    }
    KM_HIP(c, hipSetDevice(c->device));
    const km_schedule sch = resolve(c, sched_in, work);
    const int occ = km::batched_max_blocks_per_cu();
    if (occ < 1) return fail(c, KM_EHIP, "the batched kernel cannot be resident on this device");
    const int bpc = std::min(sch.blocks_per_cu, occ);
    const int grid = bpc * c->n_cu;
    const int S = sch.team_size;
    int rc = ensure_ws(c, n_items, n_init, grid, n_tmp);
    if (rc) return rc;
    km::BatchedWS* w = c->bws;

    // initial centres, item descriptors, and the two work lists (largest first)
    for (int i = 0; i < n_inst; ++i)
        memcpy(w->init_h + init_off[i], inst[i].init,
               sizeof(double) * (size_t)inst[i].n_restarts * inst[i].K * inst[i].d);
    std::vector<int32_t> big, small;
    for (int j = 0; j < n_items; ++j) {
        const km_instance& in = inst[items[j].inst];
        BInst& b = w->inst_h[j];
        b.X = in.X;
        b.N = in.N;
        b.ld = in.ld;
        b.d = in.d;
        b.K = in.K;
        b.R = items[j].nr;
        b.vec = ((reinterpret_cast<uintptr_t>(in.X) & 15u) == 0 && (in.ld & 3) == 0) ? 1 : 0;
        b.labels = !in.labels_out ? nullptr
                                  : (items[j].r0 == 0 ? in.labels_out : w->tmp_labels + tmp_off[j]);
        b.init = w->init + init_off[items[j].inst] + (size_t)items[j].r0 * in.K * in.d;
        (S > 1 && work[j] >= sch.big_work ? big : small).push_back(j);
    }
    const size_t off = n_init;
    auto larger = [&](int32_t a, int32_t b) { return work[a] > work[b] || (work[a] == work[b] && a < b); };
    std::sort(big.begin(), big.end(), larger);
    std::sort(small.begin(), small.end(), larger);
    std::copy(big.begin(), big.end(), w->order_h);
    std::copy(small.begin(), small.end(), w->order_h + big.size());
    const int n_teams = (S > 1 && !big.empty()) ? grid / S : 0;

    BatchState* h = w->bs_h;
    memset(h, 0, sizeof(BatchState));
    h->inst = w->inst;
    h->order_big = w->order;
    h->order_small = w->order + big.size();
    h->n_inst = n_items;
    h->n_big = n_teams ? (int32_t)big.size() : 0;
    h->n_small = (int32_t)small.size();
    if (!n_teams && !big.empty()) {
        // no teams: every item goes through the single-block list
        std::vector<int32_t> all(n_items);
        std::iota(all.begin(), all.end(), 0);
        std::sort(all.begin(), all.end(), larger);
        std::copy(all.begin(), all.end(), w->order_h);
        h->order_small = w->order;
        h->n_small = n_items;
    }
    h->team_size = n_teams ? S : 1;
    h->mfma_min_k = sch.mfma_min_k;
    h->n_teams = n_teams;
    h->max_iter = max_iter;
    h->tol = tol;
    h->minus_inf = -INFINITY;
    h->absmax = w->absmax;
    h->out = w->out;
    h->best = w->best;
    h->best_mu = w->best_mu;
    h->tpart = w->tpart;
    h->fold = w->fold;
    h->tjpart = w->tjpart;
    h->teams = w->teams;

    KM_HIP(c, hipMemcpyAsync(w->inst, w->inst_h, sizeof(BInst) * n_items, hipMemcpyHostToDevice, c->stream));
    KM_HIP(c, hipMemcpyAsync(w->order, w->order_h, sizeof(int32_t) * n_items, hipMemcpyHostToDevice, c->stream));
    KM_HIP(c, hipMemcpyAsync(w->init, w->init_h, sizeof(double) * off, hipMemcpyHostToDevice, c->stream));
    KM_HIP(c, hipMemcpyAsync(w->bs, h, sizeof(BatchState), hipMemcpyHostToDevice, c->stream));

    // {scan, persistent fit}: one graph per (grid, team size, n_inst)
    const int scan_grid = std::min(n_items, 4 * c->n_cu);
    KM_HIP(c, hipEventRecord(w->ev0, c->stream));
    bool launched = false;
    if (c->use_graph && w->coop_capture_ok) {
        if (!w->graph || w->g_grid != grid || w->g_S != h->team_size || w->g_n != n_items) {
            drop_graph(w);
            hipGraph_t g = nullptr;
            KM_HIP(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
            hipError_t e1 = km::launch_batched_scan(w->bs, n_items, scan_grid, c->cap_stream);
            hipError_t e2 = e1 == hipSuccess ? km::launch_batched_fit(w->bs, grid, c->cap_stream, true)
                                             : e1;
            hipError_t e3 = hipStreamEndCapture(c->cap_stream, &g);
            if (e2 == hipSuccess && e3 == hipSuccess && g) {
                hipGraphExec_t ex = nullptr;
                if (hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) == hipSuccess) {
                    w->graph = ex;
                    w->g_grid = grid;
                    w->g_S = h->team_size;
                    w->g_n = n_items;
                }
            }
            if (g) (void)hipGraphDestroy(g);
            if (!w->graph) {
                w->coop_capture_ok = false;  // launch directly from now on
                (void)hipGetLastError();
            }
        }
        if (w->graph) {
            KM_HIP(c, hipGraphLaunch(w->graph, c->stream));
            launched = true;
        }
    }
    if (!launched) {
        KM_HIP(c, km::launch_batched_scan(w->bs, n_items, scan_grid, c->stream));
        KM_HIP(c, km::launch_batched_fit(w->bs, grid, c->stream, true));
    }
    KM_HIP(c, hipEventRecord(w->ev1, c->stream));
    KM_HIP(c, hipMemcpyAsync(w->out_h, w->out, sizeof(BOut) * n_items * km::BK_RMAX, hipMemcpyDeviceToHost, c->stream));
    KM_HIP(c, hipMemcpyAsync(w->best_h, w->best, sizeof(int32_t) * n_items, hipMemcpyDeviceToHost, c->stream));
    KM_HIP(c, hipMemcpyAsync(w->best_mu_h, w->best_mu, sizeof(double) * n_items * km::BK_KMAX * km::DMAX,
                             hipMemcpyDeviceToHost, c->stream));
    KM_HIP(c, hipMemcpyAsync(w->error_h, &w->bs->error, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
    KM_HIP(c, hipStreamSynchronize(c->stream));
    KM_HIP(c, hipEventElapsedTime(&w->last_ms, w->ev0, w->ev1));
    if (ms_out) *ms_out = w->last_ms;
    if (*w->error_h) return fail(c, KM_EHIP, "a team barrier of the batched kernel timed out");

    // per instance: the kept restart over all of its items (smallest
    // objective, lowest restart index on ties: items and their restarts come
    // in restart order), its outcome and centres, and the copy of its labels
    // when they were written by a later item
    int nonfinite = -1, range = -1;
    int n_copies = 0;
    for (int j0 = 0; j0 < n_items;) {
        const int i = items[j0].inst;
        int j1 = j0;
        while (j1 < n_items && items[j1].inst == i) ++j1;
        km_instance& in = inst[i];
        const BOut* o0 = w->out_h + (size_t)j0 * km::BK_RMAX;
        if (o0[0].iters < 0) {
            if (o0[0].iters == -1 && nonfinite < 0) nonfinite = i;
            if (o0[0].iters == -2 && range < 0) range = i;
            j0 = j1;
            continue;
        }
        int bj = j0, br = 0;
        double bJ = 0.0;
        bool have = false;
        for (int j = j0; j < j1; ++j) {
            const BOut* o = w->out_h + (size_t)j * km::BK_RMAX;
            for (int r = 0; r < items[j].nr; ++r) {
                const int rr = items[j].r0 + r;
                if (in.restart_objective) in.restart_objective[rr] = o[r].J;
                if (in.restart_iters) in.restart_iters[rr] = o[r].iters;
                if (!have || o[r].J < bJ) {
                    have = true;
                    bJ = o[r].J;
                    bj = j;
                    br = r;
                }
            }
        }
        // the item's own kept restart is the instance's (its objective is the
        // smallest, and the first such within the item)
        const BOut& ob = w->out_h[(size_t)bj * km::BK_RMAX + br];
        in.best_restart = items[bj].r0 + br;
        memcpy(in.centroids_out, w->best_mu_h + (size_t)bj * km::BK_KMAX * km::DMAX,
               sizeof(double) * in.K * in.d);
        in.res.iters = ob.iters;
        in.res.converged = ob.converged;
        in.res.E = ob.E;
        in.res.shift_l2 = sqrt(ob.E);
        in.res.objective = ob.J;
        in.res.empty_events = ob.empty_events;
        if (in.labels_out && items[bj].r0 > 0)
            w->copies_h[n_copies++] = km::BCopy{w->tmp_labels + tmp_off[bj], in.labels_out, in.N};
        j0 = j1;
    }
    if (n_copies > 0) {
        KM_HIP(c, hipMemcpyAsync(w->copies, w->copies_h, sizeof(km::BCopy) * n_copies,
                                 hipMemcpyHostToDevice, c->stream));
        KM_HIP(c, km::launch_batched_copy_labels(w->copies, n_copies, c->stream));
        KM_HIP(c, hipStreamSynchronize(c->stream));
    }
    if (nonfinite >= 0)
        return fail(c, KM_EINVAL, "instance %d holds a NaN or an infinity", nonfinite);
    if (range >= 0) {
        km::range_error(c);
        return fail(c, KM_EUNSUPPORTED, "instance %d: %s", range, std::string(c->err).c_str());
    }
    return KM_OK;
}

// ---------------------------------------------------------------- tuner cache
std::string batch_key(int32_t n_inst, const km_instance* inst) {
    int dmask = 0, rmax = 0, kmin = 1 << 30, kmax = 0;
    int64_t nmin = INT64_MAX, nmax = 0;
    for (int i = 0; i < n_inst; ++i) {
        dmask |= 1 << inst[i].d;
        rmax = std::max(rmax, (int)inst[i].n_restarts);
        kmin = std::min(kmin, (int)inst[i].K);
        kmax = std::max(kmax, (int)inst[i].K);
        nmin = std::min(nmin, inst[i].N);
        nmax = std::max(nmax, inst[i].N);
    }
    char buf[160];
    snprintf(buf, sizeof buf, "R%d_d%s_K%d-%d_N1e%d-1e%d", rmax,
             dmask == 12 ? "23" : (dmask == 4 ? "2" : "3"), kmin, kmax,
             (int)floor(log10((double)nmin)), (int)floor(log10((double)nmax)));
    return buf;
}

bool cache_lookup(const char* path, const std::string& key, km_schedule* s) {
    FILE* f = fopen(path, "r");
    if (!f) return false;
    char line[512];
    bool found = false;
    while (fgets(line, sizeof line, f)) {
        char k[200];
        int S = 0, b = 0, g = 0, mk = 0;
        double w = 0.0;
        // one entry per line: {"key": "...", "team_size": S, "blocks_per_cu": b, "big_work": w,
        // "restart_group": g, "mfma_min_k": mk, ...}
        const int n = sscanf(line, " {\"key\": \"%199[^\"]\", \"team_size\": %d, \"blocks_per_cu\": %d, "
                                   "\"big_work\": %lf, \"restart_group\": %d, \"mfma_min_k\": %d",
                             k, &S, &b, &w, &g, &mk);
        if (n >= 4 && key == k) {
            s->team_size = S;
            s->blocks_per_cu = b;
            s->big_work = w;
            s->restart_group = n >= 5 ? g : 0;
            s->mfma_min_k = n >= 6 ? mk : 0;
            found = true;
        }
    }
    fclose(f);
    return found;
}

void cache_store(const char* path, const std::string& key, const km_schedule& s, float ms) {
    FILE* f = fopen(path, "a");
    if (!f) return;
    fprintf(f, "{\"key\": \"%s\", \"team_size\": %d, \"blocks_per_cu\": %d, \"big_work\": %.17g, "
               "\"restart_group\": %d, \"mfma_min_k\": %d, \"ms\": %.4f}\n",
            key.c_str(), s.team_size, s.blocks_per_cu, s.big_work, s.restart_group, s.mfma_min_k, ms);
    fclose(f);
}

}  // namespace

extern "C" {

int kmeans_fit_batched(kmeans_ctx* c, int32_t n_inst, km_instance* inst, double tol,
                       int32_t max_iter) {
    if (!c) return KM_EINVAL;
    c->err.clear();
    return run_batched(c, n_inst, inst, tol, max_iter, c->sched, nullptr);
}

int kmeans_set_batched_schedule(kmeans_ctx* c, const km_schedule* s) {
    if (!c || !s) return KM_EINVAL;
    if (s->team_size < 0 || s->team_size > km::BK_TEAM_MAX)
        return fail(c, KM_EINVAL, "team_size out of [0, %d]", km::BK_TEAM_MAX);
    if (s->blocks_per_cu < 0 || s->blocks_per_cu > 16)
        return fail(c, KM_EINVAL, "blocks_per_cu out of [0, 16]");
    if (!(s->big_work >= 0.0)) return fail(c, KM_EINVAL, "big_work must be >= 0");
    if (s->restart_group < 0 || s->restart_group > km::BK_RMAX)
        return fail(c, KM_EINVAL, "restart_group out of [0, %d]", km::BK_RMAX);
    if (s->mfma_min_k < 0 || s->mfma_min_k > km::BK_KMAX + 1)
        return fail(c, KM_EINVAL, "mfma_min_k out of [0, %d]", km::BK_KMAX + 1);
    c->sched = *s;
    return KM_OK;
}

int kmeans_get_batched_schedule(kmeans_ctx* c, km_schedule* s) {
    if (!c || !s) return KM_EINVAL;
    *s = c->sched;
    return KM_OK;
}

int kmeans_tune_batched(kmeans_ctx* c, int32_t n_inst, km_instance* inst, double tol,
                        int32_t max_iter, const char* cache_path, km_schedule* best) {
    if (!c) return KM_EINVAL;
    c->err.clear();
    if (n_inst < 1 || !inst) return fail(c, KM_EINVAL, "empty batch");
    const std::string key = batch_key(n_inst, inst);
    km_schedule s{};
    if (cache_path && cache_lookup(cache_path, key, &s)) {
        c->sched = s;
        if (best) *best = s;
        return KM_OK;
    }
    // candidates: no teams, or teams of 4/8/16 blocks for the top 90/70/50/30 %
    // of the work items by work; two to four resident blocks per compute unit
    // (as many as fit); every restart of an instance in one item.  Tune on
    // the whole batch where possible: the tail of the launch (the last large
    // items on single blocks) depends on the number of items per block.  Then,
    // from the fastest, restart groups of 4, 2 and 1 (with the same team
    // threshold as a share of the items), then the matrix-core keys.
    int rmax = 1;
    for (int i = 0; i < n_inst; ++i) rmax = std::max(rmax, (int)inst[i].n_restarts);
    auto threshold = [&](int g, double f) {
        const std::vector<Item> items = work_items(n_inst, inst, g);
        std::vector<double> work(items.size());
        for (size_t j = 0; j < items.size(); ++j) {
            const km_instance& in = inst[items[j].inst];
            work[j] = (double)in.N * in.K * items[j].nr;
        }
        std::sort(work.begin(), work.end());
        return std::max(1.0, work[(size_t)(f * (double)(work.size() - 1))]);
    };
    const int occ = km::batched_max_blocks_per_cu();
    struct Cand {
        km_schedule s;
        double f;  // team threshold as a quantile of the items' work (< 0: no teams)
    };
    std::vector<Cand> cand;
    for (int bpc : {2, 3, 4}) {
        if (bpc > occ && bpc > 2) break;
        cand.push_back({{1, bpc, 0.0, 0, 0}, -1.0});
        for (int S : {4, 8, 16})
            for (double f : {0.10, 0.30, 0.50, 0.70})
                cand.push_back({{S, bpc, threshold(0, f), 0, 0}, f});
    }
    float best_ms = 1e30f;
    Cand best_c = cand[0];
    // one warm-up run (allocations, code load), then one timed run per candidate
    int rc = run_batched(c, n_inst, inst, tol, max_iter, cand[0].s, nullptr);
    if (rc) return rc;
    for (const Cand& cs : cand) {
        float ms = 0.f;
        rc = run_batched(c, n_inst, inst, tol, max_iter, cs.s, &ms);
        if (rc) return rc;
        if (ms < best_ms) {
            best_ms = ms;
            best_c = cs;
        }
    }
    for (int g : {4, 2, 1}) {
        if (g >= rmax) continue;
        Cand cs = best_c;
        cs.s.restart_group = g;
        cs.s.big_work = cs.f < 0.0 ? 0.0 : threshold(g, cs.f);
        float ms = 0.f;
        rc = run_batched(c, n_inst, inst, tol, max_iter, cs.s, &ms);
        if (rc) return rc;
        if (ms < best_ms) {
            best_ms = ms;
            best_c = cs;
        }
    }
    // then the matrix-core keys for the 3-D instances from K = 16 or 24
    // (they pay only at the larger K: fewer instructions per point, but a
    // longer dependent chain per restart)
    for (int mk : {24, 16}) {
        bool any = false;
        for (int i = 0; i < n_inst; ++i) any = any || (inst[i].d == 3 && inst[i].K >= mk);
        if (!any) continue;
        Cand cs = best_c;
        cs.s.mfma_min_k = mk;
        float ms = 0.f;
        rc = run_batched(c, n_inst, inst, tol, max_iter, cs.s, &ms);
        if (rc) return rc;
        if (ms < best_ms) {
            best_ms = ms;
            best_c = cs;
        }
    }
    const km_schedule best_s = best_c.s;
    c->sched = best_s;
    if (best) *best = best_s;
    if (cache_path) cache_store(cache_path, key, best_s, best_ms);
    return KM_OK;
}

}  // extern "C"
