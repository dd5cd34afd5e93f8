/*
 * kmeans.h -- C ABI of the MI355X (gfx950) Lloyd K-means library
 * (libkmeans_mi355x.so).
 *
 * The operation is Lloyd's algorithm as defined in the paper's section "The
 * Lloyd's Algorithm": starting from K initial centres, repeat
 *   reassignment   z_i = argmin_k ||x_i - mu_k||_2^2            (every point)
 *   mean           mu_k' = sum_{z_i=k} x_i / #{i : z_i = k}      (every cluster)
 * and, as in the section "Serial Lloyd's Algorithm", after every update form
 *   E = sum_k ||mu_k' - mu_k||_2^2
 * and stop once E is below a tolerance (of the order of 1e-6 in the paper).
 * The inputs are the data set, the number of clusters and the number of
 * points; the outputs are the final cluster indicators and means (problem
 * statement and serial-algorithm sections).
 *
 * Conventions shared by every entry point
 *   - X is caller-owned DEVICE memory: d rows of N float32, row j starting at
 *     X + j*ld (structure of arrays; the paper's X in R^{d x N}).  ld >= N.
 *     When X is 16-byte aligned and ld is a multiple of 4 the kernels use
 *     128-bit loads; otherwise they fall back to 32-bit loads (same results).
 *   - Centres passed in or out are caller-owned HOST arrays of K*d float64,
 *     row-major (centre k at [k*d, k*d+d)).  float64 centres make resuming a
 *     fit from its output exact.
 *   - Labels are caller-owned DEVICE int32 arrays of N, 0-based (the paper
 *     numbers clusters 1..K).
 *   - Reassignment compares squared distances to the centres rounded to
 *     float32.  A point whose nearest centre wins by more than the rounding
 *     of the computation (a certified bound) gets that centre; near-ties are
 *     decided by the direct form (x0-m0)^2 + (x1-m1)^2 + ... +
 *     (x_{d-1}-m_{d-1})^2 evaluated in float64 (each difference, square and
 *     partial sum rounded to float64, left to right), first index of the
 *     minimum.  A certified margin is far above float64 rounding, so every
 *     label is the first-index minimum of that float64 distance, whichever
 *     scan (KM_OPT_KEYS, KM_OPT_WIDE) ran and whichever points it certified.
 *     The objective sums, in float64, the float32 direct-form distances
 *     (left to right, the first term a product, the others fused
 *     multiply-adds) to the chosen centres.
 *     Per-cluster sums are exact integer sums of the points rounded to the
 *     grid 2^-F, F = 43 - ilogb(max|x|) (so every |x| 2^F < 2^44), carried
 *     in 128 bits across blocks; the divide, E and the tolerance test are
 *     float64.  Each mean is therefore within 2^(ilogb(max|x|) - 44) <=
 *     max|x| 2^-44 per coordinate of the exact mean of its points.  Fits
 *     (kmeans_fit, kmeans_fit_batched) return KM_EUNSUPPORTED, after their
 *     scan of X and before any update, for data with max|x| >= 2^28, where
 *     that bound could exceed 1e-5 for a cluster near the origin (scale such
 *     data first); kmeans_assign takes no sums and has no such limit.
 *     Results do not depend on the launch configuration and repeat bit for
 *     bit from run to run.
 *   - An empty cluster keeps its previous centre and is counted.
 *   - Supported shapes: 1 <= d <= 32, 1 <= K <= 4096, K <= N <= 2^31 - 1.
 *     d in {2, 3} with K <= 64 runs the 2-D/3-D kernels, every other shape
 *     the general-shape kernels (same definitions, same results up to the
 *     objective's summation order).  Those keep one block's sums and centre
 *     tables in LDS when 8*K*(d+1) + 4*Kp*s + 4*Kp (the first and last
 *     rounded up to 16) + 2224 <= 65536 bytes, Kp = K rounded up to a
 *     multiple of 3, s = the padded width (d for d <= 4; then 6, 8, 12, 16,
 *     24 or 32) rounded up to a multiple of 4 (d <= 4: K <= 1024; d = 8:
 *     K <= 585; d = 16: K <= 309; d = 32: K <= 159); larger K takes their
 *     tiled form (centres staged through LDS in tiles, sums in device
 *     memory), with the same results.  kmeans_fit_batched: d in {2, 3},
 *     K <= 32, N <= 2^27, up to 8 restarts.
 *   - Every call is synchronous with respect to the host: it returns after
 *     its device work on the context's stream has completed.  There is no
 *     host synchronisation between iterations of a fit.
 *   - A context is bound to one device and one HIP stream and is not
 *     thread-safe; use one context per host thread.
 *
 * Errors: every int-returning call returns KM_OK (0) or a negative code.  All
 * argument validation happens before any device work; on error nothing on
 * the device has been modified and kmeans_last_error() describes the cause.
 * Not converging within max_iter is not an error (km_result.converged = 0).
 */
#ifndef KMEANS_MI355X_H
#define KMEANS_MI355X_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define KMEANS_ABI_VERSION 2

typedef struct kmeans_ctx kmeans_ctx;

enum km_status {
    KM_OK = 0,
    KM_EINVAL = -1,       /* invalid argument (null pointer, bad size, NaN)   */
    KM_ENODEV = -2,       /* no usable GPU, or device index out of range      */
    KM_EHIP = -3,         /* a HIP runtime call failed                        */
    KM_ENOMEM = -4,       /* device or pinned-host allocation failed          */
    KM_EUNSUPPORTED = -5  /* d or K outside what the kernels implement        */
};

/* Outcome of a fit. */
typedef struct km_result {
    int32_t iters;        /* T: updates performed (1 <= T <= max_iter)        */
    int32_t converged;    /* 1 when the last update had E < tol               */
    double E;             /* E of the last update                             */
    double shift_l2;      /* sqrt(E): Frobenius norm of the last centre shift */
    double objective;     /* sum_i min_k ||x_i - mu_k||^2 at the final centres
                             (float32 distances, summed in float64)           */
    int64_t empty_events; /* sum over the updates of clusters left empty     */
} km_result;

/* Options for kmeans_set_option. */
enum km_option {
    KM_OPT_GRAPH = 1,     /* 1 (default): replay iterations from a hipGraph;
                             0: launch each iteration kernel directly          */
    KM_OPT_UNROLL = 2,    /* iterations per graph launch (0 = automatic)       */
    KM_OPT_BLOCKS = 3,    /* grid size of the iteration kernel (0 = automatic;
                             raised to N / 2^19 blocks where smaller, so that
                             no block adds more than 2^19 points into its
                             int64 sums)                                       */
    KM_OPT_TIMING = 4,    /* 1: time the iteration launches with HIP events
                             (see kmeans_get_timing)                           */
    KM_OPT_KEYS = 5,      /* how the reassignment scan forms its keys
                             |m|^2 - 2 m.x: 0 (default) automatic, 1 vector
                             ALUs, 2 matrix cores (fp16 MFMA on hi/lo pieces
                             of the operands).  Automatic: in the 2-D/3-D
                             kernels the matrix cores for 24 < K <= 32 and
                             K > 44 (data or centres beyond about 2^36 or
                             below 2^-48 in magnitude take the vector ALUs);
                             in the general-shape kernels the matrix cores for
                             padded widths 8, 12 and 16 (7 <= d <= 16) with
                             K >= 64 whose operand tables fit in 64 KB of LDS
                             (at d = 16: K <= 256), with 2 the same shapes at
                             any K (beyond the scale range every point takes
                             the float64 re-scan).  Labels, centres, E and T
                             do not depend on it.                               */
    KM_OPT_PERSIST = 6,   /* how kmeans_fit runs its updates: 0 (default)
                             and 1: graph replays of one launch per update
                             (measured as fast or faster at every size); 2:
                             one persistent cooperative launch whenever the
                             VALU scan is used and the grid fits on the
                             device.  Results do not depend on it.             */
    KM_OPT_WIDE = 7,      /* 1: run kmeans_fit and kmeans_assign on the
                             general-shape kernels for every shape (a cross-
                             check of the two implementations); 0 (default):
                             only for shapes outside d in {2, 3}, K <= 64.     */
    KM_OPT_TRACK = 8      /* indicator tracking ("The Lloyd's Algorithm": the
                             iteration has converged once no cluster indicator
                             changes).  1: kmeans_fit keeps every point's label
                             in labels_out (required, device, N int32) from
                             update to update -- each update reads a point's
                             previous label and writes the new one where it
                             differs (4 to 8 more bytes of traffic per point
                             and update) -- counts the points whose label
                             changed (kmeans_get_changes; the first update
                             counts all N) and also stops after the first
                             update that changes none (converged = 1).  The
                             per-cluster sums are exact, so that update's E is
                             0 and the centres, labels and T are those of
                             tol = 4.9e-324 unless an update trades points
                             between clusters without changing any sum (two
                             distinct points equal on the sums' grid of
                             2^(ilogb(max|x|) - 43) swapping clusters).  0
                             (default): off.  Not with kmeans_fit_batched or
                             kmeans_fit_noalloc.                              */
};

/*
 * Create a context on HIP device `device` that enqueues all work on
 * `hip_stream` (a hipStream_t; NULL = the device's null stream).  `flags` is
 * reserved and must be 0.  On success *out owns its device workspace, pinned
 * host staging and graph cache until kmeans_destroy.
 * Returns KM_ENODEV when no GPU is present or `device` is out of range.
 */
int kmeans_create(kmeans_ctx **out, int device, void *hip_stream, uint32_t flags);

/* Release everything the context owns.  NULL is accepted. */
void kmeans_destroy(kmeans_ctx *ctx);

/* Message describing the last error on `ctx` ("" if none).  Valid until the
 * next call on the same context.  With ctx == NULL: the last error of a
 * failed kmeans_create in this thread. */
const char *kmeans_last_error(const kmeans_ctx *ctx);

/* Static name of a status code. */
const char *kmeans_status_string(int status);

/* ABI version this library implements (KMEANS_ABI_VERSION). */
int kmeans_abi_version(void);

/*
 * Host-only argument check of a fit of N points of dimension d (row stride
 * ld) into K clusters: the same rules kmeans_fit applies before any device
 * work.  Needs no GPU.  Returns KM_OK, KM_EINVAL or KM_EUNSUPPORTED.
 */
int kmeans_validate(int64_t N, int64_t ld, int32_t d, int32_t K, double tol,
                    int32_t max_iter);

/*
 * Reassignment step alone (the paper's step 2) for the given centres:
 * writes labels[i] = argmin_k ||x_i - mu_k||^2 (if labels != NULL, device)
 * and *objective = sum_i min_k ||x_i - mu_k||^2 (if objective != NULL, host).
 * `centroids` is a host array of K*d float64.
 */
int kmeans_assign(kmeans_ctx *ctx, const float *X, int64_t N, int64_t ld,
                  int32_t d, int32_t K, const double *centroids,
                  int32_t *labels, double *objective);

/*
 * Lloyd's algorithm (the paper's steps 1-3 with its error test) from the
 * host centres `init` (K*d float64) until E < tol or max_iter updates.
 * Writes the final centres to centroids_out (host, K*d float64), the labels
 * against those final centres to labels_out (device, may be NULL) and the
 * outcome to *res (may be NULL).
 * tol must be finite and >= 0 (tol = 0 runs exactly max_iter updates;
 * tol = 4.9e-324, the smallest positive double, stops at the first update
 * with E == 0: the per-cluster sums are exact, so this is the update after
 * the indicators stopped changing -- the paper's convergence criterion);
 * max_iter >= 1.  Returns KM_EINVAL (after the run) if X holds a NaN or an
 * infinity, KM_EUNSUPPORTED (after the scan) if max|x| >= 2^28.
 */
int kmeans_fit(kmeans_ctx *ctx, const float *X, int64_t N, int64_t ld,
               int32_t d, int32_t K, const double *init, double tol,
               int32_t max_iter, double *centroids_out, int32_t *labels_out,
               km_result *res);

/*
 * kmeans_fit for callers that cannot allocate memory (code that must not
 * call hipMalloc or create graphs, streams or events: tight serving loops,
 * harnesses that forbid allocation).  Same arguments, results and error
 * codes as kmeans_fit, without a context: `device` is the HIP device (made
 * current for the call, the caller's current device restored on return) and
 * `hip_stream` the stream of that device to run on (NULL: its null stream).
 * Shapes: d in {2, 3} and K <= 64, else KM_EUNSUPPORTED; N, ld, tol and
 * max_iter as kmeans_fit.  Errors are read with kmeans_last_error(NULL) (per
 * host thread).
 * Scratch: the fit's device state, partial sums, tickets and E/J history
 * live in one statically sized device array of about 8.6 MB, which the
 * library holds on every device it runs on until the process ends (no
 * history is kept for reading back; updates beyond 1024 run unrecorded).
 * The call allocates no device or host memory; the initial state is copied
 * from, and the results read back into, memory on the caller's stack.
 * Calls that overlap on one device (from two threads, or on two streams)
 * share that array and race: serialise them.
 */
int kmeans_fit_noalloc(int device, void *hip_stream, const float *X, int64_t N,
                       int64_t ld, int32_t d, int32_t K, const double *init,
                       double tol, int32_t max_iter, double *centroids_out,
                       int32_t *labels_out, km_result *res);

/* Set a km_option on the context.  Returns KM_EINVAL for an unknown option
 * or a value out of range. */
int kmeans_set_option(kmeans_ctx *ctx, int32_t option, int64_t value);

/*
 * Per-update history of the last kmeans_fit on `ctx`: E_t and the objective
 * J_t of the centres each update started from.  Copies min(cap, T) entries
 * into E and J (host, either may be NULL) and returns that count (or a
 * negative status).
 */
int kmeans_get_history(kmeans_ctx *ctx, double *E, double *J, int32_t cap);

/*
 * With KM_OPT_TRACK on during the last kmeans_fit on `ctx`: the number of
 * points whose label changed in each update (the first update: N).  Copies
 * min(cap, T) entries into `changed` (host, may be NULL) and returns that
 * count; KM_EINVAL if the last fit did not track its indicators.
 */
int kmeans_get_changes(kmeans_ctx *ctx, int64_t *changed, int32_t cap);

/*
 * With KM_OPT_TIMING on: total device time (ms, HIP events on the context's
 * stream) of the iteration launches of the last kmeans_fit, and the number of
 * iteration kernels those launches contained (for a persistent fit: the one
 * launch's time and the number of updates it performed).
 */
int kmeans_get_timing(kmeans_ctx *ctx, double *iter_ms, int64_t *iter_kernels);

/* ---------------------------------------------------------- batched fits */

/* One instance of a batched fit: its own points and K, and n_restarts
 * independent Lloyd runs from different initial centres, of which the one
 * with the smallest final objective is kept. */
typedef struct km_instance {
    const float *X;             /* device, d rows of N float32, row stride ld  */
    int64_t N;
    int64_t ld;
    int32_t d;                  /* 2 or 3                                       */
    int32_t K;                  /* 1..32                                        */
    int32_t n_restarts;         /* 1..8                                         */
    const double *init;         /* host, n_restarts*K*d initial centres          */
    double *centroids_out;      /* host, K*d: final centres of the kept restart  */
    int32_t *labels_out;        /* device, N labels of the kept restart, or NULL */
    double *restart_objective;  /* host, n_restarts final objectives, or NULL    */
    int32_t *restart_iters;     /* host, n_restarts update counts T, or NULL      */
    int32_t best_restart;       /* out: index of the kept restart                */
    km_result res;              /* out: outcome of the kept restart              */
} km_instance;

/* Launch schedule of kmeans_fit_batched (see kmeans_tune_batched). */
typedef struct km_schedule {
    int32_t team_size;          /* blocks that share one large instance (1..16; 1 = no teams) */
    int32_t blocks_per_cu;      /* persistent grid = blocks_per_cu x compute units (capped by
                                   occupancy)                                       */
    double big_work;            /* work items with N*K*restarts >= big_work go to teams */
    int32_t restart_group;      /* restart fusion: an instance's restarts run as work items of
                                   at most restart_group restarts each, every item scanning its
                                   restarts in one pass over the points (1..8; 0 = all of
                                   them in one item).  Results do not depend on it.      */
    int32_t mfma_min_k;         /* 3-D instances with K >= mfma_min_k reassign with the
                                   matrix-core keys (all their restarts' centres as rows of
                                   32-row tiles), the others with the VALU keys (1..33;
                                   33 = never; 0 = the default, KM_BATCHED_MFMA_MIN_K).
                                   Results do not depend on it.                          */
} km_schedule;

/* Default of km_schedule.mfma_min_k: the VALU keys everywhere (on the mixed
   4096-instance batch the matrix-core keys from K = 16 measured 2.6 % slower;
   on uniform batches of 3-D instances at K = 32, 15 % faster). */
#define KM_BATCHED_MFMA_MIN_K 33

/*
 * Many independent fits in one persistent launch (the points of every
 * instance must stay valid until the call returns).  Every restart follows
 * exactly the iteration of kmeans_fit (same labels, centres, E and T as a
 * kmeans_fit from the same initial centres, tol and max_iter); afterwards the
 * objective of each restart is evaluated at its final centres and the
 * smallest is kept (lowest restart index on ties).  Constraints per
 * instance: d in {2, 3}, 1 <= K <= 32, K <= N <= 2^27, 1 <= n_restarts <= 8,
 * ld >= N.  Returns KM_EINVAL if any instance holds a NaN or an infinity,
 * KM_EUNSUPPORTED if any has max|x| >= 2^28 (after the run; the other
 * instances' outputs are valid).
 */
int kmeans_fit_batched(kmeans_ctx *ctx, int32_t n_inst, km_instance *inst, double tol,
                       int32_t max_iter);

/* Set / read the schedule used by kmeans_fit_batched on this context. */
int kmeans_set_batched_schedule(kmeans_ctx *ctx, const km_schedule *s);
int kmeans_get_batched_schedule(kmeans_ctx *ctx, km_schedule *s);

/*
 * Autotuner of the batched schedule: times kmeans_fit_batched on `inst`
 * (the workload itself, or a sample of it: the end of a launch, when the last
 * large instances run on single blocks, depends on the number of instances
 * per block, so a small sample can mislead) for each candidate schedule (team
 * size 1, 4, 8, 16; teams for the top 90/70/50/30 % of work items by N*K*R;
 * 2-4 blocks per compute unit; all restarts fused), then, from the fastest,
 * restart groups of 4, 2 and 1 where the batch has more restarts per
 * instance, then the matrix-core keys for 3-D instances from K = 24 and 16
 * (km_schedule.mfma_min_k), and keeps the fastest on the context and
 * writes it to *best (may be NULL).  If cache_path is not NULL the result is
 * looked up first and stored afterwards in that JSON file, keyed by a coarse
 * signature of the batch (restarts, d mix, K and N ranges).  Results of the
 * fits do not depend on the schedule (integer cluster sums), except the last
 * bits of the objectives.
 */
int kmeans_tune_batched(kmeans_ctx *ctx, int32_t n_inst, km_instance *inst, double tol,
                        int32_t max_iter, const char *cache_path, km_schedule *best);

/* ------------------------------------------------ learned initialiser */
/*
 * A small permutation-invariant network proposes the K initial centres of a
 * 3-D instance from a sample of P of its points, to cut the number of Lloyd
 * updates (the paper notes that the initialisation steers the result and that
 * the iteration count grows with N).  Architecture, on points normalised by
 * the sample's mean and scalar standard deviation s (s^2 = mean over points
 * and coordinates of (x - mean)^2):
 *   per point  h1 = relu(x W1 + b1) (3 -> 64), h2 = relu(h1 W2 + b2) (64 -> 64)
 *   pooling    p = [mean over points of h2, max over points of h2]  (128)
 *   head       z = relu(p W3 + b3) (128 -> 256), y = z W4 + b4 (256 -> 3K)
 * y holds K normalised centres; centre = y * s + mean.  Weights are float32
 * masters used as bfloat16 copies; the per-point products run on bfloat16
 * MFMA with float32 accumulation.  Training minimises
 *   L = (1/B) sum_b sum_k |y_b[pi_b(k)] - t_b[k]|^2
 * against target centres t (normalised the same way), pi_b the least-cost
 * assignment (Hungarian matching on the device, held fixed for the gradient).
 *
 * Parameters: one caller-owned DEVICE float32 array of
 * kmeans_initnet_param_count(K) values, row-major blocks W1 [3][64], b1 [64],
 * W2 [64][64], b2 [64], W3 [128][256], b3 [256], W4 [256][3K], b4 [3K]
 * (rows = inputs).  Points: DEVICE float32 [B][P][3] (normalised); targets:
 * DEVICE float32 [B][K][3].  Shapes: 1 <= B <= 4096, P a multiple of 32 in
 * [32, 65536], 1 <= K <= 16.
 */

/* Number of floats in the parameter array for K centres (-1 if K is out of
 * range).  Needs no GPU. */
int32_t kmeans_initnet_param_count(int32_t K);

/* Forward pass: pred_out (device [B][K][3]) and optionally the pooled
 * features pool_out (device [B][128]). */
int kmeans_initnet_forward(kmeans_ctx *ctx, const float *pts, int32_t B, int32_t P,
                           int32_t K, const float *params, float *pred_out, float *pool_out);

/* Gradient of L at `params` into grad_out (device, parameter layout); the
 * loss to *loss_out (host, may be NULL) and the matching pi to match_out
 * (device [B][K], the predicted centre assigned to each target, may be NULL). */
int kmeans_initnet_grad(kmeans_ctx *ctx, const float *pts, const float *targets, int32_t B,
                        int32_t P, int32_t K, const float *params, float *grad_out,
                        double *loss_out, int32_t *match_out);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected for `step`
 * >= 1) on params with the moment arrays adam_m, adam_v (device, parameter
 * layout, zero before step 1).  *loss_out (host, may be NULL: then the call
 * returns without waiting for the device) receives the loss before the step. */
int kmeans_initnet_train_step(kmeans_ctx *ctx, const float *pts, const float *targets,
                              int32_t B, int32_t P, int32_t K, float *params, float *adam_m,
                              float *adam_v, float lr, int32_t step, double *loss_out);

/* Initial centres of one 3-D instance (X as in kmeans_fit, d = 3) from the P
 * sample points idx[0..P) (device int32 indices into [0, N); P a multiple of
 * 32 in [32, 4096]): gather, normalise, forward pass, de-normalise, into
 * centroids_out (host, K*3 float64).  The per-point layers run as up to 16
 * equal slices of the sample in parallel, pooled together (mean of the slice
 * means, max of the slice maxima), so the result equals kmeans_initnet_forward
 * on the normalised sample up to float32 summation order.  Returns KM_EINVAL
 * if the network yields a non-finite centre (callers then fall back to a
 * seeded sample of data points). */
int kmeans_init_learned(kmeans_ctx *ctx, const float *X, int64_t N, int64_t ld, int32_t K,
                        const int32_t *idx, int32_t P, const float *params,
                        double *centroids_out);

/* ------------------------------------------------------ k-means++ seeding */

/*
 * k-means++ initial centres (Arthur and Vassilvitskii, 2007): an alternative
 * to the paper's random choice of initial centres (the first step of "The
 * Lloyd's Algorithm", whose outcome the paper notes depends on that choice).  The draw is exact
 * and reproducible given the caller's K uniforms u[0..K) (host, each in
 * [0, 1)):
 *   - centre 0 is point min(N-1, floor(u[0] * N));
 *   - for j >= 1, D_i^2 is the float32 squared distance of point i to its
 *     nearest chosen centre, ((x0-c0)^2 + (x1-c1)^2) + (x2-c2)^2 with each
 *     operation rounded on its own; w_i = rint(D_i^2 * 2^G) as a 64-bit
 *     integer with G = B - ilogb(max_i D_i^2) - 1, B = 62 - ceil(log2 N);
 *     S = sum_i w_i; if S == 0 centre j is point min(N-1, floor(u[j] * N)),
 *     else with R = min(S-1, floor(u[j] * S)) it is the first point i whose
 *     inclusive prefix sum w_0 + ... + w_i exceeds R.
 * X is as in kmeans_fit (device, d rows of N float32, row stride ld).
 * Writes the chosen points to centroids_out (host, K*d float64) and their
 * indices to index_out (host, K int64; may be NULL).  Same shape limits as
 * kmeans_fit.  Returns KM_EINVAL for a u outside [0, 1) or if X holds a NaN
 * or an infinity.  Keeps a distance buffer of N floats on the context.
 */
int kmeans_pp_init(kmeans_ctx *ctx, const float *X, int64_t N, int64_t ld, int32_t d,
                   int32_t K, const double *u, double *centroids_out, int64_t *index_out);

/* ------------------------------------------------------ measured peaks */

/*
 * Measured issue rates on the context's device, for reading a kernel's
 * roofline position against what the hardware sustains rather than only
 * against published peaks: rates[0] non-packed float32 FMA (v_fma_f32),
 * rates[1] v_min3_f32 and rates[2] v_med3_f32, each in lane-operations per
 * second (16 independent chains per lane, 16 waves per SIMD, register
 * operands); rates[3] the read rate of a 1 GiB device buffer in bytes per
 * second.  Allocates and frees 1 GiB of device memory; takes about a
 * second.
 */
int kmeans_measure_peaks(kmeans_ctx *ctx, double rates[4]);

#ifdef __cplusplus
}
#endif
#endif /* KMEANS_MI355X_H */
