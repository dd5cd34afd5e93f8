// lloyd_kernels.hip -- gfx950 kernels of one Lloyd iteration.
//
// Paper: "The Lloyd's Algorithm" (reassignment argmin, mean calculation with
// the indicator function) and "Serial Lloyd's Algorithm" (error E between
// successive centres, tolerance test).
//
// Kernels
//   km_scan      one pass over X: max |x| (sets the exponent of the fixed-point
//                sums, flags NaN/Inf and data beyond their range); prepares
//                the centre tables.
//   lloyd_iter   one whole update: reassignment of every point, per-cluster
//                integer sums and counts in LDS, one partial per block, a
//                two-level reduction of the partials by the last block of each
//                group and then the last group, and in that final block the
//                float64 divide, the empty-cluster rule, E and the tolerance
//                test.  No host synchronisation between iterations.
//   lloyd_label  reassignment only: labels and the objective for the current
//                centres (final labels of a fit; the assign entry point).
//
// Reassignment: see lloyd_device.h.
//
// Determinism: the per-cluster sums are exact integer sums of rint(x 2^F)
// (|x| 2^F < 2^44, lloyd_device.h), so their value does not depend on the
// order in which points, waves or blocks add them: results are identical for
// any grid size and from run to run, without float atomics.  The
// objective (reported, not fed back) is summed per lane, reduced across the
// wave with a fixed butterfly and across waves, blocks and groups in index
// order.
#include "lloyd_device.h"
#include "lloyd_mfma.h"

namespace km {
namespace {

// Publish this block's objective partial and take a ticket; true in the last
// block of the grid to arrive (single-level; used by the label kernel).
__device__ bool finish_block(uint32_t* ticket, double* jslot, double jblock, int* sflag) {
    __syncthreads();
    if (threadIdx.x == 0) {
        st_agent(jslot, jblock);
        wait_mem();
        const uint32_t old = __hip_atomic_fetch_add(ticket, 1u, __ATOMIC_RELAXED,
                                                    __HIP_MEMORY_SCOPE_AGENT);
        *sflag = (old == gridDim.x - 1);
    }
    __syncthreads();
    return *sflag != 0;
}

// Sum of the per-block objective partials in block order; whole block.
__device__ double sum_partials(const double* __restrict__ jpart, int nb, double* sred) {
    const int tid = threadIdx.x;
    double s = 0.0;
    for (int b = tid; b < nb; b += BLOCK) s += ld_agent(&jpart[b]);
    s = wave_sum(s);
    __syncthreads();
    if ((tid & 63) == 0) sred[tid >> 6] = s;
    __syncthreads();
    double tot = 0.0;
#pragma unroll
    for (int w = 0; w < NW; ++w) tot += sred[w];
    return tot;
}

// For every entry i < nr: the sum over q < n of the partial P(q, i) (an
// i128), into out[i] (LDS).  The loads are spread over the whole block --
// each thread takes a slice of q for one entry, 8 device-coherent loads in
// flight at a time -- and the slices are added in LDS (integer sums: the
// order does not matter).  scr: LDS scratch of BLOCK values.
template <typename F>
__device__ __forceinline__ void sum_entries(int n, int nr, F P, i128* out, i128* scr) {
    const int tid = threadIdx.x;
    const int S = BLOCK / nr;                 // slices per entry (nr <= BLOCK)
    const int slice = tid / nr, i = tid - slice * nr;
    i128 s = {0ull, 0ll};
    if (slice < S) {
        const int per = (n + S - 1) / S;
        const int q0 = slice * per;
        const int q1 = q0 + per < n ? q0 + per : n;
        for (int qb = q0; qb < q1; qb += 8) {
            i128 t[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) t[u] = qb + u < q1 ? P(qb + u, i) : i128{0ull, 0ll};
#pragma unroll
            for (int u = 0; u < 8; ++u) i128_add(s, t[u]);
        }
    }
    scr[tid] = s;
    __syncthreads();
    for (int j = tid; j < nr; j += BLOCK) {
        i128 t = {0ull, 0ll};
        for (int sl = 0; sl < S; ++sl) i128_add(t, scr[sl * nr + j]);
        out[j] = t;
    }
    __syncthreads();
}

// Sum of the n float64 values p[0..n) in index order (all loads in flight at
// once, the additions by thread 0 from LDS); the result is valid in thread 0.
__device__ __forceinline__ double sum_in_order(int n, const double* p, double* sj) {
    for (int q = threadIdx.x; q < n; q += BLOCK) sj[q] = ld_agent(&p[q]);
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int q = 0; q < n; ++q) s += sj[q];
    return s;
}

// Partials handled by the last block alone when it can load them in two
// batches per thread (one-level reduction).
constexpr int ONE_LEVEL_LOADS = 16 * BLOCK;

// Two-level reduction of the block partials (integer sums | counts, and the
// objective).  Every block publishes its partial (int64: a block adds at
// most FXP_BLOCK_POINTS points); the last block of each group of GROUP
// blocks adds the group's partials in 128 bits; the last group adds the
// group sums.  With at most MAX_GROUPS blocks and ONE_LEVEL_LOADS partial
// entries in all, the last block of the grid adds the partials directly.
// Returns true in that one final block, with the grid totals in tot[0..nr)
// (LDS) and the objective in *jtot.  No two blocks add to the same address,
// so there is no contention; the integer sums are exact in any order and the
// objective is added in block, then group, order.  Partials move as
// device-coherent stores and loads (see lloyd_device.h).  acc: LDS of nr
// i128 for the group sums and the totals; scr, sj: LDS scratch of BLOCK
// i128 and MAX_GROUPS doubles.
__device__ __forceinline__ bool reduce_grid(State* __restrict__ st, const unsigned long long* blk,
                                            int nr, double jb, i128* acc, i128* scr, double* sj,
                                            double* jtot, int* sflag) {
    const int tid = threadIdx.x;
    const int b = blockIdx.x, nb = gridDim.x;
    unsigned long long* mine = st->part + (size_t)b * PART;
    for (int i = tid; i < nr; i += BLOCK) st_agent(&mine[i], blk[i]);
    if (tid == 0) st_agent(&st->jpart[b], jb);
    wait_mem();
    __syncthreads();
    const unsigned long long* part = st->part;
    auto block_partial = [&](int q, int i) {
        return i128_of((long long)ld_agent(&part[(size_t)q * PART + i]));
    };
    if (nb <= MAX_GROUPS && nb * nr <= ONE_LEVEL_LOADS) {
        // few partials: the last block of the grid adds them all (one round
        // trip of device-coherent exchanges fewer)
        if (tid == 0) {
            const uint32_t old = __hip_atomic_fetch_add(&st->ticket, 1u, __ATOMIC_RELAXED,
                                                        __HIP_MEMORY_SCOPE_AGENT);
            *sflag = (old == (uint32_t)nb - 1);
        }
        __syncthreads();
        if (!*sflag) return false;
        sum_entries(nb, nr, block_partial, acc, scr);
        const double jt = sum_in_order(nb, st->jpart, sj);
        if (tid == 0) {
            *jtot = jt;
            st_agent(&st->ticket, 0u);
        }
        __syncthreads();
        return true;
    }
    const int grp = b / GROUP, g0 = grp * GROUP;
    const int gn = (nb - g0) < GROUP ? (nb - g0) : GROUP;
    if (tid == 0) {
        const uint32_t old = __hip_atomic_fetch_add(&st->gticket[grp], 1u, __ATOMIC_RELAXED,
                                                    __HIP_MEMORY_SCOPE_AGENT);
        *sflag = (old == (uint32_t)gn - 1);
    }
    __syncthreads();
    if (!*sflag) return false;
    // last block of its group: the group's sums (128-bit, as lo / hi words)
    sum_entries(gn, nr, [&](int q, int i) { return block_partial(g0 + q, i); }, acc, scr);
    unsigned long long* gmine = st->gpart + (size_t)grp * PART * 2;
    for (int i = tid; i < nr; i += BLOCK) {
        st_agent(&gmine[2 * i], acc[i].lo);
        st_agent(&gmine[2 * i + 1], (unsigned long long)acc[i].hi);
    }
    const double jg = sum_in_order(gn, st->jpart + g0, sj);
    if (tid == 0) {
        st_agent(&st->gjpart[grp], jg);
        st_agent(&st->gticket[grp], 0u);
    }
    wait_mem();
    __syncthreads();
    const int ng = (nb + GROUP - 1) / GROUP;
    if (tid == 0) {
        const uint32_t old = __hip_atomic_fetch_add(&st->ticket, 1u, __ATOMIC_RELAXED,
                                                    __HIP_MEMORY_SCOPE_AGENT);
        *sflag = (old == (uint32_t)ng - 1);
    }
    __syncthreads();
    if (!*sflag) return false;
    // the final block
    const unsigned long long* gpart = st->gpart;
    sum_entries(ng, nr, [&](int q, int i) {
        const unsigned long long* e = &gpart[((size_t)q * PART + i) * 2];
        return i128{ld_agent(&e[0]), (long long)ld_agent(&e[1])};
    }, acc, scr);
    const double jt = sum_in_order(ng, st->gjpart, sj);
    if (tid == 0) {
        *jtot = jt;
        st_agent(&st->ticket, 0u);
    }
    __syncthreads();
    return true;
}

// ---------------------------------------------------------------- km_scan
template <int D, bool VEC>
__global__ __launch_bounds__(BLOCK) void km_scan(State* __restrict__ st) {
    __shared__ uint32_t sm[NW];
    __shared__ float sc[KPAD];
    __shared__ float sa[3 * KPAD];
    __shared__ int slast;
    const int tid = threadIdx.x;
    const float* __restrict__ X = st->X;
    const int64_t N = st->N, ld = st->ld;
    const int64_t ngroups = (N + 3) / 4;
    uint32_t m = 0;
    for (int64_t g = (int64_t)blockIdx.x * BLOCK + tid; g < ngroups;
         g += (int64_t)gridDim.x * BLOCK) {
        float x[D][4];
        const int n = load_group<D, VEC>(X, ld, N, g, x);
#pragma unroll
        for (int j = 0; j < D; ++j)
#pragma unroll
            for (int p = 0; p < 4; ++p) {
                const uint32_t b = __float_as_uint(x[j][p]) & 0x7fffffffu;
                if (p < n) m = b > m ? b : m;  // NaN bits exceed Inf bits
            }
    }
    m = wave_max(m);
    if ((tid & 63) == 0) sm[tid >> 6] = m;
    __syncthreads();
    if (tid == 0) {
        uint32_t b = 0;
        for (int w = 0; w < NW; ++w) b = sm[w] > b ? sm[w] : b;
        __hip_atomic_fetch_max(&st->absmax_bits, b, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        wait_mem();
        const uint32_t old = __hip_atomic_fetch_add(&st->scan_ticket, 1u, __ATOMIC_RELAXED,
                                                    __HIP_MEMORY_SCOPE_AGENT);
        slast = (old == gridDim.x - 1);
    }
    __syncthreads();
    if (!slast) return;
    const uint32_t a = ld_agent(&st->absmax_bits);
    prep_centres(st->mu32, st->K, KPAD, st->cand, &st->bnd, sc, sa, a);
    for (int i = tid; i < MAX_GROUPS; i += BLOCK) st->gticket[i] = 0u;
    if (tid == 0) {
        st->xe = data_exponent(a);
        if (a >= 0x7f800000u) {  // NaN or infinity in X
            st->flags |= FLAG_NONFINITE;
            st->done = 1;
        } else if (a >= FXP_RANGE_BITS) {  // beyond the fixed-point sums' range
            st->flags |= FLAG_RANGE;
            st->done = 1;
        }
        st->scan_ticket = 0;
        st->ticket = 0;
    }
}

// The reassignment scan: KT == 0 the VALU keys (assign_points), KT = 1, 2 the
// matrix-core keys with KT tiles of 32 centres (assign_points_mfma).  Both
// give the same labels.
template <int D, bool VEC, int KT, typename Sink>
__device__ __forceinline__ void scan_points(const float* __restrict__ X, int64_t ld, int64_t N,
                                            const float4* __restrict__ scand,
                                            const float4* __restrict__ smu, int K,
                                            float4 bnd, float ninf, int xe,
                                            float4* __restrict__ wq, Sink&& sink) {
    int e = 0;
    if constexpr (KT != 0) {
        if (mfma_scale(xe, bnd, e)) {
            assign_points_mfma<D, VEC, KT>(X, ld, N, scand, smu, K, bnd, e, ninf, wq, sink);
            return;
        }
    }
    // the VALU keys (also for data or centres beyond the matrix-core scale's
    // range)
    assign_points<D, VEC>(X, ld, N, scand, smu, K, bnd, ninf, wq, sink);
}

// ---------------------------------------------------------------- lloyd_iter
// LDS of one update.
// The block's per-cluster accumulators in LDS: ACC_SLOTS int64 slots hold
// `copies` = min(ACC_COPY_MAX, ACC_SLOTS / (K (d+1))) copies of the K d sums
// (the counts in a parallel 32-bit array: a block never counts 2^32 points),
// and thread t adds to copy t % copies.  With few clusters
// many lanes of a wave would add to the same slot, and LDS atomics on one
// slot serialise; the copies spread them, and are summed once per pass.
constexpr int ACC_SLOTS = 2 * KMAX * (DMAX + 1);
constexpr int ACC_COPY_MAX = 16;

struct IterSmem {
    float4 scand[KPAD];
    float4 smu[KMAX];
    // copy c at [c * KS * (d+1)], coordinate-major inside: slot j * KS + k
    // (KS = K, or 32 KT with the matrix-core scan).
    // After the pass: the group sums and grid totals of the reduction
    // (KMAX * (DMAX + 1) i128, the same bytes).
    unsigned long long sacc[ACC_SLOTS];
    unsigned int scnt[ACC_SLOTS / 2];  // counts, 32-bit: copy c at [c * KS], slot k
    // storage used in turn by the scan (re-scan queues), the block totals
    // until they are published, the reduction's scratch, and the final
    // block's update
    union {
        float4 squeue[NW][QCAP];
        unsigned long long stot[KMAX * (DMAX + 1)];
        struct {
            i128 scr[BLOCK];
            double sj[MAX_GROUPS];
        } red;
        struct {
            double sE[KMAX];
            int sEmpty[KMAX];
            float sc[KPAD];
            float sa[3 * KPAD];
        } fin;
    } u;
    double sred[NW];
    uint32_t schg[NW];  // labels changed per wave (indicator tracking)
    float4 sbnd;
    double sJ;
    int sflag;
    int sdone;
};
static_assert(sizeof(unsigned long long) * ACC_SLOTS >= sizeof(i128) * KMAX * (DMAX + 1),
              "the accumulators hold the grid totals");

// float4 through four device-coherent 32-bit accesses (lloyd_device.h).
__device__ __forceinline__ void st4_agent(float4* p, float4 v) {
    float* f = reinterpret_cast<float*>(p);
    st_agent(&f[0], v.x); st_agent(&f[1], v.y); st_agent(&f[2], v.z); st_agent(&f[3], v.w);
}
__device__ __forceinline__ float4 ld4_agent(const float4* p) {
    const float* f = reinterpret_cast<const float*>(p);
    return make_float4(ld_agent(&f[0]), ld_agent(&f[1]), ld_agent(&f[2]), ld_agent(&f[3]));
}

// Plain accesses for state that only later kernels (or the host) read, and
// device-coherent ones for state that other blocks of the same (persistent)
// kernel read.
template <bool COH, typename T>
__device__ __forceinline__ T rd(const T* p) {
    if constexpr (COH) return ld_agent(p);
    else return *p;
}
template <bool COH, typename T>
__device__ __forceinline__ void wr(T* p, T v) {
    if constexpr (COH) st_agent(p, v);
    else *p = v;
}
template <bool COH>
__device__ __forceinline__ void wr4(float4* p, float4 v) {
    if constexpr (COH) st4_agent(p, v);
    else *p = v;
}

// One reassignment + accumulation pass over the grid's points against the
// centre tables in sm (the paper's reassignment step and the numerators and
// denominators of its mean step), reduced across the grid.  Returns true in
// the one final block, with the grid's integer sums | counts in sm.sacc
// and the objective of this pass in sm.sJ.
// TRACK (indicator tracking): each point's label of the previous update is
// read from st->track, the new one written there where it differs, and the
// block's number of changed labels travels with the counts through the
// reduction: it is added, times 2^32, to cluster 0's count (a block counts
// at most 2^19 points and a fit at most 2^31 - 1, so the two fields never
// overlap).
template <int D, bool VEC, int KT, bool TRACK>
__device__ __forceinline__ bool update_pass(State* __restrict__ st, IterSmem& sm, int K, int xe,
                            float4 bnd, float ninf) {
    constexpr int R = D + 1;  // per cluster: D sums, 1 count
    const int tid = threadIdx.x, w = tid >> 6;
    const int64_t N = st->N, ld = st->ld;
    const float* __restrict__ X = st->X;
    // slots per coordinate row: K, or with the matrix-core scan the compile-
    // time 32 KT (>= K), so that the rows sit at immediate offsets
    const int KS = KT ? 32 * KT : K;
    const int KR = KS * R;
    const int copies = ACC_SLOTS / KR < ACC_COPY_MAX ? ACC_SLOTS / KR : ACC_COPY_MAX;
    for (int i = tid; i < copies * KR; i += BLOCK) sm.sacc[i] = 0ull;
    for (int i = tid; i < copies * KS; i += BLOCK) sm.scnt[i] = 0u;
    __syncthreads();

    double jl = 0.0;
    const double fscale = fxp_scale(xe);
    unsigned long long* myacc = &sm.sacc[(tid % copies) * KR];
    unsigned int* mycnt = &sm.scnt[(tid % copies) * KS];
    int32_t* __restrict__ track = st->track;
    uint32_t nchg = 0;
    scan_points<D, VEC, KT>(X, ld, N, sm.scand, sm.smu, K, bnd, ninf, xe, sm.u.squeue[w],
                            [&](int64_t i, float x0, float x1, float x2, int k, float dist) {
        if constexpr (TRACK) {
            if (track[i] != k) {
                track[i] = k;
                ++nchg;
            }
        }
        // coordinate-major slots [j * KS + k]: the 64 lanes' clusters spread
        // over the LDS banks (a cluster-major stride of 4 int64 would put
        // every cluster on one of a few bank groups)
        unsigned long long* a = &myacc[k];
        const float xs[3] = {x0, x1, x2};
#pragma unroll
        for (int j = 0; j < D; ++j)
            __hip_atomic_fetch_add(&a[j * KS], fxp_bits(xs[j], fscale), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_WORKGROUP);
        __hip_atomic_fetch_add(&mycnt[k], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        jl += (double)dist;
    });
    jl = wave_sum(jl);
    if constexpr (TRACK) nchg = wave_sum_u32(nchg);
    if ((tid & 63) == 0) {
        sm.sred[w] = jl;
        sm.schg[w] = nchg;
    }
    __syncthreads();
    // block totals, cluster-major [k * R + j]: the sums of q (each slot less
    // FXP_MAGIC_BITS per point it received) and the counts
    for (int i = tid; i < K * R; i += BLOCK) {
        const int k = i / R, j = i - k * R;
        unsigned long long n = 0ull;
        for (int c = 0; c < copies; ++c) n += sm.scnt[c * KS + k];
        unsigned long long s = n;
        if (j < D) {
            s = 0ull - n * FXP_MAGIC_BITS;
            for (int c = 0; c < copies; ++c) s += sm.sacc[c * KR + j * KS + k];
        }
        if (TRACK && i == D) {
            unsigned long long c = 0ull;
#pragma unroll
            for (int v = 0; v < NW; ++v) c += sm.schg[v];
            s += c << 32;
        }
        sm.u.stot[i] = s;
    }
    double jb = 0.0;
#pragma unroll
    for (int v = 0; v < NW; ++v) jb += sm.sred[v];
    __syncthreads();
    return reduce_grid(st, sm.u.stot, K * R, jb, reinterpret_cast<i128*>(sm.sacc), sm.u.red.scr,
                       sm.u.red.sj, &sm.sJ, &sm.sflag);
}

// The final block's update (the paper's mean-calculation step, its error E
// and tolerance test): new float64 centres (an empty cluster keeps its
// centre), E, the history, t and done; and the next pass's centre tables,
// left in sm (smu, scand, sbnd, sdone) and stored to the state.  COH: the
// state is also read by other blocks of a persistent kernel, so every access
// to it is device-coherent.
template <int D, bool COH, bool TRACK>
__device__ __forceinline__ void finalize_update(State* __restrict__ st, IterSmem& sm, int K, int xe) {
    constexpr int R = D + 1;
    const int tid = threadIdx.x;
    const i128* tot = reinterpret_cast<const i128*>(sm.sacc);
    // the state read at the end, loaded first: its round trip overlaps the
    // centres' (only this block writes these fields during the update)
    int t0 = 0, hcap = 0, max_iter = 0;
    int64_t emp0 = 0;
    double tol = 0.0;
    if (tid == 0) {
        t0 = rd<COH>(&st->t);
        emp0 = rd<COH>(&st->empty_events);
        hcap = st->hist_cap;
        max_iter = st->max_iter;
        tol = st->tol;
    }
    if (tid < K) {
        const int k = tid;
        // the count's low 32 bits (cluster 0's carries the changed labels
        // above them, see update_pass)
        const unsigned long long cnt = tot[k * R + D].lo & 0xffffffffull;
        double e = 0.0;
        float m32[DMAX] = {0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int j = 0; j < D; ++j) {
            const double old = rd<COH>(&st->mu64[k * D + j]);
            const double v = cnt ? fxp_mean(tot[k * R + j], xe, cnt) : old;
            const double sh = v - old;
            e = fma(sh, sh, e);
            wr<COH>(&st->mu64[k * D + j], v);
            m32[j] = (float)v;
        }
        const float4 m = make_float4(m32[0], m32[1], m32[2], 0.0f);
        wr4<COH>(&st->mu32[k], m);
        sm.smu[k] = m;
        sm.u.fin.sE[k] = e;
        sm.u.fin.sEmpty[k] = cnt == 0ull;
    }
    __syncthreads();
    prep_centres(sm.smu, K, KPAD, sm.scand, &sm.sbnd, sm.u.fin.sc, sm.u.fin.sa, st->absmax_bits);
    for (int i = tid; i < KPAD; i += BLOCK) wr4<COH>(&st->cand[i], sm.scand[i]);
    if (tid == 0) {
        wr4<COH>(&st->bnd, sm.sbnd);
        double E = 0.0;
        int emp = 0;
        for (int k = 0; k < K; ++k) { E += sm.u.fin.sE[k]; emp += sm.u.fin.sEmpty[k]; }
        const int t = t0;
        if (t < hcap) { st->E_hist[t] = E; st->J_hist[t] = sm.sJ; }
        int done = (E < tol || t + 1 >= max_iter) ? 1 : 0;
        if constexpr (TRACK) {
            // the paper's other criterion: no indicator changed
            const long long chg = (long long)(tot[D].lo >> 32);
            if (t < hcap) st->C_hist[t] = chg;
            st->changed = chg;
            if (chg == 0) done = 1;
        }
        wr<COH>(&st->t, t + 1);
        wr<COH>(&st->E, E);
        wr<COH>(&st->empty_events, emp0 + emp);
        wr<COH>(&st->done, done);
        sm.sdone = done;
    }
    __syncthreads();
}

static_assert(KPAD <= BLOCK && KMAX <= BLOCK, "one table entry per thread");

// One update per launch (replayed from a graph): the update's pass, then the
// final block's update of the centres.
template <int D, bool VEC, int KT, bool TRACK>
__device__ __forceinline__ void iter_body(State* __restrict__ st, IterSmem& sm) {
    const int K = st->K;
    // the centre tables' loads go out before the done test (one round trip at
    // the start of an update instead of two); KPAD and K are at most BLOCK
    const int tid = threadIdx.x;
    const float4 rc = tid < KPAD ? st->cand[tid] : make_float4(0.f, 0.f, 0.f, 0.f);
    const float4 rm = tid < K ? st->mu32[tid] : make_float4(0.f, 0.f, 0.f, 0.f);
    if (st->done) return;
    if (tid < KPAD) sm.scand[tid] = rc;
    if (tid < K) sm.smu[tid] = rm;
    __syncthreads();
    if (!update_pass<D, VEC, KT, TRACK>(st, sm, K, st->xe, st->bnd, st->minus_inf)) return;
    finalize_update<D, false, TRACK>(st, sm, K, st->xe);
}

template <int D, bool VEC, int KT>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(6, 8))) void lloyd_iter(State* __restrict__ st) {
    __shared__ IterSmem sm;
    iter_body<D, VEC, KT, false>(st, sm);
}

// The same with indicator tracking (KM_OPT_TRACK).
template <int D, bool VEC, int KT>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(6, 8))) void lloyd_iter_track(State* __restrict__ st) {
    __shared__ IterSmem sm;
    iter_body<D, VEC, KT, true>(st, sm);
}

// The whole fit in one cooperative launch (every block resident), for small
// N where a launch per update would cost more than the update.  Each update:
// the same pass and final-block update as lloyd_iter; the final block then
// publishes the round number, and every other block waits for it and
// reloads the new centre tables (device-coherent loads) before the next
// pass.  The wait is bounded: a block that polls for about a second records
// FLAG_TIMEOUT and returns, as do the others once they see it, so no wave
// spins forever.
constexpr uint32_t PERSIST_SPIN_LIMIT = 1u << 21;

template <int D, bool VEC, int KT>
__global__ __launch_bounds__(BLOCK) void lloyd_persist(State* __restrict__ st) {
    if (st->done) return;
    __shared__ IterSmem sm;
    const int tid = threadIdx.x;
    const int K = st->K;
    const int xe = st->xe;
    const float ninf = st->minus_inf;
    stage_centres(st, K, sm.scand, sm.smu);
    float4 bnd = st->bnd;
    __syncthreads();
    for (uint32_t round = 1;; ++round) {
        if (update_pass<D, VEC, KT, false>(st, sm, K, xe, bnd, ninf)) {
            finalize_update<D, true, false>(st, sm, K, xe);
            wait_mem();
            __syncthreads();
            if (tid == 0) st_agent(&st->gen, round);
        } else {
            if (tid == 0) {
                int ok = 1;
                uint32_t spins = 0;
                while (ld_agent(&st->gen) < round) {
                    __builtin_amdgcn_s_sleep(4);
                    ++spins;
                    if ((spins & 255u) == 0 && (ld_agent(&st->flags) & FLAG_TIMEOUT)) {
                        ok = 0;
                        break;
                    }
                    if (spins > PERSIST_SPIN_LIMIT) {
                        __hip_atomic_fetch_or(&st->flags, (int32_t)FLAG_TIMEOUT, __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_AGENT);
                        ok = 0;
                        break;
                    }
                }
                sm.sflag = ok;
            }
            __syncthreads();
            if (!sm.sflag) return;
            for (int i = tid; i < KPAD; i += BLOCK) sm.scand[i] = ld4_agent(&st->cand[i]);
            for (int k = tid; k < K; k += BLOCK) sm.smu[k] = ld4_agent(&st->mu32[k]);
            if (tid == 0) {
                sm.sbnd = ld4_agent(&st->bnd);
                sm.sdone = ld_agent(&st->done);
            }
        }
        __syncthreads();
        if (sm.sdone) break;
        bnd = sm.sbnd;
    }
}

// ---------------------------------------------------------------- lloyd_label
template <int D, bool VEC, int KT>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(6, 8))) void lloyd_label(State* __restrict__ st,
                                                     int32_t* __restrict__ labels) {
    if (st->flags & FLAG_NONFINITE) return;
    __shared__ float4 scand[KPAD];
    __shared__ float4 smu[KMAX];
    __shared__ float4 squeue[NW][QCAP];
    __shared__ double sred[NW];
    __shared__ int sflag;
    const int tid = threadIdx.x, w = tid >> 6;
    const int K = st->K;
    const int64_t N = st->N, ld = st->ld;
    const float* __restrict__ X = st->X;
    const float4 bnd = st->bnd;
    const float ninf = st->minus_inf;
    stage_centres(st, K, scand, smu);
    __syncthreads();
    double jl = 0.0;
    scan_points<D, VEC, KT>(X, ld, N, scand, smu, K, bnd, ninf, st->xe, squeue[w],
                            [&](int64_t i, float, float, float, int k, float dist) {
        if (labels) labels[i] = k;
        jl += (double)dist;
    });
    jl = wave_sum(jl);
    if ((tid & 63) == 0) sred[w] = jl;
    __syncthreads();
    double jb = 0.0;
#pragma unroll
    for (int v = 0; v < NW; ++v) jb += sred[v];
    if (!finish_block(&st->ticket, &st->jpart[blockIdx.x], jb, &sflag)) return;
    const double J = sum_partials(st->jpart, gridDim.x, sred);
    if (tid == 0) {
        st->J = J;
        st->ticket = 0;
    }
}

}  // namespace

#define KM_DISPATCH(KERNEL, GRID, STREAM, ...)                                        \
    do {                                                                              \
        if (d == 2 && vec)       hipLaunchKernelGGL((KERNEL<2, true>), dim3(GRID), dim3(BLOCK), 0, STREAM, __VA_ARGS__); \
        else if (d == 2)         hipLaunchKernelGGL((KERNEL<2, false>), dim3(GRID), dim3(BLOCK), 0, STREAM, __VA_ARGS__); \
        else if (d == 3 && vec)  hipLaunchKernelGGL((KERNEL<3, true>), dim3(GRID), dim3(BLOCK), 0, STREAM, __VA_ARGS__); \
        else if (d == 3)         hipLaunchKernelGGL((KERNEL<3, false>), dim3(GRID), dim3(BLOCK), 0, STREAM, __VA_ARGS__); \
        else return hipErrorInvalidValue;                                             \
    } while (0)

// The scan variants: keys 0 = VALU, 1 / 2 = matrix cores with 1 / 2 tiles of
// 32 centres.
#define KM_DISPATCH_SCAN(KERNEL, GRID, STREAM, ...)                                   \
    do {                                                                              \
        if (keys == 0) {                                                              \
            if (d == 2 && vec)      hipLaunchKernelGGL((KERNEL<2, true, 0>), dim3(GRID), dim3(BLOCK), 0, STREAM, __VA_ARGS__); \
            else if (d == 2)        hipLaunchKernelGGL((KERNEL<2, false, 0>), dim3(GRID), dim3(BLOCK), 0, STREAM, __VA_ARGS__); \
            else if (d == 3 && vec) hipLaunchKernelGGL((KERNEL<3, true, 0>), dim3(GRID), dim3(BLOCK), 0, STREAM, __VA_ARGS__); \
            else if (d == 3)        hipLaunchKernelGGL((KERNEL<3, false, 0>), dim3(GRID), dim3(BLOCK), 0, STREAM, __VA_ARGS__); \
            else return hipErrorInvalidValue;                                         \
        } else if (keys == 1) {                                                       \
            if (d == 2 && vec)      hipLaunchKernelGGL((KERNEL<2, true, 1>), dim3(GRID), dim3(BLOCK), 0, STREAM, __VA_ARGS__); \
            else if (d == 2)        hipLaunchKernelGGL((KERNEL<2, false, 1>), dim3(GRID), dim3(BLOCK), 0, STREAM, __VA_ARGS__); \
            else if (d == 3 && vec) hipLaunchKernelGGL((KERNEL<3, true, 1>), dim3(GRID), dim3(BLOCK), 0, STREAM, __VA_ARGS__); \
            else if (d == 3)        hipLaunchKernelGGL((KERNEL<3, false, 1>), dim3(GRID), dim3(BLOCK), 0, STREAM, __VA_ARGS__); \
            else return hipErrorInvalidValue;                                         \
        } else if (keys == 2) {                                                       \
            if (d == 2 && vec)      hipLaunchKernelGGL((KERNEL<2, true, 2>), dim3(GRID), dim3(BLOCK), 0, STREAM, __VA_ARGS__); \
            else if (d == 2)        hipLaunchKernelGGL((KERNEL<2, false, 2>), dim3(GRID), dim3(BLOCK), 0, STREAM, __VA_ARGS__); \
            else if (d == 3 && vec) hipLaunchKernelGGL((KERNEL<3, true, 2>), dim3(GRID), dim3(BLOCK), 0, STREAM, __VA_ARGS__); \
            else if (d == 3)        hipLaunchKernelGGL((KERNEL<3, false, 2>), dim3(GRID), dim3(BLOCK), 0, STREAM, __VA_ARGS__); \
            else return hipErrorInvalidValue;                                         \
        } else {                                                                      \
            return hipErrorInvalidValue;                                              \
        }                                                                             \
    } while (0)

hipError_t launch_scan(State* st, int d, bool vec, int grid, hipStream_t s) {
    if (grid < 1 || grid > MAX_BLOCKS) return hipErrorInvalidValue;
    KM_DISPATCH(km_scan, grid, s, st);
    return hipGetLastError();
}

hipError_t launch_iter(State* st, int d, bool vec, int keys, bool track, int grid,
                       hipStream_t s) {
    if (grid < 1 || grid > MAX_BLOCKS) return hipErrorInvalidValue;
    if (track) KM_DISPATCH_SCAN(lloyd_iter_track, grid, s, st);
    else KM_DISPATCH_SCAN(lloyd_iter, grid, s, st);
    return hipGetLastError();
}

hipError_t launch_persist(State* st, int d, bool vec, int grid, hipStream_t s) {
    if (grid < 1 || grid > MAX_BLOCKS) return hipErrorInvalidValue;
    void* args[] = {&st};
    const void* f = nullptr;
    if (d == 2 && vec) f = reinterpret_cast<const void*>(lloyd_persist<2, true, 0>);
    else if (d == 2) f = reinterpret_cast<const void*>(lloyd_persist<2, false, 0>);
    else if (d == 3 && vec) f = reinterpret_cast<const void*>(lloyd_persist<3, true, 0>);
    else if (d == 3) f = reinterpret_cast<const void*>(lloyd_persist<3, false, 0>);
    else return hipErrorInvalidValue;
    return hipLaunchCooperativeKernel(f, dim3(grid), dim3(BLOCK), args, 0, s);
}

int persist_max_blocks_per_cu(int d, bool vec) {
    const void* f = d == 2 ? (vec ? reinterpret_cast<const void*>(lloyd_persist<2, true, 0>)
                                  : reinterpret_cast<const void*>(lloyd_persist<2, false, 0>))
                           : (vec ? reinterpret_cast<const void*>(lloyd_persist<3, true, 0>)
                                  : reinterpret_cast<const void*>(lloyd_persist<3, false, 0>));
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, f, BLOCK, 0) != hipSuccess) return 0;
    return n;
}

hipError_t launch_label(State* st, int32_t* labels, int d, bool vec, int keys, int grid,
                        hipStream_t s) {
    if (grid < 1 || grid > MAX_BLOCKS) return hipErrorInvalidValue;
    KM_DISPATCH_SCAN(lloyd_label, grid, s, st, labels);
    return hipGetLastError();
}

}  // namespace km
