// batched_kernels.hip -- many independent Lloyd fits in one persistent launch.
//
// Each instance (its own X, N, d, K) runs R restarts: independent Lloyd
// iterations (the paper's reassignment and mean steps with its error test)
// from R different initial centre sets.  Every point read serves all of the
// instance's active restarts; a restart stops at E < tol or max_iter and is
// masked out of the scan.  After the last update the objective of every
// restart is evaluated at its final centres, the restart with the smallest
// objective (lowest index on ties) is kept, and its labels are written.
//
// Schedule (chosen by the host, tuned by kmeans_tune_batched): the grid is
// persistent and co-resident (cooperative launch).  Blocks [0, n_teams * S)
// form teams of S blocks that take the large instances, largest first, from
// an atomic counter; the team's blocks split the points of the instance,
// publish their integer partial sums to the team's slots, meet at a team
// barrier (an atomic counter), and every block of the team then adds the S
// partials in rank order and performs the same float64 update, so the
// centres never leave the blocks between iterations and one barrier per
// update suffices.  When the large instances run out, and from the start for
// the remaining blocks, single blocks take the small instances, again largest
// first, and run them start to finish with block barriers only.
//
// Per restart, the reassignment, the integer sums of rint(x 2^F) and the
// float64 update are the same device code as the single-instance fit, so
// centres, labels, E and T equal those of kmeans_fit from the same initial
// centres.  A block whose share of an instance exceeds FXP_BLOCK_POINTS
// points takes it in chunks of at most that many, adding each chunk's sums
// into a block-private 128-bit area in device memory (fold), so that no
// int64 slot overflows under any schedule.
#include "batched_copy.h"
#include "lloyd_device.h"

namespace km {
namespace {

enum { MODE_ACC = 0, MODE_OBJ = 1, MODE_LABEL = 2 };
constexpr int BK_ACC = BK_RMAX * BK_KMAX * (DMAX + 1);
// LDS slots for the accumulators: room for 3 copies at the largest shape and
// up to ACC_COPY_MAX copies at small ones (acc_copies).
constexpr int BK_ACC_SLOTS = 3 * BK_ACC;
constexpr int ACC_COPY_MAX = 16;
static_assert(BK_ACC % BLOCK == 0 && BK_ACC_SLOTS >= 2 * BK_ACC,
              "the accumulators hold the 128-bit totals");

// Copies of an instance's accumulators: lane l adds to copy l % copies.
// With few clusters, many of a wave's 64 lanes add to the same slot and their
// LDS atomics serialise; separate copies for lane groups cut that, and the
// copies are summed once per update.
__device__ __forceinline__ int acc_copies(int nacc) {
    const int c = BK_ACC_SLOTS / nacc;
    return c < ACC_COPY_MAX ? c : ACC_COPY_MAX;
}

struct BSmem {
    float4 scand[BK_RMAX][BK_KPAD];
    float4 smu[BK_RMAX][BK_KMAX];
    float4 sbnd[BK_RMAX];
    double mu64[BK_RMAX][BK_KMAX * DMAX];
    unsigned long long acc[BK_ACC_SLOTS];
    float4 queue[NW][QCAP];
    double jw[NW][BK_RMAX];
    double J[BK_RMAX];
    double sE[BK_RMAX][BK_KMAX];
    int sEmpty[BK_RMAX][BK_KMAX];
    float sc[KPAD];
    float sa[3 * KPAD];
    double E[BK_RMAX];
    long long empty[BK_RMAX];
    int t[BK_RMAX];
    int conv[BK_RMAX];
    int active;
    int inst;
    int flag;
};

// Team barrier: every block of the team arrives once per call; nbar counts
// the calls (the same sequence in every block of the team).  Data handed
// across it moves as device-coherent stores and loads (lloyd_device.h): each
// thread waits for its stores before the block arrives.  The wait is
// bounded: after about a second of polling, or when another team has timed
// out, the block records the error and returns false, so no wave can spin
// forever.
__device__ bool team_barrier(BatchState* __restrict__ bs, BTeam* tm, uint32_t& nbar, int S,
                             int* sflag) {
    wait_mem();
    __syncthreads();
    nbar += 1;
    if (threadIdx.x == 0) {
        __hip_atomic_fetch_add(&tm->bar, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const uint32_t target = nbar * (uint32_t)S;
        uint32_t spins = 0;
        int ok = 1;
        while (ld_agent(&tm->bar) < target) {
            __builtin_amdgcn_s_sleep(8);
            ++spins;
            if ((spins & 255u) == 0 && ld_agent(&bs->error)) {
                ok = 0;
                break;
            }
            if (spins > (1u << 21)) {
                st_agent(&bs->error, 1);
                ok = 0;
                break;
            }
        }
        *sflag = ok;
    }
    __syncthreads();
    return *sflag != 0;
}

// One pass over this block's share of the instance's points for the restarts
// in `mask`: MODE_ACC adds the points to their clusters' integer sums,
// MODE_OBJ adds the distances to jl, MODE_LABEL writes the labels.  MODE_OBJ
// and MODE_LABEL take a single restart in `mask`.
// The groups of 4 points taken are [g_lo, g_hi), strided over the team.
template <int D, int MODE>
__device__ void points_pass(const BInst& in, int rank, int S, int mask, double fscale, float ninf,
                            BSmem& sm, double& jl, int64_t g_lo, int64_t g_hi) {
    const int K = in.K;
    const int64_t N = in.N, ld = in.ld;
    const float* __restrict__ X = in.X;
    const bool vec = in.vec != 0;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const uint64_t below = (1ull << lane) - 1ull;
    float4* __restrict__ wq = sm.queue[w];
    int qn = 0;  // this wave's queue length (the same in every lane)

    // add a point's fixed-point coordinates (as fxp_bits, lloyd_device.h) and
    // a count of one to cluster k of restart r; slots are coordinate-major per
    // restart, [(r * (D + 1) + j) * K + k], so that the lanes' clusters spread
    // over the LDS banks
    const int nacc = in.R * K * (D + 1);
    unsigned long long* const myacc = &sm.acc[(lane % acc_copies(nacc)) * nacc];
    auto acc_add = [&](int r, int k, float x0, float x1, float x2) {
        unsigned long long* a = &myacc[r * (D + 1) * K + k];
        const float xs[3] = {x0, x1, x2};
#pragma unroll
        for (int j = 0; j < D; ++j)
            __hip_atomic_fetch_add(&a[j * K], fxp_bits(xs[j], fscale), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_WORKGROUP);
        __hip_atomic_fetch_add(&a[D * K], 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    };
    auto take = [&](int r, int64_t i, float x0, float x1, float x2, int k, float dist) {
        if constexpr (MODE == MODE_ACC) {
            acc_add(r, k, x0, x1, x2);
        } else if constexpr (MODE == MODE_LABEL) {
            in.labels[i] = k;
        }
        if constexpr (MODE == MODE_OBJ) jl += (double)dist;
    };
    auto drain = [&](int cnt) {
        __builtin_amdgcn_wave_barrier();
        if (lane < cnt) {
            const float4 e = wq[qn - cnt + lane];
            const int tag = __float_as_int(e.w);
            const int r = tag >> 27;
            float bd;
            int bk;
            direct_scan<D>(sm.smu[r], K, e.x, e.y, e.z, bd, bk);
            take(r, (int64_t)(tag & ((1 << 27) - 1)), e.x, e.y, e.z, bk, bd);
        }
        __builtin_amdgcn_wave_barrier();
        qn -= cnt;
    };

    const int64_t stride = (int64_t)S * BLOCK;
    for (int64_t gw = g_lo + (int64_t)rank * BLOCK + (threadIdx.x & ~63); gw < g_hi; gw += stride) {
        const int64_t g = gw + lane;
        float x[D][4];
        int n = 0;
        if (g < g_hi) {
            n = load_group_rt<D>(vec, X, ld, N, g, x);
        } else {
#pragma unroll
            for (int j = 0; j < D; ++j)
#pragma unroll
                for (int p = 0; p < 4; ++p) x[j][p] = 0.0f;
        }
#pragma unroll 1
        for (int r = 0; r < BK_RMAX; ++r) {
            if (!((mask >> r) & 1)) continue;
            float best[4];
            int arg[4];
            bool ok[4];
            nearest4<D>(sm.scand[r], sm.smu[r], K, sm.sbnd[r], ninf, x, best, arg, ok);
#pragma unroll
            for (int p = 0; p < 4; ++p) {
                const float x2 = D == 3 ? x[D - 1][p] : 0.0f;
                const bool valid = p < n;
                if (valid && ok[p]) take(r, g * 4 + p, x[0][p], x[1][p], x2, arg[p], best[p]);
                const bool f = valid && !ok[p];
                const uint64_t m = __ballot(f);
                if (m) {
                    if (f)
                        wq[qn + __popcll(m & below)] = make_float4(
                            x[0][p], x[1][p], x2, __int_as_float((r << 27) | (int)(g * 4 + p)));
                    qn += __popcll(m);
                    if (qn >= 64) drain(64);
                }
            }
        }
    }
    if (qn > 0) drain(qn);
}

// Objective partial of the block for restart r, summed over the waves in
// order, into sm.J[r].
__device__ void block_objective(BSmem& sm, int r, double jl) {
    const int w = threadIdx.x >> 6;
    const double v = wave_sum(jl);
    if ((threadIdx.x & 63) == 0) sm.jw[w][r] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
#pragma unroll
        for (int u = 0; u < NW; ++u) s += sm.jw[u][r];
        sm.J[r] = s;
    }
    __syncthreads();
}

// Run instance `inst` to completion.  rank/S: this block's place in its team
// (S = 1: alone).  Returns false when a team barrier timed out.
template <int D>
__device__ bool run_instance(BatchState* __restrict__ bs, int inst, int rank, int S, BTeam* tm,
                             unsigned long long* tpart, double* tjpart, uint32_t& nbar,
                             BSmem& sm) {
    const BInst in = bs->inst[inst];
    const int K = in.K, R = in.R;
    const int tid = threadIdx.x;
    const int nacc = R * K * (D + 1);
    const uint32_t am = bs->absmax[inst];
    const bool bad = am >= FXP_RANGE_BITS;  // non-finite, or beyond the sums' range
    const int xe = data_exponent(am);
    const double fscale = fxp_scale(xe);
    const int64_t ngroups = (in.N + 3) / 4;
    // groups of points per chunk: each block of the team takes at most
    // FXP_BLOCK_POINTS / 4 of them
    const int64_t chunk = (int64_t)S * (FXP_BLOCK_POINTS / 4);
    unsigned long long* const fold = bs->fold + (size_t)blockIdx.x * BK_ACC * 2;
    const float ninf = bs->minus_inf;
    const double tol = bs->tol;
    const int max_iter = bs->max_iter;

    for (int i = tid; i < R * K; i += BLOCK) {
        const int r = i / K, k = i - r * K;
        float m[3] = {0.f, 0.f, 0.f};
#pragma unroll
        for (int j = 0; j < D; ++j) {
            const double v = in.init[(r * K + k) * D + j];
            sm.mu64[r][k * D + j] = v;
            m[j] = (float)v;
        }
        sm.smu[r][k] = make_float4(m[0], m[1], m[2], 0.f);
    }
    if (tid < BK_RMAX) {
        sm.t[tid] = 0;
        sm.conv[tid] = 0;
        sm.E[tid] = INFINITY;
        sm.empty[tid] = 0;
    }
    if (tid == 0) sm.active = bad ? 0 : (1 << R) - 1;
    __syncthreads();
    for (int r = 0; r < R; ++r) prep_centres(sm.smu[r], K, 3 * ((K + 2) / 3), sm.scand[r], &sm.sbnd[r], sm.sc, sm.sa, am);

    double jl = 0.0;
    // ---- Lloyd updates of all active restarts
    for (;;) {
        const int active = __builtin_amdgcn_readfirstlane(sm.active);
        if (!active) break;
        const int copies = acc_copies(nacc);
        for (int64_t g0 = 0; g0 < ngroups; g0 += chunk) {
            const int64_t g1 = g0 + chunk < ngroups ? g0 + chunk : ngroups;
            for (int i = tid; i < copies * nacc; i += BLOCK) sm.acc[i] = 0ull;
            __syncthreads();
            points_pass<D, MODE_ACC>(in, rank, S, active, fscale, ninf, sm, jl, g0, g1);
            __syncthreads();
            // the chunk's sums: copies added, FXP_MAGIC_BITS removed once per
            // point (the count slot of the same restart and cluster), added to
            // the earlier chunks' in 128 bits (in this block's fold area, each
            // slot always by the same thread)
            i128 t[BK_ACC / BLOCK];
#pragma unroll
            for (int u = 0; u < BK_ACC / BLOCK; ++u) {
                const int i = tid + u * BLOCK;
                if (i >= nacc) break;
                const int rj = i / K, k = i - rj * K;
                const int r = rj / (D + 1), j = rj - r * (D + 1);
                const int ic = (r * (D + 1) + D) * K + k;
                unsigned long long n = 0ull;
                for (int c = 0; c < copies; ++c) n += sm.acc[c * nacc + ic];
                unsigned long long v = n;
                if (j < D) {
                    v = 0ull - n * FXP_MAGIC_BITS;
                    for (int c = 0; c < copies; ++c) v += sm.acc[c * nacc + i];
                }
                t[u] = i128_of((long long)v);
                if (g0 > 0) i128_add(t[u], i128{fold[2 * i], (long long)fold[2 * i + 1]});
                if (g1 < ngroups) {
                    fold[2 * i] = t[u].lo;
                    fold[2 * i + 1] = (unsigned long long)t[u].hi;
                }
            }
            __syncthreads();
            if (g1 == ngroups) {
                // the block's totals, as i128, into the accumulators' LDS
                i128* tot = reinterpret_cast<i128*>(sm.acc);
#pragma unroll
                for (int u = 0; u < BK_ACC / BLOCK; ++u) {
                    const int i = tid + u * BLOCK;
                    if (i < nacc) tot[i] = t[u];
                }
                __syncthreads();
            }
        }
        if (S > 1) {
            // the team's sums: every block's 128-bit totals, added in rank order
            const uint32_t par = nbar & 1u;
            i128* tot = reinterpret_cast<i128*>(sm.acc);
            unsigned long long* dst = tpart + ((size_t)par * S + rank) * BK_PART * 2;
            for (int i = tid; i < nacc; i += BLOCK) {
                st_agent(&dst[2 * i], tot[i].lo);
                st_agent(&dst[2 * i + 1], (unsigned long long)tot[i].hi);
            }
            if (!team_barrier(bs, tm, nbar, S, &sm.flag)) return false;
            const unsigned long long* src = tpart + (size_t)par * S * BK_PART * 2;
            for (int i = tid; i < nacc; i += BLOCK) {
                // all S device-coherent loads in flight before the first add
                unsigned long long v[2 * BK_TEAM_MAX];
#pragma unroll
                for (int q = 0; q < BK_TEAM_MAX; ++q) {
                    const unsigned long long* e = &src[((size_t)q * BK_PART + i) * 2];
                    v[2 * q] = q < S ? ld_agent(&e[0]) : 0ull;
                    v[2 * q + 1] = q < S ? ld_agent(&e[1]) : 0ull;
                }
                i128 sum = {0ull, 0ll};
#pragma unroll
                for (int q = 0; q < BK_TEAM_MAX; ++q) i128_add(sum, i128{v[2 * q], (long long)v[2 * q + 1]});
                tot[i] = sum;
            }
            __syncthreads();
        }
        // the same float64 update in every block of the team
        for (int i = tid; i < R * K; i += BLOCK) {
            const int r = i / K, k = i - r * K;
            if (!((active >> r) & 1)) continue;
            const i128* a = reinterpret_cast<const i128*>(sm.acc) + r * (D + 1) * K + k;
            const unsigned long long cnt = a[D * K].lo;
            double e = 0.0;
            float m32[3] = {0.f, 0.f, 0.f};
#pragma unroll
            for (int j = 0; j < D; ++j) {
                const double old = sm.mu64[r][k * D + j];
                const double v = cnt ? fxp_mean(a[j * K], xe, cnt) : old;
                const double sh = v - old;
                e = fma(sh, sh, e);
                sm.mu64[r][k * D + j] = v;
                m32[j] = (float)v;
            }
            sm.smu[r][k] = make_float4(m32[0], m32[1], m32[2], 0.f);
            sm.sE[r][k] = e;
            sm.sEmpty[r][k] = cnt == 0ull;
        }
        __syncthreads();
        if (tid < R && ((active >> tid) & 1)) {
            const int r = tid;
            double E = 0.0;
            int emp = 0;
            for (int k = 0; k < K; ++k) { E += sm.sE[r][k]; emp += sm.sEmpty[r][k]; }
            const int t = sm.t[r] + 1;
            sm.t[r] = t;
            sm.E[r] = E;
            sm.empty[r] += emp;
            sm.conv[r] = E < tol;
            if (E < tol || t >= max_iter) atomicAnd(&sm.active, ~(1 << r));
        }
        __syncthreads();
        const int still = __builtin_amdgcn_readfirstlane(sm.active);
        for (int r = 0; r < R; ++r)
            if ((still >> r) & 1)
                prep_centres(sm.smu[r], K, 3 * ((K + 2) / 3), sm.scand[r], &sm.sbnd[r], sm.sc, sm.sa, am);
        __syncthreads();
    }
    if (!bad) {
        // ---- objective of every restart at its final centres
        for (int r = 0; r < R; ++r) prep_centres(sm.smu[r], K, 3 * ((K + 2) / 3), sm.scand[r], &sm.sbnd[r], sm.sc, sm.sa, am);
        for (int r = 0; r < R; ++r) {
            jl = 0.0;
            points_pass<D, MODE_OBJ>(in, rank, S, 1 << r, fscale, ninf, sm, jl, 0, ngroups);
            block_objective(sm, r, jl);
        }
        if (S > 1) {
            const uint32_t par = nbar & 1u;
            double* dst = tjpart + ((size_t)par * S + rank) * BK_RMAX;
            if (tid < R) st_agent(&dst[tid], sm.J[tid]);
            if (!team_barrier(bs, tm, nbar, S, &sm.flag)) return false;
            const double* src = tjpart + (size_t)par * S * BK_RMAX;
            if (tid < R) {
                double v[BK_TEAM_MAX];
#pragma unroll
                for (int q = 0; q < BK_TEAM_MAX; ++q)
                    v[q] = q < S ? ld_agent(&src[(size_t)q * BK_RMAX + tid]) : 0.0;
                double s = 0.0;
#pragma unroll
                for (int q = 0; q < BK_TEAM_MAX; ++q) s += v[q];  // rank order
                sm.J[tid] = s;
            }
            __syncthreads();
        }
        int best = 0;
        for (int r = 1; r < R; ++r)
            if (sm.J[r] < sm.J[best]) best = r;
        best = __builtin_amdgcn_readfirstlane(best);
        // ---- labels of the kept restart
        if (in.labels)
            points_pass<D, MODE_LABEL>(in, rank, S, 1 << best, fscale, ninf, sm, jl, 0, ngroups);
        if (rank == 0) {
            if (tid < R) {
                BOut o;
                o.iters = sm.t[tid];
                o.converged = sm.conv[tid];
                o.empty_events = sm.empty[tid];
                o.E = sm.E[tid];
                o.J = sm.J[tid];
                bs->out[(size_t)inst * BK_RMAX + tid] = o;
            }
            for (int i = tid; i < K * D; i += BLOCK)
                bs->best_mu[(size_t)inst * BK_KMAX * DMAX + i] = sm.mu64[best][i];
            if (tid == 0) bs->best[inst] = best;
        }
    } else if (rank == 0 && tid < R) {
        // -1: NaN or infinity in this instance's points; -2: max|x| >= 2^28
        BOut o = {am >= 0x7f800000u ? -1 : -2, 0, 0, 0.0, 0.0};
        bs->out[(size_t)inst * BK_RMAX + tid] = o;
        if (tid == 0) bs->best[inst] = 0;
    }
    __syncthreads();
    return true;
}

__device__ bool dispatch(BatchState* __restrict__ bs, int inst, int rank, int S, BTeam* tm,
                         unsigned long long* tpart, double* tjpart, uint32_t& nbar, BSmem& sm) {
    // the instance index came through LDS: tell the compiler it is uniform so
    // that its descriptor lands in scalar registers
    inst = __builtin_amdgcn_readfirstlane(inst);
    if (bs->inst[inst].d == 2) return run_instance<2>(bs, inst, rank, S, tm, tpart, tjpart, nbar, sm);
    return run_instance<3>(bs, inst, rank, S, tm, tpart, tjpart, nbar, sm);
}

// ------------------------------------------------------------ batched_scan
// Block b scans instances b, b + grid, ...: max |x| per instance (fixed-point
// exponent, NaN/Inf detection).  Block 0 also resets the work counters and
// the team barriers for the fit that follows.
__global__ __launch_bounds__(BLOCK) void batched_scan(BatchState* __restrict__ bs) {
    __shared__ uint32_t sm[NW];
    const int tid = threadIdx.x;
    if (blockIdx.x == 0) {
        for (int i = tid; i < bs->n_teams; i += BLOCK) {
            bs->teams[i].bar = 0u;
            bs->teams[i].inst = -1;
        }
        if (tid == 0) {
            bs->big_ctr = 0u;
            bs->small_ctr = 0u;
            bs->error = 0;
        }
    }
    for (int inst = blockIdx.x; inst < bs->n_inst; inst += gridDim.x) {
        const BInst in = bs->inst[inst];
        const int64_t ngroups = (in.N + 3) / 4;
        uint32_t m = 0;
        for (int64_t g = tid; g < ngroups; g += BLOCK) {
            float x[DMAX][4];
            int n;
            if (in.d == 2) {
                float y[2][4];
                n = in.vec ? load_group<2, true>(in.X, in.ld, in.N, g, y)
                           : load_group<2, false>(in.X, in.ld, in.N, g, y);
#pragma unroll
                for (int p = 0; p < 4; ++p) { x[0][p] = y[0][p]; x[1][p] = y[1][p]; x[2][p] = 0.f; }
            } else {
                n = in.vec ? load_group<3, true>(in.X, in.ld, in.N, g, x)
                           : load_group<3, false>(in.X, in.ld, in.N, g, x);
            }
#pragma unroll
            for (int j = 0; j < DMAX; ++j)
#pragma unroll
                for (int p = 0; p < 4; ++p) {
                    const uint32_t b = __float_as_uint(x[j][p]) & 0x7fffffffu;
                    if (p < n) m = b > m ? b : m;
                }
        }
        m = wave_max(m);
        if ((tid & 63) == 0) sm[tid >> 6] = m;
        __syncthreads();
        if (tid == 0) {
            uint32_t b = 0;
            for (int v = 0; v < NW; ++v) b = sm[v] > b ? sm[v] : b;
            bs->absmax[inst] = b;
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------ batched_fit
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(3, 8))) void batched_fit(BatchState* __restrict__ bs) {
    __shared__ BSmem sm;
    const int S = bs->team_size;
    const int b = blockIdx.x;
    uint32_t nbar = 0;
    if (S > 1 && b < bs->n_teams * S) {
        const int ti = b / S, rank = b - ti * S;
        BTeam* tm = &bs->teams[ti];
        unsigned long long* tpart = bs->tpart + (size_t)ti * 2 * S * BK_PART * 2;
        double* tjpart = bs->tjpart + (size_t)ti * 2 * S * BK_RMAX;
        for (;;) {
            if (rank == 0 && threadIdx.x == 0) {
                const uint32_t idx = atomicAdd(&bs->big_ctr, 1u);
                st_agent(&tm->inst, idx < (uint32_t)bs->n_big ? bs->order_big[idx] : -1);
            }
            if (!team_barrier(bs, tm, nbar, S, &sm.flag)) return;
            if (threadIdx.x == 0) sm.inst = ld_agent(&tm->inst);
            __syncthreads();
            const int inst = sm.inst;
            __syncthreads();
            if (inst < 0) break;
            if (!dispatch(bs, inst, rank, S, tm, tpart, tjpart, nbar, sm)) return;
            // keeps the leader from publishing the next instance before every
            // block of the team has read this one
            if (!team_barrier(bs, tm, nbar, S, &sm.flag)) return;
        }
    }
    for (;;) {
        if (threadIdx.x == 0) {
            const uint32_t idx = atomicAdd(&bs->small_ctr, 1u);
            sm.inst = idx < (uint32_t)bs->n_small ? bs->order_small[idx] : -1;
        }
        __syncthreads();
        const int inst = sm.inst;
        __syncthreads();
        if (inst < 0) return;
        dispatch(bs, inst, 0, 1, nullptr, nullptr, nullptr, nbar, sm);
    }
}

}  // namespace

// Label copies (batched_copy.h): block b takes entries b, b + grid, ...
__global__ __launch_bounds__(BLOCK) void batched_copy_labels(const BCopy* __restrict__ tab, int n) {
    for (int t = blockIdx.x; t < n; t += gridDim.x) {
        const BCopy c = tab[t];
        for (int64_t i = threadIdx.x; i < c.n; i += BLOCK) c.dst[i] = c.src[i];
    }
}

hipError_t launch_batched_copy_labels(const BCopy* tab, int n, hipStream_t s) {
    if (n < 1) return hipSuccess;
    const int grid = n < 1024 ? n : 1024;
    hipLaunchKernelGGL(batched_copy_labels, dim3(grid), dim3(BLOCK), 0, s, tab, n);
    return hipGetLastError();
}

hipError_t launch_batched_scan(BatchState* bs, int n_inst, int grid, hipStream_t s) {
    if (grid < 1) return hipErrorInvalidValue;
    (void)n_inst;
    hipLaunchKernelGGL(batched_scan, dim3(grid), dim3(BLOCK), 0, s, bs);
    return hipGetLastError();
}

hipError_t launch_batched_fit(BatchState* bs, int grid, hipStream_t s, bool cooperative) {
    if (grid < 1) return hipErrorInvalidValue;
    if (cooperative) {
        void* args[] = {&bs};
        return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(batched_fit), dim3(grid),
                                          dim3(BLOCK), args, 0, s);
    }
    hipLaunchKernelGGL(batched_fit, dim3(grid), dim3(BLOCK), 0, s, bs);
    return hipGetLastError();
}

int batched_max_blocks_per_cu() {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, reinterpret_cast<const void*>(batched_fit),
                                                     BLOCK, 0) != hipSuccess)
        return 0;
    return n;
}

}  // namespace km
