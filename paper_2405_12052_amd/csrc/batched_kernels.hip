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
#include "lloyd_mfma.h"

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

// The update pass (MODE_ACC) with matrix-core keys for all active restarts of
// the instance at once: the single fit's split-fp16 keys, packed quad minima,
// VALU re-key of the winning quad and certificate (lloyd_mfma.h), so the
// labels equal the VALU pass's.  Rows of the 32-row tiles are (restart,
// centre) slots: each restart owns SW consecutive rows (SW = 8, 16 or 32 >=
// K; slots past K are pads), so a tile holds RT = 32 / SW restarts and the
// restart of every result register is known at compile time.  A wave takes 64
// points at a time (lane (c, h): points 2c and 2c + 1, "chunks" 0 and 1);
// after the two chunks' keys, lane half h finishes chunk h's point for every
// restart.  e: the common scale exponent (mfma_scale of every active
// restart).  Points [4 g_lo, min(4 g_hi, N)) in units of 64, strided over
// the team's waves.
template <int D, int SW>
__device__ void points_pass_mfma(const BInst& in, int rank, int S, int mask, double fscale,
                                 float ninf, int e, BSmem& sm, int64_t g_lo, int64_t g_hi) {
    constexpr int RT = 32 / SW;        // restarts per tile
    constexpr int NT = BK_RMAX / RT;   // tiles at most
    constexpr int QPR = SW / 8;        // quads of result registers per restart (4, 2, 1)
    constexpr float T = 16384.0f, P = 32768.0f;
    const int K = in.K, R = in.R;
    const int64_t N = in.N, ld = in.ld;
    const float* __restrict__ X = in.X;
    const bool vec = in.vec != 0;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int c = lane & 31, h = lane >> 5;
    float4* __restrict__ wq = sm.queue[w];
    int qn = 0;
    const int nacc = R * K * (D + 1);
    unsigned long long* const myacc = &sm.acc[(lane % acc_copies(nacc)) * nacc];
    const int ntiles = (R + RT - 1) / RT;

    // A operands: row c of tile t is centre c % SW of restart t RT + c / SW
    f16x8 A[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const int r = t * RT + c / SW, k = c % SW;
        const bool real = r < R && ((mask >> r) & 1) && k < K;
        A[t] = centre_operand<D>(real, real ? sm.scand[r][k] : make_float4(0.f, 0.f, 0.f, 0.f),
                                 e, h);
    }
    const uint32_t hm = h ? ~0u : 0u;
    const uint32_t q3 = h == 0 ? pack2((_Float16)T, (_Float16)T) : pack2((_Float16)T, (_Float16)P);
    const float sc = ldexpf(1.0f, e);
    const float bms = ldexpf(12.5f, 2 * e);  // matrix-key bound, as in the single fit

    auto drain = [&](int cnt) {
        __builtin_amdgcn_wave_barrier();
        if (lane < cnt) {
            const float4 q = wq[qn - cnt + lane];
            const int tag = __float_as_int(q.w);
            const int r = tag >> 27;
            float bd;
            int bk;
            direct_scan<D>(sm.smu[r], K, q.x, q.y, q.z, bd, bk);
            unsigned long long* a = &myacc[r * (D + 1) * K + bk];
            const float xs[3] = {q.x, q.y, q.z};
#pragma unroll
            for (int j = 0; j < D; ++j)
                __hip_atomic_fetch_add(&a[j * K], fxp_bits(xs[j], fscale), __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_WORKGROUP);
            __hip_atomic_fetch_add(&a[D * K], 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        }
        __builtin_amdgcn_wave_barrier();
        qn -= cnt;
    };

    const int64_t p_lo = 4 * g_lo;
    const int64_t p_hi = 4 * g_hi < N ? 4 * g_hi : N;
    // PU units of 64 points per wave and iteration: independent chains of
    // matrix products, re-keying and certificates for the scheduler to
    // interleave (few waves are resident beside this kernel's registers)
    constexpr int PU = 2;
    const int64_t nunits = (p_hi - p_lo + 63) / 64;
    const int64_t npairs = (nunits + PU - 1) / PU;
    const int wid = __builtin_amdgcn_readfirstlane(w);
    for (int64_t v = (int64_t)rank * NW + wid; v < npairs; v += (int64_t)S * NW) {
        float x0[PU], x1[PU], x2[PU];
        int64_t i[PU];
        uint64_t mv[PU];
        unsigned long long fb[PU][3];
        f16x8 B[PU][2];
#pragma unroll
        for (int pu = 0; pu < PU; ++pu) {
            const int64_t c0 = p_lo + (v * PU + pu) * 64;
            const int64_t left = p_hi - c0;
            const int rem = left <= 0 ? 0 : (left < 64 ? (int)left : 64);
            const int64_t i0 = c0 + 2 * c;  // this lane's first point of the unit
            float x[3][2];
            if (vec && rem == 64) {
#pragma unroll
                for (int j = 0; j < D; ++j) {
                    const float2 q = *reinterpret_cast<const float2*>(X + j * ld + i0);
                    x[j][0] = q.x; x[j][1] = q.y;
                }
            } else {
#pragma unroll
                for (int p = 0; p < 2; ++p) {
                    const bool inr = 2 * c + p < rem;
#pragma unroll
                    for (int j = 0; j < D; ++j) x[j][p] = inr ? X[j * ld + i0 + p] : 0.0f;
                }
            }
            if constexpr (D == 2) {
                x[2][0] = 0.0f;
                x[2][1] = 0.0f;
            }
#pragma unroll
            for (int q = 0; q < 2; ++q)
                B[pu][q] = point_operand(sel_half(hm, x[0][q], x[2][q]) * sc, x[1][q] * sc, q3);
            // this lane's point (chunk h), its fixed-point bits (one
            // conversion for every restart)
            x0[pu] = sel_half(hm, x[0][0], x[0][1]);
            x1[pu] = sel_half(hm, x[1][0], x[1][1]);
            x2[pu] = sel_half(hm, x[2][0], x[2][1]);
            i[pu] = i0 + h;
            mv[pu] = __builtin_amdgcn_ballot_w64(2 * c + h < rem);
            fb[pu][0] = fxp_bits(x0[pu], fscale);
            fb[pu][1] = fxp_bits(x1[pu], fscale);
            fb[pu][2] = D == 3 ? fxp_bits(x2[pu], fscale) : 0ull;
        }

#pragma unroll
        for (int t = 0; t < NT; ++t) {
            if (t >= ntiles) break;
            if (!((mask >> (t * RT)) & ((1 << RT) - 1))) continue;
            // per unit, restart of the tile and chunk: the smallest packed
            // quad minimum W and the second smallest L
            float W[PU][RT][2], L[PU][RT][2];
#pragma unroll
            for (int pu = 0; pu < PU; ++pu)
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const f32x16 zero16 = {};
                const f32x16 kk = __builtin_amdgcn_mfma_f32_32x32x16_f16(A[t], B[pu][q], zero16, 0, 0, 0);
                float pm[4];
                const uint32_t qmask = ~7u;
                pm[0] = quad_min<0, true>(kk[0], kk[1], kk[2], kk[3], qmask, ninf);
                pm[1] = quad_min<QPR == 1 ? 0 : 1, false>(kk[4], kk[5], kk[6], kk[7], qmask, ninf);
                pm[2] = quad_min<QPR == 4 ? 2 : 0, false>(kk[8], kk[9], kk[10], kk[11], qmask, ninf);
                pm[3] = quad_min<QPR == 4 ? 3 : (QPR == 2 ? 1 : 0), false>(kk[12], kk[13], kk[14],
                                                                           kk[15], qmask, ninf);
                if constexpr (QPR == 4) {
                    float a1, a2;
                    top2_3(pm[0], pm[1], pm[2], a1, a2);
                    W[pu][0][q] = vmin2(a1, pm[3]);
                    L[pu][0][q] = vmin2(a2, vmax2(a1, pm[3]));
                } else if constexpr (QPR == 2) {
                    W[pu][0][q] = vmin2(pm[0], pm[1]);
                    L[pu][0][q] = vmax2(pm[0], pm[1]);
                    W[pu][1][q] = vmin2(pm[2], pm[3]);
                    L[pu][1][q] = vmax2(pm[2], pm[3]);
                } else {
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        W[pu][j][q] = pm[j];
                        L[pu][j][q] = INFINITY;
                    }
                }
            }
#pragma unroll
            for (int j = 0; j < RT; ++j) {
                const int r = t * RT + j;
                if (r >= R || !((mask >> r) & 1)) continue;
                const float4* rec = sm.scand[r];
                const float4 bnd = sm.sbnd[r];
                // both units' winners and certificates first (independent
                // work), then their sums and queue entries
                int base[PU], kk4[PU];
                uint64_t mok[PU];
#pragma unroll
                for (int pu = 0; pu < PU; ++pu) {
                    // halves merged as in the single fit: after the swaps,
                    // w0 / l0 come from the h = 0 lane of the point, w1 / l1
                    // from h = 1
                    const auto ws = __builtin_amdgcn_permlane32_swap(
                        __float_as_uint(W[pu][j][0]), __float_as_uint(W[pu][j][1]), false, false);
                    const auto ls = __builtin_amdgcn_permlane32_swap(
                        __float_as_uint(L[pu][j][0]), __float_as_uint(L[pu][j][1]), false, false);
                    const float w0 = __uint_as_float(ws[0]), w1 = __uint_as_float(ws[1]);
                    const float l0 = __uint_as_float(ls[0]), l1 = __uint_as_float(ls[1]);
                    const float Wc = vmin2(w0, w1);
                    const float Lc = vmin3(vmax2(w0, w1), l0, l1);
                    const int hw = w1 < w0 ? 1 : 0;
                    // the winning quad: centres 8 g + 4 hw + 0..3 of restart r
                    const int g = QPR == 1 ? 0 : (int)(__float_as_uint(Wc) & 7u);
                    base[pu] = (g << 3) | (hw << 2);
                    const float s0 = expanded_key<D>(x0[pu], x1[pu], x2[pu], rec[base[pu]]);
                    const float s1 = expanded_key<D>(x0[pu], x1[pu], x2[pu], rec[base[pu] + 1]);
                    const float s2 = expanded_key<D>(x0[pu], x1[pu], x2[pu], rec[base[pu] + 2]);
                    const float s3 = expanded_key<D>(x0[pu], x1[pu], x2[pu], rec[base[pu] + 3]);
                    const float a3 = fminf(fminf(s0, s1), s2);
                    const float t1 = fminf(a3, s3);
                    const float t2 = fminf(__builtin_amdgcn_fmed3f(s0, s1, s2), fmaxf(a3, s3));
                    int kq = 3;
                    kq = s2 == t1 ? 2 : kq;
                    kq = s1 == t1 ? 1 : kq;
                    kq = s0 == t1 ? 0 : kq;
                    kk4[pu] = kq;
                    float b = fmaf(bnd.y, fabsf(x0[pu]), bnd.x);
                    b = fmaf(bnd.z, fabsf(x1[pu]), b);
                    if constexpr (D == 3) b = fmaf(bnd.w, fabsf(x2[pu]), b);
                    const float bm = fmaf(b, bms, 17.0f);
                    // the certificate as lane masks (no k < K test: pads key
                    // above every real centre, in the matrix keys and in the
                    // records)
                    mok[pu] = __builtin_amdgcn_ballot_w64(Lc - Wc > bm) &
                              __builtin_amdgcn_ballot_w64(t2 - t1 > b);
                }
#pragma unroll
                for (int pu = 0; pu < PU; ++pu) {
                    if (__builtin_amdgcn_inverse_ballot_w64(mv[pu] & mok[pu])) {
                        unsigned long long* a = &myacc[r * (D + 1) * K + base[pu] + kk4[pu]];
#pragma unroll
                        for (int jj = 0; jj < D; ++jj)
                            __hip_atomic_fetch_add(&a[jj * K], fb[pu][jj], __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_WORKGROUP);
                        __hip_atomic_fetch_add(&a[D * K], 1ull, __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_WORKGROUP);
                    }
                    const uint64_t m = mv[pu] & ~mok[pu];
                    if (m) {
                        const int below_m = (int)__builtin_amdgcn_mbcnt_hi(
                            (uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
                        if (__builtin_amdgcn_inverse_ballot_w64(m))
                            wq[qn + below_m] = make_float4(x0[pu], x1[pu], x2[pu],
                                                           __int_as_float((r << 27) | (int)i[pu]));
                        qn += __popcll(m);
                        if (qn >= 64) drain(64);
                    }
                }
            }
        }
    }
    if (qn > 0) drain(qn);
}

// The common scale exponent of the matrix-core keys for the active restarts
// (mfma_scale of each), or false when one falls outside its range.
__device__ __forceinline__ bool batched_mfma_scale(const BSmem& sm, int mask, int R, int xe,
                                                   int& e) {
    e = 1 << 20;
    for (int r = 0; r < R; ++r) {
        if (!((mask >> r) & 1)) continue;
        int er;
        if (!mfma_scale(xe, sm.sbnd[r], er)) return false;
        e = er < e ? er : e;
    }
    return true;
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
__device__ __attribute__((always_inline)) bool run_instance(BatchState* __restrict__ bs, int inst, int rank, int S, BTeam* tm,
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
    for (int r = 0; r < R; ++r) prep_centres(sm.smu[r], K, BK_KPAD, sm.scand[r], &sm.sbnd[r], sm.sc, sm.sa, am);

    double jl = 0.0;
    // ---- Lloyd updates of all active restarts
    for (;;) {
        const int active = __builtin_amdgcn_readfirstlane(sm.active);
        if (!active) break;
        const int copies = acc_copies(nacc);
        // the matrix-core keys for this update (labels are the same either way)
        int e_mfma = 0;
        const bool use_mfma = D == 3 && K >= bs->mfma_min_k &&
                              batched_mfma_scale(sm, active, R, xe, e_mfma);
        for (int64_t g0 = 0; g0 < ngroups; g0 += chunk) {
            const int64_t g1 = g0 + chunk < ngroups ? g0 + chunk : ngroups;
            for (int i = tid; i < copies * nacc; i += BLOCK) sm.acc[i] = 0ull;
            __syncthreads();
            if (!use_mfma)
                points_pass<D, MODE_ACC>(in, rank, S, active, fscale, ninf, sm, jl, g0, g1);
            else if (K <= 8)
                points_pass_mfma<D, 8>(in, rank, S, active, fscale, ninf, e_mfma, sm, g0, g1);
            else if (K <= 16)
                points_pass_mfma<D, 16>(in, rank, S, active, fscale, ninf, e_mfma, sm, g0, g1);
            else
                points_pass_mfma<D, 32>(in, rank, S, active, fscale, ninf, e_mfma, sm, g0, g1);
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
                prep_centres(sm.smu[r], K, BK_KPAD, sm.scand[r], &sm.sbnd[r], sm.sc, sm.sa, am);
        __syncthreads();
    }
    if (!bad) {
        // ---- objective of every restart at its final centres
        for (int r = 0; r < R; ++r) prep_centres(sm.smu[r], K, BK_KPAD, sm.scand[r], &sm.sbnd[r], sm.sc, sm.sa, am);
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
