// lloyd_kernels.hip -- gfx950 kernels of one Lloyd iteration.
//
// Paper: "The Lloyd's Algorithm" (reassignment argmin, mean calculation with
// the indicator function) and "Serial Lloyd's Algorithm" (error E between
// successive centres, tolerance test).
//
// Kernels
//   km_scan      one pass over X: max |x| (sets the fixed-point exponent G and
//                flags NaN/Inf); prepares the centre tables.
//   lloyd_iter   one whole update: reassignment of every point, per-cluster
//                integer sums and counts in LDS, one partial per block, a
//                two-level reduction of the partials by the last block of each
//                group and then the last group, and in that final block the
//                float64 divide, the empty-cluster rule, E and the tolerance
//                test.  No host synchronisation between iterations.
//   lloyd_label  reassignment only: labels and the objective for the current
//                centres (final labels of a fit; the assign entry point).
//
// Reassignment (nearest): the scan over centres uses the expanded form
//   s_k = |m_k|^2 - 2 m_k . x      (= |x - m_k|^2 - |x|^2, same argmin)
// three fused multiply-adds per centre, and keeps the smallest and second
// smallest s over triples of centres (min3 / med3) plus the triple of the
// smallest.  A rounding bound b(x) on every s_k certifies the winner: when
// the two smallest differ by more than b(x), the first index attaining the
// smallest s is the exact argmin of the squared distance to the float32
// centres.  Otherwise (points within b(x) of a tie) the point is re-scanned
// with the direct form (x0-m0)^2 + (x1-m1)^2 [+ (x2-m2)^2] in float32, first
// index of the minimum.  The distance reported (objective) is always the
// direct form to the chosen centre.
//
// Determinism: the per-cluster sums are exact integer sums of x * 2^G
// (|x| * 2^G < 2^30, rounded to nearest), so their value does not depend on
// the order in which points, waves or blocks add them: results are identical
// for any grid size and from run to run, without float atomics.  The
// objective (reported, not fed back) is summed per lane, reduced across the
// wave with a fixed butterfly and across waves, blocks and groups in index
// order.
#include "km_internal.h"

#include <math.h>

namespace km {
namespace {

constexpr int NW = BLOCK / 64;  // waves per block

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ uint32_t wave_max(uint32_t v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        uint32_t u = __shfl_xor(v, o, 64);
        v = u > v ? u : v;
    }
    return v;
}

template <typename T>
__device__ __forceinline__ T ld_agent(const T* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Fixed-point exponent: every |x| * 2^G < 2^30 for |x| <= max|x|.
__device__ __forceinline__ int scale_exponent(uint32_t absmax_bits) {
    float a = __uint_as_float(absmax_bits);
    if (!(a > 0.0f)) return 30;
    int G = 29 - ilogbf(a);  // a < 2^(ilogb(a)+1)
    return G > 120 ? 120 : G;
}

// Load the 4 consecutive points of group g (coordinates x[j][p]); returns how
// many of them exist (4 except in the last, ragged group).
template <int D, bool VEC>
__device__ __forceinline__ int load_group(const float* __restrict__ X, int64_t ld,
                                          int64_t N, int64_t g, float (&x)[D][4]) {
    const int64_t i0 = g * 4;
    if (VEC && i0 + 4 <= N) {
#pragma unroll
        for (int j = 0; j < D; ++j) {
            const float4 v = *reinterpret_cast<const float4*>(X + j * ld + i0);
            x[j][0] = v.x; x[j][1] = v.y; x[j][2] = v.z; x[j][3] = v.w;
        }
        return 4;
    }
    const int n = (int)((N - i0) < 4 ? (N - i0) : 4);
#pragma unroll
    for (int j = 0; j < D; ++j)
#pragma unroll
        for (int p = 0; p < 4; ++p) x[j][p] = p < n ? X[j * ld + i0 + p] : 0.0f;
    return n;
}

// Squared distance in the direct form, float32, left to right with FMAs.
template <int D>
__device__ __forceinline__ float direct_dist(float x0, float x1, float x2, float4 c) {
    const float d0 = x0 - c.x;
    const float d1 = x1 - c.y;
    float s = d0 * d0;
    s = fmaf(d1, d1, s);
    if constexpr (D == 3) {
        const float d2 = x2 - c.z;
        s = fmaf(d2, d2, s);
    }
    return s;
}

// min(a, b) as the median of (a, b, -inf), with -inf read from memory so that
// it stays one med3 instruction: fminf would first quiet its loop-carried
// operands (two extra instructions).
__device__ __forceinline__ float min2(float a, float b, float ninf) {
    return __builtin_amdgcn_fmed3f(a, b, ninf);
}

// Expanded-form key of one centre record {a0, a1, a2, c}.
template <int D>
__device__ __forceinline__ float expanded_key(float x0, float x1, float x2, float4 r) {
    float s = fmaf(x0, r.x, r.w);
    s = fmaf(x1, r.y, s);
    if constexpr (D == 3) s = fmaf(x2, r.z, s);
    return s;
}

// Reassignment scan of the 4 points x[.][p] (see the file header).  scand:
// the K centre records padded to ntri triples; smu: the float32 centres;
// bnd: the rounding-bound coefficients.  For every point writes ok[p]: the
// winner is certified, and then arg[p] (its index) and best[p] (the
// direct-form squared distance to it).  Points with ok[p] == false need the
// direct-form scan (direct_scan).
template <int D>
__device__ __forceinline__ void nearest4(const float4* __restrict__ scand,
                                         const float4* __restrict__ smu, int K, int ntri,
                                         float4 bnd, float ninf, const float (&x)[D][4],
                                         float (&best)[4], int (&arg)[4], bool (&ok)[4]) {
    float m1[4], m2[4];
    int tri[4];
#pragma unroll
    for (int p = 0; p < 4; ++p) { m1[p] = INFINITY; m2[p] = INFINITY; tri[p] = 0; }
    for (int g = 0; g < ntri; ++g) {
        const float4 r0 = scand[3 * g], r1 = scand[3 * g + 1], r2 = scand[3 * g + 2];
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            const float x2 = D == 3 ? x[D - 1][p] : 0.0f;
            const float s0 = expanded_key<D>(x[0][p], x[1][p], x2, r0);
            const float s1 = expanded_key<D>(x[0][p], x[1][p], x2, r1);
            const float s2 = expanded_key<D>(x[0][p], x[1][p], x2, r2);
            const float g1 = fminf(fminf(s0, s1), s2);
            const float g2 = __builtin_amdgcn_fmed3f(s0, s1, s2);
            m2[p] = __builtin_amdgcn_fmed3f(m1[p], g1, min2(m2[p], g2, ninf));
            tri[p] = g1 < m1[p] ? g : tri[p];
            m1[p] = min2(m1[p], g1, ninf);
        }
    }
#pragma unroll
    for (int p = 0; p < 4; ++p) {
        const float x0 = x[0][p], x1 = x[1][p], x2 = D == 3 ? x[D - 1][p] : 0.0f;
        // first index of the smallest key inside the winning triple
        const int k0 = 3 * tri[p];
        const float s0 = expanded_key<D>(x0, x1, x2, scand[k0]);
        const float s1 = expanded_key<D>(x0, x1, x2, scand[k0 + 1]);
        const int k = s0 == m1[p] ? k0 : (s1 == m1[p] ? k0 + 1 : k0 + 2);
        // rounding bound of the keys of this point
        float b = fmaf(bnd.y, fabsf(x0), bnd.x);
        b = fmaf(bnd.z, fabsf(x1), b);
        if constexpr (D == 3) b = fmaf(bnd.w, fabsf(x2), b);
        ok[p] = m2[p] - m1[p] > b && k < K;
        arg[p] = ok[p] ? k : 0;
        best[p] = direct_dist<D>(x0, x1, x2, smu[arg[p]]);
    }
}

// Direct-form scan of one point over all K centres: first index of the
// minimum of the float32 squared distance (the near-tie path).
template <int D>
__device__ __forceinline__ void direct_scan(const float4* __restrict__ smu, int K, float x0,
                                            float x1, float x2, float& bd, int& bk) {
    bd = INFINITY;
    bk = 0;
    for (int q = 0; q < K; ++q) {
        const float dq = direct_dist<D>(x0, x1, x2, smu[q]);
        if (dq < bd) { bd = dq; bk = q; }
    }
}

// Reassignment of every point of the grid-stride share of this thread.
// sink(i, x0, x1, x2, k, dist) receives each point with its label and
// distance.  Points that are not certified go to this wave's LDS queue wq
// (QCAP entries {x0, x1, x2, index}) and are re-scanned 64 at a time, one per
// lane, so a rare near-tie costs one lane of a full wave instead of a whole
// wave of idle lanes.
constexpr int QCAP = 128;

template <int D, bool VEC, typename Sink>
__device__ __forceinline__ void assign_points(const float* __restrict__ X, int64_t ld,
                                              int64_t N, const float4* __restrict__ scand,
                                              const float4* __restrict__ smu, int K,
                                              int ntri, float4 bnd, float ninf,
                                              float4* __restrict__ wq, Sink&& sink) {
    const int lane = threadIdx.x & 63;
    const uint64_t below = (1ull << lane) - 1ull;
    int qn = 0;  // entries in this wave's queue; the same in every lane
    auto drain = [&](int cnt) {
        __builtin_amdgcn_wave_barrier();
        if (lane < cnt) {
            const float4 e = wq[qn - cnt + lane];
            float bd;
            int bk;
            direct_scan<D>(smu, K, e.x, e.y, e.z, bd, bk);
            sink((int64_t)__float_as_int(e.w), e.x, e.y, e.z, bk, bd);
        }
        __builtin_amdgcn_wave_barrier();
        qn -= cnt;
    };
    const int64_t ngroups = (N + 3) / 4;
    // The loop bound is uniform across the wave (ballots and the queue count
    // must see every lane); lanes past the end carry no points.
    for (int64_t gw = (int64_t)blockIdx.x * BLOCK + (threadIdx.x & ~63); gw < ngroups;
         gw += (int64_t)gridDim.x * BLOCK) {
        const int64_t g = gw + lane;
        float x[D][4];
        int n = 0;
        if (g < ngroups) {
            n = load_group<D, VEC>(X, ld, N, g, x);
        } else {
#pragma unroll
            for (int j = 0; j < D; ++j)
#pragma unroll
                for (int p = 0; p < 4; ++p) x[j][p] = 0.0f;
        }
        float best[4];
        int arg[4];
        bool ok[4];
        nearest4<D>(scand, smu, K, ntri, bnd, ninf, x, best, arg, ok);
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            const float x2 = D == 3 ? x[D - 1][p] : 0.0f;
            const bool valid = p < n;
            if (valid && ok[p]) sink(g * 4 + p, x[0][p], x[1][p], x2, arg[p], best[p]);
            const bool f = valid && !ok[p];
            const uint64_t m = __ballot(f);
            if (m) {
                if (f)
                    wq[qn + __popcll(m & below)] =
                        make_float4(x[0][p], x[1][p], x2, __int_as_float((int)(g * 4 + p)));
                qn += __popcll(m);
                if (qn >= 64) drain(64);
            }
        }
    }
    if (qn > 0) drain(qn);
}

// Centre tables for the reassignment: records {-2 m, fl32(|m|^2)} padded to
// whole triples with {0, 0, 0, +inf}, and the bound coefficients
//   b(x) = 2^-20 (Cmax + 2 sum_j A_j |x_j|),  Cmax = max_k c_k, A_j = max_k |m_kj|,
// which exceeds twice the rounding error of any key (<= 4.01 u (Cmax + 2 sum_j
// A_j |x_j|), u = 2^-24: the rounding of c_k and of three FMAs).  Called by
// one whole block with the final float32 centres in m[0..K).
__device__ void prep_centres(State* __restrict__ st, const float4* m32, int K, float* sc,
                             float* sa) {
    const int tid = threadIdx.x;
    const int ntri = (K + 2) / 3;
    if (tid < 3 * ntri) {
        float4 r = make_float4(0.f, 0.f, 0.f, INFINITY);
        float c = 0.f, a0 = 0.f, a1 = 0.f, a2 = 0.f;
        if (tid < K) {
            const float4 m = m32[tid];
            const double q = __dadd_rn(__dadd_rn(__dmul_rn((double)m.x, (double)m.x),
                                                 __dmul_rn((double)m.y, (double)m.y)),
                                       __dmul_rn((double)m.z, (double)m.z));
            c = (float)q;
            r = make_float4(-2.0f * m.x, -2.0f * m.y, -2.0f * m.z, c);
            a0 = fabsf(m.x); a1 = fabsf(m.y); a2 = fabsf(m.z);
        }
        st->cand[tid] = r;
        sc[tid] = c;
        sa[3 * tid] = a0; sa[3 * tid + 1] = a1; sa[3 * tid + 2] = a2;
    }
    __syncthreads();
    if (tid == 0) {
        float cm = 0.f, am0 = 0.f, am1 = 0.f, am2 = 0.f;
        for (int k = 0; k < K; ++k) {
            cm = fmaxf(cm, sc[k]);
            am0 = fmaxf(am0, sa[3 * k]); am1 = fmaxf(am1, sa[3 * k + 1]); am2 = fmaxf(am2, sa[3 * k + 2]);
        }
        st->bnd = make_float4(ldexpf(cm, -20), ldexpf(am0, -19), ldexpf(am1, -19), ldexpf(am2, -19));
    }
}

// Stage the centre tables of the current iteration in LDS.
__device__ __forceinline__ int stage_centres(const State* __restrict__ st, int K, float4* scand,
                                             float4* smu) {
    const int ntri = (K + 2) / 3;
    for (int i = threadIdx.x; i < 3 * ntri; i += BLOCK) scand[i] = st->cand[i];
    for (int i = threadIdx.x; i < K; i += BLOCK) smu[i] = st->mu32[i];
    return ntri;
}

// Publish this block's objective partial and take a ticket; true in the last
// block of the grid to arrive (single-level; used by the label kernel).
__device__ bool finish_block(uint32_t* ticket, double* jslot, double jblock, int* sflag) {
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        *jslot = jblock;
        __threadfence();
        const uint32_t old = __hip_atomic_fetch_add(ticket, 1u, __ATOMIC_ACQ_REL,
                                                    __HIP_MEMORY_SCOPE_AGENT);
        *sflag = (old == gridDim.x - 1);
    }
    __syncthreads();
    const bool last = *sflag != 0;
    if (last) __threadfence();
    return last;
}

// Sum of the per-block objective partials in block order; whole block.
__device__ double sum_partials(const double* __restrict__ jpart, int nb, double* sred) {
    const int tid = threadIdx.x;
    double s = 0.0;
    for (int b = tid; b < nb; b += BLOCK) s += jpart[b];
    s = wave_sum(s);
    __syncthreads();
    if ((tid & 63) == 0) sred[tid >> 6] = s;
    __syncthreads();
    double tot = 0.0;
#pragma unroll
    for (int w = 0; w < NW; ++w) tot += sred[w];
    return tot;
}

// Two-level reduction of the block partials (integer sums | counts, and the
// objective).  Every block publishes its partial; the last block of each
// group of GROUP blocks adds the group's partials; the last group adds the
// group sums.  Returns true in that one final block, with the grid totals in
// tot[0..nr) (LDS) and the objective in *jtot.  No two blocks add to the same
// address, so there is no contention; the integer sums are exact in any order
// and the objective is added in block, then group, order.
__device__ bool reduce_grid(State* __restrict__ st, const unsigned long long* blk, int nr,
                            double jb, unsigned long long* tot, double* jtot, int* sflag) {
    const int tid = threadIdx.x;
    const int b = blockIdx.x, nb = gridDim.x;
    unsigned long long* mine = st->part + (size_t)b * PART;
    for (int i = tid; i < nr; i += BLOCK) mine[i] = blk[i];
    if (tid == 0) st->jpart[b] = jb;
    __threadfence();
    __syncthreads();
    const int grp = b / GROUP, g0 = grp * GROUP;
    const int gn = (nb - g0) < GROUP ? (nb - g0) : GROUP;
    if (tid == 0) {
        const uint32_t old = __hip_atomic_fetch_add(&st->gticket[grp], 1u, __ATOMIC_ACQ_REL,
                                                    __HIP_MEMORY_SCOPE_AGENT);
        *sflag = (old == (uint32_t)gn - 1);
    }
    __syncthreads();
    if (!*sflag) return false;
    __threadfence();
    // last block of its group
    for (int i = tid; i < nr; i += BLOCK) {
        unsigned long long s = 0ull;
        for (int q = 0; q < gn; ++q) s += st->part[(size_t)(g0 + q) * PART + i];
        st->gpart[(size_t)grp * PART + i] = s;
    }
    if (tid == 0) {
        double j = 0.0;
        for (int q = 0; q < gn; ++q) j += st->jpart[g0 + q];
        st->gjpart[grp] = j;
        st->gticket[grp] = 0u;
    }
    __threadfence();
    __syncthreads();
    const int ng = (nb + GROUP - 1) / GROUP;
    if (tid == 0) {
        const uint32_t old = __hip_atomic_fetch_add(&st->ticket, 1u, __ATOMIC_ACQ_REL,
                                                    __HIP_MEMORY_SCOPE_AGENT);
        *sflag = (old == (uint32_t)ng - 1);
    }
    __syncthreads();
    if (!*sflag) return false;
    __threadfence();
    // the final block
    for (int i = tid; i < nr; i += BLOCK) {
        unsigned long long s = 0ull;
        for (int q = 0; q < ng; ++q) s += st->gpart[(size_t)q * PART + i];
        tot[i] = s;
    }
    if (tid == 0) {
        double j = 0.0;
        for (int q = 0; q < ng; ++q) j += st->gjpart[q];
        *jtot = j;
        st->ticket = 0u;
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
        __threadfence();
        const uint32_t old = __hip_atomic_fetch_add(&st->scan_ticket, 1u, __ATOMIC_ACQ_REL,
                                                    __HIP_MEMORY_SCOPE_AGENT);
        slast = (old == gridDim.x - 1);
    }
    __syncthreads();
    if (!slast) return;
    __threadfence();
    prep_centres(st, st->mu32, st->K, sc, sa);
    for (int i = tid; i < MAX_GROUPS; i += BLOCK) st->gticket[i] = 0u;
    if (tid == 0) {
        const uint32_t a = ld_agent(&st->absmax_bits);
        st->G = scale_exponent(a);
        if (a >= 0x7f800000u) {  // NaN or infinity in X
            st->flags |= FLAG_NONFINITE;
            st->done = 1;
        }
        st->scan_ticket = 0;
        st->ticket = 0;
    }
}

// ---------------------------------------------------------------- lloyd_iter
template <int D, bool VEC>
__global__ __launch_bounds__(BLOCK) void lloyd_iter(State* __restrict__ st) {
    if (st->done) return;
    constexpr int R = D + 1;  // per cluster: D sums, 1 count
    __shared__ float4 scand[KPAD];
    __shared__ float4 smu[KMAX];
    __shared__ unsigned long long sacc[NW][KMAX * R];
    __shared__ unsigned long long stot[KMAX * R];
    __shared__ float4 squeue[NW][QCAP];
    __shared__ double sred[NW];
    __shared__ double sE[KMAX];
    __shared__ int sEmpty[KMAX];
    __shared__ float sc[KPAD];
    __shared__ float sa[3 * KPAD];
    __shared__ double sJ;
    __shared__ int sflag;

    const int tid = threadIdx.x, w = tid >> 6;
    const int K = st->K;
    const int G = st->G;
    const int64_t N = st->N, ld = st->ld;
    const float* __restrict__ X = st->X;
    const float4 bnd = st->bnd;
    const float ninf = st->minus_inf;

    const int ntri = stage_centres(st, K, scand, smu);
    for (int i = tid; i < NW * KMAX * R; i += BLOCK) (&sacc[0][0])[i] = 0ull;
    __syncthreads();

    double jl = 0.0;
    unsigned long long* myacc = sacc[w];
    assign_points<D, VEC>(X, ld, N, scand, smu, K, ntri, bnd, ninf, squeue[w],
                          [&](int64_t, float x0, float x1, float x2, int k, float dist) {
        unsigned long long* a = &myacc[k * R];
        const float xs[3] = {x0, x1, x2};
#pragma unroll
        for (int j = 0; j < D; ++j) {
            const long long q = (long long)__float2int_rn(ldexpf(xs[j], G));
            __hip_atomic_fetch_add(&a[j], (unsigned long long)q, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_WORKGROUP);
        }
        __hip_atomic_fetch_add(&a[D], 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        jl += (double)dist;
    });
    jl = wave_sum(jl);
    if ((tid & 63) == 0) sred[w] = jl;
    __syncthreads();
    for (int i = tid; i < K * R; i += BLOCK) {
        unsigned long long s = 0ull;
#pragma unroll
        for (int v = 0; v < NW; ++v) s += sacc[v][i];
        stot[i] = s;
    }
    double jb = 0.0;
#pragma unroll
    for (int v = 0; v < NW; ++v) jb += sred[v];
    __syncthreads();
    if (!reduce_grid(st, stot, K * R, jb, &sacc[0][0], &sJ, &sflag)) return;

    // ---- final block: the update of the paper's mean-calculation step ----
    const unsigned long long* tot = &sacc[0][0];
    if (tid < K) {
        const int k = tid;
        const unsigned long long cnt = tot[k * R + D];
        double e = 0.0;
        float m32[DMAX] = {0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int j = 0; j < D; ++j) {
            const long long s = (long long)tot[k * R + j];
            const double old = st->mu64[k * D + j];
            const double v = cnt ? ldexp((double)s, -G) / (double)cnt : old;
            const double sh = v - old;
            e = fma(sh, sh, e);
            st->mu64[k * D + j] = v;
            m32[j] = (float)v;
        }
        const float4 m = make_float4(m32[0], m32[1], m32[2], 0.0f);
        st->mu32[k] = m;
        smu[k] = m;
        sE[k] = e;
        sEmpty[k] = cnt == 0ull;
    }
    __syncthreads();
    prep_centres(st, smu, K, sc, sa);
    if (tid == 0) {
        double E = 0.0;
        int emp = 0;
        for (int k = 0; k < K; ++k) { E += sE[k]; emp += sEmpty[k]; }
        const int t = st->t;
        if (t < st->hist_cap) { st->E_hist[t] = E; st->J_hist[t] = sJ; }
        st->t = t + 1;
        st->E = E;
        st->empty_events += emp;
        st->done = (E < st->tol || t + 1 >= st->max_iter) ? 1 : 0;
    }
}

// ---------------------------------------------------------------- lloyd_label
template <int D, bool VEC>
__global__ __launch_bounds__(BLOCK) void lloyd_label(State* __restrict__ st,
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
    const int ntri = stage_centres(st, K, scand, smu);
    __syncthreads();
    double jl = 0.0;
    assign_points<D, VEC>(X, ld, N, scand, smu, K, ntri, bnd, ninf, squeue[w],
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

hipError_t launch_scan(State* st, int d, bool vec, int grid, hipStream_t s) {
    if (grid < 1 || grid > MAX_BLOCKS) return hipErrorInvalidValue;
    KM_DISPATCH(km_scan, grid, s, st);
    return hipGetLastError();
}

hipError_t launch_iter(State* st, int d, bool vec, int grid, hipStream_t s) {
    if (grid < 1 || grid > MAX_BLOCKS) return hipErrorInvalidValue;
    KM_DISPATCH(lloyd_iter, grid, s, st);
    return hipGetLastError();
}

hipError_t launch_label(State* st, int32_t* labels, int d, bool vec, int grid,
                        hipStream_t s) {
    if (grid < 1 || grid > MAX_BLOCKS) return hipErrorInvalidValue;
    KM_DISPATCH(lloyd_label, grid, s, st, labels);
    return hipGetLastError();
}

}  // namespace km
