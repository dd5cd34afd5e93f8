// lloyd_kernels.hip -- gfx950 kernels of one Lloyd iteration.
//
// Paper: "The Lloyd's Algorithm" (reassignment argmin, mean calculation with
// the indicator function) and "Serial Lloyd's Algorithm" (error E between
// successive centres, tolerance test).
//
// Kernels
//   km_scan      one pass over X: max |x| (sets the fixed-point exponent G and
//                flags NaN/Inf), clears the per-cluster accumulators.
//   lloyd_iter   one whole update: reassignment of every point (float32
//                distances, first index of the minimum), per-cluster integer
//                sums and counts in LDS, block totals added to global integer
//                accumulators, and -- in the last block to finish -- the
//                float64 divide, the empty-cluster rule, E and the tolerance
//                test.  No host synchronisation between iterations.
//   lloyd_label  reassignment only: labels and the objective for the current
//                centres (final labels of a fit; the assign entry point).
//
// Determinism: the per-cluster sums are exact integer sums of x * 2^G
// (|x| * 2^G < 2^30, rounded to nearest), so their value does not depend on
// the order in which points, waves or blocks add them: results are identical
// for any grid size and from run to run without float atomics.  The objective
// (reported, not fed back) is summed per lane, reduced across the wave with a
// fixed butterfly and across waves and blocks in index order.
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

// Reassignment of 4 points against the K centres held in LDS: squared
// distance in float32, (x0-m0)^2 + (x1-m1)^2 [+ (x2-m2)^2] accumulated left to
// right with fused multiply-adds; strict '<' keeps the lowest index on ties.
template <int D>
__device__ __forceinline__ void nearest4(const float4* __restrict__ smu, int K,
                                         const float (&x)[D][4], float (&best)[4],
                                         int (&arg)[4]) {
#pragma unroll
    for (int p = 0; p < 4; ++p) { best[p] = INFINITY; arg[p] = 0; }
#pragma unroll 2
    for (int k = 0; k < K; ++k) {
        const float4 c = smu[k];
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            const float d0 = x[0][p] - c.x;
            const float d1 = x[1][p] - c.y;
            float s = d0 * d0;
            s = fmaf(d1, d1, s);
            if constexpr (D == 3) {
                const float d2 = x[2][p] - c.z;
                s = fmaf(d2, d2, s);
            }
            if (s < best[p]) { best[p] = s; arg[p] = k; }
        }
    }
}

// Sum of the per-block objective partials in block order (fixed strided
// partition, fixed butterfly, waves in order); called by one whole block.
__device__ double sum_partials(const double* __restrict__ jpart, int nb, double* sred) {
    const int tid = threadIdx.x;
    double s = 0.0;
    for (int b = tid; b < nb; b += BLOCK)
        s += __hip_atomic_load(&jpart[b], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    s = wave_sum(s);
    __syncthreads();
    if ((tid & 63) == 0) sred[tid >> 6] = s;
    __syncthreads();
    double tot = 0.0;
#pragma unroll
    for (int w = 0; w < NW; ++w) tot += sred[w];
    return tot;
}

// Publish this block's objective partial and take a ticket; true in the last
// block of the grid to arrive.
__device__ bool finish_block(uint32_t* ticket, double* jslot, double jblock, int* slast) {
    __threadfence();  // this thread's global atomics are performed at agent scope
    __syncthreads();
    if (threadIdx.x == 0) {
        __hip_atomic_store(jslot, jblock, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __threadfence();
        const uint32_t old = __hip_atomic_fetch_add(ticket, 1u, __ATOMIC_ACQ_REL,
                                                    __HIP_MEMORY_SCOPE_AGENT);
        *slast = (old == gridDim.x - 1);
    }
    __syncthreads();
    const bool last = *slast != 0;
    if (last) __threadfence();
    return last;
}

// ---------------------------------------------------------------- km_scan
template <int D, bool VEC>
__global__ __launch_bounds__(BLOCK) void km_scan(State* __restrict__ st) {
    __shared__ uint32_t sm[NW];
    __shared__ int slast;
    const int tid = threadIdx.x;
    if (blockIdx.x == 0)
        for (int i = tid; i < KMAX * (DMAX + 1); i += BLOCK) st->acc[i] = 0ull;
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
    if (slast && tid == 0) {
        __threadfence();
        const uint32_t a = __hip_atomic_load(&st->absmax_bits, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT);
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
    __shared__ float4 smu[KMAX];
    __shared__ unsigned long long sacc[NW][KMAX * R];
    __shared__ double sred[NW];
    __shared__ double sE[KMAX];
    __shared__ int sEmpty[KMAX];
    __shared__ int slast;

    const int tid = threadIdx.x, w = tid >> 6;
    const int K = st->K;
    const int G = st->G;
    const int64_t N = st->N, ld = st->ld;
    const float* __restrict__ X = st->X;

    for (int i = tid; i < K; i += BLOCK) smu[i] = st->mu32[i];
    for (int i = tid; i < NW * KMAX * R; i += BLOCK) (&sacc[0][0])[i] = 0ull;
    __syncthreads();

    double jl = 0.0;
    const int64_t ngroups = (N + 3) / 4;
    for (int64_t g = (int64_t)blockIdx.x * BLOCK + tid; g < ngroups;
         g += (int64_t)gridDim.x * BLOCK) {
        float x[D][4];
        const int n = load_group<D, VEC>(X, ld, N, g, x);
        float best[4];
        int arg[4];
        nearest4<D>(smu, K, x, best, arg);
        float js = 0.0f;
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            if (p < n) {
                unsigned long long* a = &sacc[w][arg[p] * R];
#pragma unroll
                for (int j = 0; j < D; ++j) {
                    const long long q = (long long)__float2int_rn(ldexpf(x[j][p], G));
                    __hip_atomic_fetch_add(&a[j], (unsigned long long)q, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_WORKGROUP);
                }
                __hip_atomic_fetch_add(&a[D], 1ull, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_WORKGROUP);
                js += best[p];
            }
        }
        jl += (double)js;
    }
    __syncthreads();

    // block totals -> global integer accumulators
    for (int i = tid; i < K * R; i += BLOCK) {
        unsigned long long s = 0ull;
#pragma unroll
        for (int v = 0; v < NW; ++v) s += sacc[v][i];
        if (s) __hip_atomic_fetch_add(&st->acc[i], s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    jl = wave_sum(jl);
    if ((tid & 63) == 0) sred[w] = jl;
    __syncthreads();
    double jb = 0.0;
#pragma unroll
    for (int v = 0; v < NW; ++v) jb += sred[v];
    if (!finish_block(&st->ticket, &st->jpart[blockIdx.x], jb, &slast)) return;

    // ---- last block: the update of the paper's mean-calculation step ----
    const double J = sum_partials(st->jpart, gridDim.x, sred);
    if (tid < K) {
        const int k = tid;
        const unsigned long long cnt = __hip_atomic_exchange(
            &st->acc[k * R + D], 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        double e = 0.0;
        float m32[DMAX] = {0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int j = 0; j < D; ++j) {
            const long long s = (long long)__hip_atomic_exchange(
                &st->acc[k * R + j], 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const double old = st->mu64[k * D + j];
            const double v = cnt ? ldexp((double)s, -G) / (double)cnt : old;
            const double sh = v - old;
            e = fma(sh, sh, e);
            st->mu64[k * D + j] = v;
            m32[j] = (float)v;
        }
        st->mu32[k] = make_float4(m32[0], m32[1], m32[2], 0.0f);
        sE[k] = e;
        sEmpty[k] = cnt == 0ull;
    }
    __syncthreads();
    if (tid == 0) {
        double E = 0.0;
        int emp = 0;
        for (int k = 0; k < K; ++k) { E += sE[k]; emp += sEmpty[k]; }
        const int t = st->t;
        if (t < st->hist_cap) { st->E_hist[t] = E; st->J_hist[t] = J; }
        st->t = t + 1;
        st->E = E;
        st->empty_events += emp;
        st->done = (E < st->tol || t + 1 >= st->max_iter) ? 1 : 0;
        st->ticket = 0;
    }
}

// ---------------------------------------------------------------- lloyd_label
template <int D, bool VEC>
__global__ __launch_bounds__(BLOCK) void lloyd_label(State* __restrict__ st,
                                                     int32_t* __restrict__ labels) {
    if (st->flags & FLAG_NONFINITE) return;
    __shared__ float4 smu[KMAX];
    __shared__ double sred[NW];
    __shared__ int slast;
    const int tid = threadIdx.x, w = tid >> 6;
    const int K = st->K;
    const int64_t N = st->N, ld = st->ld;
    const float* __restrict__ X = st->X;
    for (int i = tid; i < K; i += BLOCK) smu[i] = st->mu32[i];
    __syncthreads();
    const bool lvec = labels && ((reinterpret_cast<uintptr_t>(labels) & 15u) == 0);
    double jl = 0.0;
    const int64_t ngroups = (N + 3) / 4;
    for (int64_t g = (int64_t)blockIdx.x * BLOCK + tid; g < ngroups;
         g += (int64_t)gridDim.x * BLOCK) {
        float x[D][4];
        const int n = load_group<D, VEC>(X, ld, N, g, x);
        float best[4];
        int arg[4];
        nearest4<D>(smu, K, x, best, arg);
        float js = 0.0f;
#pragma unroll
        for (int p = 0; p < 4; ++p) js += p < n ? best[p] : 0.0f;
        jl += (double)js;
        if (labels) {
            if (lvec && n == 4) {
                *reinterpret_cast<int4*>(labels + g * 4) = make_int4(arg[0], arg[1], arg[2], arg[3]);
            } else {
#pragma unroll
                for (int p = 0; p < 4; ++p)
                    if (p < n) labels[g * 4 + p] = arg[p];
            }
        }
    }
    jl = wave_sum(jl);
    if ((tid & 63) == 0) sred[w] = jl;
    __syncthreads();
    double jb = 0.0;
#pragma unroll
    for (int v = 0; v < NW; ++v) jb += sred[v];
    if (!finish_block(&st->ticket, &st->jpart[blockIdx.x], jb, &slast)) return;
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
