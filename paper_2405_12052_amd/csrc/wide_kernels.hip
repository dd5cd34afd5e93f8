// wide_kernels.hip -- the Lloyd iteration for general d (up to WD_MAX) and K
// (up to WK_MAX), see wide.h.
//
// Reassignment (the paper's argmin of the squared Euclidean distance): every
// point is compared with every centre in the direct form
//   s_k = (x_0 - m_k0)^2 + (x_1 - m_k1)^2 + ... + (x_{d-1} - m_k,d-1)^2
// in float32, left to right, the first term a product and the others fused
// multiply-adds -- the same expression, in the same order, as the direct
// form of the 2-D/3-D kernels -- and the first k attaining the minimum wins.
// Each lane holds P consecutive points in registers; the float32 centres sit
// in LDS and are read as wave-uniform (broadcast) float4s, each serving the
// P points of every lane.
//
// Mean step: the points' coordinates as integers rint(x * 2^G) (|x| * 2^G <
// 2^30) and a count of one are added to their cluster's int64 slots in LDS
// (coordinate-major, slot j * K + k); each block writes its K * (d + 1) slots
// as one row of partials.
// wide_reduce sums the rows over the grid, WCHUNK rows per thread, and adds
// the chunk sums to the totals with device-scope integer atomics; integer
// addition is exact, so the totals do not depend on the order.  The last
// block to finish divides in float64 (the paper's mean with its indicator
// function), keeps the centre of an empty cluster, computes E (sum over the
// centres of the squared shift) and applies the tolerance test.
#include "wide.h"
#include "lloyd_device.h"

namespace km {
namespace {

static_assert(WBLOCK == BLOCK, "the wide kernels use the block helpers of lloyd_device.h");

enum { WMODE_ACC = 0, WMODE_LABEL = 1 };

template <int D>
struct WShape {
    static constexpr int DS = wide_stride(D);  // floats per centre in LDS
    static constexpr int NB = DS / 4;          // float4 reads per centre
    static constexpr int P = D <= 16 ? 4 : 2;  // points per lane
};

// Load the P consecutive points starting at i0 (n of them exist) into
// x[p][j]; coordinates j >= d are zero.
template <int D, int P>
__device__ __forceinline__ void wide_load(const float* __restrict__ X, int64_t ld, int d,
                                          bool vec, int64_t i0, int n, float (&x)[P][D]) {
#pragma unroll
    for (int j = 0; j < D; ++j) {
        if (j < d) {
            const float* row = X + (int64_t)j * ld + i0;
            if (vec && n == P) {
                if constexpr (P == 4) {
                    const float4 v = *reinterpret_cast<const float4*>(row);
                    x[0][j] = v.x; x[1][j] = v.y; x[2][j] = v.z; x[3][j] = v.w;
                } else {
                    const float2 v = *reinterpret_cast<const float2*>(row);
                    x[0][j] = v.x; x[1][j] = v.y;
                }
            } else {
#pragma unroll
                for (int p = 0; p < P; ++p) x[p][j] = p < n ? row[p] : 0.0f;
            }
        } else {
#pragma unroll
            for (int p = 0; p < P; ++p) x[p][j] = 0.0f;
        }
    }
}

// Reassignment of this thread's grid-stride share of the points against the
// K centres cm (LDS, stride DS, zero padded).  MODE_ACC adds each point to
// its cluster's slots in acc (K x (d + 1)); MODE_LABEL writes labels (if not
// null).  Both add the direct-form distance to the chosen centre to jl.
template <int D, int MODE>
__device__ __forceinline__ void wide_points(const WState* __restrict__ st, const float* cm,
                                            int K, int d, int G, unsigned long long* acc,
                                            int32_t* __restrict__ labels, double& jl) {
    using S = WShape<D>;
    constexpr int P = S::P, NB = S::NB;
    const int64_t N = st->N, ld = st->ld;
    const float* __restrict__ X = st->X;
    const bool vec = st->vec != 0;
    const int64_t ngroups = (N + P - 1) / P;
    const float4* cm4 = reinterpret_cast<const float4*>(cm);
    for (int64_t g = (int64_t)blockIdx.x * WBLOCK + threadIdx.x; g < ngroups;
         g += (int64_t)gridDim.x * WBLOCK) {
        const int64_t i0 = g * P;
        const int n = (N - i0) < P ? (int)(N - i0) : P;
        float x[P][D];
        wide_load<D, P>(X, ld, d, vec, i0, n, x);
        float best[P];
        int arg[P];
#pragma unroll
        for (int p = 0; p < P; ++p) { best[p] = INFINITY; arg[p] = 0; }
        for (int k = 0; k < K; ++k) {
            float s[P];
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                const float4 m = cm4[k * NB + b];
                const float mv[4] = {m.x, m.y, m.z, m.w};
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int j = 4 * b + u;
                    if (j < D) {
#pragma unroll
                        for (int p = 0; p < P; ++p) {
                            const float t = x[p][j] - mv[u];
                            s[p] = j == 0 ? t * t : fmaf(t, t, s[p]);
                        }
                    }
                }
            }
#pragma unroll
            for (int p = 0; p < P; ++p) {
                if (s[p] < best[p]) { best[p] = s[p]; arg[p] = k; }
            }
        }
#pragma unroll
        for (int p = 0; p < P; ++p) {
            if (p < n) {
                jl += (double)best[p];
                if constexpr (MODE == WMODE_ACC) {
                    // coordinate-major slots [j * K + k]: the lanes' clusters
                    // spread over the LDS banks
                    unsigned long long* a = acc + arg[p];
#pragma unroll
                    for (int j = 0; j < D; ++j) {
                        if (j < d) {
                            const long long q = (long long)__float2int_rn(ldexpf(x[p][j], G));
                            __hip_atomic_fetch_add(&a[j * K], (unsigned long long)q,
                                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                        }
                    }
                    __hip_atomic_fetch_add(&a[d * K], 1ull, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_WORKGROUP);
                } else {
                    if (labels) labels[i0 + p] = arg[p];
                }
            }
        }
    }
}

// Sum of v over the block, waves added in index order; valid in every thread.
__device__ __forceinline__ double block_sum(double v, double* sw) {
    v = wave_sum(v);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sw[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < NW; ++w) s += sw[w];
    return s;
}

// Sum of the n float64 values v(i), i in [0, n), in a fixed order: lane l of
// wave 0 adds a contiguous run of them in index order, then thread 0 adds the
// 64 run sums in lane order.  The result is valid in thread 0.  sw: 64 LDS.
template <typename F>
__device__ __forceinline__ double ordered_sum(int n, F v, double* sw) {
    const int tid = threadIdx.x;
    if (tid < 64) {
        const int per = (n + 63) / 64;
        const int a = tid * per, b = a + per < n ? a + per : n;
        double s = 0.0;
        for (int i = a; i < b; ++i) s += v(i);
        sw[tid] = s;
    }
    __syncthreads();
    double s = 0.0;
    if (tid == 0)
        for (int l = 0; l < 64; ++l) s += sw[l];
    return s;
}

// ------------------------------------------------------------------ kernels

// Once per fit: max |x| over the data (fixed-point exponent; NaN/Inf stops
// the fit) and zeroed totals.
__global__ __launch_bounds__(WBLOCK) void wide_scan(WState* __restrict__ st) {
    const int tid = threadIdx.x;
    const int d = st->d;
    const int64_t N = st->N, ld = st->ld;
    const int nacc = st->K * (d + 1);
    const int64_t stride = (int64_t)gridDim.x * WBLOCK;
    const int64_t t0 = (int64_t)blockIdx.x * WBLOCK + tid;
    for (int64_t i = t0; i < nacc; i += stride) st->tot[i] = 0ull;
    uint32_t m = 0;
    for (int j = 0; j < d; ++j) {
        const float* __restrict__ row = st->X + (int64_t)j * ld;
        for (int64_t i = t0; i < N; i += stride) {
            const uint32_t b = __float_as_uint(row[i]) & 0x7fffffffu;
            m = b > m ? b : m;
        }
    }
    m = wave_max(m);
    if ((tid & 63) == 0 && m) {
        __hip_atomic_fetch_max(&st->absmax_bits, m, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (m >= 0x7f800000u) {
            __hip_atomic_fetch_or(&st->flags, (int32_t)FLAG_NONFINITE, __ATOMIC_RELAXED,
                                  __HIP_MEMORY_SCOPE_AGENT);
            st_agent(&st->done, 1);
        }
    }
}

// Reassignment and per-block sums of one update.
template <int D>
__global__ __launch_bounds__(WBLOCK) void wide_update(WState* __restrict__ st) {
    extern __shared__ __align__(16) unsigned char wsm[];
    if (st->done) return;
    using S = WShape<D>;
    const int tid = threadIdx.x;
    const int d = st->d, K = st->K, nacc = K * (d + 1);
    unsigned long long* acc = reinterpret_cast<unsigned long long*>(wsm);
    float* cm = reinterpret_cast<float*>(wsm + (((size_t)nacc * 8 + 15) & ~(size_t)15));
    double* sw = reinterpret_cast<double*>(cm + (size_t)K * S::DS);
    const int G = scale_exponent(st->absmax_bits);
    for (int i = tid; i < K * S::DS; i += WBLOCK) cm[i] = st->mu32[i];
    for (int i = tid; i < nacc; i += WBLOCK) acc[i] = 0ull;
    __syncthreads();
    double jl = 0.0;
    wide_points<D, WMODE_ACC>(st, cm, K, d, G, acc, nullptr, jl);
    const double jb = block_sum(jl, sw);  // also orders the LDS atomics before the copy-out
    unsigned long long* row = st->part + (size_t)blockIdx.x * nacc;
    for (int i = tid; i < nacc; i += WBLOCK) row[i] = acc[i];
    if (tid == 0) st->jpart[blockIdx.x] = jb;
}

// Totals of the partial rows, then (last block) the float64 mean step.
// Grid: x = tiles of WBLOCK slots, y = chunks of WCHUNK rows.
__global__ __launch_bounds__(WBLOCK) void wide_reduce(WState* __restrict__ st) {
    extern __shared__ __align__(16) unsigned char wsm[];
    __shared__ double sw[64];
    __shared__ int sflag;
    __shared__ int sempty;
    if (st->done) return;
    const int tid = threadIdx.x;
    const int d = st->d, K = st->K, nacc = K * (d + 1), gu = st->grid;
    unsigned long long* tot = st->tot;
    {
        const int i = blockIdx.x * WBLOCK + tid;
        const int b0 = blockIdx.y * WCHUNK;
        const int b1 = b0 + WCHUNK < gu ? b0 + WCHUNK : gu;
        if (i < nacc && b0 < b1) {
            const unsigned long long* __restrict__ col = st->part + i;
            unsigned long long v[WCHUNK];
#pragma unroll
            for (int u = 0; u < WCHUNK; ++u) v[u] = b0 + u < b1 ? col[(size_t)(b0 + u) * nacc] : 0ull;
            unsigned long long s = 0ull;
#pragma unroll
            for (int u = 0; u < WCHUNK; ++u) s += v[u];
            if (s) (void)__hip_atomic_fetch_add(&tot[i], s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
    wait_mem();
    __syncthreads();
    if (tid == 0) {
        const uint32_t nblk = gridDim.x * gridDim.y;
        const uint32_t old = __hip_atomic_fetch_add(&st->ticket, 1u, __ATOMIC_RELAXED,
                                                    __HIP_MEMORY_SCOPE_AGENT);
        sflag = old == nblk - 1;
        sempty = 0;
    }
    __syncthreads();
    if (!sflag) return;

    // ---- last block: totals into LDS (8 device-coherent loads in flight per
    // thread), then cleared for the next update
    unsigned long long* stot = reinterpret_cast<unsigned long long*>(wsm);
    double* se = reinterpret_cast<double*>(wsm + (size_t)nacc * 8);
    for (int i0 = tid; i0 < nacc; i0 += 8 * WBLOCK) {
        unsigned long long v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int i = i0 + u * WBLOCK;
            v[u] = i < nacc ? ld_agent(&tot[i]) : 0ull;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int i = i0 + u * WBLOCK;
            if (i < nacc) {
                stot[i] = v[u];
                st_agent(&tot[i], 0ull);
            }
        }
    }
    __syncthreads();
    const int G = scale_exponent(st->absmax_bits);
    const int DS = wide_stride(wide_width(d));
    int emp = 0;
    for (int k = tid; k < K; k += WBLOCK) {
        const unsigned long long* a = stot + k;   // slots [j * K + k]
        const unsigned long long cnt = a[d * K];
        double e = 0.0;
        for (int j = 0; j < d; ++j) {
            const double old = st->mu64[k * d + j];
            const double v = cnt ? ldexp((double)(long long)a[j * K], -G) / (double)cnt : old;
            const double sh = v - old;
            e = fma(sh, sh, e);
            st->mu64[k * d + j] = v;
            st->mu32[k * DS + j] = (float)v;
        }
        se[k] = e;
        emp += cnt == 0ull;
    }
    if (emp) atomicAdd(&sempty, emp);
    __syncthreads();
    const double E = ordered_sum(K, [&](int k) { return se[k]; }, sw);
    __syncthreads();
    const double* jp = st->jpart;
    const double J = ordered_sum(gu, [&](int b) { return jp[b]; }, sw);
    if (tid == 0) {
        const int t = st->t;
        if (t < st->hist_cap) {
            st->E_hist[t] = E;
            st->J_hist[t] = J;
        }
        st->t = t + 1;
        st->E = E;
        st->empty_events += sempty;
        st->done = (E < st->tol || t + 1 >= st->max_iter) ? 1 : 0;
        st_agent(&st->ticket, 0u);
    }
}

// Reassignment only: labels and the objective at the current centres.
template <int D>
__global__ __launch_bounds__(WBLOCK) void wide_label(WState* __restrict__ st,
                                                     int32_t* __restrict__ labels) {
    extern __shared__ __align__(16) unsigned char wsm[];
    __shared__ double sj[WMAX_GRID];
    __shared__ double sw[64];
    __shared__ int sflag;
    using S = WShape<D>;
    const int tid = threadIdx.x;
    const int d = st->d, K = st->K;
    float* cm = reinterpret_cast<float*>(wsm);
    const int G = scale_exponent(st->absmax_bits);
    for (int i = tid; i < K * S::DS; i += WBLOCK) cm[i] = st->mu32[i];
    __syncthreads();
    double jl = 0.0;
    wide_points<D, WMODE_LABEL>(st, cm, K, d, G, nullptr, labels, jl);
    const double jb = block_sum(jl, sw);
    if (tid == 0) {
        st_agent(&st->jpart[blockIdx.x], jb);
        wait_mem();
        const uint32_t old = __hip_atomic_fetch_add(&st->ticket, 1u, __ATOMIC_RELAXED,
                                                    __HIP_MEMORY_SCOPE_AGENT);
        sflag = old == gridDim.x - 1;
    }
    __syncthreads();
    if (!sflag) return;
    const int nb = gridDim.x;
    for (int b = tid; b < nb; b += WBLOCK) sj[b] = ld_agent(&st->jpart[b]);
    __syncthreads();
    const double J = ordered_sum(nb, [&](int b) { return sj[b]; }, sw);
    if (tid == 0) {
        st->J = J;
        st_agent(&st->ticket, 0u);
    }
}

#define KM_WIDE_DISPATCH(KERN, d, grid, lds, s, ...)                                          \
    switch (wide_width(d)) {                                                                 \
        case 1: hipLaunchKernelGGL(KERN<1>, dim3(grid), dim3(WBLOCK), lds, s, __VA_ARGS__); break;   \
        case 2: hipLaunchKernelGGL(KERN<2>, dim3(grid), dim3(WBLOCK), lds, s, __VA_ARGS__); break;   \
        case 3: hipLaunchKernelGGL(KERN<3>, dim3(grid), dim3(WBLOCK), lds, s, __VA_ARGS__); break;   \
        case 4: hipLaunchKernelGGL(KERN<4>, dim3(grid), dim3(WBLOCK), lds, s, __VA_ARGS__); break;   \
        case 6: hipLaunchKernelGGL(KERN<6>, dim3(grid), dim3(WBLOCK), lds, s, __VA_ARGS__); break;   \
        case 8: hipLaunchKernelGGL(KERN<8>, dim3(grid), dim3(WBLOCK), lds, s, __VA_ARGS__); break;   \
        case 12: hipLaunchKernelGGL(KERN<12>, dim3(grid), dim3(WBLOCK), lds, s, __VA_ARGS__); break; \
        case 16: hipLaunchKernelGGL(KERN<16>, dim3(grid), dim3(WBLOCK), lds, s, __VA_ARGS__); break; \
        case 24: hipLaunchKernelGGL(KERN<24>, dim3(grid), dim3(WBLOCK), lds, s, __VA_ARGS__); break; \
        case 32: hipLaunchKernelGGL(KERN<32>, dim3(grid), dim3(WBLOCK), lds, s, __VA_ARGS__); break; \
        default: return hipErrorInvalidValue;                                                \
    }

}  // namespace

hipError_t launch_wide_scan(WState* st, int grid, hipStream_t s) {
    if (grid < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(wide_scan, dim3(grid), dim3(WBLOCK), 0, s, st);
    return hipGetLastError();
}

hipError_t launch_wide_update(WState* st, int d, int K, int grid, hipStream_t s) {
    const size_t lds = wide_lds_bytes(d, K);
    if (grid < 1 || grid > WMAX_GRID || d < 1 || d > WD_MAX || K < 1 || K > WK_MAX ||
        lds > (size_t)WLDS_MAX)
        return hipErrorInvalidValue;
    KM_WIDE_DISPATCH(wide_update, d, grid, lds, s, st)
    return hipGetLastError();
}

hipError_t launch_wide_reduce(WState* st, int d, int K, int grid_update, hipStream_t s) {
    const int nacc = K * (d + 1);
    // LDS of the last block: the totals and one float64 per centre (no more
    // than wide_update's tables, whose centres take at least 16 bytes each)
    const size_t lds = (size_t)nacc * 8 + (size_t)K * 8;
    if (d < 1 || d > WD_MAX || K < 1 || K > WK_MAX || grid_update < 1 ||
        grid_update > WMAX_GRID || lds > (size_t)WLDS_MAX)
        return hipErrorInvalidValue;
    const dim3 grid((nacc + WBLOCK - 1) / WBLOCK, (grid_update + WCHUNK - 1) / WCHUNK);
    hipLaunchKernelGGL(wide_reduce, grid, dim3(WBLOCK), lds, s, st);
    return hipGetLastError();
}

hipError_t launch_wide_label(WState* st, int32_t* labels, int d, int K, int grid,
                             hipStream_t s) {
    const size_t lds = (size_t)K * wide_stride(wide_width(d)) * 4;
    if (grid < 1 || grid > WMAX_GRID || d < 1 || d > WD_MAX || K < 1 || K > WK_MAX ||
        lds > (size_t)WLDS_MAX)
        return hipErrorInvalidValue;
    KM_WIDE_DISPATCH(wide_label, d, grid, lds, s, st, labels)
    return hipGetLastError();
}

int wide_blocks_per_cu(int d, size_t lds) {
    int n = 0;
    hipError_t e = hipErrorInvalidValue;
    switch (wide_width(d)) {
        case 1: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, reinterpret_cast<const void*>(wide_update<1>), WBLOCK, lds); break;
        case 2: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, reinterpret_cast<const void*>(wide_update<2>), WBLOCK, lds); break;
        case 3: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, reinterpret_cast<const void*>(wide_update<3>), WBLOCK, lds); break;
        case 4: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, reinterpret_cast<const void*>(wide_update<4>), WBLOCK, lds); break;
        case 6: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, reinterpret_cast<const void*>(wide_update<6>), WBLOCK, lds); break;
        case 8: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, reinterpret_cast<const void*>(wide_update<8>), WBLOCK, lds); break;
        case 12: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, reinterpret_cast<const void*>(wide_update<12>), WBLOCK, lds); break;
        case 16: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, reinterpret_cast<const void*>(wide_update<16>), WBLOCK, lds); break;
        case 24: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, reinterpret_cast<const void*>(wide_update<24>), WBLOCK, lds); break;
        case 32: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, reinterpret_cast<const void*>(wide_update<32>), WBLOCK, lds); break;
        default: break;
    }
    return e == hipSuccess ? n : 0;
}

}  // namespace km
