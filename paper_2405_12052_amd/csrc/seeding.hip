// seeding.hip -- k-means++ initial centres (D^2 weighting) on the device.
//
// The paper starts Lloyd's algorithm from centres drawn at random from the
// data (Section 3, first step) and notes that the outcome depends on them.
// k-means++ (Arthur and Vassilvitskii, 2007) is the standard alternative:
// the first centre is a uniformly drawn point, each next one is point i with
// probability proportional to D_i^2, its squared distance to the nearest
// centre chosen so far.  This file makes that draw exact and reproducible:
//
//   * D_i^2 is computed in float32, ((x0-c0)^2 + (x1-c1)^2) + (x2-c2)^2 with
//     every operation rounded separately (no fused multiply-add);
//   * weights are integers w_i = rint(D_i^2 * 2^G), G = B - ilogb(max D^2) - 1
//     with B = 62 - ceil(log2 N), so every w_i <= 2^B and their sum fits int64;
//     sums and prefix sums are exact, so no summation order can change a draw;
//   * with S = sum w_i and the caller's uniform u in [0, 1),
//     R = min(S - 1, floor(u * S)) and the chosen point is the first i whose
//     inclusive prefix sum exceeds R (S == 0: i = min(N-1, floor(u * N))).
//
// One round is two kernels over contiguous per-block chunks of the points:
// pp_update folds the newest centre into D^2 and takes the maximum, pp_select
// sums the block's weights and, in the last block to finish, walks the block
// sums and then that block's chunk to the chosen index.  Nothing goes back to
// the host until all K indices are known.
#include "ctx.h"

#include <math.h>
#include <string.h>

using km::fail;

namespace km {
struct SeedWS {
    int64_t cap = 0;
    float* d2 = nullptr;                 // [cap]
    unsigned long long* bsum = nullptr;  // [PP_MAX_BLOCKS]
    uint32_t* maxbits = nullptr;         // [KMAX] maximum D^2 of each round
    uint32_t* ticket = nullptr;          // [KMAX]
    int64_t* cidx = nullptr;             // [KMAX] chosen indices
    double* u = nullptr;                 // [KMAX]
    int32_t* flag = nullptr;             // non-finite D^2 seen
    float* cen = nullptr;                // [KMAX * 3] the chosen points
    double* u_h = nullptr;               // pinned staging
    int64_t* cidx_h = nullptr;
    int32_t* flag_h = nullptr;
    float* cen_h = nullptr;
};

void seed_ws_free(SeedWS* w) {
    if (!w) return;
    void* dev[] = {w->d2, w->bsum, w->maxbits, w->ticket, w->cidx, w->u, w->flag, w->cen};
    for (void* p : dev)
        if (p) (void)hipFree(p);
    void* host[] = {w->u_h, w->cidx_h, w->flag_h, w->cen_h};
    for (void* p : host)
        if (p) (void)hipHostFree(p);
    delete w;
}
}  // namespace km

namespace {

constexpr int PB = 256;
constexpr int PP_MAX_BLOCKS = 2048;

struct PPArgs {
    const float* X;
    int64_t N, ld, chunk;
    int d, nb, bits;          // bits = B, the weight range
    float* d2;
    unsigned long long* bsum;
    uint32_t* maxbits;
    uint32_t* ticket;
    int64_t* cidx;
    const double* u;
    int32_t* flag;
};

__device__ __forceinline__ float sq_dist(const PPArgs& a, int64_t i, float c0, float c1, float c2) {
#pragma clang fp contract(off)
    const float t0 = a.X[i] - c0;
    const float t1 = a.X[a.ld + i] - c1;
    float s = t0 * t0 + t1 * t1;
    if (a.d == 3) {
        const float t2 = a.X[2 * a.ld + i] - c2;
        s = s + t2 * t2;
    }
    return s;
}

// Integer weight of one D^2 at scale exponent G (exact: D^2 has 24 significant
// bits and the scaling is by a power of two).
__device__ __forceinline__ unsigned long long weight(float v, int G) {
    return (unsigned long long)rint(ldexp((double)v, G));
}

__device__ __forceinline__ int weight_exponent(uint32_t maxbits, int bits) {
    const float m = __uint_as_float(maxbits);
    if (!(m > 0.0f)) return 0;
    return bits - ilogbf(m) - 1;
}

// Round j >= 1: D^2 <- min(D^2, |x - c_{j-1}|^2) (j == 1: the distance
// itself), block maximum folded into maxbits[j].
__global__ __launch_bounds__(PB) void pp_update(PPArgs a, int j) {
    const int64_t lo = (int64_t)blockIdx.x * a.chunk;
    const int64_t hi = lo + a.chunk < a.N ? lo + a.chunk : a.N;
    const int64_t ci = a.cidx[j - 1];
    const float c0 = a.X[ci], c1 = a.X[a.ld + ci], c2 = a.d == 3 ? a.X[2 * a.ld + ci] : 0.0f;
    uint32_t mx = 0u;
    for (int64_t i = lo + threadIdx.x; i < hi; i += PB) {
        float v = sq_dist(a, i, c0, c1, c2);
        if (j > 1) v = fminf(a.d2[i], v);
        a.d2[i] = v;
        const uint32_t b = __float_as_uint(v);   // v >= 0 or NaN: the bits order like the values
        mx = b > mx ? b : mx;
    }
    __shared__ uint32_t wmax[PB / 64];
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        const uint32_t t = __shfl_xor(mx, o, 64);
        mx = t > mx ? t : mx;
    }
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t m = wmax[0];
        for (int w = 1; w < PB / 64; ++w) m = wmax[w] > m ? wmax[w] : m;
        atomicMax(&a.maxbits[j], m);
    }
}

// Inclusive prefix sum over the 64 lanes of a wave.
__device__ __forceinline__ unsigned long long wave_incl_scan(unsigned long long v) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const unsigned long long t = __shfl_up(v, o, 64);
        if (lane >= o) v += t;
    }
    return v;
}

// In one wave: among n consecutive terms term(0..n), find the first index
// whose inclusive prefix sum exceeds R (0 <= R < the total).  Each lane owns a
// consecutive run of ceil(n/64) terms, read 8 at a time so that the loads of
// a run overlap; the lane whose run holds the crossing walks it.  Returns the
// index in every lane.
template <typename F>
__device__ int64_t wave_find(int64_t n, unsigned long long R, F term) {
    const int lane = threadIdx.x & 63;
    const int64_t q = (n + 63) / 64;
    const int64_t b = (int64_t)lane * q;
    const int64_t e = b + q < n ? b + q : n;
    unsigned long long tot = 0;
    for (int64_t i0 = b; i0 < e; i0 += 8) {
        unsigned long long t[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) t[u] = i0 + u < e ? term(i0 + u) : 0ull;
#pragma unroll
        for (int u = 0; u < 8; ++u) tot += t[u];
    }
    const unsigned long long incl = wave_incl_scan(tot);
    const unsigned long long hit = __ballot(incl > R);
    const int owner = hit ? __builtin_ctzll(hit) : 63;
    int64_t found = -1;
    if (lane == owner) {
        unsigned long long p = incl - tot;
        for (int64_t i0 = b; i0 < e && found < 0; i0 += 8) {
            unsigned long long t[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) t[u] = i0 + u < e ? term(i0 + u) : 0ull;
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                if (found < 0 && i0 + u < e) {
                    p += t[u];
                    if (p > R) found = i0 + u;
                }
            }
        }
        if (found < 0) found = n - 1;   // unreachable with R < total
    }
    return __shfl(found, owner, 64);
}

// Round j >= 1: per-block weight sums, then (last block) the draw.
__global__ __launch_bounds__(PB) void pp_select(PPArgs a, int j) {
    const uint32_t mb = a.maxbits[j];
    const int G = weight_exponent(mb, a.bits);
    const int64_t lo = (int64_t)blockIdx.x * a.chunk;
    const int64_t hi = lo + a.chunk < a.N ? lo + a.chunk : a.N;
    unsigned long long s = 0;
    if (mb < 0x7f800000u)
        for (int64_t i = lo + threadIdx.x; i < hi; i += PB) s += weight(a.d2[i], G);
    __shared__ unsigned long long ws[PB / 64];
    __shared__ unsigned long long sb[PP_MAX_BLOCKS];
    __shared__ bool last;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o, 64);
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (int w = 0; w < PB / 64; ++w) t += ws[w];
        // block sums travel as device-coherent stores and loads (they write
        // through and read past the per-XCD L2 caches), so no device-wide
        // fence is needed: the store completes before the ticket is taken
        __hip_atomic_store(&a.bsum[blockIdx.x], t, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __builtin_amdgcn_s_waitcnt(0);
        const uint32_t old = __hip_atomic_fetch_add(&a.ticket[j], 1u, __ATOMIC_RELAXED,
                                                    __HIP_MEMORY_SCOPE_AGENT);
        last = old == (uint32_t)(gridDim.x - 1);
    }
    __syncthreads();
    if (!last) return;
    if (mb >= 0x7f800000u) {               // NaN or infinity among the D^2
        if (threadIdx.x == 0) {
            *a.flag = 1;
            a.cidx[j] = 0;
        }
        return;
    }
    // the block sums into LDS, all loads of a thread in flight together
    {
        unsigned long long v[PP_MAX_BLOCKS / PB];
#pragma unroll
        for (int u = 0; u < PP_MAX_BLOCKS / PB; ++u) {
            const int b = threadIdx.x + u * PB;
            v[u] = b < a.nb ? __hip_atomic_load(&a.bsum[b], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                            : 0ull;
        }
#pragma unroll
        for (int u = 0; u < PP_MAX_BLOCKS / PB; ++u) {
            const int b = threadIdx.x + u * PB;
            if (b < a.nb) sb[b] = v[u];
        }
    }
    __syncthreads();
    if (threadIdx.x >= 64) return;
    unsigned long long S = 0;
    {
        unsigned long long t = 0;
        for (int b = threadIdx.x; b < a.nb; b += 64) t += sb[b];
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) t += __shfl_xor(t, o, 64);
        S = t;
    }
    const double u = a.u[j];
    int64_t chosen;
    if (S == 0) {
        const double f = floor(u * (double)a.N);
        chosen = f < (double)(a.N - 1) ? (int64_t)f : a.N - 1;
    } else {
        double f = floor(u * (double)S);
        unsigned long long R = f < (double)S ? (unsigned long long)f : S - 1;
        if (R > S - 1) R = S - 1;
        unsigned long long before = 0;
        const int64_t blk = wave_find(a.nb, R, [&](int64_t b) { return sb[b]; });
        for (int64_t b = threadIdx.x; b < blk; b += 64) before += sb[b];
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) before += __shfl_xor(before, o, 64);
        const int64_t b0 = blk * a.chunk;
        const int64_t n = (b0 + a.chunk < a.N ? b0 + a.chunk : a.N) - b0;
        const float* d2 = a.d2 + b0;
        chosen = b0 + wave_find(n, R - before, [&](int64_t i) {
            return weight(d2[i], G);   // written by the previous kernel
        });
    }
    if (threadIdx.x == 0) a.cidx[j] = chosen;
}

// The chosen points, as float32 centres [K][d].
__global__ void pp_gather(PPArgs a, int K, float* cen) {
    for (int t = threadIdx.x; t < K * a.d; t += blockDim.x) {
        const int j = t / a.d, q = t % a.d;
        cen[t] = a.X[(int64_t)q * a.ld + a.cidx[j]];
    }
}

}  // namespace

extern "C" {

int kmeans_pp_init(kmeans_ctx* c, const float* X, int64_t N, int64_t ld, int32_t d, int32_t K,
                   const double* u, double* centroids_out, int64_t* index_out) {
    if (!c) return KM_EINVAL;
    c->err.clear();
    if (N < 1 || N > 2147483647LL) return fail(c, KM_EINVAL, "N=%lld out of [1, 2^31-1]", (long long)N);
    if (ld < N) return fail(c, KM_EINVAL, "ld=%lld < N=%lld", (long long)ld, (long long)N);
    if (d != 2 && d != 3) return fail(c, KM_EUNSUPPORTED, "d=%d: only 2-D and 3-D points are implemented", d);
    if (K < 1) return fail(c, KM_EINVAL, "K=%d < 1", K);
    if (K > km::KMAX) return fail(c, KM_EUNSUPPORTED, "K=%d > %d", K, km::KMAX);
    if (K > N) return fail(c, KM_EINVAL, "K=%d > N=%lld", K, (long long)N);
    if (!u) return fail(c, KM_EINVAL, "u is NULL");
    if (!centroids_out) return fail(c, KM_EINVAL, "centroids_out is NULL");
    for (int j = 0; j < K; ++j)
        if (!(u[j] >= 0.0 && u[j] < 1.0)) return fail(c, KM_EINVAL, "u[%d] = %g is not in [0, 1)", j, u[j]);
    int rc = km::check_device_ptr(c, X, "X");
    if (rc) return rc;
    KM_HIP(c, hipSetDevice(c->device));

    if (!c->sws) {
        c->sws = new km::SeedWS();
        km::SeedWS* w = c->sws;
        if (hipMalloc(&w->bsum, sizeof(unsigned long long) * PP_MAX_BLOCKS) != hipSuccess ||
            hipMalloc(&w->maxbits, sizeof(uint32_t) * km::KMAX) != hipSuccess ||
            hipMalloc(&w->ticket, sizeof(uint32_t) * km::KMAX) != hipSuccess ||
            hipMalloc(&w->cidx, sizeof(int64_t) * km::KMAX) != hipSuccess ||
            hipMalloc(&w->u, sizeof(double) * km::KMAX) != hipSuccess ||
            hipMalloc(&w->flag, sizeof(int32_t)) != hipSuccess ||
            hipMalloc(&w->cen, sizeof(float) * km::KMAX * 3) != hipSuccess ||
            hipHostMalloc(&w->cen_h, sizeof(float) * km::KMAX * 3, 0) != hipSuccess ||
            hipHostMalloc(&w->u_h, sizeof(double) * km::KMAX, 0) != hipSuccess ||
            hipHostMalloc(&w->cidx_h, sizeof(int64_t) * km::KMAX, 0) != hipSuccess ||
            hipHostMalloc(&w->flag_h, sizeof(int32_t), 0) != hipSuccess) {
            km::seed_ws_free(w);
            c->sws = nullptr;
            return fail(c, KM_ENOMEM, "allocation of the seeding workspace failed");
        }
    }
    km::SeedWS* w = c->sws;
    if (w->cap < N) {
        if (w->d2) (void)hipFree(w->d2);
        w->d2 = nullptr;
        w->cap = 0;
        if (hipMalloc(&w->d2, sizeof(float) * (size_t)N) != hipSuccess)
            return fail(c, KM_ENOMEM, "hipMalloc of %lld distances failed", (long long)N);
        w->cap = N;
    }

    PPArgs a;
    a.X = X;
    a.N = N;
    a.ld = ld;
    a.d = d;
    int64_t nb = (N + PB * 4 - 1) / (PB * 4);
    if (nb > PP_MAX_BLOCKS) nb = PP_MAX_BLOCKS;
    a.chunk = (N + nb - 1) / nb;
    a.nb = (int)((N + a.chunk - 1) / a.chunk);
    int lg = 0;
    while ((1LL << lg) < N) ++lg;   // ceil(log2 N)
    a.bits = 62 - lg;
    a.d2 = w->d2;
    a.bsum = w->bsum;
    a.maxbits = w->maxbits;
    a.ticket = w->ticket;
    a.cidx = w->cidx;
    a.u = w->u;
    a.flag = w->flag;

    // the first centre: a uniformly drawn point
    const double f0 = floor(u[0] * (double)N);
    const int64_t i0 = f0 < (double)(N - 1) ? (int64_t)f0 : N - 1;
    memcpy(w->u_h, u, sizeof(double) * K);
    w->cidx_h[0] = i0;
    KM_HIP(c, hipMemcpyAsync(w->u, w->u_h, sizeof(double) * K, hipMemcpyHostToDevice, c->stream));
    KM_HIP(c, hipMemcpyAsync(w->cidx, w->cidx_h, sizeof(int64_t), hipMemcpyHostToDevice, c->stream));
    KM_HIP(c, hipMemsetAsync(w->maxbits, 0, sizeof(uint32_t) * km::KMAX, c->stream));
    KM_HIP(c, hipMemsetAsync(w->ticket, 0, sizeof(uint32_t) * km::KMAX, c->stream));
    KM_HIP(c, hipMemsetAsync(w->flag, 0, sizeof(int32_t), c->stream));
    for (int j = 1; j < K; ++j) {
        hipLaunchKernelGGL(pp_update, dim3(a.nb), dim3(PB), 0, c->stream, a, j);
        hipLaunchKernelGGL(pp_select, dim3(a.nb), dim3(PB), 0, c->stream, a, j);
    }
    hipLaunchKernelGGL(pp_gather, dim3(1), dim3(64), 0, c->stream, a, K, w->cen);
    KM_HIP(c, hipGetLastError());
    KM_HIP(c, hipMemcpyAsync(w->cidx_h, w->cidx, sizeof(int64_t) * K, hipMemcpyDeviceToHost, c->stream));
    KM_HIP(c, hipMemcpyAsync(w->cen_h, w->cen, sizeof(float) * K * d, hipMemcpyDeviceToHost, c->stream));
    KM_HIP(c, hipMemcpyAsync(w->flag_h, w->flag, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
    KM_HIP(c, hipStreamSynchronize(c->stream));
    if (*w->flag_h) return fail(c, KM_EINVAL, "X holds a NaN or an infinity");
    // the chosen points themselves are the centres
    for (int j = 0; j < K; ++j) {
        for (int q = 0; q < d; ++q) centroids_out[j * d + q] = (double)w->cen_h[j * d + q];
        if (index_out) index_out[j] = w->cidx_h[j];
    }
    return KM_OK;
}

}  // extern "C"
