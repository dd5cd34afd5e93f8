// wide_kernels.hip -- the Lloyd iteration for general d (up to WD_MAX) and K
// (up to WK_MAX), see wide.h.
//
// Reassignment (the paper's argmin of the squared Euclidean distance): every
// point is scored against every centre with the key m_k . x - |m_k|^2 / 2
// (d fused multiply-adds; the largest key is the nearest centre), in triples
// of centres whose best key carries the triple's number in its low bits.  A
// rounding bound on both keys of the top pair and on the float64 evaluation
// of the direct form (x_0 - m_k0)^2 + ... + (x_{d-1} - m_k,d-1)^2 certifies
// the winner when the gap exceeds it; the other points are queued per wave
// and re-scanned with that float64 direct form, first index of the minimum (the same
// near-tie rule as the 2-D/3-D kernels, so both give the same labels).  Each
// lane holds P consecutive points in registers; the float32 centres sit in
// LDS and are read as wave-uniform (broadcast) float4s, each serving the P
// points of every lane.
//
// Mean step: the points' coordinates as integers rint(x 2^F) (|x| 2^F < 2^44,
// lloyd_device.h) and a count of one are added to their cluster's int64
// slots in LDS (coordinate-major, slot j * K + k; no block takes more than
// FXP_BLOCK_POINTS points); each block writes its K * (d + 1) slots as one
// row of partials.
// wide_reduce sums the rows over the grid, WCHUNK rows per thread in 128
// bits, and adds each chunk sum to the totals as two limbs (its low 32 bits
// and the rest) with device-scope integer atomics; integer addition is exact,
// so the totals do not depend on the order.  The last
// block to finish divides in float64 (the paper's mean with its indicator
// function), keeps the centre of an empty cluster, computes E (sum over the
// centres of the squared shift) and applies the tolerance test.
#include "wide.h"
#include "lloyd_device.h"
#include "lloyd_mfma.h"

namespace km {
namespace {

static_assert(WBLOCK == BLOCK, "the wide kernels use the block helpers of lloyd_device.h");

template <int D>
struct WShape {
    static constexpr int DS = wide_stride(D);  // floats per centre in LDS
    static constexpr int NB = DS / 4;          // float4 reads per centre
    static constexpr int P = D <= 16 ? 4 : 2;  // points per lane
};

// The points are read through global-address-space pointers: flat loads
// also count against the LDS counter, so a wait for the points would wait
// for outstanding LDS operations too.
typedef const float __attribute__((address_space(1))) gfloat;
typedef float f32x4g __attribute__((ext_vector_type(4)));
typedef float f32x2g __attribute__((ext_vector_type(2)));
typedef const f32x4g __attribute__((address_space(1))) gvec4;
typedef const f32x2g __attribute__((address_space(1))) gvec2;

// The same for loads and stores of the state's arrays where a wave also
// exchanges values across lanes (LDS operations): device-coherent (relaxed,
// device scope) and plain, through global-address-space pointers.
template <typename T>
__device__ __forceinline__ T gld_agent(const T* p) {
    return __hip_atomic_load((const T __attribute__((address_space(1)))*)p, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ void gst_agent(T* p, T v) {
    __hip_atomic_store((T __attribute__((address_space(1)))*)p, v, __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ T gld(const T* p) {
    return *(const T __attribute__((address_space(1)))*)p;
}
template <typename T>
__device__ __forceinline__ void gst(T* p, T v) {
    *(T __attribute__((address_space(1)))*)p = v;
}

// Load the P consecutive points starting at i0 (n of them exist) into
// x[p][j]; coordinates j >= d are zero.
template <int D, int P>
__device__ __forceinline__ void wide_load(const float* __restrict__ X, int64_t ld, int d,
                                          bool vec, int64_t i0, int n, float (&x)[P][D]) {
#pragma unroll
    for (int j = 0; j < D; ++j) {
        if (j < d) {
            const gfloat* row = (const gfloat*)X + (int64_t)j * ld + i0;
            if (vec && n == P) {
                if constexpr (P == 4) {
                    const f32x4g v = *(const gvec4*)row;
                    x[0][j] = v.x; x[1][j] = v.y; x[2][j] = v.z; x[3][j] = v.w;
                } else {
                    const f32x2g v = *(const gvec2*)row;
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

// One point's direct-form distance to centre row c (zero padded to D).
template <int D>
__device__ __forceinline__ float wide_direct(const float (&x)[D], const float4* __restrict__ c) {
    float s = 0.0f;
#pragma unroll
    for (int b = 0; b < (D + 3) / 4; ++b) {
        const float4 m = c[b];
        const float mv[4] = {m.x, m.y, m.z, m.w};
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int j = 4 * b + u;
            if (j < D) {
                const float t = x[j] - mv[u];
                s = j == 0 ? t * t : fmaf(t, t, s);
            }
        }
    }
    return s;
}

// The same distance evaluated in float64 (differences, squares and the
// running sum each rounded to float64, left to right): the near-tie rule.
template <int D>
__device__ __forceinline__ double wide_direct64(const float (&x)[D], const float4* __restrict__ c) {
#pragma clang fp contract(off)
    double s = 0.0;
#pragma unroll
    for (int b = 0; b < (D + 3) / 4; ++b) {
        const float4 m = c[b];
        const float mv[4] = {m.x, m.y, m.z, m.w};
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int j = 4 * b + u;
            if (j < D) {
                const double t = (double)x[j] - (double)mv[u];
                s = j == 0 ? t * t : s + t * t;
            }
        }
    }
    return s;
}

// The scan of one lane's P points x against the centre triples [0, ntri) of
// a table in LDS (cm4: rows of NB float4, hh: the key constants): keys
// m_k . x - |m_k|^2 / 2 (the largest is the nearest centre), the largest of
// each triple with the triple's number within its chunk of 32 in its 5
// lowest bits, folded into the running two largest g1v, g2v; gch is the
// chunk of g1v, as a triple number counted from cbase (the first triple of
// the table).
template <int D, int P>
__device__ __forceinline__ void scan_table(const float (&x)[P][D], const float4* cm4,
                                           const float* hh, int ntri, int cbase, float pinf,
                                           float (&g1v)[P], float (&g2v)[P], int (&gch)[P]) {
    constexpr int NB = WShape<D>::NB;
    for (int c0 = 0; c0 < ntri; c0 += 32) {
        const int c1 = c0 + 32 < ntri ? c0 + 32 : ntri;
        float m1[P], m2[P];
#pragma unroll
        for (int p = 0; p < P; ++p) { m1[p] = -INFINITY; m2[p] = -INFINITY; }
        for (int t = c0; t < c1; ++t) {
            float sk[3][P];
#pragma unroll
            for (int u = 0; u < 3; ++u) {
                const int k = 3 * t + u;
                const float h = hh[k];
#pragma unroll
                for (int p = 0; p < P; ++p) sk[u][p] = h;
#pragma unroll
                for (int b = 0; b < NB; ++b) {
                    const float4 m = cm4[k * NB + b];
                    const float mv[4] = {m.x, m.y, m.z, m.w};
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int j = 4 * b + v;
                        if (j < D) {
#pragma unroll
                            for (int p = 0; p < P; ++p) sk[u][p] = fmaf(x[p][j], mv[v], sk[u][p]);
                        }
                    }
                }
            }
#pragma unroll
            for (int p = 0; p < P; ++p) {
                const float gmax = fmaxf(fmaxf(sk[0][p], sk[1][p]), sk[2][p]);
                const float gp = with_index(gmax, t - c0);
                m2[p] = __builtin_amdgcn_fmed3f(m1[p], gp, m2[p]);
                m1[p] = __builtin_amdgcn_fmed3f(m1[p], gp, pinf);
            }
        }
#pragma unroll
        for (int p = 0; p < P; ++p) {
            // merge the chunk's two largest into the running two largest
            const float hi2 = fmaxf(g2v[p], m2[p]);
            g2v[p] = __builtin_amdgcn_fmed3f(g1v[p], m1[p], hi2);
            gch[p] = m1[p] > g1v[p] ? cbase + c0 : gch[p];
            g1v[p] = fmaxf(g1v[p], m1[p]);
        }
    }
}

// Per-point constants of the certificate (see finish_points).
struct WBound {
    float kc, dc, hmax;
};

// The rounding of the two keys of a comparison: each key is d FMAs on
// -fl32(|m|^2)/2, within gamma_{d+1} mag(x) of the exact key, gamma_n =
// n u / (1 - n u), u = 2^-24, so both within (d + 1) 2^-23 mag(x) (with
// 2^-10 to spare for the float32 evaluation of mag and of the gap); and,
// with a factor of 16 to spare, twice the float64 rounding of the direct
// form of the two distances (the near-tie rule): (d + 2) 2^-53 (D1 + D2)
// with D1 + D2 <= 2 (|x|^2 + 2 |t1| + gap).
__device__ __forceinline__ WBound wide_bound(int d, const float* amax) {
    return WBound{(float)(d + 1) * 0x1.004p-23f, (float)(d + 2) * 0x1p-49f, 0.5f * amax[WD_MAX]};
}

// The end of the scan for one lane's P points: the winning triple's keys
// formed again (bit-identical) from the centre rows crow (NB float4 each,
// zero rows past K up to a whole triple) and constants hrow -- in LDS, or in
// device memory when the centres were staged in tiles -- its largest key,
// the first index attaining it and the triple's second largest; the
// certificate; certified points to sink(x, i, k, dist), the others to
// queue(flag, i) (every lane calls it, flag false for a point it does not
// queue).
template <int D, int P, typename Sink, typename Queue>
__device__ __forceinline__ void finish_points(const float (&x)[P][D], int n, int64_t i0,
                                              const float (&g1v)[P], const float (&g2v)[P],
                                              const int (&gch)[P], const float4* crow,
                                              const float* hrow, int K, int d,
                                              const float* amax, WBound wb, Sink&& sink,
                                              Queue&& queue) {
    constexpr int NB = WShape<D>::NB;
#pragma unroll
    for (int p = 0; p < P; ++p) {
        const int t = gch[p] + (int)(__float_as_uint(g1v[p]) & TRI_BITS);
        const int k0 = 3 * t;
        float s3[3];
#pragma unroll
        for (int u = 0; u < 3; ++u) {
            float v = hrow[k0 + u];
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                const float4 m = crow[(k0 + u) * NB + b];
                const float mv[4] = {m.x, m.y, m.z, m.w};
#pragma unroll
                for (int w = 0; w < 4; ++w) {
                    const int j = 4 * b + w;
                    if (j < D) v = fmaf(x[p][j], mv[w], v);
                }
            }
            s3[u] = v;
        }
        const float t1 = fmaxf(fmaxf(s3[0], s3[1]), s3[2]);
        const float t2 = __builtin_amdgcn_fmed3f(s3[0], s3[1], s3[2]);
        const int k = s3[0] == t1 ? k0 : (s3[1] == t1 ? k0 + 1 : k0 + 2);
        // certificate: the gap to the runner-up exceeds the rounding of
        // both keys and the float64 rounding of the direct form (so that
        // it, too, ranks them so).  Every other triple's largest key is
        // at most its packed maximum plus the index bits (31 units in the
        // last place, below 2^-18 of it), and that packed maximum is at
        // most g2v: so at most g2v + 2^-17 |g2v| (p + 2^-18 |p| grows
        // with p).  With a single triple g2v = -inf, the sum is a NaN and
        // fmaxf returns t2.
        const float sec = fmaxf(t2, g2v[p] + ldexpf(fabsf(g2v[p]), -17));
        const float gap = t1 - sec;
        float mag = wb.hmax, xx = 0.0f;
#pragma unroll
        for (int j = 0; j < D; ++j) {
            const float a = j < d ? amax[j] : 0.0f;
            mag = fmaf(a, fabsf(x[p][j]), mag);
            xx = fmaf(x[p][j], x[p][j], xx);
        }
        const float bound = fmaf(wb.kc, mag, wb.dc * (xx + 2.0f * fabsf(t1) + fabsf(gap)));
        const bool valid = p < n;
        const bool ok = gap > bound && k < K;
        if (valid && ok) sink(x[p], i0 + p, k, wide_direct<D>(x[p], crow + k * NB));
        queue(valid && !ok, i0 + p);
    }
}

// A wave's queue of uncertified points (wq, LDS, WQCAP entries), re-scanned
// 64 at a time, one per lane, in the float64 direct form over all K centre
// rows crow (LDS or device memory), first index of the minimum.
template <int D, typename Sink>
struct WQueue {
    const float* X;
    int64_t ld;
    int d, K;
    const float4* crow;
    int* wq;
    Sink& sink;
    int qn = 0;  // queue length (the same in every lane)

    __device__ __forceinline__ void drain(int cnt) {
        constexpr int NB = WShape<D>::NB;
        const int lane = threadIdx.x & 63;
        __builtin_amdgcn_wave_barrier();
        if (lane < cnt) {
            const int64_t i = wq[qn - cnt + lane];
            float xr[D];
#pragma unroll
            for (int j = 0; j < D; ++j) xr[j] = j < d ? X[(int64_t)j * ld + i] : 0.0f;
            double bq = INFINITY;
            int bk = 0;
#pragma unroll 1
            for (int k = 0; k < K; ++k) {
                const double dk = wide_direct64<D>(xr, crow + k * NB);
                if (dk < bq) { bq = dk; bk = k; }
            }
            sink(xr, i, bk, wide_direct<D>(xr, crow + bk * NB));
        }
        __builtin_amdgcn_wave_barrier();
        qn -= cnt;
    }
    __device__ __forceinline__ void push(bool f, int64_t i) {
        const int lane = threadIdx.x & 63;
        const uint64_t mq = __ballot(f);
        if (mq) {
            if (f) wq[qn + __popcll(mq & ((1ull << lane) - 1ull))] = (int)i;
            qn += __popcll(mq);
            if (qn >= 64) drain(64);
        }
    }
};

// Centre rows and key constants in device memory, read through the scalar
// cache where every lane reads the same address (they do not change while a
// kernel runs).
typedef const __attribute__((address_space(4))) float* cfp;

// The re-scan of the points the matrix-core scan leaves uncertified, in two
// levels.  Its certificate is wider than the VALU scan's (it covers the
// float32 sum of 3 D products), so most of those points are decided by the
// VALU keys: level 1 takes 64 queued points, one per lane, keys each against
// all K centres exactly as the VALU scan does (hh + the FMA chain over the
// coordinates), keeps the largest key t1 (first index) and the second
// largest t2, and applies the VALU scan's certificate to them.  The points
// that fail it (near-ties) go to a second queue, re-scanned 64 at a time in
// the float64 direct form (first index of the minimum).
template <int D, typename Sink>
struct WQueue2 {
    const float* X;
    int64_t ld;
    int d, K;
    cfp crow;  // K rows of WShape<D>::DS floats
    cfp hrow;
    const float* amax;
    WBound wb;
    int* wq;   // level 1 (WQCAP entries)
    int* wq2;  // level 2 (WQCAP entries)
    Sink& sink;
    int qn = 0, qn2 = 0;  // queue lengths (the same in every lane)

    __device__ __forceinline__ void load(int64_t i, float (&xr)[D]) const {
#pragma unroll
        for (int j = 0; j < D; ++j) xr[j] = j < d ? X[(int64_t)j * ld + i] : 0.0f;
    }

    __device__ __forceinline__ void drain2(int cnt) {
        constexpr int NB = WShape<D>::NB;
        const int lane = threadIdx.x & 63;
        const float4* rows = (const float4*)crow;
        __builtin_amdgcn_wave_barrier();
        if (lane < cnt) {
            const int64_t i = wq2[qn2 - cnt + lane];
            float xr[D];
            load(i, xr);
            double bq = INFINITY;
            int bk = 0;
#pragma unroll 1
            for (int k = 0; k < K; ++k) {
                const double dk = wide_direct64<D>(xr, rows + k * NB);
                if (dk < bq) { bq = dk; bk = k; }
            }
            sink(xr, i, bk, wide_direct<D>(xr, rows + bk * NB));
        }
        __builtin_amdgcn_wave_barrier();
        qn2 -= cnt;
    }

    __device__ __forceinline__ void push2(bool f, int64_t i) {
        const int lane = threadIdx.x & 63;
        const uint64_t mq = __ballot(f);
        if (mq) {
            if (f) wq2[qn2 + __popcll(mq & ((1ull << lane) - 1ull))] = (int)i;
            qn2 += __popcll(mq);
            if (qn2 >= 64) drain2(64);
        }
    }

    __device__ __forceinline__ void drain(int cnt) {
        constexpr int NB = WShape<D>::NB;
        const int lane = threadIdx.x & 63;
        __builtin_amdgcn_wave_barrier();
        bool f = false;
        int64_t i = 0;
        if (lane < cnt) {
            i = wq[qn - cnt + lane];
            float xr[D];
            load(i, xr);
            float t1 = -INFINITY, t2 = -INFINITY;
            int k1 = 0;
#pragma unroll 2
            for (int k = 0; k < K; ++k) {
                float v = hrow[k];
#pragma unroll
                for (int j = 0; j < D; ++j) v = fmaf(xr[j], crow[k * (4 * NB) + j], v);
                t2 = fmaxf(t2, fminf(t1, v));
                k1 = v > t1 ? k : k1;
                t1 = fmaxf(t1, v);
            }
            float mag = wb.hmax, xx = 0.0f;
#pragma unroll
            for (int j = 0; j < D; ++j) {
                const float a = j < d ? amax[j] : 0.0f;
                mag = fmaf(a, fabsf(xr[j]), mag);
                xx = fmaf(xr[j], xr[j], xx);
            }
            const float gap = t1 - t2;
            const float bound = fmaf(wb.kc, mag, wb.dc * (xx + 2.0f * fabsf(t1) + fabsf(gap)));
            if (gap > bound) {
                const float4* rows = (const float4*)crow;
                sink(xr, i, k1, wide_direct<D>(xr, rows + k1 * NB));
            } else {
                f = true;
            }
        }
        __builtin_amdgcn_wave_barrier();
        qn -= cnt;
        push2(f, i);
    }

    __device__ __forceinline__ void push(bool f, int64_t i) {
        const int lane = threadIdx.x & 63;
        const uint64_t mq = __ballot(f);
        if (mq) {
            if (f) wq[qn + __popcll(mq & ((1ull << lane) - 1ull))] = (int)i;
            qn += __popcll(mq);
            if (qn >= 64) drain(64);
        }
    }

    __device__ __forceinline__ void finish() {
        if (qn > 0) drain(qn);
        if (qn2 > 0) drain2(qn2);
    }
};

// Reassignment of this thread's grid-stride share of the points against the
// K centres cm (LDS, Kpad rows of stride DS, zero padded) with the key
// constants hh and the bound coefficients amax (see the file header).
// Certified points go to sink(x, i, k, dist) at once; the others are queued
// in the wave's LDS queue wq (point indices) and re-scanned in the direct
// form 64 at a time, one per lane.
template <int D, typename Sink>
__device__ __forceinline__ void wide_points(const WState* __restrict__ st, const float* cm,
                                            const float* hh, const float* amax, int K, int d,
                                            int* __restrict__ wq, Sink&& sink) {
    using S = WShape<D>;
    constexpr int P = S::P;
    const int64_t N = st->N, ld = st->ld;
    const float* __restrict__ X = st->X;
    const bool vec = st->vec != 0;
    const float pinf = st->plus_inf;
    const int ntri = (K + 2) / 3;
    const int lane = threadIdx.x & 63;
    const float4* cm4 = reinterpret_cast<const float4*>(cm);
    const WBound wb = wide_bound(d, amax);
    WQueue<D, Sink> q{X, ld, d, K, cm4, wq, sink};

    const int64_t ngroups = (N + P - 1) / P;
    // the loop runs over whole waves (the queue and its ballots need every
    // lane); lanes past the end carry no points
    for (int64_t gw = (int64_t)blockIdx.x * WBLOCK + (threadIdx.x & ~63); gw < ngroups;
         gw += (int64_t)gridDim.x * WBLOCK) {
        const int64_t g = gw + lane;
        const int64_t i0 = g * P;
        const int n = g < ngroups ? ((N - i0) < P ? (int)(N - i0) : P) : 0;
        float x[P][D];
        if (n > 0) {
            wide_load<D, P>(X, ld, d, vec, i0, n, x);
        } else {
#pragma unroll
            for (int p = 0; p < P; ++p)
#pragma unroll
                for (int j = 0; j < D; ++j) x[p][j] = 0.0f;
        }
        float g1v[P], g2v[P];
        int gch[P];
#pragma unroll
        for (int p = 0; p < P; ++p) { g1v[p] = -INFINITY; g2v[p] = -INFINITY; gch[p] = 0; }
        scan_table<D, P>(x, cm4, hh, ntri, 0, pinf, g1v, g2v, gch);
        finish_points<D, P>(x, n, i0, g1v, g2v, gch, cm4, hh, K, d, amax, wb, sink,
                            [&](bool f, int64_t i) { q.push(f, i); });
    }
    if (q.qn > 0) q.drain(q.qn);
}

// Centres per LDS tile of the tiled scan (wide.h).
template <int D>
struct WTile {
    static constexpr int KT = wide_tile_k(WShape<D>::DS);
};

// The same reassignment for K whose tables exceed one block's LDS: the
// block's threads take groups of points in step (a whole block per round,
// lanes past the end carry none), and each round stages the centres into LDS
// tile by tile (cm: WTile<D>::KT rows, hh: their constants), two barriers
// per tile, folding every tile into the running two largest keys.  The
// winning triple's keys, the certificate's direct distance and the float64
// re-scan read the centre rows and constants from device memory (st->mu32,
// st->hh: L2-resident, zero rows past K up to a whole triple).
template <int D, typename Sink>
__device__ __forceinline__ void wide_points_tiled(const WState* __restrict__ st, float* cm,
                                                  float* hh, const float* amax, int K, int d,
                                                  int* __restrict__ wq, Sink&& sink) {
    using S = WShape<D>;
    constexpr int P = S::P, DS = S::DS, KT = WTile<D>::KT;
    const int tid = threadIdx.x;
    const int64_t N = st->N, ld = st->ld;
    const float* __restrict__ X = st->X;
    const bool vec = st->vec != 0;
    const float pinf = st->plus_inf;
    const float* __restrict__ gmu = st->mu32;
    const float* __restrict__ ghh = st->hh;
    const float4* grow = reinterpret_cast<const float4*>(gmu);
    const float4* cm4 = reinterpret_cast<const float4*>(cm);
    const WBound wb = wide_bound(d, amax);
    WQueue<D, Sink> q{X, ld, d, K, grow, wq, sink};

    const int64_t ngroups = (N + P - 1) / P;
    for (int64_t base = (int64_t)blockIdx.x * WBLOCK; base < ngroups;
         base += (int64_t)gridDim.x * WBLOCK) {
        const int64_t g = base + tid;
        const int64_t i0 = g * P;
        const int n = g < ngroups ? ((N - i0) < P ? (int)(N - i0) : P) : 0;
        float x[P][D];
        if (n > 0) {
            wide_load<D, P>(X, ld, d, vec, i0, n, x);
        } else {
#pragma unroll
            for (int p = 0; p < P; ++p)
#pragma unroll
                for (int j = 0; j < D; ++j) x[p][j] = 0.0f;
        }
        float g1v[P], g2v[P];
        int gch[P];
#pragma unroll
        for (int p = 0; p < P; ++p) { g1v[p] = -INFINITY; g2v[p] = -INFINITY; gch[p] = 0; }
        for (int k0 = 0; k0 < K; k0 += KT) {
            const int kn = K - k0 < KT ? K - k0 : KT;
            const int kpn = wide_kpad(kn);
            __syncthreads();  // every wave is done with the previous tile
            for (int i = tid; i < kpn * DS; i += WBLOCK)
                cm[i] = k0 * DS + i < K * DS ? gmu[(size_t)k0 * DS + i] : 0.0f;
            for (int i = tid; i < kpn; i += WBLOCK) hh[i] = ghh[k0 + i];
            __syncthreads();
            scan_table<D, P>(x, cm4, hh, kpn / 3, k0 / 3, pinf, g1v, g2v, gch);
        }
        finish_points<D, P>(x, n, i0, g1v, g2v, gch, grow, ghh, K, d, amax, wb, sink,
                            [&](bool f, int64_t i) { q.push(f, i); });
    }
    if (q.qn > 0) q.drain(q.qn);
}

// ----------------------------------------- matrix-core keys (widths 8 to 16)
// The keys of all K centres for 64 points at a time on the matrix cores
// (v_mfma_f32_32x32x16_f16), in the convention of the 2-D/3-D matrix-core
// scan (lloyd_mfma.h): the smallest key is the nearest centre,
//   s_k = |m_k|^2 / 2 - m_k . x   (= -(the VALU scan's key)),
// all scaled by 2^(2e), with points and centres scaled by 2^e so that every
// |x'|, |m'| < 2^13.  Each scaled value is split v = vh + vl into two fp16
// pieces and the product m' x' is taken as mh xh + mh xl + ml xh (each exact
// in float32).  Rows are centres (32 to a tile), columns points (32 to a
// chunk).  Lane half h takes the coordinates [h H, h H + H) of its point,
// H = D / 2, so that both halves run the same instructions: its 8 inner
// entries of k-step s are the entries 8 s .. 8 s + 7 of the sequence
//   (mh_0, xh_0), (mh_0, xl_0), (ml_0, xh_0), (mh_1, xh_1), ...
// over its H coordinates, zero past 3 H (S = ceil(3 H / 8) steps: 2 at
// width 8, 3 at 12 and 16).  |m|^2 / 2 enters exactly, as the float32
// accumulator input (pads: 2^120, above every real key).
//
// Each lane holds, per chunk, 16 keys of one point (result register r: the
// centre 8 (r / 4) + 4 h + r % 4 of the tile).  Tiles are taken in pairs:
// the packed quad minima (lloyd_mfma.h: a 3-bit number 4 (tile % 2) + quad
// in the low mantissa bits) of a pair go through the same tournament as the
// 2-D/3-D scan, and the pair's smallest and second smallest are merged into
// the point's running W (with its pair) and L.  The two lane halves of a
// point are then merged (one lane swap per value), half h finishing chunk h,
// and the winning quad's four centres are keyed again on the VALU exactly as
// the VALU scan keys them (its t1, first index, and t2).
//
// Certificate.  mag(x) = max_k |m_k|^2 / 2 + sum_j max_k |m_kj| |x_j| bounds
// every |s_k|.  A matrix key differs from the exact key by at most e_m: the
// split remainders and the dropped ml xl leave <= 3.01 2^-22 |m'_j||x'_j| +
// 2^-25 (|m'_j| + |x'_j|) per coordinate, the float32 sum of the 3 D
// products and the accumulator input, in any order and rounded to nearest or
// toward zero, <= 3 D 2^-23 (1 + 2^-10) mag'; f16 subnormal pieces flushed
// to zero would drop < 0.5 per product.  Packing moves a quad minimum by at
// most 7 units in its last place.  So when
//   L - W > 2 (3 D + 13.05) 2^-23 (1 + 2^-10) mag' + 5 D + 2^(2e) dc (|x|^2 + 2 |t1|)
// every centre outside the winning quad is farther, in exact arithmetic,
// than the quad's nearest by more than the float64 rounding of the direct
// form (the dc term of the VALU certificate); when in addition the VALU
// certificate holds for t1 against the quad's t2, the label is the
// first-index float64 direct-form argmin.  Other points go to the float64
// re-scan.  Scales outside e in [-24, 60] (data or centres beyond about
// 2^36 or below 2^-48) send every point to the re-scan.
// Points per lane of the matrix-core scan's wave iteration.
constexpr int WMFMA_PL = 4;

template <int D>
struct WMfma {
    static constexpr int H = D / 2;            // coordinates per lane half
    static constexpr int S = (3 * H + 7) / 8;  // k-steps of 16 inner entries
};

// Scale exponent e (|x| 2^e < 2^13, |m| 2^e < 2^13) from the data exponent
// and the bound coefficients amax (LDS); false outside [-24, 60].
__device__ __forceinline__ bool wide_mfma_scale(int xe, const float* amax, int d, int& e) {
    float a = 0.0f;
    for (int j = 0; j < d; ++j) a = fmaxf(a, amax[j]);
    e = 12 - xe;
    if (a > 0.0f) {
        const int ea = 12 - ilogbf(a);
        e = ea < e ? ea : e;
    }
    return e >= -24 && e <= 60;
}

// The A operands of every tile (record ((t S + s) 2 + h) 32 + c: centre
// 32 t + c, k-step s, lane half h) and the accumulator inputs (Cs[(t 2 + h)
// 16 + r]: centre 32 t + 8 (r / 4) + 4 h + r % 4), from the float32 centres
// and key constants in device memory.  Whole block.
template <int D>
__device__ __forceinline__ void stage_mfma(const WState* __restrict__ st, int K, int d, int e,
                                           u32x4* As, float* Cs) {
    using M = WMfma<D>;
    constexpr int H = M::H, S = M::S, DS = WShape<D>::DS;
    const int KT = (K + 31) / 32;
    const float sc = ldexpf(1.0f, e);
    const float* __restrict__ gmu = st->mu32;
    for (int idx = threadIdx.x; idx < KT * 64; idx += WBLOCK) {
        const int c = idx & 31, h = (idx >> 5) & 1, t = idx >> 6;
        const int k = 32 * t + c;
        _Float16 hi[H], lo[H];
#pragma unroll
        for (int jj = 0; jj < H; ++jj) {
            const int j = h * H + jj;
            const float m = k < K && j < d ? -gmu[(size_t)k * DS + j] * sc : 0.0f;
            split_f16(m, hi[jj], lo[jj]);
        }
#pragma unroll
        for (int s = 0; s < S; ++s) {
            u32x4 r;
#pragma unroll
            for (int w = 0; w < 4; ++w) {
                _Float16 e2[2];
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    const int v = 8 * s + 2 * w + u;
                    e2[u] = v < 3 * H ? (v % 3 == 2 ? lo[v / 3] : hi[v / 3]) : (_Float16)0;
                }
                r[w] = pack2(e2[0], e2[1]);
            }
            As[((t * S + s) * 2 + h) * 32 + c] = r;
        }
    }
    const float s2 = ldexpf(1.0f, 2 * e);
    for (int idx = threadIdx.x; idx < KT * 32; idx += WBLOCK) {
        const int r = idx & 15, h = (idx >> 4) & 1, t = idx >> 5;
        const int k = 32 * t + 8 * (r >> 2) + 4 * h + (r & 3);
        Cs[idx] = k < K ? -st->hh[k] * s2 : 0x1p120f;
    }
}

// The B operand of one point for this lane half: its H scaled coordinates u.
template <int D>
__device__ __forceinline__ void point_operand_w(const float (&u)[WMfma<D>::H],
                                                f16x8 (&B)[WMfma<D>::S]) {
    using M = WMfma<D>;
    constexpr int H = M::H, S = M::S;
    _Float16 hi[H], lo[H];
#pragma unroll
    for (int jj = 0; jj < H; ++jj) split_f16(u[jj], hi[jj], lo[jj]);
#pragma unroll
    for (int s = 0; s < S; ++s) {
        u32x4 r;
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            _Float16 e2[2];
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const int v = 8 * s + 2 * w + q;
                e2[q] = v < 3 * H ? (v % 3 == 1 ? lo[v / 3] : hi[v / 3]) : (_Float16)0;
            }
            r[w] = pack2(e2[0], e2[1]);
        }
        B[s] = __builtin_bit_cast(f16x8, r);
    }
}

// The 16 keys of one tile (A: its S operands, C: its accumulator inputs)
// for one chunk of points (B).
template <int S>
__device__ __forceinline__ f32x16 tile_keys(const f16x8 (&A)[S], const f16x8 (&B)[S],
                                            const f32x16& C) {
    f32x16 acc = __builtin_amdgcn_mfma_f32_32x32x16_f16(A[0], B[0], C, 0, 0, 0);
#pragma unroll
    for (int s = 1; s < S; ++s) acc = __builtin_amdgcn_mfma_f32_32x32x16_f16(A[s], B[s], acc, 0, 0, 0);
    return acc;
}

// Reassignment with the matrix-core keys (see above) of this wave's share of
// the grid, 32 PL points at a time (PL = 2 or 4 per lane: more independent
// matrix-core chains and loads in flight per wave); same contract as
// wide_points.  As, Cs: the staged operands (stage_mfma); amax: the bound
// coefficients (LDS); e, mok: the scale and whether it is in range.  Lane
// (c, h) loads the coordinates h H .. h H + H - 1 of points PL c .. PL c +
// PL - 1 of the iteration; chunk p is the 32 points {PL c + p}.  Chunks are
// merged in pairs (2 q, 2 q + 1), lane half h finishing chunk 2 q + h.
template <int D, int PL, typename Sink>
__device__ __forceinline__ void wide_points_mfma(const WState* __restrict__ st, const u32x4* As,
                                                 const float* Cs, const float* amax, int K,
                                                 int d, int e, bool mok, int* __restrict__ wq,
                                                 int* __restrict__ wq2, Sink&& sink) {
    static_assert(PL == 2 || PL == 4, "2 or 4 points per lane");
    using M = WMfma<D>;
    constexpr int H = M::H, S = M::S, NB = WShape<D>::NB;
    constexpr int PTS = 32 * PL;  // points per wave iteration
    const int lane = threadIdx.x & 63;
    const int c = lane & 31, h = lane >> 5;
    const int64_t N = st->N, ld = st->ld;
    const float* __restrict__ X = st->X;
    const bool vec = st->vec != 0;
    const float ninf = -st->plus_inf;
    const float4* grow = reinterpret_cast<const float4*>(st->mu32);
    const float* __restrict__ ghh = st->hh;
    // the winning quads' rows and key constants, gathered through global-
    // address-space pointers (a flat load would also wait for the wave's LDS
    // operand reads)
    const gvec4* growg = (const gvec4*)st->mu32;
    const gfloat* hhg = (const gfloat*)st->hh;
    const WBound wb = wide_bound(d, amax);
    const int KT = (K + 31) / 32;
    const float sc = ldexpf(1.0f, e);
    const float s2 = ldexpf(1.0f, 2 * e);
    const float kcm = 2.0f * (3.0f * D + 13.05f) * 0x1.004p-23f;
    const float habs = 5.0f * D;
    WQueue2<D, Sink> q{X, ld, d, K, (cfp)st->mu32, (cfp)ghh,
                       amax, wb, wq, wq2, sink};

    const int64_t nchunks = (N + PTS - 1) / PTS;
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    for (int64_t ch = (int64_t)blockIdx.x * NW + wid; ch < nchunks;
         ch += (int64_t)gridDim.x * NW) {
        const int64_t i0 = ch * PTS + PL * c;  // this lane's PL points
        const int rem = N - ch * PTS < PTS ? (int)(N - ch * PTS) : PTS;
        // this half's coordinates of the lane's points (one branch for all of
        // them: vector loads, or guarded 32-bit loads at the end of the data
        // or on unaligned rows)
        float x[H][PL];
        const gfloat* xrow = (const gfloat*)X + (int64_t)(h * H) * ld + i0;
        if (vec && i0 + PL <= N) {
#pragma unroll
            for (int jj = 0; jj < H; ++jj) {
                if (h * H + jj < d) {
                    if constexpr (PL == 4) {
                        const f32x4g v = *(const gvec4*)(xrow + (int64_t)jj * ld);
                        x[jj][0] = v.x;
                        x[jj][1] = v.y;
                        x[jj][2] = v.z;
                        x[jj][3] = v.w;
                    } else {
                        const f32x2g v = *(const gvec2*)(xrow + (int64_t)jj * ld);
                        x[jj][0] = v.x;
                        x[jj][1] = v.y;
                    }
                } else {
#pragma unroll
                    for (int p = 0; p < PL; ++p) x[jj][p] = 0.0f;
                }
            }
        } else {
#pragma unroll
            for (int jj = 0; jj < H; ++jj) {
                const bool in = h * H + jj < d;
#pragma unroll
                for (int p = 0; p < PL; ++p)
                    x[jj][p] = in && i0 + p < N ? xrow[(int64_t)jj * ld + p] : 0.0f;
            }
        }
        float W[PL], L[PL];
        int G[PL];
#pragma unroll
        for (int p = 0; p < PL; ++p) { W[p] = 0.0f; L[p] = 0.0f; G[p] = 0; }
        if (mok) {
            f16x8 B[PL][S];
#pragma unroll
            for (int p = 0; p < PL; ++p) {
                float u[H];
#pragma unroll
                for (int jj = 0; jj < H; ++jj) u[jj] = x[jj][p] * sc;
                point_operand_w<D>(u, B[p]);
                W[p] = INFINITY;
                L[p] = INFINITY;
            }
            for (int g = 0; g < KT; g += 2) {
                float pm[PL][8];
#pragma unroll
                for (int tt = 0; tt < 2; ++tt) {
                    const int t = g + tt;
                    if (tt == 1 && t >= KT) {
#pragma unroll
                        for (int p = 0; p < PL; ++p)
#pragma unroll
                            for (int r = 4; r < 8; ++r) pm[p][r] = INFINITY;
                        break;
                    }
                    f16x8 A[S];
#pragma unroll
                    for (int s = 0; s < S; ++s)
                        A[s] = __builtin_bit_cast(f16x8, As[((t * S + s) * 2 + h) * 32 + c]);
                    const f32x16 C = *reinterpret_cast<const f32x16*>(Cs + (t * 2 + h) * 16);
#pragma unroll
                    for (int p = 0; p < PL; ++p) {
                        const f32x16 kk = tile_keys<S>(A, B[p], C);
                        if (tt == 0) tile_minima<0>(kk, ninf, reinterpret_cast<float(&)[4]>(pm[p][0]));
                        else tile_minima<1>(kk, ninf, reinterpret_cast<float(&)[4]>(pm[p][4]));
                    }
                }
#pragma unroll
                for (int p = 0; p < PL; ++p) {
                    float a1, a2;
                    top2_of_8(pm[p], a1, a2);
                    // into the running pair
                    L[p] = vmin3(vmax2(W[p], a1), L[p], a2);
                    G[p] = a1 < W[p] ? g : G[p];
                    W[p] = vmin2(W[p], a1);
                }
            }
        }
#pragma unroll
        for (int qq = 0; qq < PL / 2; ++qq) {
            const int p0 = 2 * qq;
            // lane half h finishes chunk p0 + h (point i0 + p0 + h): after each
            // swap, w0 is the h = 0 lane's value for that point, w1 the h = 1 lane's
            const auto ws = __builtin_amdgcn_permlane32_swap(__float_as_uint(W[p0]),
                                                              __float_as_uint(W[p0 + 1]), false, false);
            const auto ls = __builtin_amdgcn_permlane32_swap(__float_as_uint(L[p0]),
                                                              __float_as_uint(L[p0 + 1]), false, false);
            const auto gs = __builtin_amdgcn_permlane32_swap((uint32_t)G[p0], (uint32_t)G[p0 + 1],
                                                              false, false);
            const float w0 = __uint_as_float(ws[0]), w1 = __uint_as_float(ws[1]);
            const float l0 = __uint_as_float(ls[0]), l1 = __uint_as_float(ls[1]);
            const float Wc = vmin2(w0, w1);
            const float Lc = vmin3(vmax2(w0, w1), l0, l1);
            const int hw = w1 < w0 ? 1 : 0;
            const int gw = hw ? (int)gs[1] : (int)gs[0];
            // the point's coordinates: this half's H and the other half's
            float xp[D];
#pragma unroll
            for (int jj = 0; jj < H; ++jj) {
                const auto xs = __builtin_amdgcn_permlane32_swap(__float_as_uint(x[jj][p0]),
                                                                  __float_as_uint(x[jj][p0 + 1]),
                                                                  false, false);
                xp[jj] = __uint_as_float(xs[0]);
                xp[H + jj] = __uint_as_float(xs[1]);
            }
            // the winning quad: centres 32 (gw + tile) + 8 quad + 4 hw + 0..3,
            // keyed as the VALU scan keys them (rows past K: -2^127, never chosen)
            const uint32_t bits = __float_as_uint(Wc) & 7u;
            const int base = 32 * (gw + (int)(bits >> 2)) + 8 * (int)(bits & 3u) + 4 * hw;
            float s4[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int k = base + u;
                const int kk = k < K ? k : K - 1;
                float v = hhg[kk];
#pragma unroll
                for (int b = 0; b < NB; ++b) {
                    const f32x4g m = growg[kk * NB + b];
                    const float mv[4] = {m.x, m.y, m.z, m.w};
#pragma unroll
                    for (int w2 = 0; w2 < 4; ++w2) {
                        const int j = 4 * b + w2;
                        if (j < D) v = fmaf(xp[j], mv[w2], v);
                    }
                }
                s4[u] = k < K ? v : -0x1p127f;
            }
            const float a3 = fmaxf(fmaxf(s4[0], s4[1]), s4[2]);
            const float t1 = fmaxf(a3, s4[3]);
            const float t2 = fmaxf(__builtin_amdgcn_fmed3f(s4[0], s4[1], s4[2]), fminf(a3, s4[3]));
            int kq = 3;
            kq = s4[2] == t1 ? 2 : kq;
            kq = s4[1] == t1 ? 1 : kq;
            kq = s4[0] == t1 ? 0 : kq;
            const int k = base + kq;
            float mag = wb.hmax, xx = 0.0f;
#pragma unroll
            for (int j = 0; j < D; ++j) {
                const float a = j < d ? amax[j] : 0.0f;
                mag = fmaf(a, fabsf(xp[j]), mag);
                xx = fmaf(xp[j], xp[j], xx);
            }
            const float gap = t1 - t2;
            const float bound = fmaf(wb.kc, mag, wb.dc * (xx + 2.0f * fabsf(t1) + fabsf(gap)));
            const float thr = fmaf(fmaf(kcm, mag, wb.dc * (xx + 2.0f * fabsf(t1))), s2, habs);
            const int64_t i = i0 + p0 + h;
            const bool valid = PL * c + p0 + h < rem;
            const bool ok = mok && Lc - Wc > thr && gap > bound && k < K;
            if (valid && ok) sink(xp, i, k, wide_direct<D>(xp, grow + k * NB));
            q.push(valid && !ok, i);
        }
    }
    q.finish();
}

// Key tables of the float32 centres mu32 (K rows of stride DS): hh[k] =
// -fl32(sum_j m_kj^2) / 2 (the sum of squares in float64 FMAs, rounded
// once), pads up to a whole triple -2^127; amax[j] = max_k |m_kj| (j < d),
// amax[WD_MAX] = max_k fl32(sum_j m_kj^2).  Whole block; sred: LDS scratch of
// NW * (WD_MAX + 1) words.
__device__ void key_tables(const float* __restrict__ mu32, int K, int d, int DS,
                           float* __restrict__ hh, float* __restrict__ amax, uint32_t* sred) {
    const int tid = threadIdx.x, w = tid >> 6;
    const int kp = wide_kpad(K);
    // Every wave runs the same number of passes over the rows (the wave
    // maxima need all its lanes); a thread reads its row 8 coordinates per
    // round trip, and each wave keeps its per-coordinate maxima in sred.
    uint32_t cmx = 0;
    for (int k0 = 0; k0 < kp; k0 += WBLOCK) {
        const int k = k0 + tid;
        const bool in = k < K;
        double q = 0.0;
        for (int j0 = 0; j0 < d; j0 += 8) {
            float m[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) m[u] = in && j0 + u < d ? mu32[k * DS + j0 + u] : 0.0f;
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                if (j0 + u < d) {
                    q = fma((double)m[u], (double)m[u], q);
                    const uint32_t b = wave_max(__float_as_uint(m[u]) & 0x7fffffffu);
                    if ((tid & 63) == 0) {
                        uint32_t& r = sred[w * (WD_MAX + 1) + j0 + u];
                        r = k0 == 0 || b > r ? b : r;
                    }
                }
            }
        }
        if (in) {
            const float c = (float)q;
            hh[k] = -0.5f * c;
            cmx = __float_as_uint(c) > cmx ? __float_as_uint(c) : cmx;
        } else if (k < kp) {
            hh[k] = -0x1p127f;
        }
    }
    // per-wave maxima (non-negative floats order as their bits), then across
    // the waves: one barrier
    cmx = wave_max(cmx);
    if ((tid & 63) == 0) sred[w * (WD_MAX + 1) + WD_MAX] = cmx;
    __syncthreads();
    if (tid <= WD_MAX && (tid < d || tid == WD_MAX)) {
        uint32_t r = 0;
        for (int v = 0; v < NW; ++v) r = sred[v * (WD_MAX + 1) + tid] > r ? sred[v * (WD_MAX + 1) + tid] : r;
        amax[tid] = __uint_as_float(r);
    }
    __syncthreads();
}

// Stage the centres, key constants and bound coefficients in LDS.
template <int D>
__device__ __forceinline__ void stage_tables(const WState* __restrict__ st, int K, float* cm,
                                             float* hh, float* amax) {
    constexpr int DS = WShape<D>::DS;
    const int kp = wide_kpad(K);
    for (int i = threadIdx.x; i < kp * DS; i += WBLOCK) cm[i] = i < K * DS ? st->mu32[i] : 0.0f;
    for (int i = threadIdx.x; i < kp; i += WBLOCK) hh[i] = st->hh[i];
    for (int i = threadIdx.x; i <= WD_MAX; i += WBLOCK) amax[i] = st->amax[i];
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
        // the terms are fetched 8 at a time, then added one by one
        double s = 0.0;
        for (int i0 = a; i0 < b; i0 += 8) {
            double t[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) t[u] = i0 + u < b ? v(i0 + u) : 0.0;
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (i0 + u < b) s += t[u];
        }
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
// the fit), zeroed totals, and (block 0) the key tables of the initial
// centres.
__global__ __launch_bounds__(WBLOCK) void wide_scan(WState* __restrict__ st) {
    __shared__ uint32_t sred[NW * (WD_MAX + 1)];
    __shared__ uint32_t smx[NW];
    const int tid = threadIdx.x;
    if (blockIdx.x == 0)
        key_tables(st->mu32, st->K, st->d, wide_stride(wide_width(st->d)), st->hh, st->amax, sred);
    const int d = st->d;
    const int64_t N = st->N, ld = st->ld;
    const int nacc = st->K * (d + 1);
    const int64_t stride = (int64_t)gridDim.x * WBLOCK;
    const int64_t t0 = (int64_t)blockIdx.x * WBLOCK + tid;
    for (int64_t i = t0; i < 2 * nacc; i += stride) st->tot[i] = 0ull;
    // Each thread keeps 8 loads in flight (one at a time left the scan bound
    // by memory latency): of 16 bytes where the rows allow, from the first
    // whole group of 4, else of one float.
    uint32_t m = 0;
    const int64_t ng = st->vec ? N >> 2 : 0;
    for (int j = 0; j < d; ++j) {
        const float* __restrict__ row = st->X + (int64_t)j * ld;
        const float4* __restrict__ row4 = reinterpret_cast<const float4*>(row);
        for (int64_t g = t0; g < ng; g += 8 * stride) {
            float4 v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int64_t p = g + u * stride;
                v[u] = p < ng ? row4[p] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const uint32_t b0 = __float_as_uint(v[u].x) & 0x7fffffffu;
                const uint32_t b1 = __float_as_uint(v[u].y) & 0x7fffffffu;
                const uint32_t b2 = __float_as_uint(v[u].z) & 0x7fffffffu;
                const uint32_t b3 = __float_as_uint(v[u].w) & 0x7fffffffu;
                const uint32_t a = b0 > b1 ? b0 : b1, c = b2 > b3 ? b2 : b3;
                const uint32_t e = a > c ? a : c;
                m = e > m ? e : m;
            }
        }
        for (int64_t i = 4 * ng + t0; i < N; i += 8 * stride) {
            uint32_t b[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int64_t p = i + u * stride;
                b[u] = p < N ? __float_as_uint(row[p]) & 0x7fffffffu : 0u;
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) m = b[u] > m ? b[u] : m;
        }
    }
    m = wave_max(m);
    if ((tid & 63) == 0) smx[tid >> 6] = m;
    __syncthreads();
    if (tid == 0) {
        // one atomic per block, and only where it raises the stored maximum
        m = 0;
        for (int v = 0; v < NW; ++v) m = smx[v] > m ? smx[v] : m;
        if (m > ld_agent(&st->absmax_bits))
            __hip_atomic_fetch_max(&st->absmax_bits, m, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (m >= FXP_RANGE_BITS) {
            // NaN or infinity, or beyond the range of the fixed-point sums
            __hip_atomic_fetch_or(&st->flags,
                                  (int32_t)(m >= 0x7f800000u ? FLAG_NONFINITE : FLAG_RANGE),
                                  __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            st_agent(&st->done, 1);
        }
    }
}

// Reassignment and per-block sums of one update.  TRACK (indicator
// tracking): each point's previous label is read from st->track and the new
// one written there where it differs; the block's number of changed labels
// is added, times 2^32, to cluster 0's count in its partial row (a block
// counts at most 2^19 points and a fit at most 2^31 - 1, so the fields never
// overlap).
// A point's share of one update in the block's LDS sums: its fixed-point
// coordinates and a count of one into the coordinate-major slots [j K + k]
// (the lanes' clusters spread over the LDS banks), its distance into the
// thread's objective, and with TRACK its label into st->track.
template <int D, bool TRACK>
struct LdsSums {
    unsigned long long* acc;
    int K, d;
    double fscale;
    int32_t* track;
    double jl = 0.0;
    uint32_t nchg = 0;

    __device__ __forceinline__ void add(const float (&xr)[D], int64_t i, int k, float dist) {
        jl += (double)dist;
        if constexpr (TRACK) {
            if (track[i] != k) {
                track[i] = k;
                ++nchg;
            }
        }
        unsigned long long* a = acc + k;
#pragma unroll
        for (int j = 0; j < D; ++j) {
            if (j < d)
                __hip_atomic_fetch_add(&a[j * K], fxp_bits(xr[j], fscale), __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_WORKGROUP);
        }
        __hip_atomic_fetch_add(&a[d * K], 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    }

    // After the pass: the block's row of partials -- the sums of q (each
    // slot less FXP_MAGIC_BITS per point it received, the count of its
    // cluster) and the counts; with TRACK the block's changed labels added,
    // times 2^32, to cluster 0's count (a block counts at most 2^19 points
    // and a fit at most 2^31 - 1, so the fields never overlap) -- and its
    // objective partial.  q0: the waves' re-scan queues (empty by now, their
    // first words carry the per-wave counts); sw: NW doubles.  Whole block.
    __device__ __forceinline__ void publish(WState* __restrict__ st, int* q0, double* sw) {
        const int tid = threadIdx.x, nacc = K * (d + 1);
        unsigned long long chg = 0ull;
        if constexpr (TRACK) {
            const uint32_t nw = wave_sum_u32(nchg);
            if ((tid & 63) == 0) q0[(tid >> 6) * WQCAP] = (int)nw;
            __syncthreads();
#pragma unroll
            for (int v = 0; v < NW; ++v) chg += (uint32_t)q0[v * WQCAP];
        }
        const double jb = block_sum(jl, sw);  // also orders the LDS atomics before the copy-out
        unsigned long long* row = st->part + (size_t)blockIdx.x * nacc;
        for (int i = tid; i < nacc; i += WBLOCK) {
            const int k = i % K;
            unsigned long long v = i < d * K ? acc[i] - acc[d * K + k] * FXP_MAGIC_BITS : acc[i];
            if (TRACK && i == d * K) v += chg << 32;
            row[i] = v;
        }
        if (tid == 0) st->jpart[blockIdx.x] = jb;
    }
};

// Reassignment and per-block sums of one update.  TRACK (indicator
// tracking): each point's previous label is read from st->track and the new
// one written there where it differs, and the block's number of changed
// labels travels with the counts (LdsSums::publish).
template <int D, bool TRACK>
__device__ __forceinline__ void wide_update_body(WState* __restrict__ st, unsigned char* wsm) {
    using S = WShape<D>;
    const int tid = threadIdx.x;
    const int d = st->d, K = st->K, nacc = K * (d + 1);
    const int kp = wide_kpad(K);
    unsigned long long* acc = reinterpret_cast<unsigned long long*>(wsm);
    float* cm = reinterpret_cast<float*>(wsm + (((size_t)nacc * 8 + 15) & ~(size_t)15));
    float* hh = cm + (size_t)kp * S::DS;
    float* amax = hh + ((kp + 3) & ~3);
    int* q0 = reinterpret_cast<int*>(amax + 36);
    int* wq = q0 + (tid >> 6) * WQCAP;
    double* sw = reinterpret_cast<double*>(q0 + NW * WQCAP);
    stage_tables<D>(st, K, cm, hh, amax);
    for (int i = tid; i < nacc; i += WBLOCK) acc[i] = 0ull;
    __syncthreads();
    LdsSums<D, TRACK> sums{acc, K, d, fxp_scale(data_exponent(st->absmax_bits)), st->track};
    wide_points<D>(st, cm, hh, amax, K, d, wq,
                   [&](const float (&xr)[D], int64_t i, int k, float dist) { sums.add(xr, i, k, dist); });
    sums.publish(st, q0, sw);
}

// The same update with the matrix-core keys (widths 8 to 16, wide_mfma_lds_bytes
// of LDS): the A operands and accumulator inputs of every tile are staged in
// LDS in place of the float32 centre table.  FULL: d equals the width D, so
// that every per-coordinate test folds away at compile time.
template <int D, bool TRACK, bool FULL>
__device__ __forceinline__ void wide_update_mfma_body(WState* __restrict__ st, unsigned char* wsm) {
    using M = WMfma<D>;
    const int tid = threadIdx.x;
    const int d = FULL ? D : st->d, K = st->K, nacc = K * (d + 1);
    const int KT = (K + 31) / 32;
    unsigned long long* acc = reinterpret_cast<unsigned long long*>(wsm);
    u32x4* As = reinterpret_cast<u32x4*>(wsm + (((size_t)nacc * 8 + 63) & ~(size_t)63));
    float* Cs = reinterpret_cast<float*>(As + (size_t)KT * M::S * 64);
    float* amax = Cs + KT * 32;
    int* q0 = reinterpret_cast<int*>(amax + 36);
    int* wq = q0 + (tid >> 6) * WQCAP;
    int* wq2 = q0 + (NW + (tid >> 6)) * WQCAP;
    double* sw = reinterpret_cast<double*>(q0 + 2 * NW * WQCAP);
    const int xe = data_exponent(st->absmax_bits);
    for (int i = tid; i < nacc; i += WBLOCK) acc[i] = 0ull;
    for (int i = tid; i <= WD_MAX; i += WBLOCK) amax[i] = st->amax[i];
    __syncthreads();
    int e = 0;
    const bool mok = wide_mfma_scale(xe, amax, d, e);
    if (mok) stage_mfma<D>(st, K, d, e, As, Cs);
    __syncthreads();
    LdsSums<D, TRACK> sums{acc, K, d, fxp_scale(xe), st->track};
    wide_points_mfma<D, WMFMA_PL>(st, As, Cs, amax, K, d, e, mok, wq, wq2,
                        [&](const float (&xr)[D], int64_t i, int k, float dist) { sums.add(xr, i, k, dist); });
    sums.publish(st, q0, sw);
}

template <int D>
__global__ __launch_bounds__(WBLOCK) void wide_update(WState* __restrict__ st) {
    extern __shared__ __align__(16) unsigned char wsm[];
    if (st->done) return;
    wide_update_body<D, false>(st, wsm);
}

// The same with indicator tracking (KM_OPT_TRACK).
template <int D>
__global__ __launch_bounds__(WBLOCK) void wide_update_track(WState* __restrict__ st) {
    extern __shared__ __align__(16) unsigned char wsm[];
    if (st->done) return;
    wide_update_body<D, true>(st, wsm);
}

// Widths 12 and 16 run 2 waves per SIMD (LDS allows no more at K = 256): the
// compiler may then use 256 registers per lane and keeps the matrix-core
// results out of the accumulation registers.
template <int D, bool FULL>
__global__ __launch_bounds__(WBLOCK) __attribute__((amdgpu_waves_per_eu(1, D >= 12 ? 2 : 4))) void wide_update_mfma(WState* __restrict__ st) {
    extern __shared__ __align__(64) unsigned char wsm[];
    if (st->done) return;
    wide_update_mfma_body<D, false, FULL>(st, wsm);
}

template <int D, bool FULL>
__global__ __launch_bounds__(WBLOCK) __attribute__((amdgpu_waves_per_eu(1, D >= 12 ? 2 : 4))) void wide_update_mfma_track(WState* __restrict__ st) {
    extern __shared__ __align__(64) unsigned char wsm[];
    if (st->done) return;
    wide_update_mfma_body<D, true, FULL>(st, wsm);
}

// The update for shapes beyond one block's LDS (wide_tiled): the tiled scan,
// and each point's fixed-point coordinates and count added straight into the
// block's own row of partials in device memory (integer atomics of the
// block's threads only; the row is cleared first, and the next kernel,
// wide_reduce, reads it).  q = rint(x 2^F) is the bit pattern of fxp_bits
// less FXP_MAGIC_BITS, so the row holds the sums of q themselves.  TRACK as
// in wide_update_body.
template <int D, bool TRACK>
__device__ __forceinline__ void wide_update_tiled_body(WState* __restrict__ st,
                                                       unsigned char* wsm) {
    using S = WShape<D>;
    constexpr int KT = WTile<D>::KT;
    const int tid = threadIdx.x;
    const int d = st->d, K = st->K, nacc = K * (d + 1);
    float* cm = reinterpret_cast<float*>(wsm);
    float* hh = cm + (size_t)KT * S::DS;
    float* amax = hh + ((KT + 3) & ~3);
    int* q0 = reinterpret_cast<int*>(amax + 36);
    int* wq = q0 + (tid >> 6) * WQCAP;
    double* sw = reinterpret_cast<double*>(q0 + NW * WQCAP);
    const double fscale = fxp_scale(data_exponent(st->absmax_bits));
    unsigned long long* row = st->part + (size_t)blockIdx.x * nacc;
    for (int i = tid; i < nacc; i += WBLOCK) row[i] = 0ull;
    for (int i = tid; i <= WD_MAX; i += WBLOCK) amax[i] = st->amax[i];
    wait_mem();  // the cleared row is in L2 before any thread adds to it
    __syncthreads();
    double jl = 0.0;
    int32_t* __restrict__ track = st->track;
    uint32_t nchg = 0;
    wide_points_tiled<D>(st, cm, hh, amax, K, d, wq,
                         [&](const float (&xr)[D], int64_t i, int k, float dist) {
        jl += (double)dist;
        if constexpr (TRACK) {
            if (track[i] != k) {
                track[i] = k;
                ++nchg;
            }
        }
        unsigned long long* a = row + k;
#pragma unroll
        for (int j = 0; j < D; ++j) {
            if (j < d)
                __hip_atomic_fetch_add(&a[j * K], fxp_bits(xr[j], fscale) - FXP_MAGIC_BITS,
                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        }
        __hip_atomic_fetch_add(&a[d * K], 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    });
    if constexpr (TRACK) {
        nchg = wave_sum_u32(nchg);
        // per-wave counts in the first word of each wave's (drained) queue
        if ((tid & 63) == 0) q0[(tid >> 6) * WQCAP] = (int)nchg;
        __syncthreads();
        if (tid == 0) {
            unsigned long long chg = 0ull;
#pragma unroll
            for (int v = 0; v < NW; ++v) chg += (uint32_t)q0[v * WQCAP];
            if (chg)
                __hip_atomic_fetch_add(&row[d * K], chg << 32, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_WORKGROUP);
        }
    }
    const double jb = block_sum(jl, sw);
    if (tid == 0) st->jpart[blockIdx.x] = jb;
}

template <int D>
__global__ __launch_bounds__(WBLOCK) void wide_update_tiled(WState* __restrict__ st) {
    extern __shared__ __align__(16) unsigned char wsm[];
    if (st->done) return;
    wide_update_tiled_body<D, false>(st, wsm);
}

template <int D>
__global__ __launch_bounds__(WBLOCK) void wide_update_tiled_track(WState* __restrict__ st) {
    extern __shared__ __align__(16) unsigned char wsm[];
    if (st->done) return;
    wide_update_tiled_body<D, true>(st, wsm);
}

// Totals of the partial rows, then (last block) the float64 mean step.
// Grid: x = tiles of WBLOCK slots, y = chunks of WCHUNK rows.
__global__ __launch_bounds__(WBLOCK) void wide_reduce(WState* __restrict__ st) {
    extern __shared__ __align__(16) unsigned char wsm[];
    __shared__ double sw[64];
    __shared__ uint32_t sred[NW * (WD_MAX + 1)];
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
            i128 s = {0ull, 0ll};
#pragma unroll
            for (int u = 0; u < WCHUNK; ++u) i128_add(s, i128_of((long long)v[u]));
            // limbs: s = l1 2^32 + l0, 0 <= l0 < 2^32, |l1| < 2^36 (|s| < 2^68)
            const unsigned long long l0 = s.lo & 0xffffffffull;
            const long long l1 = (long long)(((unsigned long long)s.hi << 32) | (s.lo >> 32));
            if (l0) (void)__hip_atomic_fetch_add(&tot[i], l0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (l1)
                (void)__hip_atomic_fetch_add(&tot[nacc + i], (unsigned long long)l1, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT);
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

    // ---- last block: the mean step from the totals (device-coherent loads)
    // and the key tables of the new float32 centres, from the values the
    // threads hold (the arithmetic of key_tables, in its order).  A load
    // waits for every store issued before it, so each batch's loads go out
    // before the previous batch's stores, and the totals are cleared for
    // the next update at the end.
    // a total from its two limbs: l1 2^32 + l0
    auto limbs = [](unsigned long long l0, unsigned long long hi) {
        const long long l1 = (long long)hi;
        i128 v = {(unsigned long long)l1 << 32, l1 >> 32};
        i128_add(v, i128{l0, 0ll});
        return v;
    };
    double* se = reinterpret_cast<double*>(wsm);
    const int xe = data_exponent(st->absmax_bits);
    const int DS = wide_stride(wide_width(d));
    double* mu64 = st->mu64;
    float* mu32 = st->mu32;
    float* hh = st->hh;
    const int w = tid >> 6;
    int emp = 0;
    long long chg = 0;
    uint32_t cmx = 0;
    // every wave runs the same number of passes (the per-coordinate wave
    // maxima need all its lanes); lanes past K hold zeros
    for (int k0 = 0; k0 < K; k0 += WBLOCK) {
        const int k = k0 + tid;
        const bool in = k < K;
        // slots [j * K + k], j = d the count (low 32 bits; cluster 0's
        // carries the changed labels above them, see wide_update_body); the
        // limbs and the old centre go out in batches of 8 coordinates, one
        // round trip each
        constexpr int BT = 8;
        unsigned long long lo[BT], hi[BT];
        double od[BT];
        auto load_batch = [&](int j0) {
#pragma unroll
            for (int u = 0; u < BT; ++u) {
                lo[u] = 0ull;
                hi[u] = 0ull;
                od[u] = 0.0;
                if (in && j0 + u < d) {
                    lo[u] = gld_agent(&tot[(j0 + u) * K + k]);
                    hi[u] = gld_agent(&tot[nacc + (j0 + u) * K + k]);
                    od[u] = gld(&mu64[k * d + j0 + u]);
                }
            }
        };
        unsigned long long cl0 = 0ull, chi = 0ull;
        if (in) {
            cl0 = gld_agent(&tot[d * K + k]);
            chi = gld_agent(&tot[nacc + d * K + k]);
        }
        load_batch(0);
        const unsigned long long ct = limbs(cl0, chi).lo;
        const unsigned long long cnt = ct & 0xffffffffull;
        if (k == 0) chg = (long long)(ct >> 32);
        double e = 0.0, q = 0.0;
        for (int j0 = 0; j0 < d; j0 += BT) {
            double nv[BT];
#pragma unroll
            for (int u = 0; u < BT; ++u) {
                const int j = j0 + u;
                nv[u] = 0.0;
                if (j < d) {
                    const double v = cnt ? fxp_mean(limbs(lo[u], hi[u]), xe, cnt) : od[u];
                    const double sh = v - od[u];
                    e = fma(sh, sh, e);
                    nv[u] = v;
                    const float m = (float)v;
                    q = fma((double)m, (double)m, q);
                    const uint32_t bm = wave_max(__float_as_uint(m) & 0x7fffffffu);
                    if ((tid & 63) == 0) {
                        uint32_t& r = sred[w * (WD_MAX + 1) + j];
                        r = k0 == 0 || bm > r ? bm : r;
                    }
                }
            }
            if (j0 + BT < d) load_batch(j0 + BT);
#pragma unroll
            for (int u = 0; u < BT; ++u) {
                if (in && j0 + u < d) {
                    gst(&mu64[k * d + j0 + u], nv[u]);
                    gst(&mu32[k * DS + j0 + u], (float)nv[u]);
                }
            }
        }
        if (in) {
            se[k] = e;
            emp += cnt == 0ull;
            const float c = (float)q;
            gst(&hh[k], -0.5f * c);
            cmx = __float_as_uint(c) > cmx ? __float_as_uint(c) : cmx;
        }
    }
    for (int k = K + tid; k < wide_kpad(K); k += WBLOCK) gst(&hh[k], -0x1p127f);
    if (emp) atomicAdd(&sempty, emp);
    cmx = wave_max(cmx);
    if ((tid & 63) == 0) sred[w * (WD_MAX + 1) + WD_MAX] = cmx;
    __syncthreads();
    if (tid <= WD_MAX && (tid < d || tid == WD_MAX)) {
        uint32_t r = 0;
        for (int v = 0; v < NW; ++v) r = sred[v * (WD_MAX + 1) + tid] > r ? sred[v * (WD_MAX + 1) + tid] : r;
        st->amax[tid] = __uint_as_float(r);
    }
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
        int done = (E < st->tol || t + 1 >= st->max_iter) ? 1 : 0;
        if (st->track) {
            // the paper's other criterion: no indicator changed
            if (t < st->hist_cap) st->C_hist[t] = chg;
            st->changed = chg;
            if (chg == 0) done = 1;
        }
        st->done = done;
        st_agent(&st->ticket, 0u);
    }
    // the totals, zero for the next update
    for (int i = tid; i < 2 * nacc; i += WBLOCK) gst_agent(&tot[i], 0ull);
}

// Reassignment only: labels and the objective at the current centres.
template <int D>
__global__ __launch_bounds__(WBLOCK) void wide_label(WState* __restrict__ st,
                                                     int32_t* __restrict__ labels) {
    extern __shared__ __align__(16) unsigned char wsm[];
    __shared__ double sw[64];
    __shared__ int sflag;
    using S = WShape<D>;
    const int tid = threadIdx.x;
    const int d = st->d, K = st->K;
    const int kp = wide_kpad(K);
    float* cm = reinterpret_cast<float*>(wsm);
    float* hh = cm + (size_t)kp * S::DS;
    float* amax = hh + ((kp + 3) & ~3);
    int* wq = reinterpret_cast<int*>(amax + 36) + (tid >> 6) * WQCAP;
    stage_tables<D>(st, K, cm, hh, amax);
    __syncthreads();
    double jl = 0.0;
    wide_points<D>(st, cm, hh, amax, K, d, wq,
                   [&](const float (&)[D], int64_t i, int k, float dist) {
        jl += (double)dist;
        if (labels) labels[i] = k;
    });
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
    const double* jp = st->jpart;
    const double J = ordered_sum(nb, [&](int b) { return ld_agent(&jp[b]); }, sw);
    if (tid == 0) {
        st->J = J;
        st_agent(&st->ticket, 0u);
    }
}

// Reassignment only, for shapes beyond one block's LDS (the tiled scan).
template <int D>
__global__ __launch_bounds__(WBLOCK) void wide_label_tiled(WState* __restrict__ st,
                                                           int32_t* __restrict__ labels) {
    extern __shared__ __align__(16) unsigned char wsm[];
    __shared__ double sw[64];
    __shared__ int sflag;
    using S = WShape<D>;
    constexpr int KT = WTile<D>::KT;
    const int tid = threadIdx.x;
    const int d = st->d, K = st->K;
    float* cm = reinterpret_cast<float*>(wsm);
    float* hh = cm + (size_t)KT * S::DS;
    float* amax = hh + ((KT + 3) & ~3);
    int* wq = reinterpret_cast<int*>(amax + 36) + (tid >> 6) * WQCAP;
    for (int i = tid; i <= WD_MAX; i += WBLOCK) amax[i] = st->amax[i];
    __syncthreads();
    double jl = 0.0;
    wide_points_tiled<D>(st, cm, hh, amax, K, d, wq,
                         [&](const float (&)[D], int64_t i, int k, float dist) {
        jl += (double)dist;
        if (labels) labels[i] = k;
    });
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
    const double* jp = st->jpart;
    const double J = ordered_sum(nb, [&](int b) { return ld_agent(&jp[b]); }, sw);
    if (tid == 0) {
        st->J = J;
        st_agent(&st->ticket, 0u);
    }
}

// Reassignment only with the matrix-core keys.
template <int D, bool FULL>
__global__ __launch_bounds__(WBLOCK) __attribute__((amdgpu_waves_per_eu(1, D >= 12 ? 2 : 4))) void wide_label_mfma(WState* __restrict__ st,
                                                          int32_t* __restrict__ labels) {
    extern __shared__ __align__(64) unsigned char wsm[];
    __shared__ double sw[64];
    __shared__ int sflag;
    using M = WMfma<D>;
    const int tid = threadIdx.x;
    const int d = FULL ? D : st->d, K = st->K;
    const int KT = (K + 31) / 32;
    u32x4* As = reinterpret_cast<u32x4*>(wsm);
    float* Cs = reinterpret_cast<float*>(As + (size_t)KT * M::S * 64);
    float* amax = Cs + KT * 32;
    int* wq = reinterpret_cast<int*>(amax + 36) + (tid >> 6) * WQCAP;
    int* wq2 = reinterpret_cast<int*>(amax + 36) + (NW + (tid >> 6)) * WQCAP;
    for (int i = tid; i <= WD_MAX; i += WBLOCK) amax[i] = st->amax[i];
    __syncthreads();
    int e = 0;
    const bool mok = wide_mfma_scale(data_exponent(st->absmax_bits), amax, d, e);
    if (mok) stage_mfma<D>(st, K, d, e, As, Cs);
    __syncthreads();
    double jl = 0.0;
    wide_points_mfma<D, WMFMA_PL>(st, As, Cs, amax, K, d, e, mok, wq, wq2,
                        [&](const float (&)[D], int64_t i, int k, float dist) {
        jl += (double)dist;
        if (labels) labels[i] = k;
    });
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
    const double* jp = st->jpart;
    const double J = ordered_sum(nb, [&](int b) { return ld_agent(&jp[b]); }, sw);
    if (tid == 0) {
        st->J = J;
        st_agent(&st->ticket, 0u);
    }
}

// The matrix-core kernels exist for widths 8, 12 and 16.
// The matrix-core kernels exist for widths 8, 12 and 16, each for d equal to
// the width (FULL) and for narrower d.
#define KM_WIDE_MFMA_DISPATCH(KERN, d, grid, lds, s, ...)                                      \
    switch (2 * wide_width(d) + (wide_width(d) == (d) ? 1 : 0)) {                             \
        case 16: hipLaunchKernelGGL((KERN<8, false>), dim3(grid), dim3(WBLOCK), lds, s, __VA_ARGS__); break;  \
        case 17: hipLaunchKernelGGL((KERN<8, true>), dim3(grid), dim3(WBLOCK), lds, s, __VA_ARGS__); break;   \
        case 24: hipLaunchKernelGGL((KERN<12, false>), dim3(grid), dim3(WBLOCK), lds, s, __VA_ARGS__); break; \
        case 25: hipLaunchKernelGGL((KERN<12, true>), dim3(grid), dim3(WBLOCK), lds, s, __VA_ARGS__); break;  \
        case 32: hipLaunchKernelGGL((KERN<16, false>), dim3(grid), dim3(WBLOCK), lds, s, __VA_ARGS__); break; \
        case 33: hipLaunchKernelGGL((KERN<16, true>), dim3(grid), dim3(WBLOCK), lds, s, __VA_ARGS__); break;  \
        default: return hipErrorInvalidValue;                                                \
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

hipError_t launch_wide_update(WState* st, int d, int K, bool track, bool mfma, int grid,
                              hipStream_t s) {
    if (grid < 1 || grid > WMAX_GRID || d < 1 || d > WD_MAX || K < 1 || K > WK_MAX)
        return hipErrorInvalidValue;
    if (mfma) {
        if (!wide_mfma_fits(d, K)) return hipErrorInvalidValue;
        const size_t lds = wide_mfma_lds_bytes(d, K);
        if (track) {
            KM_WIDE_MFMA_DISPATCH(wide_update_mfma_track, d, grid, lds, s, st)
        } else {
            KM_WIDE_MFMA_DISPATCH(wide_update_mfma, d, grid, lds, s, st)
        }
    } else if (wide_tiled(d, K)) {
        const size_t lds = wide_tiled_lds_bytes(d);
        if (track) {
            KM_WIDE_DISPATCH(wide_update_tiled_track, d, grid, lds, s, st)
        } else {
            KM_WIDE_DISPATCH(wide_update_tiled, d, grid, lds, s, st)
        }
    } else {
        const size_t lds = wide_lds_bytes(d, K);
        if (track) {
            KM_WIDE_DISPATCH(wide_update_track, d, grid, lds, s, st)
        } else {
            KM_WIDE_DISPATCH(wide_update, d, grid, lds, s, st)
        }
    }
    return hipGetLastError();
}

hipError_t launch_wide_reduce(WState* st, int d, int K, int grid_update, hipStream_t s) {
    const int nacc = K * (d + 1);
    // LDS of the last block: one float64 per centre
    const size_t lds = (size_t)K * 8;
    if (d < 1 || d > WD_MAX || K < 1 || K > WK_MAX || grid_update < 1 ||
        grid_update > WMAX_GRID || lds > (size_t)WLDS_MAX)
        return hipErrorInvalidValue;
    const dim3 grid((nacc + WBLOCK - 1) / WBLOCK, (grid_update + WCHUNK - 1) / WCHUNK);
    hipLaunchKernelGGL(wide_reduce, grid, dim3(WBLOCK), lds, s, st);
    return hipGetLastError();
}

hipError_t launch_wide_label(WState* st, int32_t* labels, int d, int K, bool mfma, int grid,
                             hipStream_t s) {
    if (grid < 1 || grid > WMAX_GRID || d < 1 || d > WD_MAX || K < 1 || K > WK_MAX)
        return hipErrorInvalidValue;
    if (mfma) {
        if (!wide_mfma_fits(d, K)) return hipErrorInvalidValue;
        const size_t lds = wide_mfma_table_bytes(d, K);
        KM_WIDE_MFMA_DISPATCH(wide_label_mfma, d, grid, lds, s, st, labels)
    } else if (wide_tiled(d, K)) {
        const size_t lds = wide_tiled_lds_bytes(d);
        KM_WIDE_DISPATCH(wide_label_tiled, d, grid, lds, s, st, labels)
    } else {
        const size_t lds = wide_table_bytes(d, K);
        KM_WIDE_DISPATCH(wide_label, d, grid, lds, s, st, labels)
    }
    return hipGetLastError();
}

#define KM_WIDE_OCC(KERN)                                                                      \
    [](int w, size_t lds) {                                                                    \
        int n = 0;                                                                             \
        hipError_t e = hipErrorInvalidValue;                                                   \
        switch (w) {                                                                           \
            case 1: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, reinterpret_cast<const void*>(KERN<1>), WBLOCK, lds); break;   \
            case 2: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, reinterpret_cast<const void*>(KERN<2>), WBLOCK, lds); break;   \
            case 3: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, reinterpret_cast<const void*>(KERN<3>), WBLOCK, lds); break;   \
            case 4: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, reinterpret_cast<const void*>(KERN<4>), WBLOCK, lds); break;   \
            case 6: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, reinterpret_cast<const void*>(KERN<6>), WBLOCK, lds); break;   \
            case 8: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, reinterpret_cast<const void*>(KERN<8>), WBLOCK, lds); break;   \
            case 12: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, reinterpret_cast<const void*>(KERN<12>), WBLOCK, lds); break; \
            case 16: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, reinterpret_cast<const void*>(KERN<16>), WBLOCK, lds); break; \
            case 24: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, reinterpret_cast<const void*>(KERN<24>), WBLOCK, lds); break; \
            case 32: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, reinterpret_cast<const void*>(KERN<32>), WBLOCK, lds); break; \
            default: break;                                                                    \
        }                                                                                      \
        return e == hipSuccess ? n : 0;                                                        \
    }

int wide_blocks_per_cu(int d, int K, bool mfma) {
    const int w = wide_width(d);
    if (mfma) {
        if (!wide_mfma_fits(d, K)) return 0;
        const size_t lds = wide_mfma_lds_bytes(d, K);
        int n = 0;
        hipError_t e = hipErrorInvalidValue;
        switch (w) {
            case 8: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, reinterpret_cast<const void*>(wide_update_mfma<8, false>), WBLOCK, lds); break;
            case 12: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, reinterpret_cast<const void*>(wide_update_mfma<12, false>), WBLOCK, lds); break;
            case 16: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, reinterpret_cast<const void*>(wide_update_mfma<16, false>), WBLOCK, lds); break;
            default: break;
        }
        return e == hipSuccess ? n : 0;
    }
    if (wide_tiled(d, K)) return KM_WIDE_OCC(wide_update_tiled)(w, wide_tiled_lds_bytes(d));
    return KM_WIDE_OCC(wide_update)(w, wide_lds_bytes(d, K));
}

}  // namespace km
