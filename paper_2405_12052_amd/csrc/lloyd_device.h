// lloyd_device.h -- device helpers shared by the single-fit kernels
// (lloyd_kernels.hip) and the batched kernel (batched_kernels.hip): loading
// points, the certified reassignment scan, the direct-form re-scan and its
// per-wave queue, and the centre tables.  Internal to libkmeans_mi355x.so.
//
// Reassignment (nearest4): the scan over centres uses the expanded form
//   s_k = |m_k|^2 - 2 m_k . x      (= |x - m_k|^2 - |x|^2, same argmin)
// three fused multiply-adds per centre, and keeps the smallest and second
// smallest s over triples of centres (min3 / med3) plus the triple of the
// smallest.  A rounding bound b(x) on every s_k certifies the winner: when
// the two smallest differ by more than b(x), the first index attaining the
// smallest s is the exact argmin of the squared distance to the float32
// centres.  Otherwise (points within b(x) of a tie) the point is re-scanned
// with the direct form (x0-m0)^2 + (x1-m1)^2 [+ (x2-m2)^2] evaluated in
// float64, first index of the minimum.  The distance reported (objective) is
// always the float32 direct form to the chosen centre.
#pragma once

#include "km_internal.h"

#include <math.h>

namespace km {

constexpr int NW = BLOCK / 64;  // waves per block

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v) {
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

// Data that blocks of one kernel hand to each other (partial sums, tickets'
// payloads) travel as device-coherent stores and loads: relaxed atomics at
// device scope, which write through and read past the per-XCD L2 caches.
// The writer waits for its stores to complete before it signals (wait_mem),
// and the reader loads after it has seen the signal.  This replaces
// device-scope fences, each of which writes back and invalidates a whole L2.
template <typename T>
__device__ __forceinline__ T ld_agent(const T* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <typename T>
__device__ __forceinline__ void st_agent(T* p, T v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Wait until this thread's memory operations have completed.
__device__ __forceinline__ void wait_mem() { __builtin_amdgcn_s_waitcnt(0); }

// Exponent of the data's magnitude: ilogb(max|x|), so max|x| < 2^(xe+1);
// -1 for all-zero data.
__device__ __forceinline__ int data_exponent(uint32_t absmax_bits) {
    const float a = __uint_as_float(absmax_bits);
    return a > 0.0f ? ilogbf(a) : -1;
}

// ---------------------------------------------------------------------------
// Per-cluster sums in fixed point (the numerators of the paper's mean step).
//
// Every coordinate enters as the integer q = rint(x 2^F), F = FXP_BITS - 1 -
// xe, so |q| < 2^44 (x 2^F is a float32 scaled by a power of two: exact, and
// an integer once it reaches 2^23).  Integer sums are exact in any order, so
// the means do not depend on the schedule.  One int64 slot of a block never
// receives more than FXP_BLOCK_POINTS = 2^19 points between two readings
// (|sum| < 2^63); sums over blocks are carried in 128 bits.  The rounding
// moves each mean coordinate by at most 2^(xe-44) <= max|x| 2^-44 from the
// exact mean, below the 1e-5 centre tolerance of any cluster (a cluster at
// the origin included) while xe <= 27: fits refuse data with max|x| >= 2^28
// (FXP_RANGE_BITS) rather than return means that could miss it.
//
// The conversion is one float64 FMA: x 2^F + 1.5 2^52 rounds to an integer
// (the spacing of doubles in [2^52, 2^53) is 1) whose bit pattern is
// FXP_MAGIC_BITS + q for |q| < 2^51.  The accumulators add those bit patterns
// as 64-bit integers; a slot that received n points is corrected by
// subtracting n FXP_MAGIC_BITS (mod 2^64) when it is read.
// (FXP_BITS, FXP_BLOCK_POINTS and FXP_RANGE_BITS are in km_internal.h.)
constexpr double FXP_MAGIC = 0x1.8p52;
constexpr unsigned long long FXP_MAGIC_BITS = 0x4338000000000000ull;

// 2^F for data of exponent xe.
__device__ __forceinline__ double fxp_scale(int xe) { return ldexp(1.0, FXP_BITS - 1 - xe); }

// FXP_MAGIC_BITS + rint(x 2^F) (mod 2^64), scale = 2^F.
__device__ __forceinline__ unsigned long long fxp_bits(float x, double scale) {
    return (unsigned long long)__double_as_longlong(fma((double)x, scale, FXP_MAGIC));
}

// A signed 128-bit integer: value = hi 2^64 + lo.
struct i128 {
    unsigned long long lo;
    long long hi;
};

__device__ __forceinline__ i128 i128_of(long long v) {
    return i128{(unsigned long long)v, v >> 63};
}

__device__ __forceinline__ void i128_add(i128& a, const i128& b) {
    const unsigned long long lo = a.lo + b.lo;
    a.hi += b.hi + (lo < a.lo ? 1 : 0);
    a.lo = lo;
}

// The double nearest to v (|v| < 2^116): hi 2^64 and the upper 32 bits of
// lo add exactly (at most 53 significant bits), the lower 32 bits are added
// with the one rounding.
__device__ __forceinline__ double i128_to_double(const i128& v) {
    const double a = ldexp((double)v.hi, 64);
    const double b = ldexp((double)(v.lo >> 32), 32);
    const double c = (double)(v.lo & 0xffffffffull);
    return (a + b) + c;
}

// Mean of a cluster from the 128-bit sum of its q and its count n > 0:
// (S 2^-F) / n in float64.
__device__ __forceinline__ double fxp_mean(const i128& S, int xe, unsigned long long n) {
    return ldexp(i128_to_double(S), -(FXP_BITS - 1 - xe)) / (double)n;
}

// Load the 4 consecutive points of group g (coordinates x[j][p]); returns how
// many of them exist (4 except in the last, ragged group).  VEC: the rows are
// 16-byte aligned (128-bit loads).
template <int D, bool VEC>
__device__ __forceinline__ int load_group(const float* __restrict__ X, int64_t ld,
                                          int64_t N, int64_t g, float (&x)[D][4]) {
    // global-address-space loads: flat loads also count against the LDS
    // counter, so each wait for the points would wait for the block's
    // outstanding LDS atomics too
    typedef const float __attribute__((address_space(1)))* gfp;
    typedef float f32x4 __attribute__((ext_vector_type(4)));
    typedef const f32x4 __attribute__((address_space(1)))* gf4p;
    const gfp Xg = (gfp)X;
    const int64_t i0 = g * 4;
    if (VEC && i0 + 4 <= N) {
#pragma unroll
        for (int j = 0; j < D; ++j) {
            const f32x4 v = *(gf4p)(Xg + j * ld + i0);
            x[j][0] = v.x; x[j][1] = v.y; x[j][2] = v.z; x[j][3] = v.w;
        }
        return 4;
    }
    const int n = (int)((N - i0) < 4 ? (N - i0) : 4);
#pragma unroll
    for (int j = 0; j < D; ++j)
#pragma unroll
        for (int p = 0; p < 4; ++p) x[j][p] = p < n ? Xg[j * ld + i0 + p] : 0.0f;
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
// the K centre records padded to whole triples; smu: the float32 centres;
// bnd: the rounding-bound coefficients.  For every point writes ok[p]: the
// winner is certified, and then arg[p] (its index) and best[p] (the
// direct-form squared distance to it).  Points with ok[p] == false need the
// direct-form scan (direct_scan).
//
// Per triple of centres the scan keeps, per point, only the smallest key of
// the triple with the triple's index written into its 5 lowest bits (one
// and-or), the smallest of those (m1) and the second smallest (m2): four
// compare-type instructions per triple.  At the end the winning triple's
// three keys are formed again (bit-identical), giving the exact smallest key
// t1, its first index, and the triple's second smallest t2.  Every key of
// another triple is at least m2 less its index bits (at most 31 units in its
// last place, below 2^-18 |m2|), so the second smallest key over all centres
// is at least min(t2, m2 - 2^-17 |m2|), which the certificate compares with t1.
constexpr uint32_t TRI_BITS = 31u;  // ntri <= 32

// v with its 5 lowest bits replaced by the (wave-uniform) index g: one
// bitfield insert (the mask is an inline constant, g a scalar register).
__device__ __forceinline__ float with_index(float v, int g) {
    float r;
    asm("v_bfi_b32 %0, 31, %1, %2" : "=v"(r) : "s"(g), "v"(v));
    return r;
}

template <int D>
__device__ __forceinline__ void nearest4(const float4* __restrict__ scand,
                                         const float4* __restrict__ smu, int K,
                                         float4 bnd, float ninf, const float (&x)[D][4],
                                         float (&best)[4], int (&arg)[4], bool (&ok)[4]) {
    float m1[4], m2[4];
#pragma unroll
    for (int p = 0; p < 4; ++p) { m1[p] = INFINITY; m2[p] = INFINITY; }
    // whole triples; a last triple with one or two real centres (K not a
    // multiple of 3) is folded on its own below, without its pads' keys
    const int nfull = K / 3;
    for (int g = 0; g < nfull; ++g) {
        const float4 r0 = scand[3 * g], r1 = scand[3 * g + 1], r2 = scand[3 * g + 2];
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            const float x2 = D == 3 ? x[D - 1][p] : 0.0f;
            const float s0 = expanded_key<D>(x[0][p], x[1][p], x2, r0);
            const float s1 = expanded_key<D>(x[0][p], x[1][p], x2, r1);
            const float s2 = expanded_key<D>(x[0][p], x[1][p], x2, r2);
            const float g1 = fminf(fminf(s0, s1), s2);
            const float gp = with_index(g1, g);
            m2[p] = __builtin_amdgcn_fmed3f(m1[p], gp, m2[p]);
            m1[p] = min2(m1[p], gp, ninf);
        }
    }
    const int rem = K - 3 * nfull;  // the same in every lane
    if (rem != 0) {
        const float4 r0 = scand[3 * nfull], r1 = scand[3 * nfull + 1];
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            const float x2 = D == 3 ? x[D - 1][p] : 0.0f;
            float g1 = expanded_key<D>(x[0][p], x[1][p], x2, r0);
            if (rem == 2) g1 = min2(g1, expanded_key<D>(x[0][p], x[1][p], x2, r1), ninf);
            const float gp = with_index(g1, nfull);
            m2[p] = __builtin_amdgcn_fmed3f(m1[p], gp, m2[p]);
            m1[p] = min2(m1[p], gp, ninf);
        }
    }
#pragma unroll
    for (int p = 0; p < 4; ++p) {
        const float x0 = x[0][p], x1 = x[1][p], x2 = D == 3 ? x[D - 1][p] : 0.0f;
        // the winning triple's keys again: exact smallest, its first index,
        // and the triple's second smallest
        const int k0 = 3 * (int)(__float_as_uint(m1[p]) & TRI_BITS);
        const float s0 = expanded_key<D>(x0, x1, x2, scand[k0]);
        const float s1 = expanded_key<D>(x0, x1, x2, scand[k0 + 1]);
        const float s2 = expanded_key<D>(x0, x1, x2, scand[k0 + 2]);
        const float t1 = fminf(fminf(s0, s1), s2);
        const float t2 = __builtin_amdgcn_fmed3f(s0, s1, s2);
        const int k = s0 == t1 ? k0 : (s1 == t1 ? k0 + 1 : k0 + 2);
        // rounding bound of the keys of this point
        float b = fmaf(bnd.y, fabsf(x0), bnd.x);
        b = fmaf(bnd.z, fabsf(x1), b);
        if constexpr (D == 3) b = fmaf(bnd.w, fabsf(x2), b);
        // every other triple's smallest key is at least its packed minimum
        // less the index bits (31 units in the last place, below 2^-18 of it),
        // and that packed minimum is at least m2: so at least
        // m2 - 2^-17 |m2| (p - 2^-18 |p| grows with p).  With a single
        // triple m2 = +inf, the difference is a NaN and fminf returns t2.
        const float sec = fminf(t2, m2[p] - ldexpf(fabsf(m2[p]), -17));
        ok[p] = sec - t1 > b && k < K;
        arg[p] = ok[p] ? k : 0;
        best[p] = direct_dist<D>(x0, x1, x2, smu[arg[p]]);
    }
}

// load_group with the alignment known only at run time (uniform branch).
template <int D>
__device__ __forceinline__ int load_group_rt(bool vec, const float* __restrict__ X, int64_t ld,
                                             int64_t N, int64_t g, float (&x)[D][4]) {
    return vec ? load_group<D, true>(X, ld, N, g, x) : load_group<D, false>(X, ld, N, g, x);
}

// Squared distance evaluated in float64: each coordinate's difference,
// square and the running sum rounded to float64, left to right (no fused
// operations).
template <int D>
__device__ __forceinline__ double direct_dist64(float x0, float x1, float x2, float4 c) {
    // plain operators under contract(off): the _rn helpers' own bodies may be
    // contracted once inlined
#pragma clang fp contract(off)
    const double d0 = (double)x0 - (double)c.x;
    const double d1 = (double)x1 - (double)c.y;
    double s = d0 * d0 + d1 * d1;
    if constexpr (D == 3) {
        const double d2 = (double)x2 - (double)c.z;
        s = s + d2 * d2;
    }
    return s;
}

// Near-tie scan of one point over all K centres: first index of the minimum
// of the float64 squared distance (a certified winner is also that minimum,
// its margin being far above float64 rounding, so labels do not depend on
// which points were certified).  bd: the float32 direct-form distance to
// the chosen centre (the objective's term).
template <int D>
__device__ __forceinline__ void direct_scan(const float4* __restrict__ smu, int K, float x0,
                                            float x1, float x2, float& bd, int& bk) {
    double best = INFINITY;
    bk = 0;
    // rare path: kept rolled, so that its float64 registers do not set the
    // register budget of the kernels that inline it
#pragma unroll 1
    for (int q = 0; q < K; ++q) {
        const double dq = direct_dist64<D>(x0, x1, x2, smu[q]);
        if (dq < best) { best = dq; bk = q; }
    }
    bd = direct_dist<D>(x0, x1, x2, smu[bk]);
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
                                              float4 bnd, float ninf,
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
        nearest4<D>(scand, smu, K, bnd, ninf, x, best, arg, ok);
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
// whole triples with {0, 0, 0, 2^127}, and the bound coefficients
//   b(x) = 2^-21 (1 + 2^-10) (Cmax + 2 sum_j A_j |x_j|) + 2^-46 xmax sum_j |x_j|,
//   Cmax = max_k c_k, A_j = max_k |m_kj|, xmax = max |x| over the data
// (xmax_bits).  The first part is twice the rounding bound of a key
// (gamma_4 (Cmax + 2 sum_j A_j |x_j|), gamma_4 = 4u / (1 - 4u), u = 2^-24: the
// rounding of c_k and of three FMAs), with 2^-10 to spare for the float32
// evaluation of the bound and of the gap.  The second covers the float64 evaluation of the direct form
// used for near-ties: two distances D err by at most 2 (d + 2) 2^-53 D, D <=
// |x|^2 + |key|, below 2^-49 (|x|^2 + |key|); the key part lies far inside
// the first term and |x|^2 <= xmax sum_j |x_j|.  A certified winner is
// therefore also the first-index minimum of the float64 direct form.
// Written to cand[0 .. npad) (npad >= 3*ceil(K/3): records past K are pads)
// and *bnd (global or LDS).  Called by one whole block; sc and sa are LDS
// scratch of npad and 3*npad floats.
__device__ inline void prep_centres(const float4* m32, int K, int npad, float4* cand, float4* bnd,
                                    float* sc, float* sa, uint32_t xmax_bits) {
    const int tid = threadIdx.x;
    if (tid < npad) {
        // pads: a finite key far above any real one (their keys carry index
        // bits in the scan, which would turn an infinity into a NaN)
        float4 r = make_float4(0.f, 0.f, 0.f, 0x1p127f);
        float c = 0.f, a0 = 0.f, a1 = 0.f, a2 = 0.f;
        if (tid < K) {
#pragma clang fp contract(off)
            const float4 m = m32[tid];
            const double q = ((double)m.x * (double)m.x + (double)m.y * (double)m.y) +
                             (double)m.z * (double)m.z;
            c = (float)q;
            r = make_float4(-2.0f * m.x, -2.0f * m.y, -2.0f * m.z, c);
            a0 = fabsf(m.x); a1 = fabsf(m.y); a2 = fabsf(m.z);
        }
        cand[tid] = r;
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
        const float e = 0x1p-46f * __uint_as_float(xmax_bits);
        const float f = 0x1.004p-21f;
        *bnd = make_float4(cm * f, am0 * (2.0f * f) + e, am1 * (2.0f * f) + e,
                           am2 * (2.0f * f) + e);
    }
    __syncthreads();
}

// Stage the centre tables of the current iteration in LDS: all KPAD records
// (pads included, for the matrix-core scan's re-keying of a quad) and the K
// float32 centres.
__device__ __forceinline__ void stage_centres(const State* __restrict__ st, int K, float4* scand,
                                              float4* smu) {
    for (int i = threadIdx.x; i < KPAD; i += BLOCK) scand[i] = st->cand[i];
    for (int i = threadIdx.x; i < K; i += BLOCK) smu[i] = st->mu32[i];
}

}  // namespace km
