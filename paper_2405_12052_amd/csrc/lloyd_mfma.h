// lloyd_mfma.h -- reassignment scan with the expanded-form keys computed on
// the matrix cores (FP32 MFMA 32x32x2), the argmin on the VALU.
//
// The keys s_k = |m_k|^2 - 2 m_k . x of 32 points against 32 centres are
// one 32x32 product with inner dimension 4:
//   [-2 m_k0, -2 m_k1, -2 m_k2, |m_k|^2] . [x0, x1, x2, 1]
// taken as two chained v_mfma_f32_32x32x2_f32 (inner pairs (x0, x1) and
// (x2, 1)).  Operand layout of that instruction (lane l, c = l % 32,
// h = l / 32): A[m][k] comes from lane m + 32k, B[k][n] from lane n + 32k, and
// register r of the result holds row 8(r/4) + 4h + r%4, column c.  With rows
// = centres and columns = points, lane (c, h) receives 16 keys of point c per
// tile of 32 centres: centres {0-3, 8-11, 16-19, 24-27} + 4h.  K <= 64 takes
// KT = 1 or 2 centre tiles; centres past K get the key 2^127 (coefficients 0,
// constant 2^127): finite, so that packing a group number into it cannot make
// a NaN, and above any key of finite data that matters.
//
// A wave takes 128 points at a time: lane (c, h) loads coordinate h of points
// 4c .. 4c+3 with one 128-bit load (and coordinate 2 of the same points), so
// "tile" j in 0..3 is the 32 points {4c + j}.  Per tile each lane folds its
// keys into: W, the smallest group minimum with the group's number packed
// into its 5 low mantissa bits, and L, a lower bound of every other key (the
// second smallest group minimum and the smallest within-group second key;
// the groups are triples of result registers).  The two halves of a point
// are merged across lanes l and l ^ 32; two tiles at a time, so that every
// lane then finishes one point: the winning group's (at most 3) centres are
// re-keyed on the VALU with three FMAs each and the smallest wins.
//
// Certificate.  mag(x) = Cmax + 2 sum_j A_j |x_j| (Cmax, A_j as in the VALU
// scan) bounds every |key|.  A matrix-core key differs from the exact key by
// e_m <= a few 2^-24 mag(x) (4 products and sums of float32 values), packing
// moves a group minimum by at most 2^-18 mag(x) (32 units in its last place),
// and the VALU re-keying errs by e_v <= 3.01 2^-24 mag(x).  With
// L - W > beta = 2^-16 mag(x) >= 2 2^-18 mag(x) + 2 e_m + 2 e_v, every other
// key exceeds the winner's in exact arithmetic, and the re-keying of the
// winning group still orders it correctly, so the winner is the exact argmin
// of the keys of the float32 centres -- the label the VALU scan certifies.
// Points that fail the test go to the same per-wave re-scan queue as in the
// VALU scan.  Labels are therefore identical to the VALU scan's.
//
// Measured on MI355X (N = 2e8, d = 3, K = 64): the VALU instruction count
// drops by a third against the VALU scan, but the FP32 matrix-core
// instructions never execute alongside VALU instructions (the hardware's
// co-execution counter stays at zero), so their 64 cycles per 32x32 tile add
// to the VALU time and an update takes 2.44 ms against 2.00 ms.  The library
// therefore selects this scan only on request (KM_OPT_KEYS = 2).
#pragma once

#include "lloyd_device.h"

namespace km {

typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ f32x16 mfma_key(float a, float b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}

// min(a, b, c), max(a, b) and min(a, b) as single instructions: the keys are
// never signalling NaNs, so the operand quieting that the compiler adds in
// front of its own min/max/med3 for values it cannot prove canonical (packed
// keys) is not needed.
__device__ __forceinline__ float vmin3(float a, float b, float c) {
    float r;
    asm("v_min3_f32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
    return r;
}

__device__ __forceinline__ float vmax(float a, float b) {
    float r;
    asm("v_max_f32 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}

__device__ __forceinline__ float vmin(float a, float b) {
    float r;
    asm("v_min_f32 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}

// Centre of result register r (0..15) of centre tile t for lane half h.
__device__ __forceinline__ int reg_centre(int t, int r, int h) {
    return 32 * t + 8 * (r >> 2) + 4 * h + (r & 3);
}

// One group of keys (a, b, c) into the running (m1, s2, g2m):
//   g1 = min(a, b, c) with the group number `gid` in its 5 low mantissa bits,
//   s2 = second smallest g1 so far, m1 = smallest g1 so far,
//   g2m = smallest within-group second key so far.
// The within-group median is taken first, by the compiler, so that it (not
// the assembly) is the first reader of the matrix-core results and carries
// the wait for them; the assembly takes it as an input and so follows it.
template <uint32_t GID>
__device__ __forceinline__ void fold_group(float a, float b, float c, uint32_t mask, float ninf,
                                           float& m1, float& s2, float& g2m) {
    const float g2 = __builtin_amdgcn_fmed3f(a, b, c);
    float t;
    asm("v_min3_f32 %0, %4, %5, %6\n\t"
        "v_and_or_b32 %0, %0, %7, %8\n\t"
        "v_med3_f32 %1, %2, %1, %0\n\t"
        "v_min_f32 %2, %2, %0"
        : "=&v"(t), "+v"(s2), "+v"(m1)
        : "v"(g2), "v"(a), "v"(b), "v"(c), "s"(mask), "i"(GID));
    g2m = min2(g2m, g2, ninf);
}

// Fold the keys of one tile of points (per lane: KT*16 keys) into (W, L):
// groups are the register triples (0,1,2) .. (12,13,14) of each centre tile
// and the last registers (15) of all tiles.
template <int KT>
__device__ __forceinline__ void fold_keys(const f32x16 (&s)[KT], float ninf, float& W, float& L) {
    const uint32_t mask = ~31u;
    float m1 = INFINITY, s2 = INFINITY, g2m = INFINITY;
    fold_group<0>(s[0][0], s[0][1], s[0][2], mask, ninf, m1, s2, g2m);
    fold_group<1>(s[0][3], s[0][4], s[0][5], mask, ninf, m1, s2, g2m);
    fold_group<2>(s[0][6], s[0][7], s[0][8], mask, ninf, m1, s2, g2m);
    fold_group<3>(s[0][9], s[0][10], s[0][11], mask, ninf, m1, s2, g2m);
    fold_group<4>(s[0][12], s[0][13], s[0][14], mask, ninf, m1, s2, g2m);
    if constexpr (KT == 2) {
        fold_group<5>(s[1][0], s[1][1], s[1][2], mask, ninf, m1, s2, g2m);
        fold_group<6>(s[1][3], s[1][4], s[1][5], mask, ninf, m1, s2, g2m);
        fold_group<7>(s[1][6], s[1][7], s[1][8], mask, ninf, m1, s2, g2m);
        fold_group<8>(s[1][9], s[1][10], s[1][11], mask, ninf, m1, s2, g2m);
        fold_group<9>(s[1][12], s[1][13], s[1][14], mask, ninf, m1, s2, g2m);
        // the pair (15 of tile 0, 15 of tile 1), padded with +inf
        fold_group<10>(s[0][15], s[1][15], INFINITY, mask, ninf, m1, s2, g2m);
    } else {
        fold_group<5>(s[0][15], INFINITY, INFINITY, mask, ninf, m1, s2, g2m);
    }
    W = m1;
    L = vmin(s2, g2m);
}

// The (up to) three centres of group g for lane half h, in increasing order.
template <int KT>
__device__ __forceinline__ void group_centres(uint32_t g, int h, int (&c)[3]) {
    if (g < 5u * KT) {
        const int t = (int)g / 5, r = 3 * ((int)g % 5);
        c[0] = reg_centre(t, r, h);
        c[1] = reg_centre(t, r + 1, h);
        c[2] = reg_centre(t, r + 2, h);
    } else {
        c[0] = reg_centre(0, 15, h);
        c[1] = KT == 2 ? reg_centre(1, 15, h) : c[0];
        c[2] = c[1];
    }
}

// Reassignment of the points of this wave's share of the grid (chunks of 128
// points) with the MFMA keys; same contract as assign_points (sink receives
// every certified point, the others are re-scanned from the per-wave queue).
template <int D, bool VEC, int KT, typename Sink>
__device__ __forceinline__ void assign_points_mfma(const float* __restrict__ X, int64_t ld,
                                                   int64_t N, const float4* __restrict__ scand,
                                                   const float4* __restrict__ smu, int K,
                                                   float4 bnd, float ninf,
                                                   float4* __restrict__ wq, Sink&& sink) {
    const int lane = threadIdx.x & 63;
    const int c = lane & 31, h = lane >> 5;
    const uint64_t below = (1ull << lane) - 1ull;

    // A operands: centre 32t + c, coefficient h of each inner pair
    float a0[KT], a1[KT];
#pragma unroll
    for (int t = 0; t < KT; ++t) {
        const int k = 32 * t + c;
        if (k < K) {
            const float4 r = scand[k];
            a0[t] = h ? r.y : r.x;
            a1[t] = h ? r.w : r.z;
        } else {
            a0[t] = 0.0f;
            a1[t] = h ? 0x1p127f : 0.0f;
        }
    }
    // certificate threshold 2^-16 mag(x) (+ a floor far below any key gap
    // that matters, so that all-zero keys are never certified)
    const float4 bq = make_float4(ldexpf(bnd.x, 4), ldexpf(bnd.y, 4), ldexpf(bnd.z, 4),
                                  ldexpf(bnd.w, 4));
    const f32x16 zero = {};

    int qn = 0;
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

    const int64_t nchunks = (N + 127) / 128;
    for (int64_t ch = (int64_t)blockIdx.x * NW + (threadIdx.x >> 6); ch < nchunks;
         ch += (int64_t)gridDim.x * NW) {
        const int64_t i0 = ch * 128 + 4 * c;   // first of this lane's 4 points
        float xh[4], x2[4];
        if (VEC && i0 + 4 <= N) {
            const float4 v = *reinterpret_cast<const float4*>(X + h * ld + i0);
            xh[0] = v.x; xh[1] = v.y; xh[2] = v.z; xh[3] = v.w;
            if constexpr (D == 3) {
                const float4 u = *reinterpret_cast<const float4*>(X + 2 * ld + i0);
                x2[0] = u.x; x2[1] = u.y; x2[2] = u.z; x2[3] = u.w;
            }
        } else {
#pragma unroll
            for (int p = 0; p < 4; ++p) {
                const bool in = i0 + p < N;
                xh[p] = in ? X[h * ld + i0 + p] : 0.0f;
                if constexpr (D == 3) x2[p] = in ? X[2 * ld + i0 + p] : 0.0f;
            }
        }
        if constexpr (D == 2) {
#pragma unroll
            for (int p = 0; p < 4; ++p) x2[p] = 0.0f;
        }

#pragma unroll
        for (int pair = 0; pair < 2; ++pair) {
            float W[2], L[2];
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const int j = 2 * pair + q;
                const float bb = h ? 1.0f : x2[j];
                f32x16 s[KT];
#pragma unroll
                for (int t = 0; t < KT; ++t) s[t] = mfma_key(a1[t], bb, mfma_key(a0[t], xh[j], zero));
                fold_keys<KT>(s, ninf, W[q], L[q]);
            }
            // lane half h finishes tile j = 2 pair + h: take the partner's
            // half of that tile and the partner's coordinate
            const float Wo = __shfl_xor(h ? W[0] : W[1], 32, 64);
            const float Lo = __shfl_xor(h ? L[0] : L[1], 32, 64);
            const float xo = __shfl_xor(h ? xh[2 * pair] : xh[2 * pair + 1], 32, 64);
            const int j = 2 * pair + h;
            const float Wm = h ? W[1] : W[0];
            const float Lm = h ? L[1] : L[0];
            const float x0 = h ? xo : xh[j];
            const float x1 = h ? xh[j] : xo;
            const float xz = x2[j];
            // merged halves: winner, and a lower bound of every other key
            const bool mine = !(Wo < Wm);
            const float Wc = mine ? Wm : Wo;
            const float Lc = vmin3(vmax(Wm, Wo), Lm, Lo);
            const int hw = mine ? h : 1 - h;
            uint32_t g = __float_as_uint(Wc) & 31u;
            g = g < 5u * KT ? g : 5u * KT;
            int cc[3];
            group_centres<KT>(g, hw, cc);
            // re-key the group's centres on the VALU; the smallest wins
            int k = cc[0];
            float kb = expanded_key<D>(x0, x1, xz, scand[cc[0] < K ? cc[0] : 0]);
#pragma unroll
            for (int e = 1; e < 3; ++e) {
                const float v = expanded_key<D>(x0, x1, xz, scand[cc[e] < K ? cc[e] : 0]);
                const bool lt = v < kb;
                kb = lt ? v : kb;
                k = lt ? cc[e] : k;
            }
            float b = fmaf(bq.y, fabsf(x0), bq.x);
            b = fmaf(bq.z, fabsf(x1), b);
            if constexpr (D == 3) b = fmaf(bq.w, fabsf(xz), b);
            b = fmaxf(b, 1e-30f);
            const int64_t i = i0 + j;
            const bool valid = i < N;
            const bool ok = Lc - Wc > b && k < K;
            if (valid && ok) sink(i, x0, x1, xz, k, direct_dist<D>(x0, x1, xz, smu[k]));
            const bool f = valid && !ok;
            const uint64_t m = __ballot(f);
            if (m) {
                if (f) wq[qn + __popcll(m & below)] = make_float4(x0, x1, xz, __int_as_float((int)i));
                qn += __popcll(m);
                if (qn >= 64) drain(64);
            }
        }
    }
    if (qn > 0) drain(qn);
}

}  // namespace km
