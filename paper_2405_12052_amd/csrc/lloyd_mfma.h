// lloyd_mfma.h -- reassignment scan with the expanded-form keys computed on
// the matrix cores from a two-piece fp16 split of the float32 operands
// (v_mfma_f32_32x32x16_f16), the argmin on the VALU.
//
// Keys.  s_k = c_k + sum_j a_kj x_j with a_kj = -2 m_kj and c_k = fl32(|m_k|^2)
// (the records the VALU scan uses).  The points are scaled by 2^ex and the
// coefficients by 2^ea (powers of two: exact) so that every |x'|, |a'| < 2^15,
// and each is split as v = hi + lo, hi = f16(v), lo = f16(v - hi) (both
// rounded to nearest): |v - hi - lo| <= 2^-22 |v| + 2^-25.  The product a'x'
// is taken as ah xh + ah xl + al xh (each term exact in float32); the dropped
// al xl and the split remainders leave <= 3.01 2^-22 |a'||x'| + 2^-24
// (|a'| + |x'|).  The 3 terms per coordinate are 9 inner-dimension entries
// of one 32x32x16 product, and the constant c_k 2^(ea+ex) (exact) enters as
// the accumulator input, so that the result is the key scaled by 2^(ea+ex).
//
// Operand layout of the instruction (lane l, c = l % 32, h = l / 32):
// A[m][8h + i] and B[8h + i][n] are element i of lane (m or n) + 32h's
// 8-element operand, and register r of the result holds row
// 8(r/4) + 4h + r%4, column c.  Rows are centres, columns points.  Lane
// (c, h) supplies for its point the column (xh0, xl0, xh0, xh1, xl1, xh1,
// xh2, xl2) in both halves, and for its centre the row (ah0, ah0, al0, ah1,
// ah1, al1, ah2, ah2) in half 0 and (0, 0, 0, 0, 0, 0, al2, 0) in half 1:
// the 9 terms, with no lane-dependent work on the point side.  K <= 64 takes
// KT = 1 or 2 tiles of 32 centres; centres past K have zero coefficients
// and the constant 2^127 (finite, so that packing a group number into it
// cannot make a NaN, and above every real key: the scales keep those below
// 2^96).
//
// A wave takes 128 points at a time: lane (c, h) loads the D coordinates of
// points 4c .. 4c+3, so "tile" j in 0..3 is the 32 points {4c + j}.  Per tile
// each lane folds its 16 KT keys into W, the smallest group minimum with the
// group's number in its 5 low mantissa bits, and L, the second smallest
// (groups are triples of result registers; four compare-type instructions
// per triple).  The halves of a point are merged across lanes l and l ^ 32,
// two tiles at a time, so that every lane then finishes one point: the
// winning group's (at most 3) centres are re-keyed on the VALU with three
// FMAs each, giving the group's smallest key t1 (first index) and second
// smallest t2.
//
// Certificate.  Take mag'(x) = Cmax' + sum_j A'_j |x'_j| (the scaled Cmax and
// max_k |a_kj| of the VALU scan's bound), which bounds every |key|.  A matrix
// key differs from the exact key of the float32 centres by e_m <= 2.1 2^-20
// mag' + 18 (the rounding of c_k, the split remainders, and 10 float32 sums
// bounded pessimistically by 2^-23 each; 18 covers f16 subnormal inputs even
// if the matrix core flushed them), and packing moves a group minimum by at
// most 2^-18 mag'.  When L - W > 2^-16 mag' + 64 (> 2 pack + 2 e_m), every
// key outside the winning group exceeds, in exact arithmetic, the exact key
// of the group's smallest member.  When in addition t2 - t1 > b(x) (the VALU
// scan's bound, over twice the VALU key error), the re-keying orders the
// group exactly.  The winner is then the exact argmin over all centres: the
// label the VALU scan certifies.  Both bounds also carry the float64 direct
// form's term of the coefficients (prep_centres; 16 times over in the scaled
// one).  Other points go to the same per-wave
// re-scan queue, so the labels are identical to the VALU scan's.
#pragma once

#include "lloyd_device.h"

namespace km {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ f32x16 mfma_key16(f16x8 a, f16x8 b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
}

// min(a, b, c) and max(a, b), single instructions: the keys are never
// signalling NaNs, so the operand quieting that the compiler adds in front of
// its own min/max for values it cannot prove canonical is not needed.
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

// v = hi + lo (+ a remainder below 2^-22 |v| + 2^-25), both rounded to nearest.
__device__ __forceinline__ void split_f16(float v, _Float16& hi, _Float16& lo) {
    hi = (_Float16)v;
    lo = (_Float16)(v - (float)hi);
}

// Centre of result register r (0..15) of centre tile t for lane half h.
__device__ __forceinline__ int reg_centre(int t, int r, int h) {
    return 32 * t + 8 * (r >> 2) + 4 * h + (r & 3);
}

// One group of keys (a, b, c) into the running (m1, s2): the group minimum
// with the group number GID in its 5 low mantissa bits, m1 = smallest such
// value so far, s2 = second smallest.  FIRST: the group is the first one read
// from a matrix-core result; its first minimum is then the compiler's own
// instruction, which carries the wait for the matrix core (the assembly that
// follows depends on it).
template <uint32_t GID, bool FIRST>
__device__ __forceinline__ void fold_group(float a, float b, float c, uint32_t mask, float ninf,
                                           float& m1, float& s2) {
    float t;
    if constexpr (FIRST) {
        const float ab = min2(a, b, ninf);
        asm("v_min_f32 %0, %3, %4\n\t"
            "v_and_or_b32 %0, %0, %5, %6\n\t"
            "v_med3_f32 %1, %2, %1, %0\n\t"
            "v_min_f32 %2, %2, %0"
            : "=&v"(t), "+v"(s2), "+v"(m1)
            : "v"(ab), "v"(c), "s"(mask), "i"(GID));
    } else {
        asm("v_min3_f32 %0, %3, %4, %5\n\t"
            "v_and_or_b32 %0, %0, %6, %7\n\t"
            "v_med3_f32 %1, %2, %1, %0\n\t"
            "v_min_f32 %2, %2, %0"
            : "=&v"(t), "+v"(s2), "+v"(m1)
            : "v"(a), "v"(b), "v"(c), "s"(mask), "i"(GID));
    }
}

// Fold the keys of one tile of points (per lane: 16 KT keys) into (W, L):
// groups are the register triples (0,1,2) .. (12,13,14) of each centre tile
// and the last registers (15) of all tiles.
template <int KT>
__device__ __forceinline__ void fold_keys(const f32x16 (&s)[KT], float ninf, float& W, float& L) {
    const uint32_t mask = ~31u;
    float m1 = INFINITY, s2 = INFINITY;
    fold_group<0, true>(s[0][0], s[0][1], s[0][2], mask, ninf, m1, s2);
    fold_group<1, false>(s[0][3], s[0][4], s[0][5], mask, ninf, m1, s2);
    fold_group<2, false>(s[0][6], s[0][7], s[0][8], mask, ninf, m1, s2);
    fold_group<3, false>(s[0][9], s[0][10], s[0][11], mask, ninf, m1, s2);
    fold_group<4, false>(s[0][12], s[0][13], s[0][14], mask, ninf, m1, s2);
    if constexpr (KT == 2) {
        fold_group<5, true>(s[1][0], s[1][1], s[1][2], mask, ninf, m1, s2);
        fold_group<6, false>(s[1][3], s[1][4], s[1][5], mask, ninf, m1, s2);
        fold_group<7, false>(s[1][6], s[1][7], s[1][8], mask, ninf, m1, s2);
        fold_group<8, false>(s[1][9], s[1][10], s[1][11], mask, ninf, m1, s2);
        fold_group<9, false>(s[1][12], s[1][13], s[1][14], mask, ninf, m1, s2);
        // the pair (15 of tile 0, 15 of tile 1), padded with +inf
        fold_group<10, false>(s[0][15], s[1][15], INFINITY, mask, ninf, m1, s2);
    } else {
        fold_group<5, false>(s[0][15], INFINITY, INFINITY, mask, ninf, m1, s2);
    }
    W = m1;
    L = s2;
}

// The centres of group g for lane half h, in increasing order; -1 where the
// group has fewer than three.
template <int KT>
__device__ __forceinline__ void group_centres(uint32_t g, int h, int (&c)[3]) {
    if (g < 5u * KT) {
        const int t = (int)g / 5, r = 3 * ((int)g % 5);
        c[0] = reg_centre(t, r, h);
        c[1] = reg_centre(t, r + 1, h);
        c[2] = reg_centre(t, r + 2, h);
    } else {
        c[0] = reg_centre(0, 15, h);
        c[1] = KT == 2 ? reg_centre(1, 15, h) : -1;
        c[2] = -1;
    }
}

// The 8-element B column of one point (scaled coordinates), the same in both
// lane halves: (xh0, xl0, xh0, xh1, xl1, xh1, xh2, xl2).
template <int D>
__device__ __forceinline__ f16x8 point_column(float x0, float x1, float x2) {
    _Float16 h0, l0, h1, l1, h2 = 0, l2 = 0;
    split_f16(x0, h0, l0);
    split_f16(x1, h1, l1);
    if constexpr (D == 3) split_f16(x2, h2, l2);
    const f16x8 b = {h0, l0, h0, h1, l1, h1, h2, l2};
    return b;
}

// Reassignment of the points of this wave's share of the grid (chunks of 128
// points) with the matrix-core keys; same contract as assign_points (sink
// receives every certified point, the others are re-scanned from the
// per-wave queue).  xe: the exponent of the data's magnitude (every
// |x| < 2^(xe+1)).
template <int D, bool VEC, int KT, typename Sink>
__device__ __forceinline__ void assign_points_mfma(const float* __restrict__ X, int64_t ld,
                                                   int64_t N, const float4* __restrict__ scand,
                                                   const float4* __restrict__ smu, int K,
                                                   float4 bnd, float ninf, int xe,
                                                   float4* __restrict__ wq, Sink&& sink) {
    const int lane = threadIdx.x & 63;
    const int c = lane & 31, h = lane >> 5;
    const uint64_t below = (1ull << lane) - 1ull;

    // Scales: |x 2^ex| < 2^15 and |a 2^ea| < 2^15 (max |a_kj| = 2 max_kj |m_kj| <=
    // 2^21 max(bnd.yzw)); ex - ea <= 64 keeps every scaled key below 2^96.
    const float amax = ldexpf(fmaxf(fmaxf(bnd.y, bnd.z), bnd.w), 21);
    int ex = 14 - xe < 105 ? 14 - xe : 105;
    int ea = amax > 0.0f ? 14 - ilogbf(amax) : ex;
    if (ex > ea + 64) ex = ea + 64;

    // A operands (centre 32t + c) and accumulator inputs (the scaled
    // constants of the result registers' centres), fixed for the whole pass
    f16x8 A[KT];
    f32x16 C[KT];
#pragma unroll
    for (int t = 0; t < KT; ++t) {
        const int k = 32 * t + c;
        _Float16 h0 = 0, l0 = 0, h1 = 0, l1 = 0, h2 = 0, l2 = 0;
        if (k < K) {
            const float4 r = scand[k];
            split_f16(ldexpf(r.x, ea), h0, l0);
            split_f16(ldexpf(r.y, ea), h1, l1);
            if constexpr (D == 3) split_f16(ldexpf(r.z, ea), h2, l2);
        }
        const _Float16 z = 0;
        if (h == 0) {
            const f16x8 a = {h0, h0, l0, h1, h1, l1, h2, h2};
            A[t] = a;
        } else {
            const f16x8 a = {z, z, z, z, z, z, l2, z};
            A[t] = a;
        }
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int kr = reg_centre(t, r, h);
            C[t][r] = kr < K ? ldexpf(scand[kr].w, ea + ex) : 0x1p127f;
        }
    }
    // bound on the scaled gap: 2^-16 mag'(x) + 64 (the coefficients hold 2^-21
    // and 2^-20 of the magnitudes, with 2^-10 to spare)
    const float bx = ldexpf(bnd.x, 5 + ea + ex) + 64.0f;
    const float by = ldexpf(bnd.y, 5 + ea), bz = ldexpf(bnd.z, 5 + ea), bw = ldexpf(bnd.w, 5 + ea);
    const float sx = ldexpf(1.0f, ex);

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
        const int64_t i0 = ch * 128 + 4 * c;  // first of this lane's 4 points
        float x[3][4];
        if (VEC && i0 + 4 <= N) {
#pragma unroll
            for (int j = 0; j < D; ++j) {
                const float4 v = *reinterpret_cast<const float4*>(X + j * ld + i0);
                x[j][0] = v.x; x[j][1] = v.y; x[j][2] = v.z; x[j][3] = v.w;
            }
        } else {
#pragma unroll
            for (int p = 0; p < 4; ++p) {
                const bool in = i0 + p < N;
#pragma unroll
                for (int j = 0; j < D; ++j) x[j][p] = in ? X[j * ld + i0 + p] : 0.0f;
            }
        }
        if constexpr (D == 2) {
#pragma unroll
            for (int p = 0; p < 4; ++p) x[2][p] = 0.0f;
        }

#pragma unroll
        for (int pair = 0; pair < 2; ++pair) {
            float W[2], L[2];
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const int j = 2 * pair + q;
                const f16x8 B = point_column<D>(x[0][j] * sx, x[1][j] * sx, x[2][j] * sx);
                f32x16 s[KT];
#pragma unroll
                for (int t = 0; t < KT; ++t) s[t] = mfma_key16(A[t], B, C[t]);
                fold_keys<KT>(s, ninf, W[q], L[q]);
            }
            // lane half h finishes tile j = 2 pair + h: take the partner's
            // half of that tile
            const float Wo = __shfl_xor(h ? W[0] : W[1], 32, 64);
            const float Lo = __shfl_xor(h ? L[0] : L[1], 32, 64);
            const int j = 2 * pair + h;
            const float Wm = h ? W[1] : W[0];
            const float Lm = h ? L[1] : L[0];
            const float x0 = h ? x[0][2 * pair + 1] : x[0][2 * pair];
            const float x1 = h ? x[1][2 * pair + 1] : x[1][2 * pair];
            const float xz = h ? x[2][2 * pair + 1] : x[2][2 * pair];
            // merged halves: winner, and the second smallest group minimum
            const bool mine = !(Wo < Wm);
            const float Wc = mine ? Wm : Wo;
            const float Lc = vmin3(vmax(Wm, Wo), Lm, Lo);
            const int hw = mine ? h : 1 - h;
            uint32_t g = __float_as_uint(Wc) & 31u;
            g = g < 5u * KT ? g : 5u * KT;
            int cc[3];
            group_centres<KT>(g, hw, cc);
            // re-key the group's centres on the VALU: smallest (first index)
            // and second smallest
            float t1 = 0x1p127f, t2 = 0x1p127f;
            int k = K;
#pragma unroll
            for (int e = 0; e < 3; ++e) {
                const bool in = cc[e] >= 0 && cc[e] < K;
                const float v = in ? expanded_key<D>(x0, x1, xz, scand[in ? cc[e] : 0]) : 0x1p127f;
                const bool lt = v < t1;
                t2 = lt ? t1 : fminf(t2, v);
                t1 = lt ? v : t1;
                k = lt ? cc[e] : k;
            }
            float b = fmaf(bnd.y, fabsf(x0), bnd.x);
            b = fmaf(bnd.z, fabsf(x1), b);
            if constexpr (D == 3) b = fmaf(bnd.w, fabsf(xz), b);
            float bm = fmaf(by, fabsf(x0 * sx), bx);
            bm = fmaf(bz, fabsf(x1 * sx), bm);
            if constexpr (D == 3) bm = fmaf(bw, fabsf(xz * sx), bm);
            const int64_t i = i0 + j;
            const bool valid = i < N;
            const bool ok = Lc - Wc > bm && t2 - t1 > b && k < K;
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
