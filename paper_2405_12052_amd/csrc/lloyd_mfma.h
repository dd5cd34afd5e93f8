// lloyd_mfma.h -- reassignment scan with the expanded-form keys on the
// matrix cores (v_mfma_f32_32x32x16_f16, a two-piece fp16 split of the
// float32 operands), the argmin on the VALU.
//
// Keys.  s_k = c_k + sum_j a_kj x_j, a_kj = -2 m_kj, c_k = fl32(|m_k|^2): the
// records of the VALU scan.  Points and coefficients are scaled by one power
// of two 2^e (exact), chosen so that |x'| < 2^13 and |a'| < 2^14; then
// c' = c 2^(2e) < 3 2^26 and every scaled key |s'| < 2^29.2.  Each of x', a'
// is split v = vh + vl, vh = f16(v), vl = f16(v - vh) (round to nearest), and
// a'x' is taken as ah xh + ah xl + al xh (each product exact in float32).
// c' 2^-14 (< 3 2^12) is split into three f16 pieces, each multiplied by the
// exact f16 constant 2^14.  The 12 terms of a real centre are 12 of the 16
// inner-dimension entries of one 32x32x16 product (the accumulator input is
// zero); centres past K (pads) carry instead the one term 2^15 x 2^15 =
// 2^30, above every real key.
//
// Operand layout of the instruction (lane l, c = l % 32, h = l / 32):
// A[m][8h + i] and B[8h + i][n] are element i of lane (m or n) + 32h's
// 8-element operand; result register r holds row 8 (r / 4) + 4h + r % 4,
// column c.  Rows are centres, columns points.  Inner dimension:
//   k :  0    1    2    3    4    5    6    7  |  8    9   10   11   12   13   14  15
//   A :  ah0  ah0  ah1  ah1  al0  al1  c1   c2 |  ah2  ah2  0    0    al2  0    c3  p
//   B :  xh0  xl0  xh1  xl1  xh0  xh1  T    T  |  xh2  xl2  xh1  xl1  xh2  xh1  T   P
// with T = 2^14, P = 2^15, c1 + c2 + c3 = c' 2^-14, and p = P for pads (all
// other A entries of a pad zero), p = 0 for real centres.  Lane half h builds
// its B operand from u = (x0 if h = 0 else x2) and v = x1 as (uh, ul),
// (vh, vl), (uh, vh) and the constant (T, T) or (T, P): the same
// instructions in both halves.
//
// A wave takes 64 points at a time: lane (c, h) loads the coordinates of
// points 2c and 2c+1, so "chunk" j in 0..1 is the 32 points {2c + j}.  Per
// chunk each lane reduces its 16 KT keys to one minimum per quad of result
// registers (four consecutive centres; group number g = 4 t + r / 4 in the 3
// low mantissa bits: three instructions per quad), and a small tournament
// over those packed minima gives W, the smallest, and L, the second smallest
// (10 instructions for the 8 of K > 32).  The halves are merged
// with one lane swap per value (v_permlane32_swap), two chunks at a time, so
// that lane half h then finishes chunk h.  The winning quad's four
// centres (8 g + 4 hw + 0..3, hw the half that held it) are re-keyed on the
// VALU exactly as the VALU scan keys them, giving the quad's smallest key t1
// (first index) and second smallest t2.
//
// Certificate.  mag(x) = Cmax + 2 sum_j A_j |x_j| bounds every |s_k|
// (A_j = max_k |m_kj|).  A matrix key differs from the exact key of the
// float32 centres (scaled) by at most e_m: the split remainders and the
// dropped al xl leave <= 3.01 2^-22 |a'_j| |x'_j| + 2^-25 (|a'_j| + |x'_j|)
// per coordinate, the pieces of c' leave <= 2^-33 c' + 2^-11, and the sum of
// the 12 terms in float32, in any order and rounded either to nearest or
// toward zero, <= 11 2^-23 of the sum of their magnitudes:
// e_m <= 2.13 2^-20 mag' + 2^-8 (mag' = mag 2^(2e)); if the matrix core
// flushed f16 subnormal pieces to zero, each dropped product would add < 2
// (scaled units), < 8 in all.  Packing 3 bits moves a quad minimum by at
// most 7 units in its last place, <= 0.875 2^-20 mag'.  When L - W exceeds
// 2 (pack + e_m) <= 6.01 2^-20 mag' + 16.008, below 12.5 b(x) 2^(2e) + 17
// with b(x) the VALU scan's bound (b >= 2^-21 mag; the margin also covers
// the float32 rounding of L - W and of the bound), every key outside the
// winning quad
// exceeds, in exact arithmetic, the exact key of the quad's smallest member;
// when in addition t2 - t1 > b(x), the re-keying orders the quad exactly.
// The winner is then the exact argmin over all centres, and its margin is far
// above the float64 rounding of the direct form (b carries that term): the
// label of the VALU scan.  Other points go to the same per-wave re-scan queue.
//
// Range.  The scale needs 2^(2e + 4) to stay finite and normal: e in
// [-24, 60], i.e. data and centres between about 2^-48 and 2^36 in
// magnitude.  Outside it the pass takes the VALU scan.
#pragma once

#include "lloyd_device.h"

namespace km {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// min(a, b, c), single instruction: the keys are never signalling NaNs, so
// the operand quieting the compiler adds in front of its own minimum of
// values it cannot prove canonical (matrix-core results) is not needed.
__device__ __forceinline__ float vmin3(float a, float b, float c) {
    float r;
    asm("v_min3_f32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
    return r;
}

// min(a, b) and max(a, b), single instructions, for the same reason.
__device__ __forceinline__ float vmin2(float a, float b) {
    float r;
    asm("v_min_f32 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}

__device__ __forceinline__ float vmax2(float a, float b) {
    float r;
    asm("v_max_f32 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}

// The minimum of one quad of keys (a, b, c, d) with the group number GID in
// its 3 low mantissa bits.  FIRST: the quad is the first one read from a
// matrix-core result; its first minimum is then the compiler's own
// instruction, which carries the wait for the matrix core (the assembly that
// follows depends on it).
template <uint32_t GID, bool FIRST>
__device__ __forceinline__ float quad_min(float a, float b, float c, float d, uint32_t mask,
                                          float ninf) {
    float t;
    if constexpr (FIRST) {
        const float ab = min2(a, b, ninf);
        asm("v_min3_f32 %0, %1, %2, %3\n\t"
            "v_and_or_b32 %0, %0, %4, %5"
            : "=&v"(t)
            : "v"(ab), "v"(c), "v"(d), "s"(mask), "i"(GID));
    } else {
        asm("v_min3_f32 %0, %1, %2, %3\n\t"
            "v_min_f32 %0, %0, %4\n\t"
            "v_and_or_b32 %0, %0, %5, %6"
            : "=&v"(t)
            : "v"(a), "v"(b), "v"(c), "v"(d), "s"(mask), "i"(GID));
    }
    return t;
}

// The four packed quad minima of one tile of keys (per lane: 16).
template <int T>
__device__ __forceinline__ void tile_minima(const f32x16& s, float ninf, float (&p)[4]) {
    const uint32_t mask = ~7u;
    p[0] = quad_min<4 * T, true>(s[0], s[1], s[2], s[3], mask, ninf);
    p[1] = quad_min<4 * T + 1, false>(s[4], s[5], s[6], s[7], mask, ninf);
    p[2] = quad_min<4 * T + 2, false>(s[8], s[9], s[10], s[11], mask, ninf);
    p[3] = quad_min<4 * T + 3, false>(s[12], s[13], s[14], s[15], mask, ninf);
}

// Smallest and second smallest of (a, b, c) and of (a, b, c, d): the three
// values' minimum and median, then d merged in.
__device__ __forceinline__ void top2_3(float a, float b, float c, float& m1, float& m2) {
    m1 = vmin3(a, b, c);
    m2 = __builtin_amdgcn_fmed3f(a, b, c);
}

// (m1, m2) <- the two smallest of {m1, m2, u1, u2}, given m1 <= m2, u1 <= u2.
__device__ __forceinline__ void top2_merge(float& m1, float& m2, float u1, float u2) {
    m2 = vmin3(vmax2(m1, u1), m2, u2);
    m1 = vmin2(m1, u1);
}

// W, the smallest of 8 distinct values, and L, the second smallest, in 10
// instructions: groups of 3, 3 and 2 give their smallest (a1, b1, c1) and
// second smallest (a2, b2, c2); W is the smallest group minimum, and L the
// smaller of the middle group minimum (the best of the other groups) and the
// smallest second (the winning group's own runner-up, or a larger value).
__device__ __forceinline__ void top2_of_8(const float (&p)[8], float& W, float& L) {
    float a1, a2, b1, b2;
    top2_3(p[0], p[1], p[2], a1, a2);
    top2_3(p[3], p[4], p[5], b1, b2);
    const float c1 = vmin2(p[6], p[7]), c2 = vmax2(p[6], p[7]);
    W = vmin3(a1, b1, c1);
    L = vmin2(__builtin_amdgcn_fmed3f(a1, b1, c1), vmin3(a2, b2, c2));
}

// The keys of one chunk (B: its points' operand) against the KT tiles of
// centres A: W, the smallest packed quad minimum, and L, the second smallest
// (a small tournament over the 4 KT packed minima).
template <int KT>
__device__ __forceinline__ void chunk_keys(const f16x8 (&A)[KT], f16x8 B, float ninf, float& W,
                                           float& L) {
    const f32x16 zero16 = {};
    float p[4 * KT];
    const f32x16 k0 = __builtin_amdgcn_mfma_f32_32x32x16_f16(A[0], B, zero16, 0, 0, 0);
    tile_minima<0>(k0, ninf, reinterpret_cast<float(&)[4]>(p[0]));
    if constexpr (KT == 2) {
        const f32x16 k1 = __builtin_amdgcn_mfma_f32_32x32x16_f16(A[1], B, zero16, 0, 0, 0);
        tile_minima<1>(k1, ninf, reinterpret_cast<float(&)[4]>(p[4]));
        top2_of_8(p, W, L);
    } else {
        float a1, a2;
        top2_3(p[0], p[1], p[2], a1, a2);
        // d merged in: second smallest = min(a2, max(a1, d))
        L = vmin2(a2, vmax2(a1, p[3]));
        W = vmin2(a1, p[3]);
    }
}

// a in lane half 0, b in half 1 (hm: all ones in half 1), as one bitfield
// select: a ternary on array elements can become a select of their
// addresses, which puts the array in scratch memory.
__device__ __forceinline__ float sel_half(uint32_t hm, float a, float b) {
    return __uint_as_float((__float_as_uint(b) & hm) | (__float_as_uint(a) & ~hm));
}

// v = hi + lo (+ a remainder below 2^-22 |v| + 2^-25), both rounded to nearest.
__device__ __forceinline__ void split_f16(float v, _Float16& hi, _Float16& lo) {
    hi = (_Float16)v;
    lo = (_Float16)(v - (float)hi);
}

__device__ __forceinline__ uint32_t pack2(_Float16 lo, _Float16 hi) {
    const f16x2 v = {lo, hi};
    return __builtin_bit_cast(uint32_t, v);
}

// The B operand of one point for this lane half from the scaled u and v = x1
// (see the file header): (uh, ul), (vh, vl), (uh, vh) and the half's
// constant register q3.
__device__ __forceinline__ f16x8 point_operand(float u, float v, uint32_t q3) {
    _Float16 uh, ul, vh, vl;
    split_f16(u, uh, ul);
    split_f16(v, vh, vl);
    const uint32_t r0 = pack2(uh, ul), r1 = pack2(vh, vl);
    // (uh, vh): the low halves of r0 and r1, one byte permute (left to
    // itself the compiler converts uh and vh a second time)
    uint32_t r2;
    asm("v_perm_b32 %0, %1, %2, %3" : "=v"(r2) : "v"(r1), "v"(r0), "s"(0x05040100u));
    const u32x4 r = {r0, r1, r2, q3};
    return __builtin_bit_cast(f16x8, r);
}

__device__ __forceinline__ f16x8 zero_operand() {
    const u32x4 r = {0u, 0u, 0u, 0u};
    return __builtin_bit_cast(f16x8, r);
}

// The A operand of one centre row for lane half h (see the file header):
// the record r = (a0, a1, a2, c) of a real centre at scale 2^e, or a pad's
// single term P (with the half-1 constant P of the B operand: 2^30).
template <int D>
__device__ __forceinline__ f16x8 centre_operand(bool real, float4 r, int e, int h) {
    const _Float16 z = 0;
    if (real) {
        _Float16 h0, l0, h1, l1, h2, l2;
        split_f16(ldexpf(r.x, e), h0, l0);
        split_f16(ldexpf(r.y, e), h1, l1);
        split_f16(D == 3 ? ldexpf(r.z, e) : 0.0f, h2, l2);
        // c' 2^-14 in three pieces
        const float cs = ldexpf(r.w, 2 * e - 14);
        const _Float16 c1 = (_Float16)cs;
        const float r1 = cs - (float)c1;
        const _Float16 c2 = (_Float16)r1;
        const _Float16 c3 = (_Float16)(r1 - (float)c2);
        if (h == 0) {
            const f16x8 a = {h0, h0, h1, h1, l0, l1, c1, c2};
            return a;
        }
        const f16x8 a = {h2, h2, z, z, l2, z, c3, z};
        return a;
    }
    if (h == 0) return zero_operand();
    const f16x8 a = {z, z, z, z, z, z, z, (_Float16)32768.0f};
    return a;
}

// Scale exponent e of the matrix-core keys for data of exponent xe
// (max|x| < 2^(xe+1)) and centres with bnd (the VALU bound coefficients:
// bnd.y..w >= 2^-20 max_k |m_kj|); false when e falls outside [-24, 96].
__device__ __forceinline__ bool mfma_scale(int xe, float4 bnd, int& e) {
    // >= max_kj |m_kj| (bnd.y = 2^-20 (1 + 2^-10) max_k |m_k0| + ...)
    const float amax = ldexpf(fmaxf(fmaxf(bnd.y, bnd.z), bnd.w), 20);
    e = 12 - xe;                                     // |x| 2^e < 2^13
    if (amax > 0.0f) {
        const int ea = 12 - ilogbf(amax);            // |a| 2^e = 2 |m| 2^e < 2^14
        e = ea < e ? ea : e;
    }
    return e >= -24 && e <= 60;
}

// Reassignment of the points of this wave's share of the grid (chunks of 128
// points) with the matrix-core keys; same contract as assign_points (sink
// receives every certified point, the others are re-scanned from the
// per-wave queue).  scand: the centre records, KPAD of them (pads included);
// e: the scale exponent (mfma_scale).
template <int D, bool VEC, int KT, typename Sink>
__device__ __forceinline__ void assign_points_mfma(const float* __restrict__ X, int64_t ld,
                                                   int64_t N, const float4* __restrict__ scand,
                                                   const float4* __restrict__ smu, int K,
                                                   float4 bnd, int e, float ninf,
                                                   float4* __restrict__ wq, Sink&& sink) {
    const int lane = threadIdx.x & 63;
    const int c = lane & 31, h = lane >> 5;
    constexpr float T = 16384.0f, P = 32768.0f;

    // A operands (centre 32 t + c), fixed for the whole pass
    f16x8 A[KT];
#pragma unroll
    for (int t = 0; t < KT; ++t) {
        const int k = 32 * t + c;
        A[t] = centre_operand<D>(k < K, k < K ? scand[k] : make_float4(0.f, 0.f, 0.f, 0.f), e, h);
    }
    const uint32_t hm = h ? ~0u : 0u;  // lane half as a bit mask
    const uint32_t q3 = h == 0 ? pack2((_Float16)T, (_Float16)T) : pack2((_Float16)T, (_Float16)P);
    const float s = ldexpf(1.0f, e);
    // matrix-key bound in scaled units: 12.5 b(x) 2^(2e) + 17 (the absolute
    // part covers f16 subnormal pieces even if the matrix core flushed them);
    // the scale 2^(2e+4) <= 2^124 stays finite
    const float bms = ldexpf(12.5f, 2 * e);

    int qn = 0;
    auto drain = [&](int cnt) {
        __builtin_amdgcn_wave_barrier();
        if (lane < cnt) {
            const float4 q = wq[qn - cnt + lane];
            float bd;
            int bk;
            direct_scan<D>(smu, K, q.x, q.y, q.z, bd, bk);
            sink((int64_t)__float_as_int(q.w), q.x, q.y, q.z, bk, bd);
        }
        __builtin_amdgcn_wave_barrier();
        qn -= cnt;
    };

    // chunk numbers in 32 bits (N < 2^31), so the loop test is a scalar one
    const int nchunks = (int)((N + 63) / 64);
    // the points as global memory: loads from a wave-uniform base in scalar
    // registers plus the lane's 32-bit offset
    typedef const float __attribute__((address_space(1)))* gfp;
    typedef float f32x2 __attribute__((ext_vector_type(2)));
    typedef const f32x2 __attribute__((address_space(1)))* gf2p;
    const gfp Xg = (gfp)X;
    // the wave's index, known to the compiler as uniform (scalar registers)
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    // the grid stride, kept in a scalar register (reloaded from the dispatch
    // packet it would cost a wait on every outstanding LDS atomic per chunk)
    int stride = (int)gridDim.x * NW;
    asm("" : "+s"(stride));
    for (int ch = (int)blockIdx.x * NW + wid; ch < nchunks; ch += stride) {
        const int64_t c0 = (int64_t)ch * 64;
        const int64_t i0 = c0 + 2 * c;  // first of this lane's 2 points
        // points of this chunk pair that exist (wave-uniform; left > 0).  The
        // empty asm statements keep these values in scalar registers as
        // written: the compiler would otherwise turn the test into a 64-bit
        // comparison on the VALU, and fold the row base into per-lane 64-bit
        // addresses.
        const int64_t left = N - c0;
        int64_t lhi = left >> 6;
        asm("" : "+s"(lhi));
        const bool full = lhi != 0;
        const int rem = full ? 64 : (int)left;
        float x[3][2];
        if (VEC && full) {
#pragma unroll
            for (int j = 0; j < D; ++j) {
                gfp row = Xg + (j * ld + c0);
                asm("" : "+s"(row));
                const f32x2 v = *(gf2p)(row + (uint32_t)(2 * c));
                x[j][0] = v.x; x[j][1] = v.y;
            }
        } else {
#pragma unroll
            for (int p = 0; p < 2; ++p) {
                const bool in = i0 + p < N;
#pragma unroll
                for (int j = 0; j < D; ++j) x[j][p] = in ? X[j * ld + i0 + p] : 0.0f;
            }
        }
        if constexpr (D == 2) {
            x[2][0] = 0.0f;
            x[2][1] = 0.0f;
        }

        float W[2], L[2];
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const float u = sel_half(hm, x[0][q], x[2][q]) * s;
            const float v = x[1][q] * s;
            chunk_keys<KT>(A, point_operand(u, v, q3), ninf, W[q], L[q]);
        }
        // lane half h finishes chunk h.  After the swaps, in either half,
        // w0 / l0 come from the h = 0 lane of the point and w1 / l1 from the
        // h = 1 lane.
        const auto ws = __builtin_amdgcn_permlane32_swap(__float_as_uint(W[0]),
                                                          __float_as_uint(W[1]), false, false);
        const auto ls = __builtin_amdgcn_permlane32_swap(__float_as_uint(L[0]),
                                                          __float_as_uint(L[1]), false, false);
        const float w0 = __uint_as_float(ws[0]), w1 = __uint_as_float(ws[1]);
        const float l0 = __uint_as_float(ls[0]), l1 = __uint_as_float(ls[1]);
        const float Wc = vmin2(w0, w1);
        const float Lc = vmin3(vmax2(w0, w1), l0, l1);
        const int hw = w1 < w0 ? 1 : 0;
        // this lane's point: chunk h (selected, not indexed: a lane-dependent
        // index would put x in scratch memory)
        const float x0 = sel_half(hm, x[0][0], x[0][1]);
        const float x1 = sel_half(hm, x[1][0], x[1][1]);
        const float x2 = sel_half(hm, x[2][0], x[2][1]);
        // the winning quad: centres 8 g + 4 hw + 0..3 (records padded to KPAD)
        const int base = ((int)(__float_as_uint(Wc) & 7u) << 3) | (hw << 2);
        const float s0 = expanded_key<D>(x0, x1, x2, scand[base]);
        const float s1 = expanded_key<D>(x0, x1, x2, scand[base + 1]);
        const float s2 = expanded_key<D>(x0, x1, x2, scand[base + 2]);
        const float s3 = expanded_key<D>(x0, x1, x2, scand[base + 3]);
        const float a3 = fminf(fminf(s0, s1), s2);
        const float t1 = fminf(a3, s3);
        // second smallest of the four: of the first three, or max(their
        // minimum, s3)
        const float t2 = fminf(__builtin_amdgcn_fmed3f(s0, s1, s2), fmaxf(a3, s3));
        // first index attaining t1 (selects, not branches)
        int kq = 3;
        kq = s2 == t1 ? 2 : kq;
        kq = s1 == t1 ? 1 : kq;
        kq = s0 == t1 ? 0 : kq;
        const int k = base + kq;
        float b = fmaf(bnd.y, fabsf(x0), bnd.x);
        b = fmaf(bnd.z, fabsf(x1), b);
        if constexpr (D == 3) b = fmaf(bnd.w, fabsf(x2), b);
        const float bm = fmaf(b, bms, 17.0f);
        const int64_t i = i0 + h;
        // The certificate as lane masks, one ballot per comparison, combined
        // on the scalar unit (a ballot of a combined condition costs a copy
        // through a vector register).  No k < K test: a pad's matrix key,
        // 2^30, is above every real one (< 2^29.2), so the winning quad
        // holds a real centre, and a pad's record keys at 2^127, above
        // every real key, so t1 is a real centre's.
        const uint64_t mv = __builtin_amdgcn_ballot_w64(2 * c + h < rem);
        const uint64_t mok = __builtin_amdgcn_ballot_w64(Lc - Wc > bm) &
                             __builtin_amdgcn_ballot_w64(t2 - t1 > b);
        // the queue's lanes: valid and not certified
        const uint64_t m = mv & ~mok;
        if (__builtin_amdgcn_inverse_ballot_w64(mv & mok))
            sink(i, x0, x1, x2, k, direct_dist<D>(x0, x1, x2, smu[k]));
        if (m) {
            // slot: the queued lanes below this one (mbcnt)
            const int below_m = (int)__builtin_amdgcn_mbcnt_hi(
                (uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
            // this lane is queued: its bit of m, as a lane mask (no vector copy)
            if (__builtin_amdgcn_inverse_ballot_w64(m))
                wq[qn + below_m] = make_float4(x0, x1, x2, __int_as_float((int)i));
            qn += __popcll(m);
            if (qn >= 64) drain(64);
        }
    }
    if (qn > 0) drain(qn);
}

}  // namespace km
