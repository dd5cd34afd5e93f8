// initnet_kernels.hip -- the learned initialiser: a permutation-invariant
// network that maps a sample of P points of an instance (normalised by their
// mean and scalar standard deviation) to K initial centres, and its training.
//
//   per point  h1 = relu(x W1 + b1)          3 -> 64    (VALU, fp32)
//              h2 = relu(h1 W2 + b2)         64 -> 64   (BF16 MFMA 32x32x16, fp32 acc)
//   pooling    p  = [mean h2, max h2]        128        (max: first point on ties)
//   head       z  = relu(p W3 + b3)          128 -> 256
//              y  = z W4 + b4                256 -> 3K
//   loss       L  = (1/B) sum_b sum_k |y_b[pi_b(k)] - t_b[k]|^2, pi_b the
//                   least-cost assignment (Hungarian, on the device)
//
// Weights are used as bfloat16 copies of float32 masters (round to nearest
// even when loaded); the activations entering matrix products (h1, p, z) and
// the back-propagated signals entering them (dh2, dz, dy) are rounded to
// bfloat16 as well; all sums accumulate in float32.  Gradients reach the
// masters unchanged (the rounding is treated as the identity).  The head's
// products (B x 128 x 256 and B x 256 x 3K per step) run on the VALU on the
// same bfloat16 operands; the per-point products, which hold all but a
// fraction of a percent of the work, run on the matrix cores.
//
// Every sum is taken in a fixed order (lanes, waves, instances), so a step's
// gradient repeats bit for bit; there are no float atomics.
#include "initnet.h"

#include <math.h>

namespace km {
namespace net {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int NW = 4;             // waves per block
constexpr int NT = 64 * NW;       // threads per block

__device__ __forceinline__ float bfr(float f) { return (float)(__bf16)f; }

__device__ __forceinline__ f32x16 mfma(bf16x8 a, bf16x8 b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ f32x16 zero16() {
    f32x16 z;
#pragma unroll
    for (int i = 0; i < 16; ++i) z[i] = 0.0f;
    return z;
}

// Row (within the 32-row tile) of accumulator register r of lane l:
// D[8*(r/4) + 4*(l/32) + r%4][l % 32].
__device__ __forceinline__ int drow(int r, int lane) { return 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3); }

__device__ __forceinline__ void wave_sync_lds() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Layer 1 for point (x0, x1, x2) and the 8 features f0..f0+7: relu(x W1 + b1)
// as fp32 (t = b; t += x0 w0; t += x1 w1; t += x2 w2 with FMAs), rounded to
// bf16 for the MFMA operand.
__device__ __forceinline__ bf16x8 layer1_bf(const float* sW1, const float* sb1, float x0,
                                            float x1, float x2, int f0) {
    bf16x8 a;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const int f = f0 + e;
        float t = fmaf(x0, sW1[f], sb1[f]);
        t = fmaf(x1, sW1[64 + f], t);
        t = fmaf(x2, sW1[128 + f], t);
        a[e] = (__bf16)fmaxf(t, 0.0f);
    }
    return a;
}

// W2 (or its transpose) as MFMA operands held in registers: for k-step s and
// column tile t, lane l holds M[k = 16 s + 8 (l/32) + e][n = 32 t + l%32],
// e = 0..7, with M = W2 (trans = false: M[k][n] = W2[k][n]) or W2^T.
__device__ __forceinline__ void load_w2(const float* __restrict__ W2, bool trans, int lane,
                                        bf16x8 (&w)[4][2]) {
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int k = 16 * s + 8 * (lane >> 5) + e, n = 32 * t + (lane & 31);
                w[s][t][e] = (__bf16)(trans ? W2[n * NH + k] : W2[k * NH + n]);
            }
}

// ------------------------------------------------------------ net_points_fwd
// One block per instance.  pool[b] = [mean_p h2, max_p h2], argmax[b][n] =
// first point attaining the maximum of feature n.
__global__ __launch_bounds__(NT) void net_points_fwd(const float* __restrict__ pts, int P,
                                                     const float* __restrict__ params,
                                                     float* __restrict__ pool,
                                                     int32_t* __restrict__ argmax) {
    __shared__ float sW1[3 * NH];
    __shared__ float sb1[NH];
    __shared__ float ssum[NW][NH];
    __shared__ float smax[NW][NH];
    __shared__ int sarg[NW][NH];
    const int b = blockIdx.x, tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    for (int i = tid; i < 3 * NH; i += NT) sW1[i] = bfr(params[OFF_W1 + i]);
    for (int i = tid; i < NH; i += NT) sb1[i] = params[OFF_B1 + i];
    bf16x8 w2[4][2];
    load_w2(params + OFF_W2, false, lane, w2);
    float b2[2];
#pragma unroll
    for (int t = 0; t < 2; ++t) b2[t] = params[OFF_B2 + 32 * t + (lane & 31)];
    __syncthreads();
    const float* __restrict__ xb = pts + (size_t)b * P * 3;
    float sum[2] = {0.f, 0.f}, mx[2] = {-INFINITY, -INFINITY};
    int arg[2] = {0, 0};
    for (int tile = w; tile < P / 32; tile += NW) {
        const int m = tile * 32 + (lane & 31);
        const float x0 = xb[m * 3], x1 = xb[m * 3 + 1], x2 = xb[m * 3 + 2];
        bf16x8 a[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) a[s] = layer1_bf(sW1, sb1, x0, x1, x2, 16 * s + 8 * (lane >> 5));
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            f32x16 acc = zero16();
#pragma unroll
            for (int s = 0; s < 4; ++s) acc = mfma(a[s], w2[s][t], acc);
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const float h = fmaxf(acc[r] + b2[t], 0.0f);
                sum[t] += h;
                if (h > mx[t]) { mx[t] = h; arg[t] = tile * 32 + drow(r, lane); }
            }
        }
    }
    // lanes l and l+32 hold the same feature: combine (sum low + high; max
    // prefers the larger value, then the smaller point index)
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        const float os = __shfl_xor(sum[t], 32, 64);
        const float om = __shfl_xor(mx[t], 32, 64);
        const int oa = __shfl_xor(arg[t], 32, 64);
        const float lo = lane < 32 ? sum[t] : os, hi = lane < 32 ? os : sum[t];
        sum[t] = lo + hi;
        if (om > mx[t] || (om == mx[t] && oa < arg[t])) { mx[t] = om; arg[t] = oa; }
        if (lane < 32) {
            ssum[w][32 * t + lane] = sum[t];
            smax[w][32 * t + lane] = mx[t];
            sarg[w][32 * t + lane] = arg[t];
        }
    }
    __syncthreads();
    if (tid < NH) {
        float s = 0.f, m = -INFINITY;
        int a = 0;
        for (int v = 0; v < NW; ++v) {
            s += ssum[v][tid];
            if (smax[v][tid] > m || (smax[v][tid] == m && sarg[v][tid] < a)) {
                m = smax[v][tid];
                a = sarg[v][tid];
            }
        }
        pool[(size_t)b * 2 * NH + tid] = s / (float)P;
        pool[(size_t)b * 2 * NH + NH + tid] = m;
        if (argmax) argmax[(size_t)b * NH + tid] = a;
    }
}

// ------------------------------------------------------------ Hungarian
// Least-cost assignment of an n x n matrix c[i*n + j] (rows: predictions,
// columns: targets), shortest augmenting paths with potentials (the classic
// O(n^3) method of Kuhn and Munkres as refined by Jonker and Volgenant).
// Writes pi[j] = the row assigned to column j.  One thread.
__device__ void hungarian(const double* c, int n, int* pi) {
    double u[KMAXN + 1], v[KMAXN + 1], minv[KMAXN + 1];
    int p[KMAXN + 1], way[KMAXN + 1];
    bool used[KMAXN + 1];
    for (int i = 0; i <= n; ++i) { u[i] = 0.0; v[i] = 0.0; p[i] = 0; way[i] = 0; }
    for (int i = 1; i <= n; ++i) {
        // add row i: grow an alternating tree from the virtual column 0
        p[0] = i;
        int j0 = 0;
        for (int j = 0; j <= n; ++j) { minv[j] = INFINITY; used[j] = false; }
        int guard = 0;  // each pass marks one more column: at most n + 1 passes
        do {
            if (++guard > n + 1) break;
            used[j0] = true;
            const int i0 = p[j0];
            double delta = INFINITY;
            int j1 = 0;
            for (int j = 1; j <= n; ++j) {
                if (used[j]) continue;
                double cij = c[(i0 - 1) * n + (j - 1)];
                if (!(cij < 1e300)) cij = 1e300;  // NaN / inf: a huge finite cost
                const double cur = cij - u[i0] - v[j];
                if (cur < minv[j]) { minv[j] = cur; way[j] = j0; }
                if (minv[j] < delta) { delta = minv[j]; j1 = j; }
            }
            for (int j = 0; j <= n; ++j) {
                if (used[j]) { u[p[j]] += delta; v[j] -= delta; }
                else minv[j] -= delta;
            }
            j0 = j1;
        } while (p[j0] != 0);
        for (int g = 0; j0 && g <= n; ++g) {  // flip the augmenting path
            const int j1 = way[j0];
            p[j0] = p[j1];
            j0 = j1;
        }
    }
    for (int j = 1; j <= n; ++j) pi[j - 1] = (p[j] >= 1 && p[j] <= n) ? p[j] - 1 : j - 1;
}

// ------------------------------------------------------------ net_head
// One block per instance: head forward; with targets also the matching, the
// loss and the head's backward pass.  Writes per instance the bf16 operands
// the weight gradients need (poolbf, zbf, dybf, dzbf), the float32 bias
// gradients' summands (dy, dz), dpool, the loss and the matching.
__global__ __launch_bounds__(NT) void net_head(const float* __restrict__ pool, int B, int K,
                                               const float* __restrict__ params,
                                               const float* __restrict__ targets,
                                               float* __restrict__ pred, HeadOut ho) {
    __shared__ float sp[2 * NH];
    __shared__ float sz[NZ];
    __shared__ float sza[NZ];
    __shared__ float sy[3 * KMAXN];
    __shared__ float sdy[3 * KMAXN];
    __shared__ float sdz[NZ];
    __shared__ double scost[KMAXN * KMAXN];
    __shared__ int spi[KMAXN];
    const int b = blockIdx.x, tid = threadIdx.x;
    const int O = 3 * K;
    const float* W3 = params + OFF_W3;
    const float* W4 = params + OFF_W4;
    const float* b4 = params + off_b4(K);
    if (tid < 2 * NH) sp[tid] = bfr(pool[(size_t)b * 2 * NH + tid]);
    __syncthreads();
    {   // z = relu(p W3 + b3)
        const int j = tid;
        float a = params[OFF_B3 + j];
        for (int i = 0; i < 2 * NH; ++i) a = fmaf(sp[i], bfr(W3[i * NZ + j]), a);
        sza[j] = a;
        sz[j] = bfr(fmaxf(a, 0.0f));
    }
    __syncthreads();
    if (tid < O) {  // y = z W4 + b4
        float a = b4[tid];
        for (int j = 0; j < NZ; ++j) a = fmaf(sz[j], bfr(W4[j * O + tid]), a);
        sy[tid] = a;
        if (pred) pred[(size_t)b * O + tid] = a;
    }
    if (!targets) return;
    __syncthreads();
    const float* tg = targets + (size_t)b * O;
    if (tid < K * K) {  // cost[pred i][target j]
        const int i = tid / K, j = tid - i * K;
        double c = 0.0;
        for (int q = 0; q < 3; ++q) {
            const double d = (double)sy[3 * i + q] - (double)tg[3 * j + q];
            c += d * d;
        }
        scost[tid] = c;
    }
    __syncthreads();
    if (tid == 0) {
        hungarian(scost, K, spi);
        double L = 0.0;
        for (int j = 0; j < K; ++j) L += scost[spi[j] * K + j];
        ho.loss[b] = L / (double)B;
        for (int j = 0; j < K; ++j) ho.match[(size_t)b * K + j] = spi[j];
    }
    __syncthreads();
    if (tid < O) {  // dy[pi(j)] = 2 (y[pi(j)] - t[j]) / B
        const int i = tid / 3, q = tid - 3 * i;
        int j = 0;
        for (int jj = 0; jj < K; ++jj)
            if (spi[jj] == i) j = jj;
        const float g = 2.0f * (sy[tid] - tg[3 * j + q]) / (float)B;
        sdy[tid] = bfr(g);
        ho.dy[(size_t)b * O + tid] = g;
        ho.dybf[(size_t)b * O + tid] = bfr(g);
    }
    __syncthreads();
    {   // dz = (dy W4^T) * [z_pre > 0]
        const int j = tid;
        float a = 0.0f;
        for (int o = 0; o < O; ++o) a = fmaf(sdy[o], bfr(W4[j * O + o]), a);
        const float g = sza[j] > 0.0f ? a : 0.0f;
        sdz[j] = bfr(g);
        ho.dz[(size_t)b * NZ + j] = g;
        ho.dzbf[(size_t)b * NZ + j] = bfr(g);
        ho.zbf[(size_t)b * NZ + j] = sz[j];
    }
    __syncthreads();
    if (tid < 2 * NH) {  // dpool = dz W3^T
        const int i = tid;
        float a = 0.0f;
        for (int j = 0; j < NZ; ++j) a = fmaf(sdz[j], bfr(W3[i * NZ + j]), a);
        ho.dpool[(size_t)b * 2 * NH + i] = a;
        ho.poolbf[(size_t)b * 2 * NH + i] = sp[i];
    }
}

// ------------------------------------------------------------ net_points_bwd
// One block per instance: back-propagates dpool through the pooling and the
// two per-point layers.  Each wave writes its partial of dW1, db1, dW2, db2
// (layout PT_*) to part[(b * NW + w) * PT_SIZE].
__global__ __launch_bounds__(NT) void net_points_bwd(const float* __restrict__ pts, int P,
                                                     const float* __restrict__ params,
                                                     const float* __restrict__ dpool,
                                                     const int32_t* __restrict__ argmax,
                                                     float* __restrict__ part) {
    __shared__ float sW1[3 * NH];
    __shared__ float sb1[NH];
    __shared__ float sdm[NH];   // dmean / P
    __shared__ float sdx[NH];   // dmax
    __shared__ int sam[NH];     // argmax
    __shared__ __bf16 sh1T[NW][NH][32];   // h1, feature-major
    __shared__ __bf16 sdzT[NW][NH][32];   // dz2, feature-major
    __shared__ __bf16 sdz[NW][32][NH];    // dz2, point-major
    __shared__ float sxT[NW][3][32];      // points, coordinate-major
    const int b = blockIdx.x, tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    for (int i = tid; i < 3 * NH; i += NT) sW1[i] = bfr(params[OFF_W1 + i]);
    if (tid < NH) {
        sb1[tid] = params[OFF_B1 + tid];
        sdm[tid] = dpool[(size_t)b * 2 * NH + tid] / (float)P;
        sdx[tid] = dpool[(size_t)b * 2 * NH + NH + tid];
        sam[tid] = argmax[(size_t)b * NH + tid];
    }
    bf16x8 w2[4][2], w2t[4][2];
    load_w2(params + OFF_W2, false, lane, w2);
    load_w2(params + OFF_W2, true, lane, w2t);
    float b2[2];
#pragma unroll
    for (int t = 0; t < 2; ++t) b2[t] = params[OFF_B2 + 32 * t + (lane & 31)];
    __syncthreads();
    f32x16 gW2T[2][2];   // dW2^T tiles [t (h2 features)][u (h1 features)]
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int u = 0; u < 2; ++u) gW2T[t][u] = zero16();
    float gW1[2][3] = {{0.f, 0.f, 0.f}, {0.f, 0.f, 0.f}};
    float gb1[2] = {0.f, 0.f}, gb2[2] = {0.f, 0.f};
    const float* __restrict__ xb = pts + (size_t)b * P * 3;
    const int hl = lane >> 5, cl = lane & 31;
    for (int tile = w; tile < P / 32; tile += NW) {
        // (a) this lane's point: layer 1, kept feature-major in LDS
        const int m = tile * 32 + cl;
        const float x0 = xb[m * 3], x1 = xb[m * 3 + 1], x2 = xb[m * 3 + 2];
        bf16x8 a[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            a[s] = layer1_bf(sW1, sb1, x0, x1, x2, 16 * s + 8 * hl);
#pragma unroll
            for (int e = 0; e < 8; ++e) sh1T[w][16 * s + 8 * hl + e][cl] = a[s][e];
        }
        if (hl == 0) { sxT[w][0][cl] = x0; sxT[w][1][cl] = x1; sxT[w][2][cl] = x2; }
        // (b) h2 pre-activations; (c) dz2 = (dmean/P + [argmax] dmax) [h2 > 0]
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            f32x16 acc = zero16();
#pragma unroll
            for (int s = 0; s < 4; ++s) acc = mfma(a[s], w2[s][t], acc);
            const int n = 32 * t + cl;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int i = drow(r, lane);
                float g = sdm[n] + (sam[n] == tile * 32 + i ? sdx[n] : 0.0f);
                g = acc[r] + b2[t] > 0.0f ? g : 0.0f;
                gb2[t] += g;
                const __bf16 gb = (__bf16)g;
                sdzT[w][n][i] = gb;
                sdz[w][i][n] = gb;
            }
        }
        wave_sync_lds();
        // (e) dW2^T += dz2^T h1: A = dz2^T [h2 feature][point], B = h1 [point][h1 feature]
#pragma unroll
        for (int sp = 0; sp < 2; ++sp) {
            bf16x8 A[2], Bm[2];
#pragma unroll
            for (int t = 0; t < 2; ++t)
#pragma unroll
                for (int e = 0; e < 8; ++e) A[t][e] = sdzT[w][32 * t + cl][16 * sp + 8 * hl + e];
#pragma unroll
            for (int u = 0; u < 2; ++u)
#pragma unroll
                for (int e = 0; e < 8; ++e) Bm[u][e] = sh1T[w][32 * u + cl][16 * sp + 8 * hl + e];
#pragma unroll
            for (int t = 0; t < 2; ++t)
#pragma unroll
                for (int u = 0; u < 2; ++u) gW2T[t][u] = mfma(A[t], Bm[u], gW2T[t][u]);
        }
        // (f) dh1 = dz2 W2^T: A = dz2 [point][h2 feature], B = W2^T [h2 f][h1 f]
        bf16x8 A2[4];
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int e = 0; e < 8; ++e) A2[s][e] = sdz[w][cl][16 * s + 8 * hl + e];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            f32x16 d1 = zero16();
#pragma unroll
            for (int s = 0; s < 4; ++s) d1 = mfma(A2[s], w2t[s][u], d1);
            // (g) dz1 = dh1 [h1 > 0]; dW1 += x dz1, db1 += dz1
            const int n1 = 32 * u + cl;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int i = drow(r, lane);
                const float g = (float)sh1T[w][n1][i] > 0.0f ? d1[r] : 0.0f;
                gb1[u] += g;
                gW1[u][0] = fmaf(sxT[w][0][i], g, gW1[u][0]);
                gW1[u][1] = fmaf(sxT[w][1][i], g, gW1[u][1]);
                gW1[u][2] = fmaf(sxT[w][2][i], g, gW1[u][2]);
            }
        }
        wave_sync_lds();
    }
    // partials of this wave: lanes l and l+32 share their features
    float* out = part + ((size_t)b * NW + w) * PT_SIZE;
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        float v[5] = {gW1[u][0], gW1[u][1], gW1[u][2], gb1[u], gb2[u]};
#pragma unroll
        for (int q = 0; q < 5; ++q) {
            const float o = __shfl_xor(v[q], 32, 64);
            v[q] = hl == 0 ? v[q] + o : o + v[q];
        }
        if (hl == 0) {
            const int n = 32 * u + cl;
            out[PT_W1 + n] = v[0];
            out[PT_W1 + NH + n] = v[1];
            out[PT_W1 + 2 * NH + n] = v[2];
            out[PT_B1 + n] = v[3];
            out[PT_B2 + n] = v[4];
        }
    }
    // dW2[n1][n2]: tile (t, u) register r of lane l is dW2^T[32t + row][32u + l%32]
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int n2 = 32 * t + drow(r, lane), n1 = 32 * u + cl;
                out[PT_W2 + n1 * NH + n2] = gW2T[t][u][r];
            }
}

// ------------------------------------------------------------ net_reduce
// One thread per parameter: its gradient summed over instances (and waves) in
// index order; then either stored (grad != null) or applied with Adam.
__global__ __launch_bounds__(256) void net_reduce(int B, int K, const float* __restrict__ part,
                                                  HeadOut ho, float* __restrict__ grad,
                                                  float* __restrict__ params,
                                                  float* __restrict__ m, float* __restrict__ v,
                                                  AdamArgs adam) {
    const int O = 3 * K;
    const int n = param_count(K);
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    float g = 0.0f;
    if (p < OFF_W3) {
        const int q = p;  // the wave partials use the parameter layout of W1..b2
        for (int b = 0; b < B; ++b)
            for (int w = 0; w < NW; ++w) g += part[((size_t)b * NW + w) * PT_SIZE + q];
    } else if (p < OFF_B3) {
        const int i = (p - OFF_W3) / NZ, j = (p - OFF_W3) % NZ;
        for (int b = 0; b < B; ++b)
            g = fmaf(ho.poolbf[(size_t)b * 2 * NH + i], ho.dzbf[(size_t)b * NZ + j], g);
    } else if (p < OFF_W4) {
        const int j = p - OFF_B3;
        for (int b = 0; b < B; ++b) g += ho.dz[(size_t)b * NZ + j];
    } else if (p < off_b4(K)) {
        const int j = (p - OFF_W4) / O, o = (p - OFF_W4) % O;
        for (int b = 0; b < B; ++b)
            g = fmaf(ho.zbf[(size_t)b * NZ + j], ho.dybf[(size_t)b * O + o], g);
    } else {
        const int o = p - off_b4(K);
        for (int b = 0; b < B; ++b) g += ho.dy[(size_t)b * O + o];
    }
    if (grad) grad[p] = g;
    if (m) {
        const float mm = adam.beta1 * m[p] + (1.0f - adam.beta1) * g;
        const float vv = adam.beta2 * v[p] + (1.0f - adam.beta2) * g * g;
        m[p] = mm;
        v[p] = vv;
        const float mh = mm / adam.bc1, vh = vv / adam.bc2;
        params[p] -= adam.lr * mh / (sqrtf(vh) + adam.eps);
    }
}

// ------------------------------------------------------------ net_gather
// One block: gathers the P sample points idx[0..P) of X (d = 3 rows, stride
// ld), normalises them by their mean and scalar standard deviation and writes
// pts [P][3] and stats {mean0..2, s}.  Each thread keeps its points in
// registers (up to GATHER_PER points, all loads in flight together); float64
// sums per thread, then across each wave by a fixed butterfly and across
// the waves in order, so the result repeats bit for bit.
constexpr int GATHER_PER = GATHER_MAX / NT;
static_assert(GATHER_PER * NT == GATHER_MAX, "the sample must split evenly over the block");

__device__ __forceinline__ double block_sum_fixed(double v, double* sw) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sw[threadIdx.x >> 6] = v;
    __syncthreads();
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < NW; ++w) t += sw[w];
    return t;
}

__global__ __launch_bounds__(NT) void net_gather(const float* __restrict__ X, int64_t ld,
                                                 int64_t N, const int32_t* __restrict__ idx,
                                                 int P, float* __restrict__ pts,
                                                 double* __restrict__ stats) {
    __shared__ double sw[NW];
    const int tid = threadIdx.x;
    float v[GATHER_PER][3];
#pragma unroll
    for (int u = 0; u < GATHER_PER; ++u) {
        const int i = tid + u * NT;
        int64_t k = i < P ? idx[i] : 0;
        k = k < 0 ? 0 : (k >= N ? N - 1 : k);
#pragma unroll
        for (int q = 0; q < 3; ++q) v[u][q] = i < P ? X[q * ld + k] : 0.0f;
    }
    double mean[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        double s = 0.0;
#pragma unroll
        for (int u = 0; u < GATHER_PER; ++u) s += (double)v[u][q];
        mean[q] = block_sum_fixed(s, sw) / (double)P;
    }
    double s2 = 0.0;
#pragma unroll
    for (int u = 0; u < GATHER_PER; ++u)
        if (tid + u * NT < P)
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                const double dv = (double)v[u][q] - mean[q];
                s2 += dv * dv;
            }
    double sd = sqrt(block_sum_fixed(s2, sw) / (3.0 * (double)P));
    if (!(sd > 0.0)) sd = 1.0;
    if (tid == 0) {
        stats[0] = mean[0];
        stats[1] = mean[1];
        stats[2] = mean[2];
        stats[3] = sd;
    }
#pragma unroll
    for (int u = 0; u < GATHER_PER; ++u) {
        const int i = tid + u * NT;
        if (i < P)
#pragma unroll
            for (int q = 0; q < 3; ++q) pts[(size_t)i * 3 + q] = (float)(((double)v[u][q] - mean[q]) / sd);
    }
}

// ------------------------------------------------------------ inference head
// Inference of one instance whose P points were pooled as S equal slices
// (net_points_fwd with B = S): pool = [mean of the slice means, max of the
// slice maxima].  net_infer_z: block b computes z[j] for the 16 outputs
// j in [16 b, 16 b + 16), 16 threads per output each summing 8 of the 128
// inputs (all 8 weight loads in flight), combined by a fixed butterfly.
// net_infer_y: one block, y = z W4 + b4, the outputs' inputs split the same
// way.  Operands rounded to bfloat16 as in net_head.
__global__ __launch_bounds__(NT) void net_infer_z(const float* __restrict__ part, int S,
                                                  const float* __restrict__ params,
                                                  float* __restrict__ z) {
    __shared__ float sp[2 * NH];
    const int tid = threadIdx.x;
    if (tid < 2 * NH) {
        float a;
        if (tid < NH) {
            a = 0.0f;
            for (int s = 0; s < S; ++s) a += part[(size_t)s * 2 * NH + tid];
            a /= (float)S;
        } else {
            a = -INFINITY;
            for (int s = 0; s < S; ++s) a = fmaxf(a, part[(size_t)s * 2 * NH + tid]);
        }
        sp[tid] = bfr(a);
    }
    __syncthreads();
    const int j = blockIdx.x * 16 + (tid >> 4), l = tid & 15;
    const float* W3 = params + OFF_W3;
    float w[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) w[u] = W3[(size_t)(8 * l + u) * NZ + j];
    float acc = 0.0f;
#pragma unroll
    for (int u = 0; u < 8; ++u) acc = fmaf(sp[8 * l + u], bfr(w[u]), acc);
#pragma unroll
    for (int o = 8; o >= 1; o >>= 1) acc += __shfl_xor(acc, o, 16);
    if (l == 0) z[j] = bfr(fmaxf(acc + params[OFF_B3 + j], 0.0f));
}

__global__ __launch_bounds__(NT) void net_infer_y(const float* __restrict__ z, int K,
                                                  const float* __restrict__ params,
                                                  float* __restrict__ pred) {
    __shared__ float sz[NZ];
    __shared__ float sacc[NT];
    const int tid = threadIdx.x;
    const int O = 3 * K;
    sz[tid] = z[tid];                        // NT == NZ
    __syncthreads();
    // 4 threads per output (O <= 48 <= 64), 64 inputs each
    const int o = tid >> 2, l = tid & 3;
    const float* W4 = params + OFF_W4;
    float acc = 0.0f;
    if (o < O) {
        for (int j0 = 64 * l; j0 < 64 * l + 64; j0 += 16) {
            float w[16];
#pragma unroll
            for (int u = 0; u < 16; ++u) w[u] = W4[(size_t)(j0 + u) * O + o];
#pragma unroll
            for (int u = 0; u < 16; ++u) acc = fmaf(sz[j0 + u], bfr(w[u]), acc);
        }
    }
    sacc[tid] = acc;
    __syncthreads();
    if (tid < O) {
        const float* a = &sacc[4 * tid];
        pred[tid] = ((a[0] + a[1]) + (a[2] + a[3])) + params[off_b4(K) + tid];
    }
}

}  // namespace

hipError_t launch_points_fwd(const float* pts, int B, int P, const float* params, float* pool,
                             int32_t* argmax, hipStream_t s) {
    hipLaunchKernelGGL(net_points_fwd, dim3(B), dim3(NT), 0, s, pts, P, params, pool, argmax);
    return hipGetLastError();
}

hipError_t launch_head(const float* pool, int B, int K, const float* params, const float* targets,
                       float* pred, const HeadOut& ho, hipStream_t s) {
    hipLaunchKernelGGL(net_head, dim3(B), dim3(NT), 0, s, pool, B, K, params, targets, pred, ho);
    return hipGetLastError();
}

hipError_t launch_points_bwd(const float* pts, int B, int P, const float* params,
                             const float* dpool, const int32_t* argmax, float* part,
                             hipStream_t s) {
    hipLaunchKernelGGL(net_points_bwd, dim3(B), dim3(NT), 0, s, pts, P, params, dpool, argmax,
                       part);
    return hipGetLastError();
}

hipError_t launch_reduce(int B, int K, const float* part, const HeadOut& ho, float* grad,
                         float* params, float* m, float* v, const AdamArgs& adam, hipStream_t s) {
    const int n = param_count(K);
    hipLaunchKernelGGL(net_reduce, dim3((n + 255) / 256), dim3(256), 0, s, B, K, part, ho, grad,
                       params, m, v, adam);
    return hipGetLastError();
}

hipError_t launch_infer_head(const float* part, int S, int K, const float* params, float* z,
                             float* pred, hipStream_t s) {
    hipLaunchKernelGGL(net_infer_z, dim3(NZ / 16), dim3(NT), 0, s, part, S, params, z);
    hipLaunchKernelGGL(net_infer_y, dim3(1), dim3(NT), 0, s, z, K, params, pred);
    return hipGetLastError();
}

hipError_t launch_gather(const float* X, int64_t ld, int64_t N, const int32_t* idx, int P,
                         float* pts, double* stats, hipStream_t s) {
    hipLaunchKernelGGL(net_gather, dim3(1), dim3(NT), 0, s, X, ld, N, idx, P, pts, stats);
    return hipGetLastError();
}

}  // namespace net
}  // namespace km
