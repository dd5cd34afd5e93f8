// peaks.hip -- measured issue rates of the VALU instructions the reassignment
// scan is made of, and the HBM read rate, on the device at hand.  The
// roofline uses the published peaks; these measurements say how much of the
// published FP32 figure the non-packed instructions can reach.
//
// Each probe kernel runs many independent dependency chains per lane (16), a
// grid of 16 waves per SIMD, and writes one value per lane so that no work can
// be removed.  Every instruction is issued through inline assembly with
// register operands only, so that the instruction measured is exactly the one
// the kernels issue.  On gfx950 the FP32 add, multiply and FMA issue at up to
// twice the rate of the compare, select, min3 and med3 instructions.
#include "ctx.h"

namespace {

constexpr int PB = 256;

constexpr int CHAINS = 16;

template <int OP>
__global__ __launch_bounds__(PB) void issue_probe(float* __restrict__ out, int iters, float a0,
                                                  float b0) {
    float x[CHAINS];
    // operands in VGPRs (lane-dependent values)
    const float a = a0 + (float)(threadIdx.x & 1) * 1e-7f;
    const float b = b0 + (float)(threadIdx.x & 2) * 1e-7f;
#pragma unroll
    for (int u = 0; u < CHAINS; ++u) x[u] = (float)(threadIdx.x & 7) * 0.125f + (float)u;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int u = 0; u < CHAINS; ++u) {
            if constexpr (OP == 0) {
                asm volatile("v_fma_f32 %0, %0, %1, %2" : "+v"(x[u]) : "v"(a), "v"(b));
            } else if constexpr (OP == 1) {
                asm volatile("v_min3_f32 %0, %0, %1, %2" : "+v"(x[u]) : "v"(a), "v"(b));
            } else {
                asm volatile("v_med3_f32 %0, %0, %1, %2" : "+v"(x[u]) : "v"(a), "v"(b));
            }
        }
    }
    float s = 0.0f;
#pragma unroll
    for (int u = 0; u < CHAINS; ++u) s += x[u];
    out[(size_t)blockIdx.x * PB + threadIdx.x] = s;
}

__global__ __launch_bounds__(PB) void read_probe(const float4* __restrict__ src, size_t n4,
                                                 float* __restrict__ out) {
    float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
    for (size_t i = (size_t)blockIdx.x * PB + threadIdx.x; i < n4; i += (size_t)gridDim.x * PB) {
        const float4 v = src[i];
        acc.x += v.x; acc.y += v.y; acc.z += v.z; acc.w += v.w;
    }
    out[(size_t)blockIdx.x * PB + threadIdx.x] = acc.x + acc.y + acc.z + acc.w;
}

}  // namespace

extern "C" int kmeans_measure_peaks(kmeans_ctx* c, double* rates) {
    if (!c) return KM_EINVAL;
    c->err.clear();
    if (!rates) return km::fail(c, KM_EINVAL, "rates is NULL");
    KM_HIP(c, hipSetDevice(c->device));
    const int grid = c->n_cu * 16;         // 16 blocks of 4 waves per CU: 16 waves per SIMD
    const int iters = 2048;
    const size_t read_bytes = (size_t)1 << 30;
    float* out = nullptr;
    float4* src = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = KM_OK;
    if (hipMalloc(&out, sizeof(float) * (size_t)grid * PB) != hipSuccess ||
        hipMalloc(&src, read_bytes) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
        hipEventCreate(&e1) != hipSuccess) {
        rc = km::fail(c, KM_ENOMEM, "allocation for the peak probes failed");
    }
    if (!rc && hipMemsetAsync(src, 0, read_bytes, c->stream) != hipSuccess)
        rc = km::fail(c, KM_EHIP, "hipMemsetAsync failed");
    for (int op = 0; op < 4 && !rc; ++op) {
        float best = 1e30f;
        for (int rep = 0; rep < 3 && !rc; ++rep) {
            (void)hipEventRecord(e0, c->stream);
            if (op == 0) hipLaunchKernelGGL(issue_probe<0>, dim3(grid), dim3(PB), 0, c->stream, out, iters, 0.999f, 0.001f);
            else if (op == 1) hipLaunchKernelGGL(issue_probe<1>, dim3(grid), dim3(PB), 0, c->stream, out, iters, 3.0f, 5.0f);
            else if (op == 2) hipLaunchKernelGGL(issue_probe<2>, dim3(grid), dim3(PB), 0, c->stream, out, iters, 3.0f, 5.0f);
            else hipLaunchKernelGGL(read_probe, dim3(grid), dim3(PB), 0, c->stream, src, read_bytes / 16, out);
            (void)hipEventRecord(e1, c->stream);
            if (hipGetLastError() != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
                rc = km::fail(c, KM_EHIP, "peak probe %d failed", op);
                break;
            }
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            best = ms < best ? ms : best;
        }
        if (!rc) {
            const double s = best * 1e-3;
            rates[op] = op < 3 ? (double)grid * PB * iters * CHAINS / s : (double)read_bytes / s;
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (out) (void)hipFree(out);
    if (src) (void)hipFree(src);
    return rc;
}
