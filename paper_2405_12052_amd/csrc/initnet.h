// initnet.h -- layout and launchers of the learned initialiser's kernels
// (initnet_kernels.hip).  Internal to libkmeans_mi355x.so; the public
// interface is include/kmeans.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace km {
namespace net {

constexpr int NH = 64;      // per-point width
constexpr int NZ = 256;     // head width
constexpr int KMAXN = 16;   // largest K the head predicts

// Parameter layout (floats): W1 [3][64], b1 [64], W2 [64][64], b2 [64],
// W3 [128][256], b3 [256], W4 [256][3K], b4 [3K]; row-major, rows = inputs.
constexpr int OFF_W1 = 0;
constexpr int OFF_B1 = OFF_W1 + 3 * NH;
constexpr int OFF_W2 = OFF_B1 + NH;
constexpr int OFF_B2 = OFF_W2 + NH * NH;
constexpr int OFF_W3 = OFF_B2 + NH;
constexpr int OFF_B3 = OFF_W3 + 2 * NH * NZ;
constexpr int OFF_W4 = OFF_B3 + NZ;
__host__ __device__ constexpr int off_b4(int K) { return OFF_W4 + NZ * 3 * K; }
__host__ __device__ constexpr int param_count(int K) { return off_b4(K) + 3 * K; }

// Per-wave partial of the per-point gradients: the parameter layout of W1..b2.
constexpr int PT_W1 = OFF_W1, PT_B1 = OFF_B1, PT_W2 = OFF_W2, PT_B2 = OFF_B2;
constexpr int PT_SIZE = OFF_W3;

// Per-instance outputs of the head kernel (device arrays, B rows each).
struct HeadOut {
    double* loss;    // [B]      matched loss / B
    int32_t* match;  // [B][K]   predicted centre assigned to each target
    float* dy;       // [B][3K]  dL/dy
    float* dybf;     // [B][3K]  its bf16 rounding
    float* dz;       // [B][256] dL/dz_pre
    float* dzbf;     // [B][256]
    float* zbf;      // [B][256] bf16 z
    float* dpool;    // [B][128] dL/dpool
    float* poolbf;   // [B][128] bf16 pool
};

struct AdamArgs {
    float lr, beta1, beta2, eps;
    float bc1, bc2;  // 1 - beta^step
};

hipError_t launch_points_fwd(const float* pts, int B, int P, const float* params, float* pool,
                             int32_t* argmax, hipStream_t s);
hipError_t launch_head(const float* pool, int B, int K, const float* params, const float* targets,
                       float* pred, const HeadOut& ho, hipStream_t s);
hipError_t launch_points_bwd(const float* pts, int B, int P, const float* params,
                             const float* dpool, const int32_t* argmax, float* part,
                             hipStream_t s);
hipError_t launch_reduce(int B, int K, const float* part, const HeadOut& ho, float* grad,
                         float* params, float* m, float* v, const AdamArgs& adam, hipStream_t s);
hipError_t launch_gather(const float* X, int64_t ld, int64_t N, const int32_t* idx, int P,
                         float* pts, double* stats, hipStream_t s);
// Inference of one instance pooled as S equal slices (launch_points_fwd with
// B = S): head over the combined pool into pred [3K]; z: scratch of NZ floats.
hipError_t launch_infer_head(const float* part, int S, int K, const float* params, float* z,
                             float* pred, hipStream_t s);
constexpr int GATHER_MAX = 4096;   // largest sample launch_gather takes

}  // namespace net
}  // namespace km
