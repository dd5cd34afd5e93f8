// wide.h -- device state and launchers of the general-shape fit: any d in
// [1, WD_MAX] and K in [1, WK_MAX] whose per-block tables fit in LDS (the
// single-fit kernels of lloyd_kernels.hip cover d in {2, 3}, K <= 64).
// Internal to libkmeans_mi355x.so; the public interface is include/kmeans.h.
//
// The method is the same Lloyd iteration (the paper's "The Lloyd's
// Algorithm" and "Serial Lloyd's Algorithm"): reassignment by the first-index
// argmin of the squared distance to the float32 centres in the direct form
// evaluated in float64 (found through a certified expanded key, see
// wide_kernels.hip), per-cluster exact integer sums of rint(x 2^F)
// (lloyd_device.h), the float64 mean step with the empty-cluster rule, E and
// the tolerance test.  Per update two kernels run: wide_update (reassignment and
// per-block sums) and wide_reduce (the partials summed into the totals by the
// whole grid, then the mean step and the next pass's key tables in the last
// block).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace km {

constexpr int WD_MAX = 32;        // largest d
constexpr int WK_MAX = 4096;      // largest K
constexpr int WBLOCK = 256;       // threads per block of the wide kernels
constexpr int WMAX_GRID = 4096;   // cap of the update grid (rows of partials)
constexpr int WCHUNK = 32;        // partials summed per thread in wide_reduce
constexpr int WLDS_MAX = 65536;   // dynamic LDS of one wide_update block
constexpr int WQCAP = 128;        // re-scan queue entries per wave

// Compiled point widths: d is padded with zero coordinates up to the next of
// these (zeros add exactly nothing to a squared distance).
__host__ __device__ constexpr int wide_width(int d) {
    return d <= 4 ? d : d <= 6 ? 6 : d <= 8 ? 8 : d <= 12 ? 12 : d <= 16 ? 16 : d <= 24 ? 24 : 32;
}
// Floats per centre in LDS (the width rounded up to whole float4s).
__host__ __device__ constexpr int wide_stride(int D) { return (D + 3) & ~3; }

// Centres padded to whole triples (the scan takes them three at a time).
__host__ __device__ constexpr int wide_kpad(int K) { return 3 * ((K + 2) / 3); }

// LDS of the key tables and queues, shared by wide_update and wide_label:
// float32 centres Kpad * stride, the keys' constants Kpad (rounded to 16
// bytes), the bound coefficients (WD_MAX + 1, padded to 36), the per-wave
// re-scan queues and the per-wave objective partials.
__host__ __device__ constexpr size_t wide_table_bytes(int d, int K) {
    return (size_t)wide_kpad(K) * wide_stride(wide_width(d)) * 4 +
           (((size_t)wide_kpad(K) * 4 + 15) & ~(size_t)15) + 36 * 4 +
           (size_t)(WBLOCK / 64) * WQCAP * 4 + (WBLOCK / 64) * 8;
}

// LDS bytes of one wide_update block for (d, K): integer sums and counts
// K * (d + 1) int64 (rounded to 16 bytes), then the tables.
__host__ __device__ constexpr size_t wide_lds_bytes(int d, int K) {
    return (((size_t)K * (d + 1) * 8 + 15) & ~(size_t)15) + wide_table_bytes(d, K);
}

// Shapes whose sums and tables exceed WLDS_MAX take the tiled kernels: the
// centres pass through LDS in tiles of wide_tile_k(stride) rows (whole
// chunks of 32 triples, about 24 KB), the sums go to the block's row of
// partials in device memory.
__host__ __device__ constexpr int wide_tile_k(int DS) {
    return 96 * ((6144 / (96 * DS)) > 0 ? (6144 / (96 * DS)) : 1);
}
__host__ __device__ constexpr bool wide_tiled(int d, int K) {
    return wide_lds_bytes(d, K) > (size_t)WLDS_MAX;
}
// LDS of a tiled block: one tile of float32 centres and constants, the bound
// coefficients (36 floats), the per-wave re-scan queues and objective sums.
__host__ __device__ constexpr size_t wide_tiled_lds_bytes(int d) {
    return (size_t)wide_tile_k(wide_stride(wide_width(d))) * wide_stride(wide_width(d)) * 4 +
           (((size_t)wide_tile_k(wide_stride(wide_width(d))) * 4 + 15) & ~(size_t)15) + 36 * 4 +
           (size_t)(WBLOCK / 64) * WQCAP * 4 + (WBLOCK / 64) * 8;
}

// The matrix-core keys (wide_kernels.hip) for widths 8, 12 and 16: per tile
// of 32 centres, S k-steps of A operands (S = ceil(3 (width / 2) / 8): 2 at
// width 8, 3 at 12 and 16; 1 KB per step) and 32 accumulator inputs in LDS,
// in place of the float32 centre table.
__host__ __device__ constexpr bool wide_mfma_width(int d) {
    return wide_width(d) == 8 || wide_width(d) == 12 || wide_width(d) == 16;
}
__host__ __device__ constexpr int wide_mfma_steps(int d) {
    return (3 * (wide_width(d) / 2) + 7) / 8;
}
// LDS of the reassignment-only kernel: operands, accumulator inputs, bound
// coefficients, the two levels of re-scan queues and objective sums.
__host__ __device__ constexpr size_t wide_mfma_table_bytes(int d, int K) {
    return (size_t)((K + 31) / 32) * wide_mfma_steps(d) * 1024 + (size_t)((K + 31) / 32) * 128 +
           36 * 4 + (size_t)(WBLOCK / 64) * WQCAP * 4 * 2 + (WBLOCK / 64) * 8;
}
// LDS of the update kernel: the integer sums and counts first (rounded to 64
// bytes), then the tables.
__host__ __device__ constexpr size_t wide_mfma_lds_bytes(int d, int K) {
    return (((size_t)K * (d + 1) * 8 + 63) & ~(size_t)63) + wide_mfma_table_bytes(d, K);
}
__host__ __device__ constexpr bool wide_mfma_fits(int d, int K) {
    return wide_mfma_width(d) && wide_mfma_lds_bytes(d, K) <= (size_t)WLDS_MAX;
}

struct alignas(16) WState {
    // ---- problem (host-written) ----
    const float* X;        // d rows of N float32, row j at X + j*ld
    int64_t N;
    int64_t ld;
    int32_t d;
    int32_t K;
    double tol;            // stop once E < tol
    int32_t max_iter;
    int32_t hist_cap;      // entries of E_hist / J_hist
    int32_t grid;          // blocks of wide_update (rows of part)
    int32_t vec;           // rows 16-byte aligned and ld % 4 == 0
    double* mu64;          // [K * d] float64 centres, row-major
    float* mu32;           // [Kpad * stride] the same rounded to float32, zero padded
                           // (coordinates past d, rows past K up to a whole triple)
    float* hh;             // [Kpad] -|m_k|^2 / 2 of the float32 centres (pads: -2^127)
    float* amax;           // [WD_MAX + 1] max_k |m_kj| for j < d; [WD_MAX]: max_k |m_k|^2
    unsigned long long* part;  // [grid][K * (d + 1)] per-block sums | counts (int64;
                               // the tiled kernels add into it directly)
    unsigned long long* tot;   // [2][K * (d + 1)] totals as two limbs, value =
                               // tot[1][i] 2^32 + tot[0][i] (zero between updates)
    double* jpart;         // [grid] per-block objective partials
    double* E_hist;        // [hist_cap]
    double* J_hist;        // [hist_cap]
    int32_t* track;        // indicator tracking: previous labels (N int32, -1 before
                           // the first update), rewritten by every update; null: off
    int64_t* C_hist;       // [hist_cap] labels changed per update (with track)
    // ---- progress (device-written; read back by the host) ----
    int32_t t;             // updates performed
    int32_t done;          // 1: no further update runs
    int32_t flags;         // FLAG_* (km_internal.h)
    int32_t pad0;
    double E;              // E of the last update
    double J;              // objective of the last reassignment pass
    int64_t empty_events;  // clusters left empty, summed over updates
    int64_t changed;       // labels changed by the last update (with track)
    float plus_inf;        // +infinity, read at run time by the kernels
    int32_t pad1;
    // ---- device scratch ----
    uint32_t absmax_bits;  // max |x| over the data, as float bits (the exponent of
                           // the fixed-point sums, lloyd_device.h)
    uint32_t ticket;       // blocks finished in the current kernel
};

constexpr size_t kWUploadBytes = offsetof(WState, absmax_bits) + 8;
constexpr size_t kWProgressOffset = offsetof(WState, t);
constexpr size_t kWProgressBytes = offsetof(WState, absmax_bits) - offsetof(WState, t);

// Launchers (wide_kernels.hip); each returns hipErrorInvalidValue for a
// shape or grid outside the limits above.
hipError_t launch_wide_scan(WState* st, int grid, hipStream_t s);
hipError_t launch_wide_update(WState* st, int d, int K, bool track, bool mfma, int grid,
                              hipStream_t s);
hipError_t launch_wide_reduce(WState* st, int d, int K, int grid_update, hipStream_t s);
hipError_t launch_wide_label(WState* st, int32_t* labels, int d, int K, bool mfma, int grid,
                             hipStream_t s);
// Resident update blocks per compute unit for (d, K) (the matrix-core kernel
// with mfma, else the tiled kernel when wide_tiled(d, K)); 0 on error.
int wide_blocks_per_cu(int d, int K, bool mfma);

}  // namespace km
