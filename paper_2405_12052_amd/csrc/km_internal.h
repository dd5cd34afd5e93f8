// km_internal.h -- device-resident state and launcher declarations shared by
// the kernels (lloyd_kernels.hip) and the host runtime (kmeans_api.hip).
// Internal to libkmeans_mi355x.so; the public interface is include/kmeans.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace km {

constexpr int KMAX = 64;          // largest K of a single fit
constexpr int DMAX = 3;           // points are 2-D or 3-D (problem statement)
constexpr int BLOCK = 256;        // threads per block of the point kernels
constexpr int MAX_BLOCKS = 4096;  // grid cap (size of the per-block partials)
constexpr int GROUP = 32;         // blocks per first-level reduction group
constexpr int MAX_GROUPS = MAX_BLOCKS / GROUP;
constexpr int KPAD = 66;          // KMAX rounded up to whole triples of centres
constexpr int PART = KMAX * (DMAX + 1);  // int64 slots of one block partial

// Status flags written by the device.
// Fixed-point cluster sums (see lloyd_device.h): |q| < 2^FXP_BITS per
// coordinate, at most FXP_BLOCK_POINTS points per int64 slot of a block, data
// with max|x| >= 2^28 (FXP_RANGE_BITS, float32 bits) refused by fits.
constexpr int FXP_BITS = 44;
constexpr int64_t FXP_BLOCK_POINTS = (int64_t)1 << 19;
constexpr uint32_t FXP_RANGE_BITS = 0x4d800000u;

// FLAG_RANGE: max|x| >= 2^28, beyond the range in which the fixed-point
// cluster sums guarantee the centre tolerance (lloyd_device.h); fits stop
// before their first update.
enum : int32_t { FLAG_NONFINITE = 1, FLAG_TIMEOUT = 2, FLAG_RANGE = 4 };

// One fit (or one reassignment pass) lives in this struct in device memory.
// The host writes the problem fields and the initial centres before the
// first kernel; afterwards only kernels write it, and the host reads back
// the progress block with one small copy per batch of iterations.
struct alignas(16) State {
    // ---- problem (host-written) ----
    const float* X;        // d rows of N float32, row j at X + j*ld
    int64_t N;
    int64_t ld;
    int32_t d;
    int32_t K;
    double tol;            // stop once E < tol
    int32_t max_iter;
    int32_t hist_cap;      // entries of E_hist / J_hist
    double* jpart;         // [MAX_BLOCKS] per-block objective partials
    unsigned long long* part;   // [MAX_BLOCKS][PART] per-block sums | counts (int64)
    unsigned long long* gpart;  // [MAX_GROUPS][PART][2] per-group sums | counts (128-bit:
                                // lo, hi)
    double* gjpart;        // [MAX_GROUPS] per-group objective partials
    uint32_t* gticket;     // [MAX_GROUPS] blocks finished per group
    double* E_hist;        // [hist_cap]
    double* J_hist;        // [hist_cap]
    int32_t* track;        // indicator tracking (KM_OPT_TRACK): every update reads
                           // each point's previous label here and writes its new
                           // one (N int32, -1 before the first update); null: off
    int64_t* C_hist;       // [hist_cap] labels changed per update (with track)
    // ---- progress (device-written; read back by the host) ----
    int32_t t;             // updates performed
    int32_t done;          // 1: no further update runs
    int32_t flags;         // FLAG_*
    int32_t xe;            // ilogb(max|x|) (-1 for all-zero data): the fixed-point
                           // exponent of the per-cluster sums is 43 - xe
    double E;              // E of the last update
    double J;              // objective of the last reassignment-only pass
    int64_t empty_events;  // clusters left empty, summed over updates
    int64_t changed;       // labels changed by the last update (with track)
    float minus_inf;       // -infinity, read at run time by the kernels
    int32_t pad1;
    // ---- device scratch ----
    uint32_t absmax_bits;  // max |x| over the data, as float bits
    uint32_t ticket;       // blocks finished in the current kernel
    uint32_t scan_ticket;  // blocks finished in the scan kernel
    uint32_t gen;          // updates published by a persistent fit
    // ---- centres ----
    double mu64[KMAX * DMAX];          // float64 centres, row-major K x d
    float4 mu32[KMAX];                 // the same rounded to float32, padded
    // ---- derived from mu32 on the device before each reassignment ----
    float4 cand[KPAD];                 // {-2 m0, -2 m1, -2 m2, fl32(|m|^2)}; pads
                                       // {0, 0, 0, 2^127} up to a whole triple
    float4 bnd;                        // {2^-20 Cmax, 2^-19 A0, 2^-19 A1, 2^-19 A2}
};

// Bytes of State the host uploads (problem, progress and centres) and the
// progress block it reads back.
constexpr size_t kUploadBytes = offsetof(State, cand);
constexpr size_t kProgressOffset = offsetof(State, t);
constexpr size_t kProgressBytes = offsetof(State, absmax_bits) - offsetof(State, t);

// ---------------------------------------------------------------- batched fit
// Many independent instances, each with up to BK_RMAX restarts (independent
// Lloyd runs from different initial centres), in one persistent launch.
constexpr int BK_KMAX = 32;                        // K per restart
constexpr int BK_RMAX = 8;                         // restarts per instance
constexpr int BK_KPAD = 33;                        // BK_KMAX rounded up to triples
constexpr int BK_PART = BK_RMAX * BK_KMAX * (DMAX + 1);  // int64 per block partial
constexpr int BK_TEAM_MAX = 16;                    // blocks per team
constexpr int64_t BK_NMAX = (int64_t)1 << 27;      // points per instance

struct BInst {                 // one instance (host-written)
    const float* X;            // d rows of N float32, row j at X + j*ld
    int64_t N;
    int64_t ld;
    int32_t d, K, R, vec;      // vec: 16-byte aligned rows
    int32_t* labels;           // device labels of the best restart, or null
    const double* init;        // device, R*K*d initial centres
};

struct BOut {                  // one (instance, restart) result (device-written)
    int32_t iters;
    int32_t converged;
    int64_t empty_events;
    double E;                  // E of the last update
    double J;                  // objective at the final centres
};

struct alignas(64) BTeam {     // one team of blocks
    uint32_t bar;              // barrier arrivals (monotonic within a launch)
    int32_t inst;              // instance the team works on, -1 when none is left
    uint32_t pad[14];
};

struct BatchState {
    const BInst* inst;         // [n_inst]
    const int32_t* order_big;  // instances processed by teams, largest first
    const int32_t* order_small;// instances processed by single blocks, largest first
    int32_t n_inst, n_big, n_small;
    int32_t team_size;         // blocks per team (1 = no teams)
    int32_t mfma_min_k;        // instances with K >= this take the matrix-core keys
    int32_t n_teams;
    int32_t max_iter;
    double tol;
    float minus_inf;
    int32_t error;             // 1: a team barrier timed out
    uint32_t big_ctr;          // next entry of order_big
    uint32_t small_ctr;        // next entry of order_small
    uint32_t* absmax;          // [n_inst] max |x| bits per instance
    BOut* out;                 // [n_inst][BK_RMAX]
    int32_t* best;             // [n_inst] restart with the smallest objective
    double* best_mu;           // [n_inst][BK_KMAX * DMAX] its final centres
    unsigned long long* tpart; // [n_teams][2][team_size][BK_PART][2] (128-bit: lo, hi)
    unsigned long long* fold;  // [grid][BK_PART][2] block-private 128-bit chunk sums
    double* tjpart;            // [n_teams][2][team_size][BK_RMAX]
    BTeam* teams;              // [n_teams]
};

hipError_t launch_batched_scan(BatchState* bs, int n_inst, int grid, hipStream_t s);
hipError_t launch_batched_fit(BatchState* bs, int grid, hipStream_t s, bool cooperative);
int batched_max_blocks_per_cu();

// Launchers (lloyd_kernels.hip).  `vec`: X is 16-byte aligned with ld % 4 == 0.
// `keys`: 0 = VALU scan, 1 / 2 = matrix-core scan with 1 / 2 tiles of 32 centres.
hipError_t launch_scan(State* st, int d, bool vec, int grid, hipStream_t s);
hipError_t launch_iter(State* st, int d, bool vec, int keys, bool track, int grid,
                       hipStream_t s);
hipError_t launch_label(State* st, int32_t* labels, int d, bool vec, int keys, int grid,
                        hipStream_t s);
// The whole fit as one cooperative launch (VALU scan); grid must fit on the
// device at persist_max_blocks_per_cu blocks per compute unit.
hipError_t launch_persist(State* st, int d, bool vec, int grid, hipStream_t s);
int persist_max_blocks_per_cu(int d, bool vec);

}  // namespace km
