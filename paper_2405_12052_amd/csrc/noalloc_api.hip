// noalloc_api.hip -- kmeans_fit_noalloc: the fit of kmeans_fit (2-D/3-D,
// K <= 64) for callers that cannot allocate memory, e.g. serving loops or
// harnesses that forbid hipMalloc.  Everything the fit's kernels need beyond
// the caller's inputs and outputs -- the device state, the per-block and
// per-group partials, the group tickets and a bounded E/J history -- lives in
// one file-scope device array, `scratch`, whose device address is looked up
// once per device (hipGetSymbolAddress) and passed to the kernels.  No call
// allocates device or host memory, creates a graph, a stream or an event:
// the updates are launched one by one on the caller's stream, the initial
// state is copied from a host object on the call's stack, and the results
// are read back into it.
//
// Every call on one device uses that device's one copy of the array, which
// keeps the previous call's contents; calls that overlap on one device (two
// host threads, or two streams) race and give wrong results.  The state and
// the group tickets are written at the start of every call; the partials are
// fully written by each update before they are read.
#include "ctx.h"

#include <math.h>
#include <string.h>

#include <mutex>

namespace km {
namespace {
constexpr size_t align256(size_t n) { return (n + 255) / 256 * 256; }
constexpr int NA_HIST = 1024;  // E/J history entries kept (updates beyond run unrecorded)
// Layout of the scratch array (byte offsets, each 256-byte aligned).
constexpr size_t NA_STATE = 0;
constexpr size_t NA_JPART = align256(NA_STATE + sizeof(State));
constexpr size_t NA_PART = align256(NA_JPART + sizeof(double) * MAX_BLOCKS);
constexpr size_t NA_GPART = align256(NA_PART + sizeof(unsigned long long) * PART * MAX_BLOCKS);
constexpr size_t NA_GJPART = align256(NA_GPART + sizeof(unsigned long long) * 2 * PART * MAX_GROUPS);
constexpr size_t NA_GTICKET = align256(NA_GJPART + sizeof(double) * MAX_GROUPS);
constexpr size_t NA_HIST_OFF = align256(NA_GTICKET + sizeof(uint32_t) * MAX_GROUPS);
constexpr size_t NA_BYTES = align256(NA_HIST_OFF + sizeof(double) * 2 * NA_HIST);
}  // namespace
}  // namespace km

// The fit's device scratch: about 8.6 MB on every device the library runs on,
// held until the process ends.  In host code `scratch` names a host-side
// stand-in, not device memory: only the address from hipGetSymbolAddress is
// used.
static __device__ __align__(256) unsigned char scratch[km::NA_BYTES];

namespace km {
namespace {

constexpr int NA_MAX_DEVICES = 64;
struct DevScratch {
    std::once_flag once;
    int rc = KM_OK;
    unsigned char* ptr = nullptr;   // device address of `scratch` on this device
    int n_cu = 256;
};
DevScratch g_dev[NA_MAX_DEVICES];

// One fill kernel clears the group tickets (no hipMemsetAsync: callers may
// record their work into a graph).
__global__ void clear_words(uint32_t* p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

// The device address of `scratch` on `device` (current), looked up once.
int scratch_for(int device, DevScratch** out) {
    DevScratch& s = g_dev[device];
    std::call_once(s.once, [&]() {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            s.rc = fail(nullptr, KM_EHIP, "hipGetSymbolAddress of the fit's scratch failed: %s",
                        hipGetErrorString(e));
            return;
        }
        s.ptr = static_cast<unsigned char*>(p);
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, device) == hipSuccess && prop.multiProcessorCount > 0)
            s.n_cu = prop.multiProcessorCount;
    });
    if (s.rc != KM_OK) return fail(nullptr, s.rc, "the fit's scratch is unavailable on device %d",
                                   device);
    *out = &s;
    return KM_OK;
}

// Restores the calling thread's current device on every return.
struct DeviceGuard {
    int prev = -1;
    ~DeviceGuard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

#define NA_HIP(call)                                                                       \
    do {                                                                                   \
        hipError_t e_ = (call);                                                            \
        if (e_ != hipSuccess)                                                              \
            return fail(nullptr, KM_EHIP, "%s failed: %s", #call, hipGetErrorString(e_)); \
    } while (0)

}  // namespace
}  // namespace km

extern "C" int kmeans_fit_noalloc(int device, void* hip_stream, const float* X, int64_t N,
                                  int64_t ld, int32_t d, int32_t K, const double* init,
                                  double tol, int32_t max_iter, double* centroids_out,
                                  int32_t* labels_out, km_result* res) {
    using namespace km;
    int rc = validate(nullptr, N, ld, d, K, tol, max_iter);
    if (rc) return rc;
    if ((d != 2 && d != 3) || K > KMAX)
        return fail(nullptr, KM_EUNSUPPORTED,
                    "kmeans_fit_noalloc takes d in {2, 3} and K <= %d (d=%d, K=%d); its scratch "
                    "holds the state of that fit only",
                    KMAX, d, K);
    rc = check_centres(nullptr, init, K, d, "init");
    if (!rc && !centroids_out) rc = fail(nullptr, KM_EINVAL, "centroids_out is NULL");
    if (rc) return rc;
    int n_dev = 0;
    if (hipGetDeviceCount(&n_dev) != hipSuccess || n_dev < 1) {
        (void)hipGetLastError();
        return fail(nullptr, KM_ENODEV, "no HIP device available");
    }
    if (device < 0 || device >= n_dev || device >= NA_MAX_DEVICES)
        return fail(nullptr, KM_ENODEV, "device %d out of range [0, %d)", device,
                    n_dev < NA_MAX_DEVICES ? n_dev : NA_MAX_DEVICES);
    DeviceGuard guard;
    NA_HIP(hipGetDevice(&guard.prev));
    NA_HIP(hipSetDevice(device));
    rc = check_device_ptr(nullptr, X, "X");
    if (!rc && labels_out) rc = check_device_ptr(nullptr, labels_out, "labels_out");
    if (rc) return rc;
    DevScratch* s = nullptr;
    rc = scratch_for(device, &s);
    if (rc) return rc;

    hipStream_t stream = (hipStream_t)hip_stream;
    unsigned char* base = s->ptr;
    State* st = reinterpret_cast<State*>(base + NA_STATE);
    const FitBufs b{reinterpret_cast<double*>(base + NA_JPART),
                    reinterpret_cast<unsigned long long*>(base + NA_PART),
                    reinterpret_cast<unsigned long long*>(base + NA_GPART),
                    reinterpret_cast<double*>(base + NA_GJPART),
                    reinterpret_cast<uint32_t*>(base + NA_GTICKET),
                    reinterpret_cast<double*>(base + NA_HIST_OFF), nullptr, NA_HIST};
    const bool vec = vec_ok(X, ld);
    const int grid = grid_blocks(s->n_cu, 0, N);
    const int U = auto_unroll(N, max_iter);
    const int keys = auto_keys(K);  // the scan kmeans_fit takes by default

    // the initial state, from this call's stack (read back into it at the end)
    State h;
    stage_state(&h, b, X, N, ld, d, K, init, tol, max_iter);
    hipLaunchKernelGGL(clear_words, dim3((MAX_GROUPS + 255) / 256), dim3(256), 0, stream, b.gticket,
                       MAX_GROUPS);
    NA_HIP(hipGetLastError());
    NA_HIP(hipMemcpyAsync(st, &h, kUploadBytes, hipMemcpyHostToDevice, stream));
    NA_HIP(launch_scan(st, d, vec, grid, stream));
    // batches of U updates; the device stops itself once done, the host reads
    // the progress block after each batch (not at all when tol == 0)
    int launched = 0;
    while (launched < max_iter) {
        const int n = (max_iter - launched) < U ? (max_iter - launched) : U;
        for (int i = 0; i < n; ++i) NA_HIP(launch_iter(st, d, vec, keys, false, grid, stream));
        launched += n;
        if (tol > 0.0 && launched < max_iter) {
            NA_HIP(hipMemcpyAsync(reinterpret_cast<char*>(&h) + kProgressOffset,
                                  reinterpret_cast<char*>(st) + kProgressOffset, kProgressBytes,
                                  hipMemcpyDeviceToHost, stream));
            NA_HIP(hipStreamSynchronize(stream));
            if (h.done) break;
        }
    }
    NA_HIP(launch_label(st, labels_out, d, vec, keys, grid, stream));
    NA_HIP(hipMemcpyAsync(reinterpret_cast<char*>(&h) + kProgressOffset,
                          reinterpret_cast<char*>(st) + kProgressOffset,
                          kUploadBytes - kProgressOffset, hipMemcpyDeviceToHost, stream));
    NA_HIP(hipStreamSynchronize(stream));
    if (h.flags & FLAG_NONFINITE) return fail(nullptr, KM_EINVAL, "X holds a NaN or an infinity");
    if (h.flags & FLAG_RANGE) return range_error(nullptr);
    memcpy(centroids_out, h.mu64, sizeof(double) * (size_t)K * d);
    if (res) {
        res->iters = h.t;
        res->converged = h.E < tol ? 1 : 0;
        res->E = h.E;
        res->shift_l2 = sqrt(h.E);
        res->objective = h.J;
        res->empty_events = h.empty_events;
    }
    return KM_OK;
}
