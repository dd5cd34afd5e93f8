// Host stand-in for the HIP runtime header, for building the reassignment
// scan's device header (lloyd_device.h) on the CPU in tests: plain C++
// definitions of the vector types, bit casts, thread indices and the few
// builtins that header uses.  One thread, no GPU.
#pragma once

#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <string.h>

#define __device__
#define __host__
#define __global__
#define __shared__ static
#define __forceinline__ inline
#define __launch_bounds__(...)

struct float4 { float x, y, z, w; };
struct float2 { float x, y; };
struct dim3 { unsigned x = 0, y = 0, z = 0; };
inline float4 make_float4(float x, float y, float z, float w) { return float4{x, y, z, w}; }

typedef int hipError_t;
typedef void* hipStream_t;

extern thread_local dim3 threadIdx, blockIdx, blockDim, gridDim;

inline uint32_t __float_as_uint(float f) { uint32_t u; memcpy(&u, &f, 4); return u; }
inline float __uint_as_float(uint32_t u) { float f; memcpy(&f, &u, 4); return f; }
inline int __float_as_int(float f) { int u; memcpy(&u, &f, 4); return u; }
inline float __int_as_float(int u) { float f; memcpy(&f, &u, 4); return f; }
inline long long __double_as_longlong(double d) { long long u; memcpy(&u, &d, 8); return u; }

inline void __syncthreads() {}
template <typename T> inline T __shfl_xor(T v, int, int) { return v; }
inline uint64_t __ballot(int b) { return b ? 1ull : 0ull; }
inline int __popcll(unsigned long long v) { return __builtin_popcountll(v); }

// v_med3_f32: the median of three (no NaN among the scan's operands)
inline float km_host_fmed3f(float a, float b, float c) {
    const float lo = fminf(a, b), hi = fmaxf(a, b);
    return fmaxf(lo, fminf(hi, c));
}
#define __builtin_amdgcn_fmed3f km_host_fmed3f
#define __builtin_amdgcn_wave_barrier() ((void)0)
#define __builtin_amdgcn_s_waitcnt(x) ((void)(x))
#define __builtin_amdgcn_readfirstlane(x) (x)

#define __HIP_MEMORY_SCOPE_WORKGROUP 3
#define __HIP_MEMORY_SCOPE_AGENT 4
template <typename T> inline T __hip_atomic_load(const T* p, int, int) { return *p; }
template <typename T> inline void __hip_atomic_store(T* p, T v, int, int) { *p = v; }
template <typename T, typename U> inline T __hip_atomic_fetch_add(T* p, U v, int, int) {
    T o = *p; *p = (T)(o + (T)v); return o;
}
template <typename T, typename U> inline T __hip_atomic_fetch_max(T* p, U v, int, int) {
    T o = *p; if ((T)v > o) *p = (T)v; return o;
}
