// Shared device/host definitions of the HIP library (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include <algorithm>

#include "abba.h"

namespace abba {

// ---------------------------------------------------------------- bf16 ---
// Storage-only bfloat16: widened to FP32 on load, rounded to nearest even on
// store (the usual bit-level rounding: add 0x7fff plus the lsb of the kept
// half, then truncate; NaN stays a quiet NaN).
struct bf16 {
    uint16_t bits;
};

__device__ __forceinline__ float to_f32(float v) { return v; }
__device__ __forceinline__ double to_f64(double v) { return v; }
__device__ __forceinline__ float to_f32(bf16 v) { return __uint_as_float(((uint32_t)v.bits) << 16); }

template <typename T> struct acc_of { typedef float type; };
template <> struct acc_of<double> { typedef double type; };

template <typename T> __device__ __forceinline__ typename acc_of<T>::type load_as(const T *p, size_t i);
template <> __device__ __forceinline__ float load_as<float>(const float *p, size_t i) { return p[i]; }
template <> __device__ __forceinline__ double load_as<double>(const double *p, size_t i) { return p[i]; }
template <> __device__ __forceinline__ float load_as<bf16>(const bf16 *p, size_t i) { return to_f32(p[i]); }

__device__ __forceinline__ bf16 f32_to_bf16(float f) {
    uint32_t u = __float_as_uint(f);
    bf16 r;
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) {
        r.bits = (uint16_t)((u >> 16) | 0x0040u);
        return r;
    }
    u += 0x7fffu + ((u >> 16) & 1u);
    r.bits = (uint16_t)(u >> 16);
    return r;
}

template <typename T> __device__ __forceinline__ void store_as(T *p, size_t i, typename acc_of<T>::type v);
template <> __device__ __forceinline__ void store_as<float>(float *p, size_t i, float v) { p[i] = v; }
template <> __device__ __forceinline__ void store_as<double>(double *p, size_t i, double v) { p[i] = v; }
template <> __device__ __forceinline__ void store_as<bf16>(bf16 *p, size_t i, float v) { p[i] = f32_to_bf16(v); }

// ------------------------------------------------------- wave reductions ---
// Butterfly over the 64 lanes of a wavefront.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Block-wide sum for blockDim.x a multiple of 64; `red` holds one slot per
// wave.  Every thread receives the total.  The summation order is fixed
// (wave butterfly, then waves in index order), so results are deterministic.
template <typename T>
__device__ __forceinline__ T block_sum(T v, T *red) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
    v = wave_sum(v);
    __syncthreads();
    if (lane == 0) red[wid] = v;
    __syncthreads();
    T t = 0;
    for (int w = 0; w < nw; ++w) t += red[w];
    return t;
}

}  // namespace abba

// --------------------------------------------------------- host helpers ---
namespace abba {
void set_error(const char *fmt, ...);
int hip_fail(hipError_t e, const char *what);
}  // namespace abba

#define ABBA_HIP(call)                                                         \
    do {                                                                       \
        hipError_t e_ = (call);                                                \
        if (e_ != hipSuccess) return abba::hip_fail(e_, #call);                \
    } while (0)

#define ABBA_LAUNCHED(what)                                                    \
    do {                                                                       \
        hipError_t e_ = hipGetLastError();                                     \
        if (e_ != hipSuccess) return abba::hip_fail(e_, what);                 \
    } while (0)
