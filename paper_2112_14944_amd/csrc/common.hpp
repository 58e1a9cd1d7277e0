// Shared device helpers and host plumbing for the gfx950 PPR / layout library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pprviz.h"

namespace pprviz {

constexpr int kWave = 64;

// ---------------------------------------------------------------- host side

#define PPRVIZ_HIP_TRY(expr)                          \
    do {                                              \
        hipError_t _e = (expr);                       \
        if (_e != hipSuccess) return PPR_EHIP;        \
    } while (0)

// Returns PPR_EHIP when an earlier asynchronous error is pending on the device.
inline ppr_status pending_error() {
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? PPR_OK : PPR_EHIP;
}

inline ppr_status launch_status() {
    return hipGetLastError() == hipSuccess ? PPR_OK : PPR_EHIP;
}

inline size_t align_up(size_t x, size_t a = 256) { return (x + a - 1) / a * a; }

// Bump allocator over the caller's workspace (no device allocation).
struct WsCursor {
    char* base;
    size_t cap;
    size_t used = 0;
    template <typename T>
    T* take(size_t count) {
        size_t off = align_up(used);
        used = off + align_up(count * sizeof(T));
        if (base == nullptr || used > cap) return nullptr;
        return reinterpret_cast<T*>(base + off);
    }
};

struct WsSize {
    size_t used = 0;
    template <typename T>
    T* take(size_t count) {
        used = align_up(used) + align_up(count * sizeof(T));
        return nullptr;
    }
};

// ---------------------------------------------------------------- device side

// Pointers in the global address space.  Pointers that reach a kernel inside
// a struct are otherwise treated as generic (flat) pointers, whose loads also
// count against the LDS wait counter and so serialize with LDS traffic.
template <typename T>
using gcptr = const T __attribute__((address_space(1)))*;
template <typename T>
using gptr = T __attribute__((address_space(1)))*;
template <typename T>
__device__ __forceinline__ gcptr<T> as_global(const T* p) {
    return (gcptr<T>)p;
}
template <typename T>
__device__ __forceinline__ gptr<T> as_global_w(T* p) {
    return (gptr<T>)p;
}

// Broadcast lane J of every 16-lane DPP row to the whole row (row_newbcast,
// DPP control 0x150 + J on gfx90a and later).
template <int J>
__device__ __forceinline__ int row_bcast(int v) {
    return __builtin_amdgcn_update_dpp(0, v, 0x150 + J, 0xf, 0xf, false);
}
template <int J>
__device__ __forceinline__ float row_bcast(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x150 + J, 0xf, 0xf, false));
}

__device__ __forceinline__ float lds_load(const float* base_bytes_as_float, int byte_off) {
    return *reinterpret_cast<const float*>(reinterpret_cast<const char*>(base_bytes_as_float) + byte_off);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

// Fill kernel (used instead of hipMemsetAsync so that captured graphs replay
// correctly).
template <typename T>
__global__ void fill_kernel(T* __restrict__ p, T value, int64_t count) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < count; i += stride) p[i] = value;
}

template <typename T>
inline void fill(T* p, T value, int64_t count, hipStream_t s) {
    if (count <= 0) return;
    int64_t blocks = (count + 255) / 256;
    if (blocks > 16384) blocks = 16384;
    hipLaunchKernelGGL(fill_kernel<T>, dim3((unsigned)blocks), dim3(256), 0, s, p, value, count);
}

}  // namespace pprviz
