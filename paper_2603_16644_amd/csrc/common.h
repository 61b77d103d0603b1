// Shared device helpers for the gfx950 kernels: status codes, MFMA operand
// types, wavefront reductions and the bump allocator over the caller's
// workspace.  Wavefronts are 64 lanes wide throughout.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/pne.h"

#define PNE_WAVE 64

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef float v16f __attribute__((ext_vector_type(16)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef _Float16 v8h __attribute__((ext_vector_type(8)));
typedef int v8i __attribute__((ext_vector_type(8)));

#define HIP_OK(call)                                                  \
    do {                                                              \
        if ((call) != hipSuccess) return PNE_EHIP;                    \
    } while (0)

namespace pne {

// Sum over the 64 lanes of a wavefront; every lane receives the result.
template <typename T>
__device__ __forceinline__ T wave_sum(T v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, PNE_WAVE);
    return v;
}

template <typename T>
__device__ __forceinline__ T wave_max(T v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        T o = __shfl_xor(v, off, PNE_WAVE);
        v = o > v ? o : v;
    }
    return v;
}

// Block-wide sum for blockDim.x a multiple of 64 (<= 1024).  `red` is a
// __shared__ array of at least blockDim.x/64 elements.  All threads get the
// result.  Contains two barriers.
template <typename T>
__device__ __forceinline__ T block_sum(T v, T* red)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    v = wave_sum(v);
    if (lane == 0) red[w] = v;
    __syncthreads();
    T t = 0;
    for (int i = 0; i < nw; ++i) t += red[i];   // fixed order: deterministic
    __syncthreads();
    return t;
}

// Bump allocator over the caller's workspace (256-byte aligned slices).
struct Arena {
    char* base;
    size_t cap;
    size_t used;
    __host__ Arena(void* p, size_t c) : base((char*)p), cap(c), used(0) {}
    template <typename T>
    __host__ T* take(size_t count)
    {
        size_t bytes = (count * sizeof(T) + 255) & ~(size_t)255;
        T* p = base ? (T*)(base + used) : nullptr;
        used += bytes;
        return p;
    }
    __host__ bool fits() const { return used <= cap; }
};

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

}  // namespace pne
