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

// ---------------------------------------------------------------- cross-lane exchange
// Partner values without the LDS round trip of a bpermute (one VALU
// instruction per 32 bits).
//   lane_swap<32>(a, b): lanes 32..63 of a trade places with lanes 0..31 of
//     b (v_permlane32_swap); afterwards a + b holds, in lane l < 32, a(l) +
//     a(l + 32), and in lane l >= 32, b(l - 32) + b(l);
//   lane_swap<16>(a, b): the same within each half of 32 lanes at distance
//     16 (v_permlane16_swap);
//   dpp_partner<O>(v), O = 8, 4, 2, 1: the value of a partner lane on the
//     other side of lane bit O (row mirror l <-> 15 - l, half-row mirror l
//     <-> 7 - l, l ^ 2, l ^ 1; DPP moves).
// In both forms a lane and its partner combine the same two values, so a
// butterfly over bits 32 .. 1 leaves the same total in every lane.
__device__ __forceinline__ void lane_swap32x(unsigned& a, unsigned& b, bool s32)
{
    if (s32) {
        auto r = __builtin_amdgcn_permlane32_swap(a, b, false, false);
        a = r[0];
        b = r[1];
    } else {
        auto r = __builtin_amdgcn_permlane16_swap(a, b, false, false);
        a = r[0];
        b = r[1];
    }
}
template <int S, typename T>
__device__ __forceinline__ void lane_swap(T& a, T& b)
{
    static_assert(S == 32 || S == 16, "lane_swap distance");
    if constexpr (sizeof(T) == 4) {
        unsigned ua = __builtin_bit_cast(unsigned, a), ub = __builtin_bit_cast(unsigned, b);
        lane_swap32x(ua, ub, S == 32);
        a = __builtin_bit_cast(T, ua);
        b = __builtin_bit_cast(T, ub);
    } else {
        const uint64_t ab = __builtin_bit_cast(uint64_t, a), bb = __builtin_bit_cast(uint64_t, b);
        unsigned alo = (unsigned)ab, ahi = (unsigned)(ab >> 32), blo = (unsigned)bb, bhi = (unsigned)(bb >> 32);
        lane_swap32x(alo, blo, S == 32);
        lane_swap32x(ahi, bhi, S == 32);
        a = __builtin_bit_cast(T, ((uint64_t)ahi << 32) | alo);
        b = __builtin_bit_cast(T, ((uint64_t)bhi << 32) | blo);
    }
}
template <int O, typename T>
__device__ __forceinline__ T dpp_partner(T v)
{
    constexpr int CTRL = O == 8 ? 0x140 : O == 4 ? 0x141 : O == 2 ? 0x4E : 0xB1;
    static_assert(O == 8 || O == 4 || O == 2 || O == 1, "dpp_partner distance");
    if constexpr (sizeof(T) == 4) {
        return __builtin_bit_cast(T, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false));
    } else {
        const uint64_t b = __builtin_bit_cast(uint64_t, v);
        const unsigned lo = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)b, CTRL, 0xF, 0xF, false);
        const unsigned hi = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, 0xF, 0xF, false);
        return __builtin_bit_cast(T, ((uint64_t)hi << 32) | lo);
    }
}
// value of the partner across lane bit O (any O in 32 .. 1)
template <int O, typename T>
__device__ __forceinline__ T lane_partner(T v)
{
    if constexpr (O >= 16) {
        T a = v, b = v;
        lane_swap<O>(a, b);
        // lane l < O (within its group of 2 O lanes) now holds its own value
        // in a and the partner's in b; the other lanes the reverse
        return ((threadIdx.x & O) != 0) ? a : b;
    } else {
        return dpp_partner<O>(v);
    }
}

// Sum over the 64 lanes of a wavefront; every lane receives the result.
template <typename T>
__device__ __forceinline__ T wave_sum(T v)
{
    {
        T a = v, b = v;
        lane_swap<32>(a, b);
        v = a + b;
    }
    {
        T a = v, b = v;
        lane_swap<16>(a, b);
        v = a + b;
    }
    v += dpp_partner<8>(v);
    v += dpp_partner<4>(v);
    v += dpp_partner<2>(v);
    v += dpp_partner<1>(v);
    return v;
}

template <typename T>
__device__ __forceinline__ T wave_max(T v)
{
    T o = lane_partner<32>(v);
    v = o > v ? o : v;
    o = lane_partner<16>(v);
    v = o > v ? o : v;
    o = dpp_partner<8>(v);
    v = o > v ? o : v;
    o = dpp_partner<4>(v);
    v = o > v ? o : v;
    o = dpp_partner<2>(v);
    v = o > v ? o : v;
    o = dpp_partner<1>(v);
    v = o > v ? o : v;
    return v;
}

// Value of v in lane l of the wavefront (l uniform; readlane into a scalar
// register).
template <typename T>
__device__ __forceinline__ T lane_value(T v, int l)
{
    if constexpr (sizeof(T) == 8) {
        const uint64_t b = __builtin_bit_cast(uint64_t, v);
        const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, l);
        const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), l);
        return __builtin_bit_cast(T, ((uint64_t)hi << 32) | lo);
    } else {
        return __builtin_bit_cast(T, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), l));
    }
}

// Largest v over the wavefront with its index i (ties: the smaller index);
// every lane receives the pair.
template <int O, typename T, typename I>
__device__ __forceinline__ void argmax_step(T& v, I& i)
{
    const T ov = lane_partner<O>(v);
    const I oi = lane_partner<O>(i);
    if (ov > v || (ov == v && oi < i)) {
        v = ov;
        i = oi;
    }
}
template <typename T, typename I>
__device__ __forceinline__ void wave_argmax(T& v, I& i)
{
    argmax_step<32>(v, i);
    argmax_step<16>(v, i);
    argmax_step<8>(v, i);
    argmax_step<4>(v, i);
    argmax_step<2>(v, i);
    argmax_step<1>(v, i);
}

// Transposing sum of v[0..NB) (NB = 2 .. 32) over the 64 lanes: the total of
// entry e ends in every lane l with (l >> (6 - log2 NB)) & (NB - 1) == e.
// Step s halves the entries a lane carries: lanes with bit 32 >> s set keep
// the upper half, their partners the lower half, each adding the partner's
// copy.  Both candidate sums are formed explicitly (a lane-dependent choice
// between array entries would be lowered to an indexed access over the whole
// array).  Returns the lane's total; v is clobbered.
template <typename T, int NB, int STEP = 0>
__device__ __forceinline__ T wave_transpose_total(T (&v)[NB])
{
    constexpr int LOGNB = NB == 32 ? 5 : NB == 16 ? 4 : NB == 8 ? 3 : NB == 4 ? 2 : 1;
    static_assert((1 << LOGNB) == NB, "NB must be a power of two in 2 .. 32");
    if constexpr (STEP < LOGNB) {
        constexpr int o = 32 >> STEP;
        constexpr int half = NB >> (STEP + 1);
        if constexpr (o >= 16) {
#pragma unroll
            for (int i = 0; i < half; ++i) {
                T a = v[i], b = v[i + half];
                lane_swap<o>(a, b);
                v[i] = a + b;
            }
        } else {
            const bool hi = (threadIdx.x & o) != 0;
#pragma unroll
            for (int i = 0; i < half; ++i) {
                const T lo_sum = v[i] + dpp_partner<o>(v[i]);
                const T hi_sum = v[i + half] + dpp_partner<o>(v[i + half]);
                v[i] = hi ? hi_sum : lo_sum;
            }
        }
        return wave_transpose_total<T, NB, STEP + 1>(v);
    } else {
        T y = v[0];
        if constexpr (LOGNB <= 1) y += lane_partner<16>(y);
        if constexpr (LOGNB <= 2) y += lane_partner<8>(y);
        if constexpr (LOGNB <= 3) y += dpp_partner<4>(y);
        if constexpr (LOGNB <= 4) y += dpp_partner<2>(y);
        if constexpr (LOGNB <= 5) y += dpp_partner<1>(y);
        return y;
    }
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
