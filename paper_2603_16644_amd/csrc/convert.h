// Round-to-nearest-even conversions from FP32 to the narrow MFMA operand
// formats, written out on the bit patterns so that every conversion is the
// IEEE rounding of the value (no dependence on hardware conversion modes).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pne {

// FP32 -> BF16 (8 significand bits), RNE.  Inputs are finite here.
__device__ __forceinline__ uint16_t f32_to_bf16_bits(float x)
{
    uint32_t u = __float_as_uint(x);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// FP32 -> IEEE binary16, RNE (hardware conversion; default rounding mode).
__device__ __forceinline__ uint16_t f32_to_f16_bits(float x)
{
    _Float16 h = (_Float16)x;
    return __builtin_bit_cast(uint16_t, h);
}

// FP32 -> OCP E4M3 (bias 7, 3 mantissa bits, largest finite 448, no inf),
// RNE with saturation to +-448.
__device__ __forceinline__ uint8_t f32_to_e4m3_bits(float x)
{
    uint32_t sign = (__float_as_uint(x) >> 24) & 0x80u;
    float a = fminf(fabsf(x), 448.0f);
    uint32_t code;
    if (a < 0x1p-6f) {
        // subnormal grid 2^-9: k in 0..8 (k = 8 is the smallest normal, code 8)
        code = (uint32_t)rintf(a * 512.0f);
    } else {
        uint32_t u = __float_as_uint(a);
        int e = (int)((u >> 23) & 0xffu) - 127;      // -6 .. 8
        uint32_t man = u & 0x7fffffu;
        uint32_t r = man >> 20;                      // 3 kept bits
        uint32_t rem = man & 0xfffffu;
        if (rem > 0x80000u || (rem == 0x80000u && (r & 1u))) ++r;
        if (r == 8u) { r = 0u; ++e; }
        code = ((uint32_t)(e + 7) << 3) | r;
    }
    return (uint8_t)(sign | code);
}

}  // namespace pne
