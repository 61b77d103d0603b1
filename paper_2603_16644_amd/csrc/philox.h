// Counter-based Gaussian generator for the sketching matrix Omega.
//
// Philox4x32 with 10 rounds (Salmon, Moraes, Dror, Shaw, SC'11, Section 4):
// two 32x32->64-bit multiplies per round with multipliers 0xD2511F53 and
// 0xCD9E8D57, Weyl key increments 0x9E3779B9 and 0xBB67AE85.
//
// Entry (i, j) of the unscaled s x m sketch for problem `pid`:
//   key = (seed low word, seed high word), counter = (j, i/4, pid, 0);
//   the four output words feed two Box-Muller pairs (Box & Muller 1958):
//   rows 4(i/4)+0,1 from (w0, w1), rows +2,+3 from (w2, w3), with
//   U1 = ((w_a >> 8) + 1) 2^-24, U2 = (w_b >> 8) 2^-24,
//   even row sqrt(-2 ln U1) cos(2 pi U2), odd row sqrt(-2 ln U1) sin(2 pi U2).
// The transform is evaluated in FP32 with the hardware log2/sqrt/sin/cos
// (v_sin/v_cos take their argument in revolutions, so 2 pi U2 is exact).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pne {

struct Gauss4 {
    float z[4];
};

__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r > 0) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
        const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c[0];
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c[2];
        const uint32_t y0 = (uint32_t)(p1 >> 32) ^ c[1] ^ k0;
        const uint32_t y1 = (uint32_t)p1;
        const uint32_t y2 = (uint32_t)(p0 >> 32) ^ c[3] ^ k1;
        const uint32_t y3 = (uint32_t)p0;
        c[0] = y0; c[1] = y1; c[2] = y2; c[3] = y3;
    }
}

__device__ __forceinline__ void box_muller(uint32_t wa, uint32_t wb, float& even, float& odd)
{
    const float u1 = (float)((wa >> 8) + 1u) * 0x1p-24f;   // (0, 1]
    const float u2 = (float)(wb >> 8) * 0x1p-24f;          // [0, 1)
    // -2 ln u1 = -2 ln(2) log2(u1)
    const float rad = __builtin_amdgcn_sqrtf(-1.3862943611198906f * __builtin_amdgcn_logf(u1));
    even = rad * __builtin_amdgcn_cosf(u2);
    odd = rad * __builtin_amdgcn_sinf(u2);
}

// Rows 4q .. 4q+3 of column j.
__device__ __forceinline__ Gauss4 omega_quad(uint64_t seed, uint32_t pid, uint32_t q, uint32_t j)
{
    uint32_t c[4] = {j, q, pid, 0u};
    philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
    Gauss4 g;
    box_muller(c[0], c[1], g.z[0], g.z[1]);
    box_muller(c[2], c[3], g.z[2], g.z[3]);
    return g;
}

}  // namespace pne
