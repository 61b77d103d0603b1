// Single-work-group triangular solve on a vector held in LDS (FP64 or FP32),
// shared by the solve kernels and the condition estimate.
#pragma once
#include "common.h"

namespace pne {

// x (in LDS) := U^{-1} x with U(i, j) = trans ? M[j + i ld] : M[i + j ld];
// `lower` says whether U is lower triangular.  Whole work-group.
template <typename T>
__device__ inline void wg_trsv(int64_t n, const T* __restrict__ M, int64_t ld, bool lower, bool trans,
                        bool unit, T* x)
{
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    auto U = [&](int64_t i, int64_t j) -> T { return trans ? M[j + i * ld] : M[i + j * ld]; };
    if (lower) {
        for (int64_t b0 = 0; b0 < n; b0 += 64) {
            const int bw = (int)((n - b0 < 64) ? n - b0 : 64);
            if (wid == 0) {
                T xi = (lane < bw) ? x[b0 + lane] : (T)0;
                for (int k = 0; k < bw; ++k) {
                    T xk = __shfl(xi, k, 64);
                    if (!unit) xk = xk / U(b0 + k, b0 + k);
                    if (lane == k) xi = xk;
                    if (lane > k && lane < bw) xi -= U(b0 + lane, b0 + k) * xk;
                }
                if (lane < bw) x[b0 + lane] = xi;
            }
            __syncthreads();
            for (int64_t i = b0 + bw + tid; i < n; i += blockDim.x) {
                T s = 0;
                for (int k = 0; k < bw; ++k) s += U(i, b0 + k) * x[b0 + k];
                x[i] -= s;
            }
            __syncthreads();
        }
    } else {
        for (int64_t b1 = n; b1 > 0; b1 -= 64) {
            const int64_t b0 = (b1 - 64 > 0) ? b1 - 64 : 0;
            const int bw = (int)(b1 - b0);
            if (wid == 0) {
                T xi = (lane < bw) ? x[b0 + lane] : (T)0;
                for (int k = bw - 1; k >= 0; --k) {
                    T xk = __shfl(xi, k, 64);
                    if (!unit) xk = xk / U(b0 + k, b0 + k);
                    if (lane == k) xi = xk;
                    if (lane < k) xi -= U(b0 + lane, b0 + k) * xk;
                }
                if (lane < bw) x[b0 + lane] = xi;
            }
            __syncthreads();
            for (int64_t i = tid; i < b0; i += blockDim.x) {
                T s = 0;
                for (int k = 0; k < bw; ++k) s += U(i, b0 + k) * x[b0 + k];
                x[i] -= s;
            }
            __syncthreads();
        }
    }
}


}  // namespace pne
