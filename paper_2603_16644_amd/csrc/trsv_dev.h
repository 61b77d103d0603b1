// Single-work-group triangular solves on a vector held in LDS (FP64 or FP32),
// shared by the solve kernels and the condition estimate.  wg_trsv: blocked by 64:
// the diagonal block is staged in LDS and solved by one wavefront (lane i
// holds x_i; each step finalises one entry and removes it from the later
// ones), then all threads update the remaining entries with the block's
// columns.  wg_trsv_inv: the same blocking with the diagonal blocks applied
// through their precomputed inverses (one small matrix-vector product per
// block instead of 64 dependent steps).
#pragma once
#include "common.h"

namespace pne {

constexpr int TB = 64, TBL = TB + 1;  // diagonal block and its LDS leading dimension

// x (in LDS) := U^{-1} x with U(i, j) = trans ? M[j + i ld] : M[i + j ld];
// `lower` says whether U is lower triangular.  `dblk` is LDS scratch of
// TB * TBL elements.  Whole work-group.
template <typename T>
__device__ inline void wg_trsv(int64_t n, const T* __restrict__ M, int64_t ld, bool lower, bool trans,
                               bool unit, T* x, T* dblk)
{
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    auto U = [&](int64_t i, int64_t j) -> T { return trans ? M[j + i * ld] : M[i + j * ld]; };
    const int64_t nb = (n + TB - 1) / TB;
    for (int64_t bb = 0; bb < nb; ++bb) {
        const int64_t blk = lower ? bb : nb - 1 - bb;
        const int64_t b0 = blk * TB;
        const int bw = (int)((n - b0 < TB) ? n - b0 : TB);
        for (int e = tid; e < TB * TB; e += blockDim.x) {
            const int r = e % TB, c = e / TB;
            const bool in = lower ? (r >= c) : (r <= c);
            dblk[r + c * TBL] = (r < bw && c < bw && in) ? U(b0 + r, b0 + c) : (T)0;
        }
        __syncthreads();
        if (wid == 0) {
            T xi = (lane < bw) ? x[b0 + lane] : (T)0;
            for (int s = 0; s < bw; ++s) {
                const int k = lower ? s : bw - 1 - s;
                T xk = __shfl(xi, k, 64);
                if (!unit) xk = xk / dblk[k + k * TBL];
                if (lane == k) xi = xk;
                else if (lower ? (lane > k) : (lane < k)) xi -= dblk[lane + k * TBL] * xk;
            }
            if (lane < bw) x[b0 + lane] = xi;
        }
        __syncthreads();
        if (lower) {
            for (int64_t i = b0 + bw + tid; i < n; i += blockDim.x) {
                T s = 0;
                for (int k = 0; k < bw; ++k) s += U(i, b0 + k) * x[b0 + k];
                x[i] -= s;
            }
        } else {
            for (int64_t i = tid; i < b0; i += blockDim.x) {
                T s = 0;
                for (int k = 0; k < bw; ++k) s += U(i, b0 + k) * x[b0 + k];
                x[i] -= s;
            }
        }
        __syncthreads();
    }
}

// Inverse of every 64 x 64 diagonal block of op(M) (lower or upper; unit
// diagonal optional): block b goes to Dinv[b*TB*TB + r + c*TB].  One wavefront
// per block; lane c solves op(M)_bb y = e_c column by column.  Padding rows
// and columns beyond n act as the identity.
template <typename T>
__global__ __launch_bounds__(64) void inv_diag_blocks_kernel(int64_t n, const T* __restrict__ M, int64_t ld,
                                                             int lower, int trans, int unit, T* __restrict__ Dinv)
{
    __shared__ T Ub[TB * TBL];
    const int64_t b0 = (int64_t)blockIdx.x * TB;
    const int bw = (int)((n - b0 < TB) ? n - b0 : TB);
    const int lane = threadIdx.x;
    for (int e = lane; e < TB * TB; e += 64) {
        const int r = e % TB, c = e / TB;
        const bool in = lower ? (r >= c) : (r <= c);
        T v = 0;
        if (r < bw && c < bw && in) v = trans ? M[(b0 + c) + (b0 + r) * ld] : M[(b0 + r) + (b0 + c) * ld];
        if (r == c && (r >= bw || unit)) v = (T)1;
        Ub[r + c * TBL] = v;
    }
    __syncthreads();
    T y[TB];
#pragma unroll
    for (int r = 0; r < TB; ++r) y[r] = (r == lane) ? (T)1 : (T)0;
    if (lower) {
#pragma unroll
        for (int k = 0; k < TB; ++k) {
            y[k] = y[k] / Ub[k + k * TBL];
#pragma unroll
            for (int r = k + 1; r < TB; ++r) y[r] -= Ub[r + k * TBL] * y[k];
        }
    } else {
#pragma unroll
        for (int k = TB - 1; k >= 0; --k) {
            y[k] = y[k] / Ub[k + k * TBL];
#pragma unroll
            for (int r = 0; r < k; ++r) y[r] -= Ub[r + k * TBL] * y[k];
        }
    }
    T* D = Dinv + (int64_t)blockIdx.x * TB * TB;
#pragma unroll
    for (int r = 0; r < TB; ++r) D[r + lane * TB] = y[r];
}

// x (in LDS) := U^{-1} x using the inverted diagonal blocks Dinv of U
// (stored as by inv_diag_blocks_kernel for U, or for U^T when dtrans is set,
// in which case block (r, c) is read as Dinv[c + r*TB]).  U(i, j) as in
// wg_trsv.  `tmp` is LDS scratch of TB elements.  Whole work-group.
template <typename T>
__device__ inline void wg_trsv_inv(int64_t n, const T* __restrict__ M, int64_t ld, bool lower, bool trans,
                                   const T* __restrict__ Dinv, bool dtrans, T* x, T* tmp)
{
    const int tid = threadIdx.x;
    auto U = [&](int64_t i, int64_t j) -> T { return trans ? M[j + i * ld] : M[i + j * ld]; };
    const int64_t nb = (n + TB - 1) / TB;
    for (int64_t bb = 0; bb < nb; ++bb) {
        const int64_t blk = lower ? bb : nb - 1 - bb;
        const int64_t b0 = blk * TB;
        const int bw = (int)((n - b0 < TB) ? n - b0 : TB);
        const T* D = Dinv + blk * TB * TB;
        if (tid < bw) {
            T s = 0;
            for (int c = 0; c < bw; ++c) s += (dtrans ? D[c + tid * TB] : D[tid + c * TB]) * x[b0 + c];
            tmp[tid] = s;
        }
        __syncthreads();
        if (tid < bw) x[b0 + tid] = tmp[tid];
        __syncthreads();
        if (lower) {
            for (int64_t i = b0 + bw + tid; i < n; i += blockDim.x) {
                T s = 0;
                for (int k = 0; k < bw; ++k) s += U(i, b0 + k) * x[b0 + k];
                x[i] -= s;
            }
        } else {
            for (int64_t i = tid; i < b0; i += blockDim.x) {
                T s = 0;
                for (int k = 0; k < bw; ++k) s += U(i, b0 + k) * x[b0 + k];
                x[i] -= s;
            }
        }
        __syncthreads();
    }
}

}  // namespace pne
