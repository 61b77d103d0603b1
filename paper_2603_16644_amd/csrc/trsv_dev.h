// Single-work-group triangular solves on a vector held in LDS (FP64 or FP32),
// shared by the solve kernels and the condition estimate: blocked by 64, the
// diagonal blocks applied through their precomputed inverses (one small
// matrix-vector product per block instead of 64 dependent steps), then all
// threads update the remaining entries with the block's columns.
#pragma once
#include "common.h"

namespace pne {

constexpr int TB = 64, TBL = TB + 1;  // diagonal block and its LDS leading dimension

// Inverse of every 64 x 64 diagonal block of op(M) (lower or upper; unit
// diagonal optional): block b goes to Dinv[b*TB*TB + r + c*TB].  One wavefront
// per block (bx = b); lane c solves op(M)_bb y = e_c column by column.
// Padding rows and columns beyond n act as the identity.
struct InvDiagArgs {
    int64_t n;
    const void* M;
    int64_t ld;
    int lower, trans, unit;
    void* Dinv;
};
template <typename T>
struct InvDiag {
    typedef InvDiagArgs Args;
    static constexpr int NTH = 64, WPE = 0;
    static __device__ void run(const InvDiagArgs& a, int bx, int by);
};
template <typename T>
__device__ void InvDiag<T>::run(const InvDiagArgs& a, int bx, int)
{
    const int64_t n = a.n, ld = a.ld;
    const int lower = a.lower, trans = a.trans, unit = a.unit;
    const T* __restrict__ M = (const T*)a.M;
    T* __restrict__ Dinv = (T*)a.Dinv;
    __shared__ T Ub[TB * TBL];
    const int64_t b0 = (int64_t)bx * TB;
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
    T* D = Dinv + (int64_t)bx * TB * TB;
#pragma unroll
    for (int r = 0; r < TB; ++r) D[r + lane * TB] = y[r];
}

// x (in LDS) := U^{-1} x using the inverted diagonal blocks Dinv of U
// (stored as by InvDiag for U, or for U^T when dtrans is set,
// in which case block (r, c) is read as Dinv[c + r*TB]).  U(i, j) =
// trans ? M[j + i ld] : M[i + j ld]; `lower` says whether U is lower
// triangular.  `tmp` is LDS scratch of TB elements.  Whole work-group.
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
