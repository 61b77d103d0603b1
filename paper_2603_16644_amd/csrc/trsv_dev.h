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
// per block (bx = b); lane c solves op(M)_bb y = e_c by substitution in
// column order (forward for lower, backward for upper) with the block in LDS
// and the reciprocal diagonal, y in registers (static indices through
// template recursion).  Padding rows and columns beyond n act as the
// identity.
template <typename T, bool UPPER, int K>
struct InvStep {
    static __device__ __forceinline__ void run(T (&y)[TB], const T* Ub, const T* rd, T* Ys)
    {
        constexpr int k = UPPER ? TB - 1 - K : K;
        const int lane = threadIdx.x;
        const T yk = y[k] * rd[k];
        Ys[k * TBL + lane] = yk;
#pragma unroll
        for (int j = 0; j < TB; ++j)
            if (UPPER ? (j < k) : (j > k)) y[j] -= Ub[j + k * TBL] * yk;
        __syncthreads();
        InvStep<T, UPPER, K + 1>::run(y, Ub, rd, Ys);
    }
};
template <typename T, bool UPPER>
struct InvStep<T, UPPER, TB> {
    static __device__ __forceinline__ void run(T (&)[TB], const T*, const T*, T*) {}
};

struct InvDiagArgs {
    int64_t n;
    const void* M;
    int64_t ld;
    int trans, unit;
    void* Dinv;
    int64_t block0;    // first block handled (bx = 0)
};
template <typename T, bool UPPER>
struct InvDiag {
    typedef InvDiagArgs Args;
    static constexpr int NTH = 64, WPE = 0;
    static __device__ void run(const InvDiagArgs& a, int bx, int by);
};
template <typename T, bool UPPER>
__device__ void InvDiag<T, UPPER>::run(const InvDiagArgs& a, int bx, int)
{
    const int64_t n = a.n, ld = a.ld;
    const int trans = a.trans, unit = a.unit;
    const T* __restrict__ M = (const T*)a.M;
    const int64_t blk = a.block0 + bx;
    T* __restrict__ D = (T*)a.Dinv + blk * TB * TB;
    __shared__ T Ub[TB * TBL];   // Ub[r + c * TBL] = op(M)_bb(r, c)
    __shared__ T Ys[TB * TBL];   // Ys[r * TBL + c] = inverse(r, c)
    __shared__ T rd[TB];
    const int64_t b0 = blk * TB;
    const int bw = (int)((n - b0 < TB) ? n - b0 : TB);
    const int lane = threadIdx.x;
    for (int e = lane; e < TB * TB; e += 64) {
        const int r = e % TB, c = e / TB;
        const bool in = UPPER ? (r <= c) : (r >= c);
        T v = 0;
        if (r < bw && c < bw && in) v = trans ? M[(b0 + c) + (b0 + r) * ld] : M[(b0 + r) + (b0 + c) * ld];
        if (r == c && (r >= bw || unit)) v = (T)1;
        Ub[r + c * TBL] = v;
    }
    __syncthreads();
    rd[lane] = (T)1 / Ub[lane + lane * TBL];
    __syncthreads();
    T y[TB];
#pragma unroll
    for (int r = 0; r < TB; ++r) y[r] = (r == lane) ? (T)1 : (T)0;
    InvStep<T, UPPER, 0>::run(y, Ub, rd, Ys);
    for (int c = 0; c < TB; ++c) D[lane + c * TB] = Ys[lane * TBL + c];
}

// x (in LDS) := U^{-1} x using the inverted diagonal blocks Dinv of U
// (stored as by InvDiag for U, or for U^T when dtrans is set, in which case
// block (r, c) is read as Dinv[c + r*TB]).  U(i, j) = trans ? M[j + i ld] :
// M[i + j ld]; `lower` says whether U is lower triangular.  `tmp` is LDS
// scratch of TB elements.  Whole work-group.
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
