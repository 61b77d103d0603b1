// Cholesky factorization C = L L^T of the n x n PNE matrix A_p^T A_p (FP64),
// and of the FP32 Gram matrix of the condition estimate.  Blocked,
// right-looking with 64-column blocks:
//   diagonal block: unblocked Cholesky in LDS by one work-group;
//   panel below it: X := X L_JJ^{-T} (row-parallel leaf, trsm.hip);
//   trailing lower triangle: C -= X X^T (MFMA GEMM on lower tiles).
// A non-positive or non-finite pivot at global column k sets *info to
// 2000 + k + 1 (first failure only) and the factor continues as NaN.
#include "common.h"
#include "kernels.h"

namespace pne {

constexpr int CB = 64;

template <typename T>
__global__ __launch_bounds__(256) void potrf_diag_kernel(int w, T* __restrict__ C, int64_t ldc,
                                                         int32_t* __restrict__ info, int64_t c0)
{
    __shared__ T L[CB * (CB + 1)];
    const int tid = threadIdx.x;
    for (int e = tid; e < CB * CB; e += 256) {
        const int i = e % CB, j = e / CB;
        L[i + j * (CB + 1)] = (i < w && j < w && i >= j) ? C[i + (int64_t)j * ldc] : (T)0;
    }
    __syncthreads();
    for (int k = 0; k < w; ++k) {
        T d = L[k + k * (CB + 1)];
        const bool bad = !(d > (T)0) || !isfinite(d);
        if (bad && tid == 0 && *info == 0) *info = 2000 + (int32_t)(c0 + k) + 1;
        const T lkk = bad ? (T)NAN : (T)sqrt(d);
        __syncthreads();
        if (tid == 0) L[k + k * (CB + 1)] = lkk;
        if (tid > k && tid < w) L[tid + k * (CB + 1)] /= lkk;
        __syncthreads();
        // trailing update of the lower triangle: L(i, j) -= L(i, k) L(j, k), k < j <= i
        for (int e = tid; e < CB * CB; e += 256) {
            const int i = e % CB, j = e / CB;
            if (j > k && i >= j && i < w) L[i + j * (CB + 1)] -= L[i + k * (CB + 1)] * L[j + k * (CB + 1)];
        }
        __syncthreads();
    }
    for (int e = tid; e < CB * CB; e += 256) {
        const int i = e % CB, j = e / CB;
        if (i < w && j < w) C[i + (int64_t)j * ldc] = (i >= j) ? L[i + j * (CB + 1)] : (T)0;
    }
}

template <typename T>
static void gemm_t(const GemmArgs& g, hipStream_t st)
{
    if constexpr (sizeof(T) == 8) gemm_f64(g, st);
    else gemm_f32(g, st);
}

template <typename T>
void cholesky(int64_t n, T* C, int64_t ldc, int32_t* info, hipStream_t st)
{
    for (int64_t c0 = 0; c0 < n; c0 += CB) {
        const int w = (int)((n - c0 < CB) ? n - c0 : CB);
        T* D = C + c0 + c0 * ldc;
        potrf_diag_kernel<T><<<1, 256, 0, st>>>(w, D, ldc, info, c0);
        const int64_t rem = n - c0 - w;
        if (rem <= 0) break;
        T* X = C + (c0 + w) + c0 * ldc;
        trsm_leaf<T, true, false>(rem, w, X, 1, ldc, D, ldc, st);
        T* C22 = C + (c0 + w) + (c0 + w) * ldc;
        GemmArgs g{};
        g.M = rem; g.N = rem; g.K = w;
        g.A = X; g.lda = ldc; g.transA = 0;
        g.B = X; g.ldb = ldc; g.transB = 1;
        g.alpha = -1.0; g.beta = 1.0;
        g.Cin = C22; g.ldcin = ldc; g.C = C22; g.ldc = ldc;
        g.lower = 1; g.splits = 1;
        gemm_t<T>(g, st);
    }
}
template void cholesky<double>(int64_t, double*, int64_t, int32_t*, hipStream_t);
template void cholesky<float>(int64_t, float*, int64_t, int32_t*, hipStream_t);

}  // namespace pne
