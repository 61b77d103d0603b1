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
#include "launch.h"

namespace pne {

constexpr int CB = 64;

// Unblocked Cholesky of one w x w (w <= 64) diagonal block: lane i of every
// wave holds row i; wave q holds columns 16q .. 16q+15 in registers.  Step k
// (unrolled, so every register index is static): the owner wave of column k
// forms L(:, k) = C(:, k) / sqrt(C(k, k)) and publishes it in LDS; every wave
// then updates its columns j > k: L(i, j) -= L(i, k) L(j, k).
template <typename T, int K>
struct CholSteps {
    static __device__ __forceinline__ void run(int w, T (&a)[16], T* lcol, int32_t* info, int64_t c0)
    {
        if (K >= w) return;
        const int lane = threadIdx.x & 63, q = threadIdx.x >> 6;
        constexpr int QK = K >> 4, TK = K & 15;
        if (q == QK) {
            const T d = __shfl(a[TK], K, 64);
            const bool bad = !(d > (T)0) || !isfinite(d);
            if (bad && lane == 0 && *info == 0) *info = 2000 + (int32_t)(c0 + K) + 1;
            const T lkk = bad ? (T)NAN : (T)sqrt(d);
            const T rl = (T)1 / lkk;
            const T l = (lane > K) ? a[TK] * rl : (lane == K ? lkk : (T)0);
            a[TK] = l;
            lcol[lane] = l;
        }
        __syncthreads();
        const T li = lcol[lane];
#pragma unroll
        for (int t = 0; t < 16; ++t) {
            const int j = 16 * q + t;
            if (j > K) a[t] -= li * lcol[j];
        }
        __syncthreads();
        CholSteps<T, K + 1>::run(w, a, lcol, info, c0);
    }
};
template <typename T>
struct CholSteps<T, CB> {
    static __device__ __forceinline__ void run(int, T (&)[16], T*, int32_t*, int64_t) {}
};

struct PotrfDiagArgs {
    int w;
    void* C;
    int64_t ldc;
    int32_t* info;
    int64_t c0;
};
template <typename T>
struct PotrfDiag {
    typedef PotrfDiagArgs Args;
    static constexpr int NTH = 256, WPE = 0;
    static __device__ void run(const PotrfDiagArgs& a, int, int)
    {
        const int w = a.w;
        const int64_t ldc = a.ldc;
        T* __restrict__ C = (T*)a.C;
        __shared__ T lcol[CB];
        const int lane = threadIdx.x & 63, q = threadIdx.x >> 6;
        T v[16];
#pragma unroll
        for (int t = 0; t < 16; ++t) {
            const int j = 16 * q + t;
            v[t] = (lane < w && j < w && lane >= j) ? C[lane + (int64_t)j * ldc] : (T)0;
        }
        CholSteps<T, 0>::run(w, v, lcol, a.info, a.c0);
#pragma unroll
        for (int t = 0; t < 16; ++t) {
            const int j = 16 * q + t;
            if (lane < w && j < w) C[lane + (int64_t)j * ldc] = (lane >= j) ? v[t] : (T)0;
        }
    }
};

template <typename T>
static void gemm_t(Exec& ex, const GemmArgs& g)
{
    if constexpr (sizeof(T) == 8) gemm_f64(ex, g);
    else gemm_f32(ex, g);
}

template <typename T>
void cholesky(Exec& ex, int64_t n, T* C, int64_t ldc, int32_t* info)
{
    for (int64_t c0 = 0; c0 < n; c0 += CB) {
        ex.iter((uint32_t)(c0 / CB));
        const int w = (int)((n - c0 < CB) ? n - c0 : CB);
        T* D = C + c0 + c0 * ldc;
        launch<PotrfDiag<T>>(ex, 1, 1, PotrfDiagArgs{w, D, ldc, info, c0});
        const int64_t rem = n - c0 - w;
        if (rem <= 0) break;
        T* X = C + (c0 + w) + c0 * ldc;
        trsm_leaf<T, true, false>(ex, rem, w, X, 1, ldc, D, ldc);
        T* C22 = C + (c0 + w) + (c0 + w) * ldc;
        GemmArgs g{};
        g.M = rem; g.N = rem; g.K = w;
        g.A = X; g.lda = ldc; g.transA = 0;
        g.B = X; g.ldb = ldc; g.transB = 1;
        g.alpha = -1.0; g.beta = 1.0;
        g.Cin = C22; g.ldcin = ldc; g.C = C22; g.ldc = ldc;
        g.lower = 1; g.splits = 1;
        gemm_t<T>(ex, g);
    }
}
template void cholesky<double>(Exec&, int64_t, double*, int64_t, int32_t*);
template void cholesky<float>(Exec&, int64_t, float*, int64_t, int32_t*);

}  // namespace pne
