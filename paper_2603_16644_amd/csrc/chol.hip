// Cholesky factorization C = L L^T of the n x n PNE matrix A_p^T A_p (FP64),
// and of the FP32 Gram matrix of the condition estimate.  Blocked,
// right-looking with 64-column blocks:
//   diagonal block: unblocked Cholesky by one wavefront (four for FP32),
//     then the inverse L_JJ^{-1} of the block (kept: it serves the panel
//     below and the triangular solves);
//   panel below it: X := X L_JJ^{-T} (MFMA GEMM with the inverse);
//   trailing lower triangle: C -= X X^T (MFMA GEMM on lower tiles).
// A non-positive or non-finite pivot at global column k sets *info to
// 2000 + k + 1 (first failure only) and the factor continues as NaN.
#include "common.h"
#include "kernels.h"
#include "launch.h"

namespace pne {

constexpr int CB = 64;

// FP64 diagonal block by one wavefront.  Lane i holds row i (a[j] =
// C(i, j)); step K forms column K of L, L(i, K) = C(i, K) / L(K, K) with
// L(K, K) = sqrt(C(K, K)), publishes it in LDS and updates the columns
// j > K: C(i, j) -= L(i, K) L(j, K).  Register indices are compile-time
// constants (template recursion).
template <typename T, int K>
struct PotrfStep {
    static __device__ __forceinline__ void run(int w, T (&a)[CB], T* lcol, int32_t* info, int64_t c0)
    {
        if (K >= w) return;
        const int lane = threadIdx.x;
        const T d = lane_value(a[K], K);
        const bool bad = !(d > (T)0) || !isfinite(d);
        if (bad && lane == 0 && *info == 0) *info = 2000 + (int32_t)(c0 + K) + 1;
        const T lkk = bad ? (T)NAN : (T)sqrt(d);
        const T rl = (T)1 / lkk;
        const T l = (lane > K) ? a[K] * rl : (lane == K ? lkk : (T)0);
        a[K] = l;
        lcol[lane] = l;
        __syncthreads();
#pragma unroll
        for (int j = K + 1; j < CB; ++j) a[j] -= l * lcol[j];
        __syncthreads();
        PotrfStep<T, K + 1>::run(w, a, lcol, info, c0);
    }
};
template <typename T>
struct PotrfStep<T, CB> {
    static __device__ __forceinline__ void run(int, T (&)[CB], T*, int32_t*, int64_t) {}
};

// FP32 diagonal block (condition estimate) by four wavefronts: lane i of
// every wave holds row i, wave q holds columns 16q .. 16q+15; same steps as
// above with the owner wave of column K publishing it.
template <typename T, int K>
struct PotrfStep4 {
    static __device__ __forceinline__ void run(int w, T (&a)[16], T* lcol, int32_t* info, int64_t c0)
    {
        if (K >= w) return;
        const int lane = threadIdx.x & 63, q = threadIdx.x >> 6;
        constexpr int QK = K >> 4, TK = K & 15;
        if (q == QK) {
            const T d = lane_value(a[TK], K);
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
        PotrfStep4<T, K + 1>::run(w, a, lcol, info, c0);
    }
};
template <typename T>
struct PotrfStep4<T, CB> {
    static __device__ __forceinline__ void run(int, T (&)[16], T*, int32_t*, int64_t) {}
};

struct PotrfDiagArgs {
    int w;
    void* C;          // diagonal block, ld ldc (lower triangle in, L out)
    int64_t ldc;
    int32_t* info;
    int64_t c0;
};
template <typename T>
struct PotrfDiag {
    typedef PotrfDiagArgs Args;
    static constexpr bool ONE_WAVE = sizeof(T) == 8;
    static constexpr int NTH = ONE_WAVE ? 64 : 256, WPE = 0;
    static __device__ void run(const PotrfDiagArgs& p, int, int)
    {
        const int w = p.w;
        const int64_t ldc = p.ldc;
        T* __restrict__ C = (T*)p.C;
        __shared__ T lcol[CB];
        if constexpr (ONE_WAVE) {
            const int lane = threadIdx.x;
            T a[CB];
#pragma unroll
            for (int j = 0; j < CB; ++j) a[j] = (lane < w && j < w && lane >= j) ? C[lane + (int64_t)j * ldc] : (T)0;
            PotrfStep<T, 0>::run(w, a, lcol, p.info, p.c0);
#pragma unroll
            for (int j = 0; j < CB; ++j)
                if (lane < w && j < w) C[lane + (int64_t)j * ldc] = (lane >= j) ? a[j] : (T)0;
        } else {
            const int lane = threadIdx.x & 63, q = threadIdx.x >> 6;
            T a[16];
#pragma unroll
            for (int t = 0; t < 16; ++t) {
                const int j = 16 * q + t;
                a[t] = (lane < w && j < w && lane >= j) ? C[lane + (int64_t)j * ldc] : (T)0;
            }
            PotrfStep4<T, 0>::run(w, a, lcol, p.info, p.c0);
#pragma unroll
            for (int t = 0; t < 16; ++t) {
                const int j = 16 * q + t;
                if (lane < w && j < w) C[lane + (int64_t)j * ldc] = (lane >= j) ? a[t] : (T)0;
            }
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
void cholesky(Exec& ex, int64_t n, T* C, int64_t ldc, int32_t* info, T* Dinv)
{
    for (int64_t c0 = 0; c0 < n; c0 += CB) {
        ex.iter((uint32_t)(c0 / CB));
        const int w = (int)((n - c0 < CB) ? n - c0 : CB);
        T* D = C + c0 + c0 * ldc;
        T* Db = Dinv + (c0 / CB) * CB * CB;
        launch<PotrfDiag<T>>(ex, 1, 1, PotrfDiagArgs{w, D, ldc, info, c0});
        inv_diag_blocks<T>(ex, n, C, ldc, 1, 0, 0, Dinv, c0 / CB, 1);
        const int64_t rem = n - c0 - w;
        if (rem <= 0) break;
        // X := X L_JJ^{-T}: in place (each work-group reads all of its rows
        // before it writes them)
        T* X = C + (c0 + w) + c0 * ldc;
        GemmArgs p{};
        p.M = rem; p.N = w; p.K = w;
        p.A = X; p.lda = ldc; p.transA = 0;
        p.B = Db; p.ldb = CB; p.transB = 1;
        p.alpha = 1.0; p.beta = 0.0;
        p.C = X; p.ldc = ldc;
        p.splits = 1;
        gemm_t<T>(ex, p);
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
template void cholesky<double>(Exec&, int64_t, double*, int64_t, int32_t*, double*);
template void cholesky<float>(Exec&, int64_t, float*, int64_t, int32_t*, float*);

}  // namespace pne
