// Cholesky factorization C = L L^T of the n x n PNE matrix A_p^T A_p (FP64),
// and of the FP32 Gram matrix of the condition estimate.  Blocked,
// right-looking with 64-column blocks:
//   diagonal block: its factor L_JJ and the inverse L_JJ^{-1} by one
//     work-group (PotrfInv; the inverse serves the panel below and the
//     triangular solves);
//   panel below it: X := X L_JJ^{-T} (MFMA GEMM with the inverse);
//   trailing lower triangle: C -= X X^T (MFMA GEMM on lower tiles).
// A non-positive or non-finite pivot at global column k sets *info to
// 2000 + k + 1 (first failure only) and the factor continues as NaN.
#include "common.h"
#include "kernels.h"
#include "launch.h"

namespace pne {

constexpr int CB = 64;

// Diagonal block with its inverse, by one work-group of 256 threads.  The
// w x w block (padded to 64 x 64 with the identity) is held in LDS and
// factored in four steps of 16 columns (right-looking):
//   the 16 x 16 diagonal block D by one wavefront, lane i holding row i:
//     column K of L_D is formed from the pivot C(K, K) and every lane
//     updates its row with the entries L(j, K) of the other rows, read by
//     readlane (no LDS round trip per column); the same wavefront then
//     forms L_D^{-1}, lane c solving L_D y = e_c by forward substitution;
//   the rows below: L21 = A21 L_D^{-T} (all threads);
//   the trailing lower triangle: A22 -= L21 L21^T (all threads).
// The inverse of the 64 x 64 factor is then assembled by block rows,
//   X_ii = L_ii^{-1},  X_ij = -X_ii sum_{k = j .. i-1} L_ik X_kj  (j < i).
// Outputs: L in the lower triangle of the block in C (zeros above), X in
// Dinv (64 x 64, column-major; the identity on padding).
constexpr int PD_LD = CB + 1;   // LDS leading dimension of the block

struct PotrfInvArgs {
    int w;
    void* C;          // diagonal block, ld ldc (lower triangle in, L out)
    int64_t ldc;
    int32_t* info;
    int64_t c0;       // global index of the block's first column
    void* Dinv;       // 64 x 64 inverse out
};
template <typename T>
struct PotrfInv {
    typedef PotrfInvArgs Args;
    static constexpr int NTH = 256, WPE = 0;
    static __device__ void run(const PotrfInvArgs& p, int, int);
};
template <typename T>
__device__ void PotrfInv<T>::run(const PotrfInvArgs& p, int, int)
{
    __shared__ T L[CB * PD_LD];   // L[r + c * PD_LD]
    __shared__ T X[CB * PD_LD];   // inverse
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int w = p.w;
    const int64_t ldc = p.ldc;
    T* __restrict__ C = (T*)p.C;
    for (int e = tid; e < CB * CB; e += NTH) {
        const int r = e % CB, c = e / CB;
        T v = (T)0;
        if (r < w && c < w) v = (r >= c) ? C[r + c * ldc] : (T)0;
        else if (r == c) v = (T)1;
        L[r + c * PD_LD] = v;
    }
    __syncthreads();
#pragma unroll 1
    for (int kb = 0; kb < 4; ++kb) {
        const int o = 16 * kb;
        if (wid == 0) {
            T a[16];
#pragma unroll
            for (int j = 0; j < 16; ++j) a[j] = (lane < 16 && j <= lane) ? L[(o + lane) + (o + j) * PD_LD] : (T)0;
#pragma unroll
            for (int K = 0; K < 16; ++K) {
                const T d = lane_value(a[K], K);
                const bool bad = !(d > (T)0) || !isfinite(d);
                if (bad && lane == 0 && o + K < w && *p.info == 0) *p.info = 2000 + (int32_t)(p.c0 + o + K) + 1;
                const T lkk = bad ? (T)NAN : (T)sqrt(d);
                const T rl = (T)1 / lkk;
                const T l = (lane > K) ? a[K] * rl : (lane == K ? lkk : (T)0);
                a[K] = l;
#pragma unroll
                for (int j = K + 1; j < 16; ++j) a[j] -= l * lane_value(l, j);
            }
            if (lane < 16) {
#pragma unroll
                for (int j = 0; j < 16; ++j)
                    if (j <= lane) L[(o + lane) + (o + j) * PD_LD] = a[j];
            }
            // (the wavefront's own LDS writes are visible to its later reads)
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            // column `lane` of L_D^{-1}: y_r = (delta_{r, lane} - sum_{k<r}
            // L(r, k) y_k) / L(r, r), the entries of L_D read as LDS broadcasts
            T y[16];
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                T s = (lane == r) ? (T)1 : (T)0;
#pragma unroll
                for (int k = 0; k < r; ++k) s -= L[(o + r) + (o + k) * PD_LD] * y[k];
                y[r] = s / L[(o + r) + (o + r) * PD_LD];
            }
            if (lane < 16) {
#pragma unroll
                for (int r = 0; r < 16; ++r) X[(o + r) + (o + lane) * PD_LD] = y[r];
            }
        }
        __syncthreads();
        const int nr = CB - o - 16;   // rows below the diagonal block
        if (nr > 0) {
            // L21 = A21 L_D^{-T}: element (r, c) = sum_{k <= c} A21(r, k) L_D^{-1}(c, k)
            T res[3];
#pragma unroll
            for (int t = 0; t < 3; ++t) {
                const int e = tid + NTH * t;
                T s = (T)0;
                if (e < nr * 16) {
                    const int r = o + 16 + e % nr, c = e / nr;
                    for (int k = 0; k <= c; ++k) s += L[r + (o + k) * PD_LD] * X[(o + c) + (o + k) * PD_LD];
                }
                res[t] = s;
            }
            __syncthreads();
#pragma unroll
            for (int t = 0; t < 3; ++t) {
                const int e = tid + NTH * t;
                if (e < nr * 16) L[(o + 16 + e % nr) + (o + e / nr) * PD_LD] = res[t];
            }
            __syncthreads();
            // A22 -= L21 L21^T on the lower triangle
            for (int e = tid; e < nr * nr; e += NTH) {
                const int rr = e % nr, cc = e / nr;
                if (rr < cc) continue;
                T s = (T)0;
#pragma unroll
                for (int k = 0; k < 16; ++k) s += L[(o + 16 + rr) + (o + k) * PD_LD] * L[(o + 16 + cc) + (o + k) * PD_LD];
                L[(o + 16 + rr) + (o + 16 + cc) * PD_LD] -= s;
            }
            __syncthreads();
        }
    }
    // inverse by block rows
#pragma unroll 1
    for (int i = 1; i < 4; ++i) {
        const int cnt = 16 * 16 * i;   // block row i, columns 0 .. 16 i - 1
        T res[3];
        // S(r, col) = sum_{q = col .. 16 i - 1} L(16 i + r, q) X(q, col)
#pragma unroll
        for (int t = 0; t < 3; ++t) {
            const int e = tid + NTH * t;
            T s = (T)0;
            if (e < cnt) {
                const int r = e % 16, col = e / 16;
                for (int q = col; q < 16 * i; ++q) s += L[(16 * i + r) + q * PD_LD] * X[q + col * PD_LD];
            }
            res[t] = s;
        }
        __syncthreads();
#pragma unroll
        for (int t = 0; t < 3; ++t) {
            const int e = tid + NTH * t;
            if (e < cnt) X[(16 * i + e % 16) + (e / 16) * PD_LD] = res[t];
        }
        __syncthreads();
        // X_ij = -X_ii S: element (r, col) = -sum_{u <= r} X(16 i + r, 16 i + u) S(u, col)
#pragma unroll
        for (int t = 0; t < 3; ++t) {
            const int e = tid + NTH * t;
            T s = (T)0;
            if (e < cnt) {
                const int r = e % 16, col = e / 16;
                for (int u = 0; u <= r; ++u) s += X[(16 * i + r) + (16 * i + u) * PD_LD] * X[(16 * i + u) + col * PD_LD];
            }
            res[t] = -s;
        }
        __syncthreads();
#pragma unroll
        for (int t = 0; t < 3; ++t) {
            const int e = tid + NTH * t;
            if (e < cnt) X[(16 * i + e % 16) + (e / 16) * PD_LD] = res[t];
        }
        __syncthreads();
    }
    T* __restrict__ Dv = (T*)p.Dinv;
    for (int e = tid; e < CB * CB; e += NTH) {
        const int r = e % CB, c = e / CB;
        if (r < w && c < w) C[r + c * ldc] = (r >= c) ? L[r + c * PD_LD] : (T)0;
        Dv[r + c * CB] = (r >= c) ? X[r + c * PD_LD] : (T)0;
    }
}

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
        launch<PotrfInv<T>>(ex, 1, 1, PotrfInvArgs{w, D, ldc, info, c0, Db});
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
