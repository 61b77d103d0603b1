// A_p = A R_s^{-1} in FP64 (Algorithm 1, "Solve A_p = A R_s^{-1}", after
// R_s is promoted to double).  Blocked right-side substitution over column
// blocks J:
//   A_p(:, J) = A(:, J) - A_p(:, <J) R(<J, J)     (MFMA GEMM, gemm.hip)
//   A_p(:, J) := A_p(:, J) R(J, J)^{-1}           (row-parallel substitution)
// The second step keeps one row per lane in registers and runs the plain
// forward substitution y_j = (t_j - sum_{k<j} y_k R_kj) / R_jj with the
// 64 x 64 diagonal block broadcast from LDS.  The same leaf serves the
// Cholesky panel (X L^T = C, TRANS_LOWER).
#include "common.h"
#include "kernels.h"
#include "launch.h"

namespace pne {

constexpr int LEAF = 64;

struct TrsmLeafArgs {
    int64_t m;
    int w;
    void* X;
    int64_t rs, cs;
    const void* Rb;
    int64_t ldr;
};
template <typename T, bool TRANS_LOWER, bool UNIT, int NT>
struct TrsmLeaf {
    typedef TrsmLeafArgs Args;
    static constexpr int NTH = NT, WPE = 0;
    static __device__ void run(const TrsmLeafArgs& a, int bx, int by);
};
template <typename T, bool TRANS_LOWER, bool UNIT, int NT>
__device__ void TrsmLeaf<T, TRANS_LOWER, UNIT, NT>::run(const TrsmLeafArgs& a, int bx, int)
{
    const int64_t m = a.m, rs = a.rs, cs = a.cs, ldr = a.ldr;
    const int w = a.w;
    T* __restrict__ X = (T*)a.X;
    const T* __restrict__ Rb = (const T*)a.Rb;
    __shared__ T Rs[LEAF * LEAF];  // Rs[c * 64 + k] = R(k, c), k <= c
    for (int e = threadIdx.x; e < LEAF * LEAF; e += NT) {
        const int c = e / LEAF, k = e % LEAF;
        T v = 0;
        if (c < w && k <= c) v = TRANS_LOWER ? Rb[c + (int64_t)k * ldr] : Rb[k + (int64_t)c * ldr];
        if (UNIT && k == c) v = (T)1;
        Rs[e] = v;
    }
    __syncthreads();
    const int64_t i = (int64_t)bx * NT + threadIdx.x;
    if (i >= m) return;
    T x[LEAF];
#pragma unroll
    for (int c = 0; c < LEAF; ++c) x[c] = (c < w) ? X[i * rs + c * cs] : (T)0;
    // column-oriented substitution: once y_c is final it is removed from every
    // later entry; y_j still accumulates its terms in the order k = 0, 1, ...
#pragma unroll
    for (int c = 0; c < LEAF; ++c) {
        if (c < w) {
            if (!UNIT) x[c] = x[c] / Rs[c * LEAF + c];
#pragma unroll
            for (int j = c + 1; j < LEAF; ++j) x[j] -= x[c] * Rs[j * LEAF + c];
        }
    }
#pragma unroll
    for (int c = 0; c < LEAF; ++c)
        if (c < w) X[i * rs + c * cs] = x[c];
}

template <typename T, bool TL, bool UNIT>
void trsm_leaf(Exec& ex, int64_t m, int w, T* X, int64_t rs, int64_t cs, const T* Rb, int64_t ldr)
{
    if (m <= 0) return;
    const TrsmLeafArgs a{m, w, X, rs, cs, Rb, ldr};
    // short panels (factorizations) use one wavefront per work-group to
    // spread over more compute units
    if (m < 16384) launch<TrsmLeaf<T, TL, UNIT, 64>>(ex, ceil_div(m, 64), 1, a);
    else launch<TrsmLeaf<T, TL, UNIT, 256>>(ex, ceil_div(m, 256), 1, a);
}
template void trsm_leaf<double, true, false>(Exec&, int64_t, int, double*, int64_t, int64_t, const double*, int64_t);
template void trsm_leaf<float, true, false>(Exec&, int64_t, int, float*, int64_t, int64_t, const float*, int64_t);
template void trsm_leaf<double, true, true>(Exec&, int64_t, int, double*, int64_t, int64_t, const double*, int64_t);
template void trsm_leaf<double, false, false>(Exec&, int64_t, int, double*, int64_t, int64_t, const double*, int64_t);

// Column blocks of 128: one GEMM brings the block up to date with every
// earlier column, then the two 64-column halves are finished by the leaf with
// a 64-deep GEMM in between.
void trsm_right_upper(Exec& ex, int64_t m, int64_t n, const double* A, int64_t lda, const double* R,
                      int64_t ldr, double* Ap, int64_t ldap)
{
    for (int64_t c0 = 0; c0 < n; c0 += 2 * LEAF) {
        ex.iter((uint32_t)(c0 / (2 * LEAF)));
        const int w = (int)((n - c0 < 2 * LEAF) ? n - c0 : 2 * LEAF);
        GemmArgs g{};
        g.M = m; g.N = w; g.K = c0;
        g.A = Ap; g.lda = ldap; g.transA = 0;
        g.B = R + c0 * ldr; g.ldb = ldr; g.transB = 0;
        g.alpha = -1.0; g.beta = 1.0;
        g.Cin = A + c0 * lda; g.ldcin = lda;
        g.C = Ap + c0 * ldap; g.ldc = ldap;
        g.splits = 1;
        gemm_f64(ex, g);
        const int w1 = w < LEAF ? w : LEAF;
        trsm_leaf<double, false, false>(ex, m, w1, Ap + c0 * ldap, 1, ldap, R + c0 + c0 * ldr, ldr);
        if (w > LEAF) {
            const int64_t c1 = c0 + LEAF;
            GemmArgs h{};
            h.M = m; h.N = w - LEAF; h.K = LEAF;
            h.A = Ap + c0 * ldap; h.lda = ldap; h.transA = 0;
            h.B = R + c0 + c1 * ldr; h.ldb = ldr; h.transB = 0;
            h.alpha = -1.0; h.beta = 1.0;
            h.Cin = Ap + c1 * ldap; h.ldcin = ldap;
            h.C = Ap + c1 * ldap; h.ldc = ldap;
            h.splits = 1;
            gemm_f64(ex, h);
            trsm_leaf<double, false, false>(ex, m, w - LEAF, Ap + c1 * ldap, 1, ldap, R + c1 + c1 * ldr, ldr);
        }
    }
}

}  // namespace pne
