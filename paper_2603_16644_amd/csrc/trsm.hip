// A_p = A R_s^{-1} in FP64 (Algorithm 1, "Solve A_p = A R_s^{-1}", after
// R_s is promoted to double).  Recursive right-side substitution (the first
// reads of each column come from A, the results go to A_p); for
// R = [R11 R12; 0 R22]
//   A_p(:, 1) := A_p(:, 1) R11^{-1}               (recursively)
//   A_p(:, 2) -= A_p(:, 1) R12                    (MFMA GEMM, gemm.hip)
//   A_p(:, 2) := A_p(:, 2) R22^{-1}               (recursively)
// down to blocks of 64 columns, finished by row-parallel substitution.
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
    const void* Xin;   // input (element (i, c) at Xin[i*rs + c*cs_in]); null: X in place
    int64_t cs_in;
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
    const T* __restrict__ Xi = a.Xin ? (const T*)a.Xin : X;
    const int64_t csi = a.Xin ? a.cs_in : cs;
    const T* __restrict__ Rb = (const T*)a.Rb;
    // Rs[c * 64 + j] = R(c, j) for c < j (TRANS_LOWER: L(j, c)): row c of the
    // block contiguous, so the update of step c reads consecutive entries;
    // rd[c] = 1 / R(c, c)
    __shared__ __attribute__((aligned(16))) T Rs[LEAF * LEAF];
    __shared__ T rd[LEAF];
    for (int e = threadIdx.x; e < LEAF * LEAF; e += NT) {
        const int c = e / LEAF, j = e % LEAF;
        T v = 0;
        if (j < w && c <= j) v = TRANS_LOWER ? Rb[j + (int64_t)c * ldr] : Rb[c + (int64_t)j * ldr];
        if (c == j) {
            if (UNIT || c >= w) v = (T)1;
            rd[c] = (T)1 / v;
        }
        Rs[e] = v;
    }
    __syncthreads();
    const int64_t i = (int64_t)bx * NT + threadIdx.x;
    if (i >= m) return;
    T x[LEAF];
#pragma unroll
    for (int c = 0; c < LEAF; ++c) x[c] = (c < w) ? Xi[i * rs + c * csi] : (T)0;
    // column-oriented substitution: once y_c is final it is stored and
    // removed from every later entry (the stores then overlap the rest of
    // the work); y_j still accumulates its terms in the order k = 0, 1, ...
#pragma unroll
    for (int c = 0; c < LEAF; ++c) {
        if (c < w) {
            if (!UNIT) x[c] = x[c] * rd[c];
            X[i * rs + c * cs] = x[c];   // final: stored while the later columns are formed
#pragma unroll
            for (int j = c + 1; j < LEAF; ++j) x[j] -= x[c] * Rs[c * LEAF + j];
        }
    }
}

template <typename T, bool TL, bool UNIT>
void trsm_leaf(Exec& ex, int64_t m, int w, T* X, int64_t rs, int64_t cs, const T* Rb, int64_t ldr,
               const T* Xin, int64_t cs_in)
{
    if (m <= 0) return;
    const TrsmLeafArgs a{m, w, X, rs, cs, Rb, ldr, Xin, cs_in};
    // short panels (factorizations) use one wavefront per work-group to
    // spread over more compute units
    if (m < 16384) launch<TrsmLeaf<T, TL, UNIT, 64>>(ex, ceil_div(m, 64), 1, a);
    else launch<TrsmLeaf<T, TL, UNIT, 256>>(ex, ceil_div(m, 256), 1, a);
}
template void trsm_leaf<double, true, false>(Exec&, int64_t, int, double*, int64_t, int64_t, const double*, int64_t,
                                             const double*, int64_t);
template void trsm_leaf<float, true, false>(Exec&, int64_t, int, float*, int64_t, int64_t, const float*, int64_t,
                                            const float*, int64_t);
template void trsm_leaf<double, true, true>(Exec&, int64_t, int, double*, int64_t, int64_t, const double*, int64_t,
                                            const double*, int64_t);
template void trsm_leaf<double, false, false>(Exec&, int64_t, int, double*, int64_t, int64_t, const double*, int64_t,
                                              const double*, int64_t);

// Blocks of at most 128 columns: the two 64-column halves are finished by
// the leaf with a 64-deep GEMM in between.  The input comes from src (the
// original A, or A_p itself once updated) and the result goes to Ap.
static void trsm_base(Exec& ex, int64_t m, int64_t n, const double* src, int64_t lds, const double* R,
                      int64_t ldr, double* Ap, int64_t ldap, uint32_t& step)
{
    ex.iter(step++);
    const int w1 = n < LEAF ? (int)n : LEAF;
    trsm_leaf<double, false, false>(ex, m, w1, Ap, 1, ldap, R, ldr, src, lds);
    if (n > LEAF) {
        GemmArgs h{};
        h.M = m; h.N = n - LEAF; h.K = LEAF;
        h.A = Ap; h.lda = ldap; h.transA = 0;
        h.B = R + LEAF * ldr; h.ldb = ldr; h.transB = 0;
        h.alpha = -1.0; h.beta = 1.0;
        h.Cin = src + LEAF * lds; h.ldcin = lds;
        h.C = Ap + LEAF * ldap; h.ldc = ldap;
        h.splits = 1;
        gemm_f64(ex, h);
        trsm_leaf<double, false, false>(ex, m, (int)(n - LEAF), Ap + LEAF * ldap, 1, ldap,
                                        R + LEAF + LEAF * ldr, ldr, nullptr, 0);
    }
}

// Recursive halving, X = [X1 X2], R = [R11 R12; 0 R22]:
//   X1 = A1 R11^{-1};  X2 = (A2 - X1 R12) R22^{-1}.
// The off-diagonal products are large GEMMs (K = n/2, n/4, ...), which run
// far closer to the MFMA peak than a sweep of 128-column blocks would.
static void trsm_rec(Exec& ex, int64_t m, int64_t n, const double* src, int64_t lds, const double* R,
                     int64_t ldr, double* Ap, int64_t ldap, uint32_t& step)
{
    if (n <= 2 * LEAF) {
        trsm_base(ex, m, n, src, lds, R, ldr, Ap, ldap, step);
        return;
    }
    const int64_t n1 = ceil_div(n / 2, LEAF) * LEAF;
    trsm_rec(ex, m, n1, src, lds, R, ldr, Ap, ldap, step);
    ex.iter(step++);
    GemmArgs g{};
    g.M = m; g.N = n - n1; g.K = n1;
    g.A = Ap; g.lda = ldap; g.transA = 0;
    g.B = R + n1 * ldr; g.ldb = ldr; g.transB = 0;
    g.alpha = -1.0; g.beta = 1.0;
    g.Cin = src + n1 * lds; g.ldcin = lds;
    g.C = Ap + n1 * ldap; g.ldc = ldap;
    g.splits = 1;
    gemm_f64(ex, g);
    trsm_rec(ex, m, n - n1, Ap + n1 * ldap, ldap, R + n1 + n1 * ldr, ldr, Ap + n1 * ldap, ldap, step);
}

void trsm_right_upper(Exec& ex, int64_t m, int64_t n, const double* A, int64_t lda, const double* R,
                      int64_t ldr, double* Ap, int64_t ldap)
{
    uint32_t step = 0;
    trsm_rec(ex, m, n, A, lda, R, ldr, Ap, ldap, step);
}

}  // namespace pne
