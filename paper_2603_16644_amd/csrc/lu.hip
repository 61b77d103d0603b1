// LU factorization with partial pivoting P C = L U of the n x n HPNE matrix
// A_p^T A (Section 1, eq. e_hpne; the system is non-symmetric).  Blocked,
// right-looking:
//   panel (PW columns, all rows below): one 512-thread work-group with the
//     panel in registers; per column the pivot is the first row of largest
//     magnitude (wavefront argmax, ties to the smaller index), the two rows
//     are exchanged through LDS, the column is scaled and the rest of the
//     panel gets the rank-1 update;
//   the same row exchanges are applied to the other columns;
//   U12 := L11^{-1} C12 (unit lower, row-parallel leaf on U12^T);
//   C22 -= L21 U12 (MFMA GEMM).
// A zero or non-finite pivot at global column k sets *info = 3000 + k + 1
// (first only); that column's elimination is skipped.
#include "common.h"
#include "kernels.h"
#include "launch.h"

namespace pne {

constexpr int LU_THREADS = 512;
constexpr int LU_WAVES = LU_THREADS / 64;

struct LuPanelArgs {
    int64_t h;
    int w;
    double* P;
    int64_t ldc;
    int32_t* piv;
    int64_t c0;
    int32_t* info;
};
template <int RPT, int PW>
struct LuPanel {
    typedef LuPanelArgs Args;
    static constexpr int NTH = LU_THREADS, WPE = 0;
    static __device__ void run(const LuPanelArgs& a, int bx, int by);
};
template <int RPT, int PW>
__device__ void LuPanel<RPT, PW>::run(const LuPanelArgs& a, int, int)
{
    const int64_t h = a.h, ldc = a.ldc, c0 = a.c0;
    const int w = a.w;
    double* __restrict__ P = a.P;
    int32_t* __restrict__ piv = a.piv;
    int32_t* __restrict__ info = a.info;
    // rows k and p and the wavefront argmax candidates, double-buffered by
    // the parity of k: step k + 1 never overwrites what a slower thread of
    // step k still reads, so each column needs two barriers
    __shared__ double rowK[2][PW], rowP[2][PW];
    __shared__ double wv[2][LU_WAVES];
    __shared__ int64_t wi[2][LU_WAVES];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    double x[RPT][PW];
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        const int64_t r = tid + LU_THREADS * q;
#pragma unroll
        for (int c = 0; c < PW; ++c) x[q][c] = (r < h && c < w) ? P[r + c * ldc] : 0.0;
    }
    for (int k = 0; k < w; ++k) {
        const int B = k & 1;
        // argmax |x(r, k)| over r >= k, first index on ties; a NaN counts as
        // +inf, so a column holding one selects a non-finite pivot
        double best = -1.0;
        int64_t bidx = INT64_MAX;
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            const int64_t r = tid + LU_THREADS * q;
            double v = -1.0;
#pragma unroll
            for (int c = 0; c < PW; ++c)
                if (c == k) v = fabs(x[q][c]);
            if (v != v) v = INFINITY;
            if (r >= k && r < h && v > best) { best = v; bidx = r; }
        }
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            const double ov = __shfl_xor(best, off, 64);
            const int64_t oi = __shfl_xor(bidx, off, 64);
            if (ov > best || (ov == best && oi < bidx)) { best = ov; bidx = oi; }
        }
        if (lane == 0) { wv[B][wid] = best; wi[B][wid] = bidx; }
        __syncthreads();
        // every thread forms the pivot row from the candidates
        double b = wv[B][0];
        int64_t p = wi[B][0];
        for (int i = 1; i < LU_WAVES; ++i)
            if (wv[B][i] > b || (wv[B][i] == b && wi[B][i] < p)) { b = wv[B][i]; p = wi[B][i]; }
        if (p < k || p >= h) p = k;   // no candidate: keep the row in place
        if (tid == 0) piv[c0 + k] = (int32_t)(c0 + p);
        // publish rows k and p of the panel
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            const int64_t r = tid + LU_THREADS * q;
            if (r == p)
#pragma unroll
                for (int c = 0; c < PW; ++c) rowP[B][c] = x[q][c];
            if (r == k)
#pragma unroll
                for (int c = 0; c < PW; ++c) rowK[B][c] = x[q][c];
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            const int64_t r = tid + LU_THREADS * q;
            if (r == k && p != k)
#pragma unroll
                for (int c = 0; c < PW; ++c) x[q][c] = rowP[B][c];
            if (r == p && p != k)
#pragma unroll
                for (int c = 0; c < PW; ++c) x[q][c] = rowK[B][c];
        }
        double pv = 0.0;
#pragma unroll
        for (int c = 0; c < PW; ++c)
            if (c == k) pv = rowP[B][c];
        if (pv == 0.0 || !isfinite(pv)) {
            if (tid == 0 && *info == 0) *info = 3000 + (int32_t)(c0 + k) + 1;
        } else {
#pragma unroll
            for (int q = 0; q < RPT; ++q) {
                const int64_t r = tid + LU_THREADS * q;
                if (r > k && r < h) {
                    // select x(r, k) first: a division inside the selection
                    // would be evaluated for every column
                    double xk = 0.0;
#pragma unroll
                    for (int c = 0; c < PW; ++c)
                        if (c == k) xk = x[q][c];
                    const double l = xk / pv;
#pragma unroll
                    for (int c = 0; c < PW; ++c) {
                        if (c == k) x[q][c] = l;
                        if (c > k) x[q][c] -= l * rowP[B][c];
                    }
                }
            }
        }
    }
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        const int64_t r = tid + LU_THREADS * q;
        if (r < h)
#pragma unroll
            for (int c = 0; c < PW; ++c)
                if (c < w) P[r + c * ldc] = x[q][c];
    }
}

// Apply the panel's row exchanges to every column outside [c0, c0 + w).
struct LuSwap {
    struct Args {
        int64_t n;
        double* C;
        int64_t ldc;
        const int32_t* piv;
        int64_t c0;
        int w;
    };
    static constexpr int NTH = 256, WPE = 0;
    static __device__ void run(const Args& a, int bx, int by);
};
__device__ void LuSwap::run(const Args& a, int bx, int)
{
    const int64_t n = a.n, ldc = a.ldc, c0 = a.c0;
    const int w = a.w;
    double* __restrict__ C = a.C;
    const int32_t* __restrict__ piv = a.piv;
    const int64_t j = (int64_t)bx * 256 + threadIdx.x;
    if (j >= n || (j >= c0 && j < c0 + w)) return;
    double* col = C + j * ldc;
    for (int k = 0; k < w; ++k) {
        const int64_t p = piv[c0 + k];
        const int64_t r = c0 + k;
        if (p != r) { double t = col[r]; col[r] = col[p]; col[p] = t; }
    }
}

template <int RPT, int PW>
static void lu_steps(Exec& ex, int64_t n, double* C, int64_t ldc, int32_t* piv, int32_t* info, int64_t c0)
{
    ex.iter((uint32_t)c0);
    const int w = (int)((n - c0 < PW) ? n - c0 : PW);
    const int64_t h = n - c0;
    launch<LuPanel<RPT, PW>>(ex, 1, 1, LuPanelArgs{h, w, C + c0 + c0 * ldc, ldc, piv, c0, info});
    launch<LuSwap>(ex, ceil_div(n, 256), 1, LuSwap::Args{n, C, ldc, piv, c0, w});
    const int64_t rem = n - c0 - w;
    if (rem <= 0) return;
    double* C12 = C + c0 + (c0 + w) * ldc;
    // U12^T L11^T = C12^T: row j of U12^T is column j of C12 (stride 1 along
    // the row, ldc between rows)
    trsm_leaf<double, true, true>(ex, rem, w, C12, ldc, 1, C + c0 + c0 * ldc, ldc);
    GemmArgs g{};
    g.M = rem; g.N = rem; g.K = w;
    g.A = C + (c0 + w) + c0 * ldc; g.lda = ldc; g.transA = 0;
    g.B = C12; g.ldb = ldc; g.transB = 0;
    g.alpha = -1.0; g.beta = 1.0;
    double* C22 = C + (c0 + w) + (c0 + w) * ldc;
    g.Cin = C22; g.ldcin = ldc; g.C = C22; g.ldc = ldc;
    g.splits = 1;
    gemm_f64(ex, g);
}

bool lu_supported(int64_t n) { return n <= 4096; }

void lu_factor(Exec& ex, int64_t n, double* C, int64_t ldc, int32_t* piv, int32_t* info)
{
    int64_t c0 = 0;
    while (c0 < n) {
        const int64_t h = n - c0;
        if (h <= 512) { lu_steps<1, 32>(ex, n, C, ldc, piv, info, c0); c0 += 32; }
        else if (h <= 1024) { lu_steps<2, 32>(ex, n, C, ldc, piv, info, c0); c0 += 32; }
        else if (h <= 2048) { lu_steps<4, 16>(ex, n, C, ldc, piv, info, c0); c0 += 16; }
        else { lu_steps<8, 8>(ex, n, C, ldc, piv, info, c0); c0 += 8; }
    }
}

}  // namespace pne
