// LU factorization with partial pivoting P C = L U of the n x n HPNE matrix
// A_p^T A (Section 1, eq. e_hpne; the system is non-symmetric).  Blocked,
// right-looking:
//   panel (PW = 32, 16 or 8 columns, all rows below), one 512-thread work-group:
//     the panel in registers; per column the pivot is the first row of
//     largest magnitude (wavefront argmax, ties to the smaller index), the
//     two rows are exchanged through LDS, the column is scaled and the rest
//     of the panel gets the rank-1 update;
//   the other columns, one thread per column over many work-groups: the
//     panel's row exchanges (composed into one permutation of at most 2 PW
//     rows, so a column's loads are all in flight together instead of one
//     exchange after another) and, right of the panel, U12 := L11^{-1} C12
//     (unit lower forward substitution);
//   C22 -= L21 U12 (MFMA GEMM).
// A zero or non-finite pivot at global column k sets *info = 3000 + k + 1
// (first only); that column's elimination is skipped.
#include "common.h"
#include "kernels.h"
#include "launch.h"

namespace pne {

constexpr int LU_THREADS = 512;
constexpr int LU_WAVES = LU_THREADS / 64;

// Shared state of the panel kernel.  Rows k and p and the per-wavefront
// argmax candidates are double-buffered by the parity of the step, so step
// k + 1 never overwrites what a slower thread of step k still reads.
template <int PW>
struct LuShared {
    double rowK[2][PW], rowP[2][PW], rowPu[2][PW];
    double wv[2][LU_WAVES];
    int64_t wi[2][LU_WAVES];
    int32_t pivl[PW];              // pivot rows of the panel (relative to its first row)
};

// Panel of the blocked LU in one 512-thread work-group: the panel
// C(c0:n, c0:c0+w) factored in registers (partial pivoting), written back
// with its pivot rows.  LuTail then applies the exchanges to the other
// columns and forms U12; the trailing update C22 -= L21 U12 follows as an
// MFMA GEMM launch.
struct LuPanelArgs {
    int64_t n;
    int w;
    double* C;
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
    const int64_t n = a.n, ldc = a.ldc, c0 = a.c0, h = n - c0;
    const int w = a.w;
    double* __restrict__ C = a.C;
    double* __restrict__ P = C + c0 + c0 * ldc;
    __shared__ LuShared<PW> sh;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wid = tid >> 6;
    int32_t* __restrict__ info = a.info;
    double x[RPT][PW];
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        const int64_t r = tid + LU_THREADS * q;
#pragma unroll
        for (int c = 0; c < PW; ++c) x[q][c] = (r < h && c < w) ? P[r + c * ldc] : 0.0;
    }
    // Column step k with the active column at register position J (a
    // compile-time constant).  The register row is rotated left after every
    // block of steps, so that every register index stays a compile-time
    // constant; after step k the columns already factored sit at the end
    // (positions PW - k .. PW - 1) or, inside a block, before J.  Two
    // barriers per step: after the wavefront argmax candidates are published
    // (every thread then forms the pivot row itself) and after the owners of
    // rows k and p publish them.  The owner of the pivot row also publishes
    // it with the factored columns zeroed (rowPu), which the rank-1 update
    // uses, so that no thread tests column positions.
    auto colstep = [&](auto jc, int k) {
        constexpr int J = decltype(jc)::value;
        const int B = k & 1;
        // argmax |x(r, k)| over r >= k, first index on ties; a NaN counts as
        // +inf, so a column holding one selects a non-finite pivot
        double best = -1.0;
        int64_t bidx = INT64_MAX;
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            const int64_t r = tid + LU_THREADS * q;
            double v = fabs(x[q][J]);
            if (v != v) v = INFINITY;
            if (r >= k && r < h && v > best) { best = v; bidx = r; }
        }
        wave_argmax(best, bidx);
        if (lane == 0) { sh.wv[B][wid] = best; sh.wi[B][wid] = bidx; }
        __syncthreads();
        double bb = sh.wv[B][0];
        int64_t p = sh.wi[B][0];
        for (int i = 1; i < LU_WAVES; ++i)
            if (sh.wv[B][i] > bb || (sh.wv[B][i] == bb && sh.wi[B][i] < p)) { bb = sh.wv[B][i]; p = sh.wi[B][i]; }
        if (p < k || p >= h) p = k;   // no candidate: keep the row in place
        if (tid == 0) sh.pivl[k] = (int32_t)p;
        const int live = PW - k + J;  // positions J .. live - 1 are not factored yet
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            const int64_t r = tid + LU_THREADS * q;
            if (r == p)
#pragma unroll
                for (int c = 0; c < PW; ++c) {
                    sh.rowP[B][c] = x[q][c];
                    sh.rowPu[B][c] = c < live ? x[q][c] : 0.0;
                }
            if (r == k)
#pragma unroll
                for (int c = 0; c < PW; ++c) sh.rowK[B][c] = x[q][c];
        }
        __syncthreads();
        const double pv = sh.rowP[B][J];
        const bool ok = pv != 0.0 && isfinite(pv);
        if (!ok && tid == 0 && *info == 0) *info = 3000 + (int32_t)(c0 + k) + 1;
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            const int64_t r = tid + LU_THREADS * q;
            // exchange rows k and p
            if (r == k && p != k)
#pragma unroll
                for (int c = 0; c < PW; ++c) x[q][c] = sh.rowP[B][c];
            if (r == p && p != k)
#pragma unroll
                for (int c = 0; c < PW; ++c) x[q][c] = sh.rowK[B][c];
            // multiplier and rank-1 update of the rows below k
            if (ok && r > k && r < h) {
                const double l = x[q][J] / pv;
                x[q][J] = l;
#pragma unroll
                for (int c = J + 1; c < PW; ++c) x[q][c] -= l * sh.rowPu[B][c];
            }
        }
    };
    // rotate the register row left by S positions
    auto rotate = [&](auto sc) {
        constexpr int S = decltype(sc)::value;
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            double t[S];
#pragma unroll
            for (int c = 0; c < S; ++c) t[c] = x[q][c];
#pragma unroll
            for (int c = 0; c < PW - S; ++c) x[q][c] = x[q][c + S];
#pragma unroll
            for (int c = 0; c < S; ++c) x[q][PW - S + c] = t[c];
        }
    };
    // blocks of four steps (one rotation per block), then single steps
    int k = 0;
#pragma unroll 1
    for (; k + 4 <= w; k += 4) {
        colstep(std::integral_constant<int, 0>{}, k);
        colstep(std::integral_constant<int, 1>{}, k + 1);
        colstep(std::integral_constant<int, 2>{}, k + 2);
        colstep(std::integral_constant<int, 3>{}, k + 3);
        rotate(std::integral_constant<int, 4>{});
    }
#pragma unroll 1
    for (; k < w; ++k) {
        colstep(std::integral_constant<int, 0>{}, k);
        rotate(std::integral_constant<int, 1>{});
    }
    // position c now holds panel column (c + w) mod PW
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        const int64_t r = tid + LU_THREADS * q;
#pragma unroll
        for (int c = 0; c < PW; ++c) {
            int col = c + w;
            if (col >= PW) col -= PW;
            if (r < h && col < w) P[r + col * ldc] = x[q][c];
        }
    }
    if (tid < w) a.piv[c0 + tid] = (int32_t)(c0 + sh.pivl[tid]);
}

// The row exchanges of a factored panel (pivots piv[c0 .. c0+w)) applied to
// every column outside it, and U12 := L11^{-1} C12 right of it; one thread
// per column.  The exchanges, applied in order k = 0 .. w-1 to the rows
// c0 + k and piv[c0 + k], move values among at most 2 w rows: one thread
// composes them into a table (row slot s receives the value that row slot
// perm[s] held before the panel), then every column loads all the values it
// needs before it stores any.
template <int PW>
struct LuTail {
    struct Args {
        int64_t n;
        int w;
        double* C;
        int64_t ldc;
        const int32_t* piv;
        int64_t c0;
    };
    static constexpr int NTH = 64, WPE = 0;
    static __device__ void run(const Args& a, int bx, int by);
};
template <int PW>
__device__ void LuTail<PW>::run(const Args& a, int bx, int)
{
    __shared__ double L11[PW][PW + 1];
    __shared__ int32_t srow[2 * PW];   // local row of each slot (slots < w: the panel rows)
    __shared__ int32_t perm[2 * PW];
    __shared__ int32_t nslot;
    const int64_t n = a.n, ldc = a.ldc, c0 = a.c0;
    const int w = a.w;
    double* __restrict__ C = a.C;
    const int tid = threadIdx.x;
    for (int e = tid; e < PW * PW; e += NTH) {
        const int i = e % PW, l = e / PW;
        L11[i][l] = (i < w && l < i) ? C[(c0 + i) + (c0 + l) * ldc] : 0.0;
    }
    if (tid == 0) {
        int ns = w;
        for (int s = 0; s < w; ++s) { srow[s] = s; perm[s] = s; }
        for (int k = 0; k < w; ++k) {
            const int pk = a.piv[c0 + k] - (int32_t)c0;
            int sp = pk;
            if (pk >= w) {
                sp = -1;
                for (int s = w; s < ns; ++s)
                    if (srow[s] == pk) sp = s;
                if (sp < 0) { sp = ns; srow[ns] = pk; perm[ns] = ns; ++ns; }
            }
            if (sp != k) { const int t = perm[k]; perm[k] = perm[sp]; perm[sp] = t; }
        }
        nslot = ns;
    }
    __syncthreads();
    // column of this thread: the columns left of the panel, then right of it
    const int64_t jj = (int64_t)bx * NTH + tid;
    if (jj >= n - w) return;
    const int64_t j = jj < c0 ? jj : jj + w;
    double* __restrict__ col = C + j * ldc + c0;
    const int ns = nslot;
    double u[PW], vo[PW];
#pragma unroll
    for (int i = 0; i < PW; ++i) u[i] = (i < w) ? col[srow[perm[i]]] : 0.0;
#pragma unroll
    for (int s = 0; s < PW; ++s) vo[s] = (w + s < ns) ? col[srow[perm[w + s]]] : 0.0;
#pragma unroll
    for (int s = 0; s < PW; ++s)
        if (w + s < ns) col[srow[w + s]] = vo[s];
    if (j >= c0 + w) {
#pragma unroll
        for (int i = 1; i < PW; ++i) {
            double v = u[i];
#pragma unroll
            for (int l = 0; l < i; ++l) v -= L11[i][l] * u[l];
            u[i] = v;
        }
    }
#pragma unroll
    for (int i = 0; i < PW; ++i)
        if (i < w) col[i] = u[i];
}

template <int RPT, int PW>
static void lu_steps(Exec& ex, int64_t n, double* C, int64_t ldc, int32_t* piv, int32_t* info, int64_t c0)
{
    ex.iter((uint32_t)c0);
    const int w = (int)((n - c0 < PW) ? n - c0 : PW);
    launch<LuPanel<RPT, PW>>(ex, 1, 1, LuPanelArgs{n, w, C, ldc, piv, c0, info});
    if (n > w)
        launch<LuTail<PW>>(ex, ceil_div(n - w, 64), 1, typename LuTail<PW>::Args{n, w, C, ldc, piv, c0});
    const int64_t rem = n - c0 - w;
    if (rem <= 0) return;
    GemmArgs g{};
    g.M = rem; g.N = rem; g.K = w;
    g.A = C + (c0 + w) + c0 * ldc; g.lda = ldc; g.transA = 0;
    g.B = C + c0 + (c0 + w) * ldc; g.ldb = ldc; g.transB = 0;
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
