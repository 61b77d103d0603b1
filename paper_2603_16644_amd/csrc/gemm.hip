// Column-major MFMA GEMM for the FP64 (and FP32) contractions of the path:
// the off-diagonal updates of the blocked A R_s^{-1}, the Gram products
// A_p^T A_p / A_p^T A with A_p^T b, the trailing updates of the blocked
// Cholesky, LU and Householder QR, and the FP64 sketch product.
//
// C = alpha op(A) op(B) + beta Cin on 128 x BN output tiles (BN = 64 or 128),
// 256 threads = 2 x 2 waves, MFMA 16x16x4 (v_mfma_f64_16x16x4f64 or
// v_mfma_f32_16x16x4f32), K staged through LDS 16 deep with the next K tile
// prefetched into registers.  The MFMA operands are fed swapped (op(B)^T as
// the instruction's A, op(A)^T as its B) so that lane l owns output rows
// i = l % 16: consecutive lanes write consecutive addresses of the
// column-major result.  Output layout of the 16x16 result in lane l,
// register r: FP32 row 4*(l/16) + r, FP64 row l/16 + 4*r, column l % 16.  Split-K writes fixed partial buffers that a separate
// kernel reduces in a fixed order.
#include "common.h"
#include "kernels.h"
#include "tune.h"
#include "launch.h"

namespace pne {

constexpr int G_BK = 16, G_PAD = 16;

template <typename TC>
__device__ __forceinline__ auto mfma_cm(TC a, TC b,
                                        typename std::conditional<sizeof(TC) == 8, v4d, v4f>::type c)
{
    if constexpr (sizeof(TC) == 8) return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    else return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ void lower_tile(int64_t id, int64_t& ti, int64_t& tj)
{
    int64_t t = (int64_t)((sqrt(8.0 * (double)id + 1.0) - 1.0) * 0.5);
    while (t * (t + 1) / 2 > id) --t;
    while ((t + 1) * (t + 2) / 2 <= id) ++t;
    ti = t;
    tj = id - t * (t + 1) / 2;
}

template <typename TA, typename TB, typename TC, int BM, int BN, bool PARTIAL>
struct GemmCm {
    typedef GemmArgs Args;
    static constexpr int NTH = 256, WPE = BM == 64 ? 3 : 2;
    static constexpr bool PERSIST = true;   // no early return: may run as a persistent grouped launch
    static __device__ void run(const GemmArgs& g, int bx, int by);
};

template <typename TA, typename TB, typename TC, int BM, int BN, bool PARTIAL>
__device__ void GemmCm<TA, TB, TC, BM, BN, PARTIAL>::run(const GemmArgs& g, int bx, int by)
{
    typedef typename std::conditional<sizeof(TC) == 8, v4d, v4f>::type VC;
    constexpr int TM = BM / 32;                // 16-wide MFMA tiles per wave along M
    constexpr int TN = BN / 32;                // 16-wide MFMA tiles per wave along N
    constexpr int LDA_S = BM + G_PAD, LDB_S = BN + G_PAD;
    constexpr int APT = BM / 16;               // A elements per thread per K tile
    constexpr int BPT = BN / 16;               // B elements per thread per K tile
    constexpr int TPR = 256 / BM;              // threads per row of op(A) (transposed load)
    // two LDS buffers: the tile in use and the next one
    __shared__ __attribute__((aligned(16))) TC As[2][G_BK * LDA_S];
    __shared__ __attribute__((aligned(16))) TC Bs[2][G_BK * LDB_S];
    __shared__ TC bsh[2][G_BK];

    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wm = w & 1, wn = w >> 1;
    const int r16 = lane & 15, g4 = lane >> 4;

    int64_t ti, tj;
    const int64_t tiles_m = (g.M + BM - 1) / BM;
    if (PARTIAL && g.xcd_remap) {
        // Work-group L of a launch runs on XCD L % 8.  Renumber so that every
        // XCD gets a contiguous run of (K chunk, tile) work: the tiles of one
        // K chunk then read their operand panels through the same L2, which
        // cuts the L2 misses of the Gram product about threefold.
        const int64_t gxw = gridDim.x, T = gxw * gridDim.y;
        const int64_t L = bx + (int64_t)by * gxw;
        const int64_t x = L % 8, slot = L / 8, q = T / 8, r = T % 8;
        const int64_t v = x * q + (x < r ? x : r) + slot;
        bx = (int)(v % gxw);
        by = (int)(v / gxw);
    }
    // K chunk of the work-group: by, or, with a separate split of the
    // diagonal tiles (one-dimensional grid), from the work-group index: the
    // first tiles_m * splits_diag work-groups take the diagonal tiles, the
    // rest the tiles below the diagonal
    int64_t split = by, kc = g.kchunk;
    if (PARTIAL && g.lower && g.splits_diag > 0) {
        const int64_t v = bx + (int64_t)by * gridDim.x;
        const int64_t nd = tiles_m * g.splits_diag;
        if (v < nd) {
            ti = tj = v % tiles_m;
            split = v / tiles_m;
            kc = g.kchunk_diag;
        } else {
            const int64_t u = v - nd, nf = tiles_m * (tiles_m - 1) / 2;
            lower_tile(u % nf, ti, tj);
            ++ti;
            split = u / nf;
        }
    } else if (g.lower) lower_tile(bx, ti, tj);
    else { ti = bx % tiles_m; tj = bx / tiles_m; }
    const int64_t i0 = ti * BM, j0 = tj * BN;
    const int64_t kbeg = PARTIAL ? split * kc : 0;
    int64_t kend = PARTIAL ? kbeg + kc : g.K;
    if (kend > g.K) kend = g.K;

    const TA* __restrict__ A = (const TA*)g.A;
    const TB* __restrict__ B = (const TB*)g.B;
    const double* __restrict__ bv = (const double*)g.bvec;
    // op(A) bvec is formed by the work-groups of the diagonal tiles of a
    // lower-triangle product (whose upper-right wavefront has no MFMA work)
    // and otherwise by those of the first tile column
    const bool fold = (bv != nullptr) && (g.lower ? ti == tj : tj == 0);
    // 16-byte vector loads when every run of APT (A) / BPT (B) elements is aligned
    const bool vecA = sizeof(TA) == 8 && ((g.lda & 1) == 0) && (((uintptr_t)A & 15) == 0);
    const bool vecB = sizeof(TB) == 8 && ((g.ldb & 1) == 0) && (((uintptr_t)B & 15) == 0);

    // on a diagonal tile of a lower-triangle product the wavefront with the
    // upper half of the rows and the right half of the columns lies above the
    // diagonal: it skips its MFMAs (its part of C stays alpha * 0 + beta * Cin)
    const bool idle = g.lower && BN == BM && ti == tj && wm < wn;
    VC acc[TM][TN];
#pragma unroll
    for (int a = 0; a < TM; ++a)
#pragma unroll
        for (int b = 0; b < TN; ++b) acc[a][b] = (VC){0, 0, 0, 0};
    TC cpart = 0;
    // quadrant and 16-column blocks of C that the wavefront writes, and the
    // thread's column of the op(A) b fold
    int ewm = wm, ewn = wn, bmask = (1 << TN) - 1, fc = tid;

    TC ra[APT], rb[BPT], rbv = 0;
    // Load the K tile starting at k0 into registers (zero outside the matrix).
    auto gload = [&](int64_t k0) {
        if (!g.transA) {
            const int kk = tid >> 4, ib = (tid & 15) * APT;
            const int64_t k = k0 + kk;
            const TA* p = A + (i0 + ib) + k * g.lda;
            if (vecA && k < kend && i0 + ib + APT <= g.M) {
#pragma unroll
                for (int q = 0; q < APT; q += 2) {
                    const double2 v = *(const double2*)(p + q);
                    ra[q] = (TC)v.x; ra[q + 1] = (TC)v.y;
                }
            } else {
#pragma unroll
                for (int q = 0; q < APT; ++q) ra[q] = (i0 + ib + q < g.M && k < kend) ? (TC)p[q] : (TC)0;
            }
        } else {
            const int ii = tid / TPR, kb = (tid % TPR) * APT;
            const int64_t i = i0 + ii;
            const TA* p = A + (k0 + kb) + i * g.lda;
            if (vecA && i < g.M && k0 + kb + APT <= kend) {
#pragma unroll
                for (int q = 0; q < APT; q += 2) {
                    const double2 v = *(const double2*)(p + q);
                    ra[q] = (TC)v.x; ra[q + 1] = (TC)v.y;
                }
            } else {
#pragma unroll
                for (int q = 0; q < APT; ++q) ra[q] = (i < g.M && k0 + kb + q < kend) ? (TC)p[q] : (TC)0;
            }
        }
        if (!g.transB) {
            constexpr int TPC = 256 / BN;  // threads per column
            const int jj = tid / TPC, kb = (tid % TPC) * BPT;
            const int64_t j = j0 + jj;
            const TB* p = B + (k0 + kb) + j * g.ldb;
            if (vecB && j < g.N && k0 + kb + BPT <= kend) {
#pragma unroll
                for (int q = 0; q < BPT; q += 2) {
                    const double2 v = *(const double2*)(p + q);
                    rb[q] = (TC)v.x; rb[q + 1] = (TC)v.y;
                }
            } else {
#pragma unroll
                for (int q = 0; q < BPT; ++q) rb[q] = (j < g.N && k0 + kb + q < kend) ? (TC)p[q] : (TC)0;
            }
        } else {
            const int kk = tid >> 4, jb = (tid & 15) * BPT;
            const int64_t k = k0 + kk;
            const TB* p = B + (j0 + jb) + k * g.ldb;
            if (vecB && k < kend && j0 + jb + BPT <= g.N) {
#pragma unroll
                for (int q = 0; q < BPT; q += 2) {
                    const double2 v = *(const double2*)(p + q);
                    rb[q] = (TC)v.x; rb[q + 1] = (TC)v.y;
                }
            } else {
#pragma unroll
                for (int q = 0; q < BPT; ++q) rb[q] = (j0 + jb + q < g.N && k < kend) ? (TC)p[q] : (TC)0;
            }
        }
        if (fold && tid < G_BK) rbv = (k0 + tid < kend) ? (TC)bv[k0 + tid] : (TC)0;
    };
    auto sstore = [&](int buf) {
        TC* as = As[buf];
        TC* bs = Bs[buf];
        if (!g.transA) {
            const int kk = tid >> 4, ib = (tid & 15) * APT;
#pragma unroll
            for (int q = 0; q < APT; ++q) as[kk * LDA_S + ib + q] = ra[q];
        } else {
            const int ii = tid / TPR, kb = (tid % TPR) * APT;
#pragma unroll
            for (int q = 0; q < APT; ++q) as[(kb + q) * LDA_S + ii] = ra[q];
        }
        if (!g.transB) {
            constexpr int TPC = 256 / BN;
            const int jj = tid / TPC, kb = (tid % TPC) * BPT;
#pragma unroll
            for (int q = 0; q < BPT; ++q) bs[(kb + q) * LDB_S + jj] = rb[q];
        } else {
            const int kk = tid >> 4, jb = (tid & 15) * BPT;
#pragma unroll
            for (int q = 0; q < BPT; ++q) bs[kk * LDB_S + jb + q] = rb[q];
        }
        if (fold && tid < G_BK) bsh[buf][tid] = rbv;
    };

    // FP32 products with a single K tile (the QR trailing update, K = panel
    // width): fetch the Cin values of the lane together with the operands.
    constexpr bool PRE = sizeof(TC) == 4 && !PARTIAL;
    TC pre[PRE ? TM : 1][PRE ? TN : 1][PRE ? 4 : 1];
    const bool use_pre = PRE && g.Cin != nullptr && (kend - kbeg) <= G_BK;
    if constexpr (PRE) {
        if (use_pre) {
            const TC* Cin0 = (const TC*)g.Cin;
#pragma unroll
            for (int a = 0; a < TM; ++a)
#pragma unroll
                for (int b = 0; b < TN; ++b)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int64_t i = i0 + wm * (BM / 2) + a * 16 + r16;
                        const int64_t j = j0 + wn * (BN / 2) + b * 16 + 4 * g4 + r;
                        pre[a][b][r] = (i < g.M && j < g.N) ? Cin0[i + j * g.ldcin] : (TC)0;
                    }
        }
    }

    // Diagonal tiles of a lower-triangle product (FP64, 128 x 128 tiles,
    // split-K, direct launches): the two wavefronts on the diagonal take
    // the lower triangles of their quadrants (10 of 16 MFMA blocks), and the
    // other two split the quadrant below the diagonal into 32-column halves
    // (8 blocks each), so that no SIMD carries more than 10 blocks per K
    // step; nobody computes the quadrant above the diagonal.  role: 0 =
    // whole quadrant, 1 = lower triangle, 2 / 3 = left / right half.  The
    // fold runs on the two half wavefronts.  (Grouped batch launches keep
    // the plain layout, with the wavefront above the diagonal idle.)
    constexpr bool ROLES_T = sizeof(TA) == 8 && sizeof(TB) == 8 && sizeof(TC) == 8 && BM == 128 && BN == 128 && PARTIAL;
    int role = 0;
    if constexpr (ROLES_T) {
        if (g.diag_roles && g.lower && ti == tj) {
            if (wm == wn) role = 1;
            else {
                ewm = 1;
                ewn = 0;
                role = (w == 1) ? 2 : 3;
                bmask = (role == 2) ? 0x3 : 0xC;
            }
            fc = tid - 64;
        }
        role = __builtin_amdgcn_readfirstlane(role);   // (uniform per wavefront)
    }

    // Fast path (FP64 operands, full tile off the diagonal of a lower-
    // triangle product, 16-byte aligned vector loads, a K range of at least
    // two whole tiles): no bounds checks, and every step of the steady state
    // is one basic block holding the LDS stores of the next K tile, the
    // global loads of the one after it and the MFMAs of the current one, so
    // that the scheduler can interleave them and the MFMA pipe keeps running
    // while they issue.  64 x 64 tiles only: on the products of A R^-1 it
    // raised the MFMA busy share from 57 % to 64 %, while the 128 x 128
    // tiles of the Gram product ran slower with it (61 % against 64 %).
    bool fast = false;
    if constexpr (sizeof(TA) == 8 && sizeof(TB) == 8 && sizeof(TC) == 8 && BM == 64)
        fast = vecA && vecB && i0 + BM <= g.M && j0 + BN <= g.N && ((kend - kbeg) % G_BK) == 0 &&
               kend - kbeg >= 2 * G_BK && !(g.lower && ti == tj);
    if constexpr (sizeof(TA) == 8 && sizeof(TB) == 8 && sizeof(TC) == 8 && BM == 64) {
      if (fast) {
        // the transposition flags as compile-time constants (one copy of the
        // loop per combination), so that no branch splits a step
        auto run_fast = [&](auto tra, auto trb) {
            constexpr bool TRA = decltype(tra)::value, TRB = decltype(trb)::value;
            double2 va[APT / 2], vb[BPT / 2];
            auto gload_fast = [&](int64_t k0) {
                const TA* pa;
                if constexpr (!TRA) pa = A + (i0 + (tid & 15) * APT) + (k0 + (tid >> 4)) * g.lda;
                else pa = A + (k0 + (tid % TPR) * APT) + (i0 + tid / TPR) * g.lda;
#pragma unroll
                for (int q = 0; q < APT / 2; ++q) va[q] = *(const double2*)(pa + 2 * q);
                const TB* pb;
                if constexpr (!TRB) pb = B + (k0 + (tid % (256 / BN)) * BPT) + (j0 + tid / (256 / BN)) * g.ldb;
                else pb = B + (j0 + (tid & 15) * BPT) + (k0 + (tid >> 4)) * g.ldb;
#pragma unroll
                for (int q = 0; q < BPT / 2; ++q) vb[q] = *(const double2*)(pb + 2 * q);
            };
            auto sstore_fast = [&](int b) {
                TC* as = As[b];
                TC* bs = Bs[b];
#pragma unroll
                for (int q = 0; q < APT; ++q) {
                    const TC v = (q & 1) ? va[q / 2].y : va[q / 2].x;
                    if constexpr (!TRA) as[(tid >> 4) * LDA_S + (tid & 15) * APT + q] = v;
                    else as[((tid % TPR) * APT + q) * LDA_S + tid / TPR] = v;
                }
#pragma unroll
                for (int q = 0; q < BPT; ++q) {
                    const TC v = (q & 1) ? vb[q / 2].y : vb[q / 2].x;
                    if constexpr (!TRB) bs[((tid % (256 / BN)) * BPT + q) * LDB_S + tid / (256 / BN)] = v;
                    else bs[(tid >> 4) * LDB_S + (tid & 15) * BPT + q] = v;
                }
            };
            auto compute = [&](int b) {
                const TC* as = As[b];
                const TC* bs = Bs[b];
#pragma unroll
                for (int kk = 0; kk < G_BK; kk += 4) {
                    TC fa[TM], fb[TN];
#pragma unroll
                    for (int t = 0; t < TM; ++t) fa[t] = as[(kk + g4) * LDA_S + wm * (BM / 2) + t * 16 + r16];
#pragma unroll
                    for (int t = 0; t < TN; ++t) fb[t] = bs[(kk + g4) * LDB_S + wn * (BN / 2) + t * 16 + r16];
#pragma unroll
                    for (int a = 0; a < TM; ++a)
#pragma unroll
                        for (int b2 = 0; b2 < TN; ++b2) acc[a][b2] = mfma_cm<TC>(fb[b2], fa[a], acc[a][b2]);
                }
            };
            // op(A) b for the folding work-groups, b read directly (uniform
            // addresses: scalar loads)
            auto fold_step = [&](int b, int64_t k0) {
                if (fold && tid < BM) {
#pragma unroll
                    for (int kk = 0; kk < G_BK; ++kk) cpart += As[b][kk * LDA_S + tid] * (TC)bv[k0 + kk];
                }
            };
            const int64_t nk = (kend - kbeg) / G_BK;
            gload_fast(kbeg);
            sstore_fast(0);
            gload_fast(kbeg + G_BK);
            int b = 0;
            for (int64_t t = 0; t + 2 < nk; ++t) {
                __syncthreads();
                fold_step(b, kbeg + t * G_BK);
                sstore_fast(b ^ 1);                     // tile t + 1
                gload_fast(kbeg + (t + 2) * G_BK);      // tile t + 2
                compute(b);                             // tile t
                b ^= 1;
            }
            __syncthreads();
            fold_step(b, kend - 2 * G_BK);
            sstore_fast(b ^ 1);
            compute(b);
            b ^= 1;
            __syncthreads();
            fold_step(b, kend - G_BK);
            compute(b);
        };
        using F = std::false_type;
        using T_ = std::true_type;
        if (!g.transA && !g.transB) run_fast(F{}, F{});
        else if (!g.transA) run_fast(F{}, T_{});
        else if (!g.transB) run_fast(T_{}, F{});
        else run_fast(T_{}, T_{});
      }
    }

    // Gram tiles (FP64, 128 x 128, op(A) = A^T and op(B) = B: both operands
    // stored with K contiguous, 16-byte aligned, whole K tiles): the loop
    // below without bounds checks (columns past the matrix read its last
    // column, whose results are never stored), one copy per role.
    bool gram = false;
    if constexpr (ROLES_T)
        gram = g.transA && !g.transB && vecA && vecB && ((kend - kbeg) % G_BK) == 0 && kend - kbeg >= 2 * G_BK;
    if constexpr (ROLES_T) {
      if (gram) {
        const int ii = tid >> 1, kb = (tid & 1) * APT;   // row of op(A) / column of op(B), K offset
        const int64_t ca = (i0 + ii < g.M) ? i0 + ii : g.M - 1;
        const int64_t cb = (j0 + ii < g.N) ? j0 + ii : g.N - 1;
        const TA* __restrict__ pa0 = A + ca * g.lda + kb;
        const TB* __restrict__ pb0 = B + cb * g.ldb + kb;
        double2 va[APT / 2], vb[BPT / 2];
        auto gl = [&](int64_t k0) {
#pragma unroll
            for (int q = 0; q < APT / 2; ++q) va[q] = *(const double2*)(pa0 + k0 + 2 * q);
#pragma unroll
            for (int q = 0; q < BPT / 2; ++q) vb[q] = *(const double2*)(pb0 + k0 + 2 * q);
        };
        auto ss = [&](int b) {
#pragma unroll
            for (int q = 0; q < APT; ++q) As[b][(kb + q) * LDA_S + ii] = (q & 1) ? va[q / 2].y : va[q / 2].x;
#pragma unroll
            for (int q = 0; q < BPT; ++q) Bs[b][(kb + q) * LDB_S + ii] = (q & 1) ? vb[q / 2].y : vb[q / 2].x;
        };
        auto gloop = [&](auto rl) {
            constexpr int RL = decltype(rl)::value;
            const int64_t nk = (kend - kbeg) / G_BK;
            gl(kbeg);
            ss(0);
            gl(kbeg + G_BK);
            int b = 0;
            for (int64_t t = 0; t < nk; ++t) {
                __syncthreads();
                const TC* as = As[b];
                const TC* bs = Bs[b];
#pragma unroll
                for (int kk = 0; kk < G_BK; kk += 4) {
                    if (RL == 0 && idle) break;
                    TC fa[TM], fb[TN];
#pragma unroll
                    for (int u = 0; u < TM; ++u) fa[u] = as[(kk + g4) * LDA_S + ewm * (BM / 2) + u * 16 + r16];
#pragma unroll
                    for (int u = 0; u < TN; ++u) fb[u] = bs[(kk + g4) * LDB_S + ewn * (BN / 2) + u * 16 + r16];
#pragma unroll
                    for (int a = 0; a < TM; ++a)
#pragma unroll
                        for (int c = 0; c < TN; ++c) {
                            if (RL == 1 && a < c) continue;
                            if (RL == 2 && c >= TN / 2) continue;
                            if (RL == 3 && c < TN / 2) continue;
                            acc[a][c] = mfma_cm<TC>(fb[c], fa[a], acc[a][c]);
                        }
                }
                // op(A) b, b read directly (uniform addresses: scalar loads)
                if (fold && fc >= 0 && fc < BM) {
                    const int64_t k0 = kbeg + t * G_BK;
#pragma unroll
                    for (int kk = 0; kk < G_BK; ++kk) cpart += as[kk * LDA_S + fc] * (TC)bv[k0 + kk];
                }
                if (t + 1 < nk) {
                    ss(b ^ 1);
                    if (t + 2 < nk) gl(kbeg + (t + 2) * G_BK);
                }
                b ^= 1;
            }
        };
        switch (role) {
        case 0: gloop(std::integral_constant<int, 0>{}); break;
        case 1: gloop(std::integral_constant<int, 1>{}); break;
        case 2: gloop(std::integral_constant<int, 2>{}); break;
        default: gloop(std::integral_constant<int, 3>{}); break;
        }
        fast = true;   // (the K loop has run)
      }
    }

    // Pipeline: tile t is in LDS buffer t % 2 while tile t + 1 is being
    // loaded into registers; one barrier per tile.  (A diagonal tile whose
    // K chunk takes this loop keeps the plain wavefront layout.)
    if constexpr (ROLES_T) {
        if (!fast && role != 0) {
            ewm = wm;
            ewn = wn;
            bmask = (1 << TN) - 1;
            fc = tid;
        }
    }
    int buf = 0;
    if (!fast && kbeg < kend) {
        gload(kbeg);
        sstore(0);
        if (kbeg + G_BK < kend) gload(kbeg + G_BK);
    }
    for (int64_t k0 = kbeg; !fast && k0 < kend; k0 += G_BK) {
        __syncthreads();
        const TC* as = As[buf];
        const TC* bs = Bs[buf];
#pragma unroll
        for (int kk = 0; kk < G_BK; kk += 4) {
            if (idle) break;
            TC fa[TM], fb[TN];
#pragma unroll
            for (int t = 0; t < TM; ++t) fa[t] = as[(kk + g4) * LDA_S + wm * (BM / 2) + t * 16 + r16];
#pragma unroll
            for (int t = 0; t < TN; ++t) fb[t] = bs[(kk + g4) * LDB_S + wn * (BN / 2) + t * 16 + r16];
#pragma unroll
            for (int a = 0; a < TM; ++a)
#pragma unroll
                for (int b = 0; b < TN; ++b) acc[a][b] = mfma_cm<TC>(fb[b], fa[a], acc[a][b]);
        }
        if (fold && tid < BM) {
#pragma unroll
            for (int kk = 0; kk < G_BK; ++kk) cpart += as[kk * LDA_S + tid] * bsh[buf][kk];
        }
        if (k0 + G_BK < kend) {
            sstore(buf ^ 1);
            if (k0 + 2 * G_BK < kend) gload(k0 + 2 * G_BK);
        }
        buf ^= 1;
    }

    // epilogue: lane owns rows i = .. + r16; accumulator register r holds
    // column j = .. + 4*g4 + r for the FP32 MFMA and j = .. + g4 + 4*r for the
    // FP64 MFMA (their 16x16 output layouts differ).  C may alias Cin: per row
    // tile every Cin value of the lane is loaded before the first store, so
    // the loads are not serialised behind stores one by one.
    TC* C = (TC*)g.C;
    const TC* Cin = (const TC*)g.Cin;
    TC* P = PARTIAL ? (TC*)g.P + split * g.M * g.N : nullptr;
    const TC* src = PARTIAL ? (g.accumulate_partials ? P : nullptr) : Cin;
    const int64_t lds_ = PARTIAL ? g.M : g.ldcin;
#pragma unroll
    for (int a = 0; a < TM; ++a) {
        const int64_t i = i0 + ewm * (BM / 2) + a * 16 + r16;
        TC prev[TN][4];
#pragma unroll
        for (int b = 0; b < TN; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t j = j0 + ewn * (BN / 2) + b * 16 + (sizeof(TC) == 8 ? g4 + 4 * r : 4 * g4 + r);
                if constexpr (PRE) {
                    if (use_pre) { prev[b][r] = pre[a][b][r]; continue; }
                }
                prev[b][r] = (src && ((bmask >> b) & 1) && i < g.M && j < g.N) ? src[i + j * lds_] : (TC)0;
            }
        if (i >= g.M) continue;
#pragma unroll
        for (int b = 0; b < TN; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t j = j0 + ewn * (BN / 2) + b * 16 + (sizeof(TC) == 8 ? g4 + 4 * r : 4 * g4 + r);
                if (j >= g.N || !((bmask >> b) & 1)) continue;
                if (PARTIAL) P[i + j * g.M] = acc[a][b][r] + prev[b][r];
                else C[i + j * g.ldc] = (TC)g.alpha * acc[a][b][r] + (TC)g.beta * prev[b][r];
            }
    }
    if (fold && fc >= 0 && fc < BM && i0 + fc < g.M) {
        if (PARTIAL) ((TC*)g.Pc)[split * g.M + i0 + fc] = cpart;
        else ((TC*)g.cvec)[i0 + fc] = cpart;
    }
}

struct GemmReduceArgs {
    GemmArgs g;
    int bm, bn;
};
template <typename TC>
struct GemmReduce {
    typedef GemmReduceArgs Args;
    static constexpr int NTH = 256, WPE = 0;
    static __device__ void run(const Args& a, int bx, int by);
};
template <typename TC>
__device__ void GemmReduce<TC>::run(const GemmReduceArgs& a, int bx, int)
{
    const GemmArgs& g = a.g;
    const int bm = a.bm, bn = a.bn;
    const int64_t idx = (int64_t)bx * 256 + threadIdx.x;
    const TC* P = (const TC*)g.P;
    const bool dsplit = g.lower && g.splits_diag > 0;
    if (idx < g.M * g.N) {
        const int64_t i = idx % g.M, j = idx / g.M;
        // lower-triangle products: the elements on and below the diagonal
        if (!g.lower || i >= j) {
            const int64_t nz = (dsplit && i / bm == j / bn) ? g.splits_diag : g.splits;
            TC s = 0;
            for (int64_t z = 0; z < nz; ++z) s += P[z * g.M * g.N + idx];
            TC v = (TC)g.alpha * s;
            if (g.Cin) v += (TC)g.beta * ((const TC*)g.Cin)[i + j * g.ldcin];
            ((TC*)g.C)[i + j * g.ldc] = v;
        }
    }
    if (g.bvec && idx < g.M) {
        const int64_t nz = dsplit ? g.splits_diag : g.splits;
        TC s = 0;
        for (int64_t z = 0; z < nz; ++z) s += ((const TC*)g.Pc)[z * g.M + idx];
        ((TC*)g.cvec)[idx] = s;
    }
}

// Output tile of a product.  64 x 64 when K is short (the tall products of
// A R^-1, the Cholesky and LU updates: three work-groups per CU and the finer
// grid beat the higher reuse of larger tiles).  Long-K products: lower
// triangles 64 x 64 up to order 512 (128-wide tiles would spend a large
// share of their work on padding) and 128 x 128 above; others 128 x 128, or
// 128 x 64 for N <= 64.
struct TileShape {
    int bm, bn;
};
// (The 64 / 512 choices are the defaults of TuneParams; the autotuner may
// replace them per workload, see tune.h.)
static TileShape tile_shape(int64_t, int64_t N, int64_t K, int lower)
{
    const TuneParams& tp = tune_params();
    if (K < 4096) return tp.shortk_tile == 128 ? TileShape{128, 128} : TileShape{64, 64};
    if (lower) return N <= tp.lower_small_n ? TileShape{64, 64} : TileShape{128, 128};
    return N <= 64 ? TileShape{128, 64} : TileShape{128, 128};
}

int64_t gemm_tiles(int64_t M, int64_t N, int64_t K, int lower)
{
    const TileShape ts = tile_shape(M, N, K, lower);
    const int64_t tm = ceil_div(M, ts.bm), tn = ceil_div(N, ts.bn);
    if (lower) return tm * (tm + 1) / 2;  // square tiles, square problems
    return tm * tn;
}

// Split-K plan for a product with `tiles` output tiles.  Alone on the
// machine: the number of splits (chunks of at least 128 along K) whose
// work-group count fills whole waves of the machine best (256 CUs x 2
// resident work-groups), preferring more work-groups when the fill is equal.
// In a batch (kchunk_fixed > 0) every product is cut into chunks of a fixed
// length instead, so that work-groups carry similar work across members.
void plan_splitk(int64_t K, int64_t tiles, int64_t* splits, int64_t* kchunk, int64_t kchunk_fixed)
{
    if (kchunk_fixed > 0) {
        const int64_t kc = ceil_div(kchunk_fixed < K ? kchunk_fixed : K, G_BK) * G_BK;
        *kchunk = kc > 0 ? kc : G_BK;
        *splits = K > 0 ? ceil_div(K, *kchunk) : 1;
        return;
    }
    const int64_t slots = 512;
    if (tiles < 1) tiles = 1;
    int64_t maxs = K / 128;
    if (maxs < 1) maxs = 1;
    if (maxs > 4 * slots) maxs = 4 * slots;
    int64_t best = 1;
    double best_eff = -1.0;
    for (int64_t sp = 1; sp <= maxs; ++sp) {
        const int64_t wg = tiles * sp;
        const int64_t waves = (wg + slots - 1) / slots;
        if (waves > 4) break;
        double eff = (double)wg / (double)(waves * slots);
        if (eff > best_eff + 1e-9) { best_eff = eff; best = sp; }
    }
    const int64_t kc = ceil_div(ceil_div(K, best), G_BK) * G_BK;
    *kchunk = kc;
    *splits = ceil_div(K, kc);
}

// Lower triangles in 128 x 128 tiles: the off-diagonal tiles keep their
// split count sf, and the diagonal tiles, whose busiest wavefront carries 10
// of the 16 MFMA blocks (see GemmCm::run), get a split count sd of their
// own; (sf, sd) minimises the K tiles times MFMA blocks of the largest
// work-group with all work-groups resident at once (two per CU), and is
// taken when it beats the uniform plan by more than 1 %.
void plan_splitk_gram(int64_t K, int64_t n, int lower, int64_t kchunk_fixed, int64_t* splits, int64_t* kchunk,
                      int64_t* splits_diag, int64_t* kchunk_diag)
{
    plan_splitk(K, gemm_tiles(n, n, K, lower), splits, kchunk, kchunk_fixed);
    *splits_diag = 0;
    *kchunk_diag = 0;
    if (!lower || kchunk_fixed > 0 || K < 2 * G_BK || tile_shape(n, n, K, lower).bm != 128) return;
    const int64_t slots = 512;
    const int64_t tm = ceil_div(n, 128), nf = tm * (tm - 1) / 2;
    const int64_t kt = ceil_div(K, G_BK);
    int64_t maxs = K / 128;
    if (maxs < 1) maxs = 1;
    const int64_t wg_u = (nf + tm) * *splits;
    double best = (double)ceil_div(wg_u, slots) * 16.0 * (double)ceil_div(kt, *splits);
    int64_t bf = 0, bd = 0;
    for (int64_t sf = nf ? 1 : 0; sf <= maxs && nf * sf + tm <= slots; ++sf) {
        int64_t sd = (slots - nf * sf) / tm;
        if (sd > maxs) sd = maxs;
        double c = 10.0 * (double)ceil_div(kt, sd);
        if (nf) {
            const double cf = 16.0 * (double)ceil_div(kt, sf);
            if (cf > c) c = cf;
        }
        if (c < 0.99 * best) {
            best = c;
            bf = sf;
            bd = sd;
        }
        if (!nf) break;
    }
    if (!bd) return;
    if (nf) {
        *kchunk = ceil_div(ceil_div(K, bf), G_BK) * G_BK;
        *splits = ceil_div(K, *kchunk);
    } else {
        *splits = 1;
    }
    *kchunk_diag = ceil_div(ceil_div(K, bd), G_BK) * G_BK;
    *splits_diag = ceil_div(K, *kchunk_diag);
}

template <typename TC>
static void gemm_reduce_launch(Exec& ex, const GemmArgs& g)
{
    const TileShape ts = tile_shape(g.M, g.N, g.K, g.lower);
    int64_t cnt = g.M * g.N;
    if (g.bvec && g.M > cnt) cnt = g.M;
    launch<GemmReduce<TC>>(ex, ceil_div(cnt, 256), 1, GemmReduceArgs{g, ts.bm, ts.bn});
}

template <typename TA, typename TB, typename TC, bool PARTIAL>
static void gemm_tiles_launch(Exec& ex, const TileShape& ts, int64_t gx, int64_t gy, const GemmArgs& g)
{
    if (ts.bm == 64) launch<GemmCm<TA, TB, TC, 64, 64, PARTIAL>>(ex, gx, gy, g);
    else if (ts.bn == 64) launch<GemmCm<TA, TB, TC, 128, 64, PARTIAL>>(ex, gx, gy, g);
    else launch<GemmCm<TA, TB, TC, 128, 128, PARTIAL>>(ex, gx, gy, g);
}

template <typename TA, typename TB, typename TC>
static void gemm_launch(Exec& ex, const GemmArgs& g0, bool reduce)
{
    GemmArgs g = g0;
    const TileShape ts = tile_shape(g.M, g.N, g.K, g.lower);
    const int64_t tiles = gemm_tiles(g.M, g.N, g.K, g.lower);
    if (tiles == 0) return;
    const bool partial = g.splits > 1 || !reduce;
    if (!partial) {
        g.splits = 1;
        g.xcd_remap = 0;
        gemm_tiles_launch<TA, TB, TC, false>(ex, ts, tiles, 1, g);
        return;
    }
    if (g.splits < 1) g.splits = 1;
    if (g.kchunk <= 0) g.kchunk = ceil_div(ceil_div(g.K, g.splits), G_BK) * G_BK;
    // (lower-triangle products only: on the FP64 sketch product, whose
    // grid is several waves of work-groups, it made the launch slower)
    g.xcd_remap = !ex.recording() && g.splits > 1 && g.lower;
    // (direct launches only; see GemmCm::run)
    g.diag_roles = !ex.recording();
    if (g.lower && g.splits_diag > 0) {
        // one-dimensional grid: diagonal tiles x splits_diag, then the tiles
        // below the diagonal x splits
        const int64_t tm = ceil_div(g.M, (int64_t)ts.bm);
        g.xcd_remap = !ex.recording();
        gemm_tiles_launch<TA, TB, TC, true>(ex, ts, tm * g.splits_diag + (tiles - tm) * g.splits, 1, g);
    } else {
        gemm_tiles_launch<TA, TB, TC, true>(ex, ts, tiles, g.splits, g);
    }
    if (reduce) gemm_reduce_launch<TC>(ex, g);
}

void gemm_f64(Exec& ex, const GemmArgs& g) { gemm_launch<double, double, double>(ex, g, true); }
void gemm_f64_reduce(Exec& ex, const GemmArgs& g) { gemm_reduce_launch<double>(ex, g); }
void gemm_f64_partials(Exec& ex, const GemmArgs& g) { gemm_launch<double, double, double>(ex, g, false); }
void gemm_f32(Exec& ex, const GemmArgs& g) { gemm_launch<float, float, float>(ex, g, true); }
void gemm_f32_partials(Exec& ex, const GemmArgs& g) { gemm_launch<float, float, float>(ex, g, false); }
void gemm_ddf(Exec& ex, const GemmArgs& g) { gemm_launch<double, double, float>(ex, g, true); }

}  // namespace pne
