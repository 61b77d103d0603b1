// n-vector kernels of the solve and refinement steps (FP64 unless stated):
// single-work-group triangular solves (trsv_dev.h), the residual r = b - A x,
// the product y = X^T v split over rows with a fixed-order reduction, and
// small helpers.
#include "common.h"
#include "kernels.h"
#include "launch.h"
#include "trsv_dev.h"

namespace pne {

constexpr int TV_THREADS = 1024;
constexpr int TV_MAXN = 4096;   // largest n of the solvers (vector held in LDS)

size_t dinv_elems(int64_t n) { return (size_t)((n + TB - 1) / TB) * TB * TB; }

template <typename T>
void inv_diag_blocks(Exec& ex, int64_t n, const T* M, int64_t ld, int lower, int trans, int unit, T* Dinv,
                     int64_t block0, int64_t nblocks)
{
    if (nblocks < 0) nblocks = (n + TB - 1) / TB - block0;
    const InvDiagArgs a{n, M, ld, trans, unit, Dinv, block0};
    if (lower) launch<InvDiag<T, false>>(ex, nblocks, 1, a);
    else launch<InvDiag<T, true>>(ex, nblocks, 1, a);
}
template void inv_diag_blocks<double>(Exec&, int64_t, const double*, int64_t, int, int, int, double*, int64_t, int64_t);
template void inv_diag_blocks<float>(Exec&, int64_t, const float*, int64_t, int, int, int, float*, int64_t, int64_t);

// PNE solve in one work-group: L z = c, L^T y = z, R x = y, with the inverted
// diagonal blocks DL of L, DLt of L^T and DR of R.  L^T is read from its
// explicit copy Lt so that all three matrices are read by columns
// (contiguous across the threads of the update step).
struct PneSolve3 {
    struct Args {
        int64_t n;
        const double* L;
        int64_t ldl;
        const double* DL;
        const double* Lt;
        const double* DLt;
        const double* R;
        int64_t ldr;
        const double* DR;
        const double* c;
        double* x;
    };
    static constexpr int NTH = TV_THREADS, WPE = 0;
    static __device__ void run(const Args& a, int, int)
    {
        __shared__ double xs[TV_MAXN];
        __shared__ double tmp[TB];
        const int64_t n = a.n;
        for (int64_t i = threadIdx.x; i < n; i += NTH) xs[i] = a.c[i];
        __syncthreads();
        wg_trsv_inv<double>(n, a.L, a.ldl, true, false, a.DL, false, xs, tmp);
        wg_trsv_inv<double>(n, a.Lt, n, false, false, a.DLt, false, xs, tmp);
        wg_trsv_inv<double>(n, a.R, a.ldr, false, false, a.DR, false, xs, tmp);
        for (int64_t i = threadIdx.x; i < n; i += NTH) a.x[i] = xs[i];
    }
};

void pne_solve3(Exec& ex, int64_t n, const double* L, int64_t ldl, const double* DL, const double* Lt,
                const double* DLt, const double* R, int64_t ldr, const double* DR, const double* c,
                double* x)
{
    launch<PneSolve3>(ex, 1, 1, PneSolve3::Args{n, L, ldl, DL, Lt, DLt, R, ldr, DR, c, x});
}

// out(j, i) = in(i, j) through a 64 x 64 LDS tile per work-group.
struct Transpose {
    struct Args {
        int64_t r, c;
        const double* in;
        int64_t ldi;
        double* out;
        int64_t ldo;
        int64_t in_stride, out_stride;   // per blockIdx.y (batches of small matrices)
    };
    static constexpr int NTH = 256, WPE = 0;
    static __device__ void run(const Args& a, int bx, int by)
    {
        __shared__ double t[64 * 65];
        const int64_t tiles_r = (a.r + 63) / 64;
        const int64_t i0 = (bx % tiles_r) * 64, j0 = (bx / tiles_r) * 64;
        const double* __restrict__ in = a.in + by * a.in_stride;
        double* __restrict__ out = a.out + by * a.out_stride;
        for (int e = threadIdx.x; e < 64 * 64; e += NTH) {
            const int ii = e & 63, jj = e >> 6;
            const int64_t i = i0 + ii, j = j0 + jj;
            t[jj * 65 + ii] = (i < a.r && j < a.c) ? in[i + j * a.ldi] : 0.0;
        }
        __syncthreads();
        for (int e = threadIdx.x; e < 64 * 64; e += NTH) {
            const int jj = e & 63, ii = e >> 6;
            const int64_t i = i0 + ii, j = j0 + jj;
            if (i < a.r && j < a.c) out[j + i * a.ldo] = t[jj * 65 + ii];
        }
    }
};

void transpose_f64(Exec& ex, int64_t r, int64_t c, const double* in, int64_t ldi, double* out, int64_t ldo)
{
    launch<Transpose>(ex, ceil_div(r, 64) * ceil_div(c, 64), 1, Transpose::Args{r, c, in, ldi, out, ldo, 0, 0});
}

void transpose_dinv(Exec& ex, int64_t n, const double* D, double* Dt)
{
    launch<Transpose>(ex, 1, ceil_div(n, TB), Transpose::Args{TB, TB, D, TB, Dt, TB, TB * TB, TB * TB});
}

// HPNE solve: x = U^{-1} L^{-1} P c (row exchanges in order, unit lower L),
// with the inverted diagonal blocks DL (unit lower) and DU (upper).
struct LuSolve {
    struct Args {
        int64_t n;
        const double* LU;
        int64_t ld;
        const int32_t* piv;
        const double* DL;
        const double* DU;
        const double* c;
        double* x;
    };
    static constexpr int NTH = TV_THREADS, WPE = 0;
    static __device__ void run(const Args& a, int, int)
    {
        __shared__ double xs[TV_MAXN];
        __shared__ double tmp[TB];
        const int64_t n = a.n;
        for (int64_t i = threadIdx.x; i < n; i += NTH) xs[i] = a.c[i];
        __syncthreads();
        if (threadIdx.x == 0)
            for (int64_t k = 0; k < n; ++k) {
                const int64_t p = a.piv[k];
                if (p != k) { double t = xs[k]; xs[k] = xs[p]; xs[p] = t; }
            }
        __syncthreads();
        wg_trsv_inv<double>(n, a.LU, a.ld, true, false, a.DL, false, xs, tmp);
        wg_trsv_inv<double>(n, a.LU, a.ld, false, false, a.DU, false, xs, tmp);
        for (int64_t i = threadIdx.x; i < n; i += NTH) a.x[i] = xs[i];
    }
};

void lu_solve2(Exec& ex, int64_t n, const double* LU, int64_t ld, const int32_t* piv, const double* DL,
               const double* DU, const double* c, double* x)
{
    launch<LuSolve>(ex, 1, 1, LuSolve::Args{n, LU, ld, piv, DL, DU, c, x});
}

// r = b - A x, one row per thread, x staged in LDS in chunks of 4096.
struct Residual {
    struct Args {
        int64_t m, n;
        const double* A;
        int64_t lda;
        const double* b;
        const double* x;
        double* r;
    };
    static constexpr int NTH = 256, WPE = 0;
    static __device__ void run(const Args& a, int bx, int)
    {
        __shared__ double xs[4096];
        const int64_t m = a.m, n = a.n, lda = a.lda;
        const double* __restrict__ A = a.A;
        const int64_t i = (int64_t)bx * 256 + threadIdx.x;
        double acc = (i < m) ? a.b[i] : 0.0;
        for (int64_t j0 = 0; j0 < n; j0 += 4096) {
            const int64_t jw = (n - j0 < 4096) ? n - j0 : 4096;
            __syncthreads();
            for (int64_t j = threadIdx.x; j < jw; j += 256) xs[j] = a.x[j0 + j];
            __syncthreads();
            if (i < m)
                for (int64_t j = 0; j < jw; ++j) acc -= A[i + (j0 + j) * lda] * xs[j];
        }
        if (i < m) a.r[i] = acc;
    }
};

void residual(Exec& ex, int64_t m, int64_t n, const double* A, int64_t lda, const double* b, const double* x,
              double* r)
{
    launch<Residual>(ex, ceil_div(m, 256), 1, Residual::Args{m, n, A, lda, b, x, r});
}

// y = X^T v: work-group (column j, row chunk z) -> P[z * n + j]; then reduce.
constexpr int64_t GV_CHUNK = 16384;
size_t gemv_t_partials(int64_t m, int64_t n) { return (size_t)ceil_div(m, GV_CHUNK) * n; }

struct GemvT {
    struct Args {
        int64_t m, n;
        const double* X;
        int64_t ldx;
        const double* v;
        double* P;
    };
    static constexpr int NTH = 256, WPE = 0;
    static __device__ void run(const Args& a, int bx, int by)
    {
        __shared__ double red[4];
        const int64_t j = bx, z = by, m = a.m;
        const int64_t k0 = z * GV_CHUNK, k1 = (k0 + GV_CHUNK < m) ? k0 + GV_CHUNK : m;
        const double* __restrict__ X = a.X;
        const double* __restrict__ v = a.v;
        double s = 0.0;
        for (int64_t k = k0 + threadIdx.x; k < k1; k += 256) s += X[k + j * a.ldx] * v[k];
        s = block_sum(s, red);
        if (threadIdx.x == 0) a.P[z * a.n + j] = s;
    }
};

struct GemvTReduce {
    struct Args {
        int64_t n, splits;
        const double* P;
        double* y;
    };
    static constexpr int NTH = 256, WPE = 0;
    static __device__ void run(const Args& a, int bx, int)
    {
        const int64_t j = (int64_t)bx * 256 + threadIdx.x;
        if (j >= a.n) return;
        double s = 0.0;
        for (int64_t z = 0; z < a.splits; ++z) s += a.P[z * a.n + j];
        a.y[j] = s;
    }
};

void gemv_t(Exec& ex, int64_t m, int64_t n, const double* X, int64_t ldx, const double* v, double* y,
            double* P)
{
    const int64_t splits = ceil_div(m, GV_CHUNK);
    launch<GemvT>(ex, n, splits, GemvT::Args{m, n, X, ldx, v, P});
    launch<GemvTReduce>(ex, ceil_div(n, 256), 1, GemvTReduce::Args{n, splits, P, y});
}

struct Axpy {
    struct Args {
        int64_t n;
        double* x;
        const double* d;
    };
    static constexpr int NTH = 256, WPE = 0;
    static __device__ void run(const Args& a, int bx, int)
    {
        const int64_t i = (int64_t)bx * 256 + threadIdx.x;
        if (i < a.n) a.x[i] += a.d[i];
    }
};
void axpy_update(Exec& ex, int64_t n, double* x, const double* d)
{
    launch<Axpy>(ex, ceil_div(n, 256), 1, Axpy::Args{n, x, d});
}

struct NanOnInfo {
    struct Args {
        int64_t n;
        double* x;
        const int32_t* info;
    };
    static constexpr int NTH = 256, WPE = 0;
    static __device__ void run(const Args& a, int bx, int)
    {
        const int64_t i = (int64_t)bx * 256 + threadIdx.x;
        if (i < a.n && *a.info != 0) a.x[i] = __builtin_nan("");
    }
};
void fill_nan_on_info(Exec& ex, int64_t n, double* x, const int32_t* info)
{
    launch<NanOnInfo>(ex, ceil_div(n, 256), 1, NanOnInfo::Args{n, x, info});
}

struct Copy2d {
    struct Args {
        int64_t r, c;
        const double* s;
        int64_t lds;
        double* d;
        int64_t ldd;
    };
    static constexpr int NTH = 256, WPE = 0;
    static __device__ void run(const Args& a, int bx, int)
    {
        const int64_t idx = (int64_t)bx * 256 + threadIdx.x;
        if (idx >= a.r * a.c) return;
        const int64_t i = idx % a.r, j = idx / a.r;
        a.d[i + j * a.ldd] = a.s[i + j * a.lds];
    }
};
void copy_f64(Exec& ex, int64_t r, int64_t c, const double* src, int64_t lds, double* dst, int64_t ldd)
{
    launch<Copy2d>(ex, ceil_div(r * c, 256), 1, Copy2d::Args{r, c, src, lds, dst, ldd});
}

struct ZeroI32 {
    struct Args {
        int64_t n;
        int32_t* p;
    };
    static constexpr int NTH = 256, WPE = 0;
    static __device__ void run(const Args& a, int bx, int)
    {
        const int64_t i = (int64_t)bx * 256 + threadIdx.x;
        if (i < a.n) a.p[i] = 0;
    }
};
void zero_i32(Exec& ex, int64_t n, int32_t* p) { launch<ZeroI32>(ex, ceil_div(n, 256), 1, ZeroI32::Args{n, p}); }

}  // namespace pne
