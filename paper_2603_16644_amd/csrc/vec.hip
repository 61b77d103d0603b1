// n-vector kernels of the solve and refinement steps (FP64 unless stated):
// inverses of the 64 x 64 diagonal blocks (trsv_dev.h), triangular solves
// with one work-group per 64-row block, the residual r = b - A x, the
// product y = X^T v split over rows with a fixed-order reduction, and small
// helpers.
#include "common.h"
#include "kernels.h"
#include "launch.h"
#include "trsv_dev.h"

namespace pne {

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

// ---------------------------------------------------------------- multi-work-group triangular solve
// x := U^{-1} x for a triangular n x n matrix U (column-major, lower or
// upper) with the inverses D of its 64 x 64 diagonal blocks (InvDiag
// layout), one work-group per block of 64 rows.  Work-groups take their
// block in dependency order from a ticket counter (forward for lower,
// backward for upper), so every block they wait for belongs to a
// work-group that is already running.  A work-group accumulates
// U(b, j) x_j over the finished blocks j as their flags are raised,
// forms x_b = D_b (c_b - sum), publishes x_b and raises its own flag.
// flags[0] is the ticket counter and flags[1 + b] the flag of block b; all
// must be zero at launch.  Waits are bounded: a flag that is not raised
// within about 2^24 polls is passed over so that the kernel ends; the
// result is then invalid and the info word receives 4000 + k + 1 (k the
// 0-based block waited for) unless an earlier failure is already recorded,
// which also makes the solver fill x with NaN.
constexpr int LB_THREADS = 256;

__device__ __forceinline__ void lb_wait(int32_t* f, int32_t* info, int64_t block)
{
    for (uint32_t it = 0; it < (1u << 24); ++it) {
        if (__hip_atomic_load(f, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) != 0) return;
        __builtin_amdgcn_s_sleep(1);
    }
    if (info) {
        int32_t expected = 0;
        __hip_atomic_compare_exchange_strong(info, &expected, 4000 + (int32_t)block + 1, __ATOMIC_RELAXED,
                                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// One triangular solve of the chain: U x = rhs (rhs == x: in place).  With
// rhs_flags set, the right-hand side block b is the output of another solve
// of the same launch and is read once that solve has raised rhs_flags[1 + b].
struct LBSolve {
    int64_t n;
    const double* M;
    int64_t ld;
    int lower;
    const double* D;
    const double* rhs;
    double* x;
    int32_t* flags;            // flags[1 + b]: block b of x is final
    const int32_t* rhs_flags;  // null, or the flags of the solve that writes rhs
    int32_t* info;             // status word for a wait that gives up (may be null)
};

// Work-group of the t-th block (in dependency order) of solve sv.
__device__ void lb_solve_block(const LBSolve& sv, int64_t t)
{
    __shared__ double xs[TB];
    __shared__ double red[4][TB];
    __shared__ double vb[TB];
    const int tid = threadIdx.x, i = tid & 63, p = tid >> 6;
    const int64_t n = sv.n, nb = (n + TB - 1) / TB;
    const int64_t b = sv.lower ? t : nb - 1 - t;
    const int64_t r0 = b * TB;
    const int bw = (int)((n - r0 < TB) ? n - r0 : TB);
    const double* __restrict__ M = sv.M;
    double s = 0.0;
    for (int64_t q = 0; q < t; ++q) {
        const int64_t j = sv.lower ? q : nb - 1 - q;
        const int64_t c0 = j * TB;
        const int jw = (int)((n - c0 < TB) ? n - c0 : TB);
        if (tid == 0) lb_wait(sv.flags + 1 + j, sv.info, j);
        __syncthreads();
        if (tid < TB)
            xs[tid] = (tid < jw) ? __hip_atomic_load(sv.x + c0 + tid, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                                 : 0.0;
        __syncthreads();
        if (i < bw) {
            double mv[16];
#pragma unroll
            for (int kk = 0; kk < 16; ++kk) {
                const int k = 16 * p + kk;
                mv[kk] = (k < jw) ? M[(r0 + i) + (c0 + k) * sv.ld] : 0.0;
            }
#pragma unroll
            for (int kk = 0; kk < 16; ++kk) s += mv[kk] * xs[16 * p + kk];
        }
        __syncthreads();
    }
    red[p][i] = s;
    if (sv.rhs_flags && tid == 0) lb_wait(const_cast<int32_t*>(sv.rhs_flags) + 1 + b, sv.info, b);
    __syncthreads();
    if (tid < TB) {
        double rv = 0.0;
        if (tid < bw)
            rv = sv.rhs_flags ? __hip_atomic_load(sv.rhs + r0 + tid, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                              : sv.rhs[r0 + tid];
        vb[tid] = (tid < bw) ? rv - (((red[0][tid] + red[1][tid]) + red[2][tid]) + red[3][tid]) : 0.0;
    }
    __syncthreads();
    const double* Db = sv.D + b * TB * TB;
    double u = 0.0;
    {
        double dv[16];
#pragma unroll
        for (int kk = 0; kk < 16; ++kk) {
            const int k = 16 * p + kk;
            dv[kk] = (k < bw && i < bw) ? Db[i + k * TB] : 0.0;
        }
#pragma unroll
        for (int kk = 0; kk < 16; ++kk) u += dv[kk] * vb[16 * p + kk];
    }
    red[p][i] = u;
    __syncthreads();
    if (tid < bw) {
        sv.x[r0 + tid] = ((red[0][tid] + red[1][tid]) + red[2][tid]) + red[3][tid];
        __threadfence();
    }
    __syncthreads();
    if (tid == 0) __hip_atomic_store(sv.flags + 1 + b, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

struct TrsvLB {
    struct Args {
        int64_t n;
        const double* M;
        int64_t ld;
        int lower;
        const double* D;
        double* x;          // in: right-hand side; out: solution
        int32_t* flags;     // 1 + ceil(n / 64) words, zero at launch
        int32_t* info;      // status word (may be null)
    };
    static constexpr int NTH = LB_THREADS, WPE = 0;
    static __device__ void run(const Args& a, int, int)
    {
        __shared__ int32_t tk;
        if (threadIdx.x == 0) tk = atomicAdd(a.flags, 1);
        __syncthreads();
        lb_solve_block(LBSolve{a.n, a.M, a.ld, a.lower, a.D, a.x, a.x, a.flags, nullptr, a.info}, tk);
    }
};

// Two chained solves in the same direction in one launch: U1 y = c, then
// U2 x = y.  Tickets alternate between them (2k: step k of the first, 2k+1:
// step k of the second), so the second follows one block behind the first
// and every block waits only for blocks holding smaller tickets.
struct TrsvLB2 {
    struct Args {
        LBSolve s1, s2;     // s2.rhs = s1.x, s2.rhs_flags = s1.flags
        int32_t* ticket;    // zero at launch
    };
    static constexpr int NTH = LB_THREADS, WPE = 0;
    static __device__ void run(const Args& a, int, int)
    {
        __shared__ int32_t tk;
        if (threadIdx.x == 0) tk = atomicAdd(a.ticket, 1);
        __syncthreads();
        const int64_t t = tk;
        if ((t & 1) == 0) lb_solve_block(a.s1, t >> 1);
        else lb_solve_block(a.s2, t >> 1);
    }
};

size_t lb_flag_words(int64_t n) { return (size_t)((n + TB - 1) / TB) + 1; }

static void trsv_lb(Exec& ex, int64_t n, const double* M, int64_t ld, int lower, const double* D, double* x,
                    int32_t* flags, int32_t* info)
{
    launch<TrsvLB>(ex, (n + TB - 1) / TB, 1, TrsvLB::Args{n, M, ld, lower, D, x, flags, info});
}

// Row exchanges of the LU pivots applied to x in order (one work-group).
struct ApplyPivots {
    struct Args {
        int64_t n;
        const int32_t* piv;
        double* x;
    };
    static constexpr int NTH = 256, WPE = 0;
    static __device__ void run(const Args& a, int, int)
    {
        __shared__ double xs[TV_MAXN];
        for (int64_t k = threadIdx.x; k < a.n; k += NTH) xs[k] = a.x[k];
        __syncthreads();
        if (threadIdx.x == 0)
            for (int64_t k = 0; k < a.n; ++k) {
                const int64_t p = a.piv[k];
                if (p != k && p >= 0 && p < a.n) { const double t = xs[k]; xs[k] = xs[p]; xs[p] = t; }
            }
        __syncthreads();
        for (int64_t k = threadIdx.x; k < a.n; k += NTH) a.x[k] = xs[k];
    }
};

void pne_solve_lb(Exec& ex, int64_t n, const double* L, int64_t ldl, const double* DL, const double* Lt,
                  const double* DLt, const double* R, int64_t ldr, const double* DR, const double* c, double* x,
                  double* y, int32_t* flags, int32_t* info)
{
    const int64_t fw = (int64_t)lb_flag_words(n);
    zero_i32(ex, 3 * fw, flags);
    if (c != x) copy_f64(ex, n, 1, c, n, x, n);
    trsv_lb(ex, n, L, ldl, 1, DL, x, flags, info);
    // L^T y = z into y, then R x = y, in one launch (both backward)
    const LBSolve s1{n, Lt, n, 0, DLt, x, y, flags + fw, nullptr, info};
    const LBSolve s2{n, R, ldr, 0, DR, y, x, flags + 2 * fw, flags + fw, info};
    const int64_t nb = (n + TB - 1) / TB;
    launch<TrsvLB2>(ex, 2 * nb, 1, TrsvLB2::Args{s1, s2, flags + fw});
}

void upper_solve_lb(Exec& ex, int64_t n, const double* U, int64_t ld, const double* DU, const double* c, double* x,
                    int32_t* flags, int32_t* info)
{
    zero_i32(ex, (int64_t)lb_flag_words(n), flags);
    if (c != x) copy_f64(ex, n, 1, c, n, x, n);
    trsv_lb(ex, n, U, ld, 0, DU, x, flags, info);
}

void lu_solve_lb(Exec& ex, int64_t n, const double* LU, int64_t ld, const int32_t* piv, const double* DL,
                 const double* DU, const double* c, double* x, int32_t* flags, int32_t* info)
{
    const int64_t fw = (int64_t)lb_flag_words(n);
    zero_i32(ex, 2 * fw, flags);
    if (c != x) copy_f64(ex, n, 1, c, n, x, n);
    launch<ApplyPivots>(ex, 1, 1, ApplyPivots::Args{n, piv, x});
    trsv_lb(ex, n, LU, ld, 1, DL, x, flags, info);
    trsv_lb(ex, n, LU, ld, 0, DU, x, flags + fw, info);
}

// r = b - A x.  A work-group takes 64 rows; its four wavefronts take the
// columns j = q (mod 4), q = 0..3, so four times as many waves stream A as
// with one row per thread, each lane with eight loads in flight; the four
// partial sums of a row are added in q order.  x is staged in LDS in chunks
// of 1024.
constexpr int RES_ROWS = 64, RES_XCHUNK = 1024;
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
        __shared__ double xs[RES_XCHUNK];
        __shared__ double part[4][RES_ROWS];
        const int64_t m = a.m, n = a.n, lda = a.lda;
        const double* __restrict__ A = a.A;
        const int lane = threadIdx.x & 63, q = threadIdx.x >> 6;
        const int64_t i = (int64_t)bx * RES_ROWS + lane;
        const bool in = i < m;
        const double* __restrict__ Ai = A + (in ? i : 0);
        double acc = 0.0;
        for (int64_t j0 = 0; j0 < n; j0 += RES_XCHUNK) {
            const int64_t jw = (n - j0 < RES_XCHUNK) ? n - j0 : RES_XCHUNK;
            __syncthreads();
            for (int64_t j = threadIdx.x; j < jw; j += NTH) xs[j] = a.x[j0 + j];
            __syncthreads();
            if (in) {
                int64_t j = q;
                for (; j + 28 < jw; j += 32) {
                    double v[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) v[u] = Ai[(j0 + j + 4 * u) * lda];
#pragma unroll
                    for (int u = 0; u < 8; ++u) acc = fma(v[u], xs[j + 4 * u], acc);
                }
                for (; j < jw; j += 4) acc = fma(Ai[(j0 + j) * lda], xs[j], acc);
            }
        }
        part[q][lane] = acc;
        __syncthreads();
        if (q == 0 && in) a.r[i] = a.b[i] - (((part[0][lane] + part[1][lane]) + part[2][lane]) + part[3][lane]);
    }
};

void residual(Exec& ex, int64_t m, int64_t n, const double* A, int64_t lda, const double* b, const double* x,
              double* r)
{
    launch<Residual>(ex, ceil_div(m, RES_ROWS), 1, Residual::Args{m, n, A, lda, b, x, r});
}

// y = X^T v: work-group (four columns from j, row chunk z) -> P[z * n + j..];
// then a fixed-order reduction over the chunks.
constexpr int64_t GV_CHUNK = 16384;
size_t gemv_t_partials(int64_t m, int64_t n) { return (size_t)ceil_div(m, GV_CHUNK) * n; }

constexpr int GV_COLS = 4;   // columns per work-group (v read once for all four)
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
        __shared__ double red[GV_COLS][4];
        const int64_t jb = (int64_t)bx * GV_COLS, z = by, m = a.m, n = a.n, ldx = a.ldx;
        const int64_t k0 = z * GV_CHUNK, k1 = (k0 + GV_CHUNK < m) ? k0 + GV_CHUNK : m;
        const double* __restrict__ X = a.X;
        const double* __restrict__ v = a.v;
        double s[GV_COLS];
        const double* Xc[GV_COLS];
#pragma unroll
        for (int c = 0; c < GV_COLS; ++c) {
            s[c] = 0.0;
            Xc[c] = X + ((jb + c < n) ? jb + c : jb) * ldx;
        }
        for (int64_t k = k0 + threadIdx.x; k < k1; k += NTH) {
            const double vk = v[k];
#pragma unroll
            for (int c = 0; c < GV_COLS; ++c) s[c] += Xc[c][k] * vk;
        }
        const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
        for (int c = 0; c < GV_COLS; ++c) {
            const double t = wave_sum(s[c]);
            if (lane == 0) red[c][w] = t;
        }
        __syncthreads();
        if (threadIdx.x < GV_COLS && jb + threadIdx.x < n) {
            const int c = threadIdx.x;
            a.P[z * n + jb + c] = ((red[c][0] + red[c][1]) + red[c][2]) + red[c][3];
        }
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
    launch<GemvT>(ex, ceil_div(n, GV_COLS), splits, GemvT::Args{m, n, X, ldx, v, P});
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

struct CopyI32 {
    struct Args {
        int64_t n;
        const int32_t* s;
        int32_t* d;
    };
    static constexpr int NTH = 256, WPE = 0;
    static __device__ void run(const Args& a, int bx, int)
    {
        const int64_t i = (int64_t)bx * 256 + threadIdx.x;
        if (i < a.n) a.d[i] = a.s[i];
    }
};
void copy_i32(Exec& ex, int64_t n, const int32_t* src, int32_t* dst)
{
    launch<CopyI32>(ex, ceil_div(n, 256), 1, CopyI32::Args{n, src, dst});
}

// Input scan of pne_opts::check_finite: the m x n entries of A and the m of
// b, a grid-stride loop over both; any thread that meets a NaN or an
// infinity stores 5000 (every such store writes the same value).
struct AllFiniteArgs {
    int64_t m, n;
    const double* A;
    int64_t lda;
    const double* b;
    int32_t* info;
    int64_t stride;   // threads of the launch
};
struct AllFinite {
    typedef AllFiniteArgs Args;
    static constexpr int NTH = 256, WPE = 0;
    static __device__ void run(const AllFiniteArgs& a, int bx, int)
    {
        const int64_t mn = a.m * a.n;
        bool bad = false;
        for (int64_t e = (int64_t)bx * NTH + threadIdx.x; e < mn + a.m; e += a.stride) {
            double v;
            if (e < mn) {
                const int64_t j = e / a.m;
                v = a.A[(e - j * a.m) + j * a.lda];
            } else {
                v = a.b[e - mn];
            }
            bad = bad || !isfinite(v);
        }
        if (bad) *a.info = 5000;
    }
};

void all_finite(Exec& ex, int64_t m, int64_t n, const double* A, int64_t lda, const double* b, int32_t* info)
{
    int64_t g = ceil_div(m * n + m, (int64_t)AllFinite::NTH * 8);
    if (g > 4096) g = 4096;
    if (g < 1) g = 1;
    launch<AllFinite>(ex, g, 1, AllFiniteArgs{m, n, A, lda, b, info, g * AllFinite::NTH});
}

}  // namespace pne
