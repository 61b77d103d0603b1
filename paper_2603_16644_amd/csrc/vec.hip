// n-vector kernels of the solve and refinement steps (FP64 unless stated):
// single-work-group triangular solves (trsv_dev.h), the residual r = b - A x, the product y = X^T v split over
// rows with a fixed-order reduction, and small helpers.
#include "common.h"
#include "kernels.h"
#include "trsv_dev.h"

namespace pne {

constexpr int TV_THREADS = 1024;

template <typename T>
__global__ __launch_bounds__(TV_THREADS) void trsv_kernel(int64_t n, const T* __restrict__ M, int64_t ld,
                                                          int uplo, int trans, int unit, T* __restrict__ x)
{
    extern __shared__ unsigned char smem[];
    __shared__ T dblk[TB * TBL];
    T* xs = (T*)smem;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) xs[i] = x[i];
    __syncthreads();
    wg_trsv<T>(n, M, ld, (uplo == 0) != (trans != 0), trans != 0, unit != 0, xs, dblk);
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) x[i] = xs[i];
}

template <typename T>
void trsv(int64_t n, const T* M, int64_t ld, int uplo, int trans, int unit, T* x, hipStream_t st)
{
    trsv_kernel<T><<<1, TV_THREADS, n * sizeof(T), st>>>(n, M, ld, uplo, trans, unit, x);
}
template void trsv<double>(int64_t, const double*, int64_t, int, int, int, double*, hipStream_t);
template void trsv<float>(int64_t, const float*, int64_t, int, int, int, float*, hipStream_t);

size_t dinv_elems(int64_t n) { return (size_t)((n + TB - 1) / TB) * TB * TB; }

template <typename T>
void inv_diag_blocks(int64_t n, const T* M, int64_t ld, int lower, int trans, int unit, T* Dinv, hipStream_t st)
{
    inv_diag_blocks_kernel<T><<<(n + TB - 1) / TB, 64, 0, st>>>(n, M, ld, lower, trans, unit, Dinv);
}
template void inv_diag_blocks<double>(int64_t, const double*, int64_t, int, int, int, double*, hipStream_t);
template void inv_diag_blocks<float>(int64_t, const float*, int64_t, int, int, int, float*, hipStream_t);

// PNE solve in one launch: L z = c, L^T y = z, R x = y, with the inverted
// diagonal blocks DL of L and DR of R.
__global__ __launch_bounds__(TV_THREADS) void pne_solve3_kernel(int64_t n, const double* __restrict__ L,
                                                                int64_t ldl, const double* __restrict__ DL,
                                                                const double* __restrict__ R, int64_t ldr,
                                                                const double* __restrict__ DR,
                                                                const double* __restrict__ c,
                                                                double* __restrict__ x)
{
    extern __shared__ unsigned char smem[];
    __shared__ double tmp[TB];
    double* xs = (double*)smem;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) xs[i] = c[i];
    __syncthreads();
    wg_trsv_inv<double>(n, L, ldl, true, false, DL, false, xs, tmp);
    wg_trsv_inv<double>(n, L, ldl, false, true, DL, true, xs, tmp);
    wg_trsv_inv<double>(n, R, ldr, false, false, DR, false, xs, tmp);
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) x[i] = xs[i];
}

void pne_solve3(int64_t n, const double* L, int64_t ldl, const double* DL, const double* R, int64_t ldr,
                const double* DR, const double* c, double* x, hipStream_t st)
{
    pne_solve3_kernel<<<1, TV_THREADS, n * sizeof(double), st>>>(n, L, ldl, DL, R, ldr, DR, c, x);
}

// HPNE solve: x = U^{-1} L^{-1} P c (row exchanges in order, unit lower L),
// with the inverted diagonal blocks DL (unit lower) and DU (upper).
__global__ __launch_bounds__(TV_THREADS) void lu_solve_kernel(int64_t n, const double* __restrict__ LU,
                                                              int64_t ld, const int32_t* __restrict__ piv,
                                                              const double* __restrict__ DL,
                                                              const double* __restrict__ DU,
                                                              const double* __restrict__ c,
                                                              double* __restrict__ x)
{
    extern __shared__ unsigned char smem[];
    __shared__ double tmp[TB];
    double* xs = (double*)smem;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) xs[i] = c[i];
    __syncthreads();
    if (threadIdx.x == 0)
        for (int64_t k = 0; k < n; ++k) {
            const int64_t p = piv[k];
            if (p != k) { double t = xs[k]; xs[k] = xs[p]; xs[p] = t; }
        }
    __syncthreads();
    wg_trsv_inv<double>(n, LU, ld, true, false, DL, false, xs, tmp);
    wg_trsv_inv<double>(n, LU, ld, false, false, DU, false, xs, tmp);
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) x[i] = xs[i];
}

void lu_solve2(int64_t n, const double* LU, int64_t ld, const int32_t* piv, const double* DL, const double* DU,
               const double* c, double* x, hipStream_t st)
{
    lu_solve_kernel<<<1, TV_THREADS, n * sizeof(double), st>>>(n, LU, ld, piv, DL, DU, c, x);
}

// r = b - A x, one row per thread, x staged in LDS in chunks of 4096.
__global__ __launch_bounds__(256) void residual_kernel(int64_t m, int64_t n, const double* __restrict__ A,
                                                       int64_t lda, const double* __restrict__ b,
                                                       const double* __restrict__ x, double* __restrict__ r)
{
    __shared__ double xs[4096];
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    double acc = (i < m) ? b[i] : 0.0;
    for (int64_t j0 = 0; j0 < n; j0 += 4096) {
        const int64_t jw = (n - j0 < 4096) ? n - j0 : 4096;
        __syncthreads();
        for (int64_t j = threadIdx.x; j < jw; j += 256) xs[j] = x[j0 + j];
        __syncthreads();
        if (i < m)
            for (int64_t j = 0; j < jw; ++j) acc -= A[i + (j0 + j) * lda] * xs[j];
    }
    if (i < m) r[i] = acc;
}

void residual(int64_t m, int64_t n, const double* A, int64_t lda, const double* b, const double* x,
              double* r, hipStream_t st)
{
    residual_kernel<<<ceil_div(m, 256), 256, 0, st>>>(m, n, A, lda, b, x, r);
}

// y = X^T v: work-group (column j, row chunk z) -> P[z * n + j]; then reduce.
constexpr int64_t GV_CHUNK = 16384;
size_t gemv_t_partials(int64_t m, int64_t n) { return (size_t)ceil_div(m, GV_CHUNK) * n; }

__global__ __launch_bounds__(256) void gemv_t_kernel(int64_t m, int64_t n, const double* __restrict__ X,
                                                     int64_t ldx, const double* __restrict__ v,
                                                     double* __restrict__ P)
{
    __shared__ double red[4];
    const int64_t j = blockIdx.x, z = blockIdx.y;
    const int64_t k0 = z * GV_CHUNK, k1 = (k0 + GV_CHUNK < m) ? k0 + GV_CHUNK : m;
    double s = 0.0;
    for (int64_t k = k0 + threadIdx.x; k < k1; k += 256) s += X[k + j * ldx] * v[k];
    s = block_sum(s, red);
    if (threadIdx.x == 0) P[z * n + j] = s;
}

__global__ __launch_bounds__(256) void gemv_t_reduce_kernel(int64_t n, int64_t splits,
                                                            const double* __restrict__ P,
                                                            double* __restrict__ y)
{
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= n) return;
    double s = 0.0;
    for (int64_t z = 0; z < splits; ++z) s += P[z * n + j];
    y[j] = s;
}

void gemv_t(int64_t m, int64_t n, const double* X, int64_t ldx, const double* v, double* y, double* P,
            hipStream_t st)
{
    const int64_t splits = ceil_div(m, GV_CHUNK);
    gemv_t_kernel<<<dim3(n, splits), 256, 0, st>>>(m, n, X, ldx, v, P);
    gemv_t_reduce_kernel<<<ceil_div(n, 256), 256, 0, st>>>(n, splits, P, y);
}

__global__ void axpy_kernel(int64_t n, double* x, const double* d)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) x[i] += d[i];
}
void axpy_update(int64_t n, double* x, const double* d, hipStream_t st)
{
    axpy_kernel<<<ceil_div(n, 256), 256, 0, st>>>(n, x, d);
}

__global__ void nan_on_info_kernel(int64_t n, double* x, const int32_t* info)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n && *info != 0) x[i] = __builtin_nan("");
}
void fill_nan_on_info(int64_t n, double* x, const int32_t* info, hipStream_t st)
{
    nan_on_info_kernel<<<ceil_div(n, 256), 256, 0, st>>>(n, x, info);
}

__global__ void copy_kernel(int64_t n, const double* s, double* d)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) d[i] = s[i];
}
void copy_f64(int64_t n, const double* src, double* dst, hipStream_t st)
{
    copy_kernel<<<ceil_div(n, 256), 256, 0, st>>>(n, src, dst);
}

__global__ void zero_kernel(int64_t n, int32_t* p)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = 0;
}
void zero_i32(int64_t n, int32_t* p, hipStream_t st) { zero_kernel<<<ceil_div(n, 256), 256, 0, st>>>(n, p); }

}  // namespace pne
