// Householder QR of the s x n sketch A_s keeping only R_s (Algorithm 1,
// "Thin QR factorization A_s = Q_s R_s"; Section 5.2), then the promotion of
// R_s to FP64 (Algorithm 1, "Promote R_s").
//
// Blocked compact-WY form (Golub & Van Loan, Section 5.2.3):
//   panel:  one 512-thread work-group holds the h x NB panel in registers
//           (thread t owns rows t, t+512, ...) and applies NB reflectors
//           in the LAPACK convention (beta = -sign(alpha) ||x||); each
//           column needs one norm reduction and one batched reduction that
//           delivers both the dot products v^T P(:, j) of the update and the
//           V^T v column of the triangular factor T (H_1..H_NB = I - V T V^T);
//   update: Y^T = W_trail^T V (MFMA GEMM, split over rows), Z = T^T Y,
//           W_trail -= V Z (MFMA GEMM).
// Working precision: FP64 for qr_prec = FP64, FP32 otherwise.  For BF16 and
// FP16 the input is rounded to the format before the factorization and R_s
// after it (FP32 arithmetic in between).
#include "common.h"
#include "convert.h"
#include "kernels.h"

namespace pne {

template <typename T, int NB>
__device__ __forceinline__ void batched_block_sum(T (&v)[NB], T (*red)[NB], T* bc, int nw)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    constexpr int LOGNB = (NB == 32) ? 5 : (NB == 16 ? 4 : 3);
    // transpose-reduce: each halving step keeps half the entries and adds the
    // partner lane's copy of them
#pragma unroll
    for (int step = 0; step < LOGNB; ++step) {
        const int o = 32 >> step;
        const int half = NB >> (step + 1);
        const bool hi = (lane & o) != 0;
#pragma unroll
        for (int i = 0; i < half; ++i) {
            const T keep = hi ? v[i + half] : v[i];
            const T send = hi ? v[i] : v[i + half];
            v[i] = keep + __shfl_xor(send, o, 64);
        }
    }
    T s = v[0];
#pragma unroll
    for (int o = (32 >> LOGNB); o >= 1; o >>= 1) s += __shfl_xor(s, o, 64);
    const int idx = (lane >> (6 - LOGNB)) & (NB - 1);
    if ((lane & ((64 >> LOGNB) - 1)) == 0) red[wid][idx] = s;
    __syncthreads();
    if (threadIdx.x < NB) {
        T t = 0;
        for (int i = 0; i < nw; ++i) t += red[i][threadIdx.x];
        bc[threadIdx.x] = t;
    }
    __syncthreads();
}

constexpr int QR_THREADS = 512;
constexpr int QR_WAVES = QR_THREADS / 64;

template <typename T, int NB, int RPT>
__global__ __launch_bounds__(QR_THREADS) void qr_panel_kernel(int64_t h, int w, T* __restrict__ W, int64_t ldw,
                                                        T* __restrict__ V, int64_t ldv,
                                                        T* __restrict__ Tout)
{
    __shared__ T red[QR_WAVES][NB];
    __shared__ T bc[NB];
    __shared__ T rs[QR_WAVES];
    __shared__ T sc[3];
    __shared__ T Ts[NB][NB + 1];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    for (int e = tid; e < NB * NB; e += QR_THREADS) Ts[e / NB][e % NB] = 0;
    T x[RPT][NB];
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        const int64_t r = tid + QR_THREADS * q;
#pragma unroll
        for (int c = 0; c < NB; ++c) x[q][c] = (r < h && c < w) ? W[r + c * ldw] : (T)0;
    }
    for (int k = 0; k < w; ++k) {
        // sigma = sum_{r > k} x(r, k)^2
        T part = 0;
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            const int64_t r = tid + QR_THREADS * q;
#pragma unroll
            for (int c = 0; c < NB; ++c)
                if (c == k && r > k) part += x[q][c] * x[q][c];
        }
        part = wave_sum(part);
        if (lane == 0) rs[wid] = part;
        __syncthreads();
        if (tid == k) {
            T sigma = 0;
            for (int i = 0; i < QR_WAVES; ++i) sigma += rs[i];
            T alpha = 0;
#pragma unroll
            for (int c = 0; c < NB; ++c)
                if (c == k) alpha = x[0][c];
            T beta, tau, scl;
            if (sigma == (T)0) {
                beta = alpha; tau = 0; scl = 0;
            } else {
                const T nrm = sqrt(alpha * alpha + sigma);
                beta = (alpha >= (T)0) ? -nrm : nrm;
                tau = (beta - alpha) / beta;
                scl = (T)1 / (alpha - beta);
            }
            sc[0] = beta; sc[1] = tau; sc[2] = scl;
        }
        __syncthreads();
        const T beta = sc[0], tau = sc[1], scl = sc[2];
        // v: scaled below the diagonal, 1 on it, 0 above
        T vr[RPT];
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            const int64_t r = tid + QR_THREADS * q;
            T cur = 0;
#pragma unroll
            for (int c = 0; c < NB; ++c)
                if (c == k) {
                    if (r > k && tau != (T)0) x[q][c] *= scl;
                    cur = x[q][c];
                }
            vr[q] = (r > k) ? ((tau != (T)0) ? cur : (T)0) : (r == k ? (T)1 : (T)0);
        }
        // vals[c < k] = V(:, c)^T v ; vals[c > k] = v^T P(:, c)
        T vals[NB];
#pragma unroll
        for (int c = 0; c < NB; ++c) vals[c] = 0;
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            const int64_t r = tid + QR_THREADS * q;
#pragma unroll
            for (int c = 0; c < NB; ++c) {
                T vc;
                if (c < k) vc = (r > c) ? x[q][c] : (r == c ? (T)1 : (T)0);
                else if (c > k && c < w) vc = x[q][c];
                else vc = 0;
                vals[c] += vc * vr[q];
            }
        }
        batched_block_sum<T, NB>(vals, red, bc, QR_WAVES);
        // rank-1 update of the remaining panel columns
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
#pragma unroll
            for (int c = 0; c < NB; ++c)
                if (c > k && c < w) x[q][c] -= tau * bc[c] * vr[q];
        }
        // T(0:k, k) = -tau T(0:k, 0:k) (V^T v),  T(k, k) = tau
        if (tid < k) {
            T s = 0;
            for (int l = tid; l < k; ++l) s += Ts[tid][l] * bc[l];
            Ts[tid][k] = -tau * s;
        }
        if (tid == k) {
            Ts[k][k] = tau;
#pragma unroll
            for (int c = 0; c < NB; ++c)
                if (c == k) x[0][c] = beta;
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        const int64_t r = tid + QR_THREADS * q;
        if (r >= h) continue;
#pragma unroll
        for (int c = 0; c < NB; ++c) {
            if (c >= w) continue;
            const T val = x[q][c];
            W[r + c * ldw] = (r <= c) ? val : (T)0;
            V[r + c * ldv] = (r > c) ? val : (r == c ? (T)1 : (T)0);
        }
    }
    for (int e = tid; e < NB * NB; e += QR_THREADS) Tout[(e % NB) + (e / NB) * NB] = Ts[e % NB][e / NB];
}

// Z(:, j) = T^T sum_z P[z](j, :)^T for each column j of the trailing matrix.
// P[z] is (rem x NB, ld rem) = partial (W_trail^T V).
template <typename T, int NB>
__global__ __launch_bounds__(256) void qr_tz_kernel(int64_t rem, int w, const T* __restrict__ P,
                                                    int64_t splits, const T* __restrict__ Tm,
                                                    T* __restrict__ Z)
{
    __shared__ T Ts[NB * NB];
    for (int e = threadIdx.x; e < NB * NB; e += 256) Ts[e] = Tm[e];
    __syncthreads();
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= rem) return;
    T y[NB];
#pragma unroll
    for (int c = 0; c < NB; ++c) {
        T s = 0;
        if (c < w)
            for (int64_t z = 0; z < splits; ++z) s += P[z * rem * w + j + c * rem];
        y[c] = s;
    }
#pragma unroll
    for (int i = 0; i < NB; ++i) {
        if (i >= w) continue;
        T s = 0;
#pragma unroll
        for (int l = 0; l <= i; ++l) s += Ts[l + i * NB] * y[l];
        Z[i + j * NB] = s;
    }
}

template <typename T>
__global__ __launch_bounds__(256) void round_matrix_kernel(int64_t rows, int64_t cols, T* M, int64_t ld,
                                                           int prec)
{
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= rows * cols) return;
    const int64_t i = idx % rows, j = idx / rows;
    float v = (float)M[i + j * ld];
    if (prec == PNE_PREC_BF16) v = __uint_as_float((uint32_t)f32_to_bf16_bits(v) << 16);
    else if (prec == PNE_PREC_FP16) v = (float)__builtin_bit_cast(_Float16, f32_to_f16_bits(v));
    M[i + j * ld] = (T)v;
}

// R = upper triangle of W(0:n, 0:n) promoted to FP64 (rounded to BF16/FP16
// first for those precisions).
template <typename T>
__global__ __launch_bounds__(256) void extract_r_kernel(int64_t n, const T* __restrict__ W, int64_t ldw,
                                                        int prec, double* __restrict__ R, int64_t ldr)
{
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= n * n) return;
    const int64_t i = idx % n, j = idx / n;
    double v = 0.0;
    if (i <= j) {
        if constexpr (sizeof(T) == 8) {
            v = W[i + j * ldw];
        } else {
            float f = W[i + j * ldw];
            if (prec == PNE_PREC_BF16) f = __uint_as_float((uint32_t)f32_to_bf16_bits(f) << 16);
            else if (prec == PNE_PREC_FP16) f = (float)__builtin_bit_cast(_Float16, f32_to_f16_bits(f));
            v = (double)f;
        }
    }
    R[i + j * ldr] = v;
}

// First zero on the diagonal of R -> *info = 1000 + k + 1 (if no earlier failure).
__global__ __launch_bounds__(1024) void r_diag_check_kernel(int64_t n, const double* __restrict__ R,
                                                            int64_t ldr, int32_t* __restrict__ info)
{
    __shared__ int64_t wmin[16];
    int64_t mine = n;
    for (int64_t k = threadIdx.x; k < n; k += 1024)
        if (R[k + k * ldr] == 0.0 && k < mine) mine = k;
    mine = -wave_max(-mine);
    if ((threadIdx.x & 63) == 0) wmin[threadIdx.x >> 6] = mine;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t f = n;
        for (int i = 0; i < 16; ++i) f = wmin[i] < f ? wmin[i] : f;
        if (f < n && *info == 0) *info = 1000 + (int32_t)f + 1;
    }
}

struct QrShape {
    int nb, rpt;
};
// rows per thread from the fixed menu of spill-free instantiations
static int qr_rpt(int64_t s)
{
    const int need = (int)ceil_div(s, QR_THREADS);
    for (int r : {1, 2, 4, 6, 8, 12})
        if (r >= need) return r;
    return 0;
}
// panel width: 16 while the panel fits the 256 architectural VGPRs, else 8
template <typename T>
static QrShape qr_shape(int64_t s)
{
    const int rpt = qr_rpt(s);
    if (!rpt) return {0, 0};
    const int max16 = sizeof(T) == 8 ? 4 : 8;
    return {rpt <= max16 ? 16 : 8, rpt};
}

bool qr_supported(int64_t s, int prec)
{
    return prec == PNE_PREC_FP64 ? qr_shape<double>(s).nb > 0 : qr_shape<float>(s).nb > 0;
}

// upper bound of plan_splitk(h, tiles) over all panels (h <= s)
static int64_t qr_max_splits(int64_t s) { return (s / 256 > 1 ? s / 256 : 1) + 1; }

template <typename T>
static size_t qr_bytes(int64_t s, int64_t n)
{
    QrShape sh = qr_shape<T>(s);
    const int nb = sh.nb ? sh.nb : 8;
    const int64_t splits = qr_max_splits(s);
    Arena ar(nullptr, 0);
    ar.take<T>((size_t)s * nb);          // V
    ar.take<T>((size_t)nb * nb);         // T
    ar.take<T>((size_t)splits * n * nb); // partials of W^T V
    ar.take<T>((size_t)nb * n);          // Z
    return ar.used;
}

size_t qr_workspace_bytes(int64_t s, int64_t n, int prec)
{
    return prec == PNE_PREC_FP64 ? qr_bytes<double>(s, n) : qr_bytes<float>(s, n);
}

template <typename T, int NB, int RPT>
static void panel_launch(int64_t h, int w, T* Wp, int64_t ldw, T* V, int64_t ldv, T* Tm, hipStream_t st)
{
    qr_panel_kernel<T, NB, RPT><<<1, QR_THREADS, 0, st>>>(h, w, Wp, ldw, V, ldv, Tm);
}

// rows per thread: the smallest instantiated value covering the panel height
template <typename T, int NB>
static void panel_dispatch(int64_t h, int w, T* Wp, int64_t ldw, T* V, int64_t ldv, T* Tm,
                           hipStream_t st)
{
    constexpr int MAXR = (NB == 16) ? (sizeof(T) == 8 ? 4 : 8) : 12;
    const int r = qr_rpt(h);
    if (r <= 1) panel_launch<T, NB, 1>(h, w, Wp, ldw, V, ldv, Tm, st);
    else if (r <= 2) panel_launch<T, NB, 2>(h, w, Wp, ldw, V, ldv, Tm, st);
    else if (r <= 4) panel_launch<T, NB, 4>(h, w, Wp, ldw, V, ldv, Tm, st);
    else if constexpr (MAXR >= 8) {
        if (r <= 6) panel_launch<T, NB, 6>(h, w, Wp, ldw, V, ldv, Tm, st);
        else if (r <= 8) panel_launch<T, NB, 8>(h, w, Wp, ldw, V, ldv, Tm, st);
        else if constexpr (MAXR >= 12) panel_launch<T, NB, 12>(h, w, Wp, ldw, V, ldv, Tm, st);
    }
}

template <typename T>
static int qr_run(int64_t s, int64_t n, T* W, int64_t ldw, int prec, double* R, int64_t ldr,
                  int32_t* info, void* work, size_t work_bytes, hipStream_t st)
{
    if (work_bytes < qr_bytes<T>(s, n)) return PNE_EWORKSPACE;
    QrShape sh = qr_shape<T>(s);
    if (!sh.nb) return PNE_ENOTSUP;
    const int NBv = sh.nb;
    const int64_t splits_max = qr_max_splits(s);
    Arena ar(work, work_bytes);
    T* V = ar.take<T>((size_t)s * NBv);
    T* Tm = ar.take<T>((size_t)NBv * NBv);
    T* P = ar.take<T>((size_t)splits_max * n * NBv);
    T* Z = ar.take<T>((size_t)NBv * n);
    if constexpr (sizeof(T) == 4) {
        if (prec == PNE_PREC_BF16 || prec == PNE_PREC_FP16)
            round_matrix_kernel<T><<<ceil_div(s * n, 256), 256, 0, st>>>(s, n, W, ldw, prec);
    }
    for (int64_t c0 = 0; c0 < n; c0 += NBv) {
        const int w = (int)((n - c0 < NBv) ? n - c0 : NBv);
        const int64_t h = s - c0;
        T* Wp = W + c0 + c0 * ldw;
        if (NBv == 16) panel_dispatch<T, 16>(h, w, Wp, ldw, V, s, Tm, st);
        else panel_dispatch<T, 8>(h, w, Wp, ldw, V, s, Tm, st);
        const int64_t rem = n - c0 - w;
        if (rem <= 0) break;
        T* Wt = W + c0 + (c0 + w) * ldw;
        // P[z] = (W_trail^T V) over row chunks  (rem x w)
        GemmArgs g{};
        g.M = rem; g.N = w; g.K = h;
        g.A = Wt; g.lda = ldw; g.transA = 1;
        g.B = V; g.ldb = s; g.transB = 0;
        int64_t splits, kc;
        plan_splitk(h, ceil_div(rem, 128), &splits, &kc);
        g.splits = splits; g.kchunk = kc;
        g.P = P;
        if constexpr (sizeof(T) == 8) gemm_f64_partials(g, st);
        else gemm_f32_partials(g, st);
        if (NBv == 16) qr_tz_kernel<T, 16><<<ceil_div(rem, 256), 256, 0, st>>>(rem, w, P, splits, Tm, Z);
        else qr_tz_kernel<T, 8><<<ceil_div(rem, 256), 256, 0, st>>>(rem, w, P, splits, Tm, Z);
        // W_trail -= V Z
        GemmArgs u{};
        u.M = h; u.N = rem; u.K = w;
        u.A = V; u.lda = s; u.transA = 0;
        u.B = Z; u.ldb = NBv; u.transB = 0;
        u.alpha = -1.0; u.beta = 1.0;
        u.Cin = Wt; u.ldcin = ldw; u.C = Wt; u.ldc = ldw;
        u.splits = 1;
        if constexpr (sizeof(T) == 8) gemm_f64(u, st);
        else gemm_f32(u, st);
    }
    extract_r_kernel<T><<<ceil_div(n * n, 256), 256, 0, st>>>(n, W, ldw, prec, R, ldr);
    r_diag_check_kernel<<<1, 1024, 0, st>>>(n, R, ldr, info);
    return hipGetLastError() == hipSuccess ? PNE_OK : PNE_EHIP;
}

int qr_r(int64_t s, int64_t n, void* W, int64_t ldw, int prec, double* R, int64_t ldr, int32_t* info,
         void* work, size_t work_bytes, hipStream_t st)
{
    if (prec == PNE_PREC_FP64) return qr_run<double>(s, n, (double*)W, ldw, prec, R, ldr, info, work, work_bytes, st);
    return qr_run<float>(s, n, (float*)W, ldw, prec, R, ldr, info, work, work_bytes, st);
}

}  // namespace pne
