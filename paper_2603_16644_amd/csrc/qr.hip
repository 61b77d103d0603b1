// Householder QR of the s x n sketch A_s keeping only R_s (Algorithm 1,
// "Thin QR factorization A_s = Q_s R_s"; Section 5.2), then the promotion of
// R_s to FP64 (Algorithm 1, "Promote R_s").
//
// Blocked compact-WY form (Golub & Van Loan, Section 5.2.3):
//   panel:  one work-group (512 or 1024 threads) holds the h x NB panel in
//           registers (thread t owns rows t, t+NT, ...) and applies NB reflectors
//           in the LAPACK convention (beta = -sign(alpha) ||x||); each
//           column needs a single batched reduction, which delivers the norm,
//           the dot products v^T P(:, j) of the update and the V^T v column of
//           the triangular factor T (H_1..H_NB = I - V T V^T);
//   update: Y^T = W_trail^T V (MFMA GEMM, split over rows), Z = T^T Y,
//           W_trail -= V Z (MFMA GEMM).
// Working precision: FP64 for qr_prec = FP64, FP32 otherwise.  For BF16 and
// FP16 the input is rounded to the format before the factorization and R_s
// after it (FP32 arithmetic in between).
#include "common.h"
#include "convert.h"
#include "kernels.h"
#include "launch.h"

namespace pne {

template <typename T, int NB>
__device__ __forceinline__ void batched_block_sum(T (&v)[NB], T (*red)[NB], T* bc, int nw)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    constexpr int LOGNB = (NB == 32) ? 5 : (NB == 16 ? 4 : 3);
    // transpose-reduce: each halving step keeps half the entries and adds the
    // partner lane's copy of them.  Both candidate sums are formed explicitly
    // (selecting between array entries with a lane-dependent condition would
    // be lowered to an indexed access over the whole array).
#pragma unroll
    for (int step = 0; step < LOGNB; ++step) {
        const int o = 32 >> step;
        const int half = NB >> (step + 1);
        const bool hi = (lane & o) != 0;
#pragma unroll
        for (int i = 0; i < half; ++i) {
            const T lo_sum = v[i] + __shfl_xor(v[i], o, 64);
            const T hi_sum = v[i + half] + __shfl_xor(v[i + half], o, 64);
            v[i] = hi ? hi_sum : lo_sum;
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


// Panel of h rows and w <= NB columns.  For column k one batched reduction
// over the rows r > k gives
//   s_c = sum_{r>k} x(r, k) x(r, c)   for every panel column c,
// i.e. sigma = s_k, the dot products of the trailing columns (c > k) and the
// products V(:, c)^T x of the earlier reflectors (c < k).  The thread that
// owns row k then forms (LAPACK convention) beta = -sign(alpha) sqrt(alpha^2
// + sigma), tau = (beta - alpha) / beta and v = [1; x(r>k) / (alpha - beta)],
// the coefficients tau v^T P(:, c) = tau (P(k, c) + s_c / (alpha - beta)) of
// the rank-1 update and the vector V^T v that extends the triangular factor T.
template <typename T, int NB, int NT>
struct PanelShared {
    T red[NT / 64][NB];
    T bc[NB];
    T cf[NB];      // tau * v^T P(:, c) for c > k
    T gv[NB];      // V(:, i)^T v for i < k
    T sc[2];       // 1 / (alpha - beta), tau
    T Ts[NB][NB + 1];
};

// One column step of the panel (see qr_panel_kernel).  KS >= 0 makes the
// column index a compile-time constant (KS == k); KS < 0 takes k at run time.
template <typename T, int NB, int RPT, int NT, int KS>
__device__ __forceinline__ void panel_step(int k_rt, int w, T (&x)[RPT][NB], PanelShared<T, NB, NT>& sh)
{
    const int k = KS >= 0 ? KS : k_rt;
    const int tid = threadIdx.x;
    T vals[NB];
#pragma unroll
    for (int c = 0; c < NB; ++c) vals[c] = 0;
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        const int64_t r = tid + NT * q;
        T xk = 0;
#pragma unroll
        for (int c = 0; c < NB; ++c)
            if (c == k) xk = x[q][c];
        xk = (r > k) ? xk : (T)0;
#pragma unroll
        for (int c = 0; c < NB; ++c) vals[c] += xk * x[q][c];
    }
    batched_block_sum<T, NB>(vals, sh.red, sh.bc, NT / 64);
    if (tid == k) {
        T alpha = 0;
#pragma unroll
        for (int c = 0; c < NB; ++c)
            if (c == k) alpha = x[0][c];
        const T sigma = sh.bc[k];
        T beta, tau, inv;
        if (sigma == (T)0) {
            beta = alpha; tau = 0; inv = 0;
        } else {
            const T nrm = sqrt(alpha * alpha + sigma);
            beta = (alpha >= (T)0) ? -nrm : nrm;
            tau = (beta - alpha) / beta;
            inv = (T)1 / (alpha - beta);
        }
#pragma unroll
        for (int c = 0; c < NB; ++c) {
            if (c > k && c < w) sh.cf[c] = tau * (x[0][c] + sh.bc[c] * inv);
            if (c < k) sh.gv[c] = x[0][c] + sh.bc[c] * inv;
            if (c == k) x[0][c] = beta;
        }
        sh.sc[0] = inv;
        sh.sc[1] = tau;
    }
    __syncthreads();
    const T inv = sh.sc[0], tau = sh.sc[1];
    // T(0:k, k) = -tau T(0:k, 0:k) (V^T v),  T(k, k) = tau
    if (tid < k) {
        T acc = 0;
        for (int l = tid; l < k; ++l) acc += sh.Ts[tid][l] * sh.gv[l];
        sh.Ts[tid][k] = -tau * acc;
    }
    if (tid == k) sh.Ts[k][k] = tau;
    // v (stored in place of column k below the diagonal) and the update,
    // branch free: v_r = 0 above row k, 1 on it, x(r, k) / (alpha - beta) below
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        const int64_t r = tid + NT * q;
        T xk = 0;
#pragma unroll
        for (int c = 0; c < NB; ++c)
            if (c == k) xk = x[q][c];
        const T scaled = xk * inv;
        const T vr = (r > k) ? scaled : ((r == k) ? (T)1 : (T)0);
#pragma unroll
        for (int c = 0; c < NB; ++c) {
            if (c == k) x[q][c] = (r > k) ? scaled : xk;
            if (c > k && c < w) x[q][c] -= sh.cf[c] * vr;
        }
    }
}

// Steps K, K+1, ..., NB-1 with compile-time column indices.
template <typename T, int NB, int RPT, int NT, int K>
struct PanelSteps {
    static __device__ __forceinline__ void run(int w, T (&x)[RPT][NB], PanelShared<T, NB, NT>& sh)
    {
        if (K >= w) return;
        panel_step<T, NB, RPT, NT, K>(K, w, x, sh);
        PanelSteps<T, NB, RPT, NT, K + 1>::run(w, x, sh);
    }
};
template <typename T, int NB, int RPT, int NT>
struct PanelSteps<T, NB, RPT, NT, NB> {
    static __device__ __forceinline__ void run(int, T (&)[RPT][NB], PanelShared<T, NB, NT>&) {}
};

// The column loop is unrolled (static register indices) for the shapes
// where that keeps the panel free of register spills, and left rolled
// otherwise (see QR_SHAPES).
struct QrPanelArgs {
    int64_t h;
    int w;
    void* W;
    int64_t ldw;
    void* V;
    int64_t ldv;
    void* Tout;
};
template <typename T, int NB, int RPT, int NT, bool UNROLL>
struct QrPanel {
    typedef QrPanelArgs Args;
    static constexpr int NTH = NT, WPE = 0;
    static __device__ void run(const QrPanelArgs& a, int bx, int by);
};
template <typename T, int NB, int RPT, int NT, bool UNROLL>
__device__ void QrPanel<T, NB, RPT, NT, UNROLL>::run(const QrPanelArgs& a, int, int)
{
    const int64_t h = a.h, ldw = a.ldw, ldv = a.ldv;
    const int w = a.w;
    T* __restrict__ W = (T*)a.W;
    T* __restrict__ V = (T*)a.V;
    T* __restrict__ Tout = (T*)a.Tout;
    __shared__ PanelShared<T, NB, NT> sh;
    const int tid = threadIdx.x;
    for (int e = tid; e < NB * NB; e += NT) sh.Ts[e / NB][e % NB] = 0;
    T x[RPT][NB];
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        const int64_t r = tid + NT * q;
#pragma unroll
        for (int c = 0; c < NB; ++c) x[q][c] = (r < h && c < w) ? W[r + c * ldw] : (T)0;
    }
    if constexpr (UNROLL) {
        PanelSteps<T, NB, RPT, NT, 0>::run(w, x, sh);
    } else {
        for (int k = 0; k < w; ++k) panel_step<T, NB, RPT, NT, -1>(k, w, x, sh);
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        const int64_t r = tid + NT * q;
        if (r >= h) continue;
#pragma unroll
        for (int c = 0; c < NB; ++c) {
            if (c >= w) continue;
            const T val = x[q][c];
            W[r + c * ldw] = (r <= c) ? val : (T)0;
            V[r + c * ldv] = (r > c) ? val : (r == c ? (T)1 : (T)0);
        }
    }
    for (int e = tid; e < NB * NB; e += NT) Tout[(e % NB) + (e / NB) * NB] = sh.Ts[e % NB][e / NB];
}

// Z(:, j) = T^T sum_z P[z](j, :)^T for each column j of the trailing matrix.
// P[z] is (rem x w, ld rem) = partial (W_trail^T V).  A work-group handles 16
// columns: the split partials are summed by (column, entry) threads into LDS,
// then each (column, entry) thread forms one entry of T^T y.
struct QrTzArgs {
    int64_t rem;
    int w;
    const void* P;
    int64_t splits;
    const void* Tm;
    void* Z;
};
template <typename T, int NB>
struct QrTz {
    typedef QrTzArgs Args;
    static constexpr int NTH = 256, WPE = 0;
    static __device__ void run(const QrTzArgs& a, int bx, int by);
};
template <typename T, int NB>
__device__ void QrTz<T, NB>::run(const QrTzArgs& a, int bx, int)
{
    const int64_t rem = a.rem, splits = a.splits;
    const int w = a.w;
    const T* __restrict__ P = (const T*)a.P;
    const T* __restrict__ Tm = (const T*)a.Tm;
    T* __restrict__ Z = (T*)a.Z;
    __shared__ T Ts[NB * NB];
    __shared__ T ys[NB][16];
    for (int e = threadIdx.x; e < NB * NB; e += 256) Ts[e] = Tm[e];
    const int jl = threadIdx.x & 15;
    const int64_t j = (int64_t)bx * 16 + jl;
    for (int l = threadIdx.x >> 4; l < NB; l += 16) {
        T s = 0;
        if (j < rem && l < w)
            for (int64_t z = 0; z < splits; ++z) s += P[z * rem * w + j + (int64_t)l * rem];
        ys[l][jl] = s;
    }
    __syncthreads();
    for (int i = threadIdx.x >> 4; i < NB; i += 16) {
        if (j >= rem || i >= w) continue;
        T s = 0;
        for (int l = 0; l <= i; ++l) s += Ts[l + i * NB] * ys[l][jl];
        Z[i + j * NB] = s;
    }
}

struct RoundMatrixArgs {
    int64_t rows, cols;
    void* M;
    int64_t ld;
    int prec;
};
template <typename T>
struct RoundMatrix {
    typedef RoundMatrixArgs Args;
    static constexpr int NTH = 256, WPE = 0;
    static __device__ void run(const RoundMatrixArgs& a, int bx, int by);
};
template <typename T>
__device__ void RoundMatrix<T>::run(const RoundMatrixArgs& a, int bx, int)
{
    const int64_t rows = a.rows, cols = a.cols, ld = a.ld;
    const int prec = a.prec;
    T* M = (T*)a.M;
    const int64_t idx = (int64_t)bx * 256 + threadIdx.x;
    if (idx >= rows * cols) return;
    const int64_t i = idx % rows, j = idx / rows;
    float v = (float)M[i + j * ld];
    if (prec == PNE_PREC_BF16) v = __uint_as_float((uint32_t)f32_to_bf16_bits(v) << 16);
    else if (prec == PNE_PREC_FP16) v = (float)__builtin_bit_cast(_Float16, f32_to_f16_bits(v));
    M[i + j * ld] = (T)v;
}

// R = upper triangle of W(0:n, 0:n) promoted to FP64 (rounded to BF16/FP16
// first for those precisions).
struct ExtractRArgs {
    int64_t n;
    const void* W;
    int64_t ldw;
    int prec;
    double* R;
    int64_t ldr;
};
template <typename T>
struct ExtractR {
    typedef ExtractRArgs Args;
    static constexpr int NTH = 256, WPE = 0;
    static __device__ void run(const ExtractRArgs& a, int bx, int by);
};
template <typename T>
__device__ void ExtractR<T>::run(const ExtractRArgs& a, int bx, int)
{
    const int64_t n = a.n, ldw = a.ldw, ldr = a.ldr;
    const int prec = a.prec;
    const T* __restrict__ W = (const T*)a.W;
    double* __restrict__ R = a.R;
    const int64_t idx = (int64_t)bx * 256 + threadIdx.x;
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
struct RDiagCheck {
    struct Args {
        int64_t n;
        const double* R;
        int64_t ldr;
        int32_t* info;
    };
    static constexpr int NTH = 1024, WPE = 0;
    static __device__ void run(const Args& a, int bx, int by);
};
__device__ void RDiagCheck::run(const Args& a, int, int)
{
    const int64_t n = a.n, ldr = a.ldr;
    const double* __restrict__ R = a.R;
    int32_t* __restrict__ info = a.info;
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

// Panel width per factorization: 16, except FP64 sketches taller than 2048
// rows, which use 8 (register budget of the panel kernel).
template <typename T>
static int qr_nb(int64_t s)
{
    if (s > 6144) return 0;
    return (sizeof(T) == 8 && s > 2048) ? 8 : 16;
}

bool qr_supported(int64_t s, int prec)
{
    return prec == PNE_PREC_FP64 ? qr_nb<double>(s) > 0 : qr_nb<float>(s) > 0;
}

// upper bound of plan_splitk(h, tiles) over all panels (h <= s)
static int64_t qr_max_splits(int64_t s) { return (s / 128 > 1 ? s / 128 : 1) + 1; }

template <typename T>
static size_t qr_bytes(int64_t s, int64_t n)
{
    const int nb = qr_nb<T>(s) ? qr_nb<T>(s) : 8;
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

template <typename T, int NB, int RPT, int NT, bool U>
static void panel_launch(Exec& ex, int64_t h, int w, T* Wp, int64_t ldw, T* V, int64_t ldv, T* Tm)
{
    launch<QrPanel<T, NB, RPT, NT, U>>(ex, 1, 1, QrPanelArgs{h, w, Wp, ldw, V, ldv, Tm});
}

// Panel shapes (rows per thread, threads, unrolled column loop): the
// smallest instantiation covering the panel height; unrolled only where the
// compiled kernel is free of register spills.
template <typename T, int NB>
static void panel_dispatch(Exec& ex, int64_t h, int w, T* Wp, int64_t ldw, T* V, int64_t ldv, T* Tm)
{
    if constexpr (sizeof(T) == 4) {
        if (h <= 1024) panel_launch<T, NB, 1, 1024, true>(ex, h, w, Wp, ldw, V, ldv, Tm);
        else if (h <= 2048) panel_launch<T, NB, 2, 1024, true>(ex, h, w, Wp, ldw, V, ldv, Tm);
        else if (h <= 2304) panel_launch<T, NB, 3, 768, true>(ex, h, w, Wp, ldw, V, ldv, Tm);
        else if (h <= 3072) panel_launch<T, NB, 6, 512, false>(ex, h, w, Wp, ldw, V, ldv, Tm);
        else if (h <= 4096) panel_launch<T, NB, 8, 512, false>(ex, h, w, Wp, ldw, V, ldv, Tm);
        else panel_launch<T, NB, 12, 512, false>(ex, h, w, Wp, ldw, V, ldv, Tm);
    } else if constexpr (NB == 16) {
        if (h <= 1024) panel_launch<T, NB, 1, 1024, true>(ex, h, w, Wp, ldw, V, ldv, Tm);
        else panel_launch<T, NB, 4, 512, false>(ex, h, w, Wp, ldw, V, ldv, Tm);
    } else {
        if (h <= 2048) panel_launch<T, NB, 4, 512, true>(ex, h, w, Wp, ldw, V, ldv, Tm);
        else if (h <= 3072) panel_launch<T, NB, 6, 512, false>(ex, h, w, Wp, ldw, V, ldv, Tm);
        else if (h <= 4096) panel_launch<T, NB, 8, 512, false>(ex, h, w, Wp, ldw, V, ldv, Tm);
        else panel_launch<T, NB, 12, 512, false>(ex, h, w, Wp, ldw, V, ldv, Tm);
    }
}

template <typename T>
static int qr_run(Exec& ex, int64_t s, int64_t n, T* W, int64_t ldw, int prec, double* R, int64_t ldr,
                  int32_t* info, void* work, size_t work_bytes)
{
    if (work_bytes < qr_bytes<T>(s, n)) return PNE_EWORKSPACE;
    const int NBv = qr_nb<T>(s);
    if (!NBv) return PNE_ENOTSUP;
    const int64_t splits_max = qr_max_splits(s);
    Arena ar(work, work_bytes);
    T* V = ar.take<T>((size_t)s * NBv);
    T* Tm = ar.take<T>((size_t)NBv * NBv);
    T* P = ar.take<T>((size_t)splits_max * n * NBv);
    T* Z = ar.take<T>((size_t)NBv * n);
    ex.stage(ST_QR_ROUND);
    if constexpr (sizeof(T) == 4) {
        if (prec == PNE_PREC_BF16 || prec == PNE_PREC_FP16)
            launch<RoundMatrix<T>>(ex, ceil_div(s * n, 256), 1, RoundMatrixArgs{s, n, W, ldw, prec});
    }
    ex.stage(ST_QR);
    for (int64_t c0 = 0; c0 < n; c0 += NBv) {
        ex.iter((uint32_t)(c0 / NBv));
        const int w = (int)((n - c0 < NBv) ? n - c0 : NBv);
        const int64_t h = s - c0;
        T* Wp = W + c0 + c0 * ldw;
        if (NBv == 16) panel_dispatch<T, 16>(ex, h, w, Wp, ldw, V, s, Tm);
        else panel_dispatch<T, 8>(ex, h, w, Wp, ldw, V, s, Tm);
        const int64_t rem = n - c0 - w;
        if (rem <= 0) break;
        T* Wt = W + c0 + (c0 + w) * ldw;
        // P[z] = (W_trail^T V) over row chunks  (rem x w); at most
        // qr_max_splits(s) chunks (the partial buffer is sized for that)
        GemmArgs g{};
        g.M = rem; g.N = w; g.K = h;
        g.A = Wt; g.lda = ldw; g.transA = 1;
        g.B = V; g.ldb = s; g.transB = 0;
        int64_t splits, kc;
        plan_splitk(h, ceil_div(rem, 128), &splits, &kc, ex.kchunk_fixed ? 512 : 0);
        g.splits = splits; g.kchunk = kc;
        g.P = P;
        if constexpr (sizeof(T) == 8) gemm_f64_partials(ex, g);
        else gemm_f32_partials(ex, g);
        const QrTzArgs ta{rem, w, P, splits, Tm, Z};
        if (NBv == 16) launch<QrTz<T, 16>>(ex, ceil_div(rem, 16), 1, ta);
        else launch<QrTz<T, 8>>(ex, ceil_div(rem, 16), 1, ta);
        // W_trail -= V Z
        GemmArgs u{};
        u.M = h; u.N = rem; u.K = w;
        u.A = V; u.lda = s; u.transA = 0;
        u.B = Z; u.ldb = NBv; u.transB = 0;
        u.alpha = -1.0; u.beta = 1.0;
        u.Cin = Wt; u.ldcin = ldw; u.C = Wt; u.ldc = ldw;
        u.splits = 1;
        if constexpr (sizeof(T) == 8) gemm_f64(ex, u);
        else gemm_f32(ex, u);
    }
    ex.stage(ST_QR_EXTRACT);
    launch<ExtractR<T>>(ex, ceil_div(n * n, 256), 1, ExtractRArgs{n, W, ldw, prec, R, ldr});
    launch<RDiagCheck>(ex, 1, 1, RDiagCheck::Args{n, R, ldr, info});
    return launch_status(ex);
}

int qr_r(Exec& ex, int64_t s, int64_t n, void* W, int64_t ldw, int prec, double* R, int64_t ldr,
         int32_t* info, void* work, size_t work_bytes)
{
    if (prec == PNE_PREC_FP64) return qr_run<double>(ex, s, n, (double*)W, ldw, prec, R, ldr, info, work, work_bytes);
    return qr_run<float>(ex, s, n, (float*)W, ldw, prec, R, ldr, info, work, work_bytes);
}

}  // namespace pne
