// Householder QR of the s x n sketch A_s keeping only R_s (Algorithm 1,
// "Thin QR factorization A_s = Q_s R_s"; Section 6.2), then the promotion of
// R_s to FP64 (Algorithm 1, "Promote R_s").
//
// Blocked compact-WY form (Golub & Van Loan, Section 5.2.3):
//   panel:  one work-group (512 or 1024 threads) holds the h x NB panel in
//           registers (thread t owns rows t, t+NT, ...) and applies NB reflectors
//           in the LAPACK convention (beta = -sign(alpha) ||x||); each
//           column needs a single batched reduction, which delivers the norm,
//           the dot products v^T P(:, j) of the update and the V^T v column of
//           the triangular factor T (H_1..H_NB = I - V T V^T);
//   update: Y = V^T W_trail, Z = T^T Y, W_trail -= V Z in one kernel (a
//           wavefront per trailing column).
// Working precision: FP64 for qr_prec = FP64, FP32 otherwise.  For BF16 and
// FP16 the input is rounded to the format before the factorization and R_s
// after it (FP32 arithmetic in between); FP16 input is first scaled by a
// power of two that keeps R_s inside the FP16 range (QrScale).
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
    const T s = wave_transpose_total<T, NB>(v);
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
    T rowk[2][NB];     // row k of the panel, published by its owner (two steps alternate)
    T G[NB][NB + 1];   // G[k][l] = V(:, l)^T v_k for l < k
    T tauv[NB];
    T Ts[NB][NB + 1];
    T cf[NB];          // (owner-computed variant) tau v^T P(:, c) for c > k
    T gv[NB];          // (owner-computed variant) V(:, i)^T v for i < k
    T sc[2];           // (owner-computed variant) 1 / (alpha - beta), tau
};

// Which column-step variant a panel shape uses: the redundant one (two
// barriers per column) where it compiles free of register spills, the
// owner-computed one (three barriers, T built column by column) elsewhere.
template <typename T, int KS>
constexpr bool panel_redundant() { return KS >= 0 && sizeof(T) == 4; }

// One column step of the panel (see QrPanel).  KS >= 0 makes the column
// index a compile-time constant (KS == k); KS < 0 takes k at run time.  The
// owner of row k publishes the row before the reduction, so that every
// thread forms beta, tau and the update coefficients itself after it: two
// barriers per column.  The triangular factor T is assembled after the last
// column from the stored V^T v_k and tau_k.
template <typename T, int NB, int RPT, int NT, int KS>
__device__ __forceinline__ void panel_step_redundant(int k_rt, int w, T (&x)[RPT][NB], PanelShared<T, NB, NT>& sh)
{
    const int k = KS >= 0 ? KS : k_rt;
    const int tid = threadIdx.x;
    T* rk = sh.rowk[k & 1];
    if (tid == k) {
#pragma unroll
        for (int c = 0; c < NB; ++c) rk[c] = x[0][c];
    }
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
    // every thread: beta = -sign(alpha) sqrt(alpha^2 + sigma),
    // tau = (beta - alpha) / beta, v = [1; x(r>k, k) / (alpha - beta)]
    const T alpha = rk[k], sigma = sh.bc[k];
    T beta, tau, inv;
    if (sigma == (T)0) {
        beta = alpha; tau = 0; inv = 0;
    } else {
        const T nrm = sqrt(alpha * alpha + sigma);
        beta = (alpha >= (T)0) ? -nrm : nrm;
        tau = (beta - alpha) / beta;
        inv = (T)1 / (alpha - beta);
    }
    T cf[NB];   // tau v^T P(:, c) for the columns c > k
#pragma unroll
    for (int c = 0; c < NB; ++c) cf[c] = (c > k && c < w) ? tau * (rk[c] + sh.bc[c] * inv) : (T)0;
    if (tid == k) {
#pragma unroll
        for (int c = 0; c < NB; ++c) {
            if (c < k) sh.G[k][c] = rk[c] + sh.bc[c] * inv;
            if (c == k) x[0][c] = beta;
        }
        sh.tauv[k] = tau;
    }
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
            if (c > k && c < w) x[q][c] -= cf[c] * vr;
        }
    }
}

// Owner-computed variant: the thread owning row k forms beta, tau and the
// coefficients and publishes them (three barriers per column); T is built
// column by column.
template <typename T, int NB, int RPT, int NT, int KS>
__device__ __forceinline__ void panel_step_owner(int k_rt, int w, T (&x)[RPT][NB], PanelShared<T, NB, NT>& sh)
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

template <typename T, int NB, int RPT, int NT, int KS>
__device__ __forceinline__ void panel_step(int k_rt, int w, T (&x)[RPT][NB], PanelShared<T, NB, NT>& sh)
{
    if constexpr (panel_redundant<T, KS>()) panel_step_redundant<T, NB, RPT, NT, KS>(k_rt, w, x, sh);
    else panel_step_owner<T, NB, RPT, NT, KS>(k_rt, w, x, sh);
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
    void* V;          // h x NB reflectors, column-major, ld ldv
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
    constexpr bool RED = panel_redundant<T, UNROLL ? 0 : -1>();
    if constexpr (!RED)
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
    // T(i, k) = -tau_k sum_{l = i..k-1} T(i, l) (V^T v_k)_l for i < k,
    // T(k, k) = tau_k: thread i builds row i (it only reads its own row)
    if (RED && tid < NB) {
        const int i = tid;
        T trow[NB];
#pragma unroll
        for (int kk = 0; kk < NB; ++kk) {
            T v = 0;
            if (kk < w) {
                if (kk == i) {
                    v = sh.tauv[kk];
                } else if (i < kk) {
                    T acc = 0;
#pragma unroll
                    for (int l = 0; l < kk; ++l)
                        if (l >= i) acc += trow[l] * sh.G[kk][l];
                    v = -sh.tauv[kk] * acc;
                }
            }
            trow[kk] = v;
        }
#pragma unroll
        for (int kk = 0; kk < NB; ++kk) sh.Ts[i][kk] = trow[kk];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        const int64_t r = tid + NT * q;
        if (r >= h) continue;
#pragma unroll
        for (int c = 0; c < NB; ++c) {
            const T val = x[q][c];
            if (c < w) W[r + c * ldw] = (r <= c) ? val : (T)0;
            // columns of V past w are zero
            V[r + c * ldv] = (c >= w) ? (T)0 : ((r > c) ? val : (r == c ? (T)1 : (T)0));
        }
    }
    for (int e = tid; e < NB * NB; e += NT) Tout[(e % NB) + (e / NB) * NB] = sh.Ts[e % NB][e / NB];
}

// Trailing update of one panel, W_trail := (I - V T V^T)^T W_trail =
// W_trail - V (T^T (V^T W_trail)), fused in one kernel.  A work-group owns
// QU_COLS trailing columns, QU_CPW per wavefront (each V load serves QU_CPW
// columns); QU_RS wavefronts share each group of columns, lane g of split s
// walking the rows 64 s + g, 64 s + g + 64 QU_RS, ...:
//   Y(:, j) = V^T W(:, j)      NB partial dot products per lane, a
//                              transpose-reduce over the wavefront, then the
//                              QU_RS partials in a fixed order;
//   Z(:, j) = T^T Y(:, j)      from LDS;
//   W(:, j) -= V Z(:, j)       every row again.
// The row loops are unrolled so that the loads of several rows are in flight
// together.  Sums run in a fixed order (bitwise reproducible).
constexpr int QU_WAVES = 8, QU_RS = 2, QU_CPW = 4, QU_COLS = QU_WAVES / QU_RS * QU_CPW;
struct QrUpdateArgs {
    int64_t h, rem;
    void* W;          // trailing matrix, h x rem, column-major
    int64_t ldw;
    const void* V;    // h x NB, column-major, ld ldv
    int64_t ldv;
    const void* Tm;   // NB x NB upper triangular, column-major
};

// Sum of v[0..NB) over the 64 lanes: the result for entry e lands in the
// lanes with (lane >> (6 - LOGNB)) & (NB - 1) == e and is written to out[e].
template <typename T, int NB>
__device__ __forceinline__ void wave_transpose_sum(T (&v)[NB], T* out)
{
    constexpr int LOGNB = (NB == 16) ? 4 : 3;
    const int lane = threadIdx.x & 63;
    const T y = wave_transpose_total<T, NB>(v);
    const int idx = (lane >> (6 - LOGNB)) & (NB - 1);
    if ((lane & ((64 >> LOGNB) - 1)) == 0) out[idx] = y;
}

template <typename T, int NB>
struct QrUpdate {
    typedef QrUpdateArgs Args;
    static constexpr int NTH = 64 * QU_WAVES, WPE = 0;
    static __device__ void run(const QrUpdateArgs& a, int bx, int)
    {
        __shared__ T Ts[NB * NB];
        __shared__ T yp[QU_WAVES][QU_CPW][NB];
        __shared__ T zs[QU_COLS][NB];
        const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
        const int cg = wv / QU_RS, rs = wv % QU_RS;
        for (int e = threadIdx.x; e < NB * NB; e += NTH) Ts[e] = ((const T*)a.Tm)[e];
        const int64_t j0 = (int64_t)bx * QU_COLS + cg * QU_CPW;
        const T* __restrict__ V = (const T*)a.V;
        T* __restrict__ W = (T*)a.W;
        const int64_t h = a.h, ldv = a.ldv, ldw = a.ldw, rem = a.rem;
        int64_t col[QU_CPW];
#pragma unroll
        for (int q = 0; q < QU_CPW; ++q) col[q] = ((j0 + q < rem) ? j0 + q : rem - 1) * ldw;
        constexpr int STRIDE = 64 * QU_RS;
        const int64_t r0 = 64 * rs + lane;
        T v[QU_CPW][NB];
#pragma unroll
        for (int q = 0; q < QU_CPW; ++q)
#pragma unroll
            for (int c = 0; c < NB; ++c) v[q][c] = 0;
#pragma unroll 2
        for (int64_t r = r0; r < h; r += STRIDE) {
            T vr[NB], wr[QU_CPW];
#pragma unroll
            for (int c = 0; c < NB; ++c) vr[c] = V[r + c * ldv];
#pragma unroll
            for (int q = 0; q < QU_CPW; ++q) wr[q] = W[r + col[q]];
#pragma unroll
            for (int q = 0; q < QU_CPW; ++q)
#pragma unroll
                for (int c = 0; c < NB; ++c) v[q][c] += vr[c] * wr[q];
        }
#pragma unroll
        for (int q = 0; q < QU_CPW; ++q) wave_transpose_sum<T, NB>(v[q], yp[wv][q]);
        __syncthreads();
        for (int t = threadIdx.x; t < QU_COLS * NB; t += NTH) {
            const int cj = t / NB, i = t % NB;
            const int g = cj / QU_CPW, q = cj % QU_CPW;
            T z = 0;
            for (int l = 0; l <= i; ++l) {
                T y = 0;
#pragma unroll
                for (int p = 0; p < QU_RS; ++p) y += yp[g * QU_RS + p][q][l];
                z += Ts[l + i * NB] * y;
            }
            zs[cj][i] = z;
        }
        __syncthreads();
        T z[QU_CPW][NB];
#pragma unroll
        for (int q = 0; q < QU_CPW; ++q)
#pragma unroll
            for (int c = 0; c < NB; ++c) z[q][c] = zs[cg * QU_CPW + q][c];
#pragma unroll 2
        for (int64_t r = r0; r < h; r += STRIDE) {
            T vr[NB], wr[QU_CPW];
#pragma unroll
            for (int c = 0; c < NB; ++c) vr[c] = V[r + c * ldv];
#pragma unroll
            for (int q = 0; q < QU_CPW; ++q) wr[q] = W[r + col[q]];
#pragma unroll
            for (int q = 0; q < QU_CPW; ++q) {
                T s = 0;
#pragma unroll
                for (int c = 0; c < NB; ++c) s += vr[c] * z[q][c];
                if (j0 + q < rem) W[r + col[q]] = wr[q] - s;
            }
        }
    }
};

// The same update split over row chunks of QS_ROWS rows, for tall panels:
//   QrYPart:  P[chunk](:, j) = V(chunk)^T W(chunk, j)   (work-group = chunk x
//             QS_COLS columns, QS_CPW columns per wavefront, QS_ROWS / 64 rows
//             per lane with all loads issued together);
//   QrApply:  Y(:, j) = sum over chunks of P (fixed order), Z = T^T Y, then
//             W(chunk, j) -= V(chunk) Z(:, j) on the same tiling.
// Each lane touches a few rows only, so the latency of a pass is a few
// memory round trips instead of one per row.
constexpr int QS_ROWS = 256, QS_CPW = 4, QS_WAVES = 4, QS_COLS = QS_CPW * QS_WAVES;
constexpr int QS_RPL = QS_ROWS / 64;   // rows per lane
constexpr int64_t QS_SPLIT_MIN = 1024; // panels taller than this use the split update
struct QrSplitArgs {
    int64_t h, rem;
    void* W;          // trailing matrix, h x rem, column-major
    int64_t ldw;
    const void* V;    // h x NB, column-major, ld ldv
    int64_t ldv;
    const void* Tm;   // NB x NB upper triangular, column-major
    void* P;          // chunk partials: P[(chunk * rem + j) * NB + c]
};

template <typename T, int NB>
struct QrYPart {
    typedef QrSplitArgs Args;
    static constexpr int NTH = 64 * QS_WAVES, WPE = 0;
    static __device__ void run(const QrSplitArgs& a, int bx, int by)
    {
        __shared__ T ys[QS_WAVES][QS_CPW][NB];
        const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
        const int64_t rc = bx, j0 = (int64_t)by * QS_COLS + wv * QS_CPW;
        const T* __restrict__ V = (const T*)a.V;
        const T* __restrict__ W = (const T*)a.W;
        const int64_t h = a.h, ldv = a.ldv, ldw = a.ldw, rem = a.rem;
        T vr[QS_RPL][NB], wr[QS_RPL][QS_CPW];
#pragma unroll
        for (int k = 0; k < QS_RPL; ++k) {
            const int64_t r = rc * QS_ROWS + 64 * k + lane;
            const bool in = r < h;
#pragma unroll
            for (int c = 0; c < NB; ++c) vr[k][c] = in ? V[r + c * ldv] : (T)0;
#pragma unroll
            for (int q = 0; q < QS_CPW; ++q) wr[k][q] = (in && j0 + q < rem) ? W[r + (j0 + q) * ldw] : (T)0;
        }
#pragma unroll
        for (int q = 0; q < QS_CPW; ++q) {
            T v[NB];
#pragma unroll
            for (int c = 0; c < NB; ++c) {
                T t = 0;
#pragma unroll
                for (int k = 0; k < QS_RPL; ++k) t += vr[k][c] * wr[k][q];
                v[c] = t;
            }
            wave_transpose_sum<T, NB>(v, ys[wv][q]);
        }
        __syncthreads();
        T* __restrict__ P = (T*)a.P;
        for (int t = threadIdx.x; t < QS_COLS * NB; t += NTH) {
            const int cj = t / NB, c = t % NB;
            const int64_t j = (int64_t)by * QS_COLS + cj;
            if (j < rem) P[(rc * rem + j) * NB + c] = ys[cj / QS_CPW][cj % QS_CPW][c];
        }
    }
};

template <typename T, int NB>
struct QrApply {
    typedef QrSplitArgs Args;
    static constexpr int NTH = 64 * QS_WAVES, WPE = 0;
    static __device__ void run(const QrSplitArgs& a, int bx, int by)
    {
        __shared__ T Ts[NB * NB];
        __shared__ T ysum[QS_COLS][NB];
        __shared__ T zs[QS_COLS][NB];
        const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
        const int64_t rc = bx, h = a.h, rem = a.rem, ldv = a.ldv, ldw = a.ldw;
        const int64_t nchunk = (h + QS_ROWS - 1) / QS_ROWS;
        const T* __restrict__ P = (const T*)a.P;
        for (int e = threadIdx.x; e < NB * NB; e += NTH) Ts[e] = ((const T*)a.Tm)[e];
        for (int t = threadIdx.x; t < QS_COLS * NB; t += NTH) {
            const int cj = t / NB, c = t % NB;
            const int64_t j = (int64_t)by * QS_COLS + cj;
            T y = 0;
            if (j < rem) {
                // loads of 8 chunks issued together, added in chunk order
                int64_t k = 0;
                for (; k + 8 <= nchunk; k += 8) {
                    T pv[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) pv[u] = P[((k + u) * rem + j) * NB + c];
#pragma unroll
                    for (int u = 0; u < 8; ++u) y += pv[u];
                }
                for (; k < nchunk; ++k) y += P[(k * rem + j) * NB + c];
            }
            ysum[cj][c] = y;
        }
        __syncthreads();
        for (int t = threadIdx.x; t < QS_COLS * NB; t += NTH) {
            const int cj = t / NB, i = t % NB;
            T z = 0;
            for (int l = 0; l <= i; ++l) z += Ts[l + i * NB] * ysum[cj][l];
            zs[cj][i] = z;
        }
        __syncthreads();
        const int64_t j0 = (int64_t)by * QS_COLS + wv * QS_CPW;
        const T* __restrict__ V = (const T*)a.V;
        T* __restrict__ W = (T*)a.W;
        T vr[QS_RPL][NB], wr[QS_RPL][QS_CPW];
#pragma unroll
        for (int k = 0; k < QS_RPL; ++k) {
            const int64_t r = rc * QS_ROWS + 64 * k + lane;
            const bool in = r < h;
#pragma unroll
            for (int c = 0; c < NB; ++c) vr[k][c] = in ? V[r + c * ldv] : (T)0;
#pragma unroll
            for (int q = 0; q < QS_CPW; ++q) wr[k][q] = (in && j0 + q < rem) ? W[r + (j0 + q) * ldw] : (T)0;
        }
#pragma unroll
        for (int q = 0; q < QS_CPW; ++q) {
            if (j0 + q >= rem) continue;
            T z[NB];
#pragma unroll
            for (int c = 0; c < NB; ++c) z[c] = zs[wv * QS_CPW + q][c];
#pragma unroll
            for (int k = 0; k < QS_RPL; ++k) {
                const int64_t r = rc * QS_ROWS + 64 * k + lane;
                if (r >= h) continue;
                T sacc = 0;
#pragma unroll
                for (int c = 0; c < NB; ++c) sacc += vr[k][c] * z[c];
                W[r + (j0 + q) * ldw] = wr[k][q] - sacc;
            }
        }
    }
};

// FP16 QR input scale (single work-group): c = 2^(k - E) with amax =
// max |W| = f 2^E (f in [1/2, 1)) and k = 14 - t, 4^t the smallest power of
// four >= s.  Then |c W| < 2^k <= 2^14 / sqrt(s), every column of c W has
// 2-norm below 2^14, and so has every entry of its triangular factor: the
// FP16 range (largest finite 65504) holds R_s whatever the scale of A.  The
// factor is exact (a power of two) and is divided out of R_s again in FP64.
// amax = 0 or non-finite gives c = 1.
struct QrScaleArgs {
    int64_t rows, cols;
    const float* W;
    int64_t ld;
    float* scale;
};
struct QrScale {
    typedef QrScaleArgs Args;
    static constexpr int NTH = 1024, WPE = 0;
    static __device__ void run(const QrScaleArgs& a, int, int)
    {
        __shared__ float red[16];
        float mx = 0.0f;
        bool bad = false;
        for (int64_t j = 0; j < a.cols; ++j)
            for (int64_t i = threadIdx.x; i < a.rows; i += NTH) {
                const float v = fabsf(a.W[i + j * a.ld]);
                if (!(v <= 3.4e38f)) bad = true;   // inf or NaN
                else mx = fmaxf(mx, v);
            }
        bad = __syncthreads_or(bad);
        mx = wave_max(mx);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
        __syncthreads();
        if (threadIdx.x == 0) {
            float m = 0.0f;
            for (int w = 0; w < 16; ++w) m = fmaxf(m, red[w]);
            int t = 0;
            while (t < 31 && ((int64_t)1 << (2 * t)) < a.rows) ++t;
            float c = 1.0f;
            if (!bad && m > 0.0f) {
                int E;
                frexpf(m, &E);
                c = ldexpf(1.0f, (14 - t) - E);
            }
            a.scale[0] = c;
        }
    }
};

struct RoundMatrixArgs {
    int64_t rows, cols;
    void* M;
    int64_t ld;
    int prec;
    const float* scale;   // FP16: the QrScale factor applied before rounding
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
    else if (prec == PNE_PREC_FP16) v = (float)__builtin_bit_cast(_Float16, f32_to_f16_bits(v * a.scale[0]));
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
    const float* scale;   // FP16: divided out after the rounding (exact)
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
            v = (double)f;
            if (prec == PNE_PREC_FP16)
                v = (double)(float)__builtin_bit_cast(_Float16, f32_to_f16_bits(f)) / (double)a.scale[0];
        }
    }
    R[i + j * ldr] = v;
}

// First zero or non-finite diagonal entry of R -> *info = 1000 + k + 1 (if no
// earlier failure).
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
        if ((R[k + k * ldr] == 0.0 || !isfinite(R[k + k * ldr])) && k < mine) mine = k;
    mine = -wave_max(-mine);
    if ((threadIdx.x & 63) == 0) wmin[threadIdx.x >> 6] = mine;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t f = n;
        for (int i = 0; i < 16; ++i) f = wmin[i] < f ? wmin[i] : f;
        if (f < n && *info == 0) *info = 1000 + (int32_t)f + 1;
    }
}

// Widest panel of a factorization: 16, except FP64 sketches taller than 2048
// rows, which use 8 throughout (register budget of the panel kernel).
template <typename T>
static int qr_nb(int64_t s)
{
    if (s > 6144) return 0;
    return (sizeof(T) == 8 && s > 2048) ? 8 : 16;
}

// Width of the panel at height h: FP32 panels taller than 2304 rows use 8
// columns (the 16-column panel kernel would spill registers there).
template <typename T>
static int panel_nb(int64_t s, int64_t h)
{
    const int nb = qr_nb<T>(s);
    return (sizeof(T) == 4 && h > 2304) ? 8 : nb;
}

bool qr_supported(int64_t s, int prec)
{
    return prec == PNE_PREC_FP64 ? qr_nb<double>(s) > 0 : qr_nb<float>(s) > 0;
}

template <typename T>
static size_t qr_bytes(int64_t s, int64_t n)
{
    const int nb = qr_nb<T>(s) ? qr_nb<T>(s) : 8;
    Arena ar(nullptr, 0);
    ar.take<T>((size_t)s * nb);          // V
    ar.take<T>((size_t)nb * nb);         // T
    ar.take<T>((size_t)ceil_div(s, QS_ROWS) * n * nb);   // chunk partials of V^T W
    ar.take<float>(4);                                    // FP16 input scale
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
// compiled kernel is free of register spills (FP32: 16-column panels up to
// 2304 rows, 8-column panels above).
template <typename T, int NB>
static void panel_dispatch(Exec& ex, int64_t h, int w, T* Wp, int64_t ldw, T* V, int64_t ldv, T* Tm)
{
    if constexpr (sizeof(T) == 4 && NB == 8) {
        if (h <= 3072) panel_launch<T, NB, 4, 768, true>(ex, h, w, Wp, ldw, V, ldv, Tm);
        else if (h <= 4096) panel_launch<T, NB, 8, 512, true>(ex, h, w, Wp, ldw, V, ldv, Tm);
        else panel_launch<T, NB, 12, 512, false>(ex, h, w, Wp, ldw, V, ldv, Tm);
    } else if constexpr (sizeof(T) == 4) {
        if (h <= 1024) panel_launch<T, NB, 1, 1024, true>(ex, h, w, Wp, ldw, V, ldv, Tm);
        else if (h <= 2048) panel_launch<T, NB, 2, 1024, true>(ex, h, w, Wp, ldw, V, ldv, Tm);
        else panel_launch<T, NB, 3, 768, true>(ex, h, w, Wp, ldw, V, ldv, Tm);
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
    if (!NBv) return PNE_ENOTSUP;   // V holds up to NBv columns
    Arena ar(work, work_bytes);
    T* V = ar.take<T>((size_t)s * NBv);
    T* Tm = ar.take<T>((size_t)NBv * NBv);
    T* Pq = ar.take<T>((size_t)ceil_div(s, QS_ROWS) * n * NBv);
    float* qscale = ar.take<float>(4);
    ex.stage(ST_QR_ROUND);
    if constexpr (sizeof(T) == 4) {
        if (prec == PNE_PREC_FP16) launch<QrScale>(ex, 1, 1, QrScaleArgs{s, n, (const float*)W, ldw, qscale});
        if (prec == PNE_PREC_BF16 || prec == PNE_PREC_FP16)
            launch<RoundMatrix<T>>(ex, ceil_div(s * n, 256), 1, RoundMatrixArgs{s, n, W, ldw, prec, qscale});
    }
    ex.stage(ST_QR);
    int64_t c0 = 0;
    while (c0 < n) {
        ex.iter((uint32_t)c0);
        const int64_t h = s - c0;
        const int nb = panel_nb<T>(s, h);
        const int w = (int)((n - c0 < nb) ? n - c0 : nb);
        T* Wp = W + c0 + c0 * ldw;
        if (nb == 16) panel_dispatch<T, 16>(ex, h, w, Wp, ldw, V, s, Tm);
        else panel_dispatch<T, 8>(ex, h, w, Wp, ldw, V, s, Tm);
        const int64_t rem = n - c0 - w;
        if (rem > 0) {
            T* Wt = W + c0 + (c0 + w) * ldw;
            if (h > QS_SPLIT_MIN) {
                // tall: two passes over row chunks
                const QrSplitArgs u{h, rem, Wt, ldw, V, s, Tm, Pq};
                const int64_t gx = ceil_div(h, QS_ROWS), gy = ceil_div(rem, QS_COLS);
                if (nb == 16) {
                    launch<QrYPart<T, 16>>(ex, gx, gy, u);
                    launch<QrApply<T, 16>>(ex, gx, gy, u);
                } else {
                    launch<QrYPart<T, 8>>(ex, gx, gy, u);
                    launch<QrApply<T, 8>>(ex, gx, gy, u);
                }
            } else {
                const QrUpdateArgs u{h, rem, Wt, ldw, V, s, Tm};
                if (nb == 16) launch<QrUpdate<T, 16>>(ex, ceil_div(rem, QU_COLS), 1, u);
                else launch<QrUpdate<T, 8>>(ex, ceil_div(rem, QU_COLS), 1, u);
            }
        }
        c0 += w;
    }
    ex.stage(ST_QR_EXTRACT);
    launch<ExtractR<T>>(ex, ceil_div(n * n, 256), 1, ExtractRArgs{n, W, ldw, prec, R, ldr, qscale});
    launch<RDiagCheck>(ex, 1, 1, RDiagCheck::Args{n, R, ldr, info});
    return launch_status(ex);
}

void check_r_diag(Exec& ex, int64_t n, const double* R, int64_t ldr, int32_t* info)
{
    launch<RDiagCheck>(ex, 1, 1, RDiagCheck::Args{n, R, ldr, info});
}

int qr_r(Exec& ex, int64_t s, int64_t n, void* W, int64_t ldw, int prec, double* R, int64_t ldr,
         int32_t* info, void* work, size_t work_bytes)
{
    if (prec == PNE_PREC_FP64) return qr_run<double>(ex, s, n, (double*)W, ldw, prec, R, ldr, info, work, work_bytes);
    return qr_run<float>(ex, s, n, (float*)W, ldw, prec, R, ldr, info, work, work_bytes);
}

}  // namespace pne
