// Single-precision condition estimate and precision pick (Section 6.1,
// Algorithm 1 first step).
//   G = fl32(A)^T fl32(A)       FP32 MFMA SYRK, split over rows of A
//   ||G||_1                     max column sum of |G| (symmetric, lower stored)
//   G = L L^T                   FP32 blocked Cholesky (with the inverses of
//                               its 64 x 64 diagonal blocks); a bad pivot
//                               means the estimate "overflows" -> kappa0 = +inf
//   est ~ ||G^{-1}||_1          Hager's method (Hager 1984): x = (1/n) 1,
//                               (solves through the inverted 64 x 64
//                               diagonal blocks of L),
//                               at most five rounds of y = G^{-1} x,
//                               z = G^{-T} sign(y) (sign 0 = +1); stop when
//                               ||z||_inf <= z^T x, else x = e_j with j the
//                               first index of max |z_j|; est = ||y||_1
//   kappa0 = (1/2) log10(||G||_1 est)
//   pick: FP16 if kappa0 < 4, FP32 if kappa0 <= 8, else FP64.
// The factor n of the bound kappa(A)^2 <= n ||G||_1 ||G^{-1}||_1 is left out
// of kappa0 (with it, kappa(A) = 1e2 would select single precision for
// 400 <= n <= 2000, contrary to the half-precision pick reported in
// Section 7.4).
#include "common.h"
#include "kernels.h"
#include "launch.h"
#include "trsv_dev.h"

namespace pne {

__device__ __forceinline__ int32_t pick_precision(float k0)
{
    if (!(k0 == k0) || isinf(k0)) return PNE_PREC_FP64;
    if (k0 < 4.0f) return PNE_PREC_FP16;
    if (k0 <= 8.0f) return PNE_PREC_FP32;
    return PNE_PREC_FP64;
}

struct KnownKappa {
    struct Args {
        double known_kappa;
        float* k0;
        int32_t* choice;
    };
    static constexpr int NTH = 64, WPE = 0;
    static __device__ void run(const Args& a, int, int)
    {
        if (threadIdx.x == 0) {
            const float v = (float)log10(a.known_kappa);
            *a.k0 = v;
            *a.choice = pick_precision(v);
        }
    }
};

// ||G||_1 from the lower triangle of the symmetric G (column j sums |G(i,j)|
// for i >= j and |G(j,i)| for i < j).
struct Norm1Sym {
    struct Args {
        int64_t n;
        const float* G;
        int64_t ld;
        float* out;
    };
    static constexpr int NTH = 1024, WPE = 0;
    static __device__ void run(const Args& a, int bx, int by);
};
__device__ void Norm1Sym::run(const Args& a, int, int)
{
    const int64_t n = a.n, ld = a.ld;
    const float* __restrict__ G = a.G;
    float* __restrict__ out = a.out;
    __shared__ float red[16];
    float best = 0.0f;
    for (int64_t j = threadIdx.x; j < n; j += 1024) {
        float s = 0.0f;
        for (int64_t i = 0; i < n; ++i) s += fabsf(i >= j ? G[i + j * ld] : G[j + i * ld]);
        best = fmaxf(best, s);
    }
    best = wave_max(best);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = best;
    __syncthreads();
    if (threadIdx.x == 0) {
        float b = 0.0f;
        for (int i = 0; i < 16; ++i) b = fmaxf(b, red[i]);
        *out = b;
    }
}

struct Hager {
    struct Args {
        int64_t n;
        const float* L;
        int64_t ld;
        const float* DL;
        const float* g1;
        const int32_t* info;
        float* k0;
        int32_t* choice;
        int tri;        // 0: L is the Cholesky factor of G; 1: L holds an upper triangular R
    };
    static constexpr int NTH = 1024, WPE = 0;
    static __device__ void run(const Args& a, int bx, int by);
};
// Hager's iteration on M^{-1}: M = L L^T (tri = 0, y = L^{-T} L^{-1} x) or
// M = R (tri = 1, y = R^{-1} x and z = R^{-T} xi, one triangular solve each).
__device__ void Hager::run(const Args& a, int, int)
{
    const int64_t n = a.n, ld = a.ld;
    const float* __restrict__ L = a.L;
    const float* __restrict__ DL = a.DL;
    const float* __restrict__ g1 = a.g1;
    const int32_t* __restrict__ info = a.info;
    float* __restrict__ k0 = a.k0;
    int32_t* __restrict__ choice = a.choice;
    __shared__ float x[4096], y[4096], z[4096];
    __shared__ float redf[16];
    __shared__ float tmp[TB];
    __shared__ float redz[16], redd[16];
    __shared__ int64_t redi[16];
    __shared__ int stop;
    __shared__ int64_t jmax_sh;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    if (*info != 0) {
        if (tid == 0) { *k0 = __builtin_inff(); *choice = PNE_PREC_FP64; }
        return;
    }
    for (int64_t i = tid; i < n; i += 1024) x[i] = 1.0f / (float)n;
    __syncthreads();
    float est = 0.0f;
    for (int it = 0; it < 5; ++it) {
        for (int64_t i = tid; i < n; i += 1024) y[i] = x[i];
        __syncthreads();
        if (a.tri) {
            wg_trsv_inv<float>(n, L, ld, false, false, DL, false, y, tmp);
        } else {
            wg_trsv_inv<float>(n, L, ld, true, false, DL, false, y, tmp);
            wg_trsv_inv<float>(n, L, ld, false, true, DL, true, y, tmp);
        }
        float s = 0.0f;
        for (int64_t i = tid; i < n; i += 1024) s += fabsf(y[i]);
        s = block_sum(s, redf);
        est = s;
        for (int64_t i = tid; i < n; i += 1024) z[i] = (y[i] >= 0.0f) ? 1.0f : -1.0f;
        __syncthreads();
        if (a.tri) {
            wg_trsv_inv<float>(n, L, ld, true, true, DL, true, z, tmp);
        } else {
            wg_trsv_inv<float>(n, L, ld, true, false, DL, false, z, tmp);
            wg_trsv_inv<float>(n, L, ld, false, true, DL, true, z, tmp);
        }
        // ||z||_inf with its first index, and z^T x
        float zm = -1.0f, ztx = 0.0f;
        int64_t zi = INT64_MAX;
        for (int64_t i = tid; i < n; i += 1024) {
            const float a = fabsf(z[i]);
            if (a > zm) { zm = a; zi = i; }
            ztx += z[i] * x[i];
        }
        wave_argmax(zm, zi);
        ztx = wave_sum(ztx);
        if (lane == 0) { redz[wid] = zm; redi[wid] = zi; redd[wid] = ztx; }
        __syncthreads();
        if (tid == 0) {
            float bm = redz[0], d = 0.0f;
            int64_t bi = redi[0];
            for (int i = 1; i < 16; ++i)
                if (redz[i] > bm || (redz[i] == bm && redi[i] < bi)) { bm = redz[i]; bi = redi[i]; }
            for (int i = 0; i < 16; ++i) d += redd[i];
            stop = (bm <= d);
            jmax_sh = bi;
        }
        __syncthreads();
        if (stop) break;
        const int64_t jm = jmax_sh;
        for (int64_t i = tid; i < n; i += 1024) x[i] = (i == jm) ? 1.0f : 0.0f;
        __syncthreads();
    }
    if (tid == 0) {
        const float prod = (*g1) * est;
        float v = __builtin_inff();
        if (isfinite(prod) && prod > 0.0f) v = (a.tri ? 1.0f : 0.5f) * log10f(prod);
        *k0 = v;
        *choice = pick_precision(v);
    }
}

struct CePlan {
    int64_t splits, kchunk;
};
static CePlan ce_plan(int64_t m, int64_t n, int64_t kchunk_fixed)
{
    CePlan p;
    plan_splitk(m, gemm_tiles(n, n, m, 1), &p.splits, &p.kchunk, kchunk_fixed);
    return p;
}

size_t condest_workspace_bytes(int64_t m, int64_t n, int64_t kchunk_fixed)
{
    CePlan p = ce_plan(m, n, kchunk_fixed);
    Arena ar(nullptr, 0);
    ar.take<float>((size_t)n * n);              // G / L
    ar.take<float>((size_t)p.splits * n * n);   // SYRK partials
    ar.take<float>(4);                          // ||G||_1
    ar.take<int32_t>(4);                        // info
    ar.take<float>(dinv_elems(n));              // block inverses of L
    return ar.used;
}

int condest_run(Exec& ex, int64_t m, int64_t n, const double* A, int64_t lda, double known_kappa, float* dk0,
                int32_t* dchoice, void* work, size_t work_bytes)
{
    ex.stage(ST_CONDEST_GRAM);
    if (known_kappa > 0.0) {
        launch<KnownKappa>(ex, 1, 1, KnownKappa::Args{known_kappa, dk0, dchoice});
        return launch_status(ex);
    }
    if (work_bytes < condest_workspace_bytes(m, n, ex.kchunk_fixed)) return PNE_EWORKSPACE;
    if (n > 4096) return PNE_ENOTSUP;
    CePlan p = ce_plan(m, n, ex.kchunk_fixed);
    Arena ar(work, work_bytes);
    float* G = ar.take<float>((size_t)n * n);
    float* P = ar.take<float>((size_t)p.splits * n * n);
    float* g1 = ar.take<float>(4);
    int32_t* info = ar.take<int32_t>(4);
    float* DL = ar.take<float>(dinv_elems(n));
    zero_i32(ex, 1, info);
    GemmArgs g{};
    g.M = n; g.N = n; g.K = m;
    g.A = A; g.lda = lda; g.transA = 1;
    g.B = A; g.ldb = lda; g.transB = 0;
    g.alpha = 1.0; g.beta = 0.0;
    g.C = G; g.ldc = n;
    g.lower = 1;
    g.splits = p.splits; g.kchunk = p.kchunk; g.P = P;
    gemm_ddf(ex, g);
    launch<Norm1Sym>(ex, 1, 1, Norm1Sym::Args{n, G, n, g1});
    ex.stage(ST_CONDEST_FACTOR);
    cholesky<float>(ex, n, G, n, info, DL);
    ex.stage(ST_CONDEST_EST);
    launch<Hager>(ex, 1, 1, Hager::Args{n, G, n, DL, g1, info, dk0, dchoice, 0});
    return launch_status(ex);
}

// ---------------------------------------------------------------- estimate from an FP32 QR
// Library variant of the first step of Algorithm 1 that does not square
// kappa(A): the FP32 sketch A_s = Omega A (s x n, the solver's sketch in
// FP32), its FP32 Householder QR -> R, then
//   kappa0 = log10(||R||_1 est),  est ~ ||R^{-1}||_1 by the same Hager
//   iteration with one triangular solve per direction;
// a zero or non-finite diagonal of R means the estimate overflows (+inf ->
// FP64).  kappa(A_s) is within the condition number of the sketched
// orthonormal basis of kappa(A) (< 3.73 asymptotically for s = 3n), and an
// FP32 QR resolves kappa up to about 1/u_32, so the single-precision band
// of Algorithm 1 (kappa0 <= 8) is reachable, which the FP32 Gram estimate
// (breakdown from kappa ~ 4e3) is not.  W (s x n FP32) and R (n x n FP64)
// receive the sketch and R: they are exactly the preconditioner an FP32
// sketch and FP32 QR with the same seed compute.

// Rf = fl32(R) on and above the diagonal, 0 below; ||Rf||_1 into *out.
struct RToF32 {
    struct Args {
        int64_t n;
        const double* R;
        float* Rf;
    };
    static constexpr int NTH = 256, WPE = 0;
    static __device__ void run(const Args& a, int bx, int)
    {
        const int64_t n = a.n;
        const int64_t e = (int64_t)bx * 256 + threadIdx.x;
        if (e >= n * n) return;
        const int64_t i = e % n, j = e / n;
        a.Rf[e] = i <= j ? (float)a.R[i + j * n] : 0.0f;
    }
};
struct Norm1Upper {
    struct Args {
        int64_t n;
        const float* R;
        float* out;
    };
    static constexpr int NTH = 1024, WPE = 0;
    static __device__ void run(const Args& a, int, int)
    {
        __shared__ float red[16];
        float best = 0.0f;
        for (int64_t j = threadIdx.x; j < a.n; j += 1024) {
            float s = 0.0f;
            for (int64_t i = 0; i <= j; ++i) s += fabsf(a.R[i + j * a.n]);
            best = fmaxf(best, s);
        }
        best = wave_max(best);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = best;
        __syncthreads();
        if (threadIdx.x == 0) {
            float b = 0.0f;
            for (int i = 0; i < 16; ++i) b = fmaxf(b, red[i]);
            *a.out = b;
        }
    }
};

static size_t condest_qr_aux_bytes(int64_t n)
{
    Arena ar(nullptr, 0);
    ar.take<float>((size_t)n * n);      // fl32(R)
    ar.take<float>(dinv_elems(n));      // block inverses of R
    ar.take<float>(4);                  // ||R||_1
    ar.take<int32_t>(4);                // info of the QR
    return ar.used;
}

size_t condest_qr_workspace_bytes(int64_t m, int64_t n, int64_t s, int64_t kchunk_fixed)
{
    size_t w = sketch_workspace_bytes(m, n, s, PNE_PREC_FP32, 128, kchunk_fixed);
    const size_t q = qr_workspace_bytes(s, n, PNE_PREC_FP32);
    if (q > w) w = q;
    return condest_qr_aux_bytes(n) + w;
}

int condest_qr_run(Exec& ex, int64_t m, int64_t n, const double* A, int64_t lda, int64_t s, uint64_t seed,
                   uint32_t pid, float* dk0, int32_t* dchoice, float* W, double* R, void* work,
                   size_t work_bytes)
{
    if (n > 4096) return PNE_ENOTSUP;
    if (!qr_supported(s, PNE_PREC_FP32)) return PNE_ENOTSUP;
    if (work_bytes < condest_qr_workspace_bytes(m, n, s, ex.kchunk_fixed)) return PNE_EWORKSPACE;
    Arena ar(work, work_bytes);
    float* Rf = ar.take<float>((size_t)n * n);
    float* DR = ar.take<float>(dinv_elems(n));
    float* r1 = ar.take<float>(4);
    int32_t* info = ar.take<int32_t>(4);
    char* rest = (char*)work + ar.used;
    const size_t rest_bytes = work_bytes - ar.used;
    ex.stage(ST_CONDEST_GRAM);
    zero_i32(ex, 1, info);
    int rc = sketch_run(ex, m, n, A, lda, s, seed, pid, PNE_PREC_FP32, 128, W, s, nullptr, 0, rest, rest_bytes);
    if (rc) return rc;
    rc = qr_r(ex, s, n, W, s, PNE_PREC_FP32, R, n, info, rest, rest_bytes);
    if (rc) return rc;
    // (no new stage: the launches below keep counting within the QR's last
    // stage, so the launch keys of a batched recording stay increasing)
    launch<RToF32>(ex, ceil_div(n * n, 256), 1, RToF32::Args{n, R, Rf});
    inv_diag_blocks<float>(ex, n, Rf, n, 0, 0, 0, DR);
    launch<Norm1Upper>(ex, 1, 1, Norm1Upper::Args{n, Rf, r1});
    launch<Hager>(ex, 1, 1, Hager::Args{n, Rf, n, DR, r1, info, dk0, dchoice, 1});
    return launch_status(ex);
}

}  // namespace pne
