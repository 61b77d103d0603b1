// Sketch A_s = Omega A (Algorithm 1, "Sketch"; Section 6.2), Omega an
// s x m Gaussian matrix with N(0, 1/s) entries drawn from the counter-based
// generator in philox.h.
//
// Pipeline per chunk of rows of A (bounded workspace for any m):
//   1. omega_gen: Omega(:, chunk) written once in the operand format, row
//      major (each sketch row contiguous over the chunk, zero padded to a
//      multiple of 64 columns).  VALU bound; every entry is drawn once.
//   2. quantize:  A(chunk, :) converted to the operand format, column major
//      (k contiguous), with per-(block, column) scales for FP16/FP8.
//   3. gemm_lp:   partial A_s += Omega_q A_q on MFMA 16x16 tiles with FP32
//      accumulation, split over K (rows of A) into fixed partial buffers.
// A final reduction sums the partials in a fixed order (bitwise
// reproducible) and applies 1/sqrt(s).
//
// Operand rounding (identical in the CPU reference): FP64 inputs go to FP32
// first, then RNE to BF16/FP16/E4M3.  FP16 uses power-of-two scales
// 2^(floor(log2 amax) - 14) per block of A, FP8 uses amax / 448 (FP32).
#include "common.h"
#include "convert.h"
#include "kernels.h"
#include "launch.h"
#include "philox.h"
#include "profile.h"

namespace pne {

template <int OP>
struct Op;
template <>
struct Op<OPK_F32> {
    typedef float T;
    static constexpr int KI = 4;   // K per MFMA
    static constexpr int EPL = 1;  // operand elements per lane
};
template <>
struct Op<OPK_BF16> {
    typedef uint16_t T;
    static constexpr int KI = 32;
    static constexpr int EPL = 8;
};
template <>
struct Op<OPK_F16> {
    typedef uint16_t T;
    static constexpr int KI = 32;
    static constexpr int EPL = 8;
};
template <>
struct Op<OPK_FP8> {
    typedef uint8_t T;
    static constexpr int KI = 32;
    static constexpr int EPL = 8;
};
template <>
struct Op<OPK_F64> {
    typedef double T;
    static constexpr int KI = 4;
    static constexpr int EPL = 1;
};

template <int OP>
__device__ __forceinline__ typename Op<OP>::T to_op(float x)
{
    if constexpr (OP == OPK_F32) return x;
    else if constexpr (OP == OPK_BF16) return f32_to_bf16_bits(x);
    else if constexpr (OP == OPK_F16) return f32_to_f16_bits(x);
    else if constexpr (OP == OPK_FP8) return f32_to_e4m3_bits(x);
    else return (double)x;
}

// ---------------------------------------------------------------- 1. Omega
// out[i * ldk + k] = Omega(i, k0 + k) in the operand format, i < s, k < kc;
// zero for kc <= k < ldk.
constexpr int OMEGA_QUADS = 8;   // row quads per thread
struct OmegaArgs {
    uint64_t seed;
    uint32_t pid;
    int64_t s, k0, kc, ldk;
    void* out;
};
template <int OP>
struct OmegaGen {
    typedef OmegaArgs Args;
    static constexpr int NTH = 256, WPE = 0;
    static __device__ void run(const OmegaArgs& a, int bx, int by);
};
template <int OP>
__device__ void OmegaGen<OP>::run(const OmegaArgs& a, int bx, int by)
{
    typedef typename Op<OP>::T T;
    const uint64_t seed = a.seed;
    const uint32_t pid = a.pid;
    const int64_t s = a.s, k0 = a.k0, kc = a.kc, ldk = a.ldk;
    T* __restrict__ out = (T*)a.out;
    const int64_t k = (int64_t)bx * 256 + threadIdx.x;
    if (k >= ldk) return;
    // OMEGA_QUADS quads of rows (4 rows each) per thread, same column k
    for (int qq = 0; qq < OMEGA_QUADS; ++qq) {
        const int64_t q = (int64_t)by * OMEGA_QUADS + qq;
        if (4 * q >= s) break;
        T v[4];
        if (k < kc) {
            Gauss4 g = omega_quad(seed, pid, (uint32_t)q, (uint32_t)(k0 + k));
#pragma unroll
            for (int t = 0; t < 4; ++t) v[t] = to_op<OP>(g.z[t]);
        } else {
#pragma unroll
            for (int t = 0; t < 4; ++t) v[t] = (T)0;
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int64_t i = 4 * q + t;
            if (i < s) out[i * ldk + k] = v[t];
        }
    }
}

// ---------------------------------------------------------------- 2. quantize A
constexpr int QUANT_PER = 4;     // rows per thread (unscaled formats)
// Unscaled formats: Aq[j * ldk + k] = op(A(k0 + k, j)); zero padding.
struct QuantArgs {
    const double* A;
    int64_t lda, k0, kc, ldk, br, n;
    void* Aq;
    float* sc;
};
template <int OP>
struct QuantizePlain {
    typedef QuantArgs Args;
    static constexpr int NTH = 256, WPE = 0;
    static __device__ void run(const QuantArgs& a, int bx, int by);
};
template <int OP>
__device__ void QuantizePlain<OP>::run(const QuantArgs& a, int bx, int by)
{
    typedef typename Op<OP>::T T;
    const double* __restrict__ A = a.A;
    const int64_t lda = a.lda, k0 = a.k0, kc = a.kc, ldk = a.ldk;
    T* __restrict__ Aq = (T*)a.Aq;
    const int64_t j = by;
    // QUANT_PER consecutive rows per thread: two 16-byte loads and one
    // 8-byte store when the column is aligned and the rows are all in range
    const int64_t kb = ((int64_t)bx * 256 + threadIdx.x) * QUANT_PER;
    if (kb >= ldk) return;
    const double* src = A + (k0 + kb) + j * lda;
    if (sizeof(T) == 2 && kb + QUANT_PER <= kc && (((uintptr_t)src) & 15) == 0) {
        const double2 v0 = *(const double2*)src, v1 = *(const double2*)(src + 2);
        const uint32_t q0 = (uint32_t)to_op<OP>((float)v0.x) | ((uint32_t)to_op<OP>((float)v0.y) << 16);
        const uint32_t q1 = (uint32_t)to_op<OP>((float)v1.x) | ((uint32_t)to_op<OP>((float)v1.y) << 16);
        *(uint2*)(Aq + j * ldk + kb) = make_uint2(q0, q1);
        return;
    }
#pragma unroll
    for (int t = 0; t < QUANT_PER; ++t) {
        const int64_t k = kb + t;
        if (k >= ldk) break;
        const float v = (k < kc) ? (float)A[(k0 + k) + j * lda] : 0.0f;
        Aq[j * ldk + k] = to_op<OP>(v);
    }
}

template <int OP>
struct QuantizeScaled {
    typedef QuantArgs Args;
    static constexpr int NTH = 256, WPE = 0;
    static __device__ void run(const QuantArgs& a, int bx, int by);
};
template <int OP>
__device__ void QuantizeScaled<OP>::run(const QuantArgs& a, int bx, int by)
{
    const double* __restrict__ A = a.A;
    const int64_t lda = a.lda, k0 = a.k0, kc = a.kc, ldk = a.ldk, br = a.br, n = a.n;
    typename Op<OP>::T* __restrict__ Aq = (typename Op<OP>::T*)a.Aq;
    float* __restrict__ sc = a.sc;
    __shared__ float red[4];
    const int64_t kb = bx, j = by;
    const int64_t r0 = kb * br;
    float amax = 0.0f;
    for (int64_t r = r0 + threadIdx.x; r < r0 + br && r < kc; r += 256)
        amax = fmaxf(amax, fabsf((float)A[(k0 + r) + j * lda]));
    amax = wave_max(amax);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = amax;
    __syncthreads();
    amax = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
    float scale;
    if (amax == 0.0f) {
        scale = 0.0f;
    } else if constexpr (OP == OPK_F16) {
        int E;
        frexpf(amax, &E);                   // amax = f 2^E, f in [0.5, 1)
        scale = ldexpf(1.0f, (E - 1) - 14);
    } else {
        scale = amax / 448.0f;
    }
    if (threadIdx.x == 0) sc[kb * n + j] = scale;
    for (int64_t r = r0 + threadIdx.x; r < r0 + br && r < ldk; r += 256) {
        float t = 0.0f;
        if (r < kc && scale != 0.0f) t = (float)A[(k0 + r) + j * lda] / scale;
        Aq[j * ldk + r] = to_op<OP>(t);
    }
}

// ---------------------------------------------------------------- 3. MFMA product
// P[i + j*M] (+)= sum_{k in split} Om[i*ldk + k] * Aq[j*ldk + k]  (per scale
// block multiplied by sc[kb*N + j] when SCALED).  128 x 128 output tile per
// work-group, 4 waves of 64 x 64, MFMA 16x16.  The MFMA A operand is the A
// side (columns j) and the B operand the Omega side (rows i), so lane l holds
// output rows i = l % 16 (contiguous in the column-major result).
constexpr int LP_BM = 128, LP_BN = 128, LP_BK = 64;

template <int OP>
__device__ __forceinline__ v4f mfma16(const typename Op<OP>::T* a, const typename Op<OP>::T* b,
                                      v4f c)
{
    if constexpr (OP == OPK_F32) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(*a, *b, c, 0, 0, 0);
    } else if constexpr (OP == OPK_BF16) {
        v8bf av = *(const v8bf*)a, bv = *(const v8bf*)b;
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, c, 0, 0, 0);
    } else if constexpr (OP == OPK_F16) {
        v8h av = *(const v8h*)a, bv = *(const v8h*)b;
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(av, bv, c, 0, 0, 0);
    } else {
        long av = *(const long*)a, bv = *(const long*)b;
        return __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(av, bv, c, 0, 0, 0);
    }
}

struct GemmLpArgs {
    const void* Om;
    const void* Aq;
    int64_t ldk, M, N;
    const float* sc;
    int64_t br;
    float* P;
    int64_t kchunk;
    int accumulate;
};
template <int OP, bool SCALED>
struct GemmLp {
    typedef GemmLpArgs Args;
    static constexpr int NTH = 256, WPE = 0;
    static __device__ void run(const GemmLpArgs& a, int bx, int by);
};
template <int OP, bool SCALED>
__device__ void GemmLp<OP, SCALED>::run(const GemmLpArgs& a, int bx, int by)
{
    typedef typename Op<OP>::T T;
    const T* __restrict__ Om = (const T*)a.Om;
    const T* __restrict__ Aq = (const T*)a.Aq;
    const int64_t ldk = a.ldk, M = a.M, N = a.N, br = a.br, kchunk = a.kchunk;
    const float* __restrict__ sc = a.sc;
    float* __restrict__ P = a.P;
    const int accumulate = a.accumulate;
    constexpr int E = sizeof(T);
    constexpr int PADE = 16 / E;                 // 16 bytes of padding per LDS row
    constexpr int LDR = LP_BK + PADE;            // LDS row length in elements
    constexpr int VPR = LP_BK * E / 16;          // 16-byte vectors per tile row
    constexpr int VPT = LP_BM * VPR / 256;       // vectors per thread per tile
    __shared__ __attribute__((aligned(16))) T As[LP_BM * LDR];
    __shared__ __attribute__((aligned(16))) T Bs[LP_BN * LDR];

    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wm = w & 1, wn = w >> 1;
    const int64_t tiles_m = (M + LP_BM - 1) / LP_BM;
    const int64_t i0 = (int64_t)(bx % tiles_m) * LP_BM;
    const int64_t j0 = (int64_t)(bx / tiles_m) * LP_BN;
    const int64_t kbeg = (int64_t)by * kchunk;
    const int64_t kend = (kbeg + kchunk < ldk) ? kbeg + kchunk : ldk;

    v4f acc[4][4], tmp[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            acc[a][b] = (v4f){0.f, 0.f, 0.f, 0.f};
            tmp[a][b] = (v4f){0.f, 0.f, 0.f, 0.f};
        }

    uint4 ra[VPT], rb[VPT];
    auto gload = [&](int64_t k) {
#pragma unroll
        for (int q = 0; q < VPT; ++q) {
            const int v = tid + 256 * q;
            const int row = v / VPR, c = v % VPR;
            const int64_t gi = i0 + row, gj = j0 + row;
            const int64_t koff = k + (int64_t)c * (16 / E);
            ra[q] = (gi < M) ? *(const uint4*)(Om + gi * ldk + koff) : make_uint4(0, 0, 0, 0);
            rb[q] = (gj < N) ? *(const uint4*)(Aq + gj * ldk + koff) : make_uint4(0, 0, 0, 0);
        }
    };
    auto sstore = [&]() {
#pragma unroll
        for (int q = 0; q < VPT; ++q) {
            const int v = tid + 256 * q;
            const int row = v / VPR, c = v % VPR;
            *(uint4*)(As + row * LDR + c * (16 / E)) = ra[q];
            *(uint4*)(Bs + row * LDR + c * (16 / E)) = rb[q];
        }
    };

    const int r16 = lane & 15, g4 = lane >> 4;
    int steps_in_block = 0;
    const int steps_per_block = SCALED ? (int)(br / LP_BK) : 1 << 30;
    if (kbeg < kend) gload(kbeg);
    for (int64_t k = kbeg; k < kend; k += LP_BK) {
        __syncthreads();
        sstore();
        __syncthreads();
        if (k + LP_BK < kend) gload(k + LP_BK);
#pragma unroll
        for (int kk = 0; kk < LP_BK; kk += Op<OP>::KI) {
            const int ko = kk + g4 * Op<OP>::EPL;
            const T* pa[4];
            const T* pb[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                pb[t] = As + (wm * 64 + t * 16 + r16) * LDR + ko;   // Omega rows i
                pa[t] = Bs + (wn * 64 + t * 16 + r16) * LDR + ko;   // A columns j
            }
#pragma unroll
            for (int ti = 0; ti < 4; ++ti)
#pragma unroll
                for (int tj = 0; tj < 4; ++tj) {
                    if constexpr (SCALED) tmp[ti][tj] = mfma16<OP>(pa[tj], pb[ti], tmp[ti][tj]);
                    else acc[ti][tj] = mfma16<OP>(pa[tj], pb[ti], acc[ti][tj]);
                }
        }
        if constexpr (SCALED) {
            if (++steps_in_block == steps_per_block || k + LP_BK >= kend) {
                const int64_t kb = k / br;
#pragma unroll
                for (int tj = 0; tj < 4; ++tj)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int64_t j = j0 + wn * 64 + tj * 16 + 4 * g4 + r;
                        const float s = (j < N) ? sc[kb * N + j] : 0.0f;
#pragma unroll
                        for (int ti = 0; ti < 4; ++ti) {
                            acc[ti][tj][r] += tmp[ti][tj][r] * s;
                            tmp[ti][tj][r] = 0.0f;
                        }
                    }
                steps_in_block = 0;
            }
        }
    }
    float* Pp = P + (int64_t)by * M * N;
#pragma unroll
    for (int ti = 0; ti < 4; ++ti) {
        const int64_t i = i0 + wm * 64 + ti * 16 + r16;
        if (i >= M) continue;
#pragma unroll
        for (int tj = 0; tj < 4; ++tj)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t j = j0 + wn * 64 + tj * 16 + 4 * g4 + r;
                if (j < N) {
                    float v = acc[ti][tj][r];
                    if (accumulate) v += Pp[i + j * M];
                    Pp[i + j * M] = v;
                }
            }
    }
}

// Wide variant for one large unscaled sketch (BF16 or FP32 operands):
// 256 x 256 output tile per work-group of eight waves (2 x 4 waves of
// 128 x 64), K tiles of 128 bytes per row, two LDS buffers (one barrier per
// K tile) and the next tile held in registers.  Twice the MFMA work of the
// 128 x 128 tile per byte brought in from L2.
constexpr int LW_BM = 256, LW_BN = 256;
template <int OP>
struct GemmLpW {
    typedef GemmLpArgs Args;
    static constexpr int NTH = 512, WPE = 2;
    static __device__ void run(const GemmLpArgs& a, int bx, int by);
};
template <int OP>
__device__ void GemmLpW<OP>::run(const GemmLpArgs& a, int bx, int by)
{
    typedef typename Op<OP>::T T;
    const T* __restrict__ Om = (const T*)a.Om;
    const T* __restrict__ Aq = (const T*)a.Aq;
    const int64_t ldk = a.ldk, M = a.M, N = a.N, kchunk = a.kchunk;
    float* __restrict__ P = a.P;
    const int accumulate = a.accumulate;
    constexpr int E = sizeof(T);
    constexpr int BK = 128 / E;                  // K tile: 128 bytes per row
    constexpr int PADE = 16 / E;
    constexpr int LDR = BK + PADE;
    constexpr int VPR = 8;                       // 16-byte vectors per tile row
    constexpr int VPT = LW_BM * VPR / 512;       // vectors per thread per operand
    __shared__ __attribute__((aligned(16))) T As[2][LW_BM * LDR];
    __shared__ __attribute__((aligned(16))) T Bs[2][LW_BN * LDR];

    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wm = w & 1, wn = w >> 1;
    const int64_t tiles_m = (M + LW_BM - 1) / LW_BM;
    const int64_t i0 = (int64_t)(bx % tiles_m) * LW_BM;
    const int64_t j0 = (int64_t)(bx / tiles_m) * LW_BN;
    const int64_t kbeg = (int64_t)by * kchunk;
    const int64_t kend = (kbeg + kchunk < ldk) ? kbeg + kchunk : ldk;

    v4f acc[8][4];
#pragma unroll
    for (int x = 0; x < 8; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) acc[x][y] = (v4f){0.f, 0.f, 0.f, 0.f};

    uint4 ra[VPT], rb[VPT];
    auto gload = [&](int64_t k) {
#pragma unroll
        for (int q = 0; q < VPT; ++q) {
            const int v = tid + 512 * q;
            const int row = v / VPR, c = v % VPR;
            const int64_t gi = i0 + row, gj = j0 + row;
            const int64_t koff = k + (int64_t)c * (16 / E);
            ra[q] = (gi < M) ? *(const uint4*)(Om + gi * ldk + koff) : make_uint4(0, 0, 0, 0);
            rb[q] = (gj < N) ? *(const uint4*)(Aq + gj * ldk + koff) : make_uint4(0, 0, 0, 0);
        }
    };
    auto sstore = [&](int buf) {
#pragma unroll
        for (int q = 0; q < VPT; ++q) {
            const int v = tid + 512 * q;
            const int row = v / VPR, c = v % VPR;
            *(uint4*)(As[buf] + row * LDR + c * (16 / E)) = ra[q];
            *(uint4*)(Bs[buf] + row * LDR + c * (16 / E)) = rb[q];
        }
    };

    const int r16 = lane & 15, g4 = lane >> 4;
    int buf = 0;
    if (kbeg < kend) {
        gload(kbeg);
        sstore(0);
        if (kbeg + BK < kend) gload(kbeg + BK);
    }
    for (int64_t k = kbeg; k < kend; k += BK) {
        __syncthreads();
        const T* as = As[buf];
        const T* bs = Bs[buf];
#pragma unroll
        for (int kk = 0; kk < BK; kk += Op<OP>::KI) {
            const int ko = kk + g4 * Op<OP>::EPL;
            const T* pa[4];
            const T* pb[8];
#pragma unroll
            for (int t = 0; t < 8; ++t) pb[t] = as + (wm * 128 + t * 16 + r16) * LDR + ko;   // Omega rows i
#pragma unroll
            for (int t = 0; t < 4; ++t) pa[t] = bs + (wn * 64 + t * 16 + r16) * LDR + ko;    // A columns j
#pragma unroll
            for (int ti = 0; ti < 8; ++ti)
#pragma unroll
                for (int tj = 0; tj < 4; ++tj) acc[ti][tj] = mfma16<OP>(pa[tj], pb[ti], acc[ti][tj]);
        }
        if (k + BK < kend) {
            sstore(buf ^ 1);
            if (k + 2 * BK < kend) gload(k + 2 * BK);
        }
        buf ^= 1;
    }
    float* Pp = P + (int64_t)by * M * N;
#pragma unroll
    for (int ti = 0; ti < 8; ++ti) {
        const int64_t i = i0 + wm * 128 + ti * 16 + r16;
        if (i >= M) continue;
#pragma unroll
        for (int tj = 0; tj < 4; ++tj)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t j = j0 + wn * 64 + tj * 16 + 4 * g4 + r;
                if (j < N) {
                    float v = acc[ti][tj][r];
                    if (accumulate) v += Pp[i + j * M];
                    Pp[i + j * M] = v;
                }
            }
    }
}

// ---------------------------------------------------------------- 4. reduction
// As = scale * sum_split P[split]  (fixed order), written as FP32 and/or FP64.
struct SketchReduceArgs {
    const void* P;
    int64_t splits, M, N;
    double scale;
    float* o32;
    int64_t ld32;
    double* o64;
    int64_t ld64;
};
template <typename TP>
struct SketchReduce {
    typedef SketchReduceArgs Args;
    static constexpr int NTH = 256, WPE = 0;
    static __device__ void run(const SketchReduceArgs& a, int bx, int by);
};
template <typename TP>
__device__ void SketchReduce<TP>::run(const SketchReduceArgs& a, int bx, int)
{
    const TP* __restrict__ P = (const TP*)a.P;
    const int64_t splits = a.splits, M = a.M, N = a.N, ld32 = a.ld32, ld64 = a.ld64;
    const double scale = a.scale;
    float* __restrict__ o32 = a.o32;
    double* __restrict__ o64 = a.o64;
    const int64_t idx = (int64_t)bx * 256 + threadIdx.x;
    if (idx >= M * N) return;
    const int64_t i = idx % M, j = idx / M;
    TP s = 0;
    for (int64_t p = 0; p < splits; ++p) s += P[p * M * N + idx];
    if (o32) o32[i + j * ld32] = (float)(s * (TP)scale);
    if (o64) o64[i + j * ld64] = (double)s * scale;
}

// ---------------------------------------------------------------- host driver
size_t sketch_workspace_bytes(int64_t m, int64_t n, int64_t s, int prec, int64_t br, int64_t kchunk_fixed)
{
    SketchPlan p = plan_sketch(m, n, s, prec, br, kchunk_fixed);
    return p.bytes;
}

SketchPlan plan_sketch(int64_t m, int64_t n, int64_t s, int prec, int64_t br, int64_t kchunk_fixed)
{
    SketchPlan p{};
    const int op = prec_to_opk(prec);
    const int64_t E = opk_bytes(op);
    // rows of A per chunk: keep Omega_q of one chunk below ~1 GiB
    int64_t max_chunk = ((int64_t)1 << 30) / (E * (s > 0 ? s : 1));
    int64_t align = (op == OPK_FP8 || op == OPK_F16) ? (br > 64 ? br : 64) : 64;
    max_chunk = (max_chunk / align) * align;
    if (max_chunk < align) max_chunk = align;
    int64_t mpad = ceil_div(m, align) * align;
    p.chunk = mpad < max_chunk ? mpad : max_chunk;
    p.nchunks = ceil_div(m, p.chunk);
    p.ldk = p.chunk;  // multiple of 64
    if (kchunk_fixed > 0) {
        // batches: K chunks of a fixed length (a multiple of the alignment)
        int64_t kc = ceil_div(kchunk_fixed, align) * align;
        if (kc > p.ldk) kc = p.ldk;
        p.kchunk = kc;
        p.splits = ceil_div(p.ldk, kc);
    } else if (op == OPK_BF16 || op == OPK_F32) {
        // one wide-tile work-group per CU: the largest split count whose
        // work-groups fit one wave of the machine
        p.wide = 1;
        const int64_t tiles = ceil_div(s, LW_BM) * ceil_div(n, LW_BN);
        int64_t want = 256 / tiles;
        int64_t maxsplit = p.ldk / (4 * align);
        if (maxsplit < 1) maxsplit = 1;
        p.splits = want < 1 ? 1 : (want < maxsplit ? want : maxsplit);
        p.kchunk = ceil_div(ceil_div(p.ldk, p.splits), align) * align;
        p.splits = ceil_div(p.ldk, p.kchunk);
    } else {
        // split-K so that tiles x splits fills the machine
        int64_t tiles = ceil_div(s, LP_BM) * ceil_div(n, LP_BN);
        if (op == OPK_F64) tiles = ceil_div(s, 128) * ceil_div(n, 128);
        int64_t want = ceil_div(1024, tiles);
        int64_t maxsplit = p.ldk / (4 * align);
        if (maxsplit < 1) maxsplit = 1;
        p.splits = want < maxsplit ? want : maxsplit;
        if (p.splits < 1) p.splits = 1;
        p.kchunk = ceil_div(ceil_div(p.ldk, p.splits), align) * align;
        p.splits = ceil_div(p.ldk, p.kchunk);
    }
    p.op = op;
    Arena ar(nullptr, 0);
    ar.take<char>((size_t)s * p.ldk * E);                           // Omega_q
    if (op != OPK_F64) ar.take<char>((size_t)n * p.ldk * E);        // A_q
    if (op == OPK_FP8 || op == OPK_F16) ar.take<float>((size_t)ceil_div(p.ldk, br) * n);
    ar.take<char>((size_t)p.splits * s * n * (op == OPK_F64 ? 8 : 4));  // partials
    p.bytes = ar.used;
    return p;
}

// Generation of Omega (arithmetic-bound) and conversion of A (memory-bound)
// in one launch, their work-groups interleaved in proportion to their
// counts so that the two run side by side: work-group b is Omega work-group
// floor(b * G_o / G) when that index steps at b, otherwise conversion
// work-group b - floor(b * G_o / G).
struct SketchPrepArgs {
    OmegaArgs o;
    QuantArgs q;
    int64_t ogx, ogn, qgx, total;
};
template <int OP>
struct SketchPrep {
    typedef SketchPrepArgs Args;
    static constexpr int NTH = 256, WPE = 0;
    static __device__ void run(const SketchPrepArgs& a, int bx, int)
    {
        const int64_t b = bx;
        const int64_t oi = b * a.ogn / a.total, oi1 = (b + 1) * a.ogn / a.total;
        if (oi1 > oi) {
            OmegaGen<OP>::run(a.o, (int)(oi % a.ogx), (int)(oi / a.ogx));
        } else {
            const int64_t qi = b - oi;
            QuantizePlain<OP>::run(a.q, (int)(qi % a.qgx), (int)(qi / a.qgx));
        }
    }
};

template <int OP>
static void launch_chunk(Exec& ex, const SketchPlan& p, const double* A, int64_t lda, int64_t k0,
                         int64_t kc, int64_t n, int64_t s, uint64_t seed, uint32_t pid, int64_t br,
                         void* Omq, void* Aq, float* sc, void* P, int accumulate)
{
    const OmegaArgs oa{seed, pid, s, k0, kc, p.ldk, Omq};
    const int64_t ogx = ceil_div(p.ldk, 256), ogy = ceil_div(ceil_div(s, 4), OMEGA_QUADS);
    constexpr bool SC = (OP == OPK_FP8 || OP == OPK_F16);
    if constexpr (OP != OPK_F64 && !SC) {
        // Omega and the conversion of A in one launch
        const QuantArgs q{A, lda, k0, kc, p.ldk, br, n, Aq, sc};
        const int64_t qgx = ceil_div(p.ldk, 256 * QUANT_PER);
        const int64_t ogn = ogx * ogy, total = ogn + qgx * n;
        launch<SketchPrep<OP>>(ex, total, 1, SketchPrepArgs{oa, q, ogx, ogn, qgx, total});
        if (!ex.recording()) {
            prof_mark(PH_SK_OMEGA, ex.st);
            prof_mark(PH_SK_QUANT, ex.st);
        }
    } else {
        launch<OmegaGen<OP>>(ex, ogx, ogy, oa);
        if (!ex.recording()) prof_mark(PH_SK_OMEGA, ex.st);
    }
    if constexpr (OP == OPK_F64) {
        // C(s x n) = Omega_q (rows contiguous over k) * A(chunk rows)
        GemmArgs g{};
        g.M = s; g.N = n; g.K = kc;
        g.A = Omq; g.lda = p.ldk; g.transA = 1;
        g.B = A + k0; g.ldb = lda; g.transB = 0;
        g.splits = p.splits; g.kchunk = p.kchunk;
        g.P = (double*)P; g.accumulate_partials = accumulate;
        gemm_f64_partials(ex, g);
    } else {
        if constexpr (SC) {
            const QuantArgs q{A, lda, k0, kc, p.ldk, br, n, Aq, sc};
            launch<QuantizeScaled<OP>>(ex, ceil_div(p.ldk, br), n, q);
            if (!ex.recording()) prof_mark(PH_SK_QUANT, ex.st);
        }
        const GemmLpArgs ga{Omq, Aq, p.ldk, s, n, sc, br, (float*)P, p.kchunk, accumulate};
        if constexpr (!SC) {
            if (p.wide) {
                launch<GemmLpW<OP>>(ex, ceil_div(s, LW_BM) * ceil_div(n, LW_BN), p.splits, ga);
                if (!ex.recording()) prof_mark(PH_SK_GEMM, ex.st);
                return;
            }
        }
        launch<GemmLp<OP, SC>>(ex, ceil_div(s, LP_BM) * ceil_div(n, LP_BN), p.splits, ga);
    }
    if (!ex.recording()) prof_mark(PH_SK_GEMM, ex.st);
}

// A_s = Omega A in precision `prec`; writes As32 (ld32) and/or As64 (ld64).
int sketch_run(Exec& ex, int64_t m, int64_t n, const double* A, int64_t lda, int64_t s, uint64_t seed,
               uint32_t pid, int prec, int64_t br, float* As32, int64_t ld32, double* As64,
               int64_t ld64, void* work, size_t work_bytes)
{
    SketchPlan p = plan_sketch(m, n, s, prec, br, ex.kchunk_fixed);
    if (work_bytes < p.bytes) return PNE_EWORKSPACE;
    ex.stage(ST_SKETCH);
    const int64_t E = opk_bytes(p.op);
    Arena ar(work, work_bytes);
    void* Omq = ar.take<char>((size_t)s * p.ldk * E);
    void* Aq = (p.op != OPK_F64) ? (void*)ar.take<char>((size_t)n * p.ldk * E) : nullptr;
    float* sc = (p.op == OPK_FP8 || p.op == OPK_F16) ? ar.take<float>((size_t)ceil_div(p.ldk, br) * n)
                                                      : nullptr;
    void* P = ar.take<char>((size_t)p.splits * s * n * (p.op == OPK_F64 ? 8 : 4));
    for (int64_t c = 0; c < p.nchunks; ++c) {
        const int64_t k0 = c * p.chunk;
        const int64_t kc = (m - k0 < p.chunk) ? m - k0 : p.chunk;
        const int acc = c > 0;
        ex.iter((uint32_t)c);
        switch (p.op) {
        case OPK_F64: launch_chunk<OPK_F64>(ex, p, A, lda, k0, kc, n, s, seed, pid, br, Omq, Aq, sc, P, acc); break;
        case OPK_F32: launch_chunk<OPK_F32>(ex, p, A, lda, k0, kc, n, s, seed, pid, br, Omq, Aq, sc, P, acc); break;
        case OPK_BF16: launch_chunk<OPK_BF16>(ex, p, A, lda, k0, kc, n, s, seed, pid, br, Omq, Aq, sc, P, acc); break;
        case OPK_F16: launch_chunk<OPK_F16>(ex, p, A, lda, k0, kc, n, s, seed, pid, br, Omq, Aq, sc, P, acc); break;
        case OPK_FP8: launch_chunk<OPK_FP8>(ex, p, A, lda, k0, kc, n, s, seed, pid, br, Omq, Aq, sc, P, acc); break;
        }
    }
    ex.stage(ST_SKETCH_REDUCE);
    const double scale = 1.0 / sqrt((double)s);
    const SketchReduceArgs ra{P, p.splits, s, n, scale, As32, ld32, As64, ld64};
    if (p.op == OPK_F64) launch<SketchReduce<double>>(ex, ceil_div(s * n, 256), 1, ra);
    else launch<SketchReduce<float>>(ex, ceil_div(s * n, 256), 1, ra);
    if (!ex.recording()) prof_mark(PH_SK_REDUCE, ex.st);
    return launch_status(ex);
}

}  // namespace pne
