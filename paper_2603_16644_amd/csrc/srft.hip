// SRFT sketch A_s = (1/sqrt(s)) S H D A (Section 6.2, eq. e_sketch, Omega =
// S F D, with the real Hartley transform H = Re(F) - Im(F) as F):
//   m' = smallest 7-smooth integer >= m (A padded with zero rows),
//   D   random signs d_j (bit j mod 128 of Philox at counter (j/128, 0, pid, 3)),
//   S   s rows of I_m' sampled uniformly with replacement
//       (k_i = floor(w m' / 2^64), w from Philox at counter (i, 0, pid, 2)).
//
// Two real columns a, b of D A form one complex sequence z = a + i b whose
// DFT Z gives both Hartley columns at row k:
//   H a[k] = (Re Z[k] + Re Z[-k] - Im Z[k] + Im Z[-k]) / 2
//   H b[k] = (Im Z[k] + Im Z[-k] + Re Z[k] - Re Z[-k]) / 2.
// The DFT of length m' is a mixed-radix Stockham (self-sorting) FFT over the
// radices 2, 3, 4, 5, 7, 8, 16, 25, 32, smallest first:
//   pass with radix R after radices of product Ns: butterfly j < m'/R reads
//   x[j + r m'/R], multiplies by exp(-2 pi i (j mod Ns) r / (Ns R)), takes
//   the R-point DFT and writes y[(j / Ns) Ns R + (j mod Ns) + q Ns].
// The last pass is evaluated only at the sampled rows k and -k
// (Z[k] = sum_r x[(k mod Ns) + r Ns] exp(-2 pi i r k / m')), so the cost is
// (passes - 1) sweeps over the m' x n/2 complex array plus 2 s R terms per
// column pair: O(m n log m) arithmetic, HBM-bound, no power-of-two
// restriction on m.
//
// Layout of the work arrays: complex (re, im) of T, row-major [row][pair]
// (pair fastest), so every pass reads and writes whole rows of pairs.  The
// first pass reads A (column-major) through an LDS tile, applies D and the
// operand rounding (FP32, or BF16 via FP32; FP64 unrounded) and transposes.
// Arithmetic in T = float (FP32/BF16 operands) or double (FP64).
#include "common.h"
#include "convert.h"
#include "kernels.h"
#include "launch.h"
#include "philox.h"
#include "profile.h"

namespace pne {

namespace {

template <typename T>
struct Cx {
    T x, y;
};

template <typename T>
__device__ __forceinline__ void sincos_pi(T a, T* s, T* c)
{
    if constexpr (sizeof(T) == 4) sincospif(a, s, c);
    else sincospi(a, s, c);
}

// exp(-2 pi i t / N) for 0 <= t < N
template <typename T>
__device__ __forceinline__ Cx<T> unit_root(int64_t t, int64_t N)
{
    T s, c;
    sincos_pi<T>((T)(-2.0) * (T)((double)t / (double)N), &s, &c);
    return Cx<T>{c, s};
}

template <typename T>
__device__ __forceinline__ Cx<T> cmul(Cx<T> a, Cx<T> b)
{
    return Cx<T>{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}

__device__ __forceinline__ double srft_operand(double v, int prec)
{
    if (prec == PNE_PREC_FP64) return v;
    float f = (float)v;
    if (prec == PNE_PREC_BF16) f = __uint_as_float((uint32_t)f32_to_bf16_bits(f) << 16);
    return (double)f;
}

}  // namespace

// ---------------------------------------------------------------- signs
struct SrftSigns {
    struct Args {
        uint64_t seed;
        uint32_t pid;
        int64_t nwords;
        uint32_t* words;   // bit j % 32 of words[j / 32] set: d_j = -1
    };
    static constexpr int NTH = 256, WPE = 0;
    static __device__ void run(const Args& a, int bx, int)
    {
        const int64_t w = (int64_t)bx * 256 + threadIdx.x;
        if (w >= a.nwords) return;
        uint32_t c[4] = {(uint32_t)(w / 4), 0u, a.pid, 3u};
        philox4x32_10(c, (uint32_t)a.seed, (uint32_t)(a.seed >> 32));
        a.words[w] = c[w % 4];
    }
};

// ---------------------------------------------------------------- first pass
// Tile: SJ butterflies x SC column pairs per work-group (256 threads, one
// butterfly each); the R x SJ x SC inputs are staged in LDS, reading SJ
// consecutive rows of every column (coalesced).
constexpr int SJ = 32, SC = 8;
struct SrftFirstArgs {
    int64_t m, mp, n, lda;
    const double* A;
    int64_t col0;      // first column of A in this chunk (even)
    int64_t P;         // column pairs in this chunk
    int prec;
    const uint32_t* signs;
    void* out;
};
template <typename T, int R>
struct SrftFirst {
    typedef SrftFirstArgs Args;
    static constexpr int NTH = 256, WPE = 0;
    static __device__ void run(const Args& a, int bx, int by);
};
template <typename T, int R>
__device__ void SrftFirst<T, R>::run(const Args& a, int bx, int by)
{
    __shared__ T zr[R * SJ * SC], zi[R * SJ * SC];
    __shared__ Cx<T> wr[R];
    const int tid = threadIdx.x;
    const int64_t Tb = a.mp / R;
    const int64_t j0 = (int64_t)bx * SJ, c0 = (int64_t)by * SC;
    if (tid < R) wr[tid] = unit_root<T>(tid, R);
    // stage: element e -> (row offset jj, column cc2 of the 2 SC columns, r)
    for (int e = tid; e < R * SJ * 2 * SC; e += 256) {
        const int jj = e % SJ;
        const int rest = e / SJ;
        const int cc2 = rest % (2 * SC);
        const int r = rest / (2 * SC);
        const int64_t j = j0 + jj;
        const int64_t row = j + (int64_t)r * Tb;
        const int64_t col = a.col0 + 2 * c0 + cc2;
        T v = 0;
        if (j < Tb && row < a.m && col < a.n && (c0 + cc2 / 2) < a.P) {
            const double x = srft_operand(a.A[row + col * a.lda], a.prec);
            const bool neg = (a.signs[row >> 5] >> (row & 31)) & 1u;
            v = (T)(neg ? -x : x);
        }
        const int slot = (r * SJ + jj) * SC + cc2 / 2;
        if (cc2 & 1) zi[slot] = v;
        else zr[slot] = v;
    }
    __syncthreads();
    const int cc = tid % SC, jj = tid / SC;
    const int64_t j = j0 + jj, c = c0 + cc;
    if (j >= Tb || c >= a.P) return;
    Cx<T> v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = Cx<T>{zr[(r * SJ + jj) * SC + cc], zi[(r * SJ + jj) * SC + cc]};
    Cx<T>* out = (Cx<T>*)a.out;
    // first pass: Ns = 1, no twiddles; outputs at rows j R + q
    for (int q = 0; q < R; ++q) {
        Cx<T> acc{0, 0};
        int idx = 0;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const Cx<T> w = wr[idx];
            acc.x += v[r].x * w.x - v[r].y * w.y;
            acc.y += v[r].x * w.y + v[r].y * w.x;
            idx += q;
            if (idx >= R) idx -= R;
        }
        out[(j * R + q) * a.P + c] = acc;
    }
}

// ---------------------------------------------------------------- middle passes
struct SrftPassArgs {
    int64_t mp, P, Ns;
    const void* in;
    void* out;
};
template <typename T, int R>
struct SrftPass {
    typedef SrftPassArgs Args;
    static constexpr int NTH = 256, WPE = 0;
    static __device__ void run(const Args& a, int bx, int by);
};
template <typename T, int R>
__device__ void SrftPass<T, R>::run(const Args& a, int bx, int)
{
    __shared__ Cx<T> wr[R];
    const int tid = threadIdx.x;
    if (tid < R) wr[tid] = unit_root<T>(tid, R);
    __syncthreads();
    const int64_t Tb = a.mp / R;
    const int64_t e = (int64_t)bx * 256 + tid;
    if (e >= Tb * a.P) return;
    const int64_t c = e % a.P, j = e / a.P;
    const Cx<T>* in = (const Cx<T>*)a.in;
    Cx<T>* out = (Cx<T>*)a.out;
    const int64_t jm = j % a.Ns, N = a.Ns * R;
    Cx<T> v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const Cx<T> x = in[(j + r * Tb) * a.P + c];
        v[r] = r == 0 ? x : cmul(x, unit_root<T>(jm * r, N));
    }
    const int64_t base = (j / a.Ns) * N + jm;
    for (int q = 0; q < R; ++q) {
        Cx<T> acc{0, 0};
        int idx = 0;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const Cx<T> w = wr[idx];
            acc.x += v[r].x * w.x - v[r].y * w.y;
            acc.y += v[r].x * w.y + v[r].y * w.x;
            idx += q;
            if (idx >= R) idx -= R;
        }
        out[(base + q * a.Ns) * a.P + c] = acc;
    }
}

// ---------------------------------------------------------------- sampled last pass
struct SrftSampleArgs {
    int64_t mp, P, Ns, R, s, n;
    const void* in;
    uint64_t seed;
    uint32_t pid;
    int64_t col0;
    double scale;      // 1 / sqrt(s)
    float* As32;
    double* As64;
    int64_t ldas;
};
template <typename T>
struct SrftSample {
    typedef SrftSampleArgs Args;
    static constexpr int NTH = 256, WPE = 0;
    static __device__ void run(const Args& a, int bx, int by);
};
template <typename T>
__device__ void SrftSample<T>::run(const Args& a, int bx, int)
{
    const int64_t e = (int64_t)bx * 256 + threadIdx.x;
    if (e >= a.s * a.P) return;
    const int64_t c = e % a.P, i = e / a.P;
    uint32_t w[4] = {(uint32_t)i, 0u, a.pid, 2u};
    philox4x32_10(w, (uint32_t)a.seed, (uint32_t)(a.seed >> 32));
    const uint64_t u = (uint64_t)w[0] | ((uint64_t)w[1] << 32);
    const int64_t k = (int64_t)__umul64hi(u, (uint64_t)a.mp);
    const int64_t kn = k == 0 ? 0 : a.mp - k;
    const Cx<T>* in = (const Cx<T>*)a.in;
    Cx<T> z[2];
    const int64_t ks[2] = {k, kn};
    for (int h = 0; h < 2; ++h) {
        const int64_t kk = ks[h];
        const int64_t jr = kk % a.Ns;
        Cx<T> acc{0, 0};
        for (int64_t r = 0; r < a.R; ++r) {
            const Cx<T> x = in[(jr + r * a.Ns) * a.P + c];
            const Cx<T> t = unit_root<T>((r * kk) % a.mp, a.mp);
            acc.x += x.x * t.x - x.y * t.y;
            acc.y += x.x * t.y + x.y * t.x;
        }
        z[h] = acc;
    }
    const T ha = (T)0.5 * (z[0].x + z[1].x - z[0].y + z[1].y);
    const T hb = (T)0.5 * (z[0].y + z[1].y + z[0].x - z[1].x);
    const int64_t ca = a.col0 + 2 * c, cb = ca + 1;
    if (a.As64) {
        a.As64[i + ca * a.ldas] = (double)ha * a.scale;
        if (cb < a.n) a.As64[i + cb * a.ldas] = (double)hb * a.scale;
    } else {
        a.As32[i + ca * a.ldas] = (float)((double)ha * a.scale);
        if (cb < a.n) a.As32[i + cb * a.ldas] = (float)((double)hb * a.scale);
    }
}

// ---------------------------------------------------------------- host side
int64_t srft_padded_length(int64_t m)
{
    for (int64_t x = m < 1 ? 1 : m;; ++x) {
        int64_t y = x;
        for (int p : {2, 3, 5, 7})
            while (y % p == 0) y /= p;
        if (y == 1) return x;
    }
}

// Radices of m' (7-smooth) from {2,3,4,5,7,8,16,25,32}, ascending.
static int srft_radices(int64_t mp, int* r)
{
    int a = 0, b = 0, c = 0, d = 0, nr = 0;
    while (mp % 2 == 0) { mp /= 2; ++a; }
    while (mp % 3 == 0) { mp /= 3; ++b; }
    while (mp % 5 == 0) { mp /= 5; ++c; }
    while (mp % 7 == 0) { mp /= 7; ++d; }
    for (; a >= 5; a -= 5) r[nr++] = 32;
    if (a == 4) r[nr++] = 16;
    else if (a == 3) r[nr++] = 8;
    else if (a == 2) r[nr++] = 4;
    else if (a == 1) r[nr++] = 2;
    for (; c >= 2; c -= 2) r[nr++] = 25;
    if (c == 1) r[nr++] = 5;
    for (; b > 0; --b) r[nr++] = 3;
    for (; d > 0; --d) r[nr++] = 7;
    for (int i = 1; i < nr; ++i)
        for (int k = i; k > 0 && r[k - 1] > r[k]; --k) { int t = r[k]; r[k] = r[k - 1]; r[k - 1] = t; }
    return nr;
}

struct SrftPlan {
    int64_t mp, pairs, chunk;   // padded length, column pairs, pairs per chunk
    int nr, radix[48];
    size_t elem;                // bytes of one complex element
    size_t buf_bytes, bytes;
};

static SrftPlan srft_plan(int64_t m, int64_t n, int prec)
{
    SrftPlan p{};
    p.mp = srft_padded_length(m);
    p.nr = srft_radices(p.mp, p.radix);
    p.pairs = (n + 1) / 2;
    p.elem = prec == PNE_PREC_FP64 ? 16 : 8;
    const size_t budget = (size_t)512 << 20;
    int64_t ch = (int64_t)(budget / ((size_t)p.mp * p.elem));
    if (ch < 1) ch = 1;
    p.chunk = ch < p.pairs ? ch : p.pairs;
    p.buf_bytes = (size_t)p.mp * p.chunk * p.elem;
    Arena ar(nullptr, 0);
    ar.take<uint32_t>((size_t)ceil_div(p.mp, 32));
    ar.take<char>(p.buf_bytes);
    ar.take<char>(p.buf_bytes);
    p.bytes = ar.used;
    return p;
}

bool srft_supported(int prec) { return prec == PNE_PREC_FP64 || prec == PNE_PREC_FP32 || prec == PNE_PREC_BF16; }

size_t srft_workspace_bytes(int64_t m, int64_t n, int prec) { return srft_plan(m, n, prec).bytes; }

template <typename T, int R>
static void first_launch(Exec& ex, const SrftPlan& p, const SrftFirstArgs& a)
{
    launch<SrftFirst<T, R>>(ex, ceil_div(p.mp / R, SJ), ceil_div(a.P, SC), a);
}
template <typename T>
static int first_dispatch(Exec& ex, const SrftPlan& p, int R, const SrftFirstArgs& a)
{
    switch (R) {
    case 1: first_launch<T, 1>(ex, p, a); break;
    case 2: first_launch<T, 2>(ex, p, a); break;
    case 3: first_launch<T, 3>(ex, p, a); break;
    case 4: first_launch<T, 4>(ex, p, a); break;
    case 5: first_launch<T, 5>(ex, p, a); break;
    case 7: first_launch<T, 7>(ex, p, a); break;
    case 8: first_launch<T, 8>(ex, p, a); break;
    case 16: first_launch<T, 16>(ex, p, a); break;
    case 25: first_launch<T, 25>(ex, p, a); break;
    case 32: first_launch<T, 32>(ex, p, a); break;
    default: return PNE_ENOTSUP;
    }
    return PNE_OK;
}
template <typename T, int R>
static void pass_launch(Exec& ex, const SrftPlan& p, const SrftPassArgs& a)
{
    launch<SrftPass<T, R>>(ex, ceil_div((p.mp / R) * a.P, 256), 1, a);
}
template <typename T>
static int pass_dispatch(Exec& ex, const SrftPlan& p, int R, const SrftPassArgs& a)
{
    switch (R) {
    case 2: pass_launch<T, 2>(ex, p, a); break;
    case 3: pass_launch<T, 3>(ex, p, a); break;
    case 4: pass_launch<T, 4>(ex, p, a); break;
    case 5: pass_launch<T, 5>(ex, p, a); break;
    case 7: pass_launch<T, 7>(ex, p, a); break;
    case 8: pass_launch<T, 8>(ex, p, a); break;
    case 16: pass_launch<T, 16>(ex, p, a); break;
    case 25: pass_launch<T, 25>(ex, p, a); break;
    case 32: pass_launch<T, 32>(ex, p, a); break;
    default: return PNE_ENOTSUP;
    }
    return PNE_OK;
}

template <typename T>
static int srft_run_t(Exec& ex, const SrftPlan& p, int64_t m, int64_t n, const double* A, int64_t lda, int64_t s,
                      uint64_t seed, uint32_t pid, int prec, float* As32, int64_t ld32, double* As64,
                      int64_t ld64, void* work)
{
    Arena ar(work, p.bytes);
    uint32_t* signs = ar.take<uint32_t>((size_t)ceil_div(p.mp, 32));
    char* buf0 = ar.take<char>(p.buf_bytes);
    char* buf1 = ar.take<char>(p.buf_bytes);
    launch<SrftSigns>(ex, ceil_div(ceil_div(p.mp, 32), 256), 1,
                      SrftSigns::Args{seed, pid, ceil_div(p.mp, 32), signs});
    // radices of the full passes: all but the last (a single radix: a load
    // pass of radix 1, then the sampled pass of radix m')
    const int nfull = p.nr > 1 ? p.nr - 1 : 0;
    const int64_t Rlast = p.nr > 0 ? p.radix[p.nr - 1] : 1;
    for (int64_t pc = 0; pc < p.pairs; pc += p.chunk) {
        ex.iter((uint32_t)(1 + pc / p.chunk));   // (iteration 0 holds the signs)
        const int64_t P = (p.pairs - pc < p.chunk) ? p.pairs - pc : p.chunk;
        char* cur = buf0;
        char* nxt = buf1;
        const int R0 = nfull > 0 ? p.radix[0] : 1;
        int rc = first_dispatch<T>(ex, p, R0, SrftFirstArgs{m, p.mp, n, lda, A, 2 * pc, P, prec, signs, cur});
        if (rc) return rc;
        int64_t Ns = R0;
        for (int t = 1; t < nfull; ++t) {
            rc = pass_dispatch<T>(ex, p, p.radix[t], SrftPassArgs{p.mp, P, Ns, cur, nxt});
            if (rc) return rc;
            Ns *= p.radix[t];
            char* tmp = cur; cur = nxt; nxt = tmp;
        }
        SrftSampleArgs sa{p.mp, P, Ns, p.nr > 0 ? Rlast : 1, s, n, cur, seed, pid, 2 * pc,
                          1.0 / sqrt((double)s), As32, As64, As64 ? ld64 : ld32};
        launch<SrftSample<T>>(ex, ceil_div(s * P, 256), 1, sa);
    }
    if (!ex.recording()) prof_mark(PH_SK_GEMM, ex.st);   // the whole SRFT counts as the sketch product
    return launch_status(ex);
}

int srft_run(Exec& ex, int64_t m, int64_t n, const double* A, int64_t lda, int64_t s, uint64_t seed, uint32_t pid,
             int prec, float* As32, int64_t ld32, double* As64, int64_t ld64, void* work, size_t work_bytes)
{
    if (!srft_supported(prec)) return PNE_ENOTSUP;
    if ((As64 == nullptr) == (As32 == nullptr)) return PNE_EINVAL;
    const SrftPlan p = srft_plan(m, n, prec);
    if (work_bytes < p.bytes) return PNE_EWORKSPACE;
    ex.stage(ST_SKETCH);
    if (prec == PNE_PREC_FP64)
        return srft_run_t<double>(ex, p, m, n, A, lda, s, seed, pid, prec, As32, ld32, As64, ld64, work);
    return srft_run_t<float>(ex, p, m, n, A, lda, s, seed, pid, prec, As32, ld32, As64, ld64, work);
}

}  // namespace pne
