/*
 * pne_oracle.c -- TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT.
 *
 * A plain, slow, obviously correct CPU implementation of what the randomized
 * preconditioned normal equations compute, written from Garrison & Ipsen,
 * "Perturbation Analysis for Preconditioned Normal Equations in Mixed
 * Precision" (arXiv 2603.16644).  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark load this file; the GPU library never
 * does, and the two share no code.
 *
 * Conventions.
 *   - Every matrix is column-major with a leading dimension (LAPACK style):
 *     element (i, j) of X is X[i + j*ldx].
 *   - Arithmetic is IEEE binary64 unless a function says otherwise.  The
 *     low-precision paths are *emulated*: operands are rounded to the target
 *     format exactly as the GPU rounds them (round-to-nearest-even), products
 *     are then summed in binary64.
 *   - Loops run in the plain textbook order; there is no blocking, no
 *     reordering and no threading.
 *   - Numerical status follows the LAPACK style: 0 = success,
 *     1000+k: R_s(k,k) == 0, 2000+k: Cholesky breakdown at column k,
 *     3000+k: zero pivot in LU at column k (k is 1-based).
 *
 * Precision codes: 1 = FP64, 2 = FP32, 3 = FP16, 4 = BF16, 5 = FP8 (OCP e4m3),
 * 0 = AUTO (the condition-estimate heuristic of Algorithm 1 picks the code).
 *
 * Parity status of each function is documented next to it; the pins live in
 * tests/test_oracle_pins.py.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define PREC_AUTO 0
#define PREC_FP64 1
#define PREC_FP32 2
#define PREC_FP16 3
#define PREC_BF16 4
#define PREC_FP8 5

#define IDX(i, j, ld) ((size_t)(i) + (size_t)(j) * (size_t)(ld))

/* ------------------------------------------------------------------------
 * Counter-based random numbers: Philox4x32 with 10 rounds.
 * Definition: Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy
 * as 1, 2, 3", SC'11, Section 4 (Philox S-box = two 32x32->64 multiplies,
 * Weyl-sequence key schedule).  Pinned by the published known-answer vectors.
 * ---------------------------------------------------------------------- */
void oracle_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u; /* round multipliers */
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u; /* key increments    */
    uint32_t x0 = ctr_in[0], x1 = ctr_in[1], x2 = ctr_in[2], x3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) { k0 += W0; k1 += W1; }
        uint64_t p0 = (uint64_t)M0 * (uint64_t)x0;
        uint64_t p1 = (uint64_t)M1 * (uint64_t)x2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t y0 = hi1 ^ x1 ^ k0;
        uint32_t y1 = lo1;
        uint32_t y2 = hi0 ^ x3 ^ k1;
        uint32_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Standard normal entry (i, j) of the unscaled sketching matrix (i < s rows,
 * j < m columns) for problem `pid`.  One Philox call with
 *   key = (seed low 32 bits, seed high 32 bits), counter = (j, i/4, pid, 0)
 * yields four words w0..w3; rows 4*(i/4)+0,1 come from the Box-Muller pair
 * (w0, w1) and rows +2,+3 from (w2, w3) (Box & Muller, Ann. Math. Stat. 1958):
 *   U1 = ((w_a >> 8) + 1) 2^-24 in (0,1],  U2 = (w_b >> 8) 2^-24 in [0,1),
 *   z_even = sqrt(-2 ln U1) cos(2 pi U2),  z_odd = sqrt(-2 ln U1) sin(2 pi U2).
 * The Gaussian sketch of the method has entries N(0, 1/s); the 1/sqrt(s)
 * factor is applied to the product, not here. */
double oracle_omega_entry(uint64_t seed, uint32_t pid, int64_t i, int64_t j)
{
    uint32_t ctr[4] = {(uint32_t)j, (uint32_t)(i >> 2), pid, 0u};
    uint32_t key[2] = {(uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32)};
    uint32_t w[4];
    oracle_philox4x32_10(ctr, key, w);
    int pair = (int)((i & 3) >> 1);
    uint32_t wa = w[2 * pair], wb = w[2 * pair + 1];
    double u1 = ((double)(wa >> 8) + 1.0) * 0x1p-24;
    double u2 = (double)(wb >> 8) * 0x1p-24;
    double rad = sqrt(-2.0 * log(u1));
    double ang = 2.0 * M_PI * u2;
    return (i & 1) ? rad * sin(ang) : rad * cos(ang);
}

/* Materialise the unscaled s x m sketch (column-major, ld = s).  Test use only. */
void oracle_omega(uint64_t seed, uint32_t pid, int64_t s, int64_t m, double* Om)
{
    for (int64_t j = 0; j < m; ++j)
        for (int64_t i = 0; i < s; ++i) Om[IDX(i, j, s)] = oracle_omega_entry(seed, pid, i, j);
}

/* ------------------------------------------------------------------------
 * Rounding to narrower binary formats, round-to-nearest-even.
 * A format with p significand bits (implicit bit included), minimum normal
 * exponent emin and largest finite value maxv.  Values below 2^emin are
 * rounded on the subnormal grid 2^(emin-p+1).  Overflow gives +-inf, or +-maxv
 * when `saturate` is set.  (IEEE 754-2008 Section 4.3.1; OCP 8-bit floating
 * point specification v1.0 for E4M3: p = 4, emin = -6, max = 448, no inf.)
 * ---------------------------------------------------------------------- */
static double round_format(double x, int p, int emin, double maxv, int saturate)
{
    if (x == 0.0 || !isfinite(x)) return x;
    int E;
    frexp(x, &E);          /* |x| = f 2^E, f in [0.5, 1) */
    int e = E - 1;         /* 2^e <= |x| < 2^(e+1)       */
    if (e < emin) e = emin;
    double q = ldexp(1.0, e - (p - 1)); /* spacing of the grid around x */
    double r = rint(x / q) * q;         /* rint rounds half to even      */
    if (fabs(r) > maxv) r = saturate ? copysign(maxv, x) : copysign(INFINITY, x);
    return r;
}

double oracle_round_fp32(double x) { return (double)(float)x; }
double oracle_round_bf16(double x) { return round_format(x, 8, -126, 0x1.fep127, 0); }
double oracle_round_fp16(double x) { return round_format(x, 11, -14, 65504.0, 0); }
double oracle_round_e4m3(double x) { return round_format(x, 4, -6, 448.0, 1); }

/* The operand value an MFMA of precision `prec` sees for an FP64 input x:
 * x is first rounded to FP32 (the sketch converts A and the generated sketch
 * entries to FP32 first), then to the narrow format. */
static double to_operand(double x, int prec)
{
    switch (prec) {
    case PREC_FP64: return x;
    case PREC_FP32: return oracle_round_fp32(x);
    case PREC_BF16: return oracle_round_bf16(oracle_round_fp32(x));
    case PREC_FP16: return oracle_round_fp16(oracle_round_fp32(x));
    case PREC_FP8: return oracle_round_e4m3(oracle_round_fp32(x));
    default: return NAN;
    }
}

/* ------------------------------------------------------------------------
 * Sketch A_s = Omega A (Algorithm 1, "Sketch"; Section 6.2, randomized
 * preconditioner), Omega Gaussian with N(0,1/s) entries.
 *
 * Operand rounding per precision (the definition the GPU implements):
 *   FP64, FP32, BF16: Omega and A rounded elementwise (via FP32).
 *   FP16, FP8: A is split into blocks of `block_rows` rows; for block k and
 *     column j let amax = max |fl32(A_ij)| over the block.
 *       FP16: scale = 2^(floor(log2 amax) - 14)   (power of two, exact)
 *       FP8 : scale = fl32(amax / 448)
 *     q_ij = round(fl32(fl32(A_ij) / scale)) in the target format
 *     (saturating for e4m3); an all-zero block contributes 0.  The partial sum of a
 *     block is multiplied by its scale.  Omega is rounded unscaled.
 * Products are summed in FP64 here; the result is multiplied by 1/sqrt(s).
 * If Aabs != NULL it receives (1/sqrt(s)) sum |Omega_q||A_q| scale, the
 * magnitude that bounds the rounding error of any summation order.
 * ---------------------------------------------------------------------- */
int oracle_sketch(int64_t m, int64_t n, const double* A, int64_t lda, int64_t s, uint64_t seed,
                  uint32_t pid, int prec, int64_t block_rows, double* As, int64_t ldas, double* Aabs)
{
    if (m < 1 || n < 1 || s < 1 || lda < m || ldas < s) return -1;
    if (prec < PREC_FP64 || prec > PREC_FP8) return -1;
    if (block_rows < 1) block_rows = 128;
    int blocked = (prec == PREC_FP16 || prec == PREC_FP8);
    int64_t bs = blocked ? block_rows : m; /* rows that share one scale */
    double inv_sqrt_s = 1.0 / sqrt((double)s);
    double* om = (double*)malloc(sizeof(double) * (size_t)s);       /* one column of Omega */
    double* scale = (double*)malloc(sizeof(double) * (size_t)n);    /* per column of A     */
    double* P = (double*)malloc(sizeof(double) * (size_t)s * (size_t)n);  /* block partial */
    double* Pa = (double*)malloc(sizeof(double) * (size_t)s * (size_t)n);
    if (!om || !scale || !P || !Pa) { free(om); free(scale); free(P); free(Pa); return -2; }
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i < s; ++i) {
            As[IDX(i, j, ldas)] = 0.0;
            if (Aabs) Aabs[IDX(i, j, ldas)] = 0.0;
        }
    for (int64_t k0 = 0; k0 < m; k0 += bs) {
        int64_t k1 = (m - k0 < bs) ? m : k0 + bs;
        /* scales of this block of rows */
        for (int64_t j = 0; j < n; ++j) {
            scale[j] = 1.0;
            if (!blocked) continue;
            float amax = 0.0f;
            for (int64_t k = k0; k < k1; ++k) {
                float a = fabsf((float)A[IDX(k, j, lda)]);
                if (a > amax) amax = a;
            }
            if (amax == 0.0f) { scale[j] = 0.0; continue; } /* all-zero block */
            if (prec == PREC_FP16) {
                int E;
                frexpf(amax, &E); /* amax = f 2^E, f in [0.5, 1) */
                scale[j] = ldexp(1.0, (E - 1) - 14);
            } else {
                scale[j] = (double)(amax / 448.0f);
            }
        }
        for (size_t t = 0; t < (size_t)s * (size_t)n; ++t) { P[t] = 0.0; Pa[t] = 0.0; }
        /* A_s += Omega(:, k) A(k, :) for every row k of the block */
        for (int64_t k = k0; k < k1; ++k) {
            for (int64_t i = 0; i < s; ++i) om[i] = to_operand(oracle_omega_entry(seed, pid, i, k), prec);
            for (int64_t j = 0; j < n; ++j) {
                double a;
                if (!blocked) {
                    a = to_operand(A[IDX(k, j, lda)], prec);
                } else if (scale[j] == 0.0) {
                    a = 0.0;
                } else {
                    float t = (float)A[IDX(k, j, lda)] / (float)scale[j];
                    a = (prec == PREC_FP16) ? oracle_round_fp16((double)t) : oracle_round_e4m3((double)t);
                }
                for (int64_t i = 0; i < s; ++i) {
                    P[IDX(i, j, s)] += om[i] * a;
                    Pa[IDX(i, j, s)] += fabs(om[i] * a);
                }
            }
        }
        for (int64_t j = 0; j < n; ++j)
            for (int64_t i = 0; i < s; ++i) {
                As[IDX(i, j, ldas)] += P[IDX(i, j, s)] * scale[j];
                if (Aabs) Aabs[IDX(i, j, ldas)] += Pa[IDX(i, j, s)] * scale[j];
            }
    }
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i < s; ++i) {
            As[IDX(i, j, ldas)] *= inv_sqrt_s;
            if (Aabs) Aabs[IDX(i, j, ldas)] *= inv_sqrt_s;
        }
    free(om); free(scale); free(P); free(Pa);
    return 0;
}

/* ------------------------------------------------------------------------
 * Householder reflector in the LAPACK convention (Golub & Van Loan,
 * Section 5.1.2): for x = [alpha; x2] returns beta, tau and v = [1; v2] with
 * (I - tau v v^T) x = [beta; 0], beta = -sign(alpha) ||x||, sign(0) = +1.
 * If x2 == 0 no reflection is needed: tau = 0, beta = alpha.
 * ---------------------------------------------------------------------- */
static void householder(int64_t len, double* x, double* tau, double* beta)
{
    double alpha = x[0];
    double sig = 0.0;
    for (int64_t i = 1; i < len; ++i) sig += x[i] * x[i];
    if (sig == 0.0) { *tau = 0.0; *beta = alpha; return; }
    double nrm = sqrt(alpha * alpha + sig);
    double b = (alpha >= 0.0) ? -nrm : nrm;
    *tau = (b - alpha) / b;
    double sc = 1.0 / (alpha - b);
    for (int64_t i = 1; i < len; ++i) x[i] *= sc;
    x[0] = 1.0;
    *beta = b;
}

/* Thin Householder QR of the s x n matrix W (s >= n), keeping only R
 * (Algorithm 1, "Thin QR factorization A_s = Q_s R_s"; Q_s is never formed).
 * W is overwritten.  R (n x n, upper triangle; strict lower part set to 0). */
int oracle_householder_r(int64_t s, int64_t n, double* W, int64_t ldw, double* R, int64_t ldr)
{
    if (s < n || n < 1 || ldw < s || ldr < n) return -1;
    double* v = (double*)malloc(sizeof(double) * (size_t)s);
    if (!v) return -2;
    for (int64_t k = 0; k < n; ++k) {
        int64_t len = s - k;
        for (int64_t i = 0; i < len; ++i) v[i] = W[IDX(k + i, k, ldw)];
        double tau, beta;
        householder(len, v, &tau, &beta);
        W[IDX(k, k, ldw)] = beta;
        for (int64_t i = 1; i < len; ++i) W[IDX(k + i, k, ldw)] = 0.0;
        for (int64_t j = k + 1; j < n; ++j) {   /* W(k:, j) -= tau v (v^T W(k:, j)) */
            double d = 0.0;
            for (int64_t i = 0; i < len; ++i) d += v[i] * W[IDX(k + i, j, ldw)];
            d *= tau;
            for (int64_t i = 0; i < len; ++i) W[IDX(k + i, j, ldw)] -= d * v[i];
        }
    }
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i < n; ++i) R[IDX(i, j, ldr)] = (i <= j) ? W[IDX(i, j, ldw)] : 0.0;
    free(v);
    return 0;
}

/* Back substitution R x = y, R upper triangular n x n.  Returns 1000+k if
 * R(k,k) is zero or not finite (1-based k); x is then left as NaN. */
static int solve_upper(int64_t n, const double* R, int64_t ldr, const double* y, double* x)
{
    for (int64_t k = 0; k < n; ++k)
        if (R[IDX(k, k, ldr)] == 0.0 || !isfinite(R[IDX(k, k, ldr)])) {
            for (int64_t i = 0; i < n; ++i) x[i] = NAN;
            return 1000 + (int)k + 1;
        }
    for (int64_t i = n - 1; i >= 0; --i) {
        double acc = y[i];
        for (int64_t j = i + 1; j < n; ++j) acc -= R[IDX(i, j, ldr)] * x[j];
        x[i] = acc / R[IDX(i, i, ldr)];
    }
    return 0;
}

/* ------------------------------------------------------------------------
 * Least squares by Householder QR (the role of the direct QR solver the paper
 * compares against, Section 7.4; Golub & Van Loan Algorithm 5.3.2): reflect A
 * to upper triangular form, apply the same reflectors to b, back-substitute
 * R x = (Q^T b)(1:n).  This is the accuracy yardstick of every solve.
 * ---------------------------------------------------------------------- */
int oracle_qr_ls(int64_t m, int64_t n, const double* A, int64_t lda, const double* b, double* x)
{
    if (m < n || n < 1 || lda < m) return -1;
    double* W = (double*)malloc(sizeof(double) * (size_t)m * (size_t)n);
    double* c = (double*)malloc(sizeof(double) * (size_t)m);
    double* v = (double*)malloc(sizeof(double) * (size_t)m);
    if (!W || !c || !v) { free(W); free(c); free(v); return -2; }
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i < m; ++i) W[IDX(i, j, m)] = A[IDX(i, j, lda)];
    for (int64_t i = 0; i < m; ++i) c[i] = b[i];
    for (int64_t k = 0; k < n; ++k) {
        int64_t len = m - k;
        for (int64_t i = 0; i < len; ++i) v[i] = W[IDX(k + i, k, m)];
        double tau, beta;
        householder(len, v, &tau, &beta);
        W[IDX(k, k, m)] = beta;
        for (int64_t j = k + 1; j < n; ++j) {
            double d = 0.0;
            for (int64_t i = 0; i < len; ++i) d += v[i] * W[IDX(k + i, j, m)];
            d *= tau;
            for (int64_t i = 0; i < len; ++i) W[IDX(k + i, j, m)] -= d * v[i];
        }
        double d = 0.0;
        for (int64_t i = 0; i < len; ++i) d += v[i] * c[k + i];
        d *= tau;
        for (int64_t i = 0; i < len; ++i) c[k + i] -= d * v[i];
    }
    int info = solve_upper(n, W, m, c, x);
    free(W); free(c); free(v);
    return info;
}

/* ------------------------------------------------------------------------
 * Preconditioned matrix A_p = A R^{-1} (Algorithm 1, "Solve A_p = A R_s^{-1}",
 * in FP64 after promotion of R_s): each row a of A solves y R = a by forward
 * substitution, y_j = (a_j - sum_{k<j} y_k R_kj) / R_jj.
 * ---------------------------------------------------------------------- */
int oracle_precondition(int64_t m, int64_t n, const double* A, int64_t lda, const double* R,
                        int64_t ldr, double* Ap, int64_t ldap)
{
    for (int64_t k = 0; k < n; ++k)
        if (R[IDX(k, k, ldr)] == 0.0 || !isfinite(R[IDX(k, k, ldr)])) return 1000 + (int)k + 1;
    for (int64_t i = 0; i < m; ++i)
        for (int64_t j = 0; j < n; ++j) {
            double acc = A[IDX(i, j, lda)];
            for (int64_t k = 0; k < j; ++k) acc -= Ap[IDX(i, k, ldap)] * R[IDX(k, j, ldr)];
            Ap[IDX(i, j, ldap)] = acc / R[IDX(j, j, ldr)];
        }
    return 0;
}

/* C = X^T Y (n x n) and c = X^T b, X, Y m x n: the PNE matrix A_p^T A_p
 * (Y = X = A_p, eq. for PNE) or the HPNE matrix A_p^T A (Y = A). */
void oracle_gram(int64_t m, int64_t n, const double* X, int64_t ldx, const double* Y, int64_t ldy,
                 const double* b, double* C, int64_t ldc, double* c)
{
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i < n; ++i) {
            double acc = 0.0;
            for (int64_t k = 0; k < m; ++k) acc += X[IDX(k, i, ldx)] * Y[IDX(k, j, ldy)];
            C[IDX(i, j, ldc)] = acc;
        }
    if (b && c)
        for (int64_t i = 0; i < n; ++i) {
            double acc = 0.0;
            for (int64_t k = 0; k < m; ++k) acc += X[IDX(k, i, ldx)] * b[k];
            c[i] = acc;
        }
}

/* Cholesky C = L L^T of a symmetric positive definite n x n matrix (reads the
 * lower triangle; Golub & Van Loan Algorithm 4.2.1).  L overwrites the lower
 * triangle of C; the strict upper triangle is set to 0.  Returns 2000+k when
 * the k-th pivot (1-based) is not positive or not finite. */
int oracle_cholesky(int64_t n, double* C, int64_t ldc)
{
    for (int64_t j = 0; j < n; ++j) {
        double d = C[IDX(j, j, ldc)];
        for (int64_t k = 0; k < j; ++k) d -= C[IDX(j, k, ldc)] * C[IDX(j, k, ldc)];
        if (!(d > 0.0) || !isfinite(d)) return 2000 + (int)j + 1;
        double ljj = sqrt(d);
        C[IDX(j, j, ldc)] = ljj;
        for (int64_t i = j + 1; i < n; ++i) {
            double acc = C[IDX(i, j, ldc)];
            for (int64_t k = 0; k < j; ++k) acc -= C[IDX(i, k, ldc)] * C[IDX(j, k, ldc)];
            C[IDX(i, j, ldc)] = acc / ljj;
        }
    }
    for (int64_t j = 1; j < n; ++j)
        for (int64_t i = 0; i < j; ++i) C[IDX(i, j, ldc)] = 0.0;
    return 0;
}

/* Magnitude used by the pivot search: |x|, with NaN counted as +inf so that a
 * column holding a NaN selects a non-finite pivot (and reports a breakdown)
 * instead of silently passing over it. */
static double pivot_mag(double x) { return isnan(x) ? INFINITY : fabs(x); }

/* LU with partial pivoting P C = L U (Golub & Van Loan Algorithm 3.4.1):
 * at column k the pivot is the first row of largest absolute value in
 * C(k:n-1, k).  piv[k] = row swapped with k (0-based).  Returns 3000+k if the
 * pivot is zero or not finite (the elimination of that column is skipped). */
int oracle_lu(int64_t n, double* C, int64_t ldc, int32_t* piv)
{
    int info = 0;
    for (int64_t k = 0; k < n; ++k) {
        int64_t p = k;
        double best = pivot_mag(C[IDX(k, k, ldc)]);
        for (int64_t i = k + 1; i < n; ++i)
            if (pivot_mag(C[IDX(i, k, ldc)]) > best) { best = pivot_mag(C[IDX(i, k, ldc)]); p = i; }
        piv[k] = (int32_t)p;
        if (p != k)
            for (int64_t j = 0; j < n; ++j) {
                double t = C[IDX(k, j, ldc)];
                C[IDX(k, j, ldc)] = C[IDX(p, j, ldc)];
                C[IDX(p, j, ldc)] = t;
            }
        double pv = C[IDX(k, k, ldc)];
        if (pv == 0.0 || !isfinite(pv)) { if (!info) info = 3000 + (int)k + 1; continue; }
        for (int64_t i = k + 1; i < n; ++i) C[IDX(i, k, ldc)] /= pv;
        for (int64_t j = k + 1; j < n; ++j)
            for (int64_t i = k + 1; i < n; ++i)
                C[IDX(i, j, ldc)] -= C[IDX(i, k, ldc)] * C[IDX(k, j, ldc)];
    }
    return info;
}

/* Solve with a Cholesky factor: L z = c, L^T y = z. */
static void chol_solve(int64_t n, const double* L, int64_t ldl, const double* c, double* y)
{
    double* z = (double*)malloc(sizeof(double) * (size_t)n);
    for (int64_t i = 0; i < n; ++i) {
        double acc = c[i];
        for (int64_t k = 0; k < i; ++k) acc -= L[IDX(i, k, ldl)] * z[k];
        z[i] = acc / L[IDX(i, i, ldl)];
    }
    for (int64_t i = n - 1; i >= 0; --i) {
        double acc = z[i];
        for (int64_t k = i + 1; k < n; ++k) acc -= L[IDX(k, i, ldl)] * y[k];
        y[i] = acc / L[IDX(i, i, ldl)];
    }
    free(z);
}

/* Solve with an LU factorization: apply the row swaps to c, L z = P c (unit
 * lower), U x = z. */
static void lu_solve(int64_t n, const double* LU, int64_t ldlu, const int32_t* piv, const double* c,
                     double* x)
{
    double* z = (double*)malloc(sizeof(double) * (size_t)n);
    for (int64_t i = 0; i < n; ++i) z[i] = c[i];
    for (int64_t k = 0; k < n; ++k)
        if (piv[k] != k) { double t = z[k]; z[k] = z[piv[k]]; z[piv[k]] = t; }
    for (int64_t i = 0; i < n; ++i) {
        double acc = z[i];
        for (int64_t k = 0; k < i; ++k) acc -= LU[IDX(i, k, ldlu)] * z[k];
        z[i] = acc;
    }
    for (int64_t i = n - 1; i >= 0; --i) {
        double acc = z[i];
        for (int64_t k = i + 1; k < n; ++k) acc -= LU[IDX(i, k, ldlu)] * x[k];
        x[i] = acc / LU[IDX(i, i, ldlu)];
    }
    free(z);
}

/* ------------------------------------------------------------------------
 * Condition estimate in single precision (Section 6.1, Algorithm 1 first step).
 *   G = fl32(A)^T fl32(A) summed in FP32; FP32 Cholesky G = L L^T (any
 *   non-positive or non-finite pivot => the estimate "overflows");
 *   est ~ ||G^{-1}||_1 by Hager's method (W. W. Hager, "Condition estimates",
 *   SIAM J. Sci. Stat. Comput. 5, 1984): x = (1/n) 1; repeat at most five
 *   times: y = G^{-1} x, xi = sign(y) (sign 0 = +1), z = G^{-T} xi; stop if
 *   ||z||_inf <= z^T x, else x = e_j with j the first index of max |z_j|;
 *   the estimate is ||y||_1 of the last y.
 *   kappa0 = (1/2) log10(||G||_1 est)   (the factor n of the 1-norm bound
 *   kappa(A)^2 <= n ||G||_1 ||G^{-1}||_1 is reported separately as
 *   kappa0_n = (1/2) log10(n ||G||_1 est); the precision pick uses kappa0).
 * Precision pick (Algorithm 1): FP16 if kappa0 < 4, FP32 if kappa0 <= 8,
 * else FP64 (also when the estimate overflows).  known_kappa > 0 skips the
 * estimate and applies the same thresholds to log10(known_kappa).
 * Pinned: kappa0 equals (1/2) log10(||G||_1 ||G^{-1}||_1) where Hager's
 * estimate is exact (diagonal and inverse-positive G), is a lower estimate
 * within a factor 10 elsewhere, and the precision picks follow the worked
 * cases of Section 7.4.
 * ---------------------------------------------------------------------- */
static int pick_precision(float kappa0)
{
    if (!isfinite(kappa0)) return PREC_FP64;
    if (kappa0 < 4.0f) return PREC_FP16;
    if (kappa0 <= 8.0f) return PREC_FP32;
    return PREC_FP64;
}

int oracle_cond_est(int64_t m, int64_t n, const double* A, int64_t lda, double known_kappa,
                    float* kappa0_out, float* kappa0_n_out, int32_t* choice_out)
{
    if (known_kappa > 0.0) {
        float k0 = (float)log10(known_kappa);
        *kappa0_out = k0;
        if (kappa0_n_out) *kappa0_n_out = k0;
        *choice_out = pick_precision(k0);
        return 0;
    }
    float* G = (float*)malloc(sizeof(float) * (size_t)n * (size_t)n);
    float* x = (float*)malloc(sizeof(float) * (size_t)n);
    float* y = (float*)malloc(sizeof(float) * (size_t)n);
    float* z = (float*)malloc(sizeof(float) * (size_t)n);
    float* t = (float*)malloc(sizeof(float) * (size_t)n);
    if (!G || !x || !y || !z || !t) { free(G); free(x); free(y); free(z); free(t); return -2; }
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i < n; ++i) {
            float acc = 0.0f;
            for (int64_t k = 0; k < m; ++k)
                acc += (float)A[IDX(k, i, lda)] * (float)A[IDX(k, j, lda)];
            G[IDX(i, j, n)] = acc;
        }
    float g1 = 0.0f; /* ||G||_1 = max column sum of |G| */
    for (int64_t j = 0; j < n; ++j) {
        float cs = 0.0f;
        for (int64_t i = 0; i < n; ++i) cs += fabsf(G[IDX(i, j, n)]);
        if (cs > g1) g1 = cs;
    }
    /* FP32 Cholesky, lower triangle in place */
    int broke = 0;
    for (int64_t j = 0; j < n && !broke; ++j) {
        float d = G[IDX(j, j, n)];
        for (int64_t k = 0; k < j; ++k) d -= G[IDX(j, k, n)] * G[IDX(j, k, n)];
        if (!(d > 0.0f) || !isfinite(d)) { broke = 1; break; }
        float ljj = sqrtf(d);
        G[IDX(j, j, n)] = ljj;
        for (int64_t i = j + 1; i < n; ++i) {
            float acc = G[IDX(i, j, n)];
            for (int64_t k = 0; k < j; ++k) acc -= G[IDX(i, k, n)] * G[IDX(j, k, n)];
            G[IDX(i, j, n)] = acc / ljj;
        }
    }
    float k0 = INFINITY, k0n = INFINITY;
    if (!broke) {
        for (int64_t i = 0; i < n; ++i) x[i] = 1.0f / (float)n;
        float est = 0.0f;
        for (int it = 0; it < 5; ++it) {
            /* y = G^{-1} x via L t = x, L^T y = t (FP32) */
            for (int64_t i = 0; i < n; ++i) {
                float acc = x[i];
                for (int64_t k = 0; k < i; ++k) acc -= G[IDX(i, k, n)] * t[k];
                t[i] = acc / G[IDX(i, i, n)];
            }
            for (int64_t i = n - 1; i >= 0; --i) {
                float acc = t[i];
                for (int64_t k = i + 1; k < n; ++k) acc -= G[IDX(k, i, n)] * y[k];
                y[i] = acc / G[IDX(i, i, n)];
            }
            est = 0.0f;
            for (int64_t i = 0; i < n; ++i) est += fabsf(y[i]);
            /* z = G^{-T} sign(y); G is symmetric so the same two solves */
            for (int64_t i = 0; i < n; ++i) {
                float acc = (y[i] >= 0.0f) ? 1.0f : -1.0f;
                for (int64_t k = 0; k < i; ++k) acc -= G[IDX(i, k, n)] * t[k];
                t[i] = acc / G[IDX(i, i, n)];
            }
            for (int64_t i = n - 1; i >= 0; --i) {
                float acc = t[i];
                for (int64_t k = i + 1; k < n; ++k) acc -= G[IDX(k, i, n)] * z[k];
                z[i] = acc / G[IDX(i, i, n)];
            }
            float zmax = 0.0f, ztx = 0.0f;
            int64_t jmax = 0;
            for (int64_t i = 0; i < n; ++i) {
                if (fabsf(z[i]) > zmax) { zmax = fabsf(z[i]); jmax = i; }
                ztx += z[i] * x[i];
            }
            if (zmax <= ztx) break;
            for (int64_t i = 0; i < n; ++i) x[i] = 0.0f;
            x[jmax] = 1.0f;
        }
        float prod = g1 * est;
        if (isfinite(prod) && prod > 0.0f) {
            k0 = 0.5f * log10f(prod);
            k0n = 0.5f * log10f((float)n * prod);
        }
    }
    *kappa0_out = k0;
    if (kappa0_n_out) *kappa0_n_out = k0n;
    *choice_out = pick_precision(k0);
    free(G); free(x); free(y); free(z); free(t);
    return 0;
}

/* Power-of-two factor applied to the s x n sketch before it is rounded to
 * FP16 for the QR: with amax = max |fl32(A_s)| = f 2^E (f in [1/2, 1)) and
 * t the smallest integer with 4^t >= s, the factor is 2^(14 - t - E).  Then
 * every entry of the scaled sketch is below 2^14 / sqrt(s), every column
 * 2-norm (and so every entry of R_s) below 2^14, inside the FP16 range
 * (largest finite value 65504).  Returns 1 for an all-zero or non-finite
 * sketch.  (Library reading: the paper fixes no scaling for the half
 * precision QR.) */
double oracle_fp16_qr_scale(int64_t s, int64_t n, const double* As, int64_t ldas)
{
    double amax = 0.0;
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i < s; ++i) {
            double v = fabs(oracle_round_fp32(As[IDX(i, j, ldas)]));
            if (!isfinite(v)) return 1.0;
            if (v > amax) amax = v;
        }
    if (amax == 0.0) return 1.0;
    int t = 0;
    while (t < 31 && ((int64_t)1 << (2 * t)) < s) ++t;
    int E;
    frexp(amax, &E);
    return ldexp(1.0, 14 - t - E);
}

/* ------------------------------------------------------------------------
 * PNE / HPNE with a randomized preconditioner (Algorithm 1; PNE: the
 * preconditioned normal equations A_p^T A_p y = A_p^T b, R_s x = y; HPNE:
 * A_p^T A x = A_p^T b solved by LU with partial pivoting).
 *   1. precision: sketch_prec / qr_prec, AUTO = condition-estimate pick
 *   2. A_s = Omega A in the sketch precision (oracle_sketch emulation; with
 *      sketch_kind 1 the SRFT sketch oracle_srft_sketch instead)
 *   3. thin QR of A_s: A_s rounded to the QR precision, FP64 Householder,
 *      R_s rounded to the QR precision, then promoted to FP64 (Algorithm 1,
 *      "Promote R_s ... to double precision")
 *   4. A_p = A R_s^{-1} in FP64
 *   5. C = A_p^T A_p (PNE) or A_p^T A (HPNE), c = A_p^T b
 *   6. Cholesky (PNE) or LU with partial pivoting (HPNE)
 *   7. triangular solves; PNE finishes with R_s x = y
 *   8. refine_steps residual corrections: r = b - A x; the same system is
 *      solved with right-hand side A_p^T r for a correction d (PNE:
 *      d = R_s^{-1} y); x += d.  (Refinement is not part of the paper's
 *      method; it is the optional FP64 correction this library offers.)
 * Outputs x (n), optionally R_s (n x n, ldr = n), the chosen precision and
 * kappa0.  Returns the numerical status (0 or 1000+k/2000+k/3000+k).
 * ---------------------------------------------------------------------- */
int oracle_srft_sketch(int64_t m, int64_t n, const double* A, int64_t lda, int64_t s, uint64_t seed,
                       uint32_t pid, int prec, double* As, int64_t ldas);

int oracle_solve(int hpne, int64_t m, int64_t n, const double* A, int64_t lda, const double* b,
                 int64_t s, uint64_t seed, uint32_t pid, int sketch_prec, int qr_prec,
                 int64_t block_rows, int refine_steps, double known_kappa, int sketch_kind, double* x,
                 double* R_out, int32_t* prec_used, float* kappa0_out)
{
    if (m < n || n < 1 || lda < m || s < n) return -1;
    float kappa0 = NAN;
    double qscale = 1.0;
    if (sketch_prec == PREC_AUTO || qr_prec == PREC_AUTO) {
        int32_t choice;
        oracle_cond_est(m, n, A, lda, known_kappa, &kappa0, NULL, &choice);
        if (sketch_prec == PREC_AUTO) sketch_prec = choice;
        if (qr_prec == PREC_AUTO) qr_prec = choice;
    }
    if (prec_used) { prec_used[0] = sketch_prec; prec_used[1] = qr_prec; }
    if (kappa0_out) *kappa0_out = kappa0;

    size_t nn = (size_t)n * (size_t)n;
    double* As = (double*)malloc(sizeof(double) * (size_t)s * (size_t)n);
    double* R = (double*)malloc(sizeof(double) * nn);
    double* Ap = (double*)malloc(sizeof(double) * (size_t)m * (size_t)n);
    double* C = (double*)malloc(sizeof(double) * nn);
    double* c = (double*)malloc(sizeof(double) * (size_t)n);
    double* y = (double*)malloc(sizeof(double) * (size_t)n);
    double* r = (double*)malloc(sizeof(double) * (size_t)m);
    double* d = (double*)malloc(sizeof(double) * (size_t)n);
    int32_t* piv = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    int info = 0;
    if (!As || !R || !Ap || !C || !c || !y || !r || !d || !piv) { info = -2; goto done; }

    /* (the SRFT has no FP16 variant: an FP16 sketch precision runs as FP32) */
    info = sketch_kind == 1 ? oracle_srft_sketch(m, n, A, lda, s, seed, pid,
                                                 sketch_prec == PREC_FP16 ? PREC_FP32 : sketch_prec, As, s)
                            : oracle_sketch(m, n, A, lda, s, seed, pid, sketch_prec, block_rows, As, s, NULL);
    if (info) goto done;
    /* FP16 has a narrow exponent range: the sketch is scaled by a power of
     * two before the rounding and R_s unscaled after it (exact), so that the
     * precision choice depends on the conditioning only, not on the scale of
     * A (Algorithm 1 picks u_p from kappa alone). */
    qscale = (qr_prec == PREC_FP16) ? oracle_fp16_qr_scale(s, n, As, s) : 1.0;
    if (qr_prec != PREC_FP64)
        for (size_t i = 0; i < (size_t)s * (size_t)n; ++i)
            As[i] = to_operand(oracle_round_fp32(As[i]) * qscale, qr_prec);
    info = oracle_householder_r(s, n, As, s, R, n);
    if (info) goto done;
    if (qr_prec != PREC_FP64)
        for (size_t i = 0; i < nn; ++i) R[i] = to_operand(R[i], qr_prec) / qscale;
    if (R_out) memcpy(R_out, R, sizeof(double) * nn);

    info = oracle_precondition(m, n, A, lda, R, n, Ap, m);
    if (info) goto done;
    oracle_gram(m, n, Ap, m, hpne ? A : Ap, hpne ? lda : m, b, C, n, c);
    if (hpne) {
        info = oracle_lu(n, C, n, piv);
        if (info) goto done;
        lu_solve(n, C, n, piv, c, x);
    } else {
        info = oracle_cholesky(n, C, n);
        if (info) goto done;
        chol_solve(n, C, n, c, y);
        info = solve_upper(n, R, n, y, x);
        if (info) goto done;
    }
    for (int step = 0; step < refine_steps; ++step) {
        for (int64_t i = 0; i < m; ++i) {
            double acc = b[i];
            for (int64_t j = 0; j < n; ++j) acc -= A[IDX(i, j, lda)] * x[j];
            r[i] = acc;
        }
        for (int64_t j = 0; j < n; ++j) {
            double acc = 0.0;
            for (int64_t i = 0; i < m; ++i) acc += Ap[IDX(i, j, m)] * r[i];
            c[j] = acc;
        }
        if (hpne) {
            lu_solve(n, C, n, piv, c, d);
        } else {
            chol_solve(n, C, n, c, y);
            solve_upper(n, R, n, y, d);
        }
        for (int64_t j = 0; j < n; ++j) x[j] += d[j];
    }
done:
    if (info > 0)
        for (int64_t j = 0; j < n; ++j) x[j] = NAN;
    free(As); free(R); free(Ap); free(C); free(c); free(y); free(r); free(d); free(piv);
    return info;
}

/* Exposed building blocks for the pins (plain wrappers, no extra logic). */
int oracle_cholesky_solve(int64_t n, const double* L, int64_t ldl, const double* c, double* y)
{
    chol_solve(n, L, ldl, c, y);
    return 0;
}
int oracle_lu_solve(int64_t n, const double* LU, int64_t ldlu, const int32_t* piv, const double* c,
                    double* x)
{
    lu_solve(n, LU, ldlu, piv, c, x);
    return 0;
}
int oracle_upper_solve(int64_t n, const double* R, int64_t ldr, const double* y, double* x)
{
    return solve_upper(n, R, ldr, y, x);
}

/* Selected entries (rows[t], cols[t]) of the sketch A_s = Omega A, computed
 * one by one with the same operand rounding as oracle_sketch (for checks of
 * very large sketches where the full product is too slow on the CPU). */
int oracle_sketch_entries(int64_t m, const double* A, int64_t lda, int64_t s, uint64_t seed,
                          uint32_t pid, int prec, int64_t block_rows, int64_t count,
                          const int64_t* rows, const int64_t* cols, double* out, double* out_abs)
{
    if (m < 1 || s < 1 || lda < m || prec < PREC_FP64 || prec > PREC_FP8) return -1;
    if (block_rows < 1) block_rows = 128;
    int blocked = (prec == PREC_FP16 || prec == PREC_FP8);
    int64_t bs = blocked ? block_rows : m;
    for (int64_t t = 0; t < count; ++t) {
        int64_t i = rows[t], j = cols[t];
        double acc = 0.0, aacc = 0.0;
        for (int64_t k0 = 0; k0 < m; k0 += bs) {
            int64_t k1 = (m - k0 < bs) ? m : k0 + bs;
            double scale = 1.0;
            if (blocked) {
                float amax = 0.0f;
                for (int64_t k = k0; k < k1; ++k) {
                    float a = fabsf((float)A[IDX(k, j, lda)]);
                    if (a > amax) amax = a;
                }
                if (amax == 0.0f) continue;
                if (prec == PREC_FP16) {
                    int E;
                    frexpf(amax, &E);
                    scale = ldexp(1.0, (E - 1) - 14);
                } else {
                    scale = (double)(amax / 448.0f);
                }
            }
            double p = 0.0, pa = 0.0;
            for (int64_t k = k0; k < k1; ++k) {
                double om = to_operand(oracle_omega_entry(seed, pid, i, k), prec);
                double a;
                if (!blocked) {
                    a = to_operand(A[IDX(k, j, lda)], prec);
                } else {
                    float tq = (float)A[IDX(k, j, lda)] / (float)scale;
                    a = (prec == PREC_FP16) ? oracle_round_fp16((double)tq) : oracle_round_e4m3((double)tq);
                }
                p += om * a;
                pa += fabs(om * a);
            }
            acc += p * scale;
            aacc += pa * scale;
        }
        out[t] = acc / sqrt((double)s);
        if (out_abs) out_abs[t] = aacc / sqrt((double)s);
    }
    return 0;
}

/* ------------------------------------------------------------------------
 * Not-normal equations (Section 5.2, eq. e_nne): B^T A x = B^T b for an
 * m x n matrix B of rank n with the column space of A.  In exact arithmetic
 * x is the least-squares solution for any such B (A = B C with C
 * nonsingular, so B^T A = B^T B C is nonsingular and the equations are
 * equivalent to A^T A x = A^T b); B = A_p gives the HPNE, B = A the normal
 * equations.  Steps: C = B^T A, c = B^T b (FP64), LU with partial pivoting
 * (first index of the largest magnitude), L U x = P c; then refine_steps
 * corrections r = b - A x, d = (B^T A)^{-1} B^T r through the same LU,
 * x += d (the library's optional FP64 correction, as for the HPNE).
 * Returns 0 or 3000+k for a zero or non-finite pivot (x is then NaN).
 * ---------------------------------------------------------------------- */
int oracle_nne(int64_t m, int64_t n, const double* A, int64_t lda, const double* B, int64_t ldb,
               const double* b, int refine_steps, double* x)
{
    if (m < n || n < 1 || lda < m || ldb < m || refine_steps < 0) return -1;
    size_t nn = (size_t)n * (size_t)n;
    double* C = (double*)malloc(sizeof(double) * nn);
    double* c = (double*)malloc(sizeof(double) * (size_t)n);
    double* r = (double*)malloc(sizeof(double) * (size_t)m);
    double* d = (double*)malloc(sizeof(double) * (size_t)n);
    int32_t* piv = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    int info = 0;
    if (!C || !c || !r || !d || !piv) { info = -2; goto done; }
    oracle_gram(m, n, B, ldb, A, lda, b, C, n, c);
    info = oracle_lu(n, C, n, piv);
    if (info) goto done;
    lu_solve(n, C, n, piv, c, x);
    for (int step = 0; step < refine_steps; ++step) {
        for (int64_t i = 0; i < m; ++i) {
            double acc = b[i];
            for (int64_t j = 0; j < n; ++j) acc -= A[IDX(i, j, lda)] * x[j];
            r[i] = acc;
        }
        for (int64_t j = 0; j < n; ++j) {
            double acc = 0.0;
            for (int64_t i = 0; i < m; ++i) acc += B[IDX(i, j, ldb)] * r[i];
            c[j] = acc;
        }
        lu_solve(n, C, n, piv, c, d);
        for (int64_t j = 0; j < n; ++j) x[j] += d[j];
    }
done:
    if (info > 0)
        for (int64_t j = 0; j < n; ++j) x[j] = NAN;
    free(C); free(c); free(r); free(d); free(piv);
    return info;
}

/* ------------------------------------------------------------------------
 * Condition estimate from a single-precision QR (library variant of the
 * first step of Algorithm 1; Section 6.1 estimates kappa(A) through the
 * 1-norm condition number of A^T A, which squares it).  Here:
 *   A_s = Omega A (s x n) with the FP32 sketch (oracle_sketch, prec FP32),
 *   rounded to FP32; Householder QR of fl32(A_s) in FP32 arithmetic
 *   (plain float loops, LAPACK reflector convention) giving R (FP32);
 *   ||R||_1 = max column sum of |R|;
 *   est ~ ||R^{-1}||_1 by Hager's method as in oracle_cond_est, with
 *   y = R^{-1} x (back substitution) and z = R^{-T} sign(y) (forward
 *   substitution with R^T), FP32;
 *   kappa0 = log10(||R||_1 est)   (no square root: R is not a Gram matrix);
 *   a zero or non-finite diagonal of R, or a non-finite product, means the
 *   estimate overflows (kappa0 = +inf).  Same thresholds as Algorithm 1.
 * kappa(A_s) differs from kappa(A) by at most the condition number of the
 * sketched orthonormal basis (below 3.73 asymptotically for s = 3n, the
 * Marchenko-Pastur edge (1 + sqrt(n/s)) / (1 - sqrt(n/s))), so kappa0 is
 * within about 0.6 of log10 kappa_1(A_s) ~ log10 kappa(A) -- without the
 * squaring, the FP32 QR resolves kappa(A) up to about 1/u_32 ~ 1.7e7.
 * Parity unpinned for the exact value (Hager is an estimate); pinned by the
 * precision picks and the lower-bound property of Hager's estimate.
 * ---------------------------------------------------------------------- */
int oracle_cond_est_qr(int64_t m, int64_t n, const double* A, int64_t lda, int64_t s, uint64_t seed,
                       uint32_t pid, float* kappa0_out, int32_t* choice_out)
{
    if (m < n || n < 1 || lda < m || s < n) return -1;
    double* As = (double*)malloc(sizeof(double) * (size_t)s * (size_t)n);
    float* W = (float*)malloc(sizeof(float) * (size_t)s * (size_t)n);
    float* v = (float*)malloc(sizeof(float) * (size_t)s);
    float* x = (float*)malloc(sizeof(float) * (size_t)n);
    float* y = (float*)malloc(sizeof(float) * (size_t)n);
    float* z = (float*)malloc(sizeof(float) * (size_t)n);
    int rc = 0;
    float k0 = INFINITY;
    if (!As || !W || !v || !x || !y || !z) { rc = -2; goto done; }
    rc = oracle_sketch(m, n, A, lda, s, seed, pid, PREC_FP32, 128, As, s, NULL);
    if (rc) goto done;
    for (size_t i = 0; i < (size_t)s * (size_t)n; ++i) W[i] = (float)As[i];
    /* FP32 Householder QR, R in the upper triangle of W */
    for (int64_t k = 0; k < n; ++k) {
        int64_t len = s - k;
        for (int64_t i = 0; i < len; ++i) v[i] = W[IDX(k + i, k, s)];
        float alpha = v[0], sig = 0.0f;
        for (int64_t i = 1; i < len; ++i) sig += v[i] * v[i];
        if (sig == 0.0f) continue;                    /* no reflection needed */
        float nrm = sqrtf(alpha * alpha + sig);
        float beta = (alpha >= 0.0f) ? -nrm : nrm;
        float tau = (beta - alpha) / beta;
        float sc = 1.0f / (alpha - beta);
        for (int64_t i = 1; i < len; ++i) v[i] *= sc;
        v[0] = 1.0f;
        W[IDX(k, k, s)] = beta;
        for (int64_t j = k + 1; j < n; ++j) {
            float d = 0.0f;
            for (int64_t i = 0; i < len; ++i) d += v[i] * W[IDX(k + i, j, s)];
            d *= tau;
            for (int64_t i = 0; i < len; ++i) W[IDX(k + i, j, s)] -= d * v[i];
        }
    }
    int ok = 1;
    for (int64_t k = 0; k < n; ++k) {
        float dkk = W[IDX(k, k, s)];
        if (dkk == 0.0f || !isfinite(dkk)) ok = 0;
    }
    if (ok) {
        float r1 = 0.0f;
        for (int64_t j = 0; j < n; ++j) {
            float cs = 0.0f;
            for (int64_t i = 0; i <= j; ++i) cs += fabsf(W[IDX(i, j, s)]);
            if (cs > r1) r1 = cs;
        }
        for (int64_t i = 0; i < n; ++i) x[i] = 1.0f / (float)n;
        float est = 0.0f;
        for (int it = 0; it < 5; ++it) {
            for (int64_t i = n - 1; i >= 0; --i) {          /* R y = x */
                float acc = x[i];
                for (int64_t j = i + 1; j < n; ++j) acc -= W[IDX(i, j, s)] * y[j];
                y[i] = acc / W[IDX(i, i, s)];
            }
            est = 0.0f;
            for (int64_t i = 0; i < n; ++i) est += fabsf(y[i]);
            for (int64_t i = 0; i < n; ++i) {               /* R^T z = sign(y) */
                float acc = (y[i] >= 0.0f) ? 1.0f : -1.0f;
                for (int64_t j = 0; j < i; ++j) acc -= W[IDX(j, i, s)] * z[j];
                z[i] = acc / W[IDX(i, i, s)];
            }
            float zmax = 0.0f, ztx = 0.0f;
            int64_t jmax = 0;
            for (int64_t i = 0; i < n; ++i) {
                if (fabsf(z[i]) > zmax) { zmax = fabsf(z[i]); jmax = i; }
                ztx += z[i] * x[i];
            }
            if (zmax <= ztx) break;
            for (int64_t i = 0; i < n; ++i) x[i] = 0.0f;
            x[jmax] = 1.0f;
        }
        float prod = r1 * est;
        if (isfinite(prod) && prod > 0.0f) k0 = log10f(prod);
    }
done:
    if (kappa0_out) *kappa0_out = k0;
    if (choice_out) *choice_out = pick_precision(k0);
    free(As); free(W); free(v); free(x); free(y); free(z);
    return rc;
}

/* ------------------------------------------------------------------------
 * Subsampled randomized trigonometric transform (Section 6.2, eq. e_sketch:
 * Omega = S F D), in its real form: F is the discrete Hartley transform
 * (H)_{kj} = cas(2 pi k j / m') = cos + sin of that angle, which equals
 * Re(F) - Im(F) of the DFT matrix F_{kj} = exp(-2 pi i k j / m') and is
 * orthogonal up to the factor sqrt(m') -- a real trigonometric transform of
 * the kind Section 7.1 names ("subsampled trigonometric transform").
 *   m' = the smallest 7-smooth integer >= m (A is padded with zero rows:
 *        the sketch of the padded matrix is a sketch of A);
 *   D  = diag(d_j), d_j = +-1 for j < m': bit (j mod 128) of the 128-bit
 *        Philox4x32-10 output at key (seed), counter (j / 128, 0, pid, 3)
 *        (word (j mod 128) / 32, bit j mod 32; bit 1 -> -1);
 *   S  = rows k_0..k_{s-1} of I_{m'} sampled uniformly with replacement:
 *        k_i = floor(w m' / 2^64), w = w0 + 2^32 w1 from Philox at key
 *        (seed), counter (i, 0, pid, 2);
 *   A_s = (1 / sqrt(s)) S H D A  (E[Omega^T Omega] = I: H / sqrt(m') is
 *        orthogonal and each sampled row carries the factor sqrt(m' / s)).
 * Operands: A rounded to the sketch precision via FP32 (FP32, BF16; FP64
 * unrounded), products summed in FP64 with the angle reduced exactly
 * ((j k) mod m' in integers).
 * ---------------------------------------------------------------------- */
int64_t oracle_next_smooth(int64_t m)
{
    for (int64_t x = (m < 1 ? 1 : m);; ++x) {
        int64_t y = x;
        static const int primes[4] = {2, 3, 5, 7};
        for (int p = 0; p < 4; ++p)
            while (y % primes[p] == 0) y /= primes[p];
        if (y == 1) return x;
    }
}

int oracle_srft_sign(uint64_t seed, uint32_t pid, int64_t j)
{
    uint32_t ctr[4] = {(uint32_t)(j / 128), 0u, pid, 3u};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t w[4];
    oracle_philox4x32_10(ctr, key, w);
    int64_t b = j % 128;
    return ((w[b / 32] >> (b % 32)) & 1u) ? -1 : 1;
}

int64_t oracle_srft_index(uint64_t seed, uint32_t pid, int64_t i, int64_t mp)
{
    uint32_t ctr[4] = {(uint32_t)i, 0u, pid, 2u};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t w[4];
    oracle_philox4x32_10(ctr, key, w);
    uint64_t u = (uint64_t)w[0] | ((uint64_t)w[1] << 32);
    return (int64_t)(((unsigned __int128)u * (unsigned __int128)(uint64_t)mp) >> 64);
}

int oracle_srft_sketch(int64_t m, int64_t n, const double* A, int64_t lda, int64_t s, uint64_t seed,
                       uint32_t pid, int prec, double* As, int64_t ldas)
{
    if (m < 1 || n < 1 || s < 1 || lda < m || ldas < s) return -1;
    if (prec != PREC_FP64 && prec != PREC_FP32 && prec != PREC_BF16) return -1;
    int64_t mp = oracle_next_smooth(m);
    double* da = (double*)malloc(sizeof(double) * (size_t)m);
    if (!da) return -2;
    const double pi = 3.14159265358979323846;
    for (int64_t c = 0; c < n; ++c) {
        for (int64_t j = 0; j < m; ++j)
            da[j] = oracle_srft_sign(seed, pid, j) * to_operand(A[IDX(j, c, lda)], prec);
        for (int64_t i = 0; i < s; ++i) {
            int64_t k = oracle_srft_index(seed, pid, i, mp);
            double acc = 0.0;
            for (int64_t j = 0; j < m; ++j) {
                int64_t t = (int64_t)(((unsigned __int128)(uint64_t)j * (uint64_t)k) % (uint64_t)mp);
                double ang = 2.0 * pi * (double)t / (double)mp;
                acc += (cos(ang) + sin(ang)) * da[j];
            }
            As[IDX(i, c, ldas)] = acc / sqrt((double)s);
        }
    }
    free(da);
    return 0;
}

/* Selected entries (rows[t], cols[t]) of the SRFT sketch, each computed as in
 * oracle_srft_sketch (checks of very large sketches). */
int oracle_srft_entries(int64_t m, const double* A, int64_t lda, int64_t s, uint64_t seed, uint32_t pid,
                        int prec, int64_t count, const int64_t* rows, const int64_t* cols, double* out)
{
    if (m < 1 || s < 1 || lda < m) return -1;
    if (prec != PREC_FP64 && prec != PREC_FP32 && prec != PREC_BF16) return -1;
    int64_t mp = oracle_next_smooth(m);
    const double pi = 3.14159265358979323846;
    for (int64_t t = 0; t < count; ++t) {
        int64_t k = oracle_srft_index(seed, pid, rows[t], mp);
        double acc = 0.0;
        for (int64_t j = 0; j < m; ++j) {
            int64_t r = (int64_t)(((unsigned __int128)(uint64_t)j * (uint64_t)k) % (uint64_t)mp);
            double ang = 2.0 * pi * (double)r / (double)mp;
            acc += (cos(ang) + sin(ang)) * oracle_srft_sign(seed, pid, j) * to_operand(A[IDX(j, cols[t], lda)], prec);
        }
        out[t] = acc / sqrt((double)s);
    }
    return 0;
}
