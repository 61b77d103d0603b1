// FP64 Householder-QR least-squares solver on the GPU: the direct method the
// paper compares PNE/HPNE against (Section 7.4, a QR solver built from
// geqrf, orgqr and trsm).  Here Q is never formed: the QR of the augmented
// matrix [A b] yields R and Q^T b together, and
//   [A b] = Q [R_A  c; 0  rho]   =>   x = R_A^{-1} c,  rho = ||b - A x||.
// The tall QR is a tree of Householder QRs (TSQR, Demmel, Grigori,
// Hoemmen, Langou 2012): the rows of [A b] are cut into blocks of at most
// 6144 rows, every block is factored (its R lands in a stacked buffer), then
// groups of stacked R factors are factored again until one R remains.  All
// blocks of a level are factored together: their launches are recorded and
// merged into grouped launches (launch.h), one level after the other.  Every
// factorization is the library's blocked Householder QR in FP64 (qr.hip);
// R_A x = c uses the block-parallel triangular solve.
#include <algorithm>
#include <vector>

#include "common.h"
#include "kernels.h"
#include "launch.h"

namespace pne {

namespace {

constexpr int64_t QRLS_HMAX = 6144;   // tallest block of the FP64 QR kernels

// W (h x N1, ld h) = rows [r0, r0 + rows) of [A b], zero below.
struct AugCopy {
    struct Args {
        int64_t h, rows, n, r0, lda;
        const double* A;
        const double* b;
        double* W;
    };
    static constexpr int NTH = 256, WPE = 0;
    static __device__ void run(const Args& a, int bx, int by)
    {
        const int64_t i = (int64_t)bx * 256 + threadIdx.x;
        const int64_t j = by;   // column 0..n (n = b)
        if (i >= a.h) return;
        double v = 0.0;
        if (i < a.rows) v = j < a.n ? a.A[(a.r0 + i) + j * a.lda] : a.b[a.r0 + i];
        a.W[i + j * a.h] = v;
    }
};

struct QrlsPlan {
    int64_t N1;                  // n + 1
    int64_t nb1, rows1, h1;      // level-1 blocks, rows per block, padded height
    int64_t G;                   // R factors per group above level 1
    std::vector<int64_t> counts; // blocks at every level (level 1 first)
    size_t qrws;                 // QR workspace of one block
};

QrlsPlan qrls_plan(int64_t m, int64_t n)
{
    QrlsPlan p;
    p.N1 = n + 1;
    const int64_t target = std::min<int64_t>(QRLS_HMAX, std::max<int64_t>(4 * p.N1, 2048));
    p.nb1 = std::max<int64_t>(1, ceil_div(m, target));
    p.rows1 = ceil_div(m, p.nb1);
    p.h1 = std::max(p.rows1, p.N1);
    p.G = QRLS_HMAX / p.N1;
    int64_t c = p.nb1;
    p.counts.push_back(c);
    while (c > 1) {
        c = ceil_div(c, p.G);
        p.counts.push_back(c);
    }
    p.qrws = std::max(qr_workspace_bytes(p.h1, p.N1, PNE_PREC_FP64),
                      qr_workspace_bytes(std::min<int64_t>(p.G, p.nb1) * p.N1, p.N1, PNE_PREC_FP64));
    return p;
}

struct QrlsBuffers {
    double *W1, *Sa, *Sb, *DR, *x;
    int32_t *flags, *linfo;
    char *qrws, *tables;
    size_t table_cap;
};

size_t qrls_layout(const QrlsPlan& p, int64_t n, void* base, size_t cap, QrlsBuffers* out, size_t tables)
{
    QrlsBuffers b{};
    Arena ar(base, cap);
    const int64_t N1 = p.N1;
    b.W1 = ar.take<double>((size_t)p.nb1 * p.h1 * N1);
    b.Sa = ar.take<double>((size_t)p.nb1 * N1 * N1);
    b.Sb = ar.take<double>((size_t)p.nb1 * N1 * N1);
    b.DR = ar.take<double>(dinv_elems(n));
    b.x = ar.take<double>(N1);
    b.flags = ar.take<int32_t>(lb_flag_words(n));
    b.linfo = ar.take<int32_t>((size_t)p.nb1);
    b.qrws = ar.take<char>((size_t)p.nb1 * ((p.qrws + 255) & ~(size_t)255));
    b.tables = ar.take<char>(tables);
    b.table_cap = tables;
    if (out) *out = b;
    return ar.used;
}

// Records one level: level 1 copies and factors row blocks of [A b] (R into
// Sa); level l > 1 factors groups of G stacked R factors of `in` (ld
// cnt_in N1) in place and writes their R into `outS` (ld cnt_out N1).
int record_level(Recorder& rec, const QrlsPlan& p, int level, int64_t m, int64_t n, const double* A, int64_t lda,
                 const double* bvec, const QrlsBuffers& b, const double* in, double* outS)
{
    const int64_t N1 = p.N1;
    const int64_t cnt_out = p.counts[level];
    const int64_t cnt_in = level == 0 ? 0 : p.counts[level - 1];
    const size_t qstride = (p.qrws + 255) & ~(size_t)255;
    for (int64_t g = 0; g < cnt_out; ++g) {
        Exec ex;
        ex.rec = &rec;
        ex.member = (int32_t)g;
        ex.stage(ST_QR_ROUND);
        double* W;
        int64_t h, ldw;
        if (level == 0) {
            const int64_t r0 = g * p.rows1;
            const int64_t rows = std::min(p.rows1, m - r0);
            h = p.h1;
            W = b.W1 + (size_t)g * p.h1 * N1;
            ldw = h;
            launch<AugCopy>(ex, ceil_div(h, 256), N1, AugCopy::Args{h, rows, n, r0, lda, A, bvec, W});
        } else {
            const int64_t k = std::min(p.G, cnt_in - g * p.G);   // R factors in this group
            h = k * N1;
            ldw = cnt_in * N1;
            W = const_cast<double*>(in) + g * p.G * N1;
        }
        int rc = qr_r(ex, h, N1, W, ldw, PNE_PREC_FP64, outS + g * N1, cnt_out * N1, b.linfo + g,
                      b.qrws + g * qstride, p.qrws);
        if (rc) return rc;
    }
    return PNE_OK;
}

size_t table_bytes(const Recorder& rec)
{
    size_t t = 256;
    for (const LaunchRec& r : rec.recs) t += r.args_size + 8 + 4 + 16 + 256 + 32;
    return t;
}

// Largest table of any level (sizing pass, no device pointers touched).
size_t qrls_table_bound(const QrlsPlan& p, int64_t m, int64_t n)
{
    QrlsBuffers b;
    qrls_layout(p, n, (void*)(uintptr_t)0x100000, SIZE_MAX / 4, &b, 0);
    size_t best = 0;
    for (size_t l = 0; l < p.counts.size(); ++l) {
        Recorder rec;
        record_level(rec, p, (int)l, m, n, (const double*)(uintptr_t)0x100000, m, (const double*)(uintptr_t)0x100000,
                     b, b.Sa, b.Sb);
        best = std::max(best, table_bytes(rec));
    }
    return best;
}

pne_status qrls_check(int64_t m, int64_t n, int64_t lda)
{
    if (n < 1 || m < n || lda < m) return PNE_EINVAL;
    if (n + 1 > QRLS_HMAX / 2 || n > 4096) return PNE_ENOTSUP;
    return PNE_OK;
}

}  // namespace

}  // namespace pne

using namespace pne;

extern "C" {

size_t qr_ls_workspace_size(int64_t m, int64_t n)
{
    if (qrls_check(m, n, m) != PNE_OK) return 0;
    const QrlsPlan p = qrls_plan(m, n);
    return qrls_layout(p, n, nullptr, 0, nullptr, qrls_table_bound(p, m, n));
}

pne_status qr_ls_solve(int64_t m, int64_t n, const double* dA, int64_t lda, const double* db, double* dx,
                       void* dwork, size_t work_bytes, int32_t* dinfo, pne_stream_t stream)
{
    pne_status chk = qrls_check(m, n, lda);
    if (chk) return chk;
    if (!dA || !db || !dx || !dinfo || !dwork) return PNE_EINVAL;
    const QrlsPlan p = qrls_plan(m, n);
    const size_t tb = qrls_table_bound(p, m, n);
    QrlsBuffers b;
    if (work_bytes < qrls_layout(p, n, dwork, work_bytes, &b, tb)) return PNE_EWORKSPACE;
    hipStream_t st = (hipStream_t)stream;
    Exec ex;
    ex.st = st;
    zero_i32(ex, 1, dinfo);
    // the tree: level 1 writes Sa; every next level reads one stacked buffer
    // and writes the other
    double* bufs[2] = {b.Sa, b.Sb};
    for (size_t l = 0; l < p.counts.size(); ++l) {
        Recorder rec;
        const double* in = l == 0 ? nullptr : bufs[(l - 1) & 1];
        int rc = record_level(rec, p, (int)l, m, n, dA, lda, db, b, in, bufs[l & 1]);
        if (rc) return (pne_status)rc;
        rc = run_recorded(rec, b.tables, b.table_cap, st);
        if (rc) return (pne_status)rc;
    }
    // final R of [A b]: R_A = R(0:n, 0:n), c = R(0:n, n); ld N1 (one block)
    const double* R = bufs[(p.counts.size() - 1) & 1];
    const int64_t ldr = p.N1;
    check_r_diag(ex, n, R, ldr, dinfo);
    inv_diag_blocks<double>(ex, n, R, ldr, 0, 0, 0, b.DR);
    upper_solve_lb(ex, n, R, ldr, b.DR, R + n * ldr, dx, b.flags, dinfo);
    fill_nan_on_info(ex, n, dx, dinfo);
    return hipGetLastError() == hipSuccess ? PNE_OK : PNE_EHIP;
}

}  // extern "C"
