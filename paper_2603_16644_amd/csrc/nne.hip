// Not-normal equations B^T A x = B^T b (Section 5.2, eq. e_nne) for a
// caller-supplied B of rank n with the column space of A.  The HPNE is the
// special case B = A_p (Remark in Section 5.2), so the solve runs the HPNE
// kernels after the preconditioner:
//   C = B^T A, c = B^T b   split-K FP64 MFMA product with the B^T b fold
//                          and a fixed-order reduction
//   P C = L U              LU with partial pivoting (first index of the
//                          largest magnitude), info 3000+k
//   L U x = P c            block-parallel triangular solves
//   refine_steps x         r = b - A x, g = B^T r, same solves, x += d
// Everything in FP64 on the caller's stream, scratch from the caller's
// workspace.
#include "common.h"
#include "kernels.h"
#include "profile.h"

namespace pne {
namespace {

struct NneBuffers {
    double *P, *Pc, *C, *c, *r, *y, *d, *gv, *dinv1, *dinv2;
    int32_t *piv, *flags;
    int64_t splits, kchunk;
};

size_t nne_layout(int64_t m, int64_t n, void* base, NneBuffers* out)
{
    NneBuffers b{};
    plan_splitk(m, gemm_tiles(n, n, m, 0), &b.splits, &b.kchunk);
    Arena ar(base, 0);
    b.P = ar.take<double>((size_t)b.splits * n * n);
    b.Pc = ar.take<double>((size_t)b.splits * n);
    b.C = ar.take<double>((size_t)n * n);
    b.c = ar.take<double>(n);
    b.r = ar.take<double>(m);
    b.y = ar.take<double>(n);
    b.d = ar.take<double>(n);
    b.gv = ar.take<double>(gemv_t_partials(m, n));
    b.dinv1 = ar.take<double>(dinv_elems(n));
    b.dinv2 = ar.take<double>(dinv_elems(n));
    b.piv = ar.take<int32_t>(n);
    b.flags = ar.take<int32_t>(2 * lb_flag_words(n));
    if (out) *out = b;
    return ar.used;
}

pne_status nne_check(int64_t m, int64_t n, int64_t lda, int64_t ldb, int32_t refine_steps)
{
    if (n < 1 || m < n || lda < m || ldb < m || refine_steps < 0) return PNE_EINVAL;
    if (!lu_supported(n) || n > 4096) return PNE_ENOTSUP;
    return PNE_OK;
}

}  // namespace
}  // namespace pne

using namespace pne;

extern "C" {

size_t nne_workspace_size(int64_t m, int64_t n)
{
    if (nne_check(m, n, m, m, 0) != PNE_OK) return 0;
    return nne_layout(m, n, nullptr, nullptr);
}

pne_status nne_solve(int64_t m, int64_t n, const double* dA, int64_t lda, const double* dB, int64_t ldb,
                     const double* db, double* dx, int32_t refine_steps, void* dwork, size_t work_bytes,
                     int32_t* dinfo, pne_stream_t stream)
{
    pne_status chk = nne_check(m, n, lda, ldb, refine_steps);
    if (chk) return chk;
    if (!dA || !dB || !db || !dx || !dinfo || !dwork) return PNE_EINVAL;
    NneBuffers b;
    if (work_bytes < nne_layout(m, n, dwork, &b)) return PNE_EWORKSPACE;
    Exec ex;
    ex.st = (hipStream_t)stream;
    zero_i32(ex, 1, dinfo);
    GemmArgs g{};
    g.M = n; g.N = n; g.K = m;
    g.A = dB; g.lda = ldb; g.transA = 1;
    g.B = dA; g.ldb = lda; g.transB = 0;
    g.alpha = 1.0; g.beta = 0.0;
    g.C = b.C; g.ldc = n;
    g.lower = 0;
    g.splits = b.splits; g.kchunk = b.kchunk;
    g.P = b.P; g.Pc = b.Pc;
    g.bvec = db; g.cvec = b.c;
    gemm_f64_partials(ex, g);
    gemm_f64_reduce(ex, g);
    lu_factor(ex, n, b.C, n, b.piv, dinfo);
    inv_diag_blocks<double>(ex, n, b.C, n, 1, 0, 1, b.dinv1);
    inv_diag_blocks<double>(ex, n, b.C, n, 0, 0, 0, b.dinv2);
    lu_solve_lb(ex, n, b.C, n, b.piv, b.dinv1, b.dinv2, b.c, dx, b.flags, dinfo);
    for (int32_t k = 0; k < refine_steps; ++k) {
        residual(ex, m, n, dA, lda, db, dx, b.r);
        gemv_t(ex, m, n, dB, ldb, b.r, b.y, b.gv);
        lu_solve_lb(ex, n, b.C, n, b.piv, b.dinv1, b.dinv2, b.y, b.d, b.flags, dinfo);
        axpy_update(ex, n, dx, b.d);
    }
    fill_nan_on_info(ex, n, dx, dinfo);
    return hipGetLastError() == hipSuccess ? PNE_OK : PNE_EHIP;
}

}  // extern "C"
