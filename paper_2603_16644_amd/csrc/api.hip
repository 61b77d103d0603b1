// C ABI (include/pne.h): argument checks, workspace layout and the launch
// sequences of Algorithm 1 for PNE and HPNE.  Everything runs on the
// caller's stream from the caller's workspace; nothing here allocates.
#include <math.h>
#include <string.h>

#include "common.h"
#include "kernels.h"
#include "profile.h"

using namespace pne;

namespace {

struct Problem {
    int64_t m, n, lda, s;
    int sketch_prec, qr_prec;
    int hpne;
    int refine;
    int64_t br;
};

bool valid_prec(int p, bool allow_auto, bool allow_fp8)
{
    if (p == PNE_PREC_AUTO) return allow_auto;
    if (p == PNE_PREC_FP8E4M3) return allow_fp8;
    return p >= PNE_PREC_FP64 && p <= PNE_PREC_BF16;
}

// Candidate precisions for sizing: AUTO may resolve to FP16, FP32 or FP64.
void candidates(int p, int* out, int* cnt)
{
    if (p == PNE_PREC_AUTO) {
        out[0] = PNE_PREC_FP16; out[1] = PNE_PREC_FP32; out[2] = PNE_PREC_FP64;
        *cnt = 3;
    } else {
        out[0] = p;
        *cnt = 1;
    }
}

struct Buffers {
    void* scratch;      // shared by sketch / QR / Gram partials / condition estimate
    void* W;            // QR working matrix s x n (FP32 or FP64)
    double* R;          // n x n
    double* Ap;         // m x n, ld m
    double* C;          // n x n
    double* c;          // n
    int32_t* piv;       // n
    double* y;          // n
    double* d;          // n
    double* r;          // m
    double* gv;         // gemv partials
    double* dinv1;      // block inverses: Cholesky factor L, or unit lower L of the LU
    double* dinv2;      // block inverses: R_s (PNE) or U (HPNE)
    float* k0;          // condition estimate
    int32_t* choice;
};

size_t scratch_bytes(const Problem& p, int sk, int qr)
{
    size_t b = sketch_workspace_bytes(p.m, p.n, p.s, sk, p.br);
    size_t q = qr_workspace_bytes(p.s, p.n, qr);
    if (q > b) b = q;
    int64_t splits, kc;
    plan_splitk(p.m, gemm_tiles(p.n, p.n, !p.hpne, 128), &splits, &kc);
    size_t g = ((size_t)splits * p.n * p.n + (size_t)splits * p.n) * sizeof(double) + 512;
    if (g > b) b = g;
    return b;
}

size_t layout(const Problem& p, void* base, size_t cap, Buffers* out, bool with_condest)
{
    int sk[3], qr[3], nsk, nqr;
    candidates(p.sketch_prec, sk, &nsk);
    candidates(p.qr_prec, qr, &nqr);
    size_t scr = 0;
    bool any64 = false;
    for (int i = 0; i < nsk; ++i)
        for (int j = 0; j < nqr; ++j) {
            size_t b = scratch_bytes(p, sk[i], qr[j]);
            if (b > scr) scr = b;
            if (qr[j] == PNE_PREC_FP64) any64 = true;
        }
    if (with_condest) {
        size_t ce = condest_workspace_bytes(p.m, p.n);
        if (ce > scr) scr = ce;
    }
    Arena ar(base, cap);
    Buffers b{};
    b.scratch = ar.take<char>(scr);
    b.W = ar.take<char>((size_t)p.s * p.n * (any64 ? 8 : 4));
    b.R = ar.take<double>((size_t)p.n * p.n);
    b.Ap = ar.take<double>((size_t)p.m * p.n);
    b.C = ar.take<double>((size_t)p.n * p.n);
    b.c = ar.take<double>(p.n);
    b.piv = ar.take<int32_t>(p.n);
    b.y = ar.take<double>(p.n);
    b.d = ar.take<double>(p.n);
    b.r = ar.take<double>(p.m);
    b.gv = ar.take<double>(gemv_t_partials(p.m, p.n));
    b.dinv1 = ar.take<double>(dinv_elems(p.n));
    b.dinv2 = ar.take<double>(dinv_elems(p.n));
    b.k0 = ar.take<float>(4);
    b.choice = ar.take<int32_t>(4);
    if (out) *out = b;
    return ar.used;
}

pne_status check_common(int64_t m, int64_t n, const void* dA, int64_t lda, const pne_opts* o)
{
    if (!o || !dA) return PNE_EINVAL;
    if (n < 1 || m < n || lda < m) return PNE_EINVAL;
    const int64_t s = o->s ? o->s : 3 * n;
    if (s < n) return PNE_EINVAL;
    if (!valid_prec(o->sketch_prec, true, true)) return PNE_EINVAL;
    if (!valid_prec(o->qr_prec, true, false)) return PNE_EINVAL;
    if (o->refine_steps < 0) return PNE_EINVAL;
    const bool scaled = o->sketch_prec == PNE_PREC_FP8E4M3 || o->sketch_prec == PNE_PREC_FP16 ||
                        o->sketch_prec == PNE_PREC_AUTO;
    if (scaled && (o->block_rows < 64 || o->block_rows % 64 != 0)) return PNE_EINVAL;
    if (n > 4096) return PNE_ENOTSUP;
    int qr[3], nqr;
    candidates(o->qr_prec, qr, &nqr);
    for (int j = 0; j < nqr; ++j)
        if (!qr_supported(s, qr[j])) return PNE_ENOTSUP;
    return PNE_OK;
}

Problem make_problem(int64_t m, int64_t n, int64_t lda, const pne_opts* o, int hpne)
{
    Problem p;
    p.m = m; p.n = n; p.lda = lda;
    p.s = o->s ? o->s : 3 * n;
    p.sketch_prec = o->sketch_prec;
    p.qr_prec = o->qr_prec;
    p.hpne = hpne;
    p.refine = o->refine_steps;
    p.br = o->block_rows > 0 ? o->block_rows : 128;
    return p;
}

// Resolve AUTO through the condition estimate (one host synchronisation).
pne_status resolve_precision(const Problem& p, const double* dA, const pne_opts* o, const Buffers& b,
                             size_t scratch_cap, hipStream_t st, int* sk, int* qr, float* k0)
{
    *sk = p.sketch_prec;
    *qr = p.qr_prec;
    *k0 = NAN;
    if (*sk != PNE_PREC_AUTO && *qr != PNE_PREC_AUTO) return PNE_OK;
    int rc = condest_run(p.m, p.n, dA, p.lda, o->known_kappa, b.k0, b.choice, b.scratch, scratch_cap, st);
    if (rc) return (pne_status)rc;
    float hk0;
    int32_t hch;
    HIP_OK(hipMemcpyAsync(&hk0, b.k0, sizeof(float), hipMemcpyDeviceToHost, st));
    HIP_OK(hipMemcpyAsync(&hch, b.choice, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    HIP_OK(hipStreamSynchronize(st));
    if (*sk == PNE_PREC_AUTO) *sk = hch;
    if (*qr == PNE_PREC_AUTO) *qr = hch;
    *k0 = hk0;
    return PNE_OK;
}

size_t scratch_cap_of(const Buffers& b) { return (size_t)((char*)b.W - (char*)b.scratch); }

// sketch + QR -> b.R; returns status
pne_status run_precond(const Problem& p, const double* dA, const pne_opts* o, int sk, int qr,
                       const Buffers& b, int32_t* dinfo, hipStream_t st)
{
    const bool w64 = (qr == PNE_PREC_FP64);
    const size_t cap = scratch_cap_of(b);
    int rc = sketch_run(p.m, p.n, dA, p.lda, p.s, o->seed, o->problem_id, sk, p.br,
                        w64 ? nullptr : (float*)b.W, p.s, w64 ? (double*)b.W : nullptr, p.s,
                        b.scratch, cap, st);
    if (rc) return (pne_status)rc;
    rc = qr_r(p.s, p.n, b.W, p.s, qr, b.R, p.n, dinfo, b.scratch, cap, st);
    return (pne_status)rc;
}

pne_status solve_impl(int hpne, int64_t m, int64_t n, const double* dA, int64_t lda, const double* db,
                      double* dx, const pne_opts* o, void* dwork, size_t work_bytes, int32_t* dinfo,
                      pne_info* hinfo, hipStream_t st)
{
    pne_status chk = check_common(m, n, dA, lda, o);
    if (chk) return chk;
    if (!db || !dx || !dinfo || !dwork) return PNE_EINVAL;
    if (hpne && !lu_supported(n)) return PNE_ENOTSUP;
    Problem p = make_problem(m, n, lda, o, hpne);
    Buffers b;
    const size_t need = layout(p, dwork, work_bytes, &b, true);
    if (work_bytes < need) return PNE_EWORKSPACE;
    prof_reset();
    prof_mark(PH_START, st);
    zero_i32(1, dinfo, st);
    int sk, qr;
    float k0;
    pne_status rc = resolve_precision(p, dA, o, b, scratch_cap_of(b), st, &sk, &qr, &k0);
    if (rc) return rc;
    prof_mark(PH_CONDEST, st);
    rc = run_precond(p, dA, o, sk, qr, b, dinfo, st);
    if (rc) return rc;
    prof_mark(PH_QR, st);
    // A_p = A R_s^{-1}
    trsm_right_upper(m, n, dA, lda, b.R, n, b.Ap, m, st);
    prof_mark(PH_TRSM, st);
    // C = A_p^T A_p (PNE, lower tiles) or A_p^T A (HPNE); c = A_p^T b
    int64_t splits, kc;
    plan_splitk(m, gemm_tiles(n, n, !hpne, 128), &splits, &kc);
    GemmArgs g{};
    g.M = n; g.N = n; g.K = m;
    g.A = b.Ap; g.lda = m; g.transA = 1;
    g.B = hpne ? (const void*)dA : (const void*)b.Ap; g.ldb = hpne ? lda : m; g.transB = 0;
    g.alpha = 1.0; g.beta = 0.0;
    g.C = b.C; g.ldc = n;
    g.lower = !hpne;
    g.splits = splits; g.kchunk = kc;
    g.P = b.scratch;
    g.Pc = (double*)b.scratch + (size_t)splits * n * n;
    g.bvec = db; g.cvec = b.c;
    gemm_f64_partials(g, st);
    prof_mark(PH_GRAM_GEMM, st);
    gemm_f64_reduce(g, st);
    prof_mark(PH_GRAM_REDUCE, st);
    if (hpne) {
        lu_factor(n, b.C, n, b.piv, dinfo, st);
        inv_diag_blocks<double>(n, b.C, n, 1, 0, 1, b.dinv1, st);
        inv_diag_blocks<double>(n, b.C, n, 0, 0, 0, b.dinv2, st);
    } else {
        cholesky<double>(n, b.C, n, dinfo, st);
        inv_diag_blocks<double>(n, b.C, n, 1, 0, 0, b.dinv1, st);
        inv_diag_blocks<double>(n, b.R, n, 0, 0, 0, b.dinv2, st);
    }
    prof_mark(PH_FACTOR, st);
    if (hpne) lu_solve2(n, b.C, n, b.piv, b.dinv1, b.dinv2, b.c, dx, st);
    else pne_solve3(n, b.C, n, b.dinv1, b.R, n, b.dinv2, b.c, dx, st);
    prof_mark(PH_SOLVE, st);
    for (int k = 0; k < p.refine; ++k) {
        residual(m, n, dA, lda, db, dx, b.r, st);
        gemv_t(m, n, b.Ap, m, b.r, b.y, b.gv, st);
        if (hpne) lu_solve2(n, b.C, n, b.piv, b.dinv1, b.dinv2, b.y, b.d, st);
        else pne_solve3(n, b.C, n, b.dinv1, b.R, n, b.dinv2, b.y, b.d, st);
        axpy_update(n, dx, b.d, st);
    }
    fill_nan_on_info(n, dx, dinfo, st);
    prof_mark(PH_REFINE, st);
    if (hipGetLastError() != hipSuccess) return PNE_EHIP;
    if (hinfo) {
        hinfo->sketch_prec_used = sk;
        hinfo->qr_prec_used = qr;
        hinfo->kappa0 = k0;
        hinfo->refine_steps_run = p.refine;
    }
    return PNE_OK;
}

}  // namespace

extern "C" {

void pne_default_opts(pne_opts* o)
{
    if (!o) return;
    memset(o, 0, sizeof(*o));
    o->s = 0;
    o->seed = 0;
    o->problem_id = 0;
    o->sketch_prec = PNE_PREC_AUTO;
    o->qr_prec = PNE_PREC_AUTO;
    o->known_kappa = 0.0;
    o->refine_steps = 1;
    o->block_rows = 128;
}

const char* pne_status_string(pne_status st)
{
    switch (st) {
    case PNE_OK: return "ok";
    case PNE_EINVAL: return "invalid argument";
    case PNE_ENOMEM: return "out of host memory";
    case PNE_EHIP: return "HIP runtime error";
    case PNE_EWORKSPACE: return "workspace too small";
    case PNE_ENOTSUP: return "unsupported size or option";
    }
    return "unknown status";
}

size_t pne_workspace_size(int64_t m, int64_t n, const pne_opts* o, int hpne)
{
    if (check_common(m, n, (const void*)1, m, o) != PNE_OK) return 0;
    Problem p = make_problem(m, n, m, o, hpne);
    return layout(p, nullptr, 0, nullptr, true);
}

pne_status pne_solve(int64_t m, int64_t n, const double* dA, int64_t lda, const double* db, double* dx,
                     const pne_opts* o, void* dwork, size_t work_bytes, int32_t* dinfo, pne_info* hinfo,
                     pne_stream_t stream)
{
    return solve_impl(0, m, n, dA, lda, db, dx, o, dwork, work_bytes, dinfo, hinfo, (hipStream_t)stream);
}

pne_status hpne_solve(int64_t m, int64_t n, const double* dA, int64_t lda, const double* db, double* dx,
                      const pne_opts* o, void* dwork, size_t work_bytes, int32_t* dinfo, pne_info* hinfo,
                      pne_stream_t stream)
{
    return solve_impl(1, m, n, dA, lda, db, dx, o, dwork, work_bytes, dinfo, hinfo, (hipStream_t)stream);
}

size_t sketch_precond_workspace_size(int64_t m, int64_t n, const pne_opts* o)
{
    if (check_common(m, n, (const void*)1, m, o) != PNE_OK) return 0;
    Problem p = make_problem(m, n, m, o, 0);
    return layout(p, nullptr, 0, nullptr, true);
}

pne_status sketch_precond(int64_t m, int64_t n, const double* dA, int64_t lda, const pne_opts* o,
                          double* dR, int64_t ldr, void* dwork, size_t work_bytes, int32_t* dinfo,
                          pne_info* hinfo, pne_stream_t stream)
{
    hipStream_t st = (hipStream_t)stream;
    pne_status chk = check_common(m, n, dA, lda, o);
    if (chk) return chk;
    if (!dR || ldr < n || !dinfo || !dwork) return PNE_EINVAL;
    Problem p = make_problem(m, n, lda, o, 0);
    Buffers b;
    const size_t need = layout(p, dwork, work_bytes, &b, true);
    if (work_bytes < need) return PNE_EWORKSPACE;
    zero_i32(1, dinfo, st);
    int sk, qr;
    float k0;
    pne_status rc = resolve_precision(p, dA, o, b, scratch_cap_of(b), st, &sk, &qr, &k0);
    if (rc) return rc;
    rc = run_precond(p, dA, o, sk, qr, b, dinfo, st);
    if (rc) return rc;
    for (int64_t j = 0; j < n; ++j)
        HIP_OK(hipMemcpyAsync(dR + j * ldr, b.R + j * n, n * sizeof(double), hipMemcpyDeviceToDevice, st));
    if (hinfo) {
        hinfo->sketch_prec_used = sk;
        hinfo->qr_prec_used = qr;
        hinfo->kappa0 = k0;
        hinfo->refine_steps_run = 0;
    }
    return PNE_OK;
}

size_t cond_est_workspace_size(int64_t m, int64_t n)
{
    if (n < 1 || m < n || n > 4096) return 0;
    return condest_workspace_bytes(m, n);
}

pne_status cond_est(int64_t m, int64_t n, const double* dA, int64_t lda, float* dkappa0, int32_t* dchoice,
                    void* dwork, size_t work_bytes, pne_stream_t stream)
{
    if (!dA || !dkappa0 || !dchoice || !dwork) return PNE_EINVAL;
    if (n < 1 || m < n || lda < m) return PNE_EINVAL;
    if (n > 4096) return PNE_ENOTSUP;
    if (work_bytes < condest_workspace_bytes(m, n)) return PNE_EWORKSPACE;
    return (pne_status)condest_run(m, n, dA, lda, 0.0, dkappa0, dchoice, dwork, work_bytes,
                                   (hipStream_t)stream);
}

size_t pne_sketch_workspace_size(int64_t m, int64_t n, int64_t s, int32_t prec)
{
    if (n < 1 || m < 1 || s < 1 || !valid_prec(prec, false, true)) return 0;
    return sketch_workspace_bytes(m, n, s, prec, 128) + 1024;
}

pne_status pne_sketch(int64_t m, int64_t n, const double* dA, int64_t lda, int64_t s, uint64_t seed,
                      uint32_t problem_id, int32_t prec, int32_t block_rows, double* dAs, int64_t ldas,
                      void* dwork, size_t work_bytes, pne_stream_t stream)
{
    if (!dA || !dAs || !dwork) return PNE_EINVAL;
    if (n < 1 || m < 1 || s < 1 || lda < m || ldas < s) return PNE_EINVAL;
    if (!valid_prec(prec, false, true)) return PNE_EINVAL;
    const bool scaled = prec == PNE_PREC_FP8E4M3 || prec == PNE_PREC_FP16;
    const int64_t br = block_rows > 0 ? block_rows : 128;
    if (scaled && br % 64 != 0) return PNE_EINVAL;
    if (work_bytes < sketch_workspace_bytes(m, n, s, prec, br)) return PNE_EWORKSPACE;
    return (pne_status)sketch_run(m, n, dA, lda, s, seed, problem_id, prec, br, nullptr, 0, dAs, ldas,
                                  dwork, work_bytes, (hipStream_t)stream);
}

size_t pne_batched_workspace_size(int64_t batch, const pne_problem_desc* hdesc, const pne_opts* o, int hpne)
{
    if (batch < 1 || !hdesc || !o) return 0;
    size_t best = 0;
    for (int64_t i = 0; i < batch; ++i) {
        size_t b = pne_workspace_size(hdesc[i].m, hdesc[i].n, o, hpne);
        if (b == 0) return 0;
        if (b > best) best = b;
    }
    return best;
}

pne_status pne_solve_batched(int64_t batch, const pne_problem_desc* hdesc, const double* dA_base,
                             const double* db_base, double* dx_base, const pne_opts* o, int hpne,
                             void* dwork, size_t work_bytes, int32_t* dinfo, pne_stream_t stream)
{
    if (batch < 1 || !hdesc || !dA_base || !db_base || !dx_base || !o || !dinfo || !dwork) return PNE_EINVAL;
    for (int64_t i = 0; i < batch; ++i) {
        const pne_problem_desc& d = hdesc[i];
        pne_status chk = check_common(d.m, d.n, dA_base, d.lda, o);
        if (chk) return chk;
        if (d.a_offset < 0 || d.b_offset < 0 || d.x_offset < 0) return PNE_EINVAL;
    }
    if (work_bytes < pne_batched_workspace_size(batch, hdesc, o, hpne)) return PNE_EWORKSPACE;
    for (int64_t i = 0; i < batch; ++i) {
        const pne_problem_desc& d = hdesc[i];
        pne_opts oi = *o;
        oi.problem_id = (uint32_t)i;
        pne_status rc = solve_impl(hpne, d.m, d.n, dA_base + d.a_offset, d.lda, db_base + d.b_offset,
                                   dx_base + d.x_offset, &oi, dwork, work_bytes, dinfo + i, nullptr,
                                   (hipStream_t)stream);
        if (rc) return rc;
    }
    return PNE_OK;
}

}  // extern "C"
