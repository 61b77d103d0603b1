// C ABI (include/pne.h): argument checks, workspace layout and the launch
// sequences of Algorithm 1 for PNE and HPNE.  Everything runs on the
// caller's stream from the caller's workspace; nothing here allocates.
#include <math.h>
#include <string.h>

#include <vector>

#include "common.h"
#include "kernels.h"
#include "profile.h"
#include "tune.h"

using namespace pne;

namespace {

struct Problem {
    int64_t m, n, lda, s;
    int sketch_prec, qr_prec;
    int hpne;
    int refine;
    int64_t br;
    int64_t kchunk_fixed;   // 0: one problem on the machine; > 0: batch planning
    int cond_method;        // 0: FP32 Gram estimate (Section 6.1); 1: FP32 QR of the sketch
    int sketch_kind;        // 0: Gaussian; 1: SRFT (Hartley transform)
};

// Precision the SRFT sketch runs in for a requested sketch precision: FP16
// has no SRFT variant (its range would need scaling) and runs as FP32.
inline int srft_prec(int sk) { return sk == PNE_PREC_FP16 ? PNE_PREC_FP32 : sk; }

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
    double* t;          // n (intermediate vector of the chained solves)
    double* r;          // m
    double* gv;         // gemv partials
    double* dinv1;      // block inverses: Cholesky factor L, or unit lower L of the LU
    double* dinv2;      // block inverses: R_s (PNE) or U (HPNE)
    double* Lt;         // PNE: L^T (n x n)
    double* dinv1t;     // PNE: block inverses of L^T
    int32_t* flags;     // block flags of the triangular solves
    float* k0;          // condition estimate
    int32_t* choice;
};

// Leading dimension of A_p: m rounded up to even, so that its columns start
// on 16-byte boundaries (16-byte loads in its products).
int64_t ap_ld(int64_t m) { return (m + 1) & ~(int64_t)1; }

size_t scratch_bytes(const Problem& p, int sk, int qr)
{
    size_t b = p.sketch_kind == 1 ? srft_workspace_bytes(p.m, p.n, srft_prec(sk))
                                  : sketch_workspace_bytes(p.m, p.n, p.s, sk, p.br, p.kchunk_fixed);
    size_t q = qr_workspace_bytes(p.s, p.n, qr);
    if (q > b) b = q;
    int64_t splits, kc, sd, kcd;
    plan_splitk_gram(p.m, p.n, !p.hpne, p.kchunk_fixed, &splits, &kc, &sd, &kcd);
    if (sd > splits) splits = sd;
    size_t g = ((size_t)splits * p.n * p.n + (size_t)splits * p.n) * sizeof(double) + 512;
    if (g > b) b = g;
    return b;
}

// Workspace of one problem; `own_k0` = false leaves k0/choice out (the batch
// keeps them in arrays of its own).
size_t layout(const Problem& p, void* base, size_t cap, Buffers* out, bool with_condest, bool own_k0 = true)
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
        size_t ce = p.cond_method == 1 ? condest_qr_workspace_bytes(p.m, p.n, p.s, p.kchunk_fixed)
                                       : condest_workspace_bytes(p.m, p.n, p.kchunk_fixed);
        if (ce > scr) scr = ce;
    }
    Arena ar(base, cap);
    Buffers b{};
    b.scratch = ar.take<char>(scr);
    b.W = ar.take<char>((size_t)p.s * p.n * (any64 ? 8 : 4));
    b.R = ar.take<double>((size_t)p.n * p.n);
    b.Ap = ar.take<double>((size_t)ap_ld(p.m) * p.n);
    b.C = ar.take<double>((size_t)p.n * p.n);
    b.c = ar.take<double>(p.n);
    b.piv = ar.take<int32_t>(p.n);
    b.y = ar.take<double>(p.n);
    b.d = ar.take<double>(p.n);
    b.t = ar.take<double>(p.n);
    b.r = ar.take<double>(p.m);
    b.gv = ar.take<double>(gemv_t_partials(p.m, p.n));
    b.dinv1 = ar.take<double>(dinv_elems(p.n));
    b.dinv2 = ar.take<double>(dinv_elems(p.n));
    if (!p.hpne) {
        b.Lt = ar.take<double>((size_t)p.n * p.n);
        b.dinv1t = ar.take<double>(dinv_elems(p.n));
    }
    b.flags = ar.take<int32_t>(3 * lb_flag_words(p.n));
    if (own_k0) {
        b.k0 = ar.take<float>(4);
        b.choice = ar.take<int32_t>(4);
    }
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
    if (o->cond_method != 0 && o->cond_method != 1) return PNE_EINVAL;
    if (o->sketch_kind != 0 && o->sketch_kind != 1) return PNE_EINVAL;
    if (o->sketch_kind == 1 && o->sketch_prec == PNE_PREC_FP8E4M3) return PNE_ENOTSUP;
    if (o->cond_method == 1 && !qr_supported(s, PNE_PREC_FP32)) return PNE_ENOTSUP;
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

Problem make_problem(int64_t m, int64_t n, int64_t lda, const pne_opts* o, int hpne, int64_t kchunk_fixed = 0)
{
    Problem p;
    p.m = m; p.n = n; p.lda = lda;
    p.s = o->s ? o->s : 3 * n;
    p.sketch_prec = o->sketch_prec;
    p.qr_prec = o->qr_prec;
    p.hpne = hpne;
    p.refine = o->refine_steps;
    p.br = o->block_rows > 0 ? o->block_rows : 128;
    p.kchunk_fixed = kchunk_fixed;
    p.cond_method = o->cond_method;
    p.sketch_kind = o->sketch_kind;
    return p;
}

inline void mark(Exec& ex, int phase)
{
    if (!ex.recording()) prof_mark(phase, ex.st);
}

// The condition estimate of one problem into b.k0 / b.choice: the FP32 Gram
// estimate of Section 6.1, or (cond_method 1, no known kappa) the estimate
// from the FP32 QR of the FP32 sketch, which leaves that sketch in b.W and
// its R factor in b.R.
int run_condest(Exec& ex, const Problem& p, const double* dA, const pne_opts* o, uint32_t pid, const Buffers& b,
                size_t scratch_cap)
{
    if (p.cond_method == 1 && !(o->known_kappa > 0.0))
        return condest_qr_run(ex, p.m, p.n, dA, p.lda, p.s, o->seed, pid, b.k0, b.choice, (float*)b.W, b.R,
                              b.scratch, scratch_cap);
    return condest_run(ex, p.m, p.n, dA, p.lda, o->known_kappa, b.k0, b.choice, b.scratch, scratch_cap);
}

// With the QR estimate and both precisions AUTO, an FP32 pick means the
// estimate already computed the preconditioner (FP32 sketch, FP32 QR, same
// seed and rows): R_s is in b.R and is reused as it stands.
bool precond_from_condest(const Problem& p, const pne_opts* o, int sk, int qr)
{
    return p.cond_method == 1 && p.sketch_kind == 0 && !(o->known_kappa > 0.0) && p.sketch_prec == PNE_PREC_AUTO &&
           p.qr_prec == PNE_PREC_AUTO && sk == PNE_PREC_FP32 && qr == PNE_PREC_FP32;
}

// Resolve AUTO through the condition estimate (one host synchronisation).
pne_status resolve_precision(Exec& ex, const Problem& p, const double* dA, const pne_opts* o, const Buffers& b,
                             size_t scratch_cap, int* sk, int* qr, float* k0)
{
    *sk = p.sketch_prec;
    *qr = p.qr_prec;
    *k0 = NAN;
    if (*sk != PNE_PREC_AUTO && *qr != PNE_PREC_AUTO) return PNE_OK;
    int rc = run_condest(ex, p, dA, o, o->problem_id, b, scratch_cap);
    if (rc) return (pne_status)rc;
    float hk0;
    int32_t hch;
    HIP_OK(hipMemcpyAsync(&hk0, b.k0, sizeof(float), hipMemcpyDeviceToHost, ex.st));
    HIP_OK(hipMemcpyAsync(&hch, b.choice, sizeof(int32_t), hipMemcpyDeviceToHost, ex.st));
    HIP_OK(hipStreamSynchronize(ex.st));
    if (*sk == PNE_PREC_AUTO) *sk = hch;
    if (*qr == PNE_PREC_AUTO) *qr = hch;
    *k0 = hk0;
    return PNE_OK;
}

size_t scratch_cap_of(const Buffers& b) { return (size_t)((char*)b.W - (char*)b.scratch); }

// sketch + QR -> b.R
pne_status run_precond(Exec& ex, const Problem& p, const double* dA, uint64_t seed, uint32_t pid, int sk,
                       int qr, const Buffers& b, int32_t* dinfo)
{
    const bool w64 = (qr == PNE_PREC_FP64);
    const size_t cap = scratch_cap_of(b);
    int rc = p.sketch_kind == 1
                 ? srft_run(ex, p.m, p.n, dA, p.lda, p.s, seed, pid, srft_prec(sk), w64 ? nullptr : (float*)b.W, p.s,
                            w64 ? (double*)b.W : nullptr, p.s, b.scratch, cap)
                 : sketch_run(ex, p.m, p.n, dA, p.lda, p.s, seed, pid, sk, p.br, w64 ? nullptr : (float*)b.W, p.s,
                              w64 ? (double*)b.W : nullptr, p.s, b.scratch, cap);
    if (rc) return (pne_status)rc;
    rc = qr_r(ex, p.s, p.n, b.W, p.s, qr, b.R, p.n, dinfo, b.scratch, cap);
    mark(ex, PH_QR);
    return (pne_status)rc;
}

// A_p = A R_s^{-1}, C = A_p^T A_p (PNE, lower tiles) or A_p^T A (HPNE) and
// c = A_p^T b (Algorithm 1 "Solve A_p" and the normal-equation matrices).
void run_gram(Exec& ex, const Problem& p, const double* dA, const double* db, const Buffers& b)
{
    const int64_t m = p.m, n = p.n, lda = p.lda;
    const int hpne = p.hpne;
    ex.stage(ST_TRSM);
    const int64_t ldap = ap_ld(m);
    trsm_right_upper(ex, m, n, dA, lda, b.R, n, b.Ap, ldap);
    mark(ex, PH_TRSM);
    ex.stage(ST_GRAM);
    int64_t splits, kc, sd, kcd;
    plan_splitk_gram(m, n, !hpne, ex.kchunk_fixed, &splits, &kc, &sd, &kcd);
    GemmArgs g{};
    g.M = n; g.N = n; g.K = m;
    g.A = b.Ap; g.lda = ldap; g.transA = 1;
    g.B = hpne ? (const void*)dA : (const void*)b.Ap; g.ldb = hpne ? lda : ldap; g.transB = 0;
    g.alpha = 1.0; g.beta = 0.0;
    g.C = b.C; g.ldc = n;
    g.lower = !hpne;
    g.splits = splits; g.kchunk = kc;
    g.splits_diag = sd; g.kchunk_diag = kcd;
    g.P = b.scratch;
    g.Pc = (double*)b.scratch + (size_t)(sd > splits ? sd : splits) * n * n;
    g.bvec = db; g.cvec = b.c;
    gemm_f64_partials(ex, g);
    mark(ex, PH_GRAM_GEMM);
    ex.stage(ST_GRAM_REDUCE);
    gemm_f64_reduce(ex, g);
    mark(ex, PH_GRAM_REDUCE);
}

// Cholesky (PNE) or LU with partial pivoting (HPNE) of C in place, then the
// inverses of the 64 x 64 diagonal blocks the triangular solves use.
void run_factor(Exec& ex, const Problem& p, const Buffers& b, int32_t* dinfo)
{
    const int64_t n = p.n;
    const int hpne = p.hpne;
    ex.stage(ST_FACTOR);
    if (hpne) lu_factor(ex, n, b.C, n, b.piv, dinfo);
    else cholesky<double>(ex, n, b.C, n, dinfo, b.dinv1);
    ex.stage(ST_FACTOR_INV);
    if (hpne) {
        inv_diag_blocks<double>(ex, n, b.C, n, 1, 0, 1, b.dinv1);
        inv_diag_blocks<double>(ex, n, b.C, n, 0, 0, 0, b.dinv2);
    } else {
        inv_diag_blocks<double>(ex, n, b.R, n, 0, 0, 0, b.dinv2);
        transpose_f64(ex, n, n, b.C, n, b.Lt, n);
        transpose_dinv(ex, n, b.dinv1, b.dinv1t);
    }
    mark(ex, PH_FACTOR);
}

// A_p, Gram, factorization, solves and refinement (Algorithm 1 after the
// preconditioner) for one problem.
pne_status run_solve(Exec& ex, const Problem& p, const double* dA, const double* db, double* dx,
                     const Buffers& b, int32_t* dinfo)
{
    const int64_t m = p.m, n = p.n, lda = p.lda;
    const int hpne = p.hpne;
    run_gram(ex, p, dA, db, b);
    run_factor(ex, p, b, dinfo);
    ex.stage(ST_SOLVE);
    if (hpne) lu_solve_lb(ex, n, b.C, n, b.piv, b.dinv1, b.dinv2, b.c, dx, b.flags, dinfo);
    else pne_solve_lb(ex, n, b.C, n, b.dinv1, b.Lt, b.dinv1t, b.R, n, b.dinv2, b.c, dx, b.t, b.flags, dinfo);
    mark(ex, PH_SOLVE);
    ex.stage(ST_REFINE);
    for (int k = 0; k < p.refine; ++k) {
        ex.iter((uint32_t)k);
        residual(ex, m, n, dA, lda, db, dx, b.r);
        gemv_t(ex, m, n, b.Ap, ap_ld(m), b.r, b.y, b.gv);
        if (hpne) lu_solve_lb(ex, n, b.C, n, b.piv, b.dinv1, b.dinv2, b.y, b.d, b.flags, dinfo);
        else pne_solve_lb(ex, n, b.C, n, b.dinv1, b.Lt, b.dinv1t, b.R, n, b.dinv2, b.y, b.d, b.t, b.flags, dinfo);
        axpy_update(ex, n, dx, b.d);
    }
    ex.stage(ST_FINISH);
    fill_nan_on_info(ex, n, dx, dinfo);
    mark(ex, PH_REFINE);
    return PNE_OK;
}

// pne_opts::check_finite: each problem's A (m x n, ld lda) and b scanned
// for non-finite entries (AllFinite writes 5000 to its info word), the info
// words read back; PNE_EINVAL if any is set.
pne_status check_finite_inputs(hipStream_t st, int64_t count, const int64_t* m, const int64_t* n,
                               const double* const* A, const int64_t* lda, const double* const* b, int32_t* dinfo)
{
    Exec ex;
    ex.st = st;
    zero_i32(ex, count, dinfo);
    for (int64_t i = 0; i < count; ++i) all_finite(ex, m[i], n[i], A[i], lda[i], b[i], dinfo + i);
    std::vector<int32_t> h((size_t)count);
    if (hipMemcpyAsync(h.data(), dinfo, (size_t)count * sizeof(int32_t), hipMemcpyDeviceToHost, st) != hipSuccess)
        return PNE_EHIP;
    if (hipStreamSynchronize(st) != hipSuccess) return PNE_EHIP;
    for (int32_t v : h)
        if (v != 0) return PNE_EINVAL;
    return PNE_OK;
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
    Exec ex;
    ex.st = st;
    if (o->check_finite) {
        const pne_status fc = check_finite_inputs(st, 1, &m, &n, &dA, &lda, &db, dinfo);
        if (fc) return fc;
    }
    prof_reset();
    prof_mark(PH_START, st);
    ex.stage(ST_INIT);
    zero_i32(ex, 1, dinfo);
    int sk, qr;
    float k0;
    pne_status rc = resolve_precision(ex, p, dA, o, b, scratch_cap_of(b), &sk, &qr, &k0);
    if (rc) return rc;
    mark(ex, PH_CONDEST);
    if (!precond_from_condest(p, o, sk, qr)) {
        rc = run_precond(ex, p, dA, o->seed, o->problem_id, sk, qr, b, dinfo);
        if (rc) return rc;
    }
    rc = run_solve(ex, p, dA, db, dx, b, dinfo);
    if (rc) return rc;
    if (hipGetLastError() != hipSuccess) return PNE_EHIP;
    if (hinfo) {
        hinfo->sketch_prec_used = sk;
        hinfo->qr_prec_used = qr;
        hinfo->kappa0 = k0;
        hinfo->refine_steps_run = p.refine;
    }
    return PNE_OK;
}

// ---------------------------------------------------------------- batches
// Row chunk of the split-K products in a batch: every member's long products
// are cut into pieces of TuneParams::batch_kchunk rows (8192 unless the
// autotuner chose another length for the workload), so that work-groups
// carry similar work across members of very different sizes.
inline int64_t batch_kchunk() { return tune_params().batch_kchunk; }

struct BatchLayout {
    float* k0;              // [batch] condition estimates
    int32_t* choice;        // [batch] precision picks
    std::vector<Buffers> buf;
    std::vector<Problem> prob;
    char* tables;           // group tables
    size_t table_cap;
    size_t fixed_bytes;     // everything but the tables
};

bool batch_auto(const pne_opts* o) { return o->sketch_prec == PNE_PREC_AUTO || o->qr_prec == PNE_PREC_AUTO; }

void batch_layout(int64_t batch, const pne_problem_desc* hd, const pne_opts* o, int hpne, void* base, size_t cap,
                  BatchLayout* L)
{
    Arena ar(base, cap);
    L->k0 = ar.take<float>(batch);
    L->choice = ar.take<int32_t>(batch);
    L->buf.resize(batch);
    L->prob.resize(batch);
    const bool with_ce = batch_auto(o);
    for (int64_t i = 0; i < batch; ++i) {
        L->prob[i] = make_problem(hd[i].m, hd[i].n, hd[i].lda, o, hpne, batch_kchunk());
        const size_t need = layout(L->prob[i], nullptr, 0, nullptr, with_ce, false);
        char* region = ar.take<char>(need);
        layout(L->prob[i], region, need, &L->buf[i], with_ce, false);
        L->buf[i].k0 = L->k0 ? L->k0 + i : nullptr;
        L->buf[i].choice = L->choice ? L->choice + i : nullptr;
    }
    L->fixed_bytes = ar.used;
    L->tables = base ? (char*)base + ar.used : nullptr;
    L->table_cap = cap > ar.used ? cap - ar.used : 0;
}

// Upper bound of the group-table bytes of a recording: every record adds its
// arguments and two int32 entries, and at most one group header, one
// alignment pad and one 256-byte table alignment.
size_t table_bound(const Recorder& rec)
{
    size_t b = 256;
    for (const LaunchRec& r : rec.recs) b += r.args_size + 8 + 4 + 16 + 256 + 32;
    return b;
}

// Records the launches of every member (main pipeline with the resolved
// precisions sk/qr per member).
pne_status record_batch(Recorder& rec, int64_t batch, const pne_problem_desc* hd, const double* dA_base,
                        const double* db_base, double* dx_base, const pne_opts* o, const BatchLayout& L,
                        const int32_t* sk, const int32_t* qr, int32_t* dinfo)
{
    // (members whose QR estimate already computed the FP32 preconditioner
    // skip the sketch and QR)
    for (int64_t i = 0; i < batch; ++i) {
        Exec ex;
        ex.rec = &rec;
        ex.member = (int32_t)i;
        ex.kchunk_fixed = batch_kchunk();
        const Problem& p = L.prob[i];
        const double* A = dA_base ? dA_base + hd[i].a_offset : nullptr;
        const double* b = db_base ? db_base + hd[i].b_offset : nullptr;
        double* x = dx_base ? dx_base + hd[i].x_offset : nullptr;
        pne_status rc = PNE_OK;
        if (!precond_from_condest(p, o, sk[i], qr[i])) {
            rc = run_precond(ex, p, A, o->seed, (uint32_t)hd[i].problem_id, sk[i], qr[i], L.buf[i],
                             dinfo ? dinfo + i : nullptr);
            if (rc) return rc;
        }
        rc = run_solve(ex, p, A, b, x, L.buf[i], dinfo ? dinfo + i : nullptr);
        if (rc) return rc;
    }
    return PNE_OK;
}

pne_status record_condest(Recorder& rec, int64_t batch, const pne_problem_desc* hd, const double* dA_base,
                          const pne_opts* o, const BatchLayout& L)
{
    for (int64_t i = 0; i < batch; ++i) {
        Exec ex;
        ex.rec = &rec;
        ex.member = (int32_t)i;
        ex.kchunk_fixed = batch_kchunk();
        const Problem& p = L.prob[i];
        const Buffers& b = L.buf[i];
        int rc = run_condest(ex, p, dA_base ? dA_base + hd[i].a_offset : nullptr, o, (uint32_t)hd[i].problem_id, b,
                             scratch_cap_of(b));
        if (rc) return (pne_status)rc;
    }
    return PNE_OK;
}

pne_status check_batch(int64_t batch, const pne_problem_desc* hd, const pne_opts* o, int hpne)
{
    if (batch < 1 || batch > (1 << 24) || !hd || !o) return PNE_EINVAL;
    for (int64_t i = 0; i < batch; ++i) {
        const pne_problem_desc& d = hd[i];
        pne_status chk = check_common(d.m, d.n, (const void*)1, d.lda, o);
        if (chk) return chk;
        if (d.a_offset < 0 || d.b_offset < 0 || d.x_offset < 0) return PNE_EINVAL;
        if (d.problem_id < 0 || d.problem_id > (int64_t)UINT32_MAX) return PNE_EINVAL;
        if (hpne && !lu_supported(d.n)) return PNE_ENOTSUP;
    }
    return PNE_OK;
}

size_t batched_size(int64_t batch, const pne_problem_desc* hd, const pne_opts* o, int hpne)
{
    if (check_batch(batch, hd, o, hpne) != PNE_OK) return 0;
    // sizing pass: a placeholder base address (never dereferenced) gives the
    // drivers non-null buffers with their real capacities
    BatchLayout L;
    batch_layout(batch, hd, o, hpne, (void*)(uintptr_t)0x100000, SIZE_MAX / 4, &L);
    // table bound over every precision a member may use, plus the condition
    // estimate's tables (a plan keeps both resident)
    int sk[3], qr[3], nsk, nqr;
    candidates(o->sketch_prec, sk, &nsk);
    candidates(o->qr_prec, qr, &nqr);
    size_t tb = 0;
    std::vector<int32_t> vs(batch), vq(batch);
    for (int a = 0; a < nsk; ++a)
        for (int c = 0; c < nqr; ++c) {
            if (o->sketch_prec == PNE_PREC_AUTO && o->qr_prec == PNE_PREC_AUTO && a != c) continue;
            for (int64_t i = 0; i < batch; ++i) { vs[i] = sk[a]; vq[i] = qr[c]; }
            Recorder rec;
            if (record_batch(rec, batch, hd, nullptr, nullptr, nullptr, o, L, vs.data(), vq.data(), nullptr))
                return 0;
            size_t b = table_bound(rec);
            if (b > tb) tb = b;
        }
    if (batch_auto(o)) {
        Recorder rec;
        if (record_condest(rec, batch, hd, nullptr, o, L)) return 0;
        tb += table_bound(rec);
    }
    return L.fixed_bytes + tb;
}

// Tuned parameters of a batched workload (the cache entry of its key, else
// the defaults).
TuneParams batch_tune(int64_t batch, const pne_problem_desc* hd, const pne_opts* o, int hpne)
{
    double sn = 0.0, sm = 0.0;
    for (int64_t i = 0; i < batch; ++i) { sn += (double)hd[i].n; sm += (double)hd[i].m; }
    TuneParams tp;
    tune_lookup(tune_key_batched(hpne, o->sketch_prec, o->qr_prec, batch, sn / batch, sm / batch), &tp);
    return tp;
}

}  // namespace

// A batched solve prepared once and executed any number of times: the
// precisions (AUTO resolved at creation), the tuned launch parameters, and
// the grouped launch sequence with its tables resident in the workspace.
struct pne_batch_plan_s {
    int64_t batch = 0;
    int32_t* dinfo = nullptr;
    char* dtables = nullptr;
    std::vector<pne::LaunchGroup> ce_groups;    // condition estimate (AUTO)
    std::vector<pne::LaunchGroup> main_groups;  // the solves
    pne::TuneParams tune;
    bool rerun_ce = false;   // some member takes its preconditioner from the estimate
    hipGraphExec_t gexec = nullptr;
    ~pne_batch_plan_s()
    {
        if (gexec) (void)hipGraphExecDestroy(gexec);
    }
};

namespace {

// Builds a plan: records, groups and uploads the launch sequence (one wait
// for the upload; with AUTO the estimate runs once and its picks are read
// back).  Runs under the tuned parameters of the workload.
pne_status plan_create(int64_t batch, const pne_problem_desc* hd, const double* dA_base, const double* db_base,
                       double* dx_base, const pne_opts* o, int hpne, void* dwork, size_t work_bytes, int32_t* dinfo,
                       hipStream_t st, const TuneParams& tp, pne_batch_plan_s** out)
{
    *out = nullptr;
    pne_status chk = check_batch(batch, hd, o, hpne);
    if (chk) return chk;
    if (!dA_base || !db_base || !dx_base || !dinfo || !dwork) return PNE_EINVAL;
    TuneScope scope(tp);
    if (work_bytes < batched_size(batch, hd, o, hpne)) return PNE_EWORKSPACE;
    BatchLayout L;
    batch_layout(batch, hd, o, hpne, dwork, work_bytes, &L);
    std::vector<int32_t> sk(batch, o->sketch_prec), qr(batch, o->qr_prec);
    GroupSeq ce, mainseq;
    size_t toff = 0;
    if (batch_auto(o)) {
        Recorder rec;
        pne_status rc = record_condest(rec, batch, hd, dA_base, o, L);
        if (rc) return rc;
        rc = (pne_status)build_groups(rec, &ce);
        if (rc) return rc;
        if (ce.blob.size() > L.table_cap) return PNE_EWORKSPACE;
        HIP_OK(hipMemcpyAsync(L.tables, ce.blob.data(), ce.blob.size(), hipMemcpyHostToDevice, st));
        enqueue_groups(ce.groups, L.tables, st, false);
        std::vector<int32_t> ch(batch);
        HIP_OK(hipMemcpyAsync(ch.data(), L.choice, batch * sizeof(int32_t), hipMemcpyDeviceToHost, st));
        HIP_OK(hipStreamSynchronize(st));
        if (hipGetLastError() != hipSuccess) return PNE_EHIP;
        for (int64_t i = 0; i < batch; ++i) {
            if (sk[i] == PNE_PREC_AUTO) sk[i] = ch[i];
            if (qr[i] == PNE_PREC_AUTO) qr[i] = ch[i];
        }
        toff = (ce.blob.size() + 255) & ~(size_t)255;
    }
    Recorder rec;
    pne_status rc = record_batch(rec, batch, hd, dA_base, db_base, dx_base, o, L, sk.data(), qr.data(), dinfo);
    if (rc) return rc;
    rc = (pne_status)build_groups(rec, &mainseq);
    if (rc) return rc;
    if (toff + mainseq.blob.size() > L.table_cap) return PNE_EWORKSPACE;
    if (!mainseq.blob.empty()) {
        HIP_OK(hipMemcpyAsync(L.tables + toff, mainseq.blob.data(), mainseq.blob.size(), hipMemcpyHostToDevice, st));
        HIP_OK(hipStreamSynchronize(st));   // the host blobs are released on return
    }
    pne_batch_plan_s* plan = new (std::nothrow) pne_batch_plan_s;
    if (!plan) return PNE_ENOMEM;
    plan->batch = batch;
    plan->dinfo = dinfo;
    plan->dtables = L.tables;
    plan->ce_groups = ce.groups;
    plan->main_groups = mainseq.groups;
    for (LaunchGroup& g : plan->main_groups) g.off += toff;
    plan->tune = tp;
    for (int64_t i = 0; i < batch; ++i)
        if (precond_from_condest(L.prob[i], o, sk[i], qr[i])) plan->rerun_ce = true;
    *out = plan;
    return PNE_OK;
}

// Enqueues a plan: clear the info words, then every grouped launch (kernel
// launches only).  run_ce = false skips the condition estimate (it has just
// run at creation on the same data).
pne_status plan_execute(pne_batch_plan_s* plan, hipStream_t st, bool run_ce)
{
    TuneScope scope(plan->tune);   // launch forms (persistent or not) chosen with the plan
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cs) != hipSuccess) return PNE_EHIP;
    const bool marks = cs == hipStreamCaptureStatusNone;
    if (marks) {
        prof_reset();
        prof_mark(PH_START, st);
    }
    Exec ex0;
    ex0.st = st;
    zero_i32(ex0, plan->batch, plan->dinfo);
    if (run_ce) enqueue_groups(plan->ce_groups, plan->dtables, st, false);
    if (marks) prof_mark(PH_CONDEST, st);
    enqueue_groups(plan->main_groups, plan->dtables, st, marks);
    return hipGetLastError() == hipSuccess ? PNE_OK : PNE_EHIP;
}

pne_status solve_batched(int64_t batch, const pne_problem_desc* hd, const double* dA_base, const double* db_base,
                         double* dx_base, const pne_opts* o, int hpne, void* dwork, size_t work_bytes,
                         int32_t* dinfo, hipStream_t st)
{
    pne_status chk = check_batch(batch, hd, o, hpne);
    if (chk) return chk;
    if (o->check_finite) {
        if (!dA_base || !db_base || !dinfo) return PNE_EINVAL;
        std::vector<int64_t> m(batch), n(batch), lda(batch);
        std::vector<const double*> A(batch), b(batch);
        for (int64_t i = 0; i < batch; ++i) {
            m[i] = hd[i].m;
            n[i] = hd[i].n;
            lda[i] = hd[i].lda;
            A[i] = dA_base + hd[i].a_offset;
            b[i] = db_base + hd[i].b_offset;
        }
        const pne_status fc = check_finite_inputs(st, batch, m.data(), n.data(), A.data(), lda.data(), b.data(), dinfo);
        if (fc) return fc;
    }
    pne_batch_plan_s* plan = nullptr;
    pne_status rc = plan_create(batch, hd, dA_base, db_base, dx_base, o, hpne, dwork, work_bytes, dinfo, st,
                                batch_tune(batch, hd, o, hpne), &plan);
    if (rc) return rc;
    rc = plan_execute(plan, st, false);
    delete plan;
    return rc;
}

}  // namespace

namespace pne {

// Workspace bytes of one PNE/HPNE solve (argument checks of solve_impl that
// need no device pointers); used by the no-allocation entry point.
pne_status solve_workspace(int hpne, int64_t m, int64_t n, int64_t lda, const pne_opts* o, size_t* need)
{
    pne_status chk = check_common(m, n, (const void*)1, lda, o);
    if (chk) return chk;
    if (hpne && !lu_supported(n)) return PNE_ENOTSUP;
    *need = layout(make_problem(m, n, lda, o, hpne), nullptr, 0, nullptr, true);
    return PNE_OK;
}

pne_status solve_entry(int hpne, int64_t m, int64_t n, const double* dA, int64_t lda, const double* db,
                       double* dx, const pne_opts* o, void* dwork, size_t work_bytes, int32_t* dinfo,
                       pne_info* hinfo, hipStream_t st)
{
    return solve_impl(hpne, m, n, dA, lda, db, dx, o, dwork, work_bytes, dinfo, hinfo, st);
}

}  // namespace pne

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
    o->cond_method = 0;
    o->sketch_kind = 0;
    o->check_finite = 0;
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
    Exec ex;
    ex.st = st;
    zero_i32(ex, 1, dinfo);
    int sk, qr;
    float k0;
    pne_status rc = resolve_precision(ex, p, dA, o, b, scratch_cap_of(b), &sk, &qr, &k0);
    if (rc) return rc;
    if (!precond_from_condest(p, o, sk, qr)) {
        rc = run_precond(ex, p, dA, o->seed, o->problem_id, sk, qr, b, dinfo);
        if (rc) return rc;
    }
    copy_f64(ex, n, n, b.R, n, dR, ldr);
    if (hipGetLastError() != hipSuccess) return PNE_EHIP;
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
    Exec ex;
    ex.st = (hipStream_t)stream;
    return (pne_status)condest_run(ex, m, n, dA, lda, 0.0, dkappa0, dchoice, dwork, work_bytes);
}

size_t cond_est_qr_workspace_size(int64_t m, int64_t n, int64_t s)
{
    if (n < 1 || m < n || n > 4096) return 0;
    if (s == 0) s = 3 * n;
    if (s < n || !qr_supported(s, PNE_PREC_FP32)) return 0;
    Arena ar(nullptr, 0);
    ar.take<float>((size_t)s * n);
    ar.take<double>((size_t)n * n);
    return ar.used + condest_qr_workspace_bytes(m, n, s);
}

pne_status cond_est_qr(int64_t m, int64_t n, const double* dA, int64_t lda, int64_t s, uint64_t seed,
                       float* dkappa0, int32_t* dchoice, void* dwork, size_t work_bytes, pne_stream_t stream)
{
    if (!dA || !dkappa0 || !dchoice || !dwork) return PNE_EINVAL;
    if (n < 1 || m < n || lda < m) return PNE_EINVAL;
    if (s == 0) s = 3 * n;
    if (s < n) return PNE_EINVAL;
    if (n > 4096 || !qr_supported(s, PNE_PREC_FP32)) return PNE_ENOTSUP;
    if (work_bytes < cond_est_qr_workspace_size(m, n, s)) return PNE_EWORKSPACE;
    Arena ar(dwork, work_bytes);
    float* W = ar.take<float>((size_t)s * n);
    double* R = ar.take<double>((size_t)n * n);
    Exec ex;
    ex.st = (hipStream_t)stream;
    return (pne_status)condest_qr_run(ex, m, n, dA, lda, s, seed, 0, dkappa0, dchoice, W, R, (char*)dwork + ar.used,
                                      work_bytes - ar.used);
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
    Exec ex;
    ex.st = (hipStream_t)stream;
    return (pne_status)sketch_run(ex, m, n, dA, lda, s, seed, problem_id, prec, br, nullptr, 0, dAs, ldas,
                                  dwork, work_bytes);
}

size_t pne_sketch_srft_workspace_size(int64_t m, int64_t n, int32_t prec)
{
    if (n < 1 || m < 1 || !srft_supported(prec)) return 0;
    return srft_workspace_bytes(m, n, prec);
}

pne_status pne_sketch_srft(int64_t m, int64_t n, const double* dA, int64_t lda, int64_t s, uint64_t seed,
                           uint32_t problem_id, int32_t prec, double* dAs, int64_t ldas, void* dwork,
                           size_t work_bytes, pne_stream_t stream)
{
    if (!dA || !dAs || !dwork) return PNE_EINVAL;
    if (n < 1 || m < 1 || s < 1 || lda < m || ldas < s) return PNE_EINVAL;
    if (!srft_supported(prec)) return PNE_ENOTSUP;
    if (work_bytes < srft_workspace_bytes(m, n, prec)) return PNE_EWORKSPACE;
    Exec ex;
    ex.st = (hipStream_t)stream;
    return (pne_status)srft_run(ex, m, n, dA, lda, s, seed, problem_id, prec, nullptr, 0, dAs, ldas, dwork,
                                work_bytes);
}

static Problem gram_problem(int64_t m, int64_t n, int64_t lda, int hpne)
{
    pne_opts o;
    pne_default_opts(&o);
    o.s = n;
    o.sketch_prec = PNE_PREC_FP64;
    o.qr_prec = PNE_PREC_FP64;
    o.refine_steps = 0;
    return make_problem(m, n, lda, &o, hpne);
}

size_t pne_gram_workspace_size(int64_t m, int64_t n, int hpne)
{
    if (n < 1 || m < n || n > 4096) return 0;
    return layout(gram_problem(m, n, m, hpne), nullptr, 0, nullptr, false);
}

pne_status pne_gram(int64_t m, int64_t n, const double* dA, int64_t lda, const double* db, const double* dR,
                    int64_t ldr, int hpne, int factor, double* dC, int64_t ldc, double* dc, int32_t* dpiv,
                    void* dwork, size_t work_bytes, int32_t* dinfo, pne_stream_t stream)
{
    if (!dA || !db || !dR || !dC || !dc || !dinfo || !dwork) return PNE_EINVAL;
    if (n < 1 || m < n || lda < m || ldr < n || ldc < n) return PNE_EINVAL;
    if (n > 4096) return PNE_ENOTSUP;
    if (hpne && factor && !dpiv) return PNE_EINVAL;
    Problem p = gram_problem(m, n, lda, hpne ? 1 : 0);
    Buffers b;
    if (work_bytes < layout(p, dwork, work_bytes, &b, false)) return PNE_EWORKSPACE;
    Exec ex;
    ex.st = (hipStream_t)stream;
    zero_i32(ex, 1, dinfo);
    copy_f64(ex, n, n, dR, ldr, b.R, n);
    run_gram(ex, p, dA, db, b);
    if (factor) run_factor(ex, p, b, dinfo);
    copy_f64(ex, n, n, b.C, n, dC, ldc);
    copy_f64(ex, n, 1, b.c, n, dc, n);
    if (factor && hpne) copy_i32(ex, n, b.piv, dpiv);
    return hipGetLastError() == hipSuccess ? PNE_OK : PNE_EHIP;
}

size_t pne_batched_workspace_size(int64_t batch, const pne_problem_desc* hdesc, const pne_opts* o, int hpne)
{
    if (check_batch(batch, hdesc, o, hpne) != PNE_OK) return 0;
    TuneScope scope(batch_tune(batch, hdesc, o, hpne));
    return batched_size(batch, hdesc, o, hpne);
}

pne_status pne_batch_plan_create(int64_t batch, const pne_problem_desc* hdesc, const double* dA_base,
                                 const double* db_base, double* dx_base, const pne_opts* o, int hpne, void* dwork,
                                 size_t work_bytes, int32_t* dinfo, pne_stream_t stream, pne_batch_plan* plan)
{
    if (!plan) return PNE_EINVAL;
    *plan = nullptr;
    pne_status chk = check_batch(batch, hdesc, o, hpne);
    if (chk) return chk;
    return plan_create(batch, hdesc, dA_base, db_base, dx_base, o, hpne, dwork, work_bytes, dinfo,
                       (hipStream_t)stream, batch_tune(batch, hdesc, o, hpne), plan);
}

pne_status pne_batch_plan_execute(pne_batch_plan plan, pne_stream_t stream)
{
    if (!plan) return PNE_EINVAL;
    return plan_execute(plan, (hipStream_t)stream, plan->rerun_ce);
}

pne_status pne_batch_plan_execute_graph(pne_batch_plan plan, pne_stream_t stream)
{
    if (!plan || !stream) return PNE_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    if (!plan->gexec) {
        hipGraph_t g = nullptr;
        HIP_OK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
        pne_status rc = plan_execute(plan, st, plan->rerun_ce);
        const hipError_t e = hipStreamEndCapture(st, &g);
        if (rc) {
            if (g) (void)hipGraphDestroy(g);
            return rc;
        }
        if (e != hipSuccess || !g) return PNE_EHIP;
        const hipError_t ei = hipGraphInstantiate(&plan->gexec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (ei != hipSuccess) {
            plan->gexec = nullptr;
            return PNE_EHIP;
        }
    }
    HIP_OK(hipGraphLaunch(plan->gexec, st));
    return PNE_OK;
}

void pne_batch_plan_destroy(pne_batch_plan plan) { delete plan; }

// Candidate settings of the autotuner: the batch row chunk, the tile of the
// short-K products (A R^-1, factor updates) and the order up to which
// lower-triangle long-K products (the Gram matrices) use 64 x 64 tiles.
static std::vector<TuneParams> tune_candidates()
{
    std::vector<TuneParams> c;
    for (int64_t kc : {4096, 8192, 16384})
        for (int st : {64, 128})
            for (int ln : {512, 1024})
                for (int pe : {0, 1}) {
                    TuneParams p;
                    p.batch_kchunk = kc;
                    p.shortk_tile = st;
                    p.lower_small_n = ln;
                    p.persistent = pe;
                    c.push_back(p);
                }
    return c;
}

size_t pne_autotune_batched_workspace_size(int64_t batch, const pne_problem_desc* hdesc, const pne_opts* o,
                                           int hpne)
{
    if (check_batch(batch, hdesc, o, hpne) != PNE_OK) return 0;
    size_t best = 0;
    for (const TuneParams& p : tune_candidates()) {
        TuneScope scope(p);
        const size_t b = batched_size(batch, hdesc, o, hpne);
        if (b == 0) return 0;
        if (b > best) best = b;
    }
    return best;
}

pne_status pne_autotune_batched(int64_t batch, const pne_problem_desc* hdesc, const double* dA_base,
                                const double* db_base, double* dx_base, const pne_opts* o, int hpne, void* dwork,
                                size_t work_bytes, int32_t* dinfo, pne_stream_t stream, pne_tune_result* result)
{
    pne_status chk = check_batch(batch, hdesc, o, hpne);
    if (chk) return chk;
    if (!dA_base || !db_base || !dx_base || !dinfo || !dwork) return PNE_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    hipEvent_t e0, e1;
    HIP_OK(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return PNE_EHIP;
    }
    TuneParams best;
    double best_ms = -1.0;
    pne_status rc = PNE_OK;
    for (const TuneParams& p : tune_candidates()) {
        pne_batch_plan_s* plan = nullptr;
        rc = plan_create(batch, hdesc, dA_base, db_base, dx_base, o, hpne, dwork, work_bytes, dinfo, st, p, &plan);
        if (rc == PNE_EWORKSPACE) { rc = PNE_OK; continue; }   // needs more than the caller gave
        if (rc) break;
        // one warm-up execution, then the median of three timed ones
        rc = plan_execute(plan, st, plan->rerun_ce);
        double t[3] = {0, 0, 0};
        for (int k = 0; k < 3 && !rc; ++k) {
            if (hipEventRecord(e0, st) != hipSuccess) { rc = PNE_EHIP; break; }
            rc = plan_execute(plan, st, plan->rerun_ce);
            if (rc) break;
            float ms = 0.0f;
            if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&ms, e0, e1) != hipSuccess) { rc = PNE_EHIP; break; }
            t[k] = ms;
        }
        delete plan;
        if (rc) break;
        if (t[0] > t[1]) { double x = t[0]; t[0] = t[1]; t[1] = x; }
        if (t[1] > t[2]) { double x = t[1]; t[1] = t[2]; t[2] = x; }
        if (t[0] > t[1]) { double x = t[0]; t[0] = t[1]; t[1] = x; }
        if (best_ms < 0.0 || t[1] < best_ms) { best_ms = t[1]; best = p; }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    if (best_ms < 0.0) return PNE_EWORKSPACE;
    double sn = 0.0, sm = 0.0;
    for (int64_t i = 0; i < batch; ++i) { sn += (double)hdesc[i].n; sm += (double)hdesc[i].m; }
    const bool stored = tune_store(tune_key_batched(hpne, o->sketch_prec, o->qr_prec, batch, sn / batch, sm / batch),
                                   best, best_ms);
    if (result) {
        result->batch_kchunk = best.batch_kchunk;
        result->shortk_tile = best.shortk_tile;
        result->lower_small_n = best.lower_small_n;
        result->persistent = best.persistent;
        result->ms = best_ms;
        result->stored = stored ? 1 : 0;
    }
    return PNE_OK;
}

pne_status pne_solve_batched(int64_t batch, const pne_problem_desc* hdesc, const double* dA_base,
                             const double* db_base, double* dx_base, const pne_opts* o, int hpne,
                             void* dwork, size_t work_bytes, int32_t* dinfo, pne_stream_t stream)
{
    return solve_batched(batch, hdesc, dA_base, db_base, dx_base, o, hpne, dwork, work_bytes, dinfo,
                         (hipStream_t)stream);
}

}  // extern "C"
