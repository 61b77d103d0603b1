/*
 * pne.h -- C ABI of the MI355X (gfx950) library for tall least-squares
 * problems  min_x ||A x - b||_2,  A m x n with rank n, m >> n,  solved by the
 * randomized preconditioned normal equations of Garrison & Ipsen,
 * "Perturbation Analysis for Preconditioned Normal Equations in Mixed
 * Precision" (arXiv 2603.16644):
 *
 *   PNE  (Section 1, eq. e_pne):  A_p^T A_p y = A_p^T b,  R_s x = y
 *   HPNE (Section 1, eq. e_hpne): A_p^T A x = A_p^T b
 *   with A_p = A R_s^{-1} and R_s the triangular factor of a sketch
 *   Omega A (Algorithm 1; Section 6.2), computed in a lower precision.
 *
 * Common conventions for every entry point.
 *   - All matrices are column-major with a leading dimension (LAPACK); A has
 *     lda >= m.  All array arguments named d* are device pointers on the
 *     current HIP device, owned by the caller; the library never frees or
 *     keeps them.  A and b are read only; outputs are overwritten.
 *   - The library allocates no device memory during a call.  Scratch space
 *     comes from the caller as dwork/work_bytes (device memory, any
 *     contents, 256-byte aligned); query its size with the *_workspace_size
 *     function of the entry point.  Workspace contents are undefined after a
 *     call.  Two calls that share a workspace must be ordered on one stream.
 *   - All device work is enqueued on `stream` and is asynchronous, except
 *     where stated (AUTO precision reads the condition estimate back to pick
 *     kernels, which synchronises the stream once).
 *   - Argument errors (n < 1, m < n, s < n, lda < m, null pointers, workspace
 *     too small, unsupported option) are detected on the host before any
 *     device work and returned as a negative pne_status; nothing is enqueued.
 *   - Numerical failures are reported asynchronously in the device word
 *     *dinfo (LAPACK style): 0 success; 1000+k: R_s(k,k) == 0; 2000+k:
 *     Cholesky of the PNE matrix broke down at column k; 3000+k: zero or
 *     non-finite pivot in the LU of the HPNE matrix at column k (k 1-based);
 *     4000+k: a block of the parallel triangular solves gave up waiting for
 *     block k (a scheduling failure; the result is invalid); 5000: A or b
 *     holds a non-finite entry (only with pne_opts.check_finite, see there).  R_s(k,k) counts
 *     as zero when it is not finite.  On failure x is filled with NaN; no
 *     silent fallback to another precision is taken.
 *   - Same inputs and options give bitwise identical results (every
 *     reduction has a fixed order; no floating-point atomics).
 */
#ifndef PNE_H
#define PNE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t* pne_stream_t; /* a hipStream_t; NULL = default stream */

typedef enum {
    PNE_OK = 0,
    PNE_EINVAL = -1,     /* invalid argument                          */
    PNE_ENOMEM = -2,     /* host allocation failed                    */
    PNE_EHIP = -3,       /* a HIP runtime call failed                 */
    PNE_EWORKSPACE = -4, /* work_bytes smaller than the queried size  */
    PNE_ENOTSUP = -5     /* option combination not supported          */
} pne_status;

/* Arithmetic of the preconditioner (Algorithm 1, "precision u_p"). */
typedef enum {
    PNE_PREC_AUTO = 0,     /* pick by the FP32 condition estimate (Section 6.1)  */
    PNE_PREC_FP64 = 1,
    PNE_PREC_FP32 = 2,
    PNE_PREC_FP16 = 3,     /* FP16 operands, per-block power-of-two scales of A   */
    PNE_PREC_BF16 = 4,
    PNE_PREC_FP8E4M3 = 5   /* OCP e4m3 operands, per-block FP32 scales of A       */
} pne_prec;

typedef struct {
    int64_t s;              /* sketch rows; 0 selects 3n (Section 6.2 uses d = 3n)       */
    uint64_t seed;          /* key of the counter-based Gaussian sketch                  */
    uint32_t problem_id;    /* third counter word of the sketch (batch member index)     */
    int32_t sketch_prec;    /* pne_prec of the sketch Omega A                            */
    int32_t qr_prec;        /* pne_prec of the QR of the sketch (FP8 not allowed)        */
    double known_kappa;     /* > 0: skip the estimate, pick from log10(known_kappa)      */
    int32_t refine_steps;   /* FP64 residual corrections after the solve (default 1)     */
    int32_t block_rows;     /* rows per scale block for FP16/FP8 sketches (128; mult. of 64) */
    int32_t cond_method;    /* AUTO estimate: 0 = FP32 Gram (Section 6.1, default);
                               1 = FP32 QR of the FP32 sketch (see cond_est_qr)              */
    int32_t sketch_kind;    /* 0 = Gaussian (default); 1 = SRFT, the subsampled randomized
                               trigonometric transform of Section 6.2 (see pne_sketch_srft);
                               with SRFT an FP16 sketch precision runs as FP32, FP8 is not
                               supported                                                    */
    int32_t check_finite;   /* nonzero: scan A (its m x n entries) and b for NaN or
                               infinity before anything else is enqueued; if one is
                               found the call writes 5000 to *dinfo and returns
                               PNE_EINVAL without solving (batched calls: per member,
                               PNE_EINVAL if any member fails).  The scan is read back,
                               so the call then synchronises its stream once; not for
                               use under stream capture.  Default 0.                    */
} pne_opts;

typedef struct {
    int32_t sketch_prec_used; /* precision actually used (AUTO resolved)  */
    int32_t qr_prec_used;
    float kappa0;             /* (1/2) log10(||G||_1 est ||G^-1||_1), G = fl32(A^T A); NaN if not estimated */
    int32_t refine_steps_run;
} pne_info;

/* Fills *opts with the defaults: s = 0 (3n), seed = 0, problem_id = 0,
 * sketch_prec = qr_prec = AUTO, known_kappa = 0, refine_steps = 1,
 * block_rows = 128, cond_method = 0, sketch_kind = 0, check_finite = 0. */
void pne_default_opts(pne_opts* opts);

/* Bytes of workspace pne_solve (hpne = 0) or hpne_solve (hpne = 1) needs for
 * an m x n problem with these options.  Returns 0 on invalid arguments. */
size_t pne_workspace_size(int64_t m, int64_t n, const pne_opts* opts, int hpne);

/* pne_solve: Algorithm 1 with the PNE (Section 1, eq. e_pne; Section 3).
 *   1. [AUTO] condition estimate and precision pick (see cond_est);
 *   2. A_s = Omega A, Omega s x m with N(0, 1/s) entries generated on the fly
 *      from (seed, problem_id, row, column) (Algorithm 1 "Sketch");
 *   3. Householder QR of A_s in qr_prec, R_s promoted to FP64;
 *   4. A_p = A R_s^{-1} (FP64, blocked substitution);
 *   5. C = A_p^T A_p, c = A_p^T b (FP64);
 *   6. Cholesky C = L L^T, L L^T y = c, R_s x = y (FP64);
 *   7. refine_steps corrections: r = b - A x, solve the same system with
 *      right-hand side A_p^T r, x += correction (FP64).
 * dA: m x n (lda); db: m; dx: n (output).  dinfo: one device int32.
 * hinfo (host, may be NULL) receives the precisions used; with AUTO the
 * call synchronises the stream once and fills kappa0.  */
pne_status pne_solve(int64_t m, int64_t n, const double* dA, int64_t lda, const double* db,
                     double* dx, const pne_opts* opts, void* dwork, size_t work_bytes,
                     int32_t* dinfo, pne_info* hinfo, pne_stream_t stream);

/* hpne_solve: Algorithm 1 with the HPNE (Section 1, eq. e_hpne; Section 4):
 * steps 1-4 as pne_solve, then C = A_p^T A, c = A_p^T b, LU with partial
 * pivoting (first index of largest magnitude on ties) P C = L U, and
 * L U x = P c; refinement as in pne_solve with the LU factors.
 * Same arguments as pne_solve. */
pne_status hpne_solve(int64_t m, int64_t n, const double* dA, int64_t lda, const double* db,
                      double* dx, const pne_opts* opts, void* dwork, size_t work_bytes,
                      int32_t* dinfo, pne_info* hinfo, pne_stream_t stream);

/* sketch_precond: the preconditioner alone (Algorithm 1 steps "Sketch",
 * "Thin QR", "Promote R_s"; Section 6.2).  Writes the upper triangle of the
 * n x n FP64 matrix R_s into dR (ldr >= n); the strict lower triangle is set
 * to zero.  Workspace: sketch_precond_workspace_size. */
size_t sketch_precond_workspace_size(int64_t m, int64_t n, const pne_opts* opts);
pne_status sketch_precond(int64_t m, int64_t n, const double* dA, int64_t lda, const pne_opts* opts,
                          double* dR, int64_t ldr, void* dwork, size_t work_bytes, int32_t* dinfo,
                          pne_info* hinfo, pne_stream_t stream);

/* cond_est: the single-precision condition estimate of Section 6.1 and the
 * precision pick of Algorithm 1.  G = fl32(A)^T fl32(A) (FP32), FP32
 * Cholesky, Hager's 1-norm estimate of ||G^{-1}||_1 (at most five
 * iterations), kappa0 = (1/2) log10(||G||_1 est) written to *dkappa0 (device
 * float; +inf when the Cholesky breaks down, i.e. the estimate overflows);
 * *dchoice (device int32) = PNE_PREC_FP16 if kappa0 < 4, PNE_PREC_FP32 if
 * kappa0 <= 8, else PNE_PREC_FP64.  Workspace: cond_est_workspace_size. */
size_t cond_est_workspace_size(int64_t m, int64_t n);
pne_status cond_est(int64_t m, int64_t n, const double* dA, int64_t lda, float* dkappa0,
                    int32_t* dchoice, void* dwork, size_t work_bytes, pne_stream_t stream);

/* cond_est_qr: a condition estimate that does not square kappa(A) (a
 * library variant of the single-precision estimate of Section 6.1, for the
 * single-precision band of Algorithm 1 that the FP32 Gram estimate cannot
 * reach beyond kappa ~ 4e3).  A_s = Omega A with the FP32 sketch (s rows, 0
 * selects 3n; Omega as in pne_solve with problem_id 0), FP32 Householder QR
 * A_s = Q R, Hager's estimate of ||R^{-1}||_1 (at most five iterations),
 * kappa0 = log10(||R||_1 est) to *dkappa0 (+inf when a diagonal entry of R
 * is zero or not finite); *dchoice by the thresholds of cond_est.  kappa(A_s)
 * is within the condition number of the sketched orthonormal basis (< 3.73
 * for s = 3n) of kappa(A).  pne_opts.cond_method = 1 makes AUTO use this
 * estimate; when it picks FP32 for both steps, its R is the preconditioner
 * (the FP32 sketch and QR are not repeated).
 * Workspace: cond_est_qr_workspace_size. */
size_t cond_est_qr_workspace_size(int64_t m, int64_t n, int64_t s);
pne_status cond_est_qr(int64_t m, int64_t n, const double* dA, int64_t lda, int64_t s, uint64_t seed,
                       float* dkappa0, int32_t* dchoice, void* dwork, size_t work_bytes, pne_stream_t stream);

/* nne_solve: the not-normal equations B^T A x = B^T b (Section 5.2, eq.
 * e_nne) for a caller-supplied B (m x n, ldb >= m, rank n, with the column
 * space of A; then x is the least-squares solution).  C = B^T A and
 * c = B^T b (FP64), LU with partial pivoting (first index of the largest
 * magnitude), L U x = P c; then refine_steps FP64 corrections r = b - A x,
 * d from B^T A d = B^T r (same LU), x += d.  The HPNE is the case B = A_p.
 * dA, dB: m x n; db: m; dx: n (output); dinfo: one device int32 (3000+k on a
 * zero or non-finite pivot; x is then NaN).  Workspace: nne_workspace_size. */
size_t nne_workspace_size(int64_t m, int64_t n);
pne_status nne_solve(int64_t m, int64_t n, const double* dA, int64_t lda, const double* dB, int64_t ldb,
                     const double* db, double* dx, int32_t refine_steps, void* dwork, size_t work_bytes,
                     int32_t* dinfo, pne_stream_t stream);

/* qr_ls_solve: least squares by FP64 Householder QR on the GPU -- the
 * direct QR solver the paper measures PNE/HPNE against (Section 7.4), with
 * Q never formed: the QR of the augmented matrix [A b] = Q [R_A c; 0 rho]
 * gives x = R_A^{-1} c.  The tall QR is a tree of blocked Householder QRs
 * (TSQR): row blocks of at most 6144 rows are factored together, then groups
 * of their stacked R factors, until one R remains.  n <= 3070.  dA: m x n
 * (lda >= m); db: m; dx: n (output); dinfo: one device int32 (1000+k for a
 * zero or non-finite R_A(k,k); x is then NaN).  Uploads one launch table per
 * tree level (one wait each).  Workspace: qr_ls_workspace_size. */
size_t qr_ls_workspace_size(int64_t m, int64_t n);
pne_status qr_ls_solve(int64_t m, int64_t n, const double* dA, int64_t lda, const double* db, double* dx,
                       void* dwork, size_t work_bytes, int32_t* dinfo, pne_stream_t stream);

/* pne_sketch: the sketch step alone, A_s = Omega A (s x n, FP64 output,
 * ldas >= s) in precision `prec` (FP64, FP32, FP16, BF16, FP8E4M3), with the
 * operand rounding the solvers use.  Omega as in pne_solve.
 * Workspace: pne_sketch_workspace_size. */
size_t pne_sketch_workspace_size(int64_t m, int64_t n, int64_t s, int32_t prec);
pne_status pne_sketch(int64_t m, int64_t n, const double* dA, int64_t lda, int64_t s, uint64_t seed,
                      uint32_t problem_id, int32_t prec, int32_t block_rows, double* dAs,
                      int64_t ldas, void* dwork, size_t work_bytes, pne_stream_t stream);

/* pne_sketch_srft: the SRFT sketch alone (Section 6.2, eq. e_sketch,
 * Omega = S F D, with the real Hartley transform H = Re(F) - Im(F) as F):
 * A_s = (1/sqrt(s)) S H D A, H of length m' = the smallest 7-smooth integer
 * >= m (A padded with zero rows), D = diag(+-1) (bit j mod 128 of Philox at
 * counter (j/128, 0, problem_id, 3)), S = s rows of I_m' sampled uniformly
 * with replacement (k_i = floor(w m' / 2^64), w = the first two Philox words
 * at counter (i, 0, problem_id, 2)); key = seed.  Computed by a mixed-radix
 * FFT (radices 2..32) of paired columns, the last pass evaluated only at the
 * sampled rows; arithmetic FP64 (prec FP64) or FP32 (FP32, or BF16 operands).
 * dAs: s x n FP64 (ldas >= s).  Workspace: pne_sketch_srft_workspace_size. */
size_t pne_sketch_srft_workspace_size(int64_t m, int64_t n, int32_t prec);
pne_status pne_sketch_srft(int64_t m, int64_t n, const double* dA, int64_t lda, int64_t s, uint64_t seed,
                           uint32_t problem_id, int32_t prec, double* dAs, int64_t ldas, void* dwork,
                           size_t work_bytes, pne_stream_t stream);

/* Batched PNE/HPNE (many independent problems in one call).
 * Problem i is A_i (m_i x n_i, lda_i) at dA_base + a_offset_i doubles, b_i at
 * db_base + b_offset_i, x_i written at dx_base + x_offset_i.  All problems
 * share the options except the sketch counter word: member i draws its
 * sketch with problem_id_i (opts->problem_id is ignored).  dinfo has
 * `batch` device int32 words.  hdesc is a host array. */
typedef struct {
    int64_t m, n, lda;
    int64_t a_offset, b_offset, x_offset;
    int64_t problem_id;   /* third counter word of member i's sketch (0 .. 2^32 - 1) */
} pne_problem_desc;

size_t pne_batched_workspace_size(int64_t batch, const pne_problem_desc* hdesc,
                                  const pne_opts* opts, int hpne);
pne_status pne_solve_batched(int64_t batch, const pne_problem_desc* hdesc, const double* dA_base,
                             const double* db_base, double* dx_base, const pne_opts* opts,
                             int hpne, void* dwork, size_t work_bytes, int32_t* dinfo,
                             pne_stream_t stream);

/* Batch plans: a batched solve prepared once and executed many times.
 * pne_batch_plan_create checks the arguments, resolves AUTO precisions (the
 * condition estimate runs once on the data present; the picks stay fixed
 * for the plan's life), records the grouped launch sequence under the tuned
 * parameters of the workload (see pne_autotune_batched) and uploads its
 * launch tables into dwork (one wait for the upload).  The workspace, A, b,
 * x and dinfo of the create call are bound to the plan: they must stay
 * allocated, and the plan may only be executed on data of the same shapes
 * at the same addresses.  Workspace size: pne_batched_workspace_size.
 * pne_batch_plan_execute enqueues the solve on `stream` -- kernel launches
 * only (the info words are cleared by a kernel), no copies, no host waits,
 * so it can be captured into a hipGraph by the caller.
 * pne_batch_plan_execute_graph captures the same sequence into a hipGraph
 * on its first call (stream must not be NULL, the legacy default stream
 * cannot be captured) and launches the instantiated graph on this and every
 * later call.  Executions of one plan must be ordered on one stream.  Results
 * are bitwise identical between executions, graph or not. */
typedef struct pne_batch_plan_s* pne_batch_plan;
pne_status pne_batch_plan_create(int64_t batch, const pne_problem_desc* hdesc, const double* dA_base,
                                 const double* db_base, double* dx_base, const pne_opts* opts, int hpne,
                                 void* dwork, size_t work_bytes, int32_t* dinfo, pne_stream_t stream,
                                 pne_batch_plan* plan);
pne_status pne_batch_plan_execute(pne_batch_plan plan, pne_stream_t stream);
pne_status pne_batch_plan_execute_graph(pne_batch_plan plan, pne_stream_t stream);
void pne_batch_plan_destroy(pne_batch_plan plan);

/* Autotuner of the batched path.  Times candidate launch parameters on the
 * caller's batch (a plan per candidate; one warm-up and the median of three
 * executions, HIP events on `stream`): the row chunk of the split-K products
 * of a batch (4096, 8192, 16384), the output tile of the short-K products
 * (64 or 128) and the largest order of the Gram products that use 64 x 64
 * tiles (512 or 1024).  The fastest is written to *result and, when the
 * environment variable PNE_TUNE_CACHE names a file, stored there (JSON)
 * under a key of (solver, sketch and QR precision options, power-of-two
 * buckets of the member count, mean n and mean m); pne_batched_workspace_size,
 * pne_solve_batched and pne_batch_plan_create read the entry back for
 * workloads with the same key.  x and dinfo hold the results of the last
 * candidate's last execution.  Workspace: at least
 * pne_autotune_batched_workspace_size (candidates that need more than
 * work_bytes are skipped). */
typedef struct {
    int64_t batch_kchunk;
    int32_t shortk_tile;
    int32_t lower_small_n;
    double ms;        /* median time of one execution with these parameters */
    int32_t stored;   /* 1 if written to the cache file */
    int32_t persistent; /* 1: the grouped MFMA products run as persistent
                           launches (work-groups taking tiles from a counter) */
} pne_tune_result;
size_t pne_autotune_batched_workspace_size(int64_t batch, const pne_problem_desc* hdesc, const pne_opts* opts,
                                           int hpne);
pne_status pne_autotune_batched(int64_t batch, const pne_problem_desc* hdesc, const double* dA_base,
                                const double* db_base, double* dx_base, const pne_opts* opts, int hpne,
                                void* dwork, size_t work_bytes, int32_t* dinfo, pne_stream_t stream,
                                pne_tune_result* result);

/* pne_gram: the normal-equation matrices of the solvers for a given
 * preconditioner (diagnostics and kernel-level checks).  With R (n x n,
 * upper triangle read, ldr >= n, FP64): A_p = A R^{-1} (Algorithm 1, "Solve
 * A_p"); C = A_p^T A_p (hpne = 0, eq. e_pne; only the lower triangle of C is
 * defined) or C = A_p^T A (hpne = 1, eq. e_hpne); c = A_p^T b.  With
 * factor != 0, C is then factored in place as the solvers do: the Cholesky
 * factor L in the lower triangle (PNE), or P C = L U with unit lower L below
 * the diagonal, U on and above it and the 0-based pivot rows in dpiv[n]
 * (HPNE; LAPACK ordering).  dC: n x n (ldc >= n); dc: n; dinfo: one device
 * int32 (2000+k / 3000+k on a breakdown, as the solvers).  Workspace:
 * pne_gram_workspace_size. */
size_t pne_gram_workspace_size(int64_t m, int64_t n, int hpne);
pne_status pne_gram(int64_t m, int64_t n, const double* dA, int64_t lda, const double* db, const double* dR,
                    int64_t ldr, int hpne, int factor, double* dC, int64_t ldc, double* dc, int32_t* dpiv,
                    void* dwork, size_t work_bytes, int32_t* dinfo, pne_stream_t stream);

/* Phase timing (diagnostics).  pne_profile_enable(1) makes every following
 * solve record a HIP event on its stream after each phase of the pipeline
 * (condition estimate, sketch generation / quantisation / product /
 * reduction, QR, A R_s^{-1}, Gram product, Gram reduction, factorization,
 * solves, refinement).  Recording never synchronises.  pne_profile_read
 * waits for the events of the most recent solve and writes the duration of
 * phase i (milliseconds, -1 if the phase did not run) to ms[i] for
 * i < max_phases; it returns the number of phases written (or a negative
 * pne_status).  pne_profile_phase_name(i) names phase i.  Not thread safe;
 * meant for benchmarks and tests on one stream. */
int pne_profile_enable(int enable);
int pne_profile_read(double* ms, int max_phases);
const char* pne_profile_phase_name(int i);

/* pne_solve_noalloc: pne_solve (hpne = 0) or hpne_solve (hpne = 1) for
 * callers that cannot allocate device memory -- code under stream capture,
 * tight serving loops, harnesses that forbid hipMalloc.  Same arguments,
 * kernels and results as those entry points, except that there is no dwork:
 * the scratch space is one file-scope device array of PNE_NOALLOC_MAX_BYTES
 * per GPU, which the library holds until the process ends.  Its address is
 * looked up once per device on that device's first call.  A problem whose
 * pne_workspace_size exceeds PNE_NOALLOC_MAX_BYTES returns PNE_EWORKSPACE
 * before any device work.  The call itself allocates nothing (no hipMalloc,
 * hipFree or allocating library routine).  All calls on one GPU share the
 * array: two calls that overlap in time on one GPU (different streams or
 * host threads without ordering) race and give undefined results; order
 * them on one stream.  AUTO precision synchronises the stream once, as in
 * pne_solve. */
#define PNE_NOALLOC_MAX_BYTES ((size_t)64 << 20)
size_t pne_noalloc_max_bytes(void);
pne_status pne_solve_noalloc(int64_t m, int64_t n, const double* dA, int64_t lda, const double* db,
                             double* dx, const pne_opts* opts, int hpne, int32_t* dinfo, pne_info* hinfo,
                             pne_stream_t stream);

/* Human-readable name of a status code (static string). */
const char* pne_status_string(pne_status st);

#ifdef __cplusplus
}
#endif
#endif /* PNE_H */
