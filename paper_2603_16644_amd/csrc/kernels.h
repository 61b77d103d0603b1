// Internal host-side interfaces between the kernel files and the C ABI layer.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.h"
#include "launch.h"

namespace pne {

// Operand kinds of the sketch product.
enum { OPK_F64 = 0, OPK_F32 = 1, OPK_BF16 = 2, OPK_F16 = 3, OPK_FP8 = 4 };

inline int prec_to_opk(int prec)
{
    switch (prec) {
    case PNE_PREC_FP64: return OPK_F64;
    case PNE_PREC_FP32: return OPK_F32;
    case PNE_PREC_BF16: return OPK_BF16;
    case PNE_PREC_FP16: return OPK_F16;
    default: return OPK_FP8;
    }
}
inline int64_t opk_bytes(int op)
{
    switch (op) {
    case OPK_F64: return 8;
    case OPK_F32: return 4;
    case OPK_BF16:
    case OPK_F16: return 2;
    default: return 1;
    }
}

// ---------------------------------------------------------------- sketch
struct SketchPlan {
    int op;
    int64_t chunk, nchunks, ldk, splits, kchunk;
    int wide;       // 256 x 256 product tiles (one large unscaled sketch)
    size_t bytes;
};
// kchunk_fixed > 0: split the product over rows of A in chunks of this
// length (batches) instead of filling the machine with one sketch
SketchPlan plan_sketch(int64_t m, int64_t n, int64_t s, int prec, int64_t br, int64_t kchunk_fixed = 0);
size_t sketch_workspace_bytes(int64_t m, int64_t n, int64_t s, int prec, int64_t br,
                              int64_t kchunk_fixed = 0);
int sketch_run(Exec& ex, int64_t m, int64_t n, const double* A, int64_t lda, int64_t s, uint64_t seed,
               uint32_t pid, int prec, int64_t br, float* As32, int64_t ld32, double* As64,
               int64_t ld64, void* work, size_t work_bytes);

// SRFT sketch (srft.hip): A_s = (1/sqrt(s)) S H D A with the Hartley
// transform of length srft_padded_length(m); precisions FP64, FP32, BF16.
int64_t srft_padded_length(int64_t m);
bool srft_supported(int prec);
size_t srft_workspace_bytes(int64_t m, int64_t n, int prec);
int srft_run(Exec& ex, int64_t m, int64_t n, const double* A, int64_t lda, int64_t s, uint64_t seed, uint32_t pid,
             int prec, float* As32, int64_t ld32, double* As64, int64_t ld64, void* work, size_t work_bytes);

// ---------------------------------------------------------------- GEMM
// Column-major C = alpha op(A) op(B) + beta Cin (C may alias Cin).
// With splits > 1 the raw products go to partial buffers P[z] (M x N, ld M)
// and gemm_reduce_* forms C.  `lower` restricts work to output tiles on or
// below the diagonal (square tiles).  With bvec != null the
// work-groups of the first tile column also form op(A) bvec into Pc[z]
// (n-vector partials), reduced into cvec.
struct GemmArgs {
    int64_t M, N, K;
    const void* A; int64_t lda; int transA;
    const void* B; int64_t ldb; int transB;
    double alpha, beta;
    const void* Cin; int64_t ldcin;
    void* C; int64_t ldc;
    int lower;
    int64_t splits, kchunk;
    void* P; int accumulate_partials;
    const void* bvec; void* Pc; void* cvec;
    int xcd_remap;    // set by the launcher (direct split-K lower-triangle launches)
    // lower-triangle split-K only: the diagonal tiles cut K into splits_diag
    // chunks of kchunk_diag (0: as the other tiles); see plan_splitk_gram
    int64_t splits_diag, kchunk_diag;
    int diag_roles;   // set by the launcher: split the diagonal tiles' work over all wavefronts
};
// element types: d = double, f = float; "ddf" = A, B stored double, computed in float
void gemm_f64(Exec& ex, const GemmArgs& g);           // full path incl. reduce
void gemm_f64_partials(Exec& ex, const GemmArgs& g);  // partials only (no reduce)
void gemm_f64_reduce(Exec& ex, const GemmArgs& g);    // reduce of the partials
void gemm_f32(Exec& ex, const GemmArgs& g);
void gemm_f32_partials(Exec& ex, const GemmArgs& g);
void gemm_ddf(Exec& ex, const GemmArgs& g);           // fl32(A)^T fl32(B) etc.
// split-K plan: splits and kchunk for a long-K product with `tiles` output
// tiles (kchunk_fixed > 0: fixed chunk length, for batches)
void plan_splitk(int64_t K, int64_t tiles, int64_t* splits, int64_t* kchunk, int64_t kchunk_fixed = 0);
int64_t gemm_tiles(int64_t M, int64_t N, int64_t K, int lower);
// split-K plan of the FP64 Gram product (n x n, K = m; lower-triangle tiles
// when `lower`): plan_splitk, or for lower triangles in 128 x 128 tiles a
// separate split of the diagonal tiles (whose wavefronts carry less MFMA
// work) when that shortens the largest work-group.  Partial buffers hold
// max(splits, splits_diag) slices.
void plan_splitk_gram(int64_t K, int64_t n, int lower, int64_t kchunk_fixed, int64_t* splits, int64_t* kchunk,
                      int64_t* splits_diag, int64_t* kchunk_diag);

// ---------------------------------------------------------------- TRSM / factorizations
// Ap = A R^{-1}, R upper n x n (FP64), blocked substitution.
void trsm_right_upper(Exec& ex, int64_t m, int64_t n, const double* A, int64_t lda, const double* R,
                      int64_t ldr, double* Ap, int64_t ldap);
// row-parallel substitution on a block of <= 64 columns: X := X R^{-1}
// (R upper, TL = false) or X := X L^{-T} (L lower, TL = true); element
// (i, c) of X at X[i*rs + c*cs]; UNIT: unit diagonal.  With Xin the input is
// read from Xin[i*rs + c*cs_in] (X is then output only).
template <typename T, bool TL, bool UNIT>
void trsm_leaf(Exec& ex, int64_t m, int w, T* X, int64_t rs, int64_t cs, const T* Rb, int64_t ldr,
               const T* Xin = nullptr, int64_t cs_in = 0);
// Cholesky (lower, in place) of the n x n matrix C; info word gets 2000+k.
// Dinv (dinv_elems(n) values) receives the inverses of the 64 x 64 diagonal
// blocks of L in the layout of inv_diag_blocks.
template <typename T>
void cholesky(Exec& ex, int64_t n, T* C, int64_t ldc, int32_t* info, T* Dinv);
// LU with partial pivoting in place; piv 0-based; info 3000+k.
void lu_factor(Exec& ex, int64_t n, double* C, int64_t ldc, int32_t* piv, int32_t* info);
// Householder QR (R only) of the s x n matrix W (in place); R (FP64, n x n,
// upper, ldr) rounded to qr_prec; info 1000+k for a zero diagonal.
size_t qr_workspace_bytes(int64_t s, int64_t n, int prec);
int qr_r(Exec& ex, int64_t s, int64_t n, void* W, int64_t ldw, int prec, double* R, int64_t ldr,
         int32_t* info, void* work, size_t work_bytes);
bool qr_supported(int64_t s, int prec);

// ---------------------------------------------------------------- vectors
// inverses of the 64 x 64 diagonal blocks of op(M) (dinv_elems(n) values);
// blocks block0 .. block0 + nblocks - 1 (nblocks < 0: to the end)
size_t dinv_elems(int64_t n);
template <typename T>
void inv_diag_blocks(Exec& ex, int64_t n, const T* M, int64_t ld, int lower, int trans, int unit, T* Dinv,
                     int64_t block0 = 0, int64_t nblocks = -1);
// x = R^{-1} L^{-T} L^{-1} c (PNE: Cholesky factor L, preconditioner R, with
// L^T stored explicitly as Lt) and x = U^{-1} L^{-1} P c (HPNE: LU with unit
// lower L), with the inverses DL, DLt, DR, DU of the 64 x 64 diagonal blocks;
// one work-group per 64-row block and per-block flags (flags: 3 *
// lb_flag_words(n) int32 for the PNE solve, 2 * ... for the LU solve; any
// contents on entry).  c and x may alias.  A wait between blocks that gives
// up writes 4000 + block + 1 to *info (if still zero; info may be null).
size_t lb_flag_words(int64_t n);
void pne_solve_lb(Exec& ex, int64_t n, const double* L, int64_t ldl, const double* DL, const double* Lt,
                  const double* DLt, const double* R, int64_t ldr, const double* DR, const double* c, double* x,
                  double* y, int32_t* flags, int32_t* info);   // y: n-vector scratch (L^T y = z)
void lu_solve_lb(Exec& ex, int64_t n, const double* LU, int64_t ld, const int32_t* piv, const double* DL,
                 const double* DU, const double* c, double* x, int32_t* flags, int32_t* info);
// x = U^{-1} c (U upper, DU the inverses of its 64 x 64 diagonal blocks);
// flags: lb_flag_words(n) int32; c and x may alias.
void upper_solve_lb(Exec& ex, int64_t n, const double* U, int64_t ld, const double* DU, const double* c, double* x,
                    int32_t* flags, int32_t* info);
// *info = 1000 + k + 1 for the first zero or non-finite R(k, k) (if still 0)
void check_r_diag(Exec& ex, int64_t n, const double* R, int64_t ldr, int32_t* info);
// out (c x r, ldo) = in^T (in r x c, ldi)
void transpose_f64(Exec& ex, int64_t r, int64_t c, const double* in, int64_t ldi, double* out, int64_t ldo);
// transposes of the 64 x 64 blocks of a block-inverse array (dinv_elems(n))
void transpose_dinv(Exec& ex, int64_t n, const double* D, double* Dt);
bool lu_supported(int64_t n);
// r = b - A x
void residual(Exec& ex, int64_t m, int64_t n, const double* A, int64_t lda, const double* b, const double* x,
              double* r);
// y = X^T v (X m x n), split over m with partials P (splits x n)
size_t gemv_t_partials(int64_t m, int64_t n);
void gemv_t(Exec& ex, int64_t m, int64_t n, const double* X, int64_t ldx, const double* v, double* y,
            double* P);
void axpy_update(Exec& ex, int64_t n, double* x, const double* d);   // x += d
void fill_nan_on_info(Exec& ex, int64_t n, double* x, const int32_t* info);
// dst(:, j) = src(:, j) for an r x c column-major block
void copy_f64(Exec& ex, int64_t r, int64_t c, const double* src, int64_t lds, double* dst, int64_t ldd);
void zero_i32(Exec& ex, int64_t n, int32_t* p);
// *info = 5000 if A (m x n, ld lda) or b (m) holds a NaN or an infinity
void all_finite(Exec& ex, int64_t m, int64_t n, const double* A, int64_t lda, const double* b, int32_t* info);
void copy_i32(Exec& ex, int64_t n, const int32_t* src, int32_t* dst);

// ---------------------------------------------------------------- batches
// One grouped launch: the kernel, its table at byte offset `off` of the
// device table area, the member count, the total work-group count and the
// pipeline stage (for phase marks).
struct LaunchGroup {
    GroupLaunchFn fn;
    size_t off;
    int count;
    int64_t total;
    uint32_t stage;
};
struct GroupSeq {
    std::vector<char> blob;             // host copy of the group tables
    std::vector<LaunchGroup> groups;    // in launch order
};
// Merge the recorded launches of a batch into grouped launches (host only).
int build_groups(const Recorder& rec, GroupSeq* out);
// Enqueue grouped launches whose tables sit at dtables (kernel launches
// only; phase marks when `marks`).
void enqueue_groups(const std::vector<LaunchGroup>& groups, const char* dtables, hipStream_t st, bool marks);
// build_groups, copy the tables to dtables (cap bytes; one wait for the
// copy) and enqueue them on st (batched.hip).
int run_recorded(const Recorder& rec, char* dtables, size_t cap, hipStream_t st);

// ---------------------------------------------------------------- condition estimate
size_t condest_workspace_bytes(int64_t m, int64_t n, int64_t kchunk_fixed = 0);
int condest_run(Exec& ex, int64_t m, int64_t n, const double* A, int64_t lda, double known_kappa, float* dk0,
                int32_t* dchoice, void* work, size_t work_bytes);
// estimate from the FP32 QR of the FP32 sketch (s rows, seed, pid); W (s x n
// FP32, ld s) and R (n x n FP64) receive the sketch and its R factor
size_t condest_qr_workspace_bytes(int64_t m, int64_t n, int64_t s, int64_t kchunk_fixed = 0);
int condest_qr_run(Exec& ex, int64_t m, int64_t n, const double* A, int64_t lda, int64_t s, uint64_t seed,
                   uint32_t pid, float* dk0, int32_t* dchoice, float* W, double* R, void* work,
                   size_t work_bytes);

// ---------------------------------------------------------------- single solves (api.hip)
// workspace bytes of one PNE (hpne = 0) / HPNE (hpne = 1) solve, after the
// host-side argument checks of the solvers
pne_status solve_workspace(int hpne, int64_t m, int64_t n, int64_t lda, const pne_opts* o, size_t* need);
// pne_solve / hpne_solve on a given workspace
pne_status solve_entry(int hpne, int64_t m, int64_t n, const double* dA, int64_t lda, const double* db,
                       double* dx, const pne_opts* o, void* dwork, size_t work_bytes, int32_t* dinfo,
                       pne_info* hinfo, hipStream_t st);

}  // namespace pne
