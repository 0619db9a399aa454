/*
 * htred.h -- C ABI of the MI355X (gfx950) Householder Hessenberg-triangular
 * reduction library, libhtred.so.
 *
 * Method: Bujanovic, Karlsson, Kressner, "A Householder-based algorithm for
 * Hessenberg-triangular reduction" (HouseHT).  Given A and an upper
 * triangular B (both n x n), the library computes orthogonal Q and Z with
 *     H = Q^T A Z   upper Hessenberg,     T = Q^T B Z   upper triangular
 * (problem statement of Sec. 1 and the opening of Sec. 3; Algorithm 1).
 * Columns of A are reduced by Householder reflectors from the left; the
 * matching column of B is reduced by an opposite reflector from the right,
 * built from a solve with B (Sec. 2.2, Lemma 2.1).  Reflectors are gathered
 * in panels of nb columns with B kept in the factored form of eq. (tildeB)
 * (Sec. 3.2) and then absorbed into A, B, Q, Z as block-reflector products
 * (Sec. 3.3).
 *
 * Conventions for every entry point:
 *   - matrices are FP64, column-major, on the device (HIP device pointers);
 *     leading dimensions must be >= max(1, n);
 *   - the caller owns every buffer; the library keeps no pointer after the
 *     call returns;
 *   - work is enqueued on `stream` (a hipStream_t passed as void*; NULL is
 *     the default stream).  Unless stated otherwise a call returns after
 *     its work is enqueued; host-side results (stats) force a stream sync;
 *   - return value 0 is success; a negative value -i flags argument i as
 *     invalid (LAPACK INFO style, 1-based argument position); positive
 *     values are HT_ERR_* codes below.  ht_strerror() names every code.
 */
#ifndef HTRED_H
#define HTRED_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Positive error codes. */
#define HT_OK              0
#define HT_ERR_HIP         1  /* a HIP runtime call failed */
#define HT_ERR_WORKSPACE   2  /* workspace too small or misaligned */
#define HT_ERR_NONFINITE   3  /* NaN or Inf found in A or B on entry */
#define HT_ERR_UNSUPPORTED 4  /* option combination not implemented */
#define HT_ERR_NOLIB       5  /* device code for this GPU is missing */
#define HT_ERR_TOO_LARGE   6  /* ht_reduce_noalloc: the order needs more than the
                                 library's fixed scratch (HT_NOALLOC_SCRATCH_BYTES) */

/* How Q and Z are produced. */
typedef enum {
    HT_QZ_IDENTITY = 0,   /* Q, Z are set to I on entry (Sec. 3 opening) */
    HT_QZ_ACCUMULATE = 1, /* Q <- Q_in * Q, Z <- Z_in * Z */
    HT_QZ_NONE = 2        /* not computed (pointer may be NULL) */
} ht_qz_mode;

/* Arithmetic of the trailing block-reflector updates (absorption, Sec. 3.3:
 * the window applications and rank-k corrections).  Panel reduction, solves,
 * chain factorisations and the T/S factors are always native FP64.
 * The split forms emulate each FP64 product with n_slices fixed-point digit
 * slices per operand (per-row / per-column power-of-two exponents over
 * chunks of 32 contraction indices) multiplied on the low-precision matrix
 * cores with exact FP32 accumulation and recombined in FP64:
 *   BF16: 7-bit digits, n_slices 1..8, default 8 (56 bits);
 *   FP8:  4-bit digits, n_slices 1..14, default 14 (56 bits).
 * Per entry the error is about (n_slices + 3) 2^{-bits n_slices} times
 * |op(A)| |op(B)|.  ht_reduce_batched supports HT_PREC_FP64 only. */
typedef enum {
    HT_PREC_FP64 = 0,        /* native FP64 (MFMA) */
    HT_PREC_SPLIT_BF16 = 1,  /* FP64 emulated with BF16 slices, FP32 accumulate */
    HT_PREC_SPLIT_FP8 = 2    /* FP64 emulated with FP8-E4M3 slices */
} ht_precision;

typedef struct {
    int32_t struct_size;     /* = sizeof(ht_options); checked */
    int32_t nb;              /* panel width (number of reflectors per absorption);
                                0 = default 64.  Must be 1..128. */
    int32_t max_ir;          /* iterative-refinement steps before a panel is cut
                                short (Sec. 3.2.2 c): default 10 */
    int32_t qmode;           /* ht_qz_mode for Q */
    int32_t zmode;           /* ht_qz_mode for Z */
    int32_t prec;            /* ht_precision */
    int32_t n_slices;        /* slices per operand for split precision; 0 = auto */
    int32_t flags;           /* HT_FLAG_* bits */
    double  ir_tol_factor;   /* IR stops when ||r||/||x|| <= f * u * ||B||_F;
                                default 2.0 (Sec. 2.3) */
    uint64_t seed;           /* stream for the zero-diagonal perturbation rho
                                (Sec. 3.2.1) */
    int32_t batch_block;     /* ht_reduce_batched: reflectors per block of the
                                Householder QR that re-triangularises B after a
                                panel; 0 = default 32.  Must be 1..64. */
    int32_t batch_wg_per_cu; /* ht_reduce_batched: resident workgroups per
                                compute unit (each reduces one pencil at a
                                time); 0 = default 3.  Must be 1..3. */
    int32_t ilo;             /* ht_reduce: first column to reduce (0-based),
                                default 0.  Columns 0..ilo-1 must already be in
                                final form: A(i, j) = 0 for i > j + 1 and for
                                i > ilo when j < ilo (B upper triangular as
                                always), as after ht_preprocess.  Only columns
                                ilo..n-3 are reduced; the transformations act on
                                rows / columns ilo+1..n-1, on every row of A and
                                B above them and on all of Q and Z. */
    int32_t ell;             /* ht_reduce: blocks per absorption window (Sec. 3.5,
                                accelerated reduction of V2 and U2); 0 or 2 =
                                the basic scheme (Sec. 3.3).  l >= 3 keeps B
                                block upper triangular between panels, with
                                diagonal blocks of order (l-1) nb, and needs
                                (l-1) nb <= 128.  Its solves are block back
                                substitutions through LU decompositions with
                                partial pivoting, without the overflow-safe
                                scaling of the basic scheme: use it for
                                pencils whose solves stay within the FP64
                                range.  Zero diagonal entries of B are not
                                perturbed (Sec. 3.2.1); an exactly singular
                                diagonal block gets the pivot eps ||B||_F, and
                                refinement judges the solves. */
} ht_options;

/* flags */
#define HT_FLAG_CHECK_FINITE 1  /* scan A, B for NaN/Inf on entry (syncs) */
#define HT_FLAG_PROFILE      2  /* time kernel classes with HIP events (stats) */
#define HT_FLAG_SOLVE_SOLO   4  /* triangular solves on one workgroup, without
                                   helper workgroups (slower; for testing) */

/* Kernel classes reported in ht_stats.prof_* when HT_FLAG_PROFILE is set.
 * prof_work is the algorithmic work of the class: flops for the
 * contraction classes (WY, CHAIN), bytes for the streaming classes. */
#define HT_PROF_WY     0  /* block-reflector updates by general products (flops) */
#define HT_PROF_TRSV   1  /* triangular solves with B (bytes of B read) */
#define HT_PROF_TRMV   2  /* residual products with B (bytes of B read) */
#define HT_PROF_YGEMV  3  /* Y = A V T columns (bytes of A read) */
#define HT_PROF_CHAIN  4  /* QL/QR/RQ chain factorisations (flops) */
#define HT_PROF_SWEEP  5  /* fused MFMA sweeps of chain windows over rows (flops) */
#define HT_PROF_NCLASS 8

typedef struct {
    int64_t columns;          /* columns reduced */
    int64_t cols_extra_ir;    /* columns that needed at least one IR step */
    int64_t ir_steps;         /* total IR correction steps */
    int64_t ir_failures;      /* columns whose IR did not converge (panel cut) */
    int64_t absorptions;      /* number of absorptions (panels) */
    int64_t scaled_solves;    /* solves that needed overflow rescaling */
    double  flops;            /* flops executed, counted from launch shapes */
    double  ms_total;         /* wall time of the call (ms), host clock */
    double  prof_ms[HT_PROF_NCLASS];       /* summed launch durations (HIP events) */
    double  prof_work[HT_PROF_NCLASS];     /* algorithmic flops or bytes */
    int64_t prof_launches[HT_PROF_NCLASS]; /* launches timed */
} ht_stats;

/* Fills *opt with the defaults listed above: the refinement limits of
 * Sec. 2.3 and Sec. 3.2.2 (at most 10 steps, tolerance 2 u ||B||_F) and the
 * panel width of Sec. 3.2 / Sec. 3.3 (64).  Returns 0 (-1 for a NULL opt). */
int ht_default_options(ht_options *opt);

/* Device workspace (bytes) ht_reduce needs for order n with these options
 * (opt may be NULL for the defaults): the panel factors U, V, Y, S, T of
 * Sec. 3.2 and the window transforms of the absorption chains of Sec. 3.3.
 * Returns 0 for invalid options or n outside 0..2^30. */
size_t ht_workspace_size(int64_t n, const ht_options *opt);

/*
 * ht_reduce -- HouseHT reduction of one pencil (Algorithm 1 with the panel
 * reduction of Sec. 3.2 and the absorption of Sec. 3.3).
 *
 *   A  (in/out)  n x n, lda:  A on entry, H on exit (exact zeros below the
 *                first subdiagonal).
 *   B  (in/out)  n x n, ldb:  upper triangular B on entry (the strictly lower
 *                triangle is ignored), T on exit (exact zeros below the
 *                diagonal).  An exactly zero (or subnormal) diagonal entry
 *                met by a solve is replaced by 2 u rho ||B||_F, rho ~ N(0,1)
 *                (Sec. 3.2.1, Remark 2.2): T is then exact for B + Delta_0.
 *   Q, Z (out or in/out per qmode/zmode)  n x n, ldq/ldz.
 *   opt   options or NULL for defaults.
 *   stats NULL, or receives counters; a non-NULL stats makes the call wait
 *         for the stream.
 *   workspace / ws_bytes: NULL/0 lets the library allocate (and free)
 *         device memory itself; otherwise at least ht_workspace_size bytes,
 *         256-byte aligned, owned by the caller.
 *   stream hipStream_t (void*), NULL = default stream.
 *
 * Q and Z: with HT_QZ_IDENTITY they are set to I first (the problem
 * statement's Q e1 = Z e1 = e1); with HT_QZ_ACCUMULATE the caller's Q_in and
 * Z_in are multiplied from the right (Q <- Q_in Q, Z <- Z_in Z: every update
 * of Q and Z in Sec. 3.3 is a right multiplication over all n rows), so a
 * preceding orthogonal transformation (e.g. the QR factorisation that made
 * B triangular) is carried along; with HT_QZ_NONE they are not touched.
 * Leading dimensions must also be <= INT32_MAX (-6..-9 otherwise).
 *
 * The host reads each panel column's refinement verdict (Sec. 3.2.2 c)
 * through a 256-byte pinned host buffer that the call allocates and frees
 * itself, one column late: the next column is already enqueued, and is
 * rolled back and redone when the verdict asks for refinement.  So the call
 * waits for `stream` about once per reflector pair and per refinement step
 * and is not graph-capturable (ht_reduce_batched is).  The call keeps no
 * state between calls: concurrent calls from several host threads on
 * different streams (with different workspaces) are independent.
 * HT_FLAG_CHECK_FINITE uses a word at the end of the caller's workspace, or
 * a 4-byte device allocation when the library allocates.
 * Results are deterministic: no floating-point atomics are used.
 */
int ht_reduce(double *A, double *B, double *Q, double *Z, int64_t n,
              int64_t lda, int64_t ldb, int64_t ldq, int64_t ldz,
              const ht_options *opt, ht_stats *stats,
              void *workspace, size_t ws_bytes, void *stream);

/*
 * ht_triangularize_b -- the first step of the QZ algorithm (Sec. 1): an
 * orthogonal Q0 with B = Q0 R, R upper triangular, applied to the pencil:
 *   B (in/out)  n x n general matrix on entry, R on exit (exact zeros below
 *               the diagonal);
 *   A (in/out)  n x n, replaced by Q0^T A;
 *   Q           Q0 (qmode HT_QZ_IDENTITY), Q_in Q0 (HT_QZ_ACCUMULATE) or
 *               untouched (HT_QZ_NONE, Q may be NULL).
 * The pencil is then ready for ht_reduce with qmode HT_QZ_ACCUMULATE.  The
 * QR factorisation runs in panels of opt->nb columns, each factored by the
 * window chain of Sec. 3.3.2 b (the chain that triangularises U2) and
 * applied by the same block-reflector sweeps as the absorption.  FP64 only
 * (HT_ERR_UNSUPPORTED for a split precision); zmode is ignored.  workspace /
 * ws_bytes as for ht_reduce (ht_workspace_size bytes for the same options,
 * or NULL to let the library allocate).  Asynchronous on `stream` unless the
 * library allocates (then it waits before freeing).  Returns -1..-3 for a
 * NULL A, B or Q (Q only when formed), -5 for n outside 0..2^30, -6 / -7 /
 * -8 for bad lda / ldb / ldq, -10 for invalid options.
 */
int ht_triangularize_b(double *A, double *B, double *Q, int64_t n, int64_t lda,
                       int64_t ldb, int64_t ldq, const ht_options *opt,
                       void *workspace, size_t ws_bytes, void *stream);

/*
 * ht_preprocess -- the zero-column preprocessing of Sec. 3.5: when the upper
 * triangular B has l > 1 zero columns, a permutation Z0 moves them to the
 * front (Q0 = Z0 when B is diagonal, so that it stays diagonal, else
 * Q0 = I), the QR factorisation of the first l columns of Q0^T A Z0 gives
 * Q1 with
 *     (Q0 Q1)^T A Z0 = [A11 A12; 0 A22],   (Q0 Q1)^T B Z0 = [0 B12; 0 B22],
 * A11 upper triangular, and B22 is made upper triangular again by the QR of
 * ht_triangularize_b (Q2), applied to A22.  On exit A and B hold the new
 * pencil, Q = Q0 Q1 diag(I, Q2) and Z = Z0 (times Q_in / Z_in with
 * HT_QZ_ACCUMULATE), and *ilo = l: the leading l x l part is in generalised
 * Schur form (l infinite eigenvalues) and ht_reduce with opt->ilo = l and
 * qmode = zmode = HT_QZ_ACCUMULATE finishes the reduction of the whole
 * pencil.  With fewer than two zero columns nothing is changed (Q, Z set
 * per their modes) and *ilo = 0.  Allocates an n x n temporary and reads
 * the zero-column pattern back to the host (waits for `stream`).  FP64
 * only.  Returns as ht_triangularize_b, plus -4 / -9 for a NULL Z or bad
 * ldz and -11 for a NULL ilo.
 */
int ht_preprocess(double *A, double *B, double *Q, double *Z, int64_t n, int64_t lda,
                  int64_t ldb, int64_t ldq, int64_t ldz, const ht_options *opt,
                  int32_t *ilo, void *workspace, size_t ws_bytes, void *stream);

/* Size of the fixed device scratch of ht_reduce_noalloc (per GPU). */
#define HT_NOALLOC_SCRATCH_BYTES (64u << 20)

/*
 * ht_reduce_noalloc -- ht_reduce for callers that cannot allocate memory
 * (tight serving loops, harnesses that forbid hipMalloc / hipHostMalloc).
 * Same arguments, results and return codes as ht_reduce (same kernels),
 * without the workspace arguments: the device workspace is a fixed array of
 * HT_NOALLOC_SCRATCH_BYTES (64 MiB) inside the library, one per GPU, held
 * until the process ends.  Orders whose workspace (ht_workspace_size for
 * the same options) exceeds it return HT_ERR_TOO_LARGE: it holds orders up
 * to 2248 at nb = 128, 4984 at nb = 64 and 9958 at nb = 32.
 * The call allocates nothing: refinement verdicts are read into pageable
 * host memory of the call, HT_FLAG_CHECK_FINITE uses a word of the array,
 * and HT_FLAG_PROFILE (which creates HIP events) returns HT_ERR_UNSUPPORTED.
 * Every call on a GPU uses that GPU's one array, which keeps the previous
 * call's contents (the call clears what must start at zero): calls that
 * overlap on one GPU (several host threads or streams) race and must be
 * serialised by the caller.  The first call on each device resolves the
 * array's device address (hipGetSymbolAddress) once.
 */
int ht_reduce_noalloc(double *A, double *B, double *Q, double *Z, int64_t n,
                      int64_t lda, int64_t ldb, int64_t ldq, int64_t ldz,
                      const ht_options *opt, ht_stats *stats, void *stream);

/*
 * ht_reduce_batched -- independent HT reductions of `batch` small pencils in
 * one persistent launch (HT reduction inside deflation windows, Sec. 1).
 *
 *   n_dev[i]  order of pencil i (device int32 array), 0 <= n <= 512;
 *   A_dev, B_dev, Q_dev, Z_dev: device arrays of device pointers, pencil i
 *             column-major with leading dimension ld_dev[i] (device int32);
 *             A, B in/out as in ht_reduce, Q and Z set (identity start);
 *   info_dev  device int32 array: 0 per success;
 *   nmax      host-side upper bound of n_dev (sizes the launch);
 *   opt       max_ir, ir_tol_factor and seed as in ht_reduce; nb is the panel
 *             width of every pencil's reduction as given (1..128), and
 *             nb = 0 runs one panel over each whole pencil; opt NULL takes
 *             ht_default_options (nb 64, batch_block 32, batch_wg_per_cu 3).
 *             A panel that ends before the last column is absorbed and B's
 *             trailing block is re-triangularised by a blocked Householder
 *             QR (batch_block reflectors per block) whose transformations go
 *             to A and Q.  batch_wg_per_cu workgroups per compute unit stay
 *             resident and take pencils, largest order first.
 * No host synchronisation and no allocation inside: the call can be
 * captured in a hipGraph.  workspace (256-byte aligned) must hold
 * ht_batched_workspace_size(batch, nmax, opt) bytes for the same options:
 * one scratch area per resident workgroup (ht_batched_workspace_size
 * returns 0 for invalid sizes or options).
 * Returns -1 for batch < 0, -2 for a NULL n_dev, -3 for a NULL A_dev or
 * B_dev, -5 for a NULL Q_dev or Z_dev, -7 for a NULL ld_dev, -8 for a NULL
 * info_dev, -9 for nmax outside 0..512, -10 for invalid options,
 * HT_ERR_UNSUPPORTED for a split precision, HT_ERR_WORKSPACE for a missing,
 * misaligned or too small workspace, HT_ERR_HIP if the launch fails.  A
 * pencil whose order, leading dimension or pointers are invalid gets
 * info = -1 and is left untouched.
 */
size_t ht_batched_workspace_size(int32_t batch, int32_t nmax, const ht_options *opt);
int ht_reduce_batched(int32_t batch, const int32_t *n_dev,
                      double *const *A_dev, double *const *B_dev,
                      double *const *Q_dev, double *const *Z_dev,
                      const int32_t *ld_dev, int32_t *info_dev, int32_t nmax,
                      const ht_options *opt, void *workspace, size_t ws_bytes,
                      void *stream);

/*
 * ht_batched_pencil_stats -- per-pencil record of the last ht_reduce_batched
 * call that used `workspace` (same batch): waits for `stream`, then writes
 * out[8 i + 0..7] (host array of 8*batch int64) for pencil i:
 *   0, 1  start and end in nanoseconds of the device wall clock, relative
 *         to the earliest start in the batch;
 *   2     number of panels (absorptions) of its reduction;
 *   3     number of iterative-refinement steps (Sec. 3.2.2);
 *   4, 5, 6  nanoseconds spent in the factored solves, in the residuals and
 *         in the absorptions (the two-sided panel updates);
 *   7     nanoseconds spent re-triangularising B after a panel.
 * Returns -1 for a NULL workspace, -2 for batch < 0, -3 for a NULL out,
 * HT_ERR_HIP if the copy fails.  Meaningless before the batched call ran.
 */
int ht_batched_pencil_stats(const void *workspace, int32_t batch, int64_t *out, void *stream);

/*
 * ht_check -- the acceptance quantities of a reduction (Theorem A.1 and its
 * corollary), computed on the device with the library's FP64 products:
 *   out[0] = ||Q H Z^T - A0||_F / ||A0||_F,  out[1] = ||Q T Z^T - B0||_F / ||B0||_F,
 *   out[2] = ||Q^T Q - I||_F,                 out[3] = ||Z^T Z - I||_F.
 * A0, B0 (the input pencil), H, T, Q, Z: device pointers, n x n, column-major,
 * common leading dimension ld >= max(1, n); out: host array of 4 doubles.
 * Allocates two n x n temporaries (hipMalloc) and waits for `stream`.
 * Returns -1..-6 for a NULL matrix (in argument order), -7 for n < 0, -8 for
 * ld < n, -9 for a NULL out, HT_ERR_HIP if an allocation or copy fails.
 */
int ht_check(const double *A0, const double *B0, const double *H, const double *T,
             const double *Q, const double *Z, int64_t n, int64_t ld, double *out,
             void *stream);

/*
 * ht_wy_gemm -- one product of the block-reflector (WY) updates of Sec. 2.4
 * and Sec. 3.3 (window applications, rank-k corrections) as ht_reduce computes it for
 * `prec`:  C = alpha op(A) op(B) + beta C  (op(X) = X or X^T per transA /
 * transB != 0), op(A) m x k, op(B) k x n, C m x n; device pointers,
 * column-major, FP64 storage; beta == 0 ignores C's contents.  Exposed so
 * that the split products can be validated on their own.  n_slices as in
 * ht_options (0 = default).  Asynchronous on `stream`.  Returns -1 for an
 * unknown prec, -2 for n_slices out of range, -5/-6/-7 for negative m/n/k,
 * -10/-12/-15 for a leading dimension below the stored rows, -9/-11/-14
 * for a NULL operand with non-empty shape.
 */
int ht_wy_gemm(int32_t prec, int32_t n_slices, int32_t transA, int32_t transB,
               int64_t m, int64_t n, int64_t k, double alpha,
               const double *A, int64_t lda, const double *B, int64_t ldb,
               double beta, double *C, int64_t ldc, void *stream);

/* Library utility (no passage of the paper): human-readable name of a
 * return code; never NULL. */
const char *ht_strerror(int code);

/* Library utility (no passage of the paper): version string, e.g.
 * "htred 0.1 gfx950". */
const char *ht_version(void);

#ifdef __cplusplus
}
#endif
#endif /* HTRED_H */
