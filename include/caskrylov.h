/*
 * caskrylov: SpMV-driven Krylov solvers with a cascaded kernel predictor and
 * asynchronous kernel switching, for AMD Instinct MI355X (gfx950).
 *
 * The method is that of "Cascaded Prediction and Asynchronous Execution of
 * Iterative Algorithms on Heterogeneous Platforms" (Gao, Liu, Wang, Ji,
 * Huang; arXiv 2411.10143):
 *   - solve A x = b with CG or restarted GMRES, whose dominant kernel is
 *     sparse matrix-vector multiplication (Introduction);
 *   - choose the SpMV configuration in three cascaded stages -- storage
 *     format, then algorithm, then kernel parameter -- from 15 matrix
 *     features (Section III-B-1, feature table; Section III-C-1, cascaded
 *     prediction figure);
 *   - start the solve at once on a default configuration and swap in each
 *     stage's choice at the next iteration boundary after it is ready, while
 *     features, inference and format conversion run concurrently
 *     (Section III-C-2, asynchronous execution).
 *
 * Conventions for every entry point
 *   - Pointers named d_* are DEVICE pointers (hipMalloc'd or torch-allocated
 *     HIP memory on the current device); all others are host pointers.
 *   - Index arrays are int32; values are IEEE binary64 unless "f32" says so.
 *   - Every call returns ck_status and never aborts, throws or exits.  On a
 *     non-OK status, ck_last_error() returns a thread-local message.
 *   - HIP failures return CK_E_HIP (the hipError_t text is in the message).
 *   - Streams: hipStream_t values owned by the caller; 0 is the null stream.
 *     Enqueued work is ordered on the given stream only.
 */
#ifndef CASKRYLOV_H
#define CASKRYLOV_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    CK_OK = 0,
    CK_E_INVALID = -1,        /* bad argument or malformed CSR              */
    CK_E_NOMEM = -2,          /* device allocation failed                   */
    CK_E_HIP = -3,            /* a HIP runtime call failed                  */
    CK_E_NOT_CONVERGED = -4,  /* iteration budget spent above tolerance     */
    CK_E_BREAKDOWN = -5,      /* CG: p.Ap <= 0 (A not SPD); GMRES: singular */
    CK_E_UNSUPPORTED = -6,    /* e.g. ELL refused because of padding fill   */
    CK_E_CANCELLED = -7       /* work abandoned before it finished          */
} ck_status;

/* Opaque matrix handle: owns device copies of the CSR arrays and of every
 * other format built from them. */
typedef struct ck_matrix *ck_handle;

/* ---- SpMV configuration space (Section III-B-2, configuration figure) ----
 * format    : CK_FMT_CSR, CK_FMT_ELL, CK_FMT_COO, CK_FMT_DIA (diagonals) or
 *             CK_FMT_HYB (ELL part plus the remainder of long rows); the
 *             five formats Section III-B-2 names
 * algorithm : for CSR only -- CK_ALG_SCALAR (one lane per row, row block
 *             staged through LDS), CK_ALG_VECTOR (`lanes` lanes per row),
 *             CK_ALG_MERGE (merge-path load balancing), CK_ALG_PANEL (column
 *             panels sized so each XCD's L2 holds its slice of x; a
 *             panel-major copy made by spmv_convert)
 * lanes     : for CSR-vector, 1, 2, 4, 8, 16, 32 or 64 lanes per row
 * stages_done: how many cascade stages produced this configuration (0-3)
 * Fourteen configurations in all: 7 CSR-vector lane counts, CSR-scalar,
 * CSR-merge, ELL, COO, CSR-panel, DIA, HYB.  ck_config_id() numbers them
 * 0..13 in that order. */
enum { CK_FMT_CSR = 0, CK_FMT_ELL = 1, CK_FMT_COO = 2, CK_FMT_DIA = 3, CK_FMT_HYB = 4 };
enum { CK_ALG_SCALAR = 0, CK_ALG_VECTOR = 1, CK_ALG_MERGE = 2, CK_ALG_PANEL = 3 };
#define CK_NUM_CONFIGS 14

typedef struct {
    int32_t format;
    int32_t algorithm;
    int32_t lanes;
    int32_t stages_done;
} ck_config;

/* ---- Features (feature table, Section III-B-1) ----
 * Integer accumulators are exact.  The derived values are computed on the
 * host from the integers only:
 *   density = nnz/(nrows*ncols)        mean = nnz/nrows
 *   sd = sqrt(nrows*sum_r2 - sum_r^2)/nrows (radicand exact in 128 bits)
 *   cov = sd/mean (0 if mean = 0)      maxavg = max_r - mean
 *   distavg = span_sum/nrows           clusteravg = cluster_sum/nrows
 *   fill = nrows*max_r/nnz             diagfill = nrows*ndiag/nnz (0 if nnz=0)
 * span_sum = sum over rows of (last column - first column); cluster_sum =
 * sum over rows of the longest run of consecutive column indices; ndiag =
 * number of distinct (column - row) among stored entries; diag_nnz = stored
 * main-diagonal entries; hist[0] = empty rows, hist[b] = rows with length in
 * [2^(b-1), 2^b), hist[15] open-ended; is_symmetric = square with every
 * stored a_ij matched by a stored a_ji of equal value. */
typedef struct {
    int64_t nrows, ncols, nnz, sum_r, sum_r2, max_r, min_r, span_sum, cluster_sum,
        ndiag, diag_nnz, hist[16], is_symmetric;
    double density, mean, sd, cov, maxavg, distavg, clusteravg, fill, diagfill;
} ck_features;

/* ---- Solver options and results ---- */
enum { CK_PREC_FP64 = 0, CK_PREC_MIXED = 1 };
/* Execution modes (ck_solve_opts.async; ignored when use_config = 1):
 *   CK_EXEC_DEFAULT    the whole solve on the default configuration;
 *   CK_EXEC_ASYNC      start on the default configuration while features,
 *                      inference and conversion run on a side stream, and
 *                      swap each stage's choice in at the next iteration
 *                      boundary (Section III-C-2);
 *   CK_EXEC_SEQUENTIAL features, cascade and conversion first, then the
 *                      whole solve on the prediction (the sequential form
 *                      the asynchronous one is compared with, Section IV);
 *                      their times count in t_total_us and switch_iter[t]
 *                      = 0 for every stage that took effect. */
enum { CK_EXEC_DEFAULT = 0, CK_EXEC_ASYNC = 1, CK_EXEC_SEQUENTIAL = 2 };
/* Overhead-aware conversion (ck_solve_opts.overhead_aware = 1 with
 * CK_EXEC_ASYNC in FP64; the overhead-conscious selection discussed among
 * the paper's related work): a decision that needs a new copy of the matrix
 * (ELL, COO, DIA, HYB, CSR-panel) waits for the solver's residual reports
 * of the first eight or more iterations, extrapolates the remaining
 * iterations R (ck_overhead_gate), and is converted only if 0.25 * R is at
 * least the conversion's cost in products; otherwise the solve keeps its
 * configuration (conversion_gated = 1 in the result). */

typedef struct {
    double tol;            /* stop when ||b - A x||_2 / ||b||_2 <= tol        */
    int32_t max_iter;      /* budget of SpMV-bearing iterations               */
    int32_t restart;       /* GMRES restart length m (<= 64); CG ignores it   */
    int32_t precision;     /* CK_PREC_FP64 or CK_PREC_MIXED (FP32 inner solve
                              + FP64 refinement; needs CK_KEEP_FP32)          */
    int32_t async;         /* CK_EXEC_DEFAULT, CK_EXEC_ASYNC or
                              CK_EXEC_SEQUENTIAL (see below)                  */
    int32_t check_every;   /* iterations between host convergence polls       */
    int32_t use_config;    /* 1: run every SpMV with `config` (async ignored) */
    ck_config config;
    int32_t overhead_aware; /* CK_EXEC_ASYNC, FP64 only: convert a decision's
                              format only if the remaining iterations,
                              extrapolated from the residual's decay, can
                              repay the conversion (see below)              */
    int32_t known_start;   /* CK_EXEC_DEFAULT / _ASYNC: start from the start
                              tree's configuration (ck_start_config) instead
                              of the default one                           */
} ck_solve_opts;

typedef struct {
    int32_t status;          /* ck_status of the solve                        */
    int32_t iterations;      /* SpMV-bearing iterations performed             */
    int32_t switch_iter[3];  /* iteration at which stage 1/2/3's choice took
                                effect; -1 if it never did                    */
    int32_t outer_steps;     /* restarts (CG) / cycles (GMRES) / refinements  */
    double true_relres;      /* ||b - A x||/||b|| recomputed in FP64 at exit  */
    double t_features_us, t_infer_us, t_convert_us, t_total_us;
    ck_config final_config;
    int32_t conversion_gated;    /* overhead-aware gate: -1 not consulted,
                                    0 converted, 1 conversion skipped        */
    int32_t est_remaining_iters; /* the gate's estimate (-1 if none)         */
} ck_solve_result;

/* Flags for spmv_create */
#define CK_KEEP_FP32 0x1u  /* also keep an FP32 copy of the values (mixed)   */

/* Device memory for a handle, supplied by the caller (e.g. a framework's
 * caching allocator).  alloc(bytes, s, ctx) returns `bytes` of device memory
 * on the current device, aligned to at least 256 bytes, to be used in stream
 * order on s (and, once that use has finished, on any stream), or NULL on
 * failure (the call that needed it then returns CK_E_NOMEM).  free(p, s, ctx)
 * gives back a block; s is the stream it was allocated for, and the library
 * calls free only when no work that uses the block can still be pending, so
 * it may be reused at once.  Both may be called from threads the library
 * creates (the asynchronous executor's side thread) and on streams it
 * creates, concurrently with the caller's thread. */
typedef struct {
    void *(*alloc)(size_t bytes, hipStream_t s, void *ctx);
    void (*free)(void *p, hipStream_t s, void *ctx);
    void *ctx;
} ck_allocator;

/* ------------------------------------------------------------------------ */

/* spmv_create -- ingest a CSR matrix (problem statement A x = b, Introduction;
 * the CSR format of the configuration space, Section III-B-2).
 * d_rowptr int32[nrows+1], d_col int32[nnz], d_val double[nnz] on the device.
 * The arrays are COPIED (the caller may free them afterwards) and validated:
 * rowptr[0] = 0, nondecreasing, rowptr[nrows] = nnz, 0 <= col < ncols,
 * columns strictly increasing inside each row.  Malformed input gives
 * CK_E_INVALID and *out = NULL.  Blocks until the copy is validated.
 * The active configuration starts as ck_default_config().
 * alloc: where every device block the handle needs comes from -- its copies
 * of the matrix in every format, feature and conversion temporaries, product
 * carries, and the workspaces of solves on it.  The struct is copied; its
 * functions and ctx must stay valid until spmv_destroy returns.  NULL: a
 * per-device cache of blocks inside the library (hipMalloc'd, kept across
 * handles up to 16 GiB, so ingest and destroy map no new pages). */
ck_status spmv_create(ck_handle *out, int64_t nrows, int64_t ncols, int64_t nnz,
                      const int32_t *d_rowptr, const int32_t *d_col, const double *d_val,
                      uint32_t flags, const ck_allocator *alloc, hipStream_t s);

/* spmv_destroy -- release every device copy (to the handle's allocator, or
 * to the library's cache).  The caller must have finished all work that uses
 * the handle; nothing is synchronised again.  NULL is ignored. */
void spmv_destroy(ck_handle h);

/* spmv_features -- the 15 features of the feature table (Section III-B-1),
 * computed by GPU kernels on stream s; blocks until *out is filled. */
ck_status spmv_features(ck_handle h, ck_features *out, hipStream_t s);

/* ck_features_ex -- spmv_features with flags.  CK_FEAT_NO_SYMMETRY skips the
 * symmetry test (a search of row j for every stored (i, j), and the one pass
 * that reads the values): is_symmetric is then -1 and every other field is
 * the same.  The cascade does not use is_symmetric; the asynchronous
 * executor's feature pass skips it in the same way. */
#define CK_FEAT_NO_SYMMETRY 0x1u
ck_status ck_features_ex(ck_handle h, ck_features *out, uint32_t flags, hipStream_t s);

/* spmv_select -- host-only cascaded inference (Section III-C-1): stage 1
 * format, stage 2 CSR algorithm (only if CSR; scalar, vector, merge or
 * panel), stage 3 lanes (only if CSR-vector).  model_path: a cascade model
 * file, or NULL for the default model: the file named by the environment
 * variable CK_CASCADE_MODEL if set, else cascade_model.txt next to the
 * library (the async executor and the request loop use the default model).
 * A stage that does not run keeps the default configuration's value for its
 * field.  *out->stages_done = stages run. */
ck_status spmv_select(const ck_features *f, const char *model_path, ck_config *out);

/* ck_select_stages -- the same inference, reporting each stage's raw class:
 * stage[0] format, stage[1] algorithm (-1 if not run), stage[2] log2(lanes)
 * (-1 if not run). */
ck_status ck_select_stages(const ck_features *f, const char *model_path, int32_t stage[3]);

/* ck_eval_stage -- one stage's tree alone, without the cascade's gating
 * (stage 0 format, 1 CSR algorithm, 2 log2(lanes)); *cls = its class.  For
 * single-stage ablations of the cascade (Section IV compares predicting one
 * part of the configuration with predicting all three). */
ck_status ck_eval_stage(const ck_features *f, const char *model_path, int32_t stage,
                        int32_t *cls);

/* ck_select_device -- the device-resident cascade: the feature pass (no
 * symmetry test), the derivation of the 15 model inputs and the walk of the
 * default model's three trees (Section III-C-1, cascaded-prediction figure)
 * all run on the GPU, stream-ordered on s, with no host round trip; the
 * derivation is the host cascade's, so the outcome equals spmv_select on
 * ck_features_ex(CK_FEAT_NO_SYMMETRY).  Writes 8 int32 to DEVICE memory
 * d_out: format, algorithm, lanes, stages run (a ck_config), then the three
 * raw stage classes as ck_select_stages reports them, then the
 * configuration id.  Returns without blocking, except that the first call
 * on a device uploads the model's node tables.  The feature scratch is kept
 * with the handle (until spmv_destroy), so calls on one handle must be
 * ordered (one stream, or synchronised). */
ck_status ck_select_device(ck_handle h, int32_t *d_out, hipStream_t s);

/* ck_cascade_eval_device -- the same tree walk for `count` rows of 15 model
 * inputs (DEVICE array d_f15, row-major, feature-table order): d_ids[r] =
 * the configuration id the cascade picks for row r.  Stream-ordered. */
ck_status ck_cascade_eval_device(const double *d_f15, int64_t count, int32_t *d_ids,
                                 hipStream_t s);

/* ck_start_config -- the starting configuration from the inputs known
 * without a pass over the entries (nrows, ncols, nnz, density, mean row
 * length): the model's optional "start" tree, which names one of the CSR
 * configurations that need no copy of the matrix (ids 0..8: CSR-vector,
 * CSR-scalar, CSR-merge).  Without a start tree in the model, or for
 * nrows = 0, the default configuration below.  *from_tree (may be NULL) = 1
 * if the tree decided.  A known-features-only first stage, as the paper's
 * related work discusses for cheap, early decisions (Sections II-B, V). */
ck_status ck_start_config(int64_t nrows, int64_t ncols, int64_t nnz, const char *model_path,
                          ck_config *out, int32_t *from_tree);

/* ck_default_config -- the configuration a solve starts from before any
 * prediction: CSR-vector with lanes = clamp(2^floor(log2(max(1, nnz/nrows))),
 * 2, 64), which needs only the O(1) features. */
ck_status ck_default_config(ck_handle h, ck_config *out);

/* spmv_convert -- build the format `cfg` needs (Section III-C-1: a format
 * switch converts the matrix).  CSR needs nothing.  ELL: column-major,
 * K = longest row, pitch = nrows rounded up to 64, padding column -1 and
 * value +0.0; refused with CK_E_UNSUPPORTED when K*pitch > 8*nnz.  COO: a
 * row-index array (column and value arrays are shared with CSR).  CSR-panel:
 * panel-major copy of the column and value arrays, P column panels of
 * ceil(ncols/P) columns (see ck_panel_layout), with per-panel row pointers
 * (P*nrows + 1 int32), or, when at most 3/4 of the P*nrows panel rows hold
 * entries, pointers and matrix-row indices of the non-empty ones only.  DIA: the ndiag distinct offsets
 * col - row of the stored entries (int32, ascending) and ndiag*pitch values,
 * diagonal k of row i at k*pitch + i, +0.0 where no entry is stored
 * (pitch = nrows rounded up to 64); refused with CK_E_UNSUPPORTED when
 * ndiag*pitch > 8*nnz.  HYB: the ELL layout of width K = the largest k with
 * 3*#{rows of length >= k} >= nrows (Bell and Garland's rule), plus the
 * ascending list of rows longer than K (their entries K.. stay in the CSR
 * arrays).  A DIA product multiplies the +0.0 of an absent slot by x like
 * a stored value, so a non-finite x_j also reaches rows that store nothing
 * in column j.  Runs on s and returns when the copy is built (it then
 * serves any stream).  Idempotent. */
ck_status spmv_convert(ck_handle h, const ck_config *cfg, hipStream_t s);

/* ck_set_active / ck_get_active -- the configuration spmv_apply uses when
 * given NULL.  Setting a format that has not been converted gives
 * CK_E_INVALID. */
ck_status ck_set_active(ck_handle h, const ck_config *cfg);
ck_status ck_get_active(ck_handle h, ck_config *out);

/* spmv_apply -- y = alpha*A*x + beta*y (the SpMV kernel of every Krylov
 * iteration, Introduction).  cfg = NULL uses the active configuration; the
 * format it names must have been converted.  beta = 0: y is not read.
 * d_x has ncols entries, d_y nrows; they must not overlap.  Asynchronous:
 * enqueued on s, returns at once. */
ck_status spmv_apply(ck_handle h, const ck_config *cfg, double alpha, const double *d_x,
                     double beta, double *d_y, hipStream_t s);

/* spmv_apply_noalloc -- spmv_apply that allocates nothing, for callers that
 * cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid allocation).  Same arguments, result and
 * kernels as spmv_apply.  The workspace of the configurations that need one
 * (CSR-merge and COO carries, CSR-panel partial vectors) comes from a fixed
 * 64 MiB device array inside the library, one per GPU, held until the
 * process ends; a product that would need more returns CK_E_UNSUPPORTED
 * (CSR-merge and COO always fit; CSR-panel fits while panels x nrows x 8
 * bytes stays well under 64 MiB).  The first call on a device looks the
 * array's address up (no allocation).  Every call on one GPU shares that
 * array: calls that overlap on one GPU (on different streams, or from
 * different threads without ordering) race and must not be issued.  The
 * format `cfg` names must have been converted beforehand (spmv_convert
 * allocates). */
ck_status spmv_apply_noalloc(ck_handle h, const ck_config *cfg, double alpha, const double *d_x,
                             double beta, double *d_y, hipStream_t s);

/* spmv_apply_f32 -- the same product on the FP32 copy of the values (handle
 * created with CK_KEEP_FP32), FP32 vectors and FP32 accumulation. */
ck_status spmv_apply_f32(ck_handle h, const ck_config *cfg, float alpha, const float *d_x,
                         float beta, float *d_y, hipStream_t s);

/* cg_solve -- conjugate gradient (Hestenes-Stiefel) for SPD A, x0 in d_x
 * (Introduction names CG as one of the two target solvers).  Stops when the
 * recurred residual reaches opts->tol, then confirms on the true residual
 * b - A x, restarting from the current x (at most 3 times) if needed.
 * p.Ap <= 0 gives CK_E_BREAKDOWN.  opts->async = 1 runs the asynchronous
 * executor (Section III-C-2).  MIXED precision: FP64 refinement around FP32
 * CG segments.  Blocks until the result is final; d_x then holds x.
 * Small systems run in one launch: FP64 solves of at most 4096 rows with
 * neither async nor use_config run on a single 1024-thread workgroup whose
 * product takes one lane per row (final_config reports CSR-vector with 1
 * lane; known_start does not change this path); other systems of at most 16384 rows with a CSR-vector configuration
 * and no async run on the request loop's batched kernel. */
ck_status cg_solve(ck_handle h, const double *d_b, double *d_x, const ck_solve_opts *opts,
                   ck_solve_result *res, hipStream_t s);

/* gmres_solve -- restarted GMRES(m), x0 in d_x, no preconditioner (the
 * solver of the paper's evaluation, Section IV).  Each cycle starts from the
 * true residual; Arnoldi uses classical Gram-Schmidt applied twice; the
 * Givens least-squares update runs on the device.  MIXED precision: each
 * FP64 refinement step runs one FP32 GMRES(m) cycle on r/||r||.  Systems of
 * at most 16384 rows with a CSR-vector configuration, m <= 32 and no async
 * run in one launch of the request loop's batched kernel. */
ck_status gmres_solve(ck_handle h, const double *d_b, double *d_x, const ck_solve_opts *opts,
                      ck_solve_result *res, hipStream_t s);

/* ck_export_ell -- copy the ELL arrays (after spmv_convert to ELL) into
 * caller buffers d_col int32[K*pitch], d_val double[K*pitch]; with NULL
 * buffers only *K and *pitch are returned. */
ck_status ck_export_ell(ck_handle h, int32_t *d_col, double *d_val, int64_t *K,
                        int64_t *pitch, hipStream_t s);

/* ck_overhead_gate -- the overhead-aware conversion rule on host values
 * (host only; the asynchronous executor applies the same rule to the
 * latest report at iteration >= 8 and the latest report at least 4
 * iterations before it): from two residual reports (iteration t0, relative
 * residual r0) and (t1, r1), t0 < t1, *remaining = 2 (t1 - t0)
 * ln(tol / r1) / ln(r1 / r0), twice the iterations the geometric decay
 * needs from r1 down to tol (a Krylov residual falls fastest early; 0 if
 * r1 <= tol, 1e9 if the residual did not decrease); *cost = the modelled
 * bytes of the conversion to `target` over one product's bytes, plus 2
 * (features f give the sizes); *convert = 1 iff 0.25 * remaining >= cost. */
ck_status ck_overhead_gate(const ck_features *f, const ck_config *target, int32_t t0, double r0,
                           int32_t t1, double r1, double tol, double *remaining, double *cost,
                           int32_t *convert);

/* ck_export_dia -- after spmv_convert to DIA: *ndiag and *pitch, and (if
 * non-NULL) the offsets into d_off int32[ndiag] and the values into d_val
 * double[ndiag*pitch] (layout as spmv_convert describes). */
ck_status ck_export_dia(ck_handle h, int32_t *d_off, double *d_val, int64_t *ndiag,
                        int64_t *pitch, hipStream_t s);

/* ck_export_hyb -- after spmv_convert to HYB: the width *K, *pitch, the
 * number of long rows *ntail and the lanes per long row of the remainder
 * pass *lanes, and (if non-NULL) the ELL part into d_col int32[K*pitch] and
 * d_val double[K*pitch] and the long rows into d_rows int32[ntail]. */
ck_status ck_export_hyb(ck_handle h, int32_t *d_col, double *d_val, int32_t *d_rows, int64_t *K,
                        int64_t *pitch, int64_t *ntail, int32_t *lanes, hipStream_t s);

/* ck_export_coo_rows -- copy the COO row array (after spmv_convert to COO)
 * into d_row int32[nnz]. */
ck_status ck_export_coo_rows(ck_handle h, int32_t *d_row, hipStream_t s);

/* ck_panel_layout -- the CSR-panel copy's shape (after spmv_convert to
 * CSR-panel), to host memory: *panels = P, *width = columns per panel,
 * *stored_rows = panel rows kept (P*nrows in the dense layout, the number
 * of non-empty panel rows in the row-list one).  P is 8q with at most 2 MB
 * of FP64 x per panel, or 4 when x fits four slices of 2.5 MB, the longest
 * row is at most 4x ceil(nnz/nrows) and more than 3/4 of the 4*nrows panel
 * rows hold entries.  CK_E_INVALID without a CSR-panel copy. */
ck_status ck_panel_layout(ck_handle h, int32_t *panels, int64_t *width, int64_t *stored_rows);

/* ck_dot -- deterministic two-stage FP64 dot product of two device vectors
 * (the inner product kernel of the Krylov loop, Introduction); result to
 * the device scalar d_out.  Same inputs give the same bits on every call. */
ck_status ck_dot(int64_t n, const double *d_x, const double *d_y, double *d_out, hipStream_t s);

/* ck_config_id / ck_config_from_id -- number the 14 configurations 0..13:
 * CSR-vector lanes 1,2,4,...,64 = 0..6, CSR-scalar = 7, CSR-merge = 8,
 * ELL = 9, COO = 10, CSR-panel = 11, DIA = 12, HYB = 13.  Invalid input
 * gives -1 / CK_E_INVALID. */
int32_t ck_config_id(const ck_config *cfg);
ck_status ck_config_from_id(int32_t id, ck_config *out);

/* ck_kernel_name -- the device symbol of the SpMV kernel that a configuration
 * launches (for matching profiler output); fp32 selects the FP32 variant.
 * DIA's kernel is specialised for the matrix's diagonal count: its name ends
 * in ", ND>", ND being 3, 5, 7, 9, 13, 15, 19 or 27, or 0 for any other
 * count.  Writes a
 * NUL-terminated string of at most cap bytes. */
ck_status ck_kernel_name(const ck_config *cfg, int32_t fp32, char *buf, size_t cap);

/* ck_spmv_bytes -- algorithmic bytes of one product on this matrix:
 * nnz*(s+4) + 4*(nrows+1) + s*ncols + s*nrows [+ s*nrows if beta != 0],
 * s = 8 (FP64) or 4 (FP32).  Format padding is not counted. */
int64_t ck_spmv_bytes(ck_handle h, int32_t fp32, int32_t beta_nonzero);

/* ck_time_spmv -- the offline timing protocol (Section III-B-2: the time of
 * a configuration is the mean over repeated products): enqueue `warmup`
 * products, then `reps` products y = A x (alpha = 1, beta = 0) back to back
 * with configuration cfg on stream s, bracketed by HIP events recorded on s.
 * fp32 = 1 uses the FP32 values and float vectors.  Blocks; *us_per_call is
 * the mean microseconds per product over the reps.  The format must have
 * been converted (spmv_convert). */
ck_status ck_time_spmv(ck_handle h, const ck_config *cfg, int32_t fp32, const void *d_x,
                       void *d_y, int32_t warmup, int32_t reps, hipStream_t s,
                       double *us_per_call);

/* ---- Request loop (serving) ----------------------------------------------
 * Solve requests on a pool of registered matrices, processed by a scheduler
 * thread inside the library.  This is the iterative-solver use of the
 * method with many right-hand sides and matrices arriving over time: every
 * matrix gets its features and cascaded prediction once (then cached), stays
 * resident in device memory while the budget allows (least-recently-used
 * idle matrices are evicted), and its requests run either in a slot of a
 * batched kernel (n <= small_n: one workgroup per system, chunk_iters
 * iterations per launch, new requests joining between launches) or as a
 * full cg_solve / gmres_solve on a worker stream.  Symmetric matrices are
 * solved with CG, the others with GMRES(restart).  x0 = 0.  Admission is in
 * arrival order within each of the two paths; a request waiting only for a
 * free slot or worker does not hold back the other path, and one waiting for
 * memory holds back both.  The budget covers resident matrices (with their
 * converted copies: a decision whose copy does not fit runs the default
 * configuration) and request workspaces; idle matrices are evicted least
 * recently used first.  A request that does not fit even when nothing else
 * is in flight completes at once with status CK_E_NOMEM. */
typedef struct ck_server *ck_server_t;

typedef struct {
    int64_t budget_bytes;    /* device memory for resident matrices + workspaces   */
    int32_t max_slots;       /* batched slots (<= 4096)                             */
    int32_t chunk_iters;     /* iterations per slot per batched launch              */
    int32_t small_n;         /* systems with n <= small_n use the batched path      */
    int32_t large_workers;   /* concurrent large solves (1..16), one stream each    */
    int32_t precision;       /* CK_PREC_MIXED (FP32 inner, FP64 refinement) or FP64 */
    int32_t restart;         /* GMRES m (the batched path caps it at 32)            */
    int32_t max_iter;        /* per request; <= 0 means 100000                      */
    double tol;              /* ||b - A x|| / ||b|| target                          */
} ck_server_opts;

typedef struct {
    int64_t tag;             /* the caller's tag from ck_server_submit              */
    int32_t matrix_id, status, iterations;
    int32_t path;            /* 0 batched slot, 1 worker-stream solve               */
    int32_t config_id;       /* cached configuration of the matrix (ck_config_id)   */
    int32_t pad;
    double true_relres;      /* FP64 relative residual at exit                      */
    double t_submit_us, t_admit_us, t_done_us;   /* ck_server_clock_us() times     */
} ck_completion;

/* prediction_cache_hits counts admissions that found the matrix's features
 * and cascade decision already cached; prediction_cache_misses counts the
 * feature extractions and predictions actually run.  The latency fields
 * cover the completions since the server was created or since the last
 * ck_server_reset_stats (window_completed of them): latency = t_done_us -
 * t_submit_us of each completion; p50/p99 are its quantiles, interpolated
 * linearly between the closest ranks; solves_per_s = window_completed /
 * (latest t_done_us - earliest t_submit_us in the window).  Requests
 * completed with an error (e.g. CK_E_NOMEM) count too. */
typedef struct {
    int64_t submitted, completed, queued, in_flight, resident_matrices, evictions,
        bytes_in_use, batched_launches, prediction_cache_hits, prediction_cache_misses;
    int64_t window_completed;
    double p50_latency_us, p99_latency_us, solves_per_s;
} ck_server_stats;

/* ck_server_create -- start a request loop on the current device. */
ck_status ck_server_create(const ck_server_opts *opts, ck_server_t *out);
/* ck_server_add_matrix -- register a square CSR matrix under `id`.  The
 * device arrays stay owned by the caller and must outlive the server (an
 * evicted matrix is re-ingested from them). */
ck_status ck_server_add_matrix(ck_server_t s, int32_t id, int64_t n, int64_t nnz,
                               const int32_t *d_rowptr, const int32_t *d_col,
                               const double *d_val);
/* ck_server_submit -- enqueue a solve of A_id x = b; returns at once.  d_b and
 * d_x (n doubles each) must stay valid until the completion is polled. */
ck_status ck_server_submit(ck_server_t s, int32_t matrix_id, const double *d_b, double *d_x,
                           int64_t tag);
/* ck_server_poll -- move up to cap completions into out; returns the count. */
int32_t ck_server_poll(ck_server_t s, ck_completion *out, int32_t cap);
/* ck_server_drain -- wait until every submitted request has completed. */
ck_status ck_server_drain(ck_server_t s, double timeout_s);
ck_status ck_server_get_stats(ck_server_t s, ck_server_stats *out);
/* ck_server_reset_stats -- start a new latency window (the counters of
 * ck_server_stats are not reset). */
ck_status ck_server_reset_stats(ck_server_t s);
/* ck_server_clock_us -- microseconds since the server was created. */
double ck_server_clock_us(ck_server_t s);
/* ck_server_destroy -- stop the loop, free everything (pending requests are
 * dropped). */
void ck_server_destroy(ck_server_t s);

/* ck_last_error -- message for the last non-OK status on this thread. */
const char *ck_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* CASKRYLOV_H */
