/*
 * sscs.h -- C ABI of libsscs, an MI355X (gfx950) implementation of the
 * per-iteration hot path of SuperSCS (Sopasakis, Menounou, Patrinos,
 * "SuperSCS: fast and accurate large-scale conic optimization", arXiv 1903.06477).
 *
 * Problem (Sec. III, problem (P)):   minimise <c, x>  subject to  b - A x = s,  s in K,
 * dual (Sec. III, problem (D)):      minimise <b, y>  subject to  y in K*,  A^T y + c = 0.
 * The solver applies Douglas-Rachford splitting to the homogeneous self-dual
 * embedding (Sec. III-A, IV-A, equation (drs)) with the SuperMann steps of
 * Algorithm 1 and the directions of Sec. IV-D (Algorithm 2, Anderson).
 *
 * Conventions for every entry point
 *   - Integers are int32 unless noted; reals are double at the boundary.
 *   - A is given in CSR, 0-based, column indices sorted and in range, no duplicates.
 *   - Rows of A, b, s and y are ordered by cone block:
 *         zero (z rows) | R+ (l rows) | SOC q[0] | ... | PSD s[0] | ... | exp (3 each)
 *     SOC blocks are (x, t) with t LAST (Sec. II (iii)).
 *     PSD blocks of order k hold k(k+1)/2 entries: the column-major lower
 *     triangle of the symmetric matrix with off-diagonal entries multiplied by
 *     sqrt(2), i.e. the inverse of the paper's mat operator (Sec. II (ii)).
 *     exp blocks are (x1, x2, x3) in cl{x1 >= x2 exp(x3/x2), x2 > 0} (Sec. II (v)).
 *   - The HSDE state u = (chi, psi, tau) has length N = n + m + 1 (Sec. III-A).
 *   - Ownership: inputs are borrowed for the duration of a call; create copies
 *     (uploads) them, so the caller may free them afterwards.  Outputs are
 *     caller-allocated.  Workspaces are library-owned and released by destroy.
 *     The library never frees caller memory.
 *   - Vector arguments of solve / component entry points live on the host,
 *     or on the device when settings.data_on_device is non-zero.
 *   - Every call is enqueued on the stream given at create (NULL: the null
 *     stream) and returns after that stream has finished the call's work.
 *     One workspace may be used by one thread at a time.
 *   - Return value: SSCS_OK (0) or a negative error code.  No C++ exception
 *     crosses the ABI.  sscs_error_string() describes a code; after
 *     SSCS_E_HIP it also names the last HIP error seen by the library.
 */
#ifndef SSCS_H
#define SSCS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Error codes. */
#define SSCS_OK              0
#define SSCS_E_INVALID      (-1)  /* bad sizes, cone sizes not summing to m, bad CSR, bad settings */
#define SSCS_E_NOMEM        (-2)  /* device or host allocation failed */
#define SSCS_E_HIP          (-3)  /* a HIP runtime call failed */
#define SSCS_E_UNSUPPORTED  (-4)  /* valid input this build does not handle */
#define SSCS_E_DEVICE       (-5)  /* the device engine reported an internal failure
                                     (for example a grid barrier that did not complete) */

/* Solver outcome, info.status (Sec. IV-C; "no conclusion" cases map to the limits). */
#define SSCS_SOLVED          1
#define SSCS_INFEASIBLE      2
#define SSCS_UNBOUNDED       3
#define SSCS_MAX_ITERS       4
#define SSCS_TIME_LIMIT      5
#define SSCS_NUMERICAL       6

/* Directions (Sec. IV-D). */
#define SSCS_DIR_RB          0   /* modified restarted Broyden, Algorithm 2 */
#define SSCS_DIR_AA          1   /* Anderson's acceleration */
#define SSCS_DIR_RESIDUAL    2   /* d = -R u (K0 with c0 = 1 gives plain DRS) */
#define SSCS_DIR_ZERO        3   /* d = 0: every step is the hyperplane (K2) step */
#define SSCS_DIR_AA_QR       5   /* Anderson's acceleration with t from an updated QR
                                    factorisation of Xi (Sec. IV-D-2) */
#define SSCS_DIR_SCS         4   /* not Algorithm 1: SCS's splitting, Douglas-Rachford on
                                    N_C + Q (Sec. IV-A) relaxed by lambda, no SuperMann
                                    steps; the state is z, the candidate Pi_C(z) */

/* Precision of the linear step (Sec. IV-A, indirect solve). */
/* Linear step (I + Q)^{-1} (Sec. IV-A): the reduced system I + A^T A of the
 * HSDE solved iteratively or directly. */
#define SSCS_LINSYS_CG       0   /* conjugate gradients, Jacobi preconditioned, warm-started */
#define SSCS_LINSYS_DIRECT   1   /* I + A^T A formed and factored (dense Cholesky L L^T) once
                                    on the device at create, and its inverse L^{-T} L^{-1}
                                    formed from the factor (n <= SSCS_DIRECT_NMAX, FP64,
                                    single instances); each linear step is then one dense
                                    product with it */
#define SSCS_DIRECT_NMAX  4096

#define SSCS_PREC_FP64       0   /* FP64 everywhere */
#define SSCS_PREC_MIXED      1   /* the CG iterations apply I + A^T A with FP32 copies of
                                    A's values (FP64 vectors, accumulation and scalar
                                    recurrences); each linear step's residual is recomputed
                                    with the FP64 operator and the CG restarted from it (up
                                    to four refinement rounds) until that FP64 residual
                                    meets the CG tolerance.  Projections, residuals,
                                    termination and directions stay FP64. */

/* Problem data (Sec. III, problem (P)).  Host pointers. */
typedef struct {
    int32_t m, n;                 /* A is m x n */
    int64_t nnz;
    const int32_t *rowptr;        /* m + 1 entries */
    const int32_t *colind;        /* nnz entries, sorted within each row */
    const double  *val;           /* nnz entries */
    const double  *b;             /* m */
    const double  *c;             /* n */
} sscs_data;

/* Cone K as block sizes (Sec. II).  Host pointers. */
typedef struct {
    int32_t z;                    /* zero-cone rows; dual cone is the whole space */
    int32_t l;                    /* nonnegative-orthant rows */
    int32_t nq; const int32_t *q; /* second-order cone sizes, each >= 1, t last */
    int32_t ns; const int32_t *s; /* PSD orders k >= 1 (k(k+1)/2 rows each) */
    int32_t ep;                   /* number of exponential cones (3 rows each) */
} sscs_cone;

/* Settings: Algorithm 1 inputs c0, c1, q, sigma, lambda, epsilon; Sec. IV-D
 * parameters thetabar and mem; limits; linear-step options. */
typedef struct {
    double  eps;                  /* tolerance on pr, dr, gap, ic, uc (Sec. IV-C) */
    int32_t direction;            /* SSCS_DIR_* */
    int32_t mem;                  /* memory length, 1..16 */
    double  c0, c1, q, sigma, lambda, thetabar;
    int32_t ls_max;               /* backtracking cap; after it, u+ = u - lambda R u */
    int64_t max_iters;
    double  max_time_s;           /* <= 0: no time limit */
    int32_t precision;            /* SSCS_PREC_* */
    double  cg_tol;               /* relative residual tolerance of each CG solve */
    int32_t cg_max;               /* CG iteration cap per solve */
    int32_t data_on_device;       /* vector arguments are device pointers */
    int32_t record_trace;         /* keep per-iteration ||Ru|| and step kinds */
    double  aa_reg;               /* Anderson Gram regularisation, times tr(G)/k */
    double  cg_adapt;             /* 0: every CG solve to cg_tol; > 0: inexact linear steps,
                                     CG tolerance cg_adapt * ||R u|| / ||u|| clamped to
                                     [cg_tol, 1e-3] (the first solve uses 1e-6) */
    int32_t cg_d_match;           /* with cg_adapt > 0: 1 = the CG for the direction's
                                     linear step (d~ of Sec. IV-B) stops at the same absolute
                                     residual as that iteration's u~ solve, so the trial
                                     points u~ + alpha d~ carry the error of u~ alone;
                                     0 = at the relative tolerance of its own right-hand
                                     side (a much tighter absolute accuracy) */
    int32_t check_every;          /* termination test (Sec. IV-C) every check_every-th
                                     iteration and at the iteration cap; 0 or 1: every
                                     iteration.  A time limit is noticed at a tested
                                     iteration. */
    int32_t workgroups;           /* 0: the library sizes the grid; k >= 1: single-instance
                                     solves run on k workgroups (1: the one-workgroup
                                     kernel), capped by what stays co-resident.  Read at
                                     create; update_settings may not change it. */
    int32_t linsys;               /* SSCS_LINSYS_*; read at create, update_settings may not
                                     change it.  DIRECT: SSCS_E_UNSUPPORTED when n exceeds
                                     SSCS_DIRECT_NMAX, with SSCS_PREC_MIXED, for batches and
                                     for sscs_solve_noalloc; cg_* settings are then unused
                                     and cg_iters reports 0 */
} sscs_settings;

/* Result of a solve. */
typedef struct {
    int32_t status;               /* SSCS_SOLVED ... SSCS_NUMERICAL */
    int64_t iters;                /* iterations nu performed */
    int64_t k0, k1, k2, km;       /* accepted step kinds (km: backtracking cap reached) */
    int64_t backtracks;
    int64_t cg_iters;             /* total CG iterations */
    double  pr, dr, gap, ic, uc;  /* last termination measures (Sec. IV-C) */
    double  pobj, dobj;           /* <c,x> and -<b,y> of the returned triplet */
    double  res_fp;               /* ||R u|| at the last iterate */
    double  setup_s, solve_s;     /* wall time of create and of solve */
} sscs_info;

struct sscs_work;
struct sscs_batch;
typedef struct sscs_work  sscs_work;
typedef struct sscs_batch sscs_batch;

/* Fills *st with defaults: eps 1e-6, AA mem 5, c0 0.99 (0.1 is the paper's
 * advice for RB, Sec. IV-D-1), c1 0.9999, q 0.999, sigma 0.01, lambda 1.5,
 * thetabar 0.1, ls_max 10, FP64, cg_tol 1e-10, cg_max 500, aa_reg 1e-12,
 * cg_adapt 0, cg_d_match 1, check_every 1, workgroups 0, linsys CG.  Algorithm 1 leaves
 * c1, q and lambda open; with c1 = q = 0.99 and lambda = 1 Anderson can stall
 * in K2 steps and restarted Broyden in steps at the backtracking cap. */
int sscs_default_settings(sscs_settings *st);

/* Validates and uploads (A, b, c, K), builds A^T and the per-instance
 * constants of the linear step.  hip_stream is a hipStream_t or NULL.
 * SSCS_E_INVALID if the cone rows do not add up to m, CSR is malformed,
 * a cone size is < 1, or a setting is out of range. */
int sscs_create(const sscs_data *data, const sscs_cone *cone, const sscs_settings *st,
                void *hip_stream, sscs_work **out);

/* Runs Algorithm 1 from u0 (length N; NULL = cold start (0, 0, 1)).
 * Writes x (n), y (m), s (m): the candidate of Sec. IV-C when solved or
 * stopped, the normalised certificate y (<b,y> = -1) when infeasible, or
 * (x, s) with <c,x> = -1 when unbounded; unused outputs are NaN.
 * info may be NULL. */
int sscs_solve(sscs_work *w, const double *u0, double *x, double *y, double *s, sscs_info *info);

/* Replaces the settings used by later calls (same checks as create; the
 * precision cannot change after create). */
int sscs_update_settings(sscs_work *w, const sscs_settings *st);

/* Replaces b and c (lengths m and n) keeping A and K (a parametric family). */
int sscs_update_bc(sscs_work *w, const double *b, const double *c);

int sscs_destroy(sscs_work *w);

/* Component entry points, each one call of the device code the solve uses. */
/* out = (I + Q)^{-1} r, the linear step of equation (drs), r and out of length N. */
int sscs_linear_step(sscs_work *w, const double *r, double *out);
/* out = Pi_{K*}(in), in and out of length m (Sec. IV-A, projection step). */
int sscs_project_dual_cone(sscs_work *w, const double *in, double *out);
/* ut = (I + Q)^{-1} u and Ru = ut - Pi_C(2 ut - u) (R = I - T, Sec. IV-B), length N each.
 * ut may be NULL. */
int sscs_residual(sscs_work *w, const double *u, double *ut, double *Ru);
/* y = A x (transpose = 0, x of length n) or y = A^T x (transpose = 1, x of length m). */
int sscs_spmv(sscs_work *w, int32_t transpose, const double *x, double *y);
/* Repeats the SpMV of sscs_spmv reps times on device-resident buffers
 * (benchmarking); returns the elapsed milliseconds measured by HIP events
 * on the workspace stream. */
int sscs_spmv_bench(sscs_work *w, int32_t transpose, int32_t reps, double *ms);

/* Per-iteration record of the last solve (settings.record_trace != 0):
 * res[i] = ||R u^i||, kind[i] in {0:K0, 1:K1, 2:K2, 3:KM, -1: stopped},
 * ls[i] = backtracks, eta[i] and r_safe[i] = the safeguards of Algorithm 1
 * after the step of iteration i.  Copies min(cap, iterations + 1) records
 * into every non-NULL output (host arrays); *count gets the number available. */
int sscs_get_trace(sscs_work *w, int64_t cap, double *res, int32_t *kind, int32_t *ls,
                   double *eta, double *r_safe, int64_t *count);

/* Batched solves: count independent instances in one persistent launch, one
 * workgroup per instance taken from a device work queue.  Instances whose
 * rowptr, colind and val pointers equal those of instance 0 share one device
 * copy of A.  Packed vectors concatenate per-instance vectors in instance
 * order (u0: N_i each; x: n_i; y, s: m_i).  Settings (including
 * data_on_device) are shared; settings.workgroups does not apply.  The
 * batched engine runs the FP64 operator (SSCS_E_UNSUPPORTED for
 * SSCS_PREC_MIXED).  PSD blocks of a batched instance are limited to order 64
 * (SSCS_E_UNSUPPORTED above).  Each instance's time limit (max_time_s) runs
 * from the moment a workgroup takes it from the queue. */
int sscs_batch_create(int32_t count, const sscs_data *data, const sscs_cone *cones,
                      const sscs_settings *st, void *hip_stream, sscs_batch **out);
/* Replaces b and c of every instance (packed like y and x). */
int sscs_batch_update_bc(sscs_batch *bt, const double *b_packed, const double *c_packed);
int sscs_batch_solve(sscs_batch *bt, const double *u0_packed, double *x_packed,
                     double *y_packed, double *s_packed, sscs_info *infos);
int sscs_batch_destroy(sscs_batch *bt);
/* Tunes the batch's SpMV segment width (lanes per row; Sec. IV-A's products
 * by A and A^T inside the linear step) by timing, per size class: instances
 * are classed by the width the mean-row-length rule gives their A (a power
 * of two in 1..64); each class runs alone for `iters` iterations (cold
 * start, eps 0 so that none stops early) at that width times 1/4, 1/2, 1, 2
 * and 4 (powers of two within 1..64, A^T's width scaled alike), twice each,
 * and keeps the fastest; later sscs_batch_solve calls use the kept widths.
 * The timing runs' results are discarded.  Outputs (host): *n_classes; for
 * class c < min(cap, *n_classes), in increasing rule width: class_seg[c] =
 * the rule's width, chosen_seg[c] = the kept width, ms[5 c + j] = the better
 * time in ms of candidate j (factor 2^(j-2); -1 outside 1..64).  class_seg,
 * chosen_seg and ms may be NULL.  Returns SSCS_E_INVALID for iters < 1. */
int sscs_batch_autotune(sscs_batch *bt, int32_t iters, int32_t cap, int32_t *n_classes,
                        int32_t *class_seg, int32_t *chosen_seg, double *ms);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): one
 * instance solved by the batched engine exactly as sscs_batch_create +
 * sscs_batch_solve + sscs_batch_destroy would solve it as a batch of one,
 * with every device buffer (A and its transpose, b, c, the cone tables, the
 * iteration vectors, the queue and the result) carved from a static 32 MiB
 * device array instead of allocated.  Arguments are those of sscs_create and
 * sscs_solve: data and cone are host arrays; u0 (may be NULL), x, y, s are
 * host arrays, or device arrays when st->data_on_device is set.
 * SSCS_E_UNSUPPORTED when the instance does not fit the 32 MiB (about
 * 12 nnz(A) * 2 + 8 (2 mem + 16) (n + m) bytes), for PSD orders above 64 and
 * for mixed precision.  Calls no hipMalloc / hipFree.  Each GPU holds one
 * copy of the array until the process ends and every call on that GPU uses
 * it, so calls that overlap on one GPU race: one call at a time per GPU.
 * Work is enqueued on hip_stream and the call returns after it finished. */
int sscs_solve_noalloc(const sscs_data *data, const sscs_cone *cone, const sscs_settings *st,
                       void *hip_stream, const double *u0, double *x, double *y, double *s,
                       sscs_info *info);

const char *sscs_error_string(int code);

#ifdef __cplusplus
}
#endif

#endif /* SSCS_H */
