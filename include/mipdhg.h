/*
 * mipdhg: restarted PDHG for standard-form linear programs on one MI355X.
 *
 * Problem (paper, Section 2):  min c^T x  s.t.  A x = b, x >= 0, with A of
 * size m x n; its dual is max b^T y s.t. A^T y + z = c, z >= 0.  The solver
 * returns (x, y, z), the residuals r_P = b - A x and r_D = c - A^T y - z, and
 * stops when the three relative tests of Section 2 hold:
 *     ||r_P||_2 <= eps (1 + ||b||_2),  ||r_D||_2 <= eps (1 + ||c||_2),
 *     |c^T x - b^T y| <= eps (1 + |c^T x| + |b^T y|).
 * The tests and every reported figure are computed in float64 on the original
 * (unscaled) model, as Sections 2.1 and 4.3 ask, whatever the precision of the
 * iterations.  z is max(c - A^T y, 0), the z >= 0 that minimises ||r_D||.
 * The general form Section 2 mentions (bounds lo <= x <= hi, rows of sense
 * =, >= or <=) is accepted through the optional fields of mipdhg_lp and
 * handled implicitly; the quantities above then take their general-form
 * meaning (see mipdhg_lp and mipdhg_solve).  Infeasible and unbounded LPs are
 * reported through certificate tests (see infeas_tol).
 *
 * The PDHG itself (Section 4.1 only says it follows cuPDLP+) is: diagonal
 * scaling (Ruiz infinity-norm passes plus one Pock-Chambolle pass), a constant
 * step from a power-iteration estimate of ||A||_2, a primal weight re-balanced
 * at restarts (smoothed, or by a PID controller), reflected Halpern
 * iterations, and fixed-point-residual restarts.  A stopped solve can be
 * resumed from its workspace (option resume).
 *
 * Conventions for every entry point
 *  - All array arguments are DEVICE pointers (hipMalloc'd or torch tensors on
 *    the current HIP device) owned by the caller; the library neither frees nor
 *    retains them.  Structs (mipdhg_lp, mipdhg_options, mipdhg_info) live in
 *    host memory.  `stream` is a hipStream_t (NULL = the legacy default
 *    stream); all device work is enqueued on it.
 *  - Calls are synchronous with respect to the host: they return when the
 *    results are in the output buffers.
 *  - Inputs are float64 with int32 CSR indices (so nnz < 2^31).  A is CSR with
 *    m rows; the caller also passes A^T as CSR with n rows (the same matrix,
 *    transposed).  Column indices need not be sorted; duplicates are not
 *    allowed.
 *  - Return value >= 0 is a solver status (MIPDHG_OPTIMAL ...
 *    DUAL_INFEASIBLE); the outputs then hold the last evaluated point and
 *    info is filled.  A
 *    negative value is an error: no output is written, and
 *    mipdhg_last_error() returns a message (thread-local).
 *  - Re-entrant for distinct workspaces; two calls that share a workspace must
 *    not overlap.
 */
#ifndef MIPDHG_H
#define MIPDHG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* solver status (>= 0) */
#define MIPDHG_OPTIMAL 0         /* the three tests hold at eps_rel            */
#define MIPDHG_ITER_LIMIT 1      /* max_iter reached                           */
#define MIPDHG_TIME_LIMIT 2      /* time_limit_s reached                       */
#define MIPDHG_NUMERICAL 3       /* a NaN/Inf appeared in an evaluation        */
#define MIPDHG_PRIMAL_INFEASIBLE 4 /* the change of the evaluated y since the
                                    previous evaluation is a Farkas ray (see
                                    infeas_tol)                                */
#define MIPDHG_DUAL_INFEASIBLE 5   /* the change of the evaluated x is a
                                    recession direction with c^T d < 0        */
#define MIPDHG_IN_PROGRESS 6       /* batched solve: the instance used up this
                                    call's block of iterations
                                    (batch_block_iters); its state is in the
                                    workspace and a call with resume = 1
                                    continues it                              */
/* errors (< 0) */
#define MIPDHG_ERR_INVALID_ARG -1   /* null pointer, bad size or option       */
#define MIPDHG_ERR_BAD_CSR -2       /* row pointers or column indices invalid */
#define MIPDHG_ERR_TRANSPOSE -3     /* A^T is not the transpose of A          */
#define MIPDHG_ERR_HIP -4           /* a HIP runtime call failed              */
#define MIPDHG_ERR_WORKSPACE -5     /* workspace smaller than required        */
#define MIPDHG_ERR_UNSUPPORTED -6   /* option combination not supported       */
#define MIPDHG_ERR_NONFINITE -7     /* NaN/Inf in A, b or c                   */

/* iteration precision (storage of the scaled A values and of the iterate
 * vectors; the termination tests are float64 in every mode) */
#define MIPDHG_FP64 0        /* everything float64                                    */
#define MIPDHG_FP32 1        /* A values, x, y stored in float32; SpMV sums and the
                                per-row updates computed in float64, rounded once   */
#define MIPDHG_FP32_BF16A 2  /* as FP32, but the scaled A values stored as bfloat16   */
#define MIPDHG_FP32_ACC32 3  /* float32 storage AND float32 SpMV sums and updates     */
#define MIPDHG_FP32_A 4      /* A values stored in float32, iterate vectors, sums and
                                updates in float64 (reaches tighter tolerances than
                                FP32 at 4 more bytes per vector entry); single-LP
                                solve only                                           */

/* One LP in the standard form of Section 2, or in the general form that
 * section mentions (bounds on x and inequality rows, handled implicitly: the
 * primal step projects onto the bounds, the dual step keeps y_i >= 0 on >=
 * rows and y_i <= 0 on <= rows, and the evaluation measures each row's
 * violation, the reduced costs the bounds allow and the dual objective with
 * the bound terms).  Device pointers. */
#define MIPDHG_SENSE_EQ 0   /* (A x)_i = b_i  */
#define MIPDHG_SENSE_GE 1   /* (A x)_i >= b_i */
#define MIPDHG_SENSE_LE 2   /* (A x)_i <= b_i */
typedef struct mipdhg_lp {
    int32_t m, n;            /* rows and columns of A                      */
    int64_t nnz;             /* nonzeros of A (= of A^T)                   */
    const int32_t *a_rowptr; /* [m+1], a_rowptr[0] = 0, a_rowptr[m] = nnz  */
    const int32_t *a_col;    /* [nnz] column index of each entry, in [0,n) */
    const double *a_val;     /* [nnz]                                      */
    const int32_t *at_rowptr;/* [n+1] CSR of A^T                           */
    const int32_t *at_col;   /* [nnz] in [0, m)                            */
    const double *at_val;    /* [nnz]                                      */
    const double *b;         /* [m] right-hand side                        */
    const double *c;         /* [n] objective                              */
    /* General form: all three NULL is the standard form.  lo NULL means
     * x >= 0, hi NULL no upper bounds, sense NULL all equalities.  Bounds
     * may be infinite (lo = -INFINITY, hi = +INFINITY) but not NaN, with
     * lo < +inf, hi > -inf, lo <= hi; checked with `validate`
     * (INVALID_ARG).  Single-LP solve (tile kernels, spmv_kind 0 or 2) only. */
    const double *lo;        /* [n] lower bounds of x                      */
    const double *hi;        /* [n] upper bounds of x                      */
    const int8_t *sense;     /* [m] MIPDHG_SENSE_* of each row             */
} mipdhg_lp;

/* Options.  Fill with mipdhg_default_options() and change what you need. */
typedef struct mipdhg_options {
    int32_t precision;      /* MIPDHG_FP64 / FP32 / FP32_BF16A / FP32_ACC32 [0] */
    int32_t ruiz_iters;     /* Ruiz infinity-norm passes                  [10] */
    int32_t pock_chambolle; /* one Pock-Chambolle (alpha=1) pass after     [1] */
    int32_t power_iters;    /* power iterations for ||A~||_2             [100] */
    int32_t eval_every;     /* iterations between evaluations             [64] */
    double step_safety;     /* eta = step_safety / sigma_hat            [0.95] */
    double reflect_rho;     /* reflection in [0,1]                       [1.0] */
    int32_t halpern;        /* Halpern anchoring on/off                    [1] */
    int32_t restarts;       /* restarts on/off                             [1] */
    double beta_suff;       /* restart if R <= beta_suff R0              [0.2] */
    double beta_nec;        /* ... or R <= beta_nec R0 and R > R_prev    [0.8] */
    double beta_art;        /* ... or epoch length >= beta_art t        [0.36] */
    double pw_theta;        /* primal-weight smoothing                   [0.5] */
    int64_t max_iter;       /* iteration limit                       [1000000] */
    double time_limit_s;    /* wall-clock limit, seconds (paper: 1e4)    [1e4] */
    int32_t validate;       /* check CSR, finiteness and A^T consistency   [1] */
    int32_t use_graph;      /* replay hipGraphs of eval_every iterations   [1] */
    int32_t spmv_kind;      /* iteration SpMVs: 0 = nnz-balanced LDS tiles, one
                               workgroup per tile; 1 = lane groups per row
                               (lanes_a/lanes_at); 2 = the same LDS tiles walked
                               by a persistent grid of resident workgroups;
                               3 = the dual step on a panel layout of A (row
                               groups of narrow column span, each panel of the
                               gathered vector staged in LDS, row sums per
                               panel added in panel order), the primal step on
                               A^T's LDS tiles as with 0; 4 = the dual step as
                               with 3 and the primal step on a row-panel
                               layout of A^T (groups of rows whose columns,
                               apart from a short common tail such as a
                               block-angular LP's linking rows, fit one
                               panel of LDS; every row summed whole and its
                               epilogue run where its sum ends; its layout
                               takes longer to build than 3's, so it pays on
                               long solves and the autotuner does not try
                               it); UNSUPPORTED when the matrix does not fit
                               the layouts                                 [0] */
    int32_t tile_nnz;       /* LDS tiles: nonzeros per tile, 256..8192 (0 = 2048) */
    int32_t tile_rows;      /* LDS tiles: rows per tile, 1..512 (0 = 512)           */
    int32_t short_row;      /* LDS tile row sums: 0 or -1 = every thread reduces an equal chunk of
                               the tile's products with a segmented scan across threads (default);
                               > 0 = rows up to this length summed by one thread each, longer
                               rows by a wavefront each */
    int32_t lanes_a;        /* lanes per row for A SpMVs (0 = planner)     [0] */
    int32_t lanes_at;       /* lanes per row for A^T SpMVs (0 = planner)   [0] */
    int32_t long_row;       /* rows longer than this use a whole wave (0 = planner) */
    int32_t kernel_timing;  /* per-launch durations of the primal/dual kernels in info:
                               1 = hipEvents around every launch of the solve (disables
                               graphs); 2 = after the solve, 256 back-to-back launches of
                               each kernel between two events (no per-launch event cost;
                               the solve's outputs are not changed)             [0] */
    /* Debug trace of the scaled iterates after each of the first trace_iters
     * iterations (device float64 arrays, row-major [trace_iters][n or m]):
     * the state (x, y) after the update and the projected point (x_hat, y_hat).
     * Any of the four may be NULL.  Tracing disables graphs. */
    int32_t trace_iters;    /*                                             [0] */
    double *trace_x, *trace_y, *trace_xhat, *trace_yhat;
    /* Optional warm start in the original space (device float64, may be NULL). */
    const double *x_init;   /* [n], must be >= 0 */
    const double *y_init;   /* [m] */
    /* Order of the nonzeros inside each LDS tile of the iteration's scaled
     * copies (spmv_kind 0 and 2): 0 = sorted by gather index, so that the
     * lanes of a load fall on few cache lines (costs 6 more workspace bytes
     * per nonzero and copy); 1 = row-major.  Results are bitwise identical. [0] */
    int32_t gather_order;
    /* 1 = continue the solve whose state the workspace holds (same LP, same
     * options but eps_rel, max_iter and time_limit_s; checked by a
     * fingerprint) instead of starting from (0, 0).  max_iter counts all
     * iterations, those already done included.  A solve stopped at an
     * evaluation (optimal or at its iteration limit) skipped that evaluation's
     * restart decision; it is taken again under the new tolerance, so a solve
     * stopped at a multiple of eval_every and resumed gives bitwise the
     * result of one uninterrupted solve with the resumed tolerance and limit.
     * The outputs are written at evaluations: a resumed solve whose first
     * decision already stops it leaves them as the stopped solve wrote them,
     * so pass the same output arrays.  A state that does not match (other
     * sizes, options, b or c norms or step size) is INVALID_ARG, and so is
     * one that stopped on non-finite values.  Not with x_init, y_init or
     * tracing; a kernel_timing = 2 solve is not resumable.  The batched
     * solve resumes too (see batch_block_iters); the unrolled entry points
     * do not (UNSUPPORTED).                                                 [0] */
    int32_t resume;
    /* Infeasibility certificates (the paper does not treat infeasible LPs;
     * this is the library's own test).  At every evaluation after the first,
     * with (d, e) the change of the evaluated (x, y) since the previous
     * evaluation: PRIMAL_INFEASIBLE when v = b^T e + sum_j lo_j mu_j^+ -
     * hi_j mu_j^- > 0 and || (-A^T e - mu, part of e outside its rows' sign
     * cones) || <= infeas_tol * v, with mu = -A^T e projected onto the
     * cones the bounds allow; DUAL_INFEASIBLE when c^T d < 0 and || (part of
     * A d outside the rows' recession cones, part of d outside the bounds'
     * recession cones) || <= infeas_tol * |c^T d|.  0 turns the tests off.
     * With float32 iterates (rounding ~6e-8 relative, growing with the
     * drifting iterate of an infeasible LP) use about 1e-5: at 1e-8 such a
     * run may drift until it overflows (NUMERICAL).
     * Single-LP solve only (the batched and unrolled solves ignore it). [1e-8] */
    double infeas_tol;
    /* Primal weight as a PID controller on e = log(omega) - log(dy/dx) at
     * each update: omega <- exp(log(omega) - (pw_theta e + pw_ki I +
     * pw_kd (e - e_prev))), I the sum of the errors so far (this one
     * included), e_prev the previous update's error (0 at the first).  Both
     * 0: the smoothing rule of pw_theta alone.                      [0, 0] */
    double pw_ki, pw_kd;
    /* LDS tiles of A^T (the primal SpMV and the column-side evaluation) when
     * they should differ from A's: 0 = the value of tile_nnz, tile_rows,
     * short_row.  mipdhg_autotune picks both sides.              [0, 0, 0] */
    int32_t tile_nnz_at, tile_rows_at, short_row_at;
    /* 1 = restart to the epoch's average: the projected points of the
     * current epoch are averaged (equal weights) and a restart moves the
     * state and the anchor to that average instead of the last projected
     * point; the primal-weight update measures the average's distances.  The
     * restart tests and the evaluated point are unchanged.  Meant with
     * halpern = 0; single-LP solve with spmv_kind 0 only.               [0] */
    int32_t restart_avg;
    /* spmv_kind 3: entries of the gathered vector one panel stages in LDS, a
     * power of two from 64 up to 128 KB worth (0 = 128 KB worth: 32,768 in
     * float32, 16,384 in float64); smaller panels exist to test the layout on
     * small matrices.                                                     [0] */
    int32_t panel_width;
    /* Step rule: 0 = eta = step_safety / sigma_hat from the power iteration,
     * held fixed; 1 = the adaptive step with rejection of PDLP, the solver
     * family Section 4.1 builds on: the step starts at 1 / max |A~_ij|, every
     * iteration is an attempt z' = T(z) with the current eta, accepted when
     * eta <= eta_bar = (omega ||x' - x||^2 + ||y' - y||^2 / omega) /
     * (2 |(y' - y)^T A~ (x' - x)|) and rejected (z unchanged) otherwise, and
     * the next attempt uses min((1 - (t + 1)^-0.3) eta_bar,
     * (1 + (t + 1)^-0.6) eta), t the attempt's 1-based number.  Attempts
     * count as iterations (limit, evaluations, restart rule); an evaluation
     * measures the current iterate and takes the fixed-point residual of its
     * attempt.  Needs plain PDHG (halpern 0, reflect_rho 0, restart_avg 0;
     * INVALID_ARG otherwise) and spmv_kind 0 (UNSUPPORTED otherwise); single-LP
     * solve only.                                                          [0] */
    int32_t step_rule;
    /* step_rule 1: the first step, > 0 (0 = 1 / max |A~_ij|)              [0] */
    double step0;
    /* Batched solve, > 0: two concurrent launches.  Instances whose y and
     * x_bar (the vectors kept in LDS) fit in batch_split bytes run in
     * 256-thread workgroups at the occupancy that size allows; the others
     * run in 1024-thread workgroups (four times the threads on each row and
     * column).  0 = one launch of 256-thread workgroups sized by the largest
     * instance.  The narrow class's results are bitwise those of the single
     * launch; the wide class sums over other thread partitions, so its
     * iterates agree to rounding.  mipdhg_autotune_batched picks the
     * fastest.                                                              [0] */
    int32_t batch_split;
    /* Batched solve, > 0: iterations per call.  Each unfinished instance
     * stops at its first evaluation at least batch_block_iters iterations
     * after it started in this call, saves its state (iterates, anchors,
     * primal weight, steps, restart bookkeeping, iteration count) in the
     * workspace and reports MIPDHG_IN_PROGRESS.  A call with resume = 1 on
     * the same batch, workspace, output arrays and options (eps_rel and
     * max_iter may change) continues every instance in progress, skips the
     * finished ones (their outputs and reports stand) and gives bitwise the
     * result of one uninterrupted solve.  A workspace that does not hold
     * this batch's state under these options (checked by a fingerprint of
     * the offsets and options) is INVALID_ARG, and the state is left as it
     * was.  A resumed call skips the device validation the first call did.
     * 0 = run every instance to the end.                                    [0] */
    int32_t batch_block_iters;
} mipdhg_options;

/* Per-solve report (host struct). */
typedef struct mipdhg_info {
    int32_t status;
    int32_t restarts;
    int64_t iters;          /* iteration t at which the returned point was evaluated */
    double rp_norm, rd_norm;/* ||r_P||_2, ||r_D||_2 on the original model          */
    double gap;             /* |c^T x - dobj|                                       */
    double pobj, dobj;      /* c^T x; b^T y (general form: plus the bound terms
                               sum_j lo_j z_j^+ - hi_j z_j^- over finite bounds)     */
    double rel_rp, rel_rd, rel_gap; /* the three ratios of Section 2 (<= eps: pass) */
    double rp_inf, rd_inf;  /* infinity norms                                       */
    double xz;              /* x^T z (general form: sum_j z_j^+ (x_j - lo_j) +
                               z_j^- (hi_j - x_j) over finite bounds)                */
    double max_violation;   /* max(rp_inf, rd_inf, xz / (1 + |c^T x|)), Section 4.3 */
    double b_norm, c_norm;  /* ||b||_2, ||c||_2                                     */
    double sigma_hat;       /* power-iteration estimate of ||D_r A D_c||_2 (0 with
                               step_rule 1, which runs no power iteration)           */
    double eta;             /* step, tau * sigma = eta^2 (step_rule 1: the step the
                               next attempt would take)                              */
    double omega0, omega;   /* initial and final primal weight                      */
    double ms_setup, ms_iter, ms_total; /* wall time: validation+scaling+step, loop, all */
    double bytes_per_iter;  /* algorithmic bytes of one iteration: A and A^T values and
                               indices, row pointers, each vector read or written once */
    double bytes_primal, bytes_dual; /* the same, split by kernel                     */
    double ms_primal, ms_dual;       /* with kernel_timing: mean duration per launch  */
    int64_t n_primal, n_dual;        /* with kernel_timing: launches timed            */
    int32_t lanes_a, lanes_at, long_a, long_at; /* SpMV plan used                   */
    double ms_graph;        /* part of ms_iter spent capturing and instantiating the
                               iteration block's hipGraph                            */
    int64_t rejected;       /* step_rule 1: attempts whose step was rejected        */
} mipdhg_info;

/* Fill `opt` with the defaults shown in brackets above. */
void mipdhg_default_options(mipdhg_options *opt);

/* Bytes of device workspace mipdhg_solve needs for this LP and options.
 * Returns 0 or MIPDHG_ERR_INVALID_ARG. */
int mipdhg_workspace_size(const mipdhg_lp *lp, const mipdhg_options *opt, size_t *bytes);

/* Solve one LP to eps_rel (Section 2 tests).  Outputs (device float64, all
 * required): x[n], y[m], z[n], r_p[m], r_d[n] in the original space.
 * General form: z = c - A^T y projected onto the cone the bounds allow
 * (free where both bounds are finite, >= 0 with only lo, <= 0 with only hi,
 * 0 if x_j is free), r_d = c - A^T y - z, and r_p_i is b_i - (A x)_i for
 * equality rows and its violating part (max(., 0) on >= rows, min(., 0) on
 * <= rows) otherwise.
 * d_row[m], d_col[n] (nullable): the scaling, D_r A D_c being the scaled
 * matrix the iterations run on; x~ = x / d_col, y~ = y / d_row, z~ = z * d_col
 * is the solution of the scaled LP that Algorithm 1 (Section 3.1) consumes.
 * `workspace` is a device buffer of at least mipdhg_workspace_size() bytes,
 * 256-byte aligned.  `info` (nullable) receives the report. */
int mipdhg_solve(const mipdhg_lp *lp, const mipdhg_options *opt, double eps_rel,
                 void *workspace, size_t workspace_bytes, void *stream,
                 double *x, double *y, double *z, double *r_p, double *r_d,
                 double *d_row, double *d_col, mipdhg_info *info);

/* Checkpoint of a solve (for the callers that want to keep a stopped solve
 * beyond its workspace, e.g. on disk): the part of the workspace that
 * options.resume continues from -- control block, iterates, anchors,
 * projected points, the previous evaluated point and the last evaluation's
 * partial sums -- for the LP sizes and options given (the same as the
 * solve's).  mipdhg_state_size gives its bytes; export copies it from a
 * workspace to `dst`, import from `src` into a workspace of at least
 * mipdhg_workspace_size() bytes; `dst`/`src` may be host or device memory.
 * After an import, mipdhg_solve with resume = 1 on the same LP and options
 * continues the exported solve as if it had never stopped (its outputs are
 * written at the next evaluation).  Both are synchronous on `stream`.
 * Errors: INVALID_ARG (NULL, buffer too small), WORKSPACE (too small), HIP. */
int mipdhg_state_size(const mipdhg_lp *lp, const mipdhg_options *opt, size_t *bytes);
int mipdhg_state_export(const mipdhg_lp *lp, const mipdhg_options *opt, const void *workspace,
                        size_t workspace_bytes, void *dst, size_t dst_bytes, void *stream);
int mipdhg_state_import(const mipdhg_lp *lp, const mipdhg_options *opt, void *workspace, size_t workspace_bytes,
                        const void *src, size_t src_bytes, void *stream);

/* Many independent LPs, stacked as the diagonal blocks of one block-diagonal
 * LP: instance i owns rows [row_off[i], row_off[i+1]), columns
 * [col_off[i], col_off[i+1]) and nonzeros [nnz_off[i], nnz_off[i+1]) of both
 * A and A^T, whose column indices are global (block-diagonal).  The offset
 * arrays are HOST arrays of count+1 entries starting at 0 and ending at m, n,
 * nnz of `whole`; every instance has at least one row and one column. */
typedef struct mipdhg_batch {
    int32_t count;
    const int32_t *row_off;  /* host [count+1] */
    const int32_t *col_off;  /* host [count+1] */
    const int64_t *nnz_off;  /* host [count+1] */
    mipdhg_lp whole;         /* device arrays of the block-diagonal LP */
} mipdhg_batch;

/* Bytes of device workspace mipdhg_solve_batched needs. */
int mipdhg_batch_workspace_size(const mipdhg_batch *batch, const mipdhg_options *opt, size_t *bytes);

/* Solve every instance i of the batch to its own eps_rel[i] (eps_rel: HOST
 * array of `count` tolerances, each finite and >= 0; the Section 2 tests,
 * each instance on its own norms), in one persistent kernel launch: one workgroup
 * per instance at a time, instances taken largest first from a queue, each
 * with its own scaling, step, primal weight, restarts and termination.
 * Outputs are the stacked per-instance vectors (device float64, same layout as
 * the rows/columns of `whole`): x[n], y[m], z[n], r_p[m], r_d[n].  info
 * (nullable) is a HOST array of `count` reports.  The return value is the
 * largest status over the instances (0 when all are OPTIMAL) or an error.
 * An instance needs (m_i + n_i) * sizeof(iterate) bytes of LDS, at most
 * 150 KiB; larger instances return MIPDHG_ERR_UNSUPPORTED.  Every precision
 * but FP32_A (UNSUPPORTED); as in the single-LP solve, each instance's
 * iteration is held relative to its epoch's anchor, whose residuals are
 * formed in float64 on `whole`.  Tracing, warm starts and kernel timing are
 * not available here.  With batch_block_iters
 * the solve runs in resumable blocks: the return value is
 * MIPDHG_IN_PROGRESS while any instance is unfinished. */
int mipdhg_solve_batched(const mipdhg_batch *batch, const mipdhg_options *opt, const double *eps_rel,
                         void *workspace, size_t workspace_bytes, void *stream,
                         double *x, double *y, double *z, double *r_p, double *r_d,
                         mipdhg_info *info);

/* ---- Differentiable unrolled PDHG (batched) ------------------------------
 * x_K(c, b): exactly K iterations of the solve's PDHG from (0, 0) on every
 * instance of `batch` (no termination test), x_K = D_c x_hat of iteration K
 * in the original space.  Restarts are decided by the usual rule at every
 * eval_every-th iteration and, with the per-epoch steps, recorded on the tape;
 * they are constants of the map, which is then piecewise linear in (c, b).
 * The tape (device, caller-owned, >= mipdhg_unrolled_tape_size bytes, 256-byte
 * aligned) also holds the scaling, the scaled values and a checkpoint of the
 * state every ckpt_every iterations; the backward pass recomputes each
 * checkpoint segment and sweeps it in reverse (the adjoint of the iteration
 * map, with the projection masks of the recomputed iterations).  b and c are
 * batch->whole.b / .c.  Instances must fit in LDS as for the batched solve. */
int mipdhg_unrolled_tape_size(const mipdhg_batch *batch, const mipdhg_options *opt, int32_t K,
                              int32_t ckpt_every, size_t *bytes);

/* Forward pass; writes x_K (device float64 [n]).  replay = 1 re-runs the map
 * with the restart schedule and steps already on the tape (for finite
 * differences of the frozen map) instead of deciding them. */
int mipdhg_unrolled_forward(const mipdhg_batch *batch, const mipdhg_options *opt, int32_t K,
                            int32_t ckpt_every, int32_t replay, void *tape, size_t tape_bytes,
                            void *stream, double *x_K);

/* Backward pass for a loss L with dL/dx_K = grad_xK (device float64 [n]):
 * writes dL/dc (device float64 [n]) and dL/db ([m]).  Needs the tape of the
 * forward pass with the same batch, options, K and ckpt_every. */
int mipdhg_unrolled_backward(const mipdhg_batch *batch, const mipdhg_options *opt, int32_t K,
                             int32_t ckpt_every, void *tape, size_t tape_bytes, const double *grad_xK,
                             void *stream, double *grad_c, double *grad_b);

/* The schedule a forward pass recorded on its tape for instance `inst`: the
 * iterations at which it restarted (HOST int32 restart_at, ascending) and
 * the step sizes (tau, sigma) of every epoch (HOST double taus, sigmas, one
 * more than the restarts); *n_restarts receives the count.  These are the
 * constants of the map the forward and backward passes differentiate; a
 * float64 reference run with them reproduces the map.  capacity is the
 * length of taus and sigmas (restart_at holds capacity - 1): INVALID_ARG if
 * the schedule has more epochs.  Copies from the tape on `stream` and waits. */
int mipdhg_unrolled_schedule(const mipdhg_batch *batch, const mipdhg_options *opt, int32_t K,
                             int32_t ckpt_every, const void *tape, size_t tape_bytes, int32_t inst,
                             void *stream, int32_t capacity, int32_t *restart_at, double *taus,
                             double *sigmas, int32_t *n_restarts);

/* ---- Centered warm start (Algorithm 1, Section 3.1) ----------------------
 * Maps a PDHG solution of the SCALED LP to the interior-point start (x', z')
 * (y passes through unchanged): mu_target = max(x^T z / n, mu_min); each pair
 * is lifted to alpha_min, then the smaller of x_j, z_j moves toward
 * mu_target / (the other) and the other toward mu_target / (the new value),
 * each by at most delta_max.  The paper's settings are mu_min = 1e-6,
 * delta_max = 1e-4, alpha_min = 1e-6.  If d_col (device [n]) is given, x and z
 * are original-space outputs of mipdhg_solve and are first scaled
 * (x~ = x / d_col, z~ = z * d_col); otherwise they are already scaled.
 * Outputs x_out, z_out (device [n]) are in the scaled space; mu_target (host,
 * nullable) receives the target.  workspace: device, 256-byte aligned, at
 * least mipdhg_center_workspace_size(n) bytes. */
size_t mipdhg_center_workspace_size(int32_t n);
int mipdhg_center_start(int32_t n, const double *x, const double *z, const double *d_col, double mu_min,
                        double delta_max, double alpha_min, void *workspace, size_t workspace_bytes,
                        void *stream, double *x_out, double *z_out, double *mu_target);

/* mipdhg_center_start without a workspace, for callers that cannot allocate
 * device memory (code under HIP graph capture, serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, kernels and results as
 * mipdhg_center_start; its scratch (partial sums, target, scaled copies) is a
 * fixed device array of the library, 33.6 MB, held by every GPU the library
 * runs on until the process ends.  n may be at most
 * mipdhg_center_noalloc_max_n() (2,097,152 pairs); larger n returns
 * MIPDHG_ERR_INVALID_ARG before any device work.  The call allocates nothing.
 * Calls on one GPU share its scratch array: calls that overlap on one GPU
 * (from several threads or streams) race and must be serialised by the
 * caller; sequential calls are independent (nothing in the scratch is read
 * before it is written). */
int32_t mipdhg_center_noalloc_max_n(void);
int mipdhg_center_start_noalloc(int32_t n, const double *x, const double *z, const double *d_col, double mu_min,
                                double delta_max, double alpha_min, void *stream, double *x_out, double *z_out,
                                double *mu_target);

/* The re-clamp of Algorithm 1's recovery loop (run after the caller has
 * raised alpha_min tenfold because the interior-point step was too small):
 * x_j <- max(x_j, alpha_min), z_j <- max(z_j, alpha_min), in place. */
int mipdhg_center_reclamp(int32_t n, double alpha_min, void *stream, double *x_io, double *z_io);

/* sizeof of the public structs, for bindings that mirror them:
 * which = 0 mipdhg_lp, 1 mipdhg_options, 2 mipdhg_info, 3 mipdhg_batch,
 * 4 mipdhg_ipm_options, 5 mipdhg_ipm_info; 0 for anything else. */
size_t mipdhg_sizeof(int which);

/* Times every candidate shape of the two iteration SpMVs on this LP (lane
 * groups; LDS tiles of 1024..8192 nonzeros, 256 or 512 rows, chunked or
 * short-row-32 sums, one workgroup per tile or persistent; tiles sized
 * so that their count is 4..8 per compute unit, from the row pointers; the
 * dual step on A's panel layout, spmv_kind 3, whose primal step is kind 0's
 * and takes kind 0's fastest primal shape, and whose A tiles, which the
 * power iteration and the evaluations still use, take kind 0's fastest dual
 * shape): each
 * runs `iters` iterations, then 256 back-to-back launches of each kernel
 * timed with hipEvents (kernel_timing = 2).  For each spmv_kind it takes
 * the fastest shape of the dual kernel (A's tiles) and of the primal kernel
 * (A^T's tiles) separately, and writes the kind with the smallest sum into
 * opt (spmv_kind, tile_nnz, tile_rows, short_row for A, the *_at fields for
 * A^T).  A side keeps the default shape (2,048 nonzeros, 512 rows, chunked
 * sums) unless another is more than 3 % faster, so that the choice does not
 * flip with timing noise.  best_ms (host, nullable) receives that primal +
 * dual time per iteration.  Arguments as for mipdhg_solve, whose output buffers are used as
 * scratch; candidates whose workspace does not fit are skipped, so a
 * workspace that runs all of them holds the larger of
 * mipdhg_workspace_size() of opt with tile_nnz = 512, tile_rows = 256 (the
 * smallest tiles) and with spmv_kind = 3 (the panel layout). */
int mipdhg_autotune(const mipdhg_lp *lp, mipdhg_options *opt, int32_t iters, void *workspace,
                    size_t workspace_bytes, void *stream, double *x, double *y, double *z, double *r_p,
                    double *r_d, double *best_ms);

/* mipdhg_autotune with its choice cached by matrix signature: the device
 * (architecture and compute units), the precision and the options that change
 * the candidates, m, n, nnz, and the sparsity structure (hashes of the row
 * pointers and column indices of A and A^T; the values do not enter).  A
 * signature seen before in this process, or found in the text file cache_path
 * (nullable; one line per signature, the last line of a signature wins),
 * fills opt without timing anything (*hit = 1); otherwise the tuner runs, and
 * its choice is kept for the process and appended to cache_path (*hit = 0).
 * Arguments otherwise as for mipdhg_autotune (the first 8 bytes of the
 * workspace are used for the hash). */
int mipdhg_autotune_cached(const mipdhg_lp *lp, mipdhg_options *opt, int32_t iters, const char *cache_path,
                           void *workspace, size_t workspace_bytes, void *stream, double *x, double *y, double *z,
                           double *r_p, double *r_d, double *best_ms, int32_t *hit);

/* ------------------------------------------------------------------------
 * Interior-point consumer of the centered start (Section 3.1).  The paper
 * warm-starts a barrier solver from Algorithm 1's point and counts its
 * iterations (Section 4.6).  This one is Mehrotra's primal-dual
 * predictor-corrector on the scaled LP min c~^T x, A~ x = b~, x >= 0
 * (A~ = D_r A D_c, b~ = D_r b, c~ = D_c c; D_r, D_c as mipdhg_solve returns
 * them, NULL for ones): normal equations (A~ X Z^-1 A~^T) dy = rhs formed
 * dense on the device and factored by Cholesky (a pivot that is not positive
 * is replaced by 1e128 and counted), the predictor and corrector sharing the
 * factor, steps step_frac of the way to the boundary (at most 1), separate
 * for x and for (y, z); it stops when the three relative tests of Section 2
 * hold at tol on the scaled LP.  Standard form, m <= 16384 (the dense matrix);
 * A's rows must list their columns in increasing order.  Device pointers,
 * float64; the workspace is 256-byte aligned, of mipdhg_ipm_workspace_size()
 * bytes or more.  Returns the status (MIPDHG_OPTIMAL, MIPDHG_ITER_LIMIT,
 * MIPDHG_NUMERICAL) or a negative error. */
typedef struct mipdhg_ipm_options {
    double tol;           /* the relative tests of Section 2 on the scaled LP   [1e-8]   */
    int32_t max_iter;     /* Newton steps                                        [100]    */
    int32_t max_lifts;    /* warm start: tenfold raises of alpha_min at most     [12]     */
    double step_frac;     /* fraction of the step to the boundary, in (0, 1)     [0.9995] */
    double min_step;      /* warm start: a first step min(a_p, a_d) below this
                             raises alpha_min (Section 3.1: 1e-6)                [1e-6]   */
    double mu_min, delta_max, alpha_min; /* Algorithm 1's parameters   [1e-6, 1e-4, 1e-6] */
} mipdhg_ipm_options;

typedef struct mipdhg_ipm_info {
    int32_t status;       /* as returned                                                 */
    int32_t iters;        /* Newton steps of the run that was kept                       */
    int32_t lifts;        /* warm start: tenfold raises of alpha_min                     */
    int32_t pivots_replaced;
    double alpha_min;     /* warm start: the value the kept run started from             */
    double mu_target;     /* warm start: Algorithm 1's mu_target                         */
    double first_step_p, first_step_d; /* the first iteration's steps                   */
    double rel_rp, rel_rd, rel_gap;    /* the three relative measures at the end (scaled) */
    double pobj, dobj;    /* c~^T x~ = c^T x and b~^T y~ = b^T y at the end              */
    double mu;            /* x^T z / n at the end (scaled)                               */
    double ms_total;      /* wall time of the call                                       */
} mipdhg_ipm_info;

void mipdhg_ipm_default_options(mipdhg_ipm_options *opt);
int mipdhg_ipm_workspace_size(const mipdhg_lp *lp, size_t *bytes);

/* From the scaled-space point (x_start, y_start, z_start), x, z > 0, or from
 * Mehrotra's heuristic point when all three are NULL (cold start).  Outputs
 * x, y, z (n, m, n) in the original space: x = D_c x~, y = D_r y~,
 * z = z~ / D_c. */
int mipdhg_ipm_solve(const mipdhg_lp *lp, const double *d_row, const double *d_col, const double *x_start,
                     const double *y_start, const double *z_start, const mipdhg_ipm_options *opt, void *workspace,
                     size_t workspace_bytes, void *stream, double *x, double *y, double *z, mipdhg_ipm_info *info);

/* The hybrid of Section 3.1 from a PDHG solution (x, y, z) in the original
 * space (as mipdhg_solve returns it, with its d_row, d_col): Algorithm 1's
 * centered point (x', y / D_r, z') of the scaled point, then the
 * interior-point method from it; while the first step of a run is below
 * min_step, alpha_min grows tenfold (at most max_lifts times), x' and z' are
 * lifted to it, and the method runs again from the lifted point.  Outputs
 * and result as for mipdhg_ipm_solve. */
int mipdhg_ipm_warm(const mipdhg_lp *lp, const double *d_row, const double *d_col, const double *x_pdhg,
                    const double *y_pdhg, const double *z_pdhg, const mipdhg_ipm_options *opt, void *workspace,
                    size_t workspace_bytes, void *stream, double *x, double *y, double *z, mipdhg_ipm_info *info);

/* Not an operation of the method: a plain streaming read of `bytes` bytes of
 * device memory at buf (16-byte aligned, a positive multiple of 16), with the
 * non-temporal 16-byte vector loads the SpMV kernels stream their matrices
 * with, by `blocks` workgroups of 256 threads on `stream`.  It writes one
 * 32-bit word per wave (blocks * 4 words) to the device array out, the XOR of
 * the words the wave read.  Timed, it gives the read rate a kernel reaches on
 * the device, the ceiling the iteration kernels are measured against; under
 * a hardware counter it gives the counter's reading for a known number of
 * bytes read.  Asynchronous; INVALID_ARG on a bad argument. */
int mipdhg_read_probe(const void *buf, size_t bytes, int32_t blocks, void *stream, uint32_t *out);

/* Times mipdhg_solve_batched on this batch with each candidate batch_split
 * (0, 2, 4, 8, 16, 32 KB: one launch, or the instances whose vectors fit the
 * budget in narrow workgroups beside wide workgroups for the others) and
 * writes the fastest into opt->batch_split (0 kept unless another is more
 * than 3 % faster).  The candidates' results agree to rounding (bitwise for
 * the narrow class); the outputs hold the last candidate's.  Arguments as for
 * mipdhg_solve_batched; best_ms (host, nullable) receives the chosen
 * candidate's kernel time. */
int mipdhg_autotune_batched(const mipdhg_batch *bt, mipdhg_options *opt, const double *eps_rel, void *workspace,
                            size_t workspace_bytes, void *stream, double *x, double *y, double *z, double *r_p,
                            double *r_d, double *best_ms);

/* Text for a status or error code. */
const char *mipdhg_status_string(int code);

/* Message for the last error returned on this thread ("" if none). */
const char *mipdhg_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* MIPDHG_H */
