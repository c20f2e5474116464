/* pdlp.h -- restarted PDHG for linear programming on one AMD MI355X (gfx950).
 *
 * Method: Lu & Yang, "cuPDLP.jl: A GPU Implementation of Restarted
 * Primal-Dual Hybrid Gradient for Linear Programming in Julia" (arXiv
 * 2311.12180).  The solver runs Algorithm 1 (restarted PDHG) with Algorithm 2
 * (adaptive step size), the diagonal preconditioning and primal-weight rules of
 * Section 2.2, the KKT-error restart scheme of Section 3.4 (eq. (kkt)) and the
 * relative-KKT termination test of Section 4.1, entirely on the GPU: the
 * problem crosses to the device once and the solution comes back once
 * (Section 3.2).
 *
 * The LP (Section 2, eq. (lp)), in the user orientation of this interface:
 *     min  c'x
 *     s.t. a_i x  = b_i   (row_type PDLP_ROW_EQ)
 *          a_i x >= b_i   (row_type PDLP_ROW_GE)
 *          a_i x <= b_i   (row_type PDLP_ROW_LE)
 *          l <= x <= u    (l_j may be -INFINITY, u_j may be +INFINITY)
 * A is m x n in CSR form (int32 row_ptr[m+1], int32 col_idx[nnz], double val[nnz]).
 *
 * Dual sign convention of the returned y and reduced costs lambda
 * (stationarity c = A'y + lambda): y is free on EQ rows, y >= 0 on GE rows,
 * y <= 0 on LE rows; lambda_j >= 0 where x_j sits at its lower bound and
 * lambda_j <= 0 at its upper bound.
 *
 * Every function returns an int: 0 (PDLP_OK) on success, a negative PDLP_ERR_*
 * code on failure; no function throws or aborts.  Non-convergence is not an
 * error: pdlp_solve returns PDLP_OK and info.status tells why it stopped.
 * A handle is not thread-safe; distinct handles on distinct streams may run
 * concurrently.
 */
#ifndef PDLP_H
#define PDLP_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pdlp_handle pdlp_handle;   /* opaque; owns every device buffer */

enum { PDLP_ROW_EQ = 0, PDLP_ROW_GE = 1, PDLP_ROW_LE = 2 };       /* int8 row_type */
enum { PDLP_MEM_HOST = 0, PDLP_MEM_DEVICE = 1 };                  /* where problem arrays live */
enum { PDLP_A_FP64 = 0, PDLP_A_FP32 = 1 };                        /* matrix values in the steps */
enum { PDLP_OPTIMAL = 1, PDLP_ITER_LIMIT = 2, PDLP_TIME_LIMIT = 3, PDLP_NUMERICAL_ERROR = 4,
       PDLP_PRIMAL_INFEASIBLE = 5, PDLP_DUAL_INFEASIBLE = 6 };
enum {
  PDLP_OK = 0,
  PDLP_ERR_ARG = -1,          /* NULL pointer, bad size or option */
  PDLP_ERR_DATA = -2,         /* malformed CSR, non-finite data, l > u, bad row type */
  PDLP_ERR_HIP = -3,          /* a HIP runtime call failed (no device, launch failure) */
  PDLP_ERR_OOM = -4,          /* device or pinned host allocation failed */
  PDLP_ERR_STATE = -5,        /* call out of order (e.g. get_solution before solve) */
  PDLP_ERR_UNSUPPORTED = -6
};

/* The LP.  All arrays are read during pdlp_create only (deep copy).
 * mem = PDLP_MEM_HOST: host pointers.  mem = PDLP_MEM_DEVICE: device pointers
 * of the current HIP device (e.g. torch tensor data_ptr()s), copied on the
 * given stream.  Sizes: m >= 0, n >= 1, 0 <= nnz < 2^31.  Column indices of a
 * row may come in any order but must be distinct and in [0, n). */
typedef struct {
  int32_t m, n;
  int64_t nnz;
  int32_t mem;
  const int32_t* row_ptr;     /* [m+1], row_ptr[0] = 0, nondecreasing, row_ptr[m] = nnz */
  const int32_t* col_idx;     /* [nnz] */
  const double* val;          /* [nnz], finite */
  const double* c;            /* [n], finite */
  const double* b;            /* [m], finite */
  const double* l;            /* [n], finite or -INFINITY */
  const double* u;            /* [n], finite or +INFINITY, l <= u */
  const int8_t* row_type;     /* [m], PDLP_ROW_* */
} pdlp_problem;

/* Options; pdlp_default_options fills the defaults shown. */
typedef struct {
  double eps_rel;             /* 1e-4: relative KKT tolerance of Section 4.1 */
  int64_t max_iter;           /* 1000000: accepted PDHG steps (>= 0) */
  double time_limit_s;        /* 3600 */
  int32_t eval_period;        /* 64: restart/termination check every P accepted steps (>= 1) */
  int32_t ruiz_iters;         /* 10: Ruiz inf-norm passes (Section 2.2) */
  double pc_alpha;            /* 1.0: Pock-Chambolle alpha in [0, 2]; < 0 skips the pass */
  double pw_theta;            /* 0.5: primal-weight smoothing in [0, 1] */
  double eps_zero;            /* 1e-10: the "small nonzero tolerance" of the primal weight */
  double beta_suff;           /* 0.2 restart criterion (i) */
  double beta_nec;            /* 0.8 restart criterion (ii) */
  double beta_art;            /* 0.36 restart criterion (iii) */
  int32_t a_precision;        /* PDLP_A_FP64, or PDLP_A_FP32: the scaled matrix is rounded to
                                 FP32 for the PDHG steps (products accumulate in FP64); the
                                 restart / termination evaluations use the FP64 matrix */
  int32_t kkt_omega_power;    /* 2: KKT_omega weights omega^2 and omega^-2 as in eq. (kkt); 1 */
  int32_t trace;              /* capacity of the decision trace (attempts and evaluations), 0 = off */
  int32_t poll_every;         /* 1: graph launches between two reads of the 8-byte status word
                                 (fewer are launched once the graphs in flight can reach max_iter) */
  int32_t graph;              /* 1: the inner loop is a captured hipGraph; 0: the same kernels
                                 launched one by one (for callers that cannot use graphs) */
  int32_t spmv_layout;        /* -1: chosen per matrix at create by timing the step passes (default);
                                 0: row blocks; 1: column panels (one per XCD) with a second pass
                                 that adds each row's panel sums; 2: row blocks with contiguous
                                 block ranges per XCD; plus 4: a persistent grid (one workgroup
                                 per 8 waves of every CU, looping over the row blocks); plus 8:
                                 the step passes take blocks of 6144 nonzeros instead of 3072
                                 (the evaluation passes keep 3072); or 3, 19, 35: the step pass
                                 runs on LDS-staged column panels -- the rows with at least 256
                                 nonzeros (numbered first by row_order) are cut into panels of
                                 16,384 columns whose slice of the gathered vector a workgroup of
                                 256, 512 or 1024 threads copies into LDS once, the other rows
                                 with two nonzeros or more take eight column panels (one per
                                 XCD), rows of one nonzero are summed directly -- with column
                                 panels on a persistent grid
                                 for the evaluation passes (with the FP64 matrix, the
                                 evaluation's rows of K run instead as two staged passes of
                                 one gathered vector each: K x_bar, then K x with the
                                 residuals); or 64, 80, 96: the step pass runs
                                 on SELL-64 chunks -- 64 consecutive rows stored
                                 lane-interleaved, one row per lane, zero-padded to the chunk's
                                 longest row (built automatically when the padding stays within
                                 1/8, the matrix gives at least four chunks per CU and no row is
                                 longer than 16 times the mean plus 64; with row_order the rows
                                 of K' come by descending length) --
                                 in workgroups of 1024 or 512 threads that first copy the
                                 leading 8192 entries of the gathered vector into LDS (64, 80),
                                 or of 256 threads without that copy (96); the evaluation passes
                                 over that matrix run on the same chunks (their two gathered
                                 vectors share the LDS copy).  The timing at create tries every
                                 combination on matrices with 2^20 nonzeros or more.  The
                                 layout changes the order of floating-point sums; fix it for
                                 bitwise reproducibility across handles.  This field applies to
                                 K, and to K' unless spmv_layout_kt says otherwise */
  int32_t batch_lanes;        /* batch handles: how each LP's rows are swept.  0 = chosen per LP
                                 class by timing capped solves at pdlp_create_batch (default);
                                 -1 = LDS-tiled row blocks for every LP; 1..64 (a power of two) =
                                 that many lanes per row for every row */
  int32_t batch_grid;         /* batch handles: workgroups of the persistent launch, 0 = chosen by
                                 timing (default) */
  int32_t spmv_layout_kt;     /* -2: K' follows spmv_layout (default); otherwise as spmv_layout,
                                 for K' alone */
  int32_t batch_handoff;      /* batch handles: an LP that has taken this many accepted steps stops
                                 in the persistent launch at its next evaluation (default 2048, 0 =
                                 never).  If at most 8 x handoff_streams LPs stopped, the
                                 single-LP kernels finish them, handoff_streams at a time on
                                 streams of their own (same state, same iteration); otherwise
                                 they continue in a new persistent launch with the threshold
                                 doubled (the same arithmetic as if they had not stopped), and so
                                 on until few enough remain */
  int32_t handoff_streams;    /* batch handles: LPs finished at once after the hand-off, each on a
                                 stream of its own (1..16, default 8), the LPs farthest from the
                                 tolerance first */
  int32_t detect_infeas;      /* 1 (default): test infeasibility certificates at every
                                 infeas_every-th evaluation (Section 2.2, "periodically"): the last
                                 accepted step and the epoch displacement
                                 z - z^{n,0} as candidate rays, Farkas' lemma on the unscaled LP;
                                 0: never (an infeasible LP then runs to a limit) */
  double eps_infeas;          /* tolerance of the certificate tests (default 1e-8): a dual ray y
                                 (clipped to the sign of each inequality row, lam =
                                 proj_Lambda(-A'y)) needs b'y + l'lam+ - u'lam- > 0 and
                                 ||A'y + lam|| <= eps times it; a primal ray x (projected onto the
                                 recession cone of [l, u]) needs c'x < 0 and its violation of the
                                 row cones <= eps |c'x|; each objective must also exceed eps times
                                 the sum of the magnitudes of its terms */
  int32_t infeas_every;       /* evaluations per certificate test, >= 1 (default 4: the two extra
                                 products cost ~3 % of the run when done at every evaluation) */
  int32_t presolve;           /* single-LP handles: 1 = presolve-lite at pdlp_create (fixed and
                                 empty columns, empty and singleton rows, until none applies) and
                                 the exact postsolve in pdlp_get_solution; the device solves the
                                 reduced LP (its relative errors are the reduced LP's; objectives
                                 are reported for the user's LP).  An LP that presolve finds
                                 infeasible or reduces to no column is solved as given.
                                 pdlp_get_iterate and pdlp_get_scaling return
                                 PDLP_ERR_UNSUPPORTED then.  Default 0; batch handles: 0 only */
  int32_t restart_metric;     /* 0 (default): KKT_omega restarts (Section 3.4, the paper's);
                                 1: PDLP's normalized duality gap rho_r(z) = max {L(x, yh) -
                                 L(xh, y) : zh in Z, ||zh - z||_omega <= r} / r, the metric the
                                 paper's KKT restarts replace; its trust-region problem is solved
                                 at each evaluation by 24 passes over the vectors (a multiplier
                                 search), for both candidates at once.  The candidates, criteria,
                                 betas and primal weight update are those of the KKT scheme, the
                                 reference value being the restart point's rho (+inf before the
                                 first restart).  Termination is unchanged (Section 4.1) */
  int32_t row_order;          /* single-LP handles: 1 (default) = the device numbers the rows by
                                 descending number of nonzeros, equal counts by first column
                                 (after the scaling, so D1, D2 and K~ are unchanged): on LPs with
                                 skewed row lengths the gathers of y and of x then hit the caches
                                 far more often.  On LPs with 2^20 nonzeros or more whose
                                 columns in the given order would fill 64-column chunks with
                                 more than 1/8 padding, it first renumbers the columns: sorted
                                 by descending number of nonzeros, cut into groups of 64, the
                                 groups dealt out over the column range (16,384-column
                                 strides), so that the rows of K' fill SELL-64 chunks with
                                 little padding while every wide column range keeps columns of
                                 every count.  2 = the same at any size.  Only the order of
                                 floating-point sums changes; every vector crossing this
                                 interface (x, y, reduced costs, D1, D2, K~, warm starts) stays
                                 in the caller's order.  0 = the given order.  Batch handles
                                 keep the given order */
} pdlp_options;

typedef struct {
  int32_t status;             /* PDLP_OPTIMAL / ITER_LIMIT / TIME_LIMIT / NUMERICAL_ERROR */
  int32_t returned_avg;       /* 1 if the returned point is the epoch's weighted average */
  int64_t iterations;         /* accepted PDHG steps */
  int64_t attempts;           /* step attempts of Algorithm 2 (>= iterations) */
  int64_t restarts;
  int64_t evaluations;
  double rel_kkt, rel_gap, rel_pres, rel_dres;   /* Section 4.1, on the original LP */
  double primal_obj, dual_obj;
  double omega, eta_hat;      /* primal weight and step size at exit */
  double setup_s;             /* pdlp_create: upload, transpose, scaling, layout choice */
  double solve_s;             /* pdlp_solve wall time */
  int32_t layout_k, layout_kt;  /* layouts in use for K and K' (values of spmv_layout: 0, 1, 2,
                                   plus 4 for a persistent grid, plus 8 for the wide step tiles,
                                   or 3, 19, 35 for LDS-staged step passes, or 64, 80, 96 for
                                   SELL-64 step passes);
                                   for an LP of a batch: its sweeps of K and K' (see
                                   pdlp_batch_schedule) */
  int64_t handoff_k;          /* an LP of a batch: accepted steps when the single-LP kernels took
                                 it over (0: it ended in the persistent launch) */
  double ray_obj, ray_res;    /* PRIMAL_INFEASIBLE: b'y + l'lam+ - u'lam- and ||A'y + lam|| of the
                                 returned unit dual ray; DUAL_INFEASIBLE: c'x and the row-cone
                                 violation of the returned unit primal ray; 0 otherwise */
  int32_t ray_source;         /* the candidate that certified: 0 the last accepted step, 1 the
                                 epoch displacement */
  int32_t m_solved, n_solved; /* rows and columns of the LP the device solved (after presolve) */
  int32_t reserved;
} pdlp_info;

/* Scaled-space state of the current iterate (for parity checks and resume). */
typedef struct {
  int64_t iterations, attempts, restarts, evaluations;
  double eta_hat, omega, sum_eta, kkt0;
} pdlp_iter_state;

/* Fill *o with the defaults listed above.  PDLP_ERR_ARG if o is NULL. */
int pdlp_default_options(pdlp_options* o);

/* Validate and upload the LP, transpose it on the device (both K and K' are
 * kept in CSR), negate LE rows into the >= form of eq. (primal-dual), and run
 * the Section 2.2 preconditioning (ruiz_iters Ruiz passes, then one
 * Pock-Chambolle pass) on the device.  o = NULL means defaults.  hip_stream is
 * a hipStream_t (NULL: the default stream); every device operation of the
 * handle runs on it, and create synchronizes it before returning.  On success
 * *out owns all device memory; on failure *out is NULL and
 * pdlp_last_error(NULL) describes the problem. */
int pdlp_create(const pdlp_problem* p, const pdlp_options* o, void* hip_stream, pdlp_handle** out);

/* Starting point for the next pdlp_solve (Section 4.1 uses the zero vector;
 * this replaces it): x0[n] and y0[m] in the user orientation on the host, or
 * NULL for the default (proj_X(0), 0); omega0 <= 0 keeps the default primal
 * weight ||c~||/||q~||.  x0 is projected onto the bounds and y0 onto the sign
 * constraints of its rows.  PDLP_ERR_DATA if a value is not finite. */
int pdlp_set_warm_start(pdlp_handle* h, const double* x0, const double* y0, double omega0);

/* Run Algorithm 1 from the starting point until the Section 4.1 test holds
 * (rel KKT <= eps_rel for the current or the average iterate) or a limit is
 * hit.  Each call starts afresh from the starting point.  The inner loop is a
 * captured hipGraph of attempt slots plus the restart/termination evaluation;
 * the host reads only an 8-byte status word between graph launches. */
int pdlp_solve(pdlp_handle* h);

/* For callers that cannot allocate device memory during a solve (serving
 * loops and harnesses that forbid allocation once set up): pdlp_solve with
 * the same kernels, results and status, launched one by one (no graph is
 * instantiated), with every reduction partial and segment sum of the solve
 * in a static device array of the library (64 MiB per GPU, held until the
 * process ends) instead of the handle's own buffers.  It calls no hipMalloc,
 * hipFree or other allocating routine; the handle (created by pdlp_create,
 * which allocates) still owns the problem, the iterates and the outputs.
 * Call it with the handle's device current (else PDLP_ERR_STATE).
 * PDLP_ERR_UNSUPPORTED if the LP's partial sums need more than 64 MiB (the
 * message gives the size) or on a batch handle (PDLP_ERR_STATE).  Every call
 * on one GPU shares that array and clears it first: calls that overlap on one
 * GPU, from any handle or thread, race. */
int pdlp_solve_noalloc(pdlp_handle* h);

/* Change the termination test of later solves: eps_rel >= 0, max_iter >= 0
 * accepted steps, time_limit_s > 0 (same meaning as in pdlp_options).
 * PDLP_ERR_ARG for values out of range; the handle keeps its old values then. */
int pdlp_set_termination(pdlp_handle* h, double eps_rel, int64_t max_iter, double time_limit_s);

/* The reductions pdlp_create makes with presolve = 1, computed on the host
 * (no device needed; for inspection and tests): keep_row[m], keep_col[n] (1
 * kept, 0 removed); every column's final bounds lo[n], hi[n] and, for a
 * removed column, its value x_fixed[n]; the right-hand sides b_reduced[m]
 * after the reductions (meaningful for kept rows); *offset, the objective of
 * the removed columns.  *status = 0, or PDLP_PRIMAL_INFEASIBLE /
 * PDLP_DUAL_INFEASIBLE when presolve itself finds the LP so (the outputs then
 * hold the state at that point).  Any output may be NULL.  Returns PDLP_OK or
 * the error of pdlp_create's validation. */
int pdlp_presolve(const pdlp_problem* p, int32_t* status, uint8_t* keep_row, uint8_t* keep_col, double* lo,
                  double* hi, double* x_fixed, double* b_reduced, double* offset);

/* Copy the solution of the last pdlp_solve to host buffers: x[n], y[m]
 * (user orientation) and reduced_cost[n] (lambda = proj_Lambda(c - A'y)); any
 * of them and info may be NULL.  After PDLP_PRIMAL_INFEASIBLE, y is the unit
 * dual ray and reduced_cost its multipliers lam (A'y + lam ~ 0); after
 * PDLP_DUAL_INFEASIBLE, x is the unit primal ray.  PDLP_ERR_STATE before the
 * first solve. */
int pdlp_get_solution(pdlp_handle* h, double* x, double* y, double* reduced_cost, pdlp_info* info);

/* The current iterate in the scaled >= form (x~[n], y~[m]; NULL to skip) and
 * the step state.  Valid after pdlp_solve. */
int pdlp_get_iterate(pdlp_handle* h, double* x_hat, double* y_hat, pdlp_iter_state* st);

/* The preconditioner D1[m], D2[n] and the scaled >=-form values D1 K D2 in the
 * CSR order of the input (val_scaled[nnz]); NULL to skip any. */
int pdlp_get_scaling(pdlp_handle* h, double* D1, double* D2, double* val_scaled);

/* Decision trace of the last solve (needs options.trace > 0).  Attempts:
 * k (accepted steps before the attempt), eta, eta_bar, accepted.  Evaluations:
 * k, KKT_omega(current), KKT_omega(average), candidate (1 = average), restart
 * reason (0 none, 1 sufficient, 2 necessary, 3 artificial), omega after.
 * Arrays hold up to `cap` entries; *n_att / *n_eval receive the counts. */
int pdlp_get_trace(pdlp_handle* h, int64_t cap, int64_t* n_att, int64_t* att_k, double* att_eta,
                   double* att_etabar, int8_t* att_acc, int64_t* n_eval, int64_t* ev_k,
                   double* ev_kkt_cur, double* ev_kkt_avg, int8_t* ev_cand, int8_t* ev_reason,
                   double* ev_omega);

/* Time the two PDHG step kernels: continue the last solve for `attempts`
 * attempt pairs launched eagerly on the handle's stream, each bracketed by HIP
 * events, and return the mean duration (milliseconds) of the primal-step
 * kernel (K' product fused with the x update) and of the dual-step kernel
 * (K product fused with the y update and the step-size decision).  The
 * attempts are real PDHG steps of the solve.  PDLP_ERR_STATE before a solve. */
int pdlp_profile_attempts(pdlp_handle* h, int32_t attempts, double* ms_primal, double* ms_dual);

/* Algorithmic bytes moved by one primal-step and one dual-step kernel launch
 * (matrix stream, row pointers, one read of each gathered vector, the per-row
 * vector reads and writes). */
int pdlp_step_bytes(pdlp_handle* h, double* bytes_primal, double* bytes_dual);

/* ---- Batches: many independent LPs solved by one persistent launch ----
 *
 * The LPs are packed block-diagonally (LP k owns the next m_k rows and n_k
 * columns); Algorithm 1 with its own restarts, primal weight and Section 4.1
 * termination runs for each LP, all with the options of the handle.  A
 * workgroup takes the next LP from a device queue (most nonzeros first), keeps
 * its scalar state on chip, and sweeps its rows with a per-LP number of lanes
 * per row taken from the batch schedule.  Every LP is preconditioned on its own
 * (the Section 2.2 scalings act row- and column-wise, so packing does not
 * mix LPs). */

/* Create a handle for ps[0 .. count-1] (each validated as in pdlp_create; the
 * error message names the first bad LP).  The totals of rows, columns and
 * nonzeros must stay below 2^31.  Unless batch_lanes and batch_grid are both
 * fixed, create times capped solves (64 accepted steps per LP) to choose the
 * schedule.  Single-LP entry points (pdlp_solve, pdlp_get_solution,
 * pdlp_get_iterate, pdlp_set_warm_start, pdlp_profile_attempts,
 * pdlp_step_bytes) return PDLP_ERR_STATE on a batch handle; pdlp_get_scaling
 * returns the packed arrays and pdlp_get_trace the trace of LP 0. */
int pdlp_create_batch(const pdlp_problem* ps, int32_t count, const pdlp_options* o, void* hip_stream,
                      pdlp_handle** out);

/* Warm start of LP idx (x0[n_idx], y0[m_idx], user orientation), or of every
 * LP when idx = -1 (x0, y0 packed in LP order, omega0 for all).  NULL for x0
 * or y0 means zero for that part; both NULL clears the warm start.
 * PDLP_ERR_ARG for idx out of range, PDLP_ERR_DATA for non-finite values. */
int pdlp_set_warm_start_batch(pdlp_handle* h, int32_t idx, const double* x0, const double* y0, double omega0);

/* Solve every LP of the batch from its starting point in one persistent launch
 * (or a few: see batch_handoff); the last LPs still running after
 * batch_handoff (or a multiple of it) accepted steps are finished by the
 * single-LP kernels (handoff_streams at a time, each on a library-owned stream,
 * over its own slice of the packed arrays), and the call returns when every LP
 * has ended.  time_limit_s bounds the whole solve (an LP still running then ends
 * with PDLP_TIME_LIMIT); an LP whose attempts are rejected 1000 times in a row
 * in the persistent launch, or that accepts no step over 64 polls after the
 * hand-off, ends with PDLP_NUMERICAL_ERROR. */
int pdlp_solve_batch(pdlp_handle* h);

/* Solution of LP idx (x[n_idx], y[m_idx], reduced_cost[n_idx], *info), or of
 * every LP when idx = -1 (packed in LP order, info[count]).  solve_s is the
 * time of the whole batch solve.  PDLP_ERR_STATE before pdlp_solve_batch. */
int pdlp_get_solution_batch(pdlp_handle* h, int32_t idx, double* x, double* y, double* reduced_cost,
                            pdlp_info* info);

/* Schedule of the persistent launch: lanes[2*count] (the sweep of each LP's
 * rows of K and of K': 0 = LDS-tiled row blocks of up to 4096 nonzeros, L > 0
 * = L lanes per row) and the number of workgroups; NULL to skip either. */
int pdlp_batch_schedule(pdlp_handle* h, int32_t* lanes, int32_t* grid);

/* Last error message of h, or of the last failed pdlp_create on this thread
 * when h is NULL.  Never NULL. */
const char* pdlp_last_error(const pdlp_handle* h);

/* Release every resource of h.  NULL-safe. */
void pdlp_destroy(pdlp_handle* h);

#ifdef __cplusplus
}
#endif
#endif /* PDLP_H */
