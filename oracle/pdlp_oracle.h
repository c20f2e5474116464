/* Plain CPU FP64 restarted-PDHG oracle (Lu & Yang, cuPDLP.jl, arXiv 2311.12180).
 *
 * TEST INFRASTRUCTURE ONLY: this library exists to check the HIP solver.  Only
 * the tests, the smoke check and the benchmark's CPU-baseline leg may load it.
 * It shares no code, header, table or helper with the GPU library.
 *
 * The LP is taken in the user orientation of Section 2, eq. (lp):
 *   min c'x  s.t.  rows typed EQ (a_i x = b_i), GE (a_i x >= b_i), LE (a_i x <= b_i),
 *                  l <= x <= u  (l may be -inf, u may be +inf).
 * CSR arrays: row_ptr[m+1], col_idx[nnz], val[nnz]; row_type[m] in {0 EQ, 1 GE, 2 LE}.
 * Dual vectors y are returned in the user orientation: c = A'y + lambda at optimum.
 */
#ifndef PDLP_ORACLE_H
#define PDLP_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int32_t m, n;
  int64_t nnz;
  const int32_t* row_ptr;
  const int32_t* col_idx;
  const double* val;
  const double* c;
  const double* b;
  const double* l;
  const double* u;
  const int8_t* row_type;
} orc_problem;

typedef struct {
  double eps_rel;         /* relative KKT tolerance of the termination test */
  int64_t max_iter;       /* accepted steps */
  double time_limit_s;
  int32_t eval_period;    /* restart/termination evaluation every P accepted steps */
  int32_t ruiz_iters;
  double pc_alpha;        /* Pock-Chambolle alpha (<0: no Pock-Chambolle pass) */
  double pw_theta;        /* primal-weight smoothing */
  double eps_zero;
  double beta_suff, beta_nec, beta_art;
  int32_t a_precision;    /* 0: FP64 matrix in the steps, 1: FP32-rounded scaled matrix in the steps */
  int32_t kkt_omega_power;/* 2: weights omega^2, 1/omega^2 as printed; 1: omega, 1/omega */
  int32_t threads;        /* OpenMP threads, 0 = runtime default */
  int32_t detect_infeas;  /* 1: test the infeasibility certificates */
  double eps_infeas;      /* tolerance of the certificate tests */
  int32_t infeas_every;   /* test at every infeas_every-th evaluation (after the first step) */
  int32_t restart_metric; /* 0: KKT error (the paper's), 1: normalized duality gap (PDLP's) */
} orc_options;

typedef struct {
  int32_t status;         /* 1 optimal, 2 iteration limit, 3 time limit, 4 numerical error,
                             5 primal infeasible (y holds a dual ray), 6 dual infeasible (x holds a primal ray) */
  int32_t returned_avg;   /* 1 if the returned point is the average iterate */
  int64_t iterations, attempts, restarts, evaluations;
  double rel_kkt, rel_gap, rel_pres, rel_dres, primal_obj, dual_obj;
  double omega, eta_hat, sum_eta, kkt0, setup_s, solve_s;
  int32_t threads_used;
  int32_t ray_source;     /* status 5/6: 0 the last accepted step, 1 the epoch displacement */
  double ray_obj, ray_res;/* status 5/6: the ray's objective and residual norm, for the unit-norm ray */
} orc_info;

/* Optional decision trace: caller-owned arrays of the given capacities. */
typedef struct {
  int64_t cap_att, n_att;
  int64_t* att_k; double* att_eta; double* att_etabar; int8_t* att_acc;
  int64_t cap_eval, n_eval;
  int64_t* ev_k; double* ev_kkt_cur; double* ev_kkt_avg; int8_t* ev_cand; int8_t* ev_reason;
  double* ev_omega;
} orc_trace;

void orc_default_options(orc_options* o);

/* Full solve.  x[n], y[m] (user orientation), rc[n] may be NULL.  x_hat[n], y_hat[m]
 * (optional) receive the final *current* iterate in the scaled, >=-form space. */
int orc_solve(const orc_problem* p, const orc_options* o, double* x, double* y, double* rc,
              orc_info* info, orc_trace* tr, double* x_hat, double* y_hat);

/* Diagonal preconditioning alone: D1[m], D2[n], and the scaled >=-form values
 * (LE rows negated) in the CSR order of the input. */
int orc_rescale(const orc_problem* p, int32_t ruiz_iters, double pc_alpha,
                double* D1, double* D2, double* val_scaled);

/* One PDHG step of eq. (pdhg) with fixed tau, sigma on the >=-form problem
 * given by (K, q, c, l, u, ineq).  Returns x'[n], y'[m]. */
int orc_pdhg_step(int32_t m, int32_t n, const int32_t* row_ptr, const int32_t* col_idx,
                  const double* val, const double* q, const double* c, const double* l,
                  const double* u, const int8_t* ineq, const double* x, const double* y,
                  double tau, double sigma, double* x_out, double* y_out);

/* Termination quantities on the given (user-orientation) LP at (x, y):
 * out[0..9] = rel_kkt, rel_gap, rel_pres, rel_dres, primal_obj, dual_obj,
 *             ||r_p||, ||r_d||, |gap|, kkt_omega (with the given omega and power). */
int orc_evaluate(const orc_problem* p, const double* x, const double* y, double omega,
                 int32_t omega_power, double* out);

/* Farkas test of a candidate direction (x_dir[n], y_dir[m], user orientation)
 * on the LP, with tolerance eps.  out[0..7] = dual-ray objective
 * b'y + l'lam+ - u'lam-, ||A'y + lam||, ||y||, primal-ray objective c'x, norm
 * of x's violation of the row cones, ||x||, the sums of the magnitudes of the
 * terms of the two objectives, after the projections (y clipped to
 * the sign of each inequality row, lam = proj_Lambda(-A'y), x projected onto
 * the recession cone of [l, u]).  ray_x[n], ray_y[m], lam[n] (each may be
 * NULL) receive the projected rays and multipliers.  Returns 1 when y
 * certifies primal infeasibility, else 2 when x certifies dual infeasibility,
 * else 0; -1 for a bad problem. */
int orc_ray_test(const orc_problem* p, const double* x_dir, const double* y_dir, double eps, double* out,
                 double* ray_x, double* ray_y, double* lam);

/* Normalized duality gap rho_r(z) of the scaled LP at the scaled point
 * (x[n], y[m]) with K~x, K~'y given (kx[m], kty[n]), primal weight omega and
 * radius r (the restart metric of restart_metric = 1; see the solver's
 * description of it).  Returns -1 on a bad problem. */
double orc_normalized_gap(const orc_problem* p, int32_t ruiz_iters, double pc_alpha, const double* x,
                          const double* y, double omega, double r);

/* Reduced costs lambda = proj_Lambda(c - A'y) at (user-orientation) y. */
int orc_reduced_costs(const orc_problem* p, const double* y, double* lam);

/* Restart test of the KKT-based scheme: 0 none, 1 sufficient decay,
 * 2 necessary decay without local progress, 3 long inner loop. */
int orc_restart_reason(double kkt_cand, double kkt0, double kkt_prev, int64_t t, int64_t k,
                       double beta_suff, double beta_nec, double beta_art);

/* Primal-weight update at a restart (geometric smoothing in log space). */
double orc_primal_weight_update(double dx, double dy, double omega, double theta, double eps_zero);

#ifdef __cplusplus
}
#endif
#endif
