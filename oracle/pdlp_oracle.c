/* Plain CPU FP64 restarted-PDHG oracle for LP.
 *
 * TEST INFRASTRUCTURE ONLY.  It is the yardstick the HIP solver is checked
 * against; the product never loads it.  It shares no code with the GPU path.
 *
 * It follows the method of Lu & Yang, "cuPDLP.jl: a GPU implementation of
 * restarted PDHG for linear programming in Julia" (arXiv 2311.12180), step by
 * step and without any fusion:
 *   Section 2 eq. (lp), eq. (primal-dual)  -- LP and saddle-point form
 *   Section 2.1 eq. (pdhg) + reparametrisation tau = eta/omega, sigma = eta*omega
 *   Section 2.2 Algorithm 1 (restarted PDHG), Algorithm 2 (adaptive step),
 *               preconditioning (Ruiz then Pock-Chambolle), primal weight
 *   Section 3.4 eq. (kkt), restart candidate, restart criteria (i)-(iii)
 *   Section 4.1 termination on the original (unscaled) LP, zero start.
 * Readings taken where the paper is silent or garbled (each one is an option
 * where it is a constant):
 *   - the denominator 2 (y'-y)'K(x'-x) of the step bound is used in absolute
 *     value; a zero denominator gives an infinite bound;
 *   - the exponents of Algorithm 2 use the 1-based count k+2 with 0-based k
 *     (with k+1 the first factor 1-1^-0.3 is zero);
 *   - the primal-weight update smooths in log space:
 *     omega <- exp(theta log(dy/dx) + (1-theta) log omega), theta = 0.5;
 *   - the average of Algorithm 1 sums the accepted steps of the current epoch,
 *     weighted by their step sizes;
 *   - lambda = proj_Lambda(c - K'y), Lambda_j allowing positive values only
 *     where l_j is finite and negative values only where u_j is finite;
 *     0 * inf := 0 in l'lambda+ and u'lambda-;
 *   - restart and termination are evaluated every `eval_period` accepted steps
 *     (and at the iteration limit); both the current and the average iterate
 *     are tested for termination and the one with the smaller relative KKT
 *     error is returned;
 *   - ||K||_inf of the initial step size is the largest |entry| of the scaled K;
 *   - 10 Ruiz passes (inf-norm) then one Pock-Chambolle pass with alpha = 1;
 *   - KKT_omega weights omega^2 and 1/omega^2 as printed;
 *   - at an epoch's first evaluation the previous candidate KKT is KKT(z^{n,0});
 *   - the candidate comparison KKT(current) < KKT(average) treats a relative
 *     difference below 1e-12 as a tie, which goes to the average;
 *   - the start is proj_X(0), y = 0;
 *   - infeasibility detection (Section 2.2 names the two sequences, says they
 *     are checked periodically and defers the test to its citation): at every
 *     infeas_every-th evaluation (default 4) that does not terminate,
 *     the last accepted step z - z_prev and the epoch displacement z - z^{n,0}
 *     (the normalized iterate without its 1/t, which the scale-free tests
 *     ignore) are each tested on the unscaled LP against Farkas' lemma:
 *     y (inequality entries clipped at 0) with lam = proj_Lambda(-K'y) is a
 *     dual ray when q'y + l'lam+ - u'lam- > 0 and ||K'y + lam|| <= eps times
 *     it; x projected onto the recession cone of [l, u] is a primal ray when
 *     c'x < 0 and the norm of Kx's violation of (=0 on EQ, >=0 on the other
 *     rows) is <= eps |c'x|; in both, the ray objective must also exceed eps
 *     times the sum of the magnitudes of its terms (a sign that cancellation
 *     cannot produce: with every variable boxed, lam absorbs all of K'y and
 *     the objective's sign is the whole test).  Primal infeasibility is tested
 *     first, the step before the displacement; the unit-norm ray is returned;
 *   - restart_metric = 1 replaces KKT_omega in the restart scheme by the
 *     normalized duality gap of PDLP, which Section 3.4 says the KKT error
 *     replaces: rho_r(z) = max { L(x, yh) - L(xh, y) : zh in Z,
 *     ||zh - z||_omega <= r } / r on the scaled LP, with
 *     ||d||_omega^2 = omega ||dx||^2 + ||dy||^2 / omega.  The objective is
 *     linear in d = zh - z with gradient g = (K'y - c, q - Kx); its maximiser
 *     is d(lam) = proj_{Z - z}(W^-1 g / lam), W = diag(omega, 1/omega), for the
 *     lam at which ||d(lam)||_omega = r (or the box corner when the ball does
 *     not bind).  It is solved exactly: the breakpoints at which coordinates
 *     of d reach their bounds are sorted and ||d||_omega = r is solved on the
 *     interval between two of them, where ||d||^2 is a quadratic in 1/lam
 *     (no iteration).  The candidate is the iterate with the smaller
 *     rho_{||z - z^{n,0}||}(z) (ties to the average); criteria (i)-(iii) as for
 *     KKT with rho in place of KKT, the reference value being the restart
 *     point's rho (the candidate's at the restart, with the radius to the
 *     previous restart point), +inf before the first restart.
 * Sums are taken in a fixed blocked order (blocks of 4096, serial within and
 * across blocks) so that results do not depend on the thread count.  Built
 * with -ffp-contract=off: every product and sum is rounded on its own.
 */
#include "pdlp_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define RBLK 4096

static double now_s(void) {
  struct timespec ts;
  clock_gettime(CLOCK_MONOTONIC, &ts);
  return (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
}

static void* xalloc(size_t count, size_t sz) {
  return calloc(count > 0 ? count : 1, sz);
}

/* ---------------------------------------------------------------- sums */

static double blocked_sum(int64_t n, const double* a) {
  int64_t nb = (n + RBLK - 1) / RBLK;
  if (nb == 0) return 0.0;
  double* part = (double*)xalloc((size_t)nb, sizeof(double));
#pragma omp parallel for schedule(static)
  for (int64_t b = 0; b < nb; ++b) {
    int64_t i0 = b * RBLK, i1 = i0 + RBLK < n ? i0 + RBLK : n;
    double s = 0.0;
    for (int64_t i = i0; i < i1; ++i) s += a[i];
    part[b] = s;
  }
  double s = 0.0;
  for (int64_t b = 0; b < nb; ++b) s += part[b];
  free(part);
  return s;
}

static double dot(int64_t n, const double* a, const double* b) {
  double* t = (double*)xalloc((size_t)n, sizeof(double));
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) t[i] = a[i] * b[i];
  double s = blocked_sum(n, t);
  free(t);
  return s;
}

static double sumsq(int64_t n, const double* a) { return dot(n, a, a); }

static double dist2(int64_t n, const double* a, const double* b) {
  double* t = (double*)xalloc((size_t)n, sizeof(double));
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) { double d = a[i] - b[i]; t[i] = d * d; }
  double s = blocked_sum(n, t);
  free(t);
  return s;
}

/* ---------------------------------------------------------------- CSR */

typedef struct {
  int32_t nr, nc;
  int64_t nnz;
  int32_t* rp;
  int32_t* ci;
  double* v;
  float* vf;   /* FP32-rounded copy of v (FP32-A mode), may be NULL */
} csr;

static void csr_free(csr* A) {
  free(A->rp); free(A->ci); free(A->v); free(A->vf);
  memset(A, 0, sizeof(*A));
}

/* y = A x, each row summed serially in storage order */
static void spmv(const csr* A, const double* x, double* y) {
#pragma omp parallel for schedule(dynamic, 512)
  for (int32_t i = 0; i < A->nr; ++i) {
    double s = 0.0;
    for (int64_t p = A->rp[i]; p < A->rp[i + 1]; ++p) s += A->v[p] * x[A->ci[p]];
    y[i] = s;
  }
}

/* the same product with the FP32-rounded values, converted to FP64 per product */
static void spmv_f(const csr* A, const double* x, double* y) {
#pragma omp parallel for schedule(dynamic, 512)
  for (int32_t i = 0; i < A->nr; ++i) {
    double s = 0.0;
    for (int64_t p = A->rp[i]; p < A->rp[i + 1]; ++p) s += (double)A->vf[p] * x[A->ci[p]];
    y[i] = s;
  }
}

/* pattern of A' (rows of A' sorted by the row index of A); perm[q] = position in A */
static void transpose(const csr* A, csr* T, int64_t* perm) {
  T->nr = A->nc; T->nc = A->nr; T->nnz = A->nnz;
  T->rp = (int32_t*)xalloc((size_t)A->nc + 1, sizeof(int32_t));
  T->ci = (int32_t*)xalloc((size_t)A->nnz, sizeof(int32_t));
  T->v = (double*)xalloc((size_t)A->nnz, sizeof(double));
  T->vf = NULL;
  int64_t* pos = (int64_t*)xalloc((size_t)A->nc + 1, sizeof(int64_t));
  for (int64_t p = 0; p < A->nnz; ++p) pos[A->ci[p] + 1]++;
  for (int32_t j = 0; j < A->nc; ++j) pos[j + 1] += pos[j];
  for (int32_t j = 0; j <= A->nc; ++j) T->rp[j] = (int32_t)pos[j];
  for (int32_t i = 0; i < A->nr; ++i)
    for (int64_t p = A->rp[i]; p < A->rp[i + 1]; ++p) {
      int64_t q = pos[A->ci[p]]++;
      T->ci[q] = i;
      T->v[q] = A->v[p];
      if (perm) perm[q] = p;
    }
  free(pos);
}

/* ---------------------------------------------------------------- LP */

typedef struct {
  int32_t m, n;
  csr K0, K0t;       /* unscaled >=-form matrix (LE rows negated) and its transpose */
  csr K, Kt;         /* scaled K~ = D1 K D2 and its transpose */
  double *q0, *c0, *l0, *u0;
  double *q, *c, *l, *u;
  int8_t* ineq;      /* 1 for GE and LE rows */
  int8_t* le;
  double *D1, *D2;
  double qnorm0, cnorm0;
} lp_t;

static void lp_free(lp_t* P) {
  csr_free(&P->K0); csr_free(&P->K0t); csr_free(&P->K); csr_free(&P->Kt);
  free(P->q0); free(P->c0); free(P->l0); free(P->u0);
  free(P->q); free(P->c); free(P->l); free(P->u);
  free(P->ineq); free(P->le); free(P->D1); free(P->D2);
  memset(P, 0, sizeof(*P));
}

/* Section 2 eq. (primal-dual): K = (G; A), q = (h; b); LE rows a x <= b are
 * the >= rows (-a) x >= -b. */
static int lp_normalize(const orc_problem* p, lp_t* P) {
  memset(P, 0, sizeof(*P));
  if (p->m < 0 || p->n < 1 || p->nnz < 0) return -1;
  P->m = p->m; P->n = p->n;
  int32_t m = p->m, n = p->n;
  int64_t nnz = p->nnz;
  P->K0.nr = m; P->K0.nc = n; P->K0.nnz = nnz;
  P->K0.rp = (int32_t*)xalloc((size_t)m + 1, sizeof(int32_t));
  P->K0.ci = (int32_t*)xalloc((size_t)nnz, sizeof(int32_t));
  P->K0.v = (double*)xalloc((size_t)nnz, sizeof(double));
  P->q0 = (double*)xalloc((size_t)m, sizeof(double));
  P->ineq = (int8_t*)xalloc((size_t)m, 1);
  P->le = (int8_t*)xalloc((size_t)m, 1);
  memcpy(P->K0.rp, p->row_ptr, sizeof(int32_t) * ((size_t)m + 1));
  memcpy(P->K0.ci, p->col_idx, sizeof(int32_t) * (size_t)nnz);
  for (int32_t i = 0; i < m; ++i) {
    int le = p->row_type[i] == 2;
    P->le[i] = (int8_t)le;
    P->ineq[i] = (int8_t)(p->row_type[i] != 0);
    P->q0[i] = le ? -p->b[i] : p->b[i];
    for (int64_t k = p->row_ptr[i]; k < p->row_ptr[i + 1]; ++k)
      P->K0.v[k] = le ? -p->val[k] : p->val[k];
  }
  transpose(&P->K0, &P->K0t, NULL);
  P->c0 = (double*)xalloc((size_t)n, sizeof(double));
  P->l0 = (double*)xalloc((size_t)n, sizeof(double));
  P->u0 = (double*)xalloc((size_t)n, sizeof(double));
  memcpy(P->c0, p->c, sizeof(double) * (size_t)n);
  memcpy(P->l0, p->l, sizeof(double) * (size_t)n);
  memcpy(P->u0, p->u, sizeof(double) * (size_t)n);
  P->qnorm0 = sqrt(sumsq(m, P->q0));
  P->cnorm0 = sqrt(sumsq(n, P->c0));
  return 0;
}

/* Section 2.2, preconditioning: K~ = D1 K D2 by `ruiz` Ruiz passes
 * (d1_i = 1/sqrt(max_j |K_ij|), d2_j = 1/sqrt(max_i |K_ij|), 1 for empty
 * rows/columns) and then one Pock-Chambolle pass (d1_i = 1/sqrt(sum_j
 * |K_ij|^(2-alpha)), d2_j = 1/sqrt(sum_i |K_ij|^alpha)).  Each pass computes
 * both factors from the same matrix and then applies K_ij *= d1_i * d2_j.
 * c~ = D2 c, q~ = D1 q, l~ = l / D2, u~ = u / D2. */
static void lp_scale(lp_t* P, int ruiz, double alpha) {
  int32_t m = P->m, n = P->n;
  int64_t nnz = P->K0.nnz;
  csr* K = &P->K;
  K->nr = m; K->nc = n; K->nnz = nnz;
  K->rp = (int32_t*)xalloc((size_t)m + 1, sizeof(int32_t));
  K->ci = (int32_t*)xalloc((size_t)nnz, sizeof(int32_t));
  K->v = (double*)xalloc((size_t)nnz, sizeof(double));
  K->vf = NULL;
  memcpy(K->rp, P->K0.rp, sizeof(int32_t) * ((size_t)m + 1));
  memcpy(K->ci, P->K0.ci, sizeof(int32_t) * (size_t)nnz);
  memcpy(K->v, P->K0.v, sizeof(double) * (size_t)nnz);
  int64_t* perm = (int64_t*)xalloc((size_t)nnz, sizeof(int64_t));
  transpose(K, &P->Kt, perm);
  P->D1 = (double*)xalloc((size_t)m, sizeof(double));
  P->D2 = (double*)xalloc((size_t)n, sizeof(double));
  for (int32_t i = 0; i < m; ++i) P->D1[i] = 1.0;
  for (int32_t j = 0; j < n; ++j) P->D2[j] = 1.0;
  double* d1 = (double*)xalloc((size_t)m, sizeof(double));
  double* d2 = (double*)xalloc((size_t)n, sizeof(double));
  const csr* Kt = &P->Kt;
  int passes = ruiz + (alpha >= 0.0 ? 1 : 0);
  for (int it = 0; it < passes; ++it) {
    int pc = it >= ruiz;
#pragma omp parallel for schedule(dynamic, 512)
    for (int32_t i = 0; i < m; ++i) {
      double r = 0.0;
      for (int64_t p = K->rp[i]; p < K->rp[i + 1]; ++p) {
        double a = fabs(K->v[p]);
        if (!pc) r = a > r ? a : r;
        else r += (alpha == 1.0) ? a : pow(a, 2.0 - alpha);
      }
      d1[i] = r > 0.0 ? 1.0 / sqrt(r) : 1.0;
    }
#pragma omp parallel for schedule(dynamic, 512)
    for (int32_t j = 0; j < n; ++j) {
      double s = 0.0;
      for (int64_t q = Kt->rp[j]; q < Kt->rp[j + 1]; ++q) {
        double a = fabs(K->v[perm[q]]);
        if (!pc) s = a > s ? a : s;
        else s += (alpha == 1.0) ? a : pow(a, alpha);
      }
      d2[j] = s > 0.0 ? 1.0 / sqrt(s) : 1.0;
    }
#pragma omp parallel for schedule(dynamic, 512)
    for (int32_t i = 0; i < m; ++i)
      for (int64_t p = K->rp[i]; p < K->rp[i + 1]; ++p) K->v[p] = K->v[p] * (d1[i] * d2[K->ci[p]]);
    for (int32_t i = 0; i < m; ++i) P->D1[i] *= d1[i];
    for (int32_t j = 0; j < n; ++j) P->D2[j] *= d2[j];
  }
  for (int64_t q = 0; q < nnz; ++q) P->Kt.v[q] = K->v[perm[q]];
  free(perm); free(d1); free(d2);
  P->q = (double*)xalloc((size_t)m, sizeof(double));
  P->c = (double*)xalloc((size_t)n, sizeof(double));
  P->l = (double*)xalloc((size_t)n, sizeof(double));
  P->u = (double*)xalloc((size_t)n, sizeof(double));
  for (int32_t i = 0; i < m; ++i) P->q[i] = P->D1[i] * P->q0[i];
  for (int32_t j = 0; j < n; ++j) {
    P->c[j] = P->D2[j] * P->c0[j];
    P->l[j] = P->l0[j] / P->D2[j];
    P->u[j] = P->u0[j] / P->D2[j];
  }
}

static void lp_round_fp32(lp_t* P) {
  P->K.vf = (float*)xalloc((size_t)P->K.nnz, sizeof(float));
  P->Kt.vf = (float*)xalloc((size_t)P->Kt.nnz, sizeof(float));
  for (int64_t p = 0; p < P->K.nnz; ++p) P->K.vf[p] = (float)P->K.v[p];
  for (int64_t p = 0; p < P->Kt.nnz; ++p) P->Kt.vf[p] = (float)P->Kt.v[p];
}

/* ---------------------------------------------------------------- pieces */

static double clampd(double v, double lo, double hi) {
  if (v < lo) v = lo;
  if (v > hi) v = hi;
  return v;
}

/* proj_Lambda(g): positive part allowed only at a finite lower bound,
 * negative part only at a finite upper bound */
static double proj_lambda(double g, double l, double u) {
  int lf = isfinite(l), uf = isfinite(u);
  if (lf && uf) return g;
  if (lf) return g > 0.0 ? g : 0.0;
  if (uf) return g < 0.0 ? g : 0.0;
  return 0.0;
}

typedef struct {
  double rp2, rd2, pobj, dobj;
} parts_t;

/* Residual pieces of eq. (kkt) on the >=-form LP (K, q, c, l, u) at (x, y)
 * with Kx and K'y given:
 *   primal residual (K_eq x - q_eq ; [q_ineq - K_ineq x]^+),
 *   lambda = proj_Lambda(c - K'y), dual residual c - K'y - lambda,
 *   primal objective c'x, dual objective q'y + l'lambda^+ - u'lambda^-. */
static parts_t kkt_parts(int32_t m, int32_t n, const double* q, const double* c, const double* l,
                         const double* u, const int8_t* ineq, const double* x, const double* y,
                         const double* Kx, const double* Kty) {
  parts_t r;
  double* tm = (double*)xalloc((size_t)m, sizeof(double));
  double* tn = (double*)xalloc((size_t)n, sizeof(double));
#pragma omp parallel for schedule(static)
  for (int32_t i = 0; i < m; ++i) {
    double v = Kx[i] - q[i];
    if (ineq[i]) v = (q[i] - Kx[i]) > 0.0 ? (q[i] - Kx[i]) : 0.0;
    tm[i] = v * v;
  }
  r.rp2 = blocked_sum(m, tm);
#pragma omp parallel for schedule(static)
  for (int32_t j = 0; j < n; ++j) {
    double g = c[j] - Kty[j];
    double d = g - proj_lambda(g, l[j], u[j]);
    tn[j] = d * d;
  }
  r.rd2 = blocked_sum(n, tn);
  r.pobj = dot(n, c, x);
#pragma omp parallel for schedule(static)
  for (int32_t j = 0; j < n; ++j) {
    double lam = proj_lambda(c[j] - Kty[j], l[j], u[j]);
    double lp = lam > 0.0 ? lam : 0.0, lm = lam < 0.0 ? -lam : 0.0;
    tn[j] = (lp > 0.0 ? l[j] * lp : 0.0) - (lm > 0.0 ? u[j] * lm : 0.0);
  }
  r.dobj = dot(m, q, y) + blocked_sum(n, tn);
  free(tm); free(tn);
  return r;
}

static double kkt_omega(parts_t p, double omega, int power) {
  double w = power == 1 ? omega : omega * omega;
  double gap = p.dobj - p.pobj;
  return sqrt(w * p.rp2 + p.rd2 / w + gap * gap);
}

typedef struct {
  double rel_kkt, rel_gap, rel_p, rel_d, pobj, dobj;
} rel_t;

/* Section 4.1: the relative termination quantities on the original LP. */
static rel_t relative_errors(parts_t p, double qnorm, double cnorm) {
  rel_t r;
  r.pobj = p.pobj; r.dobj = p.dobj;
  r.rel_gap = fabs(p.dobj - p.pobj) / (1.0 + fabs(p.dobj) + fabs(p.pobj));
  r.rel_p = sqrt(p.rp2) / (1.0 + qnorm);
  r.rel_d = sqrt(p.rd2) / (1.0 + cnorm);
  r.rel_kkt = r.rel_gap;
  if (r.rel_p > r.rel_kkt) r.rel_kkt = r.rel_p;
  if (r.rel_d > r.rel_kkt) r.rel_kkt = r.rel_d;
  if (isnan(r.rel_gap) || isnan(r.rel_p) || isnan(r.rel_d)) r.rel_kkt = NAN;
  return r;
}

typedef struct {
  parts_t scaled;   /* on the scaled LP: drives KKT_omega */
  rel_t rel;        /* on the original LP: drives termination */
} eval_t;

/* Evaluate a scaled iterate (xh, yh): scaled KKT pieces with K~ (FP64) and the
 * unscaled termination quantities with a separate unscaled copy of K at
 * x = D2 xh, y = D1 yh. */
static eval_t evaluate_point(const lp_t* P, const double* xh, const double* yh, double* wm,
                             double* wn, double* wm2, double* wn2) {
  eval_t e;
  int32_t m = P->m, n = P->n;
  spmv(&P->K, xh, wm);
  spmv(&P->Kt, yh, wn);
  e.scaled = kkt_parts(m, n, P->q, P->c, P->l, P->u, P->ineq, xh, yh, wm, wn);
  double* xo = (double*)xalloc((size_t)n, sizeof(double));
  double* yo = (double*)xalloc((size_t)m, sizeof(double));
  for (int32_t j = 0; j < n; ++j) xo[j] = P->D2[j] * xh[j];
  for (int32_t i = 0; i < m; ++i) yo[i] = P->D1[i] * yh[i];
  spmv(&P->K0, xo, wm2);
  spmv(&P->K0t, yo, wn2);
  parts_t pu = kkt_parts(m, n, P->q0, P->c0, P->l0, P->u0, P->ineq, xo, yo, wm2, wn2);
  e.rel = relative_errors(pu, P->qnorm0, P->cnorm0);
  free(xo); free(yo);
  return e;
}

/* ---------------------------------------------------------------- infeasibility */

static int check_problem(const orc_problem* p);

typedef struct {
  double dro, dro_abs, r2, ny2;  /* dual ray: q'y + l'lam+ - u'lam-, the sum of its terms' magnitudes,
                                    ||K'y + lam||^2, ||y||^2 */
  double pro, pro_abs, v2, nx2;  /* primal ray: c'x, sum |c_j x_j|, ||violation of Kx||^2, ||x||^2 */
} rays_t;

/* Farkas quantities of a candidate direction (xd, yd) on the unscaled
 * >=-form LP (K0, q0, c0, l0, u0).  Dual ray: y = yd with its inequality
 * entries clipped at 0; g = -K0'y; lam = proj_Lambda(g); residual g - lam,
 * i.e. K0'y + lam; objective q0'y + l0'lam+ - u0'lam- (0 * inf := 0).
 * Primal ray: x = xd projected onto the recession cone of [l0, u0] (0 where
 * both bounds are finite, max(., 0) / min(., 0) where only l0 / only u0 is);
 * violation of K0 x: the entry itself on EQ rows, min(entry, 0) on the other
 * rows; objective c0'x.  xr, yr, lam receive the projected rays. */
static rays_t ray_parts(const lp_t* P, const double* xd, const double* yd, double* xr, double* yr,
                        double* lam, double* wm, double* wn) {
  rays_t r;
  int32_t m = P->m, n = P->n;
  double* tm = (double*)xalloc((size_t)m, sizeof(double));
  double* tn = (double*)xalloc((size_t)n, sizeof(double));
  for (int32_t i = 0; i < m; ++i) yr[i] = (P->ineq[i] && yd[i] < 0.0) ? 0.0 : yd[i];
  spmv(&P->K0t, yr, wn);
  for (int32_t j = 0; j < n; ++j) {
    double g = -wn[j];
    lam[j] = proj_lambda(g, P->l0[j], P->u0[j]);
    double d = g - lam[j];
    tn[j] = d * d;
  }
  r.r2 = blocked_sum(n, tn);
  for (int32_t j = 0; j < n; ++j) {
    double lp = lam[j] > 0.0 ? lam[j] : 0.0, lm = lam[j] < 0.0 ? -lam[j] : 0.0;
    tn[j] = (lp > 0.0 ? P->l0[j] * lp : 0.0) - (lm > 0.0 ? P->u0[j] * lm : 0.0);
  }
  r.dro = dot(m, P->q0, yr) + blocked_sum(n, tn);
  for (int32_t j = 0; j < n; ++j) {
    double lp = lam[j] > 0.0 ? lam[j] : 0.0, lm = lam[j] < 0.0 ? -lam[j] : 0.0;
    tn[j] = (lp > 0.0 ? fabs(P->l0[j]) * lp : 0.0) + (lm > 0.0 ? fabs(P->u0[j]) * lm : 0.0);
  }
  for (int32_t i = 0; i < m; ++i) tm[i] = fabs(P->q0[i] * yr[i]);
  r.dro_abs = blocked_sum(m, tm) + blocked_sum(n, tn);
  r.ny2 = sumsq(m, yr);
  for (int32_t j = 0; j < n; ++j) {
    int lf = isfinite(P->l0[j]), uf = isfinite(P->u0[j]);
    double v = xd[j];
    if (lf && uf) v = 0.0;
    else if (lf) v = v > 0.0 ? v : 0.0;
    else if (uf) v = v < 0.0 ? v : 0.0;
    xr[j] = v;
  }
  spmv(&P->K0, xr, wm);
  for (int32_t i = 0; i < m; ++i) {
    double v = wm[i];
    if (P->ineq[i]) v = v < 0.0 ? v : 0.0;
    tm[i] = v * v;
  }
  r.v2 = blocked_sum(m, tm);
  r.pro = dot(n, P->c0, xr);
  for (int32_t j = 0; j < n; ++j) tn[j] = fabs(P->c0[j] * xr[j]);
  r.pro_abs = blocked_sum(n, tn);
  r.nx2 = sumsq(n, xr);
  free(tm); free(tn);
  return r;
}

/* A ray's objective must exceed eps times the magnitudes it is summed from
 * (so that cancellation cannot fake its sign) and bound its residual by the
 * factor eps. */
static int ray_dual_ok(rays_t r, double eps) {
  return r.dro > eps * r.dro_abs && r.dro > 0.0 && sqrt(r.r2) <= eps * r.dro;
}
static int ray_primal_ok(rays_t r, double eps) {
  return -r.pro > eps * r.pro_abs && r.pro < 0.0 && sqrt(r.v2) <= eps * -r.pro;
}

int orc_ray_test(const orc_problem* p, const double* x_dir, const double* y_dir, double eps, double* out,
                 double* ray_x, double* ray_y, double* lam) {
  if (check_problem(p)) return -1;
  lp_t P;
  if (lp_normalize(p, &P)) return -1;
  int32_t m = P.m, n = P.n;
  double* yd = (double*)xalloc((size_t)m, sizeof(double));
  double* xr = (double*)xalloc((size_t)n, sizeof(double));
  double* yr = (double*)xalloc((size_t)m, sizeof(double));
  double* lm = (double*)xalloc((size_t)n, sizeof(double));
  double* wm = (double*)xalloc((size_t)m, sizeof(double));
  double* wn = (double*)xalloc((size_t)n, sizeof(double));
  for (int32_t i = 0; i < m; ++i) yd[i] = P.le[i] ? -y_dir[i] : y_dir[i];
  rays_t r = ray_parts(&P, x_dir, yd, xr, yr, lm, wm, wn);
  out[0] = r.dro; out[1] = sqrt(r.r2); out[2] = sqrt(r.ny2);
  out[3] = r.pro; out[4] = sqrt(r.v2); out[5] = sqrt(r.nx2);
  out[6] = r.dro_abs; out[7] = r.pro_abs;
  if (ray_x) memcpy(ray_x, xr, sizeof(double) * (size_t)n);
  if (ray_y) for (int32_t i = 0; i < m; ++i) ray_y[i] = P.le[i] ? -yr[i] : yr[i];
  if (lam) memcpy(lam, lm, sizeof(double) * (size_t)n);
  int v = ray_dual_ok(r, eps) ? 1 : (ray_primal_ok(r, eps) ? 2 : 0);
  free(yd); free(xr); free(yr); free(lm); free(wm); free(wn);
  lp_free(&P);
  return v;
}

/* ---------------------------------------------------------------- normalized duality gap */

/* One coordinate of the trust-region problem of rho_r: with s = 1/lam the
 * maximiser's coordinate is d(s) = clip(a s, lo, hi), a = (W^-1 g)_j, weight w
 * (omega for x, 1/omega for y), gradient g; it reaches its bound (the one a
 * points to) at the breakpoint s = bound / a. */
typedef struct {
  double t;      /* breakpoint (+inf when that bound is infinite) */
  double a, w, g, bound;
} gap_coord;

static int cmp_breakpoint(const void* p, const void* q) {
  double a = ((const gap_coord*)p)->t, b = ((const gap_coord*)q)->t;
  return (a > b) - (a < b);
}

/* rho_r at the scaled point (x, y) with K~x = kx, K~'y = kty, solved exactly.
 * The objective L(x, yh) - L(xh, y) is linear in d = zh - z with gradient
 * g = (K'y - c, q - Kx).  Over the box Z - z intersected with the ball
 * ||d||_omega <= r its maximiser is d(s) = proj_{Z - z}(s W^-1 g) at the
 * largest s >= 0 with ||d(s)||_omega <= r (s = inf when the ball never binds).
 * ||d(s)||_omega^2 = A s^2 + C on each interval between consecutive
 * breakpoints, A summing w a^2 over the coordinates not yet at their bound and
 * C summing w bound^2 over those at it; it does not decrease with s.  The
 * breakpoints are sorted, the interval on which ||d||^2 reaches r^2 is found,
 * its A and C are summed afresh and s = sqrt((r^2 - C) / A) solved there. */
static double normalized_gap(const lp_t* P, const double* x, const double* y, const double* kx,
                             const double* kty, double omega, double r) {
  if (!(r > 0.0)) return 0.0;
  int32_t m = P->m, n = P->n;
  gap_coord* cs = (gap_coord*)xalloc((size_t)n + (size_t)m, sizeof(gap_coord));
  int64_t nc = 0;
  for (int32_t j = 0; j < n; ++j) {
    double g = kty[j] - P->c[j], a = g / omega;
    if (a == 0.0) continue;
    double b = a > 0.0 ? P->u[j] - x[j] : P->l[j] - x[j];
    gap_coord e = {isfinite(b) ? b / a : INFINITY, a, omega, g, b};
    cs[nc++] = e;
  }
  for (int32_t i = 0; i < m; ++i) {
    double g = P->q[i] - kx[i], a = g * omega;
    if (a == 0.0) continue;
    double b = a > 0.0 ? INFINITY : (P->ineq[i] ? -y[i] : -INFINITY);
    gap_coord e = {isfinite(b) ? b / a : INFINITY, a, 1.0 / omega, g, b};
    cs[nc++] = e;
  }
  qsort(cs, (size_t)nc, sizeof(gap_coord), cmp_breakpoint);
  double r2 = r * r;
  /* the first breakpoint index `cut` such that ||d(t_cut)||^2 >= r^2: the
   * coordinates before it are at their bounds on the crossing interval */
  double A = 0.0, C = 0.0;
  for (int64_t q = 0; q < nc; ++q) A += cs[q].w * cs[q].a * cs[q].a;
  int64_t cut = 0;
  while (cut < nc && isfinite(cs[cut].t)) {
    double t = cs[cut].t;
    if (A * t * t + C >= r2) break;
    A -= cs[cut].w * cs[cut].a * cs[cut].a;
    C += cs[cut].w * cs[cut].bound * cs[cut].bound;
    ++cut;
  }
  /* sums of the crossing interval taken afresh (the running ones above only
   * locate it); every coordinate from `cut` on is free there */
  double* ta = (double*)xalloc((size_t)nc + 1, sizeof(double));
  double* tc = (double*)xalloc((size_t)nc + 1, sizeof(double));
  for (int64_t q = 0; q < nc; ++q) {
    ta[q] = q >= cut ? cs[q].w * (cs[q].a * cs[q].a) : 0.0;
    tc[q] = q < cut ? cs[q].w * (cs[q].bound * cs[q].bound) : 0.0;
  }
  A = blocked_sum(nc, ta);
  C = blocked_sum(nc, tc);
  double s = INFINITY;   /* the ball does not bind: every coordinate at its bound */
  if (cut < nc) s = A > 0.0 ? sqrt((r2 - C > 0.0 ? r2 - C : 0.0) / A) : 0.0;
  for (int64_t q = 0; q < nc; ++q) {
    double d;
    if (q < cut || !isfinite(s)) d = cs[q].bound;
    else {
      d = cs[q].a * s;
      if (cs[q].a > 0.0 ? d > cs[q].bound : d < cs[q].bound) d = cs[q].bound;
    }
    ta[q] = cs[q].g * d;
  }
  double G = blocked_sum(nc, ta);
  free(cs); free(ta); free(tc);
  return G / r;
}

static double weighted_dist(int32_t n, int32_t m, const double* x, const double* x0, const double* y,
                            const double* y0, double omega) {
  return sqrt(omega * dist2(n, x, x0) + dist2(m, y, y0) / omega);
}

double orc_normalized_gap(const orc_problem* p, int32_t ruiz_iters, double pc_alpha, const double* x,
                          const double* y, double omega, double r) {
  if (check_problem(p)) return -1.0;
  lp_t P;
  if (lp_normalize(p, &P)) return -1.0;
  lp_scale(&P, ruiz_iters, pc_alpha);
  double* kx = (double*)xalloc((size_t)P.m, sizeof(double));
  double* kty = (double*)xalloc((size_t)P.n, sizeof(double));
  spmv(&P.K, x, kx);
  spmv(&P.Kt, y, kty);
  double rho = normalized_gap(&P, x, y, kx, kty, omega, r);
  free(kx); free(kty);
  lp_free(&P);
  return rho;
}

int orc_restart_reason(double kc, double kkt0, double kprev, int64_t t, int64_t k,
                       double beta_suff, double beta_nec, double beta_art) {
  /* Section 3.4, restart criteria */
  if (kc <= beta_suff * kkt0) return 1;                    /* (i) sufficient decay */
  if (kc <= beta_nec * kkt0 && kc > kprev) return 2;       /* (ii) necessary decay, no local progress */
  if ((double)t >= beta_art * (double)k) return 3;         /* (iii) long inner loop */
  return 0;
}

double orc_primal_weight_update(double dx, double dy, double omega, double theta, double eps_zero) {
  /* Section 2.2, primal weight update, smoothed in log space */
  if (dx > eps_zero && dy > eps_zero) return exp(theta * log(dy / dx) + (1.0 - theta) * log(omega));
  return omega;
}

void orc_default_options(orc_options* o) {
  o->eps_rel = 1e-4;
  o->max_iter = 1000000;
  o->time_limit_s = 3600.0;
  o->eval_period = 64;
  o->ruiz_iters = 10;
  o->pc_alpha = 1.0;
  o->pw_theta = 0.5;
  o->eps_zero = 1e-10;
  o->beta_suff = 0.2;
  o->beta_nec = 0.8;
  o->beta_art = 0.36;
  o->a_precision = 0;
  o->kkt_omega_power = 2;
  o->threads = 0;
  o->detect_infeas = 1;
  o->eps_infeas = 1e-8;
  o->infeas_every = 4;
  o->restart_metric = 0;
}

static int check_problem(const orc_problem* p) {
  if (!p || p->m < 0 || p->n < 1 || p->nnz < 0) return -1;
  if (!p->row_ptr || (p->nnz > 0 && (!p->col_idx || !p->val))) return -1;
  if (!p->c || !p->l || !p->u || (p->m > 0 && (!p->b || !p->row_type))) return -1;
  if (p->row_ptr[0] != 0 || p->row_ptr[p->m] != p->nnz) return -1;
  return 0;
}

int orc_rescale(const orc_problem* p, int32_t ruiz_iters, double pc_alpha, double* D1, double* D2,
                double* val_scaled) {
  if (check_problem(p)) return -1;
  lp_t P;
  if (lp_normalize(p, &P)) return -1;
  lp_scale(&P, ruiz_iters, pc_alpha);
  memcpy(D1, P.D1, sizeof(double) * (size_t)P.m);
  memcpy(D2, P.D2, sizeof(double) * (size_t)P.n);
  memcpy(val_scaled, P.K.v, sizeof(double) * (size_t)P.K.nnz);
  lp_free(&P);
  return 0;
}

int orc_pdhg_step(int32_t m, int32_t n, const int32_t* rp, const int32_t* ci, const double* v,
                  const double* q, const double* c, const double* l, const double* u,
                  const int8_t* ineq, const double* x, const double* y, double tau, double sigma,
                  double* x_out, double* y_out) {
  /* eq. (pdhg): x' = proj_X(x - tau (c - K'y)); y' = proj_Y(y + sigma (q - K(2x' - x))) */
  double* kty = (double*)xalloc((size_t)n, sizeof(double));
  double* w = (double*)xalloc((size_t)n, sizeof(double));
  for (int32_t i = 0; i < m; ++i)
    for (int64_t p = rp[i]; p < rp[i + 1]; ++p) kty[ci[p]] += v[p] * y[i];
  for (int32_t j = 0; j < n; ++j) {
    x_out[j] = clampd(x[j] - tau * (c[j] - kty[j]), l[j], u[j]);
    w[j] = 2.0 * x_out[j] - x[j];
  }
  for (int32_t i = 0; i < m; ++i) {
    double s = 0.0;
    for (int64_t p = rp[i]; p < rp[i + 1]; ++p) s += v[p] * w[ci[p]];
    double yi = y[i] + sigma * (q[i] - s);
    if (ineq[i] && yi < 0.0) yi = 0.0;
    y_out[i] = yi;
  }
  free(kty); free(w);
  return 0;
}

int orc_evaluate(const orc_problem* p, const double* x, const double* y, double omega,
                 int32_t omega_power, double* out) {
  if (check_problem(p)) return -1;
  lp_t P;
  if (lp_normalize(p, &P)) return -1;
  int32_t m = P.m, n = P.n;
  double* yk = (double*)xalloc((size_t)m, sizeof(double));
  double* kx = (double*)xalloc((size_t)m, sizeof(double));
  double* kty = (double*)xalloc((size_t)n, sizeof(double));
  for (int32_t i = 0; i < m; ++i) yk[i] = P.le[i] ? -y[i] : y[i];
  spmv(&P.K0, x, kx);
  spmv(&P.K0t, yk, kty);
  parts_t pu = kkt_parts(m, n, P.q0, P.c0, P.l0, P.u0, P.ineq, x, yk, kx, kty);
  rel_t r = relative_errors(pu, P.qnorm0, P.cnorm0);
  out[0] = r.rel_kkt; out[1] = r.rel_gap; out[2] = r.rel_p; out[3] = r.rel_d;
  out[4] = r.pobj; out[5] = r.dobj;
  out[6] = sqrt(pu.rp2); out[7] = sqrt(pu.rd2); out[8] = fabs(pu.dobj - pu.pobj);
  out[9] = kkt_omega(pu, omega, omega_power);
  free(yk); free(kx); free(kty);
  lp_free(&P);
  return 0;
}

int orc_reduced_costs(const orc_problem* p, const double* y, double* lam) {
  if (check_problem(p)) return -1;
  lp_t P;
  if (lp_normalize(p, &P)) return -1;
  double* yk = (double*)xalloc((size_t)P.m, sizeof(double));
  double* kty = (double*)xalloc((size_t)P.n, sizeof(double));
  for (int32_t i = 0; i < P.m; ++i) yk[i] = P.le[i] ? -y[i] : y[i];
  spmv(&P.K0t, yk, kty);
  for (int32_t j = 0; j < P.n; ++j) lam[j] = proj_lambda(P.c0[j] - kty[j], P.l0[j], P.u0[j]);
  free(yk); free(kty);
  lp_free(&P);
  return 0;
}

/* ---------------------------------------------------------------- solve */

int orc_solve(const orc_problem* p, const orc_options* opt, double* x_user, double* y_user,
              double* rc, orc_info* info, orc_trace* tr, double* x_hat, double* y_hat) {
  orc_options o;
  if (opt) o = *opt; else orc_default_options(&o);
  if (check_problem(p) || o.eval_period < 1 || o.max_iter < 0 || o.infeas_every < 1 ||
      (o.restart_metric != 0 && o.restart_metric != 1)) return -1;
#ifdef _OPENMP
  if (o.threads > 0) omp_set_num_threads(o.threads);
#endif
  double t_start = now_s();
  lp_t P;
  if (lp_normalize(p, &P)) return -1;
  lp_scale(&P, o.ruiz_iters, o.pc_alpha);
  if (o.a_precision == 1) lp_round_fp32(&P);
  int32_t m = P.m, n = P.n;
  const csr* Ks = &P.K;
  const csr* Kts = &P.Kt;
  void (*step_spmv)(const csr*, const double*, double*) = o.a_precision == 1 ? spmv_f : spmv;

  double* x = (double*)xalloc((size_t)n, sizeof(double));
  double* y = (double*)xalloc((size_t)m, sizeof(double));
  double* xn = (double*)xalloc((size_t)n, sizeof(double));
  double* yn = (double*)xalloc((size_t)m, sizeof(double));
  double* x0 = (double*)xalloc((size_t)n, sizeof(double));
  double* y0 = (double*)xalloc((size_t)m, sizeof(double));
  double* xs = (double*)xalloc((size_t)n, sizeof(double));
  double* ys = (double*)xalloc((size_t)m, sizeof(double));
  double* xa = (double*)xalloc((size_t)n, sizeof(double));
  double* ya = (double*)xalloc((size_t)m, sizeof(double));
  double* kty = (double*)xalloc((size_t)n, sizeof(double));
  double* w = (double*)xalloc((size_t)n, sizeof(double));
  double* kw = (double*)xalloc((size_t)m, sizeof(double));
  double* dx = (double*)xalloc((size_t)n, sizeof(double));
  double* dy = (double*)xalloc((size_t)m, sizeof(double));
  double* kdx = (double*)xalloc((size_t)m, sizeof(double));
  double* wm = (double*)xalloc((size_t)m, sizeof(double));
  double* wn = (double*)xalloc((size_t)n, sizeof(double));
  double* wm2 = (double*)xalloc((size_t)m, sizeof(double));
  double* wn2 = (double*)xalloc((size_t)n, sizeof(double));
  /* infeasibility candidates: unscaled directions and their projected rays */
  double* cdx = (double*)xalloc((size_t)n, sizeof(double));
  double* cdy = (double*)xalloc((size_t)m, sizeof(double));
  double* rx[2] = {(double*)xalloc((size_t)n, sizeof(double)), (double*)xalloc((size_t)n, sizeof(double))};
  double* ry[2] = {(double*)xalloc((size_t)m, sizeof(double)), (double*)xalloc((size_t)m, sizeof(double))};
  double* rl[2] = {(double*)xalloc((size_t)n, sizeof(double)), (double*)xalloc((size_t)n, sizeof(double))};
  rays_t ray = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  int ray_src = 0;

  /* Section 4.1 initialisation: the zero vector, projected onto X */
  for (int32_t j = 0; j < n; ++j) x[j] = clampd(0.0, P.l[j], P.u[j]);
  memcpy(x0, x, sizeof(double) * (size_t)n);

  /* Algorithm 1, initialization: step size 1/||K~||_inf, primal weight ||c~|| / ||q~|| */
  double kmax = 0.0;
  for (int64_t q = 0; q < Ks->nnz; ++q) kmax = fabs(Ks->v[q]) > kmax ? fabs(Ks->v[q]) : kmax;
  double eta_hat = kmax > 0.0 ? 1.0 / kmax : 1.0;
  double cn = sqrt(sumsq(n, P.c)), qn = sqrt(sumsq(m, P.q));
  double omega = (cn > o.eps_zero && qn > o.eps_zero) ? cn / qn : 1.0;

  int64_t k = 0, t = 0, attempts = 0, restarts = 0, evals = 0, k_last_eval = 0;
  double sum_eta = 0.0;
  int status = 0, ret_avg = 0;
  rel_t ret_rel;
  double setup_end = now_s();

  eval_t e0 = evaluate_point(&P, x, y, wm, wn, wm2, wn2);
  ret_rel = e0.rel;
  /* the restart metric's reference value (rho: +inf before the first restart) */
  double kkt0 = o.restart_metric == 1 ? INFINITY : kkt_omega(e0.scaled, omega, o.kkt_omega_power), kkt_prev = kkt0;
  if (!isfinite(e0.rel.rel_kkt)) status = 4;
  else if (e0.rel.rel_kkt <= o.eps_rel) status = 1;
  else if (o.max_iter == 0) status = 2;

  while (!status) {
    /* Algorithm 2: one PDHG step with the adaptive step-size heuristic */
    double eta = eta_hat, eta_next = eta_hat;
    double tau = 0.0, sigma = 0.0;
    for (;;) {
      attempts++;
      tau = eta / omega;
      sigma = eta * omega;
      step_spmv(Kts, y, kty);
#pragma omp parallel for schedule(static)
      for (int32_t j = 0; j < n; ++j) {
        xn[j] = clampd(x[j] - tau * (P.c[j] - kty[j]), P.l[j], P.u[j]);
        w[j] = 2.0 * xn[j] - x[j];
        dx[j] = xn[j] - x[j];
      }
      step_spmv(Ks, w, kw);
#pragma omp parallel for schedule(static)
      for (int32_t i = 0; i < m; ++i) {
        double yi = y[i] + sigma * (P.q[i] - kw[i]);
        if (P.ineq[i] && yi < 0.0) yi = 0.0;
        yn[i] = yi;
        dy[i] = yi - y[i];
      }
      step_spmv(Ks, dx, kdx);
      double nx = sumsq(n, dx), ny = sumsq(m, dy);
      double num = omega * nx + ny / omega;
      double den = 2.0 * fabs(dot(m, dy, kdx));
      double eta_bar = den > 0.0 ? num / den : INFINITY;
      double kk = (double)(k + 2);
      double a = (1.0 - pow(kk, -0.3)) * eta_bar, b = (1.0 + pow(kk, -0.6)) * eta;
      eta_next = a < b ? a : b;
      int acc = eta <= eta_bar;
      if (tr && tr->n_att < tr->cap_att) {
        int64_t s = tr->n_att++;
        tr->att_k[s] = k; tr->att_eta[s] = eta; tr->att_etabar[s] = eta_bar; tr->att_acc[s] = (int8_t)acc;
      }
      if (!isfinite(num) || isnan(den) || isnan(eta_next)) { status = 4; break; }
      if (acc) break;
      eta = eta_next;
    }
    if (status) break;
    /* accepted: z <- z', eta_hat <- eta', average weights += eta */
    { double* s = x; x = xn; xn = s; }
    { double* s = y; y = yn; yn = s; }
    eta_hat = eta_next;
    sum_eta += eta;
    for (int32_t j = 0; j < n; ++j) xs[j] += eta * x[j];
    for (int32_t i = 0; i < m; ++i) ys[i] += eta * y[i];
    t++; k++;
    if (now_s() - t_start > o.time_limit_s) { status = 3; ret_avg = 0; break; }
    if (k - k_last_eval < o.eval_period && k < o.max_iter) continue;

    /* evaluation: current and average iterate */
    evals++;
    k_last_eval = k;
    for (int32_t j = 0; j < n; ++j) xa[j] = xs[j] / sum_eta;
    for (int32_t i = 0; i < m; ++i) ya[i] = ys[i] / sum_eta;
    eval_t ec = evaluate_point(&P, x, y, wm, wn, wm2, wn2);
    eval_t ea = evaluate_point(&P, xa, ya, wm, wn, wm2, wn2);
    int avg_better = ea.rel.rel_kkt < ec.rel.rel_kkt;
    if (!isfinite(ec.rel.rel_kkt) || !isfinite(ea.rel.rel_kkt)) { status = 4; ret_rel = ec.rel; break; }
    if (ec.rel.rel_kkt <= o.eps_rel || ea.rel.rel_kkt <= o.eps_rel) {
      status = 1; ret_avg = avg_better; ret_rel = avg_better ? ea.rel : ec.rel; break;
    }
    if (o.detect_infeas && evals % o.infeas_every == 0) {
      /* Section 2.2, infeasibility detection: the last accepted step z - z_prev
       * (z_prev sits in xn, yn after the swap) and the epoch displacement z - z^{n,0} */
      rays_t rr[2];
      for (int sq = 0; sq < 2; ++sq) {
        const double* xb = sq ? x0 : xn;
        const double* yb = sq ? y0 : yn;
        for (int32_t j = 0; j < n; ++j) cdx[j] = P.D2[j] * (x[j] - xb[j]);
        for (int32_t i = 0; i < m; ++i) cdy[i] = P.D1[i] * (y[i] - yb[i]);
        rr[sq] = ray_parts(&P, cdx, cdy, rx[sq], ry[sq], rl[sq], wm, wn);
      }
      int kind = 0;
      for (int sq = 0; sq < 2 && !kind; ++sq)
        if (ray_dual_ok(rr[sq], o.eps_infeas)) { kind = 5; ray_src = sq; }
      for (int sq = 0; sq < 2 && !kind; ++sq)
        if (ray_primal_ok(rr[sq], o.eps_infeas)) { kind = 6; ray_src = sq; }
      if (kind) { status = kind; ray = rr[ray_src]; ret_avg = 0; ret_rel = ec.rel; break; }
    }
    if (k >= o.max_iter) { status = 2; ret_avg = avg_better; ret_rel = avg_better ? ea.rel : ec.rel; break; }
    /* restart candidate and restart criteria */
    double kc_cur, kc_avg;
    if (o.restart_metric == 1) {
      /* normalized duality gap of each iterate, radius = its distance to z^{n,0} */
      spmv(Ks, x, wm);
      spmv(Kts, y, wn);
      kc_cur = normalized_gap(&P, x, y, wm, wn, omega, weighted_dist(n, m, x, x0, y, y0, omega));
      spmv(Ks, xa, wm);
      spmv(Kts, ya, wn);
      kc_avg = normalized_gap(&P, xa, ya, wm, wn, omega, weighted_dist(n, m, xa, x0, ya, y0, omega));
    } else {
      kc_cur = kkt_omega(ec.scaled, omega, o.kkt_omega_power);
      kc_avg = kkt_omega(ea.scaled, omega, o.kkt_omega_power);
    }
    /* the current iterate only when clearly better; a relative difference below
     * 1e-12 is a rounding-level tie (one step into an epoch the average equals
     * the iterate) and goes to the average, the "otherwise" branch */
    int cand_avg = !(kc_cur < kc_avg - 1e-12 * kc_avg);
    double kc = cand_avg ? kc_avg : kc_cur;
    int reason = orc_restart_reason(kc, kkt0, kkt_prev, t, k, o.beta_suff, o.beta_nec, o.beta_art);
    if (reason) {
      const double* xc = cand_avg ? xa : x;
      const double* yc = cand_avg ? ya : y;
      double ddx = sqrt(dist2(n, xc, x0)), ddy = sqrt(dist2(m, yc, y0));
      omega = orc_primal_weight_update(ddx, ddy, omega, o.pw_theta, o.eps_zero);
      if (cand_avg) {
        memcpy(x, xa, sizeof(double) * (size_t)n);
        memcpy(y, ya, sizeof(double) * (size_t)m);
      }
      memcpy(x0, x, sizeof(double) * (size_t)n);
      memcpy(y0, y, sizeof(double) * (size_t)m);
      memset(xs, 0, sizeof(double) * (size_t)n);
      memset(ys, 0, sizeof(double) * (size_t)m);
      sum_eta = 0.0;
      t = 0;
      restarts++;
      kkt0 = o.restart_metric == 1 ? kc : kkt_omega(cand_avg ? ea.scaled : ec.scaled, omega, o.kkt_omega_power);
      kkt_prev = kkt0;
    } else {
      kkt_prev = kc;
    }
    if (tr && tr->n_eval < tr->cap_eval) {
      int64_t s = tr->n_eval++;
      tr->ev_k[s] = k; tr->ev_kkt_cur[s] = kc_cur; tr->ev_kkt_avg[s] = kc_avg;
      tr->ev_cand[s] = (int8_t)cand_avg; tr->ev_reason[s] = (int8_t)reason; tr->ev_omega[s] = omega;
    }
  }
  double t_end = now_s();

  /* output: unscale the returned point, flip LE duals back, reduced costs */
  const double* xr = x;
  const double* yr = y;
  if (ret_avg && sum_eta > 0.0) {
    for (int32_t j = 0; j < n; ++j) xa[j] = xs[j] / sum_eta;
    for (int32_t i = 0; i < m; ++i) ya[i] = ys[i] / sum_eta;
    xr = xa; yr = ya;
  }
  double* yo = (double*)xalloc((size_t)m, sizeof(double));
  for (int32_t j = 0; j < n; ++j) if (x_user) x_user[j] = P.D2[j] * xr[j];
  for (int32_t i = 0; i < m; ++i) yo[i] = P.D1[i] * yr[i];
  if (y_user) for (int32_t i = 0; i < m; ++i) y_user[i] = P.le[i] ? -yo[i] : yo[i];
  if (rc) {
    spmv(&P.K0t, yo, wn);
    for (int32_t j = 0; j < n; ++j) rc[j] = proj_lambda(P.c0[j] - wn[j], P.l0[j], P.u0[j]);
  }
  /* an infeasibility certificate replaces the side it certifies (unit 2-norm);
   * for a dual ray the reduced costs are its multipliers lam */
  double ray_obj = 0.0, ray_res = 0.0;
  if (status == 5 && ray.ny2 > 0.0) {
    double sc = 1.0 / sqrt(ray.ny2);
    if (y_user) for (int32_t i = 0; i < m; ++i) y_user[i] = (P.le[i] ? -ry[ray_src][i] : ry[ray_src][i]) * sc;
    if (rc) for (int32_t j = 0; j < n; ++j) rc[j] = rl[ray_src][j] * sc;
    ray_obj = ray.dro * sc;
    ray_res = sqrt(ray.r2) * sc;
  } else if (status == 6 && ray.nx2 > 0.0) {
    double sc = 1.0 / sqrt(ray.nx2);
    if (x_user) for (int32_t j = 0; j < n; ++j) x_user[j] = rx[ray_src][j] * sc;
    ray_obj = ray.pro * sc;
    ray_res = sqrt(ray.v2) * sc;
  }
  if (x_hat) memcpy(x_hat, x, sizeof(double) * (size_t)n);
  if (y_hat) memcpy(y_hat, y, sizeof(double) * (size_t)m);
  if (info) {
    info->status = status;
    info->returned_avg = ret_avg;
    info->iterations = k; info->attempts = attempts; info->restarts = restarts; info->evaluations = evals;
    info->rel_kkt = ret_rel.rel_kkt; info->rel_gap = ret_rel.rel_gap;
    info->rel_pres = ret_rel.rel_p; info->rel_dres = ret_rel.rel_d;
    info->primal_obj = ret_rel.pobj; info->dual_obj = ret_rel.dobj;
    info->omega = omega; info->eta_hat = eta_hat; info->sum_eta = sum_eta; info->kkt0 = kkt0;
    info->setup_s = setup_end - t_start; info->solve_s = t_end - setup_end;
#ifdef _OPENMP
    info->threads_used = omp_get_max_threads();
#else
    info->threads_used = 1;
#endif
    info->ray_source = (status == 5 || status == 6) ? ray_src : 0;
    info->ray_obj = ray_obj;
    info->ray_res = ray_res;
  }
  free(yo);
  free(x); free(y); free(xn); free(yn); free(x0); free(y0); free(xs); free(ys); free(xa); free(ya);
  free(kty); free(w); free(kw); free(dx); free(dy); free(kdx); free(wm); free(wn); free(wm2); free(wn2);
  free(cdx); free(cdy);
  for (int sq = 0; sq < 2; ++sq) { free(rx[sq]); free(ry[sq]); free(rl[sq]); }
  lp_free(&P);
  return 0;
}
