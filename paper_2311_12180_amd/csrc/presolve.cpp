// Presolve-lite on the host: the elementary reductions, applied until none
// applies, and the exact postsolve of the primal and dual solution.
//
// Per pass, in this order:
//   1. a column whose bounds coincide is fixed at that value (its entries move
//      into the right-hand sides, rows ascending; its cost into an offset);
//   2. rows ascending: a row without an active entry is dropped (0 must
//      satisfy it, else the LP is primal infeasible); a row with one active
//      entry a x_j {=, >=, <=} b becomes the bound b / a on x_j (both bounds
//      for EQ, the lower one for GE with a > 0 or LE with a < 0, else the upper
//      one), kept when tighter; a bound crossing the other by more than
//      1e-9 max(1, |v|) means primal infeasible, by less fixes the column;
//   3. a column without an active row is fixed at the bound its cost points
//      to (lower for c_j > 0, upper for c_j < 0, proj(0) for c_j = 0); an
//      infinite such bound means dual infeasible.
// Postsolve: the columns still active take the reduced solution; then every
// column, the active ones first and the removed ones in reverse order of
// removal, hands the multiplier of the bound it sits at (the reduced
// multiplier, or g_j = c_j - sum of a_ij y_i over its other rows) to the
// singleton row that set that bound (y = g / a) or to its own lambda_j.
#include <cmath>
#include <cstring>
#include <vector>

#include "pdlp_dev.h"

namespace pdlp {

namespace {

double tol_of(double v) { return 1e-9 * std::max(1.0, std::fabs(v)); }

}  // namespace

// Column-major copy of H's matrix (rows ascending inside a column).
void csc_of(const HostLP& H, std::vector<int32_t>& cp, std::vector<int32_t>& cr, std::vector<double>& cv) {
  cp.assign((size_t)H.n + 1, 0);
  for (int64_t e = 0; e < H.nnz; ++e) cp[(size_t)H.ci[(size_t)e] + 1]++;
  for (int32_t j = 0; j < H.n; ++j) cp[(size_t)j + 1] += cp[(size_t)j];
  cr.resize((size_t)std::max<int64_t>(H.nnz, 1));
  cv.resize((size_t)std::max<int64_t>(H.nnz, 1));
  std::vector<int32_t> pos(cp.begin(), cp.end() - 1);
  for (int32_t i = 0; i < H.m; ++i)
    for (int32_t e = H.rp[(size_t)i]; e < H.rp[(size_t)i + 1]; ++e) {
      const int32_t j = H.ci[(size_t)e];
      cr[(size_t)pos[(size_t)j]] = i;
      cv[(size_t)pos[(size_t)j]++] = H.v[(size_t)e];
    }
}

int presolve_lp(const HostLP& H, HostLP& R, Presolve& P) {
  const int32_t m = H.m, n = H.n;
  csc_of(H, P.cp, P.cr, P.cv);
  std::vector<double> b(H.b.begin(), H.b.begin() + m);
  P.lo.assign(H.l.begin(), H.l.begin() + n);
  P.hi.assign(H.u.begin(), H.u.begin() + n);
  P.row_on.assign((size_t)m, 1);
  P.col_on.assign((size_t)n, 1);
  P.xfix.assign((size_t)n, 0.0);
  P.lo_row.assign((size_t)n, -1);
  P.hi_row.assign((size_t)n, -1);
  P.order.clear();
  P.offset = 0.0;
  P.status = 0;
  auto fix = [&](int32_t j, double v) {
    P.xfix[(size_t)j] = v;
    for (int32_t k = P.cp[(size_t)j]; k < P.cp[(size_t)j + 1]; ++k) {
      const int32_t i = P.cr[(size_t)k];
      if (P.row_on[(size_t)i]) {
        const double t = P.cv[(size_t)k] * v;
        b[(size_t)i] = b[(size_t)i] - t;
      }
    }
    const double t = H.c[(size_t)j] * v;
    P.offset = P.offset + t;
    P.col_on[(size_t)j] = 0;
    P.order.push_back(j);
  };
  bool changed = true;
  while (changed) {
    changed = false;
    for (int32_t j = 0; j < n; ++j)
      if (P.col_on[(size_t)j] && P.lo[(size_t)j] == P.hi[(size_t)j]) {
        fix(j, P.lo[(size_t)j]);
        changed = true;
      }
    for (int32_t i = 0; i < m; ++i) {
      if (!P.row_on[(size_t)i]) continue;
      int cnt = 0;
      int32_t jj = -1;
      double aa = 0.0;
      for (int32_t e = H.rp[(size_t)i]; e < H.rp[(size_t)i + 1] && cnt < 2; ++e)
        if (P.col_on[(size_t)H.ci[(size_t)e]]) {
          ++cnt;
          jj = H.ci[(size_t)e];
          aa = H.v[(size_t)e];
        }
      const int8_t t = H.rt[(size_t)i];
      if (cnt == 0) {
        const double tl = 1e-9 * (1.0 + std::fabs(H.b[(size_t)i]));
        const double bi = b[(size_t)i];
        if ((t == PDLP_ROW_EQ && std::fabs(bi) > tl) || (t == PDLP_ROW_GE && bi > tl) ||
            (t == PDLP_ROW_LE && bi < -tl)) {
          P.status = PDLP_PRIMAL_INFEASIBLE;
          return P.status;
        }
        P.row_on[(size_t)i] = 0;
        changed = true;
      } else if (cnt == 1) {
        const double v = b[(size_t)i] / aa;
        const bool lower = t == PDLP_ROW_EQ || ((t == PDLP_ROW_GE) == (aa > 0.0));
        const bool upper = t == PDLP_ROW_EQ || !lower;
        double& lo = P.lo[(size_t)jj];
        double& hi = P.hi[(size_t)jj];
        if (lower && v > lo) {
          lo = v;
          P.lo_row[(size_t)jj] = i;
        }
        if (upper && v < hi) {
          hi = v;
          P.hi_row[(size_t)jj] = i;
        }
        if (lo > hi) {
          if (lo - hi > tol_of(v)) {
            P.status = PDLP_PRIMAL_INFEASIBLE;
            return P.status;
          }
          if (P.lo_row[(size_t)jj] == i) hi = lo;
          else lo = hi;
        }
        P.row_on[(size_t)i] = 0;
        changed = true;
      }
    }
    for (int32_t j = 0; j < n; ++j) {
      if (!P.col_on[(size_t)j]) continue;
      bool any = false;
      for (int32_t k = P.cp[(size_t)j]; k < P.cp[(size_t)j + 1] && !any; ++k) any = P.row_on[(size_t)P.cr[(size_t)k]] != 0;
      if (any) continue;
      const double cj = H.c[(size_t)j];
      double v;
      if (cj > 0.0) v = P.lo[(size_t)j];
      else if (cj < 0.0) v = P.hi[(size_t)j];
      else v = std::min(std::max(0.0, P.lo[(size_t)j]), P.hi[(size_t)j]);
      if (!std::isfinite(v)) {
        P.status = PDLP_DUAL_INFEASIBLE;
        return P.status;
      }
      fix(j, v);
      changed = true;
    }
  }
  P.b = b;
  // the reduced LP: active rows and columns in their original order
  P.rows.clear();
  P.cols.clear();
  std::vector<int32_t> newc((size_t)n, -1);
  for (int32_t j = 0; j < n; ++j)
    if (P.col_on[(size_t)j]) {
      newc[(size_t)j] = (int32_t)P.cols.size();
      P.cols.push_back(j);
    }
  for (int32_t i = 0; i < m; ++i)
    if (P.row_on[(size_t)i]) P.rows.push_back(i);
  R = HostLP{};
  R.m = (int32_t)P.rows.size();
  R.n = (int32_t)P.cols.size();
  R.rp.assign(1, 0);
  for (int32_t i : P.rows) {
    for (int32_t e = H.rp[(size_t)i]; e < H.rp[(size_t)i + 1]; ++e) {
      const int32_t j = H.ci[(size_t)e];
      if (P.col_on[(size_t)j]) {
        R.ci.push_back(newc[(size_t)j]);
        R.v.push_back(H.v[(size_t)e]);
      }
    }
    R.rp.push_back((int32_t)R.ci.size());
    R.b.push_back(b[(size_t)i]);
    R.rt.push_back(H.rt[(size_t)i]);
  }
  R.nnz = (int64_t)R.ci.size();
  for (int32_t j : P.cols) {
    R.c.push_back(H.c[(size_t)j]);
    R.l.push_back(P.lo[(size_t)j]);
    R.u.push_back(P.hi[(size_t)j]);
  }
  return 0;
}

void postsolve_lp(const HostLP& H, const Presolve& P, const double* xr, const double* yr, const double* lamr,
                  double* x, double* y, double* lam, bool ray) {
  // ray: (xr, yr, lamr) is a ray of the reduced LP; the same steps with zero
  // costs and the removed columns at 0 extend it to a ray of the given LP
  // (the objective terms of the bounds that singleton rows set move into
  // those rows' b'y, and a removed column's own multiplier absorbs the rest)
  const int32_t m = H.m, n = H.n;
  for (int32_t j = 0; j < n; ++j) {
    x[j] = ray ? 0.0 : P.xfix[(size_t)j];
    lam[j] = 0.0;
  }
  for (int32_t i = 0; i < m; ++i) y[i] = 0.0;
  for (size_t k = 0; k < P.cols.size(); ++k) x[P.cols[k]] = xr[k];
  for (size_t k = 0; k < P.rows.size(); ++k) y[P.rows[k]] = yr[k];
  auto coef = [&](int32_t i, int32_t j) {
    for (int32_t k = P.cp[(size_t)j]; k < P.cp[(size_t)j + 1]; ++k)
      if (P.cr[(size_t)k] == i) return P.cv[(size_t)k];
    return 0.0;
  };
  auto assign = [&](int32_t j, double mu) {
    if (mu == 0.0) return;
    const int32_t side = mu > 0.0 ? P.lo_row[(size_t)j] : P.hi_row[(size_t)j];
    if (side >= 0) y[side] = mu / coef(side, j);
    else lam[j] = mu;
  };
  for (size_t k = 0; k < P.cols.size(); ++k) assign(P.cols[k], lamr[k]);
  for (size_t q = P.order.size(); q-- > 0;) {
    const int32_t j = P.order[q];
    double g = ray ? 0.0 : H.c[(size_t)j];
    for (int32_t k = P.cp[(size_t)j]; k < P.cp[(size_t)j + 1]; ++k) {
      const int32_t i = P.cr[(size_t)k];
      if (i != P.lo_row[(size_t)j] && i != P.hi_row[(size_t)j]) {
        const double t = P.cv[(size_t)k] * y[i];
        g = g - t;
      }
    }
    assign(j, g);
  }
}

}  // namespace pdlp
