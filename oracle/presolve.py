"""Presolve-lite reference: plain loops, FP64.

TEST INFRASTRUCTURE ONLY (like the rest of this package): it is the yardstick
for the solver library's presolve; the product never imports it.

The paper notes that presolve helps PDLP-type solvers (Section 4, its
comparison with and without the commercial presolve); the reductions here are
the elementary ones, applied until none applies, in this fixed order per pass:

  1. a column whose bounds coincide is fixed at that value: its entries move
     into the right-hand sides (b_i -= a_ij x_j over the column's active rows,
     rows ascending) and its cost into the objective offset;
  2. rows, ascending: a row with no active entry is dropped (its right-hand
     side must be satisfied by 0, else the LP is primal infeasible); a row
     with one active entry a x_j {=, >=, <=} b becomes a bound v = b / a on
     x_j (both bounds for EQ; the lower bound for GE with a > 0 or LE with
     a < 0; the upper bound otherwise), kept only when it is tighter, and the
     row is dropped;
  3. a column with no active row is fixed at the bound its cost points to
     (lower if c_j > 0, upper if c_j < 0, proj(0) if c_j = 0); an infinite
     such bound means the LP is dual infeasible (or infeasible).

A new bound v is within the tolerance tol(v) = 1e-9 max(1, |v|) of the other
bound: equal (the column is fixed); beyond it: primal infeasible.

Postsolve (exact for these reductions): columns are visited in the reverse
order of their removal, the columns still active first.  For column j, with
g_j = c_j - sum_i a_ij y_i over the other rows (all of which have their y by
then: a row removed after column j holds its multiplier from a column removed
later still), g_j > 0 is the multiplier of x_j's lower bound and g_j < 0 of
its upper bound; it goes to the singleton row that set that bound
(y_row = g_j / a_row,j) or, if the bound is the column's own, to lambda_j.  For
a column still active, its reduced multiplier lambda_r,j plays the part of g_j.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np

import lpgen

EQ, GE, LE = lpgen.ROW_EQ, lpgen.ROW_GE, lpgen.ROW_LE


def _tol(v: float) -> float:
    return 1e-9 * max(1.0, abs(v))


@dataclasses.dataclass
class Record:
    status: str                 # "ok", "primal_infeasible", "dual_infeasible"
    row_keep: np.ndarray        # bool [m]
    col_keep: np.ndarray        # bool [n]
    xfix: np.ndarray            # [n] values of removed columns
    lo_row: np.ndarray          # [n] row that set the lower bound (-1: the column's own)
    hi_row: np.ndarray          # [n] row that set the upper bound
    col_order: list             # removed columns in removal order
    offset: float               # objective contribution of the removed columns
    lo: np.ndarray              # final bounds [n]
    hi: np.ndarray


def presolve(p) -> tuple[Optional[lpgen.Problem], Record]:
    m, n = int(p.m), int(p.n)
    rp, ci, val = np.asarray(p.row_ptr), np.asarray(p.col_idx), np.asarray(p.val, float)
    # the columns' entries (rows ascending), from the rows
    col_rows = [[] for _ in range(n)]
    for i in range(m):
        for e in range(rp[i], rp[i + 1]):
            col_rows[ci[e]].append((i, val[e]))
    b = np.array(p.b, float)
    lo = np.array(p.l, float)
    hi = np.array(p.u, float)
    rt = np.asarray(p.row_type)
    row_on = np.ones(m, bool)
    col_on = np.ones(n, bool)
    xfix = np.zeros(n)
    lo_row = np.full(n, -1, np.int64)
    hi_row = np.full(n, -1, np.int64)
    order = []
    offset = 0.0
    status = "ok"

    def rec():
        return Record(status, row_on.copy(), col_on.copy(), xfix.copy(), lo_row.copy(), hi_row.copy(),
                      list(order), offset, lo.copy(), hi.copy())

    def fix(j, v):
        nonlocal offset
        xfix[j] = v
        for i, a in col_rows[j]:
            if row_on[i]:
                b[i] -= a * v
        offset += p.c[j] * v
        col_on[j] = False
        order.append(j)

    changed = True
    while changed and status == "ok":
        changed = False
        # 1. fixed columns
        for j in range(n):
            if col_on[j] and lo[j] == hi[j]:
                fix(j, lo[j])
                changed = True
        # 2. empty and singleton rows
        for i in range(m):
            if not row_on[i]:
                continue
            act = [(ci[e], val[e]) for e in range(rp[i], rp[i + 1]) if col_on[ci[e]]]
            if len(act) == 0:
                t = 1e-9 * (1.0 + abs(p.b[i]))
                bad = (rt[i] == EQ and abs(b[i]) > t) or (rt[i] == GE and b[i] > t) or (rt[i] == LE and b[i] < -t)
                if bad:
                    status = "primal_infeasible"
                    return None, rec()
                row_on[i] = False
                changed = True
            elif len(act) == 1:
                j, a = act[0]
                v = b[i] / a
                lower = rt[i] == EQ or (rt[i] == GE) == (a > 0)
                upper = rt[i] == EQ or not lower
                if lower and v > lo[j]:
                    lo[j] = v
                    lo_row[j] = i
                if upper and v < hi[j]:
                    hi[j] = v
                    hi_row[j] = i
                if lo[j] > hi[j]:
                    if lo[j] - hi[j] > _tol(v):
                        status = "primal_infeasible"
                        return None, rec()
                    # within the tolerance: the column is fixed at the bound this row set
                    if lo_row[j] == i:
                        hi[j] = lo[j]
                    else:
                        lo[j] = hi[j]
                row_on[i] = False
                changed = True
        # 3. empty columns
        for j in range(n):
            if not col_on[j] or any(row_on[i] for i, _ in col_rows[j]):
                continue
            cj = p.c[j]
            if cj > 0:
                v = lo[j]
            elif cj < 0:
                v = hi[j]
            else:
                v = min(max(0.0, lo[j]), hi[j])
            if not np.isfinite(v):
                status = "dual_infeasible"
                return None, rec()
            fix(j, v)
            changed = True
    # the reduced LP: active rows and columns in their original order
    rows = np.flatnonzero(row_on)
    cols = np.flatnonzero(col_on)
    newc = np.full(n, -1, np.int64)
    newc[cols] = np.arange(len(cols))
    r_ptr = [0]
    r_ci, r_v = [], []
    for i in rows:
        for e in range(rp[i], rp[i + 1]):
            if col_on[ci[e]]:
                r_ci.append(newc[ci[e]])
                r_v.append(val[e])
        r_ptr.append(len(r_ci))
    q = lpgen.Problem(len(rows), len(cols), np.asarray(r_ptr, np.int32), np.asarray(r_ci, np.int32),
                      np.asarray(r_v, float), np.asarray(p.c, float)[cols], b[rows], lo[cols], hi[cols],
                      rt[rows].astype(np.int8), p.name + "+presolved")
    return q, rec()


def postsolve(p, r: Record, xr, yr, lamr):
    """Full-size (x, y, lambda) of the original LP from the reduced LP's
    solution (user orientation)."""
    m, n = int(p.m), int(p.n)
    rows = np.flatnonzero(r.row_keep)
    cols = np.flatnonzero(r.col_keep)
    x = r.xfix.copy()
    x[cols] = xr
    y = np.zeros(m)
    y[rows] = yr
    lam = np.zeros(n)
    A = p.to_scipy().tocsc()

    def assign(j, mu):
        """Give mu, the multiplier of x_j's lower bound (mu > 0) or upper
        bound (mu < 0), to the row that set that bound, or to lambda_j."""
        if mu == 0.0:
            return
        side = r.lo_row[j] if mu > 0 else r.hi_row[j]
        if side >= 0:
            y[side] = mu / A[side, j]
        else:
            lam[j] = mu

    for k, j in enumerate(cols):
        assign(j, float(lamr[k]))
    for j in reversed(r.col_order):
        g = p.c[j]
        for k in range(A.indptr[j], A.indptr[j + 1]):
            i = A.indices[k]
            if i != r.lo_row[j] and i != r.hi_row[j]:
                g -= A.data[k] * y[i]
        assign(j, g)
    return x, y, lam
