"""Exact, independent references for small LPs (test-only).

None of this code shares arithmetic with the oracle or the HIP solver:
  vertex_enumeration -- brute force over every basis of a boxed LP;
  box_lp_optimum     -- closed form of min c'x over a box;
  knapsack_optimum   -- greedy-by-ratio optimum of a fractional knapsack;
  highs_optimum      -- scipy's HiGHS (library cross-check only).
"""
from __future__ import annotations

import itertools

import numpy as np


def vertex_enumeration(A, b, row_type, c, l, u, tol=1e-9):
    """Optimal objective of min c'x, rows (EQ 0, GE 1, LE 2), l <= x <= u, all
    bounds finite, by enumerating every vertex: n linearly independent active
    constraints that include every EQ row."""
    A = np.asarray(A, float)
    m, n = A.shape
    cons = []      # (coefficient row, rhs)
    eq_rows = [i for i in range(m) if row_type[i] == 0]
    other = [i for i in range(m) if row_type[i] != 0]
    for i in other:
        cons.append((A[i], b[i]))
    for j in range(n):
        e = np.zeros(n); e[j] = 1.0
        cons.append((e, l[j]))
        cons.append((e, u[j]))
    Aeq = A[eq_rows]
    beq = np.asarray(b, float)[eq_rows]
    need = n - len(eq_rows)
    best = np.inf
    best_x = None
    for S in itertools.combinations(range(len(cons)), need):
        M = np.vstack([Aeq] + [cons[s][0][None, :] for s in S]) if S else Aeq
        r = np.concatenate([beq, [cons[s][1] for s in S]])
        if np.linalg.matrix_rank(M) < n:
            continue
        x = np.linalg.solve(M, r)
        ax = A @ x
        ok = np.all(x >= l - tol) and np.all(x <= u + tol)
        for i in range(m):
            if row_type[i] == 0:
                ok &= abs(ax[i] - b[i]) <= tol * (1 + abs(b[i]))
            elif row_type[i] == 1:
                ok &= ax[i] >= b[i] - tol
            else:
                ok &= ax[i] <= b[i] + tol
        if ok:
            v = float(c @ x)
            if v < best:
                best, best_x = v, x
    return best, best_x


def box_lp_optimum(c, l, u):
    """min c'x over l <= x <= u: x_j = l_j if c_j > 0, u_j if c_j < 0."""
    c, l, u = map(np.asarray, (c, l, u))
    x = np.where(c > 0, l, np.where(c < 0, u, np.clip(0.0, l, u)))
    return float(c @ x), x


def knapsack_optimum(v, w, W):
    """max v'x s.t. w'x <= W, 0 <= x <= 1 (w > 0, v > 0): fill by decreasing v/w."""
    order = np.argsort(-(np.asarray(v) / np.asarray(w)), kind="stable")
    cap = W
    val = 0.0
    for j in order:
        take = min(1.0, cap / w[j])
        if take <= 0:
            break
        val += take * v[j]
        cap -= take * w[j]
    return val


def highs_optimum(p):
    """scipy.optimize.linprog(method='highs') on a user-orientation Problem."""
    from scipy.optimize import linprog
    import scipy.sparse as sp
    A = sp.csr_matrix((p.val, p.col_idx, p.row_ptr), shape=(p.m, p.n))
    rt = np.asarray(p.row_type)
    eq = rt == 0
    ge = rt == 1
    le = rt == 2
    A_ub = sp.vstack([A[le], -A[ge]]) if (le.any() or ge.any()) else None
    b_ub = np.concatenate([p.b[le], -p.b[ge]]) if A_ub is not None else None
    bounds = [(None if not np.isfinite(lo) else lo, None if not np.isfinite(hi) else hi)
              for lo, hi in zip(p.l, p.u)]
    res = linprog(p.c, A_ub=A_ub, b_ub=b_ub, A_eq=A[eq] if eq.any() else None,
                  b_eq=p.b[eq] if eq.any() else None, bounds=bounds, method="highs")
    assert res.status == 0, res.message
    return float(res.fun)
