"""Seeded synthetic LP generators shared by the tests, the benchmark and smoke().

This module holds no arithmetic of the solver: it only draws random instances
of the LP form of the paper (Section 2, eq. (lp): min c'x s.t. Gx >= h, Ax = b,
l <= x <= u) in the user orientation of the C ABI (rows typed EQ / GE / LE), and
for the families that have one it builds a known optimal primal-dual pair
(x*, y*, lambda*) with c = A'y* + lambda*.

Dual sign convention (user orientation, stationarity c = A'y + lambda):
  y free on EQ rows, y >= 0 on GE rows, y <= 0 on LE rows;
  lambda >= 0 where x sits at a finite lower bound, <= 0 at a finite upper bound.

Families (all values float64, indices int32, row types int8):
  random_lp      -- rows of Poisson-like length, 8 random rows per column,
                    N(0,1) values, a constructed optimum (m=1000/n=2000 random LP).
  skewed_lp      -- power-law row lengths capped at 10,000 (the 1e6 x 2e6,
                    nnz 2e7 large skewed LP), constructed optimum.
  transportation -- S sources x T sinks, 2 unit entries per column.
  tiny_dense_lp  -- dense boxed LPs small enough for vertex enumeration.
  batch_lps      -- many random_lp instances of uneven size.
  infeasible_lp / bound_infeasible_lp / unbounded_lp -- a random_lp with a
                    planted contradiction (two rows asking a'x >= beta + gap
                    and a'x <= beta; one row no point of the box reaches) or a
                    planted improving ray (a new unbounded column that only
                    relaxes LE rows), with the planted certificate attached.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

ROW_EQ, ROW_GE, ROW_LE = 0, 1, 2


@dataclasses.dataclass
class Problem:
    m: int
    n: int
    row_ptr: np.ndarray   # int32 [m+1]
    col_idx: np.ndarray   # int32 [nnz]
    val: np.ndarray       # float64 [nnz]
    c: np.ndarray         # float64 [n]
    b: np.ndarray         # float64 [m]
    l: np.ndarray         # float64 [n], may hold -inf
    u: np.ndarray         # float64 [n], may hold +inf
    row_type: np.ndarray  # int8 [m]
    name: str = ""
    x_star: Optional[np.ndarray] = None    # known optimal primal point (user orientation)
    y_star: Optional[np.ndarray] = None    # known optimal dual point (user orientation)
    lam_star: Optional[np.ndarray] = None  # known reduced costs

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def obj_star(self) -> Optional[float]:
        if self.x_star is None:
            return None
        return float(np.dot(self.c, self.x_star))

    def to_scipy(self):
        import scipy.sparse as sp
        return sp.csr_matrix((self.val, self.col_idx, self.row_ptr), shape=(self.m, self.n))


def _csr_from_coo(m: int, n: int, rows: np.ndarray, cols: np.ndarray, vals: np.ndarray):
    """Row-major CSR with column indices sorted inside each row."""
    order = np.lexsort((cols, rows))
    rows, cols, vals = rows[order], cols[order], vals[order]
    counts = np.bincount(rows, minlength=m)
    row_ptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    assert row_ptr[-1] < 2**31
    return (row_ptr.astype(np.int32), cols.astype(np.int32), vals.astype(np.float64))


def _matvec(row_ptr, col_idx, val, x, m):
    rows = np.repeat(np.arange(m), np.diff(row_ptr))
    if not len(val):
        return np.zeros(m)
    return np.bincount(rows, weights=val * x[col_idx], minlength=m)


def _rmatvec(row_ptr, col_idx, val, y, m, n):
    rows = np.repeat(np.arange(m), np.diff(row_ptr))
    if not len(val):
        return np.zeros(n)
    return np.bincount(col_idx, weights=val * y[rows], minlength=n)


def _certify(rng, m, n, row_ptr, col_idx, val, row_type, lo, hi, frac_lo=0.15, frac_hi=0.15,
             slack_frac_le=0.5, name=""):
    """Build b, c and a known optimum (x*, y*, lambda*) for a given sparsity pattern.

    x*: frac_lo of the variables at l, frac_hi at u, the rest U(l, u).
    EQ rows: b = (Ax*)_i, y*_i ~ N(0,1).
    LE rows: a fraction slack_frac_le is slack (b = (Ax*)_i + U(0,1), y* = 0);
             the others are tight with y*_i = -U(0,1) (the multiplier of the
             negated >= row is U(0,1) >= 0).
    GE rows: likewise with the opposite signs.
    lambda*: U(0,1) at the lower bound, -U(0,1) at the upper bound, 0 inside.
    c = A'y* + lambda*.
    """
    status = rng.random(n)
    at_lo = status < frac_lo
    at_hi = (status >= frac_lo) & (status < frac_lo + frac_hi)
    x = lo + (hi - lo) * rng.random(n)
    x[at_lo] = lo[at_lo] if np.ndim(lo) else lo
    x[at_hi] = hi[at_hi] if np.ndim(hi) else hi
    ax = _matvec(row_ptr, col_idx, val, x, m)
    y = np.zeros(m)
    b = ax.copy()
    eq = row_type == ROW_EQ
    y[eq] = rng.standard_normal(int(eq.sum()))
    for t, sgn in ((ROW_LE, -1.0), (ROW_GE, 1.0)):
        idx = np.flatnonzero(row_type == t)
        if len(idx) == 0:
            continue
        perm = rng.permutation(len(idx))
        n_slack = int(round(slack_frac_le * len(idx)))
        slack_rows = idx[perm[:n_slack]]
        tight_rows = idx[perm[n_slack:]]
        s = rng.random(len(slack_rows))
        b[slack_rows] = ax[slack_rows] - sgn * s   # LE: b = Ax + s ; GE: b = Ax - s
        y[tight_rows] = sgn * rng.random(len(tight_rows))
    lam = np.zeros(n)
    lam[at_lo] = rng.random(int(at_lo.sum()))
    lam[at_hi] = -rng.random(int(at_hi.sum()))
    c = _rmatvec(row_ptr, col_idx, val, y, m, n) + lam
    return b, c, x, y, lam


def random_lp(seed: int = 0, m_eq: int = 500, m_le: int = 500, n: int = 2000,
              nnz_per_col: int = 8, ub: float = 10.0, name: str = "") -> Problem:
    """Random LP with a known optimum: each column has nnz_per_col distinct
    uniformly random rows with N(0,1) values; row types EQ and LE randomly
    interleaved; 0 <= x <= ub."""
    rng = np.random.Generator(np.random.PCG64(seed))
    m = m_eq + m_le
    row_type = np.array([ROW_EQ] * m_eq + [ROW_LE] * m_le, dtype=np.int8)
    rng.shuffle(row_type)
    k = min(nnz_per_col, m)
    if m > 0 and k > 0:
        # distinct rows per column: argsort of random keys, first k of each column
        rows = np.empty((n, k), dtype=np.int64)
        for j0 in range(0, n, 4096):
            j1 = min(n, j0 + 4096)
            keys = rng.random((j1 - j0, m))
            rows[j0:j1] = np.argpartition(keys, k - 1, axis=1)[:, :k]
        cols = np.repeat(np.arange(n), k)
        rows = rows.reshape(-1)
        vals = rng.standard_normal(n * k)
    else:
        rows = np.zeros(0, np.int64); cols = np.zeros(0, np.int64); vals = np.zeros(0)
    row_ptr, col_idx, val = _csr_from_coo(m, n, rows, cols, vals)
    l = np.zeros(n)
    u = np.full(n, ub)
    b, c, xs, ys, lam = _certify(rng, m, n, row_ptr, col_idx, val, row_type, l, u)
    return Problem(m, n, row_ptr, col_idx, val, c, b, l, u, row_type,
                   name or f"random_lp(seed={seed},m={m},n={n})", xs, ys, lam)


def config0(seed: int = 0) -> Problem:
    """m=1,000 (500 EQ, 500 LE), n=2,000 in [0,10], 8 nnz per column."""
    return random_lp(seed, 500, 500, 2000, 8, 10.0,
                     name=f"random_lp_m1000_n2000_seed{seed}")


def skewed_row_lengths(rng, m: int, nnz_target: int, cap: int) -> np.ndarray:
    """Row lengths L_i = min(cap, ceil(x_m * U_i^-2)), U_i ~ U(0,1): a power-law
    tail P(L >= k) ~ k^-1/2 (the tail of a Zipf(1.5) pmf), with x_m chosen by
    bisection so that sum(L) is as close to nnz_target as possible."""
    U = rng.random(m)
    U = np.maximum(U, 1e-300)
    inv2 = U ** -2.0

    def total(xm):
        return int(np.minimum(cap, np.ceil(xm * inv2)).sum())

    lo, hi = 1e-12, float(cap)
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if total(mid) < nnz_target:
            lo = mid
        else:
            hi = mid
    L = np.minimum(cap, np.ceil(hi * inv2)).astype(np.int64)
    return np.maximum(L, 1)


def _distinct_cols_per_row(rng, row_len: np.ndarray, n: int):
    """Uniform column indices, distinct inside each row (resampling duplicates)."""
    m = len(row_len)
    rows = np.repeat(np.arange(m, dtype=np.int64), row_len)
    cols = rng.integers(0, n, size=len(rows), dtype=np.int64)
    for _ in range(100):
        key = rows * n + cols
        order = np.argsort(key, kind="stable")
        ks = key[order]
        dup = np.zeros(len(ks), dtype=bool)
        dup[1:] = ks[1:] == ks[:-1]
        if not dup.any():
            rows, cols = rows[order], cols[order]
            return rows, cols
        bad = order[dup]
        cols[bad] = rng.integers(0, n, size=len(bad), dtype=np.int64)
    raise RuntimeError("could not draw distinct columns")


def skewed_lp(seed: int = 0, m: int = 1_000_000, n: int = 2_000_000,
              nnz_target: int = 20_000_000, cap: int = 10_000, ub: float = 10.0,
              name: str = "") -> Problem:
    """Large skewed LP: half EQ and half LE rows (interleaved), power-law row
    lengths capped at `cap`, distinct uniform columns per row, N(0,1) values,
    0 <= x <= ub, constructed optimum."""
    rng = np.random.Generator(np.random.PCG64(seed))
    row_type = np.array([ROW_EQ] * (m // 2) + [ROW_LE] * (m - m // 2), dtype=np.int8)
    rng.shuffle(row_type)
    L = skewed_row_lengths(rng, m, nnz_target, min(cap, n))
    rows, cols = _distinct_cols_per_row(rng, L, n)
    vals = rng.standard_normal(len(rows))
    row_ptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(L, out=row_ptr[1:])
    assert row_ptr[-1] < 2**31
    row_ptr = row_ptr.astype(np.int32)
    col_idx = cols.astype(np.int32)
    l = np.zeros(n)
    u = np.full(n, ub)
    b, c, xs, ys, lam = _certify(rng, m, n, row_ptr, col_idx, vals, row_type, l, u)
    return Problem(m, n, row_ptr, col_idx, vals, c, b, l, u, row_type,
                   name or f"skewed_lp(seed={seed},m={m},n={n},nnz={int(row_ptr[-1])})",
                   xs, ys, lam)


def config1(seed: int = 0) -> Problem:
    """m=1e6, n=2e6, nnz ~2e7, row lengths power-law capped at 10,000."""
    return skewed_lp(seed, name=f"skewed_lp_m1e6_n2e6_nnz2e7_seed{seed}")


def transportation(seed: int = 0, S: int = 2000, T: int = 2000, name: str = "") -> Problem:
    """Transportation LP, S sources x T sinks.  Variable x_{ij} has index
    i*T + j; rows 0..S-1 are supplies (sum_j x_ij = s_i), rows S..S+T-1 are
    demands (sum_i x_ij = d_j); every entry is 1.0; x >= 0, no upper bound.
    s ~ U(1,100), d' ~ U(1,100) rescaled so that sum d = sum s; c ~ U(0,1)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    s = rng.uniform(1.0, 100.0, S)
    d = rng.uniform(1.0, 100.0, T)
    d *= s.sum() / d.sum()
    cost = rng.random(S * T)
    m, n = S + T, S * T
    # supply rows: contiguous columns; demand rows: stride T
    sup_ptr = np.arange(S + 1, dtype=np.int64) * T
    dem_ptr = S * T + np.arange(1, T + 1, dtype=np.int64) * S
    row_ptr = np.concatenate([sup_ptr, dem_ptr]).astype(np.int64)
    assert row_ptr[-1] < 2**31
    col_sup = np.arange(S * T, dtype=np.int64)
    col_dem = (np.arange(S, dtype=np.int64)[None, :] * T + np.arange(T, dtype=np.int64)[:, None]).reshape(-1)
    col_idx = np.concatenate([col_sup, col_dem]).astype(np.int32)
    val = np.ones(2 * S * T)
    b = np.concatenate([s, d])
    row_type = np.zeros(m, dtype=np.int8)
    return Problem(m, n, row_ptr.astype(np.int32), col_idx, val, cost, b,
                   np.zeros(n), np.full(n, np.inf), row_type,
                   name or f"transportation_{S}x{T}_seed{seed}")


def config2(seed: int = 0) -> Problem:
    return transportation(seed, 2000, 2000, name=f"transportation_2000x2000_seed{seed}")


def tiny_dense_lp(seed: int, n: int = 4, m: int = 3, box: float = 5.0) -> Problem:
    """Dense LP with every bound finite (so it is bounded) and mixed row types;
    feasible by construction (b built from a random point of the box)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    A = rng.standard_normal((m, n))
    A[np.abs(A) < 0.05] = 0.3
    x0 = rng.uniform(-box * 0.5, box * 0.5, n)
    l = -box * rng.uniform(0.5, 1.0, n)
    u = box * rng.uniform(0.5, 1.0, n)
    row_type = rng.integers(0, 3, m).astype(np.int8)
    ax = A @ x0
    s = rng.uniform(0.0, 1.0, m)
    b = np.where(row_type == ROW_EQ, ax, np.where(row_type == ROW_GE, ax - s, ax + s))
    c = rng.standard_normal(n)
    rows, cols = np.nonzero(A)
    row_ptr, col_idx, val = _csr_from_coo(m, n, rows, cols, A[rows, cols])
    return Problem(m, n, row_ptr, col_idx, val, c, b, l, u, row_type, f"tiny_dense(seed={seed})")


def from_dense(A, c, b, l, u, row_type, name="dense") -> Problem:
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    rows, cols = np.nonzero(A)
    row_ptr, col_idx, val = _csr_from_coo(m, n, rows, cols, A[rows, cols])
    return Problem(m, n, row_ptr, col_idx, val, np.asarray(c, float), np.asarray(b, float),
                   np.asarray(l, float), np.asarray(u, float), np.asarray(row_type, np.int8), name)


def batch_sizes(seed: int = 0, count: int = 4096, m_lo: int = 50, m_hi: int = 2000) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64([seed, 0xB47C]))
    return rng.integers(m_lo, m_hi + 1, count)


def batch_lp(seed: int, idx: int, m: int) -> Problem:
    """LP number idx of a batch: built as random_lp with m rows (half EQ, half
    LE), n = 2m, 8 nnz per column, seeded by (seed, idx)."""
    s = np.random.SeedSequence([seed, idx]).generate_state(1)[0]
    return random_lp(int(s), m // 2, m - m // 2, 2 * m, 8, 10.0,
                     name=f"batch_lp(seed={seed},idx={idx},m={m})")


def permute(p: Problem, row_perm: np.ndarray, col_perm: np.ndarray) -> Problem:
    """The same LP with rows and columns renumbered: new row r is old row
    row_perm[r], new column j is old column col_perm[j]."""
    A = p.to_scipy().tocoo()
    inv_r = np.empty(p.m, np.int64); inv_r[row_perm] = np.arange(p.m)
    inv_c = np.empty(p.n, np.int64); inv_c[col_perm] = np.arange(p.n)
    row_ptr, col_idx, val = _csr_from_coo(p.m, p.n, inv_r[A.row], inv_c[A.col], A.data)
    q = Problem(p.m, p.n, row_ptr, col_idx, val, p.c[col_perm], p.b[row_perm],
                p.l[col_perm], p.u[col_perm], p.row_type[row_perm], p.name + "+perm")
    if p.x_star is not None:
        q.x_star = p.x_star[col_perm]
    if p.y_star is not None:
        q.y_star = p.y_star[row_perm]
    if p.lam_star is not None:
        q.lam_star = p.lam_star[col_perm]
    return q


def mixed_lp(seed: int = 0, m: int = 40, n: int = 60, density: float = 0.15,
             name: str = "") -> Problem:
    """Random sparse LP with every row type (EQ, GE, LE) and every bound type
    (both finite, lower only, upper only, free) and a constructed optimum.
    Each column has at least one entry so that free variables are bounded."""
    rng = np.random.Generator(np.random.PCG64([seed, 0x51A7]))
    mask = rng.random((m, n)) < density
    for j in range(n):
        if not mask[:, j].any():
            mask[rng.integers(0, m), j] = True
    rows, cols = np.nonzero(mask)
    vals = rng.standard_normal(len(rows))
    row_ptr, col_idx, val = _csr_from_coo(m, n, rows, cols, vals)
    row_type = rng.integers(0, 3, m).astype(np.int8)
    btype = rng.integers(0, 4, n)
    l = np.where((btype == 0) | (btype == 1), -rng.uniform(0, 5, n), -np.inf)
    u = np.where(btype == 0, l + rng.uniform(1, 10, n), np.where(btype == 2, rng.uniform(0, 5, n), np.inf))
    x = np.empty(n)
    lam = np.zeros(n)
    for j in range(n):
        if btype[j] == 0:
            s = rng.integers(0, 3)
            if s == 0:
                x[j] = l[j]; lam[j] = rng.random()
            elif s == 1:
                x[j] = u[j]; lam[j] = -rng.random()
            else:
                x[j] = rng.uniform(l[j], u[j])
        elif btype[j] == 1:
            if rng.random() < 0.5:
                x[j] = l[j]; lam[j] = rng.random()
            else:
                x[j] = l[j] + 3 * rng.exponential()
        elif btype[j] == 2:
            if rng.random() < 0.5:
                x[j] = u[j]; lam[j] = -rng.random()
            else:
                x[j] = u[j] - 3 * rng.exponential()
        else:
            x[j] = 3 * rng.standard_normal()
    ax = _matvec(row_ptr, col_idx, val, x, m)
    y = np.zeros(m)
    b = ax.copy()
    for i in range(m):
        tight = rng.random() < 0.6
        if row_type[i] == ROW_EQ:
            y[i] = rng.standard_normal()
        elif row_type[i] == ROW_GE:
            if tight:
                y[i] = rng.random()
            else:
                b[i] = ax[i] - rng.random()
        else:
            if tight:
                y[i] = -rng.random()
            else:
                b[i] = ax[i] + rng.random()
    c = _rmatvec(row_ptr, col_idx, val, y, m, n) + lam
    return Problem(m, n, row_ptr, col_idx, val, c, b, l, u, row_type,
                   name or f"mixed_lp(seed={seed},m={m},n={n})", x, y, lam)


def transport_family_lp(seed: int, idx: int, S: int = 100, T: int = 100) -> Problem:
    """LP number idx of a family of S x T transportation LPs (layout as in
    `transportation`).  The family (seed) fixes base costs C ~ U(0,1)^{SxT}
    and base demands d ~ U(1,10)^T; LP idx draws (seed, idx): c = C + N(0,
    0.05^2), supplies s ~ U(1,10)^S, demands d * U(0.8, 1.2) rescaled so
    that sum d = sum s."""
    base = np.random.Generator(np.random.PCG64([seed, 0xFA11]))
    C = base.random(S * T)
    d0 = base.uniform(1.0, 10.0, T)
    rng = np.random.Generator(np.random.PCG64([seed, 0xFA11, idx]))
    c = C + 0.05 * rng.standard_normal(S * T)
    s = rng.uniform(1.0, 10.0, S)
    d = d0 * rng.uniform(0.8, 1.2, T)
    d *= s.sum() / d.sum()
    p = transportation(0, S, T)
    return Problem(p.m, p.n, p.row_ptr, p.col_idx, p.val, c, np.concatenate([s, d]), p.l, p.u, p.row_type,
                   f"transport_family(seed={seed},idx={idx},{S}x{T})")


def gnn_init(seed: int, shapes) -> np.ndarray:
    """Initial weights of a network with the given parameter shapes (a list of
    (name, shape)), flat and representable in FP32: matrices U(-a, a) with
    a = sqrt(6 / (fan_in + fan_out)), vectors that multiply hidden states
    (2 or more entries) U(-a, a) with a = sqrt(3 / len), biases and scalars 0."""
    rng = np.random.Generator(np.random.PCG64([seed, 0x6E11]))
    out = []
    for name, shape in shapes:
        shape = tuple(shape)
        if len(shape) == 2:
            a = np.sqrt(6.0 / (shape[0] + shape[1]))
            w = rng.uniform(-a, a, shape)
        elif name.startswith("w_"):
            a = np.sqrt(3.0 / shape[0])
            w = rng.uniform(-a, a, shape)
        else:
            w = np.zeros(shape)
        out.append(w.astype(np.float32).astype(np.float64).reshape(-1))
    return np.concatenate(out)


def _append_rows(p: Problem, rows_cols, rows_vals, b_new, rt_new, name: str) -> Problem:
    """p with extra rows (lists of column indices / values) appended at the end."""
    A = p.to_scipy().tocoo()
    r = [A.row]; cc = [A.col]; v = [A.data]
    for k, (cols, vals) in enumerate(zip(rows_cols, rows_vals)):
        r.append(np.full(len(cols), p.m + k)); cc.append(np.asarray(cols)); v.append(np.asarray(vals, float))
    m = p.m + len(rows_cols)
    row_ptr, col_idx, val = _csr_from_coo(m, p.n, np.concatenate(r), np.concatenate(cc), np.concatenate(v))
    return Problem(m, p.n, row_ptr, col_idx, val, p.c.copy(), np.concatenate([p.b, b_new]), p.l.copy(),
                   p.u.copy(), np.concatenate([p.row_type, np.asarray(rt_new, np.int8)]), name)


def infeasible_lp(seed: int = 0, m: int = 200, gap: float = 1.0) -> Problem:
    """random_lp (m rows, n = 2m) plus the rows a'x >= beta + gap and
    a'x <= beta for a random sparse a: no x satisfies both.  The planted dual
    ray (user orientation) is y = 1 on the GE row, -1 on the LE row, 0 elsewhere."""
    base = batch_lp(seed, 0, m)
    rng = np.random.Generator(np.random.PCG64([seed, 0x1F5]))
    cols = np.sort(rng.choice(base.n, 8, replace=False))
    vals = rng.standard_normal(8)
    beta = float(rng.uniform(-5, 5))
    p = _append_rows(base, [cols, cols], [vals, vals], [beta + gap, beta], [ROW_GE, ROW_LE],
                     f"infeasible_lp(seed={seed},m={m})")
    yr = np.zeros(p.m); yr[-2] = 1.0; yr[-1] = -1.0
    p.y_star = yr      # the planted ray, not an optimum
    return p


def bound_infeasible_lp(seed: int = 0, m: int = 200) -> Problem:
    """random_lp (x in [0, 10]) plus a GE row with positive coefficients whose
    right-hand side exceeds the row's maximum over the box by 1."""
    base = batch_lp(seed, 0, m)
    rng = np.random.Generator(np.random.PCG64([seed, 0xB0D]))
    cols = np.sort(rng.choice(base.n, 8, replace=False))
    vals = rng.uniform(0.5, 2.0, 8)
    rhs = float(np.sum(vals * base.u[cols])) + 1.0
    p = _append_rows(base, [cols], [vals], [rhs], [ROW_GE], f"bound_infeasible_lp(seed={seed},m={m})")
    yr = np.zeros(p.m); yr[-1] = 1.0
    p.y_star = yr
    return p


def unbounded_lp(seed: int = 0, m: int = 200) -> Problem:
    """random_lp (feasible) plus a column x_new >= 0 without upper bound, cost
    -1, entering three LE rows with coefficient -1 (raising it only relaxes
    them) and no other row: c'x -> -inf along e_new."""
    base = batch_lp(seed, 0, m)
    rng = np.random.Generator(np.random.PCG64([seed, 0xDB1]))
    le_rows = np.flatnonzero(base.row_type == ROW_LE)
    rows = np.sort(rng.choice(le_rows, 3, replace=False))
    A = base.to_scipy().tocoo()
    n = base.n + 1
    row_ptr, col_idx, val = _csr_from_coo(base.m, n, np.concatenate([A.row, rows]),
                                          np.concatenate([A.col, np.full(3, base.n)]),
                                          np.concatenate([A.data, -np.ones(3)]))
    p = Problem(base.m, n, row_ptr, col_idx, val, np.concatenate([base.c, [-1.0]]), base.b.copy(),
                np.concatenate([base.l, [0.0]]), np.concatenate([base.u, [np.inf]]), base.row_type.copy(),
                f"unbounded_lp(seed={seed},m={m})")
    xr = np.zeros(n); xr[-1] = 1.0
    p.x_star = xr      # the planted ray, not an optimum
    return p
