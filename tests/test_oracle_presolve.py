"""Pins of the presolve-lite reference (oracle/presolve.py) and the library's
host presolve against it (no device needed).

What pins it:
  * closed forms of each reduction on tiny LPs (the bound a singleton row
    sets for every row type and coefficient sign, cascades, empty rows and
    columns, crossing bounds);
  * the postsolve is exact: when the reduced LP is solved in closed form (only
    bounds left) the postsolved point satisfies the original KKT conditions
    to rounding, and in general the postsolved point of an eps-solution passes
    the FP64 evaluator on the original LP and matches its known optimum;
  * the library's reductions (pdlp_presolve) equal the reference's bit for
    bit: the same rows and columns removed, the same bounds, fixed values and
    right-hand sides.
"""
import numpy as np
import pytest

import lpgen
import oracle
from oracle import presolve as PS

INF = np.inf


def _lp(A, b, rt, c, l, u, name="t"):
    return lpgen.from_dense(A, c, b, l, u, rt, name)


def test_singleton_rows_set_the_right_bound():
    # 2 x1 = 6 (fixes x1 = 3); -x2 >= -4 (x2 <= 4); -x3 <= 2 (x3 >= -2); 3 x4 <= 6 (x4 <= 2)
    p = _lp(np.diag([2.0, -1.0, -1.0, 3.0]), [6, -4, 2, 6], [0, 1, 2, 2], [1, -1, 1, -1],
            [-INF] * 4, [INF] * 4)
    q, r = PS.presolve(p)
    assert r.status == "ok" and q.m == 0
    np.testing.assert_array_equal(r.lo[1:], [-INF, -2.0, -INF])
    np.testing.assert_array_equal(r.hi[1:], [4.0, INF, 2.0])
    assert r.xfix[0] == 3.0 and not r.col_keep[0]
    # x2 (c < 0, upper 4), x3 (c > 0, lower -2), x4 (c < 0, upper 2) become empty columns
    np.testing.assert_array_equal(r.xfix, [3.0, 4.0, -2.0, 2.0])
    assert r.offset == 3.0 - 4.0 - 2.0 - 2.0
    assert r.lo_row.tolist() == [0, -1, 2, -1] and r.hi_row.tolist() == [0, 1, -1, 3]


def test_cascade_and_empty_row():
    # x1 = 2 (singleton) makes x1 + x2 = 5 a singleton: x2 = 3; then x1 + x2 + x3 >= 4
    # keeps x3 only: x3 >= -1, and the empty-after-fixing row 2 x1 - x2 >= 0 must hold (4 - 3 >= 0)
    p = _lp([[1, 0, 0], [1, 1, 0], [1, 1, 1], [2, -1, 0]], [2, 5, 4, 0], [0, 0, 1, 1], [1, 1, 1],
            [-INF] * 3, [INF] * 3)
    q, r = PS.presolve(p)
    assert r.status == "ok"
    assert r.xfix[0] == 2.0 and r.xfix[1] == 3.0
    assert r.lo[2] == -1.0 and r.lo_row[2] == 2
    # row 3 (2 x1 - x2 >= 0) with both columns fixed: 4 - 3 = 1 >= 0, dropped
    assert not r.row_keep.any()
    # x3 is then an empty column with c > 0: at its lower bound -1
    assert r.xfix[2] == -1.0 and r.offset == 2.0 + 3.0 - 1.0
    # the same LP with row 3 asking 2 x1 - x2 >= 2 (4 - 3 = 1 < 2): infeasible
    p2 = _lp([[1, 0, 0], [1, 1, 0], [1, 1, 1], [2, -1, 0]], [2, 5, 4, 2], [0, 0, 1, 1], [1, 1, 1],
             [-INF] * 3, [INF] * 3)
    assert PS.presolve(p2)[1].status == "primal_infeasible"


def test_crossing_bounds_and_empty_columns():
    # x >= 3 and x <= 2: infeasible; x >= 3 and x <= 3 + 1e-12: fixed at 3
    assert PS.presolve(_lp([[1.0], [1.0]], [3, 2], [1, 2], [1], [-INF], [INF]))[1].status == "primal_infeasible"
    q, r = PS.presolve(_lp([[1.0], [1.0]], [3, 3 + 1e-12], [1, 2], [1], [-INF], [INF]))
    assert r.status == "ok" and r.xfix[0] == 3.0
    # empty columns: c > 0 -> lower, c < 0 with no upper bound -> dual infeasible, c = 0 -> proj(0)
    q, r = PS.presolve(_lp([[0.0, 0.0, 1.0]], [1], [1], [2, 0, 1], [1, -3, 0], [5, -1, INF]))
    assert r.xfix[0] == 1.0 and r.xfix[1] == -1.0
    assert PS.presolve(_lp([[0.0, 1.0]], [1], [1], [-1, 1], [0, 0], [INF, INF]))[1].status == "dual_infeasible"


def _solve_postsolve(p, eps):
    q, r = PS.presolve(p)
    s = oracle.solve(q, eps_rel=eps, max_iter=1_000_000)
    x, y, lam = PS.postsolve(p, r, s.x, s.y, s.rc)
    return q, r, s, x, y, lam


def test_postsolve_exact_when_the_reduced_lp_is_only_bounds():
    """Every row is a singleton: the reduced LP has no rows; its solution is
    the closed-form box optimum, and the postsolved (x, y, lambda) is an exact
    KKT point of the original LP."""
    rng = np.random.default_rng(5)
    n = 12
    A = np.diag(rng.choice([-2.0, -1.0, 1.0, 3.0], n))
    rt = rng.integers(0, 3, n)
    b = rng.uniform(-3, 3, n)
    c = rng.standard_normal(n)
    p = _lp(A, b, rt, c, np.full(n, -10.0), np.full(n, 10.0))
    q, r = PS.presolve(p)
    assert q.m == 0
    # the reduced LP has no rows; its columns were emptied and fixed by presolve itself
    x, y, lam = PS.postsolve(p, r, np.zeros(q.n), np.zeros(0), np.zeros(q.n))
    e = oracle.evaluate(p, x, y)
    assert e["rel_kkt"] <= 1e-15, e
    np.testing.assert_allclose(lam, oracle.reduced_costs(p, y), atol=1e-15)


@pytest.mark.parametrize("make", [
    lambda: lpgen.skewed_lp(0, m=4000, n=8000, nnz_target=80000, cap=800),
    lambda: lpgen.skewed_lp(3, m=3000, n=6000, nnz_target=30000, cap=300),
])
def test_postsolve_of_an_eps_solution(make):
    p = make()
    q, r, s, x, y, lam = _solve_postsolve(p, 1e-8)
    assert s.status == "OPTIMAL"
    assert q.m < p.m and q.n < p.n
    e = oracle.evaluate(p, x, y)
    assert e["rel_kkt"] <= 2e-8, e
    np.testing.assert_allclose(lam, oracle.reduced_costs(p, y), atol=1e-12)
    ref = p.obj_star()
    assert abs(e["primal_obj"] - ref) <= 1e-6 * (1 + abs(ref))
    assert e["primal_obj"] == pytest.approx(s.info["primal_obj"] + r.offset, rel=1e-12)


@pytest.mark.parametrize("make", [
    lambda: lpgen.skewed_lp(0, m=4000, n=8000, nnz_target=80000, cap=800),
    lambda: lpgen.skewed_lp(7, m=2000, n=4000, nnz_target=12000, cap=200),
    lambda: lpgen.mixed_lp(2),
    lambda: lpgen.transportation(1, 12, 15),
    lambda: lpgen.bound_infeasible_lp(0, 100),
    lambda: _lp([[1, 0, 0], [1, 1, 0], [1, 1, 1], [2, -1, 0]], [2, 5, 4, 0], [0, 0, 1, 1], [1, 1, 1],
                [-INF] * 3, [INF] * 3),
    lambda: _lp([[1.0], [1.0]], [3, 2], [1, 2], [1], [-INF], [INF]),
])
def test_library_presolve_equals_reference(make):
    from paper_2311_12180_amd import pdlp as P
    p = make()
    q, r = PS.presolve(p)
    L = P.pdlp_presolve(p)
    status = {"ok": "OK", "primal_infeasible": "PRIMAL_INFEASIBLE", "dual_infeasible": "DUAL_INFEASIBLE"}
    assert L["status"] == status[r.status]
    np.testing.assert_array_equal(L["keep_row"], r.row_keep)
    np.testing.assert_array_equal(L["keep_col"], r.col_keep)
    if r.status == "ok":
        np.testing.assert_array_equal(L["lo"], r.lo)
        np.testing.assert_array_equal(L["hi"], r.hi)
        np.testing.assert_array_equal(L["x_fixed"], r.xfix)
        np.testing.assert_array_equal(L["b_reduced"][r.row_keep], q.b)
        assert L["offset"] == r.offset
