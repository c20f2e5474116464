"""GPU solves with presolve = 1 against the oracle's presolve + solve +
postsolve (oracle/presolve.py, pinned in tests/test_oracle_presolve.py).

Bars: the device solves an LP of exactly the oracle's reduced size; the
postsolved point passes the FP64 evaluator on the user's LP at the
tolerance (2 eps: the reduced LP's norms differ from the user's) and matches
the known optimum at 1e-8; the objective is within the reading-17 bars of the
oracle's presolved solve; infeasibility certificates of the reduced LP come
back as valid certificates of the user's LP; warm starts take full-size
vectors; the reduced-space queries are refused.
"""
import numpy as np
import pytest

import lpgen
from oracle import presolve as PS
from tests.farkas import check_dual_ray, check_primal_ray

pytestmark = pytest.mark.gpu

INF = np.inf


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    from paper_2311_12180_amd import pdlp
    pdlp.lib()
    return pdlp


def _skewed(seed=0, m=4000):
    return lpgen.skewed_lp(seed, m=m, n=2 * m, nnz_target=20 * m, cap=m // 5)


def _with_singletons(p, seed):
    """p plus singleton rows: a few variables bounded, a few fixed by EQ rows."""
    rng = np.random.default_rng(seed)
    cols = rng.choice(p.n - 1, 12, replace=False)   # never the last column (the planted ray)
    rows_c = [[j] for j in cols]
    vals = [[float(v)] for v in rng.choice([-2.0, -1.0, 1.0, 2.0], 12)]
    types = [lpgen.ROW_EQ] * 4 + [lpgen.ROW_GE] * 4 + [lpgen.ROW_LE] * 4
    # right-hand sides inside the column's box so the rows are satisfiable
    rhs = []
    for (j,), (a,), t in zip(rows_c, vals, types):
        lo, hi = p.l[j], min(p.u[j], 10.0)
        v = lo + 0.3 * (hi - lo) if t == lpgen.ROW_EQ else (lo + 0.1 * (hi - lo) if (t == lpgen.ROW_GE) == (a > 0)
                                                           else lo + 0.9 * (hi - lo))
        rhs.append(a * v)
    q = lpgen._append_rows(p, rows_c, vals, rhs, types, p.name + "+singletons")
    q.x_star, q.y_star = p.x_star, p.y_star
    return q


@pytest.mark.parametrize("eps", [1e-4, 1e-8])
def test_presolved_solve_matches_oracle(P, orc, eps):
    p = _skewed(0)
    q, rec = PS.presolve(p)
    opts = dict(eps_rel=eps, max_iter=1_000_000)
    r = orc.solve(q, **opts)
    xo, yo, lo = PS.postsolve(p, rec, r.x, r.y, r.rc)
    res = P.solve(p, presolve=1, time_limit_s=120.0, **opts)
    I = res.info
    print(f"eps {eps}: rows {p.m} -> {I['m_solved']}, cols {p.n} -> {I['n_solved']}; GPU {I['iterations']} "
          f"steps, oracle {r.info['iterations']}")
    assert (I["m_solved"], I["n_solved"]) == (q.m, q.n)
    assert res.status == "OPTIMAL"
    e = orc.evaluate(p, res.x, res.y)
    assert e["rel_kkt"] <= 2 * eps, e
    assert e["primal_obj"] == pytest.approx(I["primal_obj"], rel=1e-10, abs=1e-10)
    np.testing.assert_allclose(res.rc, orc.reduced_costs(p, res.y), rtol=1e-9, atol=1e-9)
    oref = r.info["primal_obj"] + rec.offset
    same_path = I["attempts"] == r.info["attempts"] and I["iterations"] == r.info["iterations"]
    tol = 1e-6 if same_path else max(1e-6, 2 * eps)
    assert abs(I["primal_obj"] - oref) <= tol * (1 + abs(oref))
    if eps <= 1e-8:
        ref = p.obj_star()
        assert abs(I["primal_obj"] - ref) <= 1e-6 * (1 + abs(ref))


def test_presolve_on_lps_without_reductions_changes_nothing(P):
    """No singleton rows, no fixed or empty columns: the same solve bitwise."""
    p = lpgen.batch_lp(4, 2, 300)
    a = P.solve(p, eps_rel=1e-6, time_limit_s=60.0)
    b = P.solve(p, eps_rel=1e-6, time_limit_s=60.0, presolve=1)
    assert (b.info["m_solved"], b.info["n_solved"]) == (p.m, p.n)
    assert a.info["iterations"] == b.info["iterations"]
    np.testing.assert_array_equal(a.x, b.x)
    np.testing.assert_array_equal(a.y, b.y)
    np.testing.assert_array_equal(a.rc, b.rc)


@pytest.mark.parametrize("gen", [lpgen.infeasible_lp, lpgen.unbounded_lp])
def test_certificates_survive_postsolve(P, orc, gen):
    """The reduced LP's ray, extended by the postsolve, certifies the user's LP."""
    p = _with_singletons(gen(2, 200), 3)
    res = P.solve(p, presolve=1, eps_rel=1e-8, max_iter=200_000, time_limit_s=60.0)
    assert res.info["m_solved"] < p.m
    r = orc.solve(p, eps_rel=1e-8, max_iter=200_000)
    assert res.status == r.status
    if res.status == "PRIMAL_INFEASIBLE":
        obj, _ = check_dual_ray(p, res.y, res.rc)
        assert np.linalg.norm(res.y) == pytest.approx(1.0, rel=1e-10)
        assert res.info["ray_obj"] == pytest.approx(obj, rel=1e-6)
    else:
        assert res.status == "DUAL_INFEASIBLE"
        check_primal_ray(p, res.x)


def test_infeasible_by_presolve_is_solved_as_given(P):
    """Presolve sees crossing bounds; the LP is then solved without presolve and
    the method returns its own certificate."""
    p = lpgen.from_dense([[1.0, 1.0], [1.0, 0.0], [1.0, 0.0]], [1, 1], [1, 3, 2], [0, 0], [INF, INF], [1, 1, 2])
    assert P.pdlp_presolve(p)["status"] == "PRIMAL_INFEASIBLE"
    res = P.solve(p, presolve=1, eps_rel=1e-8, max_iter=200_000, time_limit_s=60.0)
    assert (res.info["m_solved"], res.info["n_solved"]) == (p.m, p.n)
    assert res.status == "PRIMAL_INFEASIBLE"
    check_dual_ray(p, res.y, res.rc)


def test_warm_start_and_refused_queries(P):
    p = _skewed(1, 2000)
    h = P.pdlp_create(p, presolve=1, eps_rel=1e-6, time_limit_s=60.0)
    try:
        P.pdlp_solve(h)
        x, y, rc, I = P.pdlp_get_solution(h)
        assert I["status_name"] == "OPTIMAL" and x.shape == (p.n,) and y.shape == (p.m,)
        with pytest.raises(P.PdlpError, match="PDLP_ERR_UNSUPPORTED"):
            P.pdlp_get_iterate(h)
        with pytest.raises(P.PdlpError, match="PDLP_ERR_UNSUPPORTED"):
            P.pdlp_get_scaling(h)
        # restart from the (full-size) solution: done at the first evaluations
        P.pdlp_set_warm_start(h, x, y)
        P.pdlp_solve(h)
        I2 = P.pdlp_get_solution(h)[3]
        assert I2["status_name"] == "OPTIMAL" and I2["iterations"] <= max(64, I["iterations"] // 4)
    finally:
        P.pdlp_destroy(h)
