"""Row renumbering on the device (row_order = 1, the default for single-LP
handles; with 2 the columns are renumbered too, at any size) against the
given order (row_order = 0) and the oracle.

The renumbering happens after the scaling and every row and column vector
crossing the interface is mapped back, so: the preconditioner and the scaled
matrix are bitwise those of the given order (and the oracle's); the first
accepted steps match the oracle within max(1e-10, 10 x) its own spread under
renumbering (only summation orders differ); a warm start from the known
optimum in the caller's order ends at the first evaluation; solves re-check
with the FP64 evaluator; the iterate after a few steps agrees with the
given-order run to rounding.
"""
import numpy as np
import pytest

import lpgen
from tests import bars

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    from paper_2311_12180_amd import pdlp
    pdlp.lib()
    return pdlp


def _rel_inf(a, b):
    return float(np.abs(a - b).max(initial=0.0) / max(1.0, np.abs(b).max(initial=0.0)))


def _skewed(seed=0, m=4000):
    return lpgen.skewed_lp(seed, m=m, n=2 * m, nnz_target=20 * m, cap=m // 5)


@pytest.mark.parametrize("renum", [1, 2])
@pytest.mark.parametrize("prec", [0, 1])
def test_scaling_is_that_of_the_given_order(P, orc, prec, renum):
    p = _skewed(1)
    out = []
    for order in (0, renum):
        h = P.pdlp_create(p, row_order=order, a_precision=prec, time_limit_s=30.0)
        try:
            out.append(P.pdlp_get_scaling(h))
        finally:
            P.pdlp_destroy(h)
    for a, b in zip(*out):
        np.testing.assert_array_equal(a, b)
    E1, E2, ws = orc.rescale(p)
    np.testing.assert_array_equal(out[1][0], E1)
    np.testing.assert_array_equal(out[1][2], ws)


@pytest.mark.parametrize("renum", [1, 2])
@pytest.mark.parametrize("make", [lambda: _skewed(2), lambda: lpgen.mixed_lp(4), lambda: lpgen.transportation(3, 20, 25)])
def test_first_steps_match_oracle(P, orc, make, renum):
    p = make()
    opts = dict(eps_rel=0.0, max_iter=100)
    r = orc.solve(p, **opts)
    spread = 0.0
    for s in range(3):
        rng = np.random.default_rng(40 + s)
        rp, cp = rng.permutation(p.m), rng.permutation(p.n)
        q = orc.solve(lpgen.permute(p, rp, cp), **opts)
        if q.info["attempts"] != r.info["attempts"]:
            pytest.skip("the oracle's own decisions change under renumbering (a near-tie)")
        spread = max(spread, _rel_inf(q.x, r.x[cp]), _rel_inf(q.y, r.y[rp]))
    res = P.solve(p, row_order=renum, time_limit_s=60.0, **opts)
    tol = bars.bar(spread)
    ex, ey = _rel_inf(res.x, r.x), _rel_inf(res.y, r.y)
    print(f"{p.name}: x {ex:.1e} y {ey:.1e} (oracle spread {spread:.1e}, "
          f"error / spread {bars.ratio(max(ex, ey), spread)})")
    assert res.info["attempts"] == r.info["attempts"]
    assert ex <= tol and ey <= tol


@pytest.mark.parametrize("renum", [1, 2])
def test_iterate_agrees_with_given_order(P, renum):
    p = _skewed(3)
    its = []
    for order in (0, renum):
        h = P.pdlp_create(p, row_order=order, eps_rel=0.0, max_iter=20, time_limit_s=30.0)
        try:
            P.pdlp_solve(h)
            xh, yh, st = P.pdlp_get_iterate(h)
            its.append((xh, yh, st["attempts"]))
        finally:
            P.pdlp_destroy(h)
    assert its[0][2] == its[1][2]
    assert _rel_inf(its[1][0], its[0][0]) <= 1e-12
    assert _rel_inf(its[1][1], its[0][1]) <= 1e-12


@pytest.mark.parametrize("renum", [1, 2])
def test_warm_start_from_the_optimum_in_callers_order(P, orc, renum):
    p = _skewed(4)
    h = P.pdlp_create(p, eps_rel=1e-6, time_limit_s=60.0, row_order=renum)
    try:
        P.pdlp_solve(h)
        x, y, rc, I = P.pdlp_get_solution(h)
        assert I["status_name"] == "OPTIMAL"
        assert orc.evaluate(p, x, y)["rel_kkt"] <= 1e-6 * (1 + 1e-6)
        # the known optimum, given in the caller's row order
        P.pdlp_set_warm_start(h, p.x_star, p.y_star)
        P.pdlp_solve(h)
        x2, y2, _, I2 = P.pdlp_get_solution(h)
        # a start in the wrong row order is far from optimal and takes hundreds of steps
        assert I2["status_name"] == "OPTIMAL" and I2["iterations"] <= 64, (I2["iterations"], I["iterations"])
        if I2["iterations"] == 0:
            np.testing.assert_allclose(y2, p.y_star, rtol=0, atol=1e-9 * (1 + np.abs(p.y_star).max()))
            np.testing.assert_allclose(x2, p.x_star, rtol=0, atol=1e-9 * (1 + np.abs(p.x_star).max()))
    finally:
        P.pdlp_destroy(h)


@pytest.mark.parametrize("order", [0, 1, 2])
def test_both_orders_solve(P, orc, order):
    p = _skewed(5)
    res = P.solve(p, row_order=order, eps_rel=1e-8, time_limit_s=60.0)
    assert res.status == "OPTIMAL"
    e = orc.evaluate(p, res.x, res.y)
    assert e["rel_kkt"] <= 1e-8 * (1 + 1e-6)
    np.testing.assert_allclose(res.rc, orc.reduced_costs(p, res.y), rtol=1e-9, atol=1e-9)
    ref = p.obj_star()
    assert abs(res.info["primal_obj"] - ref) <= 1e-6 * (1 + abs(ref))


def test_presolve_with_renumbered_columns(P, orc):
    """Presolve (this LP has empty columns), then the reduced LP renumbered
    by rows and columns: the postsolved solution is the user's LP's, in the
    user's order (rel KKT within 2 eps: the reduced LP's norms differ from the
    user's), reduced costs included."""
    p = _skewed(0)
    res = P.solve(p, presolve=1, row_order=2, eps_rel=1e-8, time_limit_s=60.0)
    assert res.info["n_solved"] < p.n
    assert res.status == "OPTIMAL"
    e = orc.evaluate(p, res.x, res.y)
    assert e["rel_kkt"] <= 2e-8
    np.testing.assert_allclose(res.rc, orc.reduced_costs(p, res.y), rtol=1e-9, atol=1e-9)
    ref = p.obj_star()
    assert abs(res.info["primal_obj"] - ref) <= 1e-6 * (1 + abs(ref))
