"""Pins of the oracle's infeasibility detection (Section 2.2 names the two
sequences it watches -- the difference of consecutive iterates and the
normalized iterate -- and leaves the certificate test to its citation).

What pins it, independently of the oracle's own code:
  * Farkas' lemma, checked here from first principles on every certificate the
    oracle returns: a dual ray y (sign-feasible for each row type), lam in the
    cone Lambda with A'y + lam = 0 and b'y + l'lam+ - u'lam- > 0 proves that
    no x satisfies the rows and the bounds; a primal ray x in the recession
    cone of the bounds with Ax in the row cones and c'x < 0 proves that a
    feasible LP is unbounded.
  * Closed forms on tiny LPs (hand-computed ray quantities).
  * LPs with a planted contradiction or a planted improving ray are flagged
    with the right status; feasible LPs of every family never are.
"""
import numpy as np
import pytest

import lpgen
import oracle
from tests.farkas import check_dual_ray as _check_dual_ray, check_primal_ray as _check_primal_ray

INF = np.inf


def _lp(A, b, rt, c, l, u):
    return lpgen.from_dense(A, c, b, l, u, rt)


# ---------------------------------------------------------------- closed forms

def test_ray_test_closed_forms():
    # x1 + x2 >= 2 and x1 + x2 <= 1, x >= 0: y = (1, -1) gives A'y = 0, b'y = 1
    p = _lp([[1, 1], [1, 1]], [2, 1], [1, 2], [1, 1], [0, 0], [INF, INF])
    r = oracle.ray_test(p, np.zeros(2), np.array([1.0, -1.0]))
    assert r["verdict"] == 1
    assert r["dual_ray_obj"] == 1.0 and r["dual_ray_res"] == 0.0
    assert r["y_norm"] == pytest.approx(np.sqrt(2.0), rel=1e-15)
    assert r["dual_ray_obj_abs"] == 3.0
    # the wrong sign on the LE row is clipped away: y = (1, 0) leaves A'y = (1, 1)
    # absorbed by lam >= 0 at the lower bounds (lam = -A'y would be negative: not allowed)
    r = oracle.ray_test(p, np.zeros(2), np.array([1.0, 1.0]))
    np.testing.assert_array_equal(r["ray_y"], [1.0, 0.0])
    assert r["dual_ray_res"] == pytest.approx(np.sqrt(2.0), rel=1e-15)
    assert r["verdict"] == 0
    # x1 + x2 >= 5 with 0 <= x <= 2: y = 1, lam = -A'y = (-1, -1) at the upper
    # bounds, objective 5 - 2 - 2 = 1 > 0
    p = _lp([[1, 1]], [5], [1], [1, -1], [0, 0], [2, 2])
    r = oracle.ray_test(p, np.zeros(2), np.array([1.0]))
    assert r["verdict"] == 1 and r["dual_ray_obj"] == 1.0 and r["dual_ray_res"] == 0.0
    np.testing.assert_array_equal(r["lam"], [-1.0, -1.0])
    # with u = 3 the box reaches the row (objective 5 - 6 < 0): no certificate
    p = _lp([[1, 1]], [5], [1], [1, -1], [0, 0], [3, 3])
    r = oracle.ray_test(p, np.zeros(2), np.array([1.0]))
    assert r["verdict"] == 0 and r["dual_ray_obj"] == -1.0
    # min -x1 s.t. x1 - x2 >= 0, x >= 0: x = (1, 1) is an improving ray
    p = _lp([[1, -1]], [0], [1], [-1, 0], [0, 0], [INF, INF])
    r = oracle.ray_test(p, np.array([1.0, 1.0]), np.zeros(1))
    assert r["verdict"] == 2 and r["primal_ray_obj"] == -1.0 and r["primal_ray_res"] == 0.0
    # x = (1, 2) leaves the row cone by 1
    r = oracle.ray_test(p, np.array([1.0, 2.0]), np.zeros(1))
    assert r["verdict"] == 0 and r["primal_ray_res"] == 1.0
    # projection onto the recession cone: a boxed coordinate is zeroed, a
    # lower-bounded one clipped at 0, a free one kept
    p = _lp([[0, 0, 0]], [0], [0], [1, 1, 1], [0, 0, -INF], [1, INF, INF])
    r = oracle.ray_test(p, np.array([3.0, -2.0, -5.0]), np.zeros(1))
    np.testing.assert_array_equal(r["ray_x"], [0.0, 0.0, -5.0])
    assert r["primal_ray_obj"] == -5.0 and r["verdict"] == 2


def test_cancellation_cannot_fake_a_certificate():
    """Every variable boxed: lam absorbs all of A'y, so only the objective's
    sign decides.  A tight feasible LP (x1 >= 10 on [0, 10]) has ray
    objective exactly 0 for y = e1 -- not a certificate -- and the magnitude
    guard keeps a rounding-level positive value from being one."""
    p = _lp([[1, 0], [1, 1]], [10, 3], [1, 1], [1, 1], [0, 0], [10, 10])
    r = oracle.ray_test(p, np.zeros(2), np.array([1.0, 0.0]))
    assert r["dual_ray_obj"] == 0.0 and r["verdict"] == 0
    p2 = _lp([[1, 0], [1, 1]], [10 + 1e-12, 3], [1, 1], [1, 1], [0, 0], [10, 10])
    r = oracle.ray_test(p2, np.zeros(2), np.array([1.0, 0.0]))
    assert 0.0 < r["dual_ray_obj"] < 1e-8 * r["dual_ray_obj_abs"] and r["verdict"] == 0
    s = oracle.solve(p, eps_rel=1e-8)
    assert s.status == "OPTIMAL"


# ---------------------------------------------------------------- solves

@pytest.mark.parametrize("case", ["two_rows", "box_row", "unbounded_row", "unbounded_free"])
def test_tiny_solves_return_valid_certificates(case):
    if case == "two_rows":
        p = _lp([[1, 1], [1, 1]], [2, 1], [1, 2], [1, 1], [0, 0], [INF, INF])
    elif case == "box_row":
        p = _lp([[1, 1]], [5], [1], [1, -1], [0, 0], [2, 2])
    elif case == "unbounded_row":
        p = _lp([[1, -1]], [0], [1], [-1, 0], [0, 0], [INF, INF])
    else:
        p = _lp([[0, 1]], [1], [0], [1, 0], [-INF, 0], [INF, 5])
    r = oracle.solve(p, eps_rel=1e-8, max_iter=100000)
    if case.startswith("unbounded"):
        assert r.status == "DUAL_INFEASIBLE"
        obj = _check_primal_ray(p, r.x)
        assert np.linalg.norm(r.x) == pytest.approx(1.0, rel=1e-12)
        assert r.info["ray_obj"] == pytest.approx(obj, rel=1e-12)
    else:
        assert r.status == "PRIMAL_INFEASIBLE"
        obj, _ = _check_dual_ray(p, r.y, r.rc)
        assert np.linalg.norm(r.y) == pytest.approx(1.0, rel=1e-12)
        assert r.info["ray_obj"] == pytest.approx(obj, rel=1e-10)
    if case == "box_row":
        # one row: the ray is e1 itself
        np.testing.assert_allclose(r.y, [1.0], rtol=1e-12)
        np.testing.assert_allclose(r.rc, [-1.0, -1.0], rtol=1e-12)
    if case == "unbounded_free":
        np.testing.assert_allclose(r.x, [-1.0, 0.0], atol=1e-12)


@pytest.mark.parametrize("gen", [lpgen.infeasible_lp, lpgen.bound_infeasible_lp, lpgen.unbounded_lp])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_planted_families(gen, seed):
    p = gen(seed, 200)
    r = oracle.solve(p, eps_rel=1e-8, max_iter=200000)
    if gen is lpgen.unbounded_lp:
        assert r.status == "DUAL_INFEASIBLE", r.status
        _check_primal_ray(p, r.x)
        # the planted column is the only unbounded direction of this LP's box
        assert abs(r.x[-1]) > 0.5
    else:
        assert r.status == "PRIMAL_INFEASIBLE", r.status
        _check_dual_ray(p, r.y, r.rc)
    assert r.info["ray_source"] in (0, 1)


def test_tests_only_every_infeas_every_th_evaluation():
    """The unbounded column is certified at the first test: the first
    evaluation with infeas_every = 1, the fourth (step 256) by default, the
    third with infeas_every = 3."""
    p = lpgen.unbounded_lp(0, 200)
    for every, k in ((1, 64), (4, 256), (3, 192)):
        r = oracle.solve(p, eps_rel=1e-8, max_iter=200000, infeas_every=every)
        assert r.status == "DUAL_INFEASIBLE" and r.info["iterations"] == k, (every, r.info["iterations"])


def test_detection_off_runs_to_the_limit():
    p = lpgen.infeasible_lp(0, 200)
    r = oracle.solve(p, eps_rel=1e-8, max_iter=2000, detect_infeas=0)
    assert r.status == "ITER_LIMIT" and r.info["iterations"] == 2000


@pytest.mark.parametrize("make", [
    lambda: lpgen.batch_lp(0, 3, 300),
    lambda: lpgen.batch_lp(1, 7, 150),
    lambda: lpgen.mixed_lp(4),
    lambda: lpgen.transportation(1, 12, 15),
    lambda: lpgen.tiny_dense_lp(5),
])
def test_feasible_lps_are_never_flagged(make):
    """Feasible bounded LPs of every family solve to rel KKT 1e-8 without a
    certificate at any of their evaluations."""
    p = make()
    r = oracle.solve(p, eps_rel=1e-8, max_iter=300000)
    assert r.status == "OPTIMAL", (p.name, r.status)
