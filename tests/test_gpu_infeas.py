"""GPU infeasibility detection (Section 2.2) against the CPU FP64 oracle.

Bars:
  * the same status as the oracle (PRIMAL_INFEASIBLE / DUAL_INFEASIBLE) on
    tiny closed-form LPs and on LPs with a planted contradiction or improving
    ray, in every matrix layout and with the FP32 matrix;
  * the returned certificate is valid by Farkas' lemma, checked from the
    definitions (tests/farkas.py), and reported with its objective and
    residual (info.ray_obj / ray_res match the returned unit ray);
  * detection happens within one test period (eval_period x infeas_every
    accepted steps) of the range of steps at which the oracle detects under
    rounding-level changes (renumbered rows and columns, b and c moved by
    1e-15): that step moves with rounding (512..832 for one planted LP in the
    oracle alone, testing at every evaluation); when the
    GPU took the oracle's path, the unit ray lies within max(1e-8, 10x) the
    oracle's own spread under renumbering (the rays are iterate differences of
    a diverging run, so their small entries carry the iterates' sensitivity to
    summation order);
  * feasible LPs are unaffected (the parity suites run with detection on);
  * the batched solver, also across a hand-off, gives each LP the oracle's
    status and a valid certificate.
"""
import numpy as np
import pytest

import lpgen
from tests import bars
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


def _tiny(case):
    if case == "two_rows":
        return lpgen.from_dense([[1, 1], [1, 1]], [1, 1], [2, 1], [0, 0], [INF, INF], [1, 2], case)
    if case == "box_row":
        return lpgen.from_dense([[1, 1]], [1, -1], [5], [0, 0], [2, 2], [1], case)
    if case == "unbounded_row":
        return lpgen.from_dense([[1, -1]], [-1, 0], [0], [0, 0], [INF, INF], [1], case)
    return lpgen.from_dense([[0, 1]], [1, 0], [1], [-INF, 0], [INF, 5], [0], case)


CASES = ([("tiny", c) for c in ("two_rows", "box_row", "unbounded_row", "unbounded_free")]
         + [(g, s) for g in ("infeasible", "bound_infeasible", "unbounded") for s in (0, 1)])


def _make(kind, arg):
    if kind == "tiny":
        return _tiny(arg)
    return getattr(lpgen, f"{kind}_lp")(arg, 200)


def _check(p, status, x, y, rc, info):
    if status == "PRIMAL_INFEASIBLE":
        obj, res = check_dual_ray(p, y, rc)
        assert np.linalg.norm(y) == pytest.approx(1.0, rel=1e-10)
        assert info["ray_obj"] == pytest.approx(obj, rel=1e-8)
    else:
        assert status == "DUAL_INFEASIBLE"
        obj = check_primal_ray(p, x)
        assert np.linalg.norm(x) == pytest.approx(1.0, rel=1e-10)
        assert info["ray_obj"] == pytest.approx(obj, rel=1e-8)


def _ray(res):
    return res.y if res.status == "PRIMAL_INFEASIBLE" else res.x


def _perturbed(p, s):
    """p with b and c moved by one part in 1e15 (rounding level)."""
    import dataclasses
    f = 1.0 + (1e-15 if s % 2 == 0 else -1e-15)
    return dataclasses.replace(p, b=p.b * f, c=p.c * (2.0 - f))


def _oracle_spread(orc, p, opts, r, copies=3):
    """The oracle under rounding-level changes -- renumbered rows and columns
    (the summation order) and b, c moved by 1e-15 relative: the range of its
    detection steps, and how far its unit ray moves (None when the status,
    step or certifying candidate changes).  On an infeasible LP the iterates
    diverge along the ray, which lies (nearly) in the null space of K', so the
    step bound's denominator dy'K dx is a cancellation and the step sizes, and
    with them the detection step, move with any rounding change (a 2 x 2 LP:
    step 1280 as given, 512 with b moved by 1e-15)."""
    ks = [r.info["iterations"]]
    spread = 0.0
    for s in range(copies + 2):
        if s < copies:
            rng = np.random.default_rng(77 + s)
            rp, cp = rng.permutation(p.m), rng.permutation(p.n)
            q = orc.solve(lpgen.permute(p, rp, cp), **opts)
        else:
            rp, cp = np.arange(p.m), np.arange(p.n)
            q = orc.solve(_perturbed(p, s), **opts)
        assert q.status == r.status
        ks.append(q.info["iterations"])
        if spread is not None:
            if q.info["iterations"] != r.info["iterations"] or q.info["ray_source"] != r.info["ray_source"]:
                spread = None
            else:
                ref = _ray(r)[rp] if r.status == "PRIMAL_INFEASIBLE" else _ray(r)[cp]
                spread = max(spread, float(np.abs(_ray(q) - ref).max()))
    return min(ks), max(ks), spread


PERIOD = 64 * 4   # accepted steps between certificate tests (eval_period x infeas_every)


@pytest.mark.parametrize("kind,arg,every", [c + (4,) for c in CASES]
                         + [("infeasible", 0, 1), ("bound_infeasible", 1, 1), ("unbounded", 0, 1)])
def test_certificates_match_oracle(P, orc, kind, arg, every):
    p = _make(kind, arg)
    opts = dict(eps_rel=1e-8, max_iter=200000, infeas_every=every)
    r = orc.solve(p, **opts)
    assert r.status in ("PRIMAL_INFEASIBLE", "DUAL_INFEASIBLE")
    res = P.solve(p, time_limit_s=60.0, **opts)
    I = res.info
    print(f"{p.name}: oracle {r.status} at {r.info['iterations']} (source {r.info['ray_source']}), "
          f"GPU {res.status} at {I['iterations']} (source {I['ray_source']}), "
          f"ray obj {I['ray_obj']:.3e} res {I['ray_res']:.1e}")
    assert res.status == r.status
    _check(p, res.status, res.x, res.y, res.rc, I)
    lo, hi, spread = _oracle_spread(orc, p, opts, r)
    print(f"  oracle detection steps under renumbering: {lo}..{hi}")
    assert lo - 64 * every <= I["iterations"] <= hi + 64 * every
    if I["iterations"] == r.info["iterations"] and I["ray_source"] == r.info["ray_source"] and spread is not None:
        d = float(np.abs(_ray(res) - _ray(r)).max())
        print(f"  unit ray vs oracle {d:.1e}, oracle spread {spread:.1e}")
        assert d <= bars.bar(spread, 1e-8), (d, spread)


@pytest.mark.parametrize("layout,prec", [(1, 0), (2, 0), (0, 1), (9, 1), (64, 0), (80, 1), (96, 0)])
def test_every_layout_and_fp32_matrix(P, orc, layout, prec):
    """Column panels (two-phase kernels), XCD-remapped row blocks, SELL-64
    passes over both matrices (with rows and columns renumbered; their
    evaluation passes, the certificate tests included, run on the same
    chunks) and the FP32 matrix compute the same certificates."""
    for kind, arg in (("infeasible", 1), ("unbounded", 2)):
        p = _make(kind, arg)
        opts = dict(eps_rel=1e-8, max_iter=200000, a_precision=prec)
        r = orc.solve(p, **opts)
        order = 2 if layout & 64 else 1
        res = P.solve(p, time_limit_s=60.0, spmv_layout=layout, row_order=order, **opts)
        assert res.status == r.status, (kind, layout, prec)
        _check(p, res.status, res.x, res.y, res.rc, res.info)


def test_detection_off_runs_to_the_limit(P):
    p = lpgen.infeasible_lp(0, 200)
    res = P.solve(p, eps_rel=1e-8, max_iter=2000, detect_infeas=0, time_limit_s=60.0)
    assert res.status == "ITER_LIMIT" and res.info["iterations"] == 2000


def test_feasible_lp_unaffected(P, orc):
    """A feasible LP solves to the same point with detection on and off."""
    p = lpgen.batch_lp(2, 5, 300)
    a = P.solve(p, eps_rel=1e-8, time_limit_s=60.0)
    b = P.solve(p, eps_rel=1e-8, time_limit_s=60.0, detect_infeas=0)
    assert a.status == b.status == "OPTIMAL"
    assert a.info["iterations"] == b.info["iterations"]
    np.testing.assert_array_equal(a.x, b.x)
    np.testing.assert_array_equal(a.y, b.y)


@pytest.mark.parametrize("handoff", [0, 64])
def test_batch_certificates(P, orc, handoff):
    probs = [lpgen.batch_lp(9, 0, 150), lpgen.infeasible_lp(3, 150), lpgen.unbounded_lp(4, 120),
             lpgen.bound_infeasible_lp(5, 180), _tiny("two_rows"), _tiny("unbounded_free"),
             lpgen.batch_lp(9, 1, 90), lpgen.infeasible_lp(6, 100)]
    opts = dict(eps_rel=1e-8, max_iter=200000)
    h = P.pdlp_create_batch(probs, time_limit_s=120.0, batch_handoff=handoff, handoff_streams=3, **opts)
    P.pdlp_solve_batch(h)
    for k, p in enumerate(probs):
        x, y, rc, I = P.pdlp_get_solution_batch(h, k)
        r = orc.solve(p, **opts)
        assert I["status_name"] == r.status, (k, p.name, I["status_name"], r.status)
        if r.status != "OPTIMAL":
            _check(p, I["status_name"], x, y, rc, I)
            lo, hi, _ = _oracle_spread(orc, p, opts, r, copies=2)
            assert lo - PERIOD <= I["iterations"] <= hi + PERIOD, (k, p.name, I["iterations"], lo, hi)
