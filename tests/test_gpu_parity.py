"""GPU parity: the HIP solver (through the C ABI) against the CPU FP64 oracle.

Bars:
  * preconditioner D1, D2 and the scaled matrix: bitwise equal (both sides
    compute the same row reductions in the same order and the same products);
  * iterates after k accepted steps (k <= 100): identical decisions (every
    accept/reject, candidate and restart reason) and ||gpu - oracle||_inf /
    max(1, ||oracle||_inf) <= 1e-10 for x~ and y~ on the m=1000, n=2000
    random LP; on the other families the bar is max(1e-10, 10 x the
    oracle's own spread under a row/column renumbering), because there the
    step bound's denominator cancels and the trajectory itself amplifies
    rounding-order differences;
  * end to end: objective within 1e-6 relative of the oracle's at rel KKT
    1e-4 and 1e-8, and the returned point passes the oracle's FP64 evaluator.
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


def _long_row_lp(seed=0):
    """Random LP with a few rows longer than one LDS tile (chunked rows) and
    a dense column, plus empty rows and empty columns."""
    rng = np.random.default_rng(seed)
    m, n = 300, 9000
    rows, cols = [], []
    for i in range(m):
        if i in (3, 150):
            L = 7000 if i == 3 else 3073     # two tiles and a bit; one more than a tile (3072)
        elif i % 37 == 0:
            L = 0
        else:
            L = int(rng.integers(1, 30))
        c = rng.choice(n - 10, L, replace=False)   # last 10 columns stay empty
        rows += [i] * L
        cols += list(c)
    rows += list(range(m)); cols += [n - 11] * m    # a dense column
    rows = np.array(rows); cols = np.array(cols)
    key = rows * n + cols
    _, keep = np.unique(key, return_index=True)
    rows, cols = rows[keep], cols[keep]
    vals = rng.standard_normal(len(rows))
    row_ptr, col_idx, val = lpgen._csr_from_coo(m, n, rows, cols, vals)
    rt = rng.integers(0, 3, m).astype(np.int8)
    l = np.zeros(n); u = np.full(n, 4.0)
    b, c, xs, ys, lam = lpgen._certify(rng, m, n, row_ptr, col_idx, val, rt, l, u)
    return lpgen.Problem(m, n, row_ptr, col_idx, val, c, b, l, u, rt, "long_rows", xs, ys, lam)


PROBLEMS = {
    "random_1000x2000": lambda: lpgen.config0(0),
    "skewed_3000x6000": lambda: lpgen.skewed_lp(2, m=3000, n=6000, nnz_target=60000, cap=5000),
    "transport_30x40": lambda: lpgen.transportation(1, 30, 40),
    "mixed_bounds": lambda: lpgen.mixed_lp(1),
    "long_rows": lambda: _long_row_lp(0),
    # 3 column panels of the LDS-staged layout (16,384 columns each)
    "skewed_20000x40000": lambda: lpgen.skewed_lp(3, m=20000, n=40000, nnz_target=400000, cap=8000),
}


def _rel_inf(a, b):
    return float(np.abs(a - b).max(initial=0.0) / max(1.0, np.abs(b).max(initial=0.0)))


@pytest.mark.parametrize("name", list(PROBLEMS))
def test_scaling_is_bitwise_oracle(P, orc, name):
    p = PROBLEMS[name]()
    h = P.pdlp_create(p)
    D1, D2, vs = P.pdlp_get_scaling(h)
    oD1, oD2, ovs = orc.rescale(p)
    np.testing.assert_array_equal(D1, oD1)
    np.testing.assert_array_equal(D2, oD2)
    np.testing.assert_array_equal(vs, ovs)


def _rounding_spread(orc, p, opts, copies=4):
    """How far the oracle moves from itself when only the summation order
    changes (rows and columns renumbered, `copies` times): the method's own
    sensitivity to rounding over the same iterations.  The step bound's
    denominator dy'K dx cancels heavily at some steps, so on some LPs this is
    far above 1e-10.  Returns (oracle result, iterate spread, scalar spread,
    stable) where `stable` says every copy took the same decisions."""
    a = orc.solve(p, trace_cap=4096, **opts)
    sx = se = 0.0
    stable = True
    for s in range(copies):
        rng = np.random.default_rng(123 + s)
        rp, cp = rng.permutation(p.m), rng.permutation(p.n)
        b = orc.solve(lpgen.permute(p, rp, cp), trace_cap=4096, **opts)
        stable &= bool(np.array_equal(a.trace["att_acc"], b.trace["att_acc"])
                       and np.array_equal(a.trace["ev_cand"], b.trace["ev_cand"])
                       and np.array_equal(a.trace["ev_reason"], b.trace["ev_reason"]))
        sx = max(sx, _rel_inf(b.x_hat, a.x_hat[cp]), _rel_inf(b.y_hat, a.y_hat[rp]))
        se = max(se, abs(a.info["eta_hat"] - b.info["eta_hat"]) / a.info["eta_hat"],
                 abs(a.info["omega"] - b.info["omega"]) / a.info["omega"])
    return a, sx, se, stable


@pytest.mark.parametrize("name", list(PROBLEMS))
@pytest.mark.parametrize("period", [1, 64])
@pytest.mark.parametrize("kmax", [1, 10, 100])
def test_trajectory_matches_oracle(P, orc, name, period, kmax):
    """Identical decisions, and iterates within max(1e-10, 10 x the oracle's
    own rounding-order spread) after kmax accepted steps.  On the random LP of
    m=1000, n=2000 the spread is ~1e-14, so the bar there is 1e-10."""
    p = PROBLEMS[name]()
    opts = dict(eps_rel=0.0, max_iter=kmax, eval_period=period)
    h = P.pdlp_create(p, time_limit_s=60.0, trace=4096, **opts)
    P.pdlp_solve(h)
    xh, yh, st = P.pdlp_get_iterate(h)
    tr = P.pdlp_get_trace(h, 4096)
    r, sx, se, stable = _rounding_spread(orc, p, opts)
    if not stable:
        pytest.skip(f"{name} P={period} k={kmax}: the oracle itself takes different decisions when only "
                    "its summation order changes (a near-tie); no unique trajectory to compare")
    tol_x, tol_s = bars.bar(sx), bars.bar(se)
    ex, ey = _rel_inf(xh, r.x_hat), _rel_inf(yh, r.y_hat)
    ee = abs(st["eta_hat"] - r.info["eta_hat"]) / r.info["eta_hat"]
    print(f"{name} P={period} k={kmax}: x {ex:.2e} y {ey:.2e} eta_hat {ee:.2e} | "
          f"oracle spread x {sx:.2e} scalars {se:.2e} | tol {tol_x:.2e} {tol_s:.2e} | "
          f"error / spread {bars.ratio(max(ex, ey), sx)}")
    assert st["iterations"] == r.info["iterations"] == kmax
    np.testing.assert_array_equal(tr["att_acc"], r.trace["att_acc"])
    np.testing.assert_array_equal(tr["ev_reason"], r.trace["ev_reason"])
    np.testing.assert_array_equal(tr["ev_cand"], r.trace["ev_cand"])
    assert st["attempts"] == r.info["attempts"]
    assert st["restarts"] == r.info["restarts"]
    assert ex <= tol_x and ey <= tol_x
    assert ee <= tol_s
    assert abs(st["omega"] - r.info["omega"]) / r.info["omega"] <= tol_s
    if name == "random_1000x2000":
        assert max(ex, ey) <= 1e-10


LAYOUT_CASES = [(name, layout) for name in ("random_1000x2000", "skewed_3000x6000", "long_rows", "transport_30x40")
                for layout in (1, 2, 4, 5, 6, 8, 9, 13)]
# LDS-staged step passes of K (phase-1 workgroups of 256, 512 and 1024
# threads) on the LPs with long rows, one of them over three column panels
LAYOUT_CASES += [(name, layout) for name in ("skewed_3000x6000", "long_rows", "skewed_20000x40000")
                 for layout in (3, 19, 35)]
# SELL-64 step passes of K and K' (workgroups of 1024 and 512 threads with
# the leading 8192 gathered entries in LDS, of 256 threads without), rows and
# columns renumbered by length; on the 20000 x 40000 LP the gathered vectors
# are longer than the LDS slice, so both paths of the gather run
LAYOUT_CASES += [(name, layout) for name in ("random_1000x2000", "skewed_3000x6000", "long_rows",
                                              "transport_30x40", "skewed_20000x40000")
                 for layout in (64, 80, 96)]


@pytest.mark.parametrize("name,layout", LAYOUT_CASES)
def test_layouts_match_oracle(P, orc, name, layout):
    """Column panels (1), XCD-contiguous row blocks (2), their persistent-grid
    forms (4, 5, 6), the step passes on 6144-nonzero blocks (8, 9, 13), the
    LDS-staged step passes (3, 19, 35) and the SELL-64 step passes (64, 80,
    96, with rows and columns renumbered) follow the oracle's trajectory like
    the default layout: same decisions, iterates within the rounding-order
    bar, over 100 accepted steps."""
    p = PROBLEMS[name]()
    opts = dict(eps_rel=0.0, max_iter=100, eval_period=64)
    order = 2 if layout & 64 else 1
    h = P.pdlp_create(p, time_limit_s=60.0, trace=4096, spmv_layout=layout, row_order=order, **opts)
    P.pdlp_solve(h)
    xh, yh, st = P.pdlp_get_iterate(h)
    tr = P.pdlp_get_trace(h, 4096)
    info = P.pdlp_get_solution(h)[3]
    P.pdlp_destroy(h)
    if (layout & 3) == 3:   # LDS-staged step view of K; K' has no long rows here and keeps panels
        assert info["layout_k"] == layout
    else:
        assert (info["layout_k"], info["layout_kt"]) == (layout, layout)
    r, sx, se, stable = _rounding_spread(orc, p, opts)
    assert stable
    tol_x = bars.bar(sx)
    ex, ey = _rel_inf(xh, r.x_hat), _rel_inf(yh, r.y_hat)
    print(f"{name} layout {layout}: x {ex:.2e} y {ey:.2e} tol {tol_x:.2e} "
          f"error / spread {bars.ratio(max(ex, ey), sx)}")
    np.testing.assert_array_equal(tr["att_acc"], r.trace["att_acc"])
    np.testing.assert_array_equal(tr["ev_cand"], r.trace["ev_cand"])
    assert st["attempts"] == r.info["attempts"] and st["restarts"] == r.info["restarts"]
    assert ex <= tol_x and ey <= tol_x
    res = P.solve(p, eps_rel=1e-6, time_limit_s=60.0, max_iter=200000, spmv_layout=layout, row_order=order)
    ro = orc.solve(p, eps_rel=1e-6, max_iter=200000)
    assert res.status == "OPTIMAL"
    assert abs(res.info["primal_obj"] - ro.info["primal_obj"]) <= 1e-6 * (1 + abs(ro.info["primal_obj"]))
    assert orc.evaluate(p, res.x, res.y)["rel_kkt"] <= 1e-6 * (1 + 1e-6)


@pytest.mark.parametrize("eps", [1e-4, 1e-8])
@pytest.mark.parametrize("seed", [0, 1])
def test_random_lp_end_to_end(P, orc, eps, seed):
    p = lpgen.config0(seed)
    res = P.solve(p, eps_rel=eps, time_limit_s=60.0)
    r = orc.solve(p, eps_rel=eps)
    assert res.status == "OPTIMAL" and r.status == "OPTIMAL"
    assert res.info["rel_kkt"] <= eps
    obj = res.info["primal_obj"]
    assert abs(obj - r.info["primal_obj"]) <= 1e-6 * (1 + abs(r.info["primal_obj"]))
    e = orc.evaluate(p, res.x, res.y)
    assert e["rel_kkt"] <= eps * (1 + 1e-6)
    assert e["primal_obj"] == pytest.approx(obj, rel=1e-12, abs=1e-12)
    if eps <= 1e-8:
        assert abs(obj - p.obj_star()) <= 1e-6 * (1 + abs(p.obj_star()))
    lam = orc.reduced_costs(p, res.y)
    np.testing.assert_allclose(res.rc, lam, rtol=1e-9, atol=1e-9)


@pytest.mark.parametrize("name", ["skewed_3000x6000", "transport_30x40", "mixed_bounds", "long_rows"])
def test_other_families_end_to_end(P, orc, name):
    p = PROBLEMS[name]()
    res = P.solve(p, eps_rel=1e-6, time_limit_s=60.0, max_iter=200000)
    r = orc.solve(p, eps_rel=1e-6, max_iter=200000)
    assert res.status == r.status == "OPTIMAL"
    assert abs(res.info["primal_obj"] - r.info["primal_obj"]) <= 1e-6 * (1 + abs(r.info["primal_obj"]))
    assert orc.evaluate(p, res.x, res.y)["rel_kkt"] <= 1e-6 * (1 + 1e-6)


@pytest.mark.parametrize("layout", [-1, 80])
def test_fp32_matrix_mode(P, orc, layout):
    """FP32-rounded scaled matrix in the steps (in the default layout, and in
    the SELL-64 layout with rows and columns renumbered): trajectory parity
    with the oracle's FP32 mode, and rel KKT 1e-4 on the true (FP64) LP.  The
    objective at 1e-4 lies within max(1e-10, 10 x) the oracle's own
    objective spread under renumbering (copies that took the oracle's path)
    of the oracle's FP32-mode objective when the two took the same path (else
    2 eps), and within 2 eps of the FP64 oracle's: two points that both meet
    rel KKT eps can differ by about that much in objective, whatever the
    matrix precision."""
    p = lpgen.config0(2)
    lay = dict(spmv_layout=layout, row_order=2 if layout == 80 else 1)
    opts = dict(eps_rel=0.0, max_iter=100, eval_period=64, a_precision=1)
    h = P.pdlp_create(p, time_limit_s=60.0, **lay, **opts)
    P.pdlp_solve(h)
    xh, yh, st = P.pdlp_get_iterate(h)
    if layout == 80:
        I = P.pdlp_get_solution(h)[3]
        assert (I["layout_k"], I["layout_kt"]) == (80, 80)
    P.pdlp_destroy(h)
    r = orc.solve(p, **opts)
    assert st["attempts"] == r.info["attempts"] and st["restarts"] == r.info["restarts"]
    assert _rel_inf(xh, r.x_hat) <= 1e-10 and _rel_inf(yh, r.y_hat) <= 1e-10
    res = P.solve(p, eps_rel=1e-4, a_precision=1, time_limit_s=60.0, **lay)
    assert res.status == "OPTIMAL"
    e = orc.evaluate(p, res.x, res.y)
    assert e["rel_kkt"] <= 1e-4 * (1 + 1e-6)
    r64 = orc.solve(p, eps_rel=1e-4)
    r32 = orc.solve(p, eps_rel=1e-4, a_precision=1)
    obj = res.info["primal_obj"]
    e64 = abs(obj - r64.info["primal_obj"]) / (1 + abs(r64.info["primal_obj"]))
    e32 = abs(obj - r32.info["primal_obj"]) / (1 + abs(r32.info["primal_obj"]))
    same = res.info["iterations"] == r32.info["iterations"] and res.info["attempts"] == r32.info["attempts"]
    spread, copies = 0.0, 0
    for k in range(3):
        rng = np.random.default_rng(70 + k)
        rp, cp = rng.permutation(p.m), rng.permutation(p.n)
        q = orc.solve(lpgen.permute(p, rp, cp), eps_rel=1e-4, a_precision=1)
        if q.info["iterations"] == r32.info["iterations"] and q.info["attempts"] == r32.info["attempts"]:
            spread = max(spread, abs(q.info["primal_obj"] - r32.info["primal_obj"]) / (1 + abs(r32.info["primal_obj"])))
            copies += 1
    bar = bars.bar(spread) if (same and copies) else 2e-4
    print(f"fp32 objective error vs the FP64 oracle {e64:.1e}, vs the oracle's FP32 mode {e32:.1e} (same path {same}; "
          f"oracle spread {spread:.1e} over {copies} copies on its path, bar {bar:.1e})")
    assert e32 <= bar
    assert e64 <= 2e-4


def test_box_lp_without_rows(P):
    rng = np.random.default_rng(0)
    n = 1000
    c = rng.normal(size=n); l = -rng.random(n); u = rng.random(n)
    p = lpgen.Problem(0, n, np.zeros(1, np.int32), np.zeros(0, np.int32), np.zeros(0), c, np.zeros(0),
                      l, u, np.zeros(0, np.int8), "box")
    res = P.solve(p, eps_rel=1e-10, time_limit_s=30.0)
    assert res.status == "OPTIMAL"
    assert res.info["primal_obj"] == pytest.approx(float(np.sum(np.minimum(c * l, c * u))), rel=1e-9)


def test_single_variable(P, orc):
    p = lpgen.from_dense([[1.0]], [1.0], [1.0], [0.0], [10.0], [lpgen.ROW_GE])
    res = P.solve(p, eps_rel=1e-9, time_limit_s=30.0)
    r = orc.solve(p, eps_rel=1e-9)
    assert res.status == "OPTIMAL"
    assert res.info["iterations"] == r.info["iterations"]
    assert res.x[0] == pytest.approx(1.0, abs=1e-8)


def test_zero_start_already_optimal(P):
    p = lpgen.from_dense([[1.0, 1.0]], [1.0, 2.0], [0.0], [0.0, 0.0], [5.0, 5.0], [lpgen.ROW_GE])
    res = P.solve(p, eps_rel=1e-8, time_limit_s=30.0)
    assert res.status == "OPTIMAL" and res.info["iterations"] == 0


def test_warm_start_from_solution(P, orc):
    p = lpgen.config0(3)
    r = orc.solve(p, eps_rel=1e-8)
    h = P.pdlp_create(p, eps_rel=1e-6, time_limit_s=30.0)
    P.pdlp_set_warm_start(h, r.x, r.y, r.info["omega"])
    P.pdlp_solve(h)
    _, _, _, info = P.pdlp_get_solution(h)
    assert info["status"] == 1 and info["iterations"] <= 64
    with pytest.raises(P.PdlpError):
        P.pdlp_set_warm_start(h, np.full(p.n, np.nan))


def test_device_inputs_match_host_inputs(P):
    import torch
    p = lpgen.config0(4)
    dev = lpgen.Problem(p.m, p.n, *[torch.from_numpy(np.asarray(a)).cuda() for a in
                                    (p.row_ptr, p.col_idx, p.val, p.c, p.b, p.l, p.u, p.row_type)])
    a = P.solve(p, eps_rel=1e-6, time_limit_s=30.0)
    b = P.solve(dev, eps_rel=1e-6, time_limit_s=30.0)
    np.testing.assert_array_equal(a.x, b.x)
    np.testing.assert_array_equal(a.y, b.y)


@pytest.mark.parametrize("layout", [0, 1])
def test_run_to_run_bitwise(P, layout):
    p = lpgen.skewed_lp(5, m=4000, n=8000, nnz_target=80000, cap=4000)
    a = P.solve(p, eps_rel=1e-6, time_limit_s=30.0, spmv_layout=layout)
    b = P.solve(p, eps_rel=1e-6, time_limit_s=30.0, spmv_layout=layout)
    np.testing.assert_array_equal(a.x, b.x)
    np.testing.assert_array_equal(a.y, b.y)
    assert a.info["attempts"] == b.info["attempts"]


def test_state_errors(P):
    p = lpgen.config0(0)
    h = P.pdlp_create(p)
    with pytest.raises(P.PdlpError) as e:
        P.pdlp_get_solution(h)
    assert e.value.code == P.PDLP_ERR_STATE
    with pytest.raises(P.PdlpError):
        P.pdlp_profile_attempts(h, 4)


def test_limits(P):
    p = lpgen.config0(0)
    res = P.solve(p, eps_rel=1e-12, max_iter=100, time_limit_s=30.0)
    assert res.status == "ITER_LIMIT" and res.info["iterations"] == 100
    res = P.solve(lpgen.config0(0), eps_rel=1e-14, time_limit_s=0.05)
    assert res.status in ("TIME_LIMIT", "OPTIMAL")


def test_profile_attempts_runs(P):
    p = lpgen.config0(0)
    h = P.pdlp_create(p, eps_rel=1e-4, time_limit_s=30.0)
    P.pdlp_solve(h)
    ta, tb = P.pdlp_profile_attempts(h, 32)
    assert 0 < ta < 10 and 0 < tb < 10
    ba, bb = P.pdlp_step_bytes(h)
    assert ba > 16000 * 12 and bb > 16000 * 12
