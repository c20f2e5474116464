"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Every test here runs on the CPU.  None of them compares the oracle with a
retyped copy of its own formulas: they use closed forms, hand-derived worked
examples (tests/golden), LP duality identities, brute-force vertex
enumeration, library optima (scipy HiGHS, linear_sum_assignment) and exact
invariances.
"""
import math

import numpy as np
import pytest
import scipy.sparse as sp

import lpgen
from tests import exact


# ----------------------------------------------------------------------------- helpers

def ge_form(p):
    """>=-form data (K, q) of a user-orientation LP: LE rows negated."""
    le = p.row_type == lpgen.ROW_LE
    rows = np.repeat(np.arange(p.m), np.diff(p.row_ptr))
    val = np.where(le[rows], -p.val, p.val)
    q = np.where(le, -p.b, p.b)
    return val, q, (p.row_type != lpgen.ROW_EQ).astype(np.int8)


def read_golden(path):
    sections, cur = {}, None
    for line in open(path):
        line = line.split("#", 1)[0].strip()
        if not line:
            continue
        if line.startswith("["):
            cur = line.strip("[]")
            sections[cur] = []
            continue
        sections[cur].append(line)
    return sections


# ----------------------------------------------------------------------------- generator certificates

@pytest.mark.parametrize("maker", [
    lambda: lpgen.config0(0), lambda: lpgen.config0(3),
    lambda: lpgen.skewed_lp(1, m=3000, n=6000, nnz_target=60000, cap=800),
    lambda: lpgen.batch_lp(0, 7, 321), lambda: lpgen.mixed_lp(2),
    lambda: lpgen.mixed_lp(5, m=80, n=50),
])
def test_certificate_has_zero_kkt(orc, maker):
    """The constructed (x*, y*) satisfies the Section 4.1 tests to rounding:
    this pins the generator and the sign conventions of the oracle's residuals
    and objectives together (an error in either shows up here)."""
    p = maker()
    e = orc.evaluate(p, p.x_star, p.y_star)
    assert e["rel_kkt"] <= 1e-13
    assert abs(e["primal_obj"] - p.obj_star()) <= 1e-12 * (1 + abs(p.obj_star()))
    lam = orc.reduced_costs(p, p.y_star)
    np.testing.assert_allclose(lam, p.lam_star, atol=1e-11)


def test_wrong_dual_sign_is_detected(orc):
    """Flipping the sign of the LE-row duals (the sign-convention trap of the
    user orientation) must leave a visible dual residual or gap."""
    p = lpgen.config0(1)
    y = p.y_star.copy()
    le = p.row_type == lpgen.ROW_LE
    y[le] = -y[le]
    e = orc.evaluate(p, p.x_star, y)
    assert e["rel_kkt"] > 1e-3


def _feasible_pair_lp(seed):
    """An LP together with a primal feasible x and a dual feasible (y, lambda),
    all bound types present: q = Kx - s (s >= 0 on inequality rows, 0 on EQ),
    c = K'y + lambda with lambda in Lambda."""
    rng = np.random.default_rng(seed)
    m, n = 30, 45
    A = sp.random(m, n, density=0.2, random_state=rng, data_rvs=rng.standard_normal).toarray()
    row_type = rng.integers(0, 3, m).astype(np.int8)
    btype = rng.integers(0, 4, n)
    l = np.where(btype <= 1, -rng.uniform(0, 4, n), -np.inf)
    u = np.where(btype == 0, l + rng.uniform(1, 6, n), np.where(btype == 2, rng.uniform(0, 4, n), np.inf))
    x = np.where(np.isfinite(l) & np.isfinite(u), rng.uniform(np.where(np.isfinite(l), l, 0), np.where(np.isfinite(u), u, 1)),
                 np.where(np.isfinite(l), l + rng.exponential(2, n),
                          np.where(np.isfinite(u), u - rng.exponential(2, n), rng.normal(0, 2, n))))
    ax = A @ x
    s = rng.uniform(0, 1, m)
    b = np.where(row_type == 0, ax, np.where(row_type == 1, ax - s, ax + s))
    # dual: y free on EQ, >= 0 on GE, <= 0 on LE
    y = rng.normal(0, 1, m)
    y = np.where(row_type == 1, np.abs(y), np.where(row_type == 2, -np.abs(y), y))
    lam = rng.normal(0, 1, n)
    lam = np.where(np.isfinite(l) & np.isfinite(u), lam,
                   np.where(np.isfinite(l), np.abs(lam), np.where(np.isfinite(u), -np.abs(lam), 0.0)))
    c = A.T @ y + lam
    return lpgen.from_dense(A, c, b, l, u, row_type), x, y, lam, A


@pytest.mark.parametrize("seed", range(5))
def test_duality_gap_equals_complementarity(orc, seed):
    """Weak duality: at a primal feasible x and dual feasible (y, lambda),
    c'x - (b'y + l'lambda+ - u'lambda-) = sum_i y_i (a_i x - b_i)
    + sum_j lambda+_j (x_j - l_j) + sum_j lambda-_j (u_j - x_j) >= 0.
    The right-hand side is a different formula from the oracle's objectives."""
    p, x, y, lam, A = _feasible_pair_lp(seed)
    e = orc.evaluate(p, x, y)
    assert e["pres"] <= 1e-12 and e["dres"] <= 1e-12
    lp_, lm_ = np.maximum(lam, 0), np.maximum(-lam, 0)
    comp = float(y @ (A @ x - p.b)
                 + np.sum(np.where(lp_ > 0, lp_ * (x - np.where(np.isfinite(p.l), p.l, 0)), 0))
                 + np.sum(np.where(lm_ > 0, lm_ * (np.where(np.isfinite(p.u), p.u, 0) - x), 0)))
    assert comp >= 0
    gap = e["primal_obj"] - e["dual_obj"]
    assert gap == pytest.approx(comp, rel=1e-10, abs=1e-10)


# ----------------------------------------------------------------------------- eq. (pdhg)

@pytest.mark.parametrize("maker", [lambda: lpgen.config0(2), lambda: lpgen.mixed_lp(3)])
@pytest.mark.parametrize("tau,sigma", [(0.1, 0.1), (1.0, 3.0), (7.0, 0.05)])
def test_saddle_point_is_fixed_point_of_pdhg(orc, maker, tau, sigma):
    """A saddle point of eq. (primal-dual) is a fixed point of eq. (pdhg) for
    every tau, sigma > 0; a point that is not optimal is moved."""
    p = maker()
    val, q, ineq = ge_form(p)
    yk = np.where(p.row_type == lpgen.ROW_LE, -p.y_star, p.y_star)
    x1, y1 = orc.pdhg_step(p.row_ptr, p.col_idx, val, q, p.c, p.l, p.u, ineq, p.x_star, yk, tau, sigma)
    np.testing.assert_allclose(x1, p.x_star, rtol=0, atol=1e-11 * (1 + np.abs(p.x_star).max()))
    np.testing.assert_allclose(y1, yk, rtol=0, atol=1e-11 * (1 + np.abs(yk).max()))
    xp = p.x_star.copy()
    j = int(np.argmax(np.abs(p.lam_star) == 0))
    xp[j] += 0.1 if np.isfinite(p.u[j]) and xp[j] + 0.1 <= p.u[j] else -0.1
    x2, y2 = orc.pdhg_step(p.row_ptr, p.col_idx, val, q, p.c, p.l, p.u, ineq, xp, yk, tau, sigma)
    assert np.abs(y2 - yk).max() + np.abs(x2 - xp).max() > 1e-6


def test_pdhg_step_projections(orc):
    """Bounds hold after the primal projection; inequality duals are >= 0
    after the dual projection (Section 2.1)."""
    p = lpgen.mixed_lp(4)
    val, q, ineq = ge_form(p)
    rng = np.random.default_rng(0)
    x = rng.normal(0, 5, p.n)
    y = rng.normal(0, 5, p.m)
    x1, y1 = orc.pdhg_step(p.row_ptr, p.col_idx, val, q, p.c, p.l, p.u, ineq, x, y, 2.0, 2.0)
    assert np.all(x1 >= p.l) and np.all(x1 <= p.u)
    assert np.all(y1[ineq == 1] >= 0)


# ----------------------------------------------------------------------------- Algorithm 2

@pytest.mark.parametrize("cval", [1.0, 2.0])
def test_adaptive_step_worked_example(orc, cval):
    """Hand-derived trace of Algorithm 2 on min c x, x >= 1, 0 <= x <= 10
    (tests/golden/adaptive_step_1d.txt)."""
    import os
    g = read_golden(os.path.join(os.path.dirname(__file__), "golden", "adaptive_step_1d.txt"))
    env = {"inf": math.inf, "abs": abs}
    for line in g["defs"]:
        k, v = line.split("=", 1)
        env[k.strip()] = eval(v, {"__builtins__": {}}, env)
    p = lpgen.from_dense([[1.0]], [cval], [1.0], [0.0], [10.0], [lpgen.ROW_GE])
    r = orc.solve(p, max_iter=3, eval_period=64, trace_cap=16)
    att = g["attempts"]
    assert len(r.trace["att_k"]) == len(att)
    for i, line in enumerate(att):
        k, eta, etabar, acc = [s.strip() for s in line.split(",")]
        assert r.trace["att_k"][i] == int(k)
        assert r.trace["att_eta"][i] == pytest.approx(eval(eta, {"__builtins__": {}}, env), rel=1e-14)
        eb = eval(etabar, {"__builtins__": {}}, env)
        if math.isinf(eb):
            assert math.isinf(r.trace["att_etabar"][i])
        else:
            assert r.trace["att_etabar"][i] == pytest.approx(eb, rel=1e-13)
        assert r.trace["att_acc"][i] == int(acc)
    fin = {}
    for line in g[f"final c={int(cval)}"]:
        k, v = line.split("=", 1)
        fin[k.strip()] = eval(v, {"__builtins__": {}}, env)
    assert r.x_hat[0] == pytest.approx(fin["x_hat"], rel=1e-13)
    assert r.y_hat[0] == pytest.approx(fin["y_hat"], rel=1e-13)
    assert r.info["eta_hat"] == pytest.approx(fin["eta_hat"], rel=1e-13)
    assert r.info["sum_eta"] == pytest.approx(fin["sum_eta"], rel=1e-13)
    assert r.info["omega"] == pytest.approx(fin["omega"], rel=1e-15)
    assert r.info["iterations"] == 3 and r.info["attempts"] == 4


def _golden_env(g):
    env = {"__builtins__": {}, "inf": math.inf, "abs": abs, "min": min, "sqrt": math.sqrt, "exp": math.exp,
           "log": math.log}
    for line in g["defs"]:
        k, v = line.split("=", 1)
        env[k.strip()] = eval(v, env)
    return env


def check_evaluation_golden(orc, case):
    """Compare an oracle (module with solve()) with case A or B of
    tests/golden/evaluation_restart_1d.txt; raises AssertionError on a
    mismatch."""
    import os
    g = read_golden(os.path.join(os.path.dirname(__file__), "golden", "evaluation_restart_1d.txt"))
    env = _golden_env(g)
    for line in g["checks"]:
        assert eval(line, env), line
    opts = {k.strip(): int(v) for k, v in (s.split("=", 1) for s in g[f"{case}.options"])}
    p = lpgen.from_dense([[1.0]], [2.0], [1.0], [0.0], [math.inf], [lpgen.ROW_GE])
    r = orc.solve(p, eps_rel=0.0, detect_infeas=0, trace_cap=16, **opts)
    ev = lambda s: eval(s, env)
    att = g[f"{case}.attempts"]
    assert len(r.trace["att_k"]) == len(att)
    for i, line in enumerate(att):
        k, eta, etabar, acc = [s.strip() for s in line.split(",")]
        assert r.trace["att_k"][i] == int(k)
        assert r.trace["att_eta"][i] == pytest.approx(ev(eta), rel=1e-13)
        eb = ev(etabar)
        if math.isinf(eb):
            assert math.isinf(r.trace["att_etabar"][i])
        else:
            assert r.trace["att_etabar"][i] == pytest.approx(eb, rel=1e-12)
        assert r.trace["att_acc"][i] == int(acc)
    evs = g[f"{case}.evaluations"]
    assert len(r.trace["ev_k"]) == len(evs)
    for i, line in enumerate(evs):
        k, kc, ka, cand, reason, om = [s.strip() for s in line.split(",")]
        assert r.trace["ev_k"][i] == int(k)
        assert r.trace["ev_kkt_cur"][i] == pytest.approx(ev(kc), rel=1e-13)
        assert r.trace["ev_kkt_avg"][i] == pytest.approx(ev(ka), rel=1e-13)
        assert r.trace["ev_cand"][i] == int(cand)
        assert r.trace["ev_reason"][i] == int(reason)
        assert r.trace["ev_omega"][i] == pytest.approx(ev(om), rel=1e-14)
    fin = {k.strip(): ev(v) for k, v in (s.split("=", 1) for s in g[f"{case}.final"])}
    assert r.x_hat[0] == pytest.approx(fin["x_hat"], rel=1e-12)
    assert r.y_hat[0] == pytest.approx(fin["y_hat"], rel=1e-12)
    for key in ("eta_hat", "sum_eta", "omega", "kkt0"):
        assert r.info[key] == pytest.approx(fin[key], rel=1e-12), key
    for key in ("restarts", "iterations", "attempts"):
        assert r.info[key] == fin[key], key
    assert r.status == "ITER_LIMIT"


@pytest.mark.parametrize("case", ["A", "B"])
def test_evaluation_and_restart_worked_example(orc, case):
    """Hand-derived evaluation of Algorithm 1 on min 2x, x >= 1, x >= 0
    (tests/golden/evaluation_restart_1d.txt): the step-size-weighted average,
    KKT_omega with the omega^2 weights of eq. (kkt) for both iterates, the
    Section 3.4 candidate and criterion, the Section 2.2 primal weight update
    (case A) and its eps_zero guard (case B), KKT_0 recomputed with the new
    weight, and the next step taken from the restart point with that weight.
    tests/test_oracle_mutants.py shows that a uniform average, omega in place
    of omega^2, an inverted candidate and KKT_0 kept at the old weight each
    fail this check."""
    check_evaluation_golden(orc, case)


def test_step_bound_exceeds_inverse_spectral_norm(orc):
    """eta_bar = ||dz||_w^2 / (2|dy'K dx|) >= 1/||K||_2 for any dz (AM-GM and
    Cauchy-Schwarz), and every accepted step satisfies eta <= eta_bar."""
    p = lpgen.random_lp(4, 100, 100, 400, 6)
    D1, D2, vs = orc.rescale(p)
    Ks = sp.csr_matrix((vs, p.col_idx, p.row_ptr), shape=(p.m, p.n)).toarray()
    k2 = np.linalg.norm(Ks, 2)
    r = orc.solve(p, max_iter=400, eps_rel=1e-15, trace_cap=2000)
    eb = r.trace["att_etabar"]
    assert len(eb) >= 400
    assert np.all(eb >= (1 - 1e-12) / k2)
    acc = r.trace["att_acc"] == 1
    assert np.all(r.trace["att_eta"][acc] <= eb[acc])


# ----------------------------------------------------------------------------- restarts, primal weight

# (kkt_cand, kkt0, kkt_prev, t, k) -> reason; written from the three criteria of
# Section 3.4 with beta = (0.2, 0.8, 0.36): 1 sufficient, 2 necessary + no local
# progress, 3 long inner loop, 0 none.  Criteria are tested in that order.
RESTART_TABLE = [
    (0.10, 1.0, 0.50, 10, 100, 1),
    (0.20, 1.0, 0.10, 10, 100, 1),    # equality counts (<=)
    (0.50, 1.0, 0.40, 10, 100, 2),
    (0.50, 1.0, 0.60, 10, 100, 0),    # progress since the last check
    (0.50, 1.0, 0.50, 10, 100, 0),    # no strict increase
    (0.80, 1.0, 0.70, 10, 100, 2),    # equality counts (<=)
    (0.81, 1.0, 0.70, 10, 100, 0),
    (0.90, 1.0, 0.50, 36, 100, 3),    # t >= 0.36 k with equality
    (0.90, 1.0, 0.50, 35, 100, 0),
    (0.10, 1.0, 0.05, 50, 100, 1),    # (i) before (ii) and (iii)
    (0.50, 1.0, 0.40, 50, 100, 2),    # (ii) before (iii)
    (1.50, 1.0, 0.90, 64, 64, 3),     # first epoch: t = k
    (2.0, 10.0, 1.0, 1, 100, 1),
]


@pytest.mark.parametrize("row", RESTART_TABLE)
def test_restart_truth_table(orc, row):
    *args, want = row
    assert orc.restart_reason(*args) == want


def test_primal_weight_update_special_cases(orc):
    """theta = 1 gives dy/dx; theta = 0 keeps omega; theta = 1/2 gives the
    geometric mean sqrt(omega * dy/dx); omega = dy/dx is a fixed point;
    tiny dx or dy keep omega."""
    pw = orc.primal_weight_update
    assert pw(2.0, 6.0, 0.7, theta=1.0) == pytest.approx(3.0, rel=1e-15)
    assert pw(2.0, 6.0, 0.7, theta=0.0) == pytest.approx(0.7, rel=1e-15)
    assert pw(1.0, 9.0, 4.0, theta=0.5) == pytest.approx(6.0, rel=1e-15)
    assert pw(3.0, 6.0, 2.0, theta=0.3) == pytest.approx(2.0, rel=1e-15)
    assert pw(1e-12, 1.0, 5.0) == 5.0
    assert pw(1.0, 1e-12, 5.0) == 5.0


# ----------------------------------------------------------------------------- preconditioning

def test_ruiz_makes_diagonal_identity(orc):
    """One Ruiz pass maps diag(d) to diag(sign d) with D1 = D2 = |d|^-1/2;
    later passes and Pock-Chambolle leave the identity alone."""
    d = np.array([4.0, 0.25, -9.0, 1e3, 1e-2])
    p = lpgen.from_dense(np.diag(d), np.ones(5), np.ones(5), np.zeros(5), np.ones(5), [0] * 5)
    D1, D2, vs = orc.rescale(p, 10, 1.0)
    np.testing.assert_allclose(D1, np.abs(d) ** -0.5, rtol=1e-15)
    np.testing.assert_allclose(D2, np.abs(d) ** -0.5, rtol=1e-15)
    np.testing.assert_allclose(vs, np.sign(d), rtol=1e-15)


def test_pock_chambolle_on_sign_matrix(orc):
    """For a +-1 matrix Ruiz is a no-op; Pock-Chambolle with alpha = 1 gives
    row scale 1/sqrt(row nnz) and column scale 1/sqrt(column nnz)."""
    rng = np.random.default_rng(1)
    A = (rng.random((12, 20)) < 0.3) * rng.choice([-1.0, 1.0], (12, 20))
    A[:, A.any(0) == 0] = 0
    p = lpgen.from_dense(A, np.ones(20), np.ones(12), np.zeros(20), np.ones(20), [1] * 12)
    D1, D2, vs = orc.rescale(p, 10, 1.0)
    rc = np.count_nonzero(A, 1).astype(float)
    cc = np.count_nonzero(A, 0).astype(float)
    np.testing.assert_allclose(D1, np.where(rc > 0, rc ** -0.5, 1.0), rtol=1e-15)
    np.testing.assert_allclose(D2, np.where(cc > 0, cc ** -0.5, 1.0), rtol=1e-15)


def test_le_rows_are_negated_and_scaling_is_consistent(orc):
    """The scaled values equal D1_i * K_ij * D2_j with K the >=-form matrix
    (LE rows negated), and Ruiz alone drives every row and column inf-norm to 1."""
    p = lpgen.mixed_lp(6, m=50, n=70)
    D1, D2, vs = orc.rescale(p, 10, 1.0)
    val, _, _ = ge_form(p)
    rows = np.repeat(np.arange(p.m), np.diff(p.row_ptr))
    np.testing.assert_allclose(vs, D1[rows] * val * D2[p.col_idx], rtol=1e-13)
    assert np.all(D1 > 0) and np.all(D2 > 0)
    D1r, D2r, vr = orc.rescale(p, 30, -1.0)
    Ar = np.abs(sp.csr_matrix((vr, p.col_idx, p.row_ptr), shape=(p.m, p.n)).toarray())
    np.testing.assert_allclose(Ar.max(1), 1.0, atol=1e-6)
    np.testing.assert_allclose(Ar.max(0), 1.0, atol=1e-6)


# ----------------------------------------------------------------------------- whole method: optima

@pytest.mark.parametrize("seed", range(16))
def test_optimum_matches_vertex_enumeration(orc, seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(2, 6)); m = int(rng.integers(1, 5))
    p = lpgen.tiny_dense_lp(seed, n, m)
    A = p.to_scipy().toarray()
    best, _ = exact.vertex_enumeration(A, p.b, p.row_type, p.c, p.l, p.u)
    r = orc.solve(p, eps_rel=1e-10, max_iter=500000)
    assert r.status == "OPTIMAL"
    assert r.info["primal_obj"] == pytest.approx(best, rel=1e-7, abs=1e-7)


def test_box_lp_closed_form(orc):
    rng = np.random.default_rng(3)
    n = 50
    c = rng.normal(0, 1, n)
    l = rng.uniform(-3, 0, n)
    u = l + rng.uniform(0.5, 4, n)
    # one-sided bounds only on the side the objective pushes toward
    l[(c < 0) & (np.arange(n) % 3 == 0)] = -np.inf
    u[(c > 0) & (np.arange(n) % 3 == 1)] = np.inf
    p = lpgen.Problem(0, n, np.zeros(1, np.int32), np.zeros(0, np.int32), np.zeros(0), c,
                      np.zeros(0), l, u, np.zeros(0, np.int8), "box")
    want, _ = exact.box_lp_optimum(c, l, u)
    r = orc.solve(p, eps_rel=1e-12)
    assert r.status == "OPTIMAL"
    assert r.info["primal_obj"] == pytest.approx(want, rel=1e-10)


def test_fractional_knapsack(orc):
    rng = np.random.default_rng(5)
    n = 25
    v = rng.uniform(1, 10, n); w = rng.uniform(1, 10, n); W = 0.35 * w.sum()
    p = lpgen.from_dense(w[None, :], -v, [W], np.zeros(n), np.ones(n), [lpgen.ROW_LE])
    r = orc.solve(p, eps_rel=1e-10, max_iter=500000)
    assert r.status == "OPTIMAL"
    assert -r.info["primal_obj"] == pytest.approx(exact.knapsack_optimum(v, w, W), rel=1e-8)


def test_assignment_matches_hungarian(orc):
    from scipy.optimize import linear_sum_assignment
    rng = np.random.default_rng(11)
    k = 7
    C = rng.random((k, k))
    A = np.zeros((2 * k, k * k))
    for i in range(k):
        A[i, i * k:(i + 1) * k] = 1
        A[k + i, i::k] = 1
    p = lpgen.from_dense(A, C.reshape(-1), np.ones(2 * k), np.zeros(k * k), np.full(k * k, np.inf),
                         [0] * (2 * k))
    ri, ci = linear_sum_assignment(C)
    r = orc.solve(p, eps_rel=1e-10, max_iter=500000)
    assert r.status == "OPTIMAL"
    assert r.info["primal_obj"] == pytest.approx(C[ri, ci].sum(), rel=1e-8)


@pytest.mark.parametrize("seed", range(4))
def test_mixed_lp_matches_certificate_and_highs(orc, seed):
    p = lpgen.mixed_lp(seed)
    r = orc.solve(p, eps_rel=1e-9, max_iter=500000)
    assert r.status == "OPTIMAL"
    assert r.info["primal_obj"] == pytest.approx(p.obj_star(), rel=1e-7, abs=1e-7)
    assert r.info["primal_obj"] == pytest.approx(exact.highs_optimum(p), rel=1e-7, abs=1e-7)
    # the returned point passes the independent evaluator
    e = orc.evaluate(p, r.x, r.y)
    assert e["rel_kkt"] <= 1e-9 * 1.0001
    assert np.all(r.x >= p.l - 1e-12 * (1 + np.abs(p.l[np.isfinite(p.l)]).max()))
    assert np.all(r.y[p.row_type == lpgen.ROW_GE] >= 0) and np.all(r.y[p.row_type == lpgen.ROW_LE] <= 0)


def test_transportation_matches_highs(orc):
    p = lpgen.transportation(2, 25, 30)
    r = orc.solve(p, eps_rel=1e-9, max_iter=500000)
    assert r.status == "OPTIMAL"
    assert r.info["primal_obj"] == pytest.approx(exact.highs_optimum(p), rel=1e-7)


@pytest.mark.parametrize("eps", [1e-4, 1e-8])
def test_config0_reaches_known_optimum(orc, eps):
    p = lpgen.config0(0)
    r = orc.solve(p, eps_rel=eps)
    assert r.status == "OPTIMAL" and r.info["rel_kkt"] <= eps
    tol = 1e-3 if eps > 1e-6 else 1e-7
    assert abs(r.info["primal_obj"] - p.obj_star()) <= tol * (1 + abs(p.obj_star()))


def test_fp32_matrix_mode_reaches_1e4(orc):
    """FP32-rounded scaled matrix in the steps, FP64 everywhere else: the
    evaluation uses the FP64 matrix, so rel KKT 1e-4 is on the true LP."""
    p = lpgen.config0(1)
    r = orc.solve(p, eps_rel=1e-4, a_precision=1)
    assert r.status == "OPTIMAL"
    e = orc.evaluate(p, r.x, r.y)
    assert e["rel_kkt"] <= 1e-4 * 1.0001
    assert abs(r.info["primal_obj"] - p.obj_star()) <= 1e-3 * (1 + abs(p.obj_star()))


# ----------------------------------------------------------------------------- invariances

def test_le_row_equals_negated_ge_row(orc):
    """An LE row a x <= b and the GE row (-a) x >= -b are the same constraint:
    the trajectory is identical and the returned dual changes sign."""
    p = lpgen.config0(4)
    q = lpgen.Problem(**{f: getattr(p, f) for f in ("m", "n", "row_ptr", "col_idx", "c", "l", "u")},
                      val=p.val.copy(), b=p.b.copy(), row_type=p.row_type.copy())
    le = p.row_type == lpgen.ROW_LE
    rows = np.repeat(np.arange(p.m), np.diff(p.row_ptr))
    q.val[le[rows]] *= -1
    q.b[le] *= -1
    q.row_type[le] = lpgen.ROW_GE
    r1 = orc.solve(p, max_iter=300)
    r2 = orc.solve(q, max_iter=300)
    np.testing.assert_array_equal(r1.x_hat, r2.x_hat)
    np.testing.assert_array_equal(r1.y_hat, r2.y_hat)
    np.testing.assert_array_equal(r1.y[le], -r2.y[le])


def test_permutation_equivariance(orc):
    """Renumbering rows and columns renumbers the iterates (up to the
    rounding of reordered sums)."""
    p = lpgen.config0(5)
    rng = np.random.default_rng(0)
    rp, cp = rng.permutation(p.m), rng.permutation(p.n)
    q = lpgen.permute(p, rp, cp)
    r1 = orc.solve(p, max_iter=100)
    r2 = orc.solve(q, max_iter=100)
    assert r1.info["restarts"] == r2.info["restarts"] and r1.info["attempts"] == r2.info["attempts"]
    # norm-wise: ||a - b||_inf / max(1, ||b||_inf), the trajectory metric of the parity tests
    assert np.abs(r2.x_hat - r1.x_hat[cp]).max() / max(1, np.abs(r1.x_hat).max()) <= 1e-11
    assert np.abs(r2.y_hat - r1.y_hat[rp]).max() / max(1, np.abs(r1.y_hat).max()) <= 1e-11


def test_thread_count_does_not_change_results(orc):
    p = lpgen.config0(6)
    r1 = orc.solve(p, max_iter=200, threads=1)
    r2 = orc.solve(p, max_iter=200, threads=4)
    np.testing.assert_array_equal(r1.x_hat, r2.x_hat)
    np.testing.assert_array_equal(r1.y_hat, r2.y_hat)


def test_zero_start_optimal_terminates_immediately(orc):
    """If the start proj_X(0), y = 0 already satisfies the tests, no step is taken."""
    p = lpgen.from_dense([[1.0, 1.0]], [1.0, 2.0], [0.0], [0.0, 0.0], [5.0, 5.0], [lpgen.ROW_GE])
    r = orc.solve(p, eps_rel=1e-8)
    assert r.status == "OPTIMAL" and r.info["iterations"] == 0
