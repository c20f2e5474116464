"""Pins of the normalized duality gap (restart_metric = 1, PDLP's restart
metric that Section 3.4 says the KKT error replaces) in the oracle.

rho_r(z) = max { L(x, yh) - L(xh, y) : zh in Z, ||zh - z||_omega <= r } / r
is pinned against: its closed form when no bound binds (the dual norm of the
gradient), its closed form when only the box binds, a brute-force grid search
over a two-variable box-and-ball, a brute-force enumeration of every active set
of the box-and-ball problem on tiny LPs (exact, to rounding), zero at a saddle
point, and the monotonicity of r rho_r in r.  The restart scheme that uses it converges to the known
optimum.
"""
import numpy as np
import pytest

import lpgen
import oracle

INF = np.inf


def _gap(p, x, y, w, r):
    # no scaling (0 Ruiz passes, no Pock-Chambolle pass): the point is in the user's >=-form space
    return oracle.normalized_gap(p, x, y, w, r, ruiz_iters=0, pc_alpha=-1.0)


def test_no_bound_binds_gives_the_dual_norm():
    rng = np.random.default_rng(0)
    m, n = 4, 6
    A = rng.standard_normal((m, n)); b = rng.standard_normal(m); c = rng.standard_normal(n)
    p = lpgen.from_dense(A, c, b, [-INF] * n, [INF] * n, [0] * m)
    x = rng.standard_normal(n); y = rng.standard_normal(m)
    gx, gy = A.T @ y - c, b - A @ x
    for w, r in ((1.0, 0.5), (3.0, 0.01), (0.2, 7.0)):
        ref = np.sqrt(np.sum(gx ** 2) / w + w * np.sum(gy ** 2))
        assert _gap(p, x, y, w, r) == pytest.approx(ref, rel=1e-12)


def test_box_binds_before_the_ball():
    rng = np.random.default_rng(1)
    n = 7
    c = rng.standard_normal(n); x = rng.standard_normal(n)
    l, u = x - rng.uniform(0, 0.1, n), x + rng.uniform(0, 0.1, n)
    p = lpgen.from_dense(np.zeros((0, n)), c, np.zeros(0), l, u, [])
    r = 100.0
    box = np.sum(np.maximum(-c * (u - x), -c * (l - x)))
    assert _gap(p, x, np.zeros(0), 1.3, r) == pytest.approx(box / r, rel=1e-12)


@pytest.mark.parametrize("w,r", [(1.0, 0.3), (2.5, 0.4), (0.3, 1.0), (1.0, 5.0)])
def test_two_variables_against_a_grid(w, r):
    c = np.array([1.0, -2.0]); x = np.array([0.5, 0.2]); l = np.array([0.0, -1.0]); u = np.array([1.0, 0.5])
    p = lpgen.from_dense(np.zeros((0, 2)), c, np.zeros(0), l, u, [])
    rho = _gap(p, x, np.zeros(0), w, r)
    dx = np.linspace(l[0] - x[0], u[0] - x[0], 2001)
    dy = np.linspace(l[1] - x[1], u[1] - x[1], 2001)
    DX, DY = np.meshgrid(dx, dy)
    val = np.where(w * (DX ** 2 + DY ** 2) <= r * r, -c[0] * DX - c[1] * DY, -np.inf).max() / r
    # the grid under-estimates by at most its spacing times the gradient
    assert val - 1e-12 <= rho <= val + 2e-3


def _active_set_max(g, w, lo, hi, r):
    """max g'd over {lo <= d <= hi, sum w d^2 <= r^2} by brute force over the
    KKT forms of the maximiser: every coordinate is at its lower bound, at its
    upper bound, or free with d_j = s g_j / w_j for one common s > 0 fixed by
    the ball; the best feasible candidate is the maximum (tiny n only)."""
    import itertools
    best = -np.inf
    for pat in itertools.product((0, 1, 2), repeat=len(g)):
        d = np.zeros(len(g))
        free = [j for j, k in enumerate(pat) if k == 2]
        for j, k in enumerate(pat):
            if k < 2:
                d[j] = lo[j] if k == 0 else hi[j]
        if not np.all(np.isfinite(d)):
            continue
        if free:
            a = np.array([g[j] / w[j] for j in free])
            rest = r * r - np.sum(w * d * d)
            A = np.sum(np.array([w[j] for j in free]) * a * a)
            if rest < 0 or A == 0:
                continue
            s = np.sqrt(rest / A)
            d[free] = s * a
        if np.all(d >= lo - 1e-12) and np.all(d <= hi + 1e-12) and np.sum(w * d * d) <= r * r * (1 + 1e-12):
            best = max(best, float(g @ d))
    return best


@pytest.mark.parametrize("seed", range(12))
def test_exact_against_active_set_enumeration(seed):
    """rho_r equals the brute-force maximum over every active set of the
    box-and-ball problem to rounding, on tiny LPs whose rows and columns mix
    every bound type (so the ball binds, the box binds, or both)."""
    rng = np.random.default_rng(100 + seed)
    m, n = 2, 3
    A = rng.standard_normal((m, n)); b = rng.standard_normal(m); c = rng.standard_normal(n)
    l = np.where(rng.random(n) < 0.8, -rng.uniform(0, 1, n), -INF)
    u = np.where(rng.random(n) < 0.8, rng.uniform(0, 1, n), INF)
    rt = rng.integers(0, 2, m)                    # EQ or GE rows
    p = lpgen.from_dense(A, c, b, l, u, rt)
    x = np.clip(rng.uniform(-0.5, 0.5, n), l, u)
    y = np.where(rt == 1, np.abs(rng.standard_normal(m)), rng.standard_normal(m))
    w = float(rng.uniform(0.3, 3.0))
    gx, gy = A.T @ y - c, b - A @ x
    g = np.concatenate([gx, gy])
    wt = np.concatenate([np.full(n, w), np.full(m, 1.0 / w)])
    lo = np.concatenate([l - x, np.where(rt == 1, -y, -INF)])
    hi = np.concatenate([u - x, np.full(m, INF)])
    for r in (0.05, 0.4, 2.0, 50.0):
        ref = _active_set_max(g, wt, lo, hi, r) / r
        assert _gap(p, x, y, w, r) == pytest.approx(ref, rel=1e-12, abs=1e-15)


def test_zero_at_a_saddle_point_and_monotone_in_r():
    p = lpgen.tiny_dense_lp(3)
    s = oracle.solve(p, eps_rel=1e-12, max_iter=2_000_000, ruiz_iters=0, pc_alpha=-1.0)
    assert s.status == "OPTIMAL"
    # x_hat, y_hat are the final iterate in the >=-form space (unscaled here)
    vals = [_gap(p, s.x_hat, s.y_hat, 1.0, r) for r in (1e-3, 1e-1, 1.0, 10.0)]
    assert max(vals) <= 1e-9, vals
    rng = np.random.default_rng(2)
    x = rng.standard_normal(p.n); y = np.abs(rng.standard_normal(p.m))
    rs = [0.01, 0.1, 0.5, 1.0, 3.0]
    g = [r * _gap(p, x, y, 1.7, r) for r in rs]
    assert all(v >= -1e-12 for v in g)
    assert all(b >= a - 1e-12 for a, b in zip(g, g[1:])), g


@pytest.mark.parametrize("make", [lambda: lpgen.batch_lp(0, 0, 300), lambda: lpgen.mixed_lp(1),
                                  lambda: lpgen.transportation(1, 30, 40)])
def test_gap_restarts_reach_the_optimum(make):
    p = make()
    r = oracle.solve(p, eps_rel=1e-8, max_iter=1_000_000, restart_metric=1, trace_cap=100000)
    assert r.status == "OPTIMAL"
    e = oracle.evaluate(p, r.x, r.y)
    assert e["rel_kkt"] <= 1e-8
    ref = p.obj_star()
    if ref is not None:
        assert abs(e["primal_obj"] - ref) <= 1e-6 * (1 + abs(ref))
    assert (r.trace["ev_kkt_cur"] >= 0).all() and (r.trace["ev_kkt_avg"] >= 0).all()
    assert r.info["restarts"] >= 1
