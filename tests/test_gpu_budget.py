"""Step budgets (max_iter) across the attempt-slot boundaries of the device loop.

A solve launches full graphs (rounds of P + max(2, P/8) attempt slots, each
round closed by an evaluation) while the step budget left after the graphs in
flight reaches a full graph's steps, then short graphs of 8 attempt slots and
an evaluation.  The launch pattern must not touch the arithmetic (Algorithm 1
with the adaptive steps of Algorithm 2 and evaluations every P accepted steps,
Section 3.4): a solve with max_iter = b stops after exactly b accepted steps,
with the iterate, attempt and evaluation counts of the same solve launched
eagerly (graph = 0: whole rounds only, no short graph), bitwise, and the
oracle's attempt count.  A resumed solve (a second pdlp_solve after
pdlp_set_termination) counts its budget from where the first one stopped.
"""
import numpy as np
import pytest

import lpgen

pytestmark = pytest.mark.gpu

# 1 and 7: inside one short graph; 8 and 9: its end and one past it; 63, 64,
# 65: around one full graph's steps (P = 64); 137: two full graphs and a tail
BUDGETS = [1, 7, 8, 9, 20, 63, 64, 65, 100, 137]


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    from paper_2311_12180_amd import pdlp
    pdlp.lib()
    return pdlp


@pytest.fixture(scope="module")
def lp():
    return lpgen.config0(0)


def _run(P, p, budgets, graph, **opts):
    """Solves of p on one handle, one per entry of budgets (the first from the
    default start, the others resumed), with graphs or eager launches."""
    h = P.pdlp_create(p, eps_rel=0.0, max_iter=budgets[0], graph=graph, time_limit_s=60.0, **opts)
    out = []
    try:
        for i, b in enumerate(budgets):
            if i:
                P.pdlp_set_termination(h, 0.0, b, 60.0)
            P.pdlp_solve(h)
            x, y, st = P.pdlp_get_iterate(h)
            info = P.pdlp_get_solution(h)[3]
            out.append((x, y, st, info))
    finally:
        P.pdlp_destroy(h)
    return out


@pytest.mark.parametrize("b", BUDGETS)
def test_budget_is_exact_and_graphs_match_eager(P, orc, lp, b):
    (xg, yg, sg, ig), = _run(P, lp, [b], graph=1)
    (xe, ye, se, ie), = _run(P, lp, [b], graph=0)
    print(f"budget {b}: iterations {ig['iterations']}, attempts {ig['attempts']}, evaluations {ig['evaluations']}")
    assert ig["status_name"] == "ITER_LIMIT" and ig["iterations"] == b
    assert ie["status_name"] == "ITER_LIMIT" and ie["iterations"] == b
    for key in ("attempts", "evaluations", "restarts"):
        assert ig[key] == ie[key], key
    np.testing.assert_array_equal(xg, xe)
    np.testing.assert_array_equal(yg, ye)
    assert sg == se
    if b <= 100:   # the oracle's decisions are pinned step by step over the first 100 steps
        r = orc.solve(lp, eps_rel=0.0, max_iter=b)
        assert ig["attempts"] == r.info["attempts"]


@pytest.mark.parametrize("budgets", [[5, 20], [9, 64], [64, 65], [1, 1, 7]])
def test_resumed_budgets(P, lp, budgets):
    gr = _run(P, lp, budgets, graph=1)
    ea = _run(P, lp, budgets, graph=0)
    for b, (xg, yg, sg, ig), (xe, ye, se, ie) in zip(budgets, gr, ea):
        assert ig["iterations"] == b and ie["iterations"] == b
        assert ig["attempts"] == ie["attempts"]
        np.testing.assert_array_equal(xg, xe)
        np.testing.assert_array_equal(yg, ye)
        assert sg == se


@pytest.mark.parametrize("b", [9, 65, 137])
def test_budget_on_staged_and_sell_layouts(P, b):
    """The same on the LDS-staged dual step and the SELL-64 primal step (three
    staged column panels), layouts pinned so both handles sum in one order."""
    p = lpgen.skewed_lp(3, m=20000, n=40000, nnz_target=400000, cap=8000)
    opts = dict(spmv_layout=35, spmv_layout_kt=64, row_order=2)
    (xg, yg, sg, ig), = _run(P, p, [b], graph=1, **opts)
    (xe, ye, se, ie), = _run(P, p, [b], graph=0, **opts)
    assert (ig["layout_k"], ig["layout_kt"]) == (35, 64)
    assert ig["iterations"] == b and ie["iterations"] == b
    assert ig["attempts"] == ie["attempts"]
    np.testing.assert_array_equal(xg, xe)
    np.testing.assert_array_equal(yg, ye)
    assert sg == se
