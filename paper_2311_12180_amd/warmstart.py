"""Learned warm start: the pipeline around the network (include/pdlp_gnn.h).

  1. solve a family of LPs cold with the batched solver -> targets (x*, y*,
     final primal weight);
  2. train the network on a training part of the family (GPU kernels: forward,
     backward, Adam);
  3. predict (x0, y0, omega0) for held-out LPs and solve them from there; an
     LP whose warm solve does not end OPTIMAL is solved again cold (the cold
     solver is the fallback, and its termination test decides every prediction).

Only the C ABI is used; every numerical step runs in the HIP library."""
from __future__ import annotations

import time
from typing import Optional, Sequence

import numpy as np

from . import gnn as _G
from . import pdlp as _P


def canonical_transport_duals(y: np.ndarray, S: int) -> np.ndarray:
    """A transportation LP's duals are determined up to (u + s, v - s) for
    supply duals u (rows 0..S-1) and demand duals v; pick the s that gives
    both groups the same mean."""
    u, v = y[:S], y[S:]
    s = 0.5 * (v.mean() - u.mean())
    return np.concatenate([u + s, v - s])


def solve_batch(problems: Sequence, eps: float, stream=None, warm=None, time_limit_s: float = 600.0, **opts):
    """Solve LPs in one batched launch; warm = (x0 list, y0 list, omega0 array)
    or None.  Returns (xs, ys, infos, wall seconds of the solve)."""
    h = _P.pdlp_create_batch(list(problems), stream=stream, eps_rel=eps, max_iter=200000,
                             time_limit_s=time_limit_s, **opts)
    try:
        if warm is not None:
            x0, y0, om = warm
            for k in range(len(problems)):
                _P.pdlp_set_warm_start_batch(h, k, x0[k], y0[k], float(om[k]))
        t = time.perf_counter()
        _P.pdlp_solve_batch(h)
        dt = time.perf_counter() - t
        x, y, _, infos = _P.pdlp_get_solution_batch(h, -1)
        xs = [x[h.col_off[k]:h.col_off[k + 1]] for k in range(h.count)]
        ys = [y[h.row_off[k]:h.row_off[k + 1]] for k in range(h.count)]
    finally:
        _P.pdlp_destroy(h)
    return xs, ys, infos, dt


def balance_weights(x_t: Sequence[np.ndarray], y_t: Sequence[np.ndarray], log_omega: np.ndarray):
    """Loss weights that give each term unit scale on the training targets:
    1 / mean square of the scaled x and y targets, 1 / variance of log omega."""
    mx = float(np.mean(np.concatenate([np.asarray(v) ** 2 for v in x_t])))
    my = float(np.mean(np.concatenate([np.asarray(v) ** 2 for v in y_t]))) if len(y_t) else 1.0
    vo = float(np.var(log_omega))
    return (1.0 / mx if mx > 0 else 1.0, 1.0 / my if my > 0 else 1.0, 1.0 / vo if vo > 0 else 1.0)


def train(gs: "_G.GraphSet", n_train: int, epochs: int, batch: int, lr: float, theta0: np.ndarray,
          seed: int = 0, log=None, weights=None):
    """Adam on LPs [0, n_train) of the graph set in mini-batches of `batch`
    consecutive LPs, visited in a shuffled order each epoch.  Returns the mean
    loss per epoch and the training wall time."""
    _G.pdlp_gnn_set_params(gs, theta0)
    if weights is not None:
        _G.pdlp_gnn_set_loss_weights(gs, *weights)
    rng = np.random.default_rng(seed)
    starts = np.arange(0, n_train - batch + 1, batch)
    losses = []
    t = time.perf_counter()
    for ep in range(epochs):
        tot = 0.0
        for s in rng.permutation(starts):
            tot += _G.pdlp_gnn_train_step(gs, int(s), batch, lr)
        losses.append(tot / len(starts))
        if log:
            log(f"epoch {ep}: loss {losses[-1]:.5f}")
    return losses, time.perf_counter() - t


def predict(gs: "_G.GraphSet", first: int, count: int):
    """Per-LP lists (x0, y0) and omega0 for LPs [first, first + count)."""
    x0, y0, om = _G.pdlp_gnn_predict(gs, first, count)
    cv = gs.col_off[first:first + count + 1] - gs.col_off[first]
    cr = gs.row_off[first:first + count + 1] - gs.row_off[first]
    return ([x0[cv[k]:cv[k + 1]] for k in range(count)], [y0[cr[k]:cr[k + 1]] for k in range(count)], om)


def warm_solve_with_fallback(problems: Sequence, eps: float, warm, stream=None, **opts):
    """Warm-started batched solve; LPs that do not end OPTIMAL are solved again
    cold.  Returns (infos, warm solve seconds, fallback seconds, fallback LP
    indices)."""
    xs, ys, infos, dt = solve_batch(problems, eps, stream, warm=warm, **opts)
    bad = [k for k, i in enumerate(infos) if i["status_name"] != "OPTIMAL"]
    dt_fb = 0.0
    if bad:
        _, _, inf2, dt_fb = solve_batch([problems[k] for k in bad], eps, stream, **opts)
        for k, i in zip(bad, inf2):
            infos[k] = i
    return infos, dt, dt_fb, bad
