"""Farkas' lemma checks of infeasibility certificates, written from the
definitions alone (no solver code): used on the oracle's and on the GPU's
certificates alike."""
import numpy as np

import lpgen


def check_dual_ray(p, y, lam, tol=1e-7):
    """Farkas certificate of primal infeasibility, checked from its definition."""
    A = p.to_scipy()
    y = np.asarray(y); lam = np.asarray(lam)
    # sign of y per row type (user orientation): GE >= 0, LE <= 0, EQ free
    assert np.all(y[p.row_type == lpgen.ROW_GE] >= -1e-14)
    assert np.all(y[p.row_type == lpgen.ROW_LE] <= 1e-14)
    # lam in Lambda: positive only at a finite lower bound, negative only at a finite upper bound
    assert np.all((lam <= 1e-14) | np.isfinite(p.l))
    assert np.all((lam >= -1e-14) | np.isfinite(p.u))
    lp = np.maximum(lam, 0.0); lm = np.maximum(-lam, 0.0)
    obj = p.b @ y + np.sum(p.l[lp > 0] * lp[lp > 0]) - np.sum(p.u[lm > 0] * lm[lm > 0])
    res = np.linalg.norm(A.T @ y + lam)
    assert obj > 0.0, obj
    assert res <= tol * obj, (res, obj)
    return obj, res


def check_primal_ray(p, x, tol=1e-7):
    """Certificate of dual infeasibility (an improving ray), from its definition."""
    A = p.to_scipy()
    x = np.asarray(x)
    fl, fu = np.isfinite(p.l), np.isfinite(p.u)
    assert np.all(x[fl & fu] == 0.0)
    assert np.all(x[fl] >= 0.0) and np.all(x[fu] <= 0.0)
    ax = A @ x
    obj = p.c @ x
    viol = np.where(p.row_type == lpgen.ROW_EQ, ax,
                    np.where(p.row_type == lpgen.ROW_GE, np.minimum(ax, 0.0), np.maximum(ax, 0.0)))
    assert obj < 0.0, obj
    assert np.linalg.norm(viol) <= tol * -obj, (np.linalg.norm(viol), obj)
    return obj
