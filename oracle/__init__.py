"""ctypes front end of the plain CPU FP64 restarted-PDHG oracle.

TEST INFRASTRUCTURE ONLY.  This package is the yardstick the HIP solver is
checked against.  Only the tests, ``__graft_entry__.smoke()`` and the CPU
baseline leg of ``bench.py`` may import it; the solver library never does.
It shares no code with the GPU path.

Functions follow the paper (arXiv 2311.12180): ``solve`` runs Algorithm 1 with
Algorithm 2 steps, eq. (kkt) restarts and the Section 4.1 termination test;
``rescale`` is the Section 2.2 preconditioning; ``pdhg_step`` is eq. (pdhg);
``evaluate`` returns the Section 4.1 termination quantities; ``restart_reason``
and ``primal_weight_update`` are the Section 3.4 / 2.2 rules.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pdlp_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

STATUS = {0: "NONE", 1: "OPTIMAL", 2: "ITER_LIMIT", 3: "TIME_LIMIT", 4: "NUMERICAL_ERROR",
          5: "PRIMAL_INFEASIBLE", 6: "DUAL_INFEASIBLE"}


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain -O2, OpenMP, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
                               "-std=c11", "-D_POSIX_C_SOURCE=200809L", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Problem(C.Structure):
    _fields_ = [("m", C.c_int32), ("n", C.c_int32), ("nnz", C.c_int64),
                ("row_ptr", C.c_void_p), ("col_idx", C.c_void_p), ("val", C.c_void_p),
                ("c", C.c_void_p), ("b", C.c_void_p), ("l", C.c_void_p), ("u", C.c_void_p),
                ("row_type", C.c_void_p)]


class _Options(C.Structure):
    _fields_ = [("eps_rel", C.c_double), ("max_iter", C.c_int64), ("time_limit_s", C.c_double),
                ("eval_period", C.c_int32), ("ruiz_iters", C.c_int32), ("pc_alpha", C.c_double),
                ("pw_theta", C.c_double), ("eps_zero", C.c_double), ("beta_suff", C.c_double),
                ("beta_nec", C.c_double), ("beta_art", C.c_double), ("a_precision", C.c_int32),
                ("kkt_omega_power", C.c_int32), ("threads", C.c_int32), ("detect_infeas", C.c_int32),
                ("eps_infeas", C.c_double), ("infeas_every", C.c_int32), ("restart_metric", C.c_int32)]


class _Info(C.Structure):
    _fields_ = [("status", C.c_int32), ("returned_avg", C.c_int32), ("iterations", C.c_int64),
                ("attempts", C.c_int64), ("restarts", C.c_int64), ("evaluations", C.c_int64),
                ("rel_kkt", C.c_double), ("rel_gap", C.c_double), ("rel_pres", C.c_double),
                ("rel_dres", C.c_double), ("primal_obj", C.c_double), ("dual_obj", C.c_double),
                ("omega", C.c_double), ("eta_hat", C.c_double), ("sum_eta", C.c_double),
                ("kkt0", C.c_double), ("setup_s", C.c_double), ("solve_s", C.c_double),
                ("threads_used", C.c_int32), ("ray_source", C.c_int32), ("ray_obj", C.c_double),
                ("ray_res", C.c_double)]


class _Trace(C.Structure):
    _fields_ = [("cap_att", C.c_int64), ("n_att", C.c_int64), ("att_k", C.c_void_p),
                ("att_eta", C.c_void_p), ("att_etabar", C.c_void_p), ("att_acc", C.c_void_p),
                ("cap_eval", C.c_int64), ("n_eval", C.c_int64), ("ev_k", C.c_void_p),
                ("ev_kkt_cur", C.c_void_p), ("ev_kkt_avg", C.c_void_p), ("ev_cand", C.c_void_p),
                ("ev_reason", C.c_void_p), ("ev_omega", C.c_void_p)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(_LIB)
        L.orc_solve.argtypes = [C.POINTER(_Problem), C.POINTER(_Options), C.c_void_p, C.c_void_p,
                                C.c_void_p, C.POINTER(_Info), C.c_void_p, C.c_void_p, C.c_void_p]
        L.orc_rescale.argtypes = [C.POINTER(_Problem), C.c_int32, C.c_double, C.c_void_p,
                                  C.c_void_p, C.c_void_p]
        L.orc_pdhg_step.argtypes = [C.c_int32, C.c_int32] + [C.c_void_p] * 10 + [C.c_double, C.c_double,
                                                                                C.c_void_p, C.c_void_p]
        L.orc_evaluate.argtypes = [C.POINTER(_Problem), C.c_void_p, C.c_void_p, C.c_double,
                                   C.c_int32, C.c_void_p]
        L.orc_reduced_costs.argtypes = [C.POINTER(_Problem), C.c_void_p, C.c_void_p]
        L.orc_ray_test.argtypes = [C.POINTER(_Problem), C.c_void_p, C.c_void_p, C.c_double, C.c_void_p,
                                   C.c_void_p, C.c_void_p, C.c_void_p]
        L.orc_ray_test.restype = C.c_int
        L.orc_normalized_gap.argtypes = [C.POINTER(_Problem), C.c_int32, C.c_double, C.c_void_p, C.c_void_p,
                                         C.c_double, C.c_double]
        L.orc_normalized_gap.restype = C.c_double
        L.orc_restart_reason.argtypes = [C.c_double, C.c_double, C.c_double, C.c_int64, C.c_int64,
                                         C.c_double, C.c_double, C.c_double]
        L.orc_restart_reason.restype = C.c_int
        L.orc_primal_weight_update.argtypes = [C.c_double] * 5
        L.orc_primal_weight_update.restype = C.c_double
        L.orc_default_options.argtypes = [C.POINTER(_Options)]
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data if a is not None and a.size else None


class _Held:
    """Keeps the contiguous arrays alive while the C structure points at them."""

    def __init__(self, prob):
        self.row_ptr = np.ascontiguousarray(prob.row_ptr, dtype=np.int32)
        self.col_idx = np.ascontiguousarray(prob.col_idx, dtype=np.int32)
        self.val = np.ascontiguousarray(prob.val, dtype=np.float64)
        self.c = np.ascontiguousarray(prob.c, dtype=np.float64)
        self.b = np.ascontiguousarray(prob.b, dtype=np.float64)
        self.l = np.ascontiguousarray(prob.l, dtype=np.float64)
        self.u = np.ascontiguousarray(prob.u, dtype=np.float64)
        self.row_type = np.ascontiguousarray(prob.row_type, dtype=np.int8)
        self.s = _Problem(int(prob.m), int(prob.n), int(self.row_ptr[-1]), _p(self.row_ptr),
                          _p(self.col_idx), _p(self.val), _p(self.c), _p(self.b), _p(self.l),
                          _p(self.u), _p(self.row_type))


def default_options(**kw) -> _Options:
    o = _Options()
    lib().orc_default_options(C.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


@dataclasses.dataclass
class Result:
    x: np.ndarray
    y: np.ndarray
    rc: np.ndarray
    x_hat: np.ndarray
    y_hat: np.ndarray
    status: str
    info: dict
    trace: Optional[dict] = None


def solve(prob, trace_cap: int = 0, **opts) -> Result:
    """Solve with the oracle.  Options: eps_rel, max_iter, time_limit_s,
    eval_period, ruiz_iters, pc_alpha, pw_theta, eps_zero, beta_suff, beta_nec,
    beta_art, a_precision, kkt_omega_power, threads, detect_infeas, eps_infeas,
    infeas_every, restart_metric.
    Status PRIMAL_INFEASIBLE returns a unit dual ray in y (and its multipliers
    in rc), DUAL_INFEASIBLE a unit primal ray in x."""
    h = _Held(prob)
    o = default_options(**opts)
    m, n = int(prob.m), int(prob.n)
    x = np.zeros(n); y = np.zeros(m); rc = np.zeros(n)
    xh = np.zeros(n); yh = np.zeros(m)
    info = _Info()
    tr = None
    tarr = None
    if trace_cap > 0:
        tarr = dict(att_k=np.zeros(trace_cap, np.int64), att_eta=np.zeros(trace_cap),
                    att_etabar=np.zeros(trace_cap), att_acc=np.zeros(trace_cap, np.int8),
                    ev_k=np.zeros(trace_cap, np.int64), ev_kkt_cur=np.zeros(trace_cap),
                    ev_kkt_avg=np.zeros(trace_cap), ev_cand=np.zeros(trace_cap, np.int8),
                    ev_reason=np.zeros(trace_cap, np.int8), ev_omega=np.zeros(trace_cap))
        tr = _Trace(trace_cap, 0, _p(tarr["att_k"]), _p(tarr["att_eta"]), _p(tarr["att_etabar"]),
                    _p(tarr["att_acc"]), trace_cap, 0, _p(tarr["ev_k"]), _p(tarr["ev_kkt_cur"]),
                    _p(tarr["ev_kkt_avg"]), _p(tarr["ev_cand"]), _p(tarr["ev_reason"]),
                    _p(tarr["ev_omega"]))
    rcode = lib().orc_solve(C.byref(h.s), C.byref(o), _p(x), _p(y), _p(rc), C.byref(info),
                            C.addressof(tr) if tr is not None else None, _p(xh), _p(yh))
    if rcode != 0:
        raise ValueError("oracle rejected the problem")
    d = {f: getattr(info, f) for f, _ in _Info._fields_}
    trace = None
    if tr is not None:
        na, ne = tr.n_att, tr.n_eval
        trace = {k: v[:na] for k, v in tarr.items() if k.startswith("att")}
        trace.update({k: v[:ne] for k, v in tarr.items() if k.startswith("ev")})
    return Result(x, y, rc, xh, yh, STATUS.get(info.status, str(info.status)), d, trace)


def rescale(prob, ruiz_iters: int = 10, pc_alpha: float = 1.0):
    """D1[m], D2[n] and the scaled >=-form values (LE rows negated)."""
    h = _Held(prob)
    D1 = np.zeros(prob.m); D2 = np.zeros(prob.n); vs = np.zeros(len(h.val))
    if lib().orc_rescale(C.byref(h.s), ruiz_iters, pc_alpha, _p(D1), _p(D2), _p(vs)) != 0:
        raise ValueError("bad problem")
    return D1, D2, vs


def pdhg_step(row_ptr, col_idx, val, q, c, l, u, ineq, x, y, tau, sigma):
    """eq. (pdhg) on a >=-form LP; returns (x', y')."""
    m, n = len(q), len(c)
    arrs = [np.ascontiguousarray(a, dtype=dt) for a, dt in
            ((row_ptr, np.int32), (col_idx, np.int32), (val, np.float64), (q, np.float64),
             (c, np.float64), (l, np.float64), (u, np.float64), (ineq, np.int8), (x, np.float64),
             (y, np.float64))]
    xo = np.zeros(n); yo = np.zeros(m)
    lib().orc_pdhg_step(m, n, *[_p(a) for a in arrs], float(tau), float(sigma), _p(xo), _p(yo))
    return xo, yo


def evaluate(prob, x, y, omega: float = 1.0, omega_power: int = 2) -> dict:
    """Section 4.1 quantities on the user-orientation LP at (x, y)."""
    h = _Held(prob)
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.ascontiguousarray(y, dtype=np.float64)
    out = np.zeros(10)
    if lib().orc_evaluate(C.byref(h.s), _p(x), _p(y), float(omega), int(omega_power), _p(out)) != 0:
        raise ValueError("bad problem")
    keys = ["rel_kkt", "rel_gap", "rel_pres", "rel_dres", "primal_obj", "dual_obj",
            "pres", "dres", "gap", "kkt_omega"]
    return dict(zip(keys, out.tolist()))


def ray_test(prob, x_dir, y_dir, eps: float = 1e-8) -> dict:
    """Farkas test of a candidate direction (user orientation): verdict 1 =
    y certifies primal infeasibility, 2 = x certifies dual infeasibility,
    0 = neither; the ray quantities after projection; the projected rays."""
    h = _Held(prob)
    xd = np.ascontiguousarray(x_dir, dtype=np.float64)
    yd = np.ascontiguousarray(y_dir, dtype=np.float64)
    out = np.zeros(8)
    rx = np.zeros(prob.n); ry = np.zeros(prob.m); lam = np.zeros(prob.n)
    v = lib().orc_ray_test(C.byref(h.s), _p(xd), _p(yd), float(eps), _p(out), _p(rx), _p(ry), _p(lam))
    if v < 0:
        raise ValueError("bad problem")
    keys = ["dual_ray_obj", "dual_ray_res", "y_norm", "primal_ray_obj", "primal_ray_res", "x_norm",
            "dual_ray_obj_abs", "primal_ray_obj_abs"]
    d = dict(zip(keys, out.tolist()))
    d.update(verdict=int(v), ray_x=rx, ray_y=ry, lam=lam)
    return d


def normalized_gap(prob, x_scaled, y_scaled, omega: float, r: float, ruiz_iters: int = 10,
                   pc_alpha: float = 1.0) -> float:
    """rho_r of the scaled LP at a scaled point (x~, y~ in the >=-form space)."""
    h = _Held(prob)
    xs = np.ascontiguousarray(x_scaled, dtype=np.float64)
    ys = np.ascontiguousarray(y_scaled, dtype=np.float64)
    v = lib().orc_normalized_gap(C.byref(h.s), ruiz_iters, pc_alpha, _p(xs), _p(ys), float(omega), float(r))
    if v < 0:
        raise ValueError("bad problem")
    return v


def reduced_costs(prob, y) -> np.ndarray:
    h = _Held(prob)
    y = np.ascontiguousarray(y, dtype=np.float64)
    lam = np.zeros(prob.n)
    lib().orc_reduced_costs(C.byref(h.s), _p(y), _p(lam))
    return lam


def restart_reason(kkt_cand, kkt0, kkt_prev, t, k, beta_suff=0.2, beta_nec=0.8, beta_art=0.36) -> int:
    return int(lib().orc_restart_reason(kkt_cand, kkt0, kkt_prev, t, k, beta_suff, beta_nec, beta_art))


def primal_weight_update(dx, dy, omega, theta=0.5, eps_zero=1e-10) -> float:
    return float(lib().orc_primal_weight_update(dx, dy, omega, theta, eps_zero))
