"""Python binding of the C ABI in include/pdlp.h (argument marshalling only).

Every step of the solve runs in the HIP library libpdlp_hip.so built in-tree
for gfx950; this module only converts arguments.  Problems come as numpy
arrays (host) or torch ROCm tensors (device, copied on the current stream).
If the library is missing the import fails: there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpdlp_hip.so")

PDLP_ROW_EQ, PDLP_ROW_GE, PDLP_ROW_LE = 0, 1, 2
PDLP_MEM_HOST, PDLP_MEM_DEVICE = 0, 1
PDLP_A_FP64, PDLP_A_FP32 = 0, 1
PDLP_OPTIMAL, PDLP_ITER_LIMIT, PDLP_TIME_LIMIT, PDLP_NUMERICAL_ERROR = 1, 2, 3, 4
PDLP_PRIMAL_INFEASIBLE, PDLP_DUAL_INFEASIBLE = 5, 6
PDLP_OK, PDLP_ERR_ARG, PDLP_ERR_DATA, PDLP_ERR_HIP, PDLP_ERR_OOM, PDLP_ERR_STATE, PDLP_ERR_UNSUPPORTED = \
    0, -1, -2, -3, -4, -5, -6
STATUS = {0: "NONE", 1: "OPTIMAL", 2: "ITER_LIMIT", 3: "TIME_LIMIT", 4: "NUMERICAL_ERROR",
          5: "PRIMAL_INFEASIBLE", 6: "DUAL_INFEASIBLE"}
ERRORS = {-1: "PDLP_ERR_ARG", -2: "PDLP_ERR_DATA", -3: "PDLP_ERR_HIP", -4: "PDLP_ERR_OOM",
          -5: "PDLP_ERR_STATE", -6: "PDLP_ERR_UNSUPPORTED"}

EXPORTED = ["pdlp_default_options", "pdlp_create", "pdlp_set_warm_start", "pdlp_set_termination", "pdlp_solve",
            "pdlp_solve_noalloc",
            "pdlp_get_solution", "pdlp_get_iterate", "pdlp_get_scaling", "pdlp_get_trace",
            "pdlp_profile_attempts", "pdlp_step_bytes", "pdlp_create_batch", "pdlp_set_warm_start_batch",
            "pdlp_solve_batch", "pdlp_get_solution_batch", "pdlp_batch_schedule", "pdlp_presolve",
            "pdlp_last_error", "pdlp_destroy"]


class PdlpError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class pdlp_problem(C.Structure):
    _fields_ = [("m", C.c_int32), ("n", C.c_int32), ("nnz", C.c_int64), ("mem", C.c_int32),
                ("row_ptr", C.c_void_p), ("col_idx", C.c_void_p), ("val", C.c_void_p),
                ("c", C.c_void_p), ("b", C.c_void_p), ("l", C.c_void_p), ("u", C.c_void_p),
                ("row_type", C.c_void_p)]


class pdlp_options(C.Structure):
    _fields_ = [("eps_rel", C.c_double), ("max_iter", C.c_int64), ("time_limit_s", C.c_double),
                ("eval_period", C.c_int32), ("ruiz_iters", C.c_int32), ("pc_alpha", C.c_double),
                ("pw_theta", C.c_double), ("eps_zero", C.c_double), ("beta_suff", C.c_double),
                ("beta_nec", C.c_double), ("beta_art", C.c_double), ("a_precision", C.c_int32),
                ("kkt_omega_power", C.c_int32), ("trace", C.c_int32), ("poll_every", C.c_int32),
                ("graph", C.c_int32), ("spmv_layout", C.c_int32), ("batch_lanes", C.c_int32),
                ("batch_grid", C.c_int32), ("spmv_layout_kt", C.c_int32),
                ("batch_handoff", C.c_int32), ("handoff_streams", C.c_int32),
                ("detect_infeas", C.c_int32), ("eps_infeas", C.c_double), ("infeas_every", C.c_int32),
                ("presolve", C.c_int32), ("restart_metric", C.c_int32),
                ("row_order", C.c_int32)]


class pdlp_info(C.Structure):
    _fields_ = [("status", C.c_int32), ("returned_avg", C.c_int32), ("iterations", C.c_int64),
                ("attempts", C.c_int64), ("restarts", C.c_int64), ("evaluations", C.c_int64),
                ("rel_kkt", C.c_double), ("rel_gap", C.c_double), ("rel_pres", C.c_double),
                ("rel_dres", C.c_double), ("primal_obj", C.c_double), ("dual_obj", C.c_double),
                ("omega", C.c_double), ("eta_hat", C.c_double), ("setup_s", C.c_double),
                ("solve_s", C.c_double), ("layout_k", C.c_int32), ("layout_kt", C.c_int32),
                ("handoff_k", C.c_int64), ("ray_obj", C.c_double), ("ray_res", C.c_double),
                ("ray_source", C.c_int32), ("m_solved", C.c_int32), ("n_solved", C.c_int32),
                ("reserved", C.c_int32)]


class pdlp_iter_state(C.Structure):
    _fields_ = [("iterations", C.c_int64), ("attempts", C.c_int64), ("restarts", C.c_int64),
                ("evaluations", C.c_int64), ("eta_hat", C.c_double), ("omega", C.c_double),
                ("sum_eta", C.c_double), ("kkt0", C.c_double)]


_lib = None


def lib() -> C.CDLL:
    """Load libpdlp_hip.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_2311_12180_amd/build.py "
                              "(there is no CPU fallback)")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_double
        L.pdlp_default_options.argtypes = [C.POINTER(pdlp_options)]
        L.pdlp_create.argtypes = [C.POINTER(pdlp_problem), C.POINTER(pdlp_options), vp, C.POINTER(vp)]
        L.pdlp_set_warm_start.argtypes = [vp, vp, vp, dbl]
        L.pdlp_set_termination.argtypes = [vp, dbl, i64, dbl]
        L.pdlp_solve.argtypes = [vp]
        L.pdlp_solve_noalloc.argtypes = [vp]
        L.pdlp_get_solution.argtypes = [vp, vp, vp, vp, C.POINTER(pdlp_info)]
        L.pdlp_get_iterate.argtypes = [vp, vp, vp, C.POINTER(pdlp_iter_state)]
        L.pdlp_get_scaling.argtypes = [vp, vp, vp, vp]
        L.pdlp_get_trace.argtypes = [vp, i64, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
        L.pdlp_profile_attempts.argtypes = [vp, i32, C.POINTER(dbl), C.POINTER(dbl)]
        L.pdlp_step_bytes.argtypes = [vp, C.POINTER(dbl), C.POINTER(dbl)]
        L.pdlp_create_batch.argtypes = [C.POINTER(pdlp_problem), i32, C.POINTER(pdlp_options), vp, C.POINTER(vp)]
        L.pdlp_presolve.argtypes = [C.POINTER(pdlp_problem), C.POINTER(i32), vp, vp, vp, vp, vp, vp,
                                    C.POINTER(dbl)]
        L.pdlp_set_warm_start_batch.argtypes = [vp, i32, vp, vp, dbl]
        L.pdlp_solve_batch.argtypes = [vp]
        L.pdlp_get_solution_batch.argtypes = [vp, i32, vp, vp, vp, vp]
        L.pdlp_batch_schedule.argtypes = [vp, vp, vp]
        L.pdlp_last_error.argtypes = [vp]
        L.pdlp_last_error.restype = C.c_char_p
        L.pdlp_destroy.argtypes = [vp]
        L.pdlp_destroy.restype = None
        for name in EXPORTED:
            if name not in ("pdlp_last_error", "pdlp_destroy"):
                getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def _ptr(a):
    if a is None:
        return None
    if hasattr(a, "data_ptr"):
        return a.data_ptr() if a.numel() else None
    return a.ctypes.data if a.size else None


def pdlp_last_error(h=None) -> str:
    return lib().pdlp_last_error(h.ptr if isinstance(h, Handle) else h).decode()


def _check(rc: int, h=None):
    if rc != PDLP_OK:
        raise PdlpError(rc, pdlp_last_error(h))


def pdlp_default_options(**overrides) -> pdlp_options:
    o = pdlp_options()
    _check(lib().pdlp_default_options(C.byref(o)))
    for k, v in overrides.items():
        if not hasattr(o, k) or k.startswith("_"):
            raise KeyError(f"unknown option {k}")
        setattr(o, k, v)
    return o


class Handle:
    """Owns a pdlp_handle; destroyed explicitly or when garbage-collected."""

    def __init__(self, ptr: int, m: int, n: int, nnz: int, keep):
        self.ptr = ptr
        self.m, self.n, self.nnz = m, n, nnz
        self._keep = keep

    def __del__(self):
        try:
            pdlp_destroy(self)
        except Exception:
            pass


def _is_torch(a) -> bool:
    return hasattr(a, "data_ptr") and hasattr(a, "is_cuda")


def pdlp_create(problem, options: Optional[pdlp_options] = None, stream=None, **opts) -> Handle:
    """Create a handle for `problem` (attributes m, n, row_ptr, col_idx, val, c,
    b, l, u, row_type as numpy arrays, or torch device tensors)."""
    if options is None:
        options = pdlp_default_options(**opts)
    elif opts:
        raise ValueError("pass either options or keyword options")
    dev = _is_torch(problem.row_ptr) and problem.row_ptr.is_cuda
    if dev:
        import torch
        arrs = dict(row_ptr=problem.row_ptr.to(torch.int32).contiguous(),
                    col_idx=problem.col_idx.to(torch.int32).contiguous(),
                    val=problem.val.to(torch.float64).contiguous(),
                    c=problem.c.to(torch.float64).contiguous(), b=problem.b.to(torch.float64).contiguous(),
                    l=problem.l.to(torch.float64).contiguous(), u=problem.u.to(torch.float64).contiguous(),
                    row_type=problem.row_type.to(torch.int8).contiguous())
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        nnz = int(arrs["row_ptr"][-1].item()) if int(problem.m) >= 0 else 0
        mem = PDLP_MEM_DEVICE
    else:
        arrs = dict(row_ptr=np.ascontiguousarray(problem.row_ptr, dtype=np.int32),
                    col_idx=np.ascontiguousarray(problem.col_idx, dtype=np.int32),
                    val=np.ascontiguousarray(problem.val, dtype=np.float64),
                    c=np.ascontiguousarray(problem.c, dtype=np.float64),
                    b=np.ascontiguousarray(problem.b, dtype=np.float64),
                    l=np.ascontiguousarray(problem.l, dtype=np.float64),
                    u=np.ascontiguousarray(problem.u, dtype=np.float64),
                    row_type=np.ascontiguousarray(problem.row_type, dtype=np.int8))
        nnz = int(arrs["row_ptr"][-1]) if len(arrs["row_ptr"]) else 0
        mem = PDLP_MEM_HOST
    s = pdlp_problem(int(problem.m), int(problem.n), nnz, mem, *[_ptr(arrs[k]) for k in
                     ("row_ptr", "col_idx", "val", "c", "b", "l", "u", "row_type")])
    out = C.c_void_p()
    rc = lib().pdlp_create(C.byref(s), C.byref(options), C.c_void_p(stream) if stream else None, C.byref(out))
    _check(rc)
    return Handle(out.value, int(problem.m), int(problem.n), nnz, (arrs, options))


def _host_arrays(problem) -> dict:
    return dict(row_ptr=np.ascontiguousarray(problem.row_ptr, dtype=np.int32),
                col_idx=np.ascontiguousarray(problem.col_idx, dtype=np.int32),
                val=np.ascontiguousarray(problem.val, dtype=np.float64),
                c=np.ascontiguousarray(problem.c, dtype=np.float64),
                b=np.ascontiguousarray(problem.b, dtype=np.float64),
                l=np.ascontiguousarray(problem.l, dtype=np.float64),
                u=np.ascontiguousarray(problem.u, dtype=np.float64),
                row_type=np.ascontiguousarray(problem.row_type, dtype=np.int8))


class BatchHandle(Handle):
    """A pdlp_handle over several LPs; ms / ns / nnzs are the per-LP sizes."""

    def __init__(self, ptr: int, ms, ns, nnzs, keep):
        super().__init__(ptr, int(sum(ms)), int(sum(ns)), int(sum(nnzs)), keep)
        self.count = len(ms)
        self.ms = np.asarray(ms, np.int64)
        self.ns = np.asarray(ns, np.int64)
        self.row_off = np.concatenate([[0], np.cumsum(self.ms)])
        self.col_off = np.concatenate([[0], np.cumsum(self.ns)])


def pdlp_create_batch(problems, options: Optional[pdlp_options] = None, stream=None, **opts) -> BatchHandle:
    """Create a batch handle for a list of host problems (as for pdlp_create)."""
    if options is None:
        options = pdlp_default_options(**opts)
    elif opts:
        raise ValueError("pass either options or keyword options")
    arrs = [_host_arrays(p) for p in problems]
    structs = (pdlp_problem * max(len(arrs), 1))()
    for k, (p, a) in enumerate(zip(problems, arrs)):
        nnz = int(a["row_ptr"][-1]) if len(a["row_ptr"]) else 0
        structs[k] = pdlp_problem(int(p.m), int(p.n), nnz, PDLP_MEM_HOST, *[_ptr(a[key]) for key in
                                  ("row_ptr", "col_idx", "val", "c", "b", "l", "u", "row_type")])
    out = C.c_void_p()
    rc = lib().pdlp_create_batch(structs, len(arrs), C.byref(options), C.c_void_p(stream) if stream else None,
                                 C.byref(out))
    _check(rc)
    nnzs = [int(a["row_ptr"][-1]) for a in arrs]
    return BatchHandle(out.value, [int(p.m) for p in problems], [int(p.n) for p in problems], nnzs,
                       (arrs, structs, options))


def pdlp_set_warm_start_batch(h: BatchHandle, idx: int, x0=None, y0=None, omega0: float = 0.0):
    """Warm start of LP idx, or of all LPs (packed vectors) when idx = -1."""
    nx = h.n if idx < 0 else int(h.ns[idx])
    ny = h.m if idx < 0 else int(h.ms[idx])
    x0 = None if x0 is None else np.ascontiguousarray(x0, dtype=np.float64)
    y0 = None if y0 is None else np.ascontiguousarray(y0, dtype=np.float64)
    if x0 is not None and x0.shape != (nx,):
        raise ValueError(f"x0 must have {nx} entries")
    if y0 is not None and y0.shape != (ny,):
        raise ValueError(f"y0 must have {ny} entries")
    _check(lib().pdlp_set_warm_start_batch(h.ptr, int(idx), _ptr(x0), _ptr(y0), float(omega0)), h)


def pdlp_solve_batch(h: BatchHandle):
    _check(lib().pdlp_solve_batch(h.ptr), h)


def pdlp_get_solution_batch(h: BatchHandle, idx: int):
    """(x, y, reduced_cost, info) of LP idx; for idx = -1 the packed vectors of
    every LP and a list of info dicts."""
    nx = h.n if idx < 0 else int(h.ns[idx])
    ny = h.m if idx < 0 else int(h.ms[idx])
    x = np.zeros(nx); y = np.zeros(ny); rc = np.zeros(nx)
    cnt = h.count if idx < 0 else 1
    infos = (pdlp_info * cnt)()
    _check(lib().pdlp_get_solution_batch(h.ptr, int(idx), _ptr(x), _ptr(y), _ptr(rc), infos), h)
    if idx < 0:
        return x, y, rc, [_info_dict(i) for i in infos]
    return x, y, rc, _info_dict(infos[0])


def pdlp_batch_schedule(h: BatchHandle):
    """(lanes[count, 2] for K and K' rows, workgroups of the launch)."""
    lanes = np.zeros(2 * h.count, np.int32)
    g = C.c_int32()
    _check(lib().pdlp_batch_schedule(h.ptr, _ptr(lanes), C.byref(g)), h)
    return lanes.reshape(h.count, 2), g.value


def pdlp_presolve(problem) -> dict:
    """The reductions of presolve = 1 on the host (no device needed): status
    name, keep_row[m], keep_col[n] (bool), lo[n], hi[n], x_fixed[n],
    b_reduced[m], offset."""
    a = _host_arrays(problem)
    m, n = int(problem.m), int(problem.n)
    nnz = int(a["row_ptr"][-1]) if len(a["row_ptr"]) else 0
    ps = pdlp_problem(m, n, nnz, PDLP_MEM_HOST, *[_ptr(a[k]) for k in
                                                  ("row_ptr", "col_idx", "val", "c", "b", "l", "u", "row_type")])
    st = C.c_int32()
    kr = np.zeros(max(m, 1), np.uint8); kc = np.zeros(n, np.uint8)
    lo = np.zeros(n); hi = np.zeros(n); xf = np.zeros(n); br = np.zeros(max(m, 1)); off = C.c_double()
    _check(lib().pdlp_presolve(C.byref(ps), C.byref(st), _ptr(kr), _ptr(kc), _ptr(lo), _ptr(hi), _ptr(xf),
                               _ptr(br), C.byref(off)))
    return dict(status=STATUS.get(st.value, "OK") if st.value else "OK", keep_row=kr[:m].astype(bool),
                keep_col=kc.astype(bool), lo=lo, hi=hi, x_fixed=xf, b_reduced=br[:m], offset=off.value)


def pdlp_set_warm_start(h: Handle, x0=None, y0=None, omega0: float = 0.0):
    x0 = None if x0 is None else np.ascontiguousarray(x0, dtype=np.float64)
    y0 = None if y0 is None else np.ascontiguousarray(y0, dtype=np.float64)
    if x0 is not None and x0.shape != (h.n,):
        raise ValueError("x0 must have n entries")
    if y0 is not None and y0.shape != (h.m,):
        raise ValueError("y0 must have m entries")
    _check(lib().pdlp_set_warm_start(h.ptr, _ptr(x0), _ptr(y0), float(omega0)), h)


def pdlp_set_termination(h: Handle, eps_rel: float, max_iter: int, time_limit_s: float):
    _check(lib().pdlp_set_termination(h.ptr, float(eps_rel), int(max_iter), float(time_limit_s)), h)


def pdlp_solve(h: Handle):
    _check(lib().pdlp_solve(h.ptr), h)


def pdlp_solve_noalloc(h: Handle):
    """pdlp_solve without any device allocation (partial sums in the library's
    static device scratch; see include/pdlp.h)."""
    _check(lib().pdlp_solve_noalloc(h.ptr), h)


def _info_dict(info: pdlp_info) -> dict:
    d = {f: getattr(info, f) for f, _ in pdlp_info._fields_}
    d["status_name"] = STATUS.get(info.status, str(info.status))
    return d


def pdlp_get_solution(h: Handle):
    """(x[n], y[m], reduced_cost[n], info dict) of the last solve."""
    x = np.zeros(h.n); y = np.zeros(h.m); rc = np.zeros(h.n)
    info = pdlp_info()
    _check(lib().pdlp_get_solution(h.ptr, _ptr(x), _ptr(y), _ptr(rc), C.byref(info)), h)
    return x, y, rc, _info_dict(info)


def pdlp_get_iterate(h: Handle):
    xh = np.zeros(h.n); yh = np.zeros(h.m)
    st = pdlp_iter_state()
    _check(lib().pdlp_get_iterate(h.ptr, _ptr(xh), _ptr(yh), C.byref(st)), h)
    return xh, yh, {f: getattr(st, f) for f, _ in pdlp_iter_state._fields_}


def pdlp_get_scaling(h: Handle):
    D1 = np.zeros(h.m); D2 = np.zeros(h.n); vs = np.zeros(h.nnz)
    _check(lib().pdlp_get_scaling(h.ptr, _ptr(D1), _ptr(D2), _ptr(vs)), h)
    return D1, D2, vs


def pdlp_get_trace(h: Handle, cap: int) -> dict:
    na = C.c_int64(); ne = C.c_int64()
    t = dict(att_k=np.zeros(cap, np.int64), att_eta=np.zeros(cap), att_etabar=np.zeros(cap),
             att_acc=np.zeros(cap, np.int8), ev_k=np.zeros(cap, np.int64), ev_kkt_cur=np.zeros(cap),
             ev_kkt_avg=np.zeros(cap), ev_cand=np.zeros(cap, np.int8), ev_reason=np.zeros(cap, np.int8),
             ev_omega=np.zeros(cap))
    _check(lib().pdlp_get_trace(h.ptr, cap, C.byref(na), _ptr(t["att_k"]), _ptr(t["att_eta"]),
                                _ptr(t["att_etabar"]), _ptr(t["att_acc"]), C.byref(ne), _ptr(t["ev_k"]),
                                _ptr(t["ev_kkt_cur"]), _ptr(t["ev_kkt_avg"]), _ptr(t["ev_cand"]),
                                _ptr(t["ev_reason"]), _ptr(t["ev_omega"])), h)
    out = {k: v[:na.value] for k, v in t.items() if k.startswith("att")}
    out.update({k: v[:ne.value] for k, v in t.items() if k.startswith("ev")})
    return out


def pdlp_profile_attempts(h: Handle, attempts: int):
    a = C.c_double(); b = C.c_double()
    _check(lib().pdlp_profile_attempts(h.ptr, int(attempts), C.byref(a), C.byref(b)), h)
    return a.value, b.value


def pdlp_step_bytes(h: Handle):
    a = C.c_double(); b = C.c_double()
    _check(lib().pdlp_step_bytes(h.ptr, C.byref(a), C.byref(b)), h)
    return a.value, b.value


def pdlp_destroy(h: Handle):
    if h is not None and h.ptr:
        lib().pdlp_destroy(h.ptr)
        h.ptr = None


@dataclasses.dataclass
class Result:
    x: np.ndarray
    y: np.ndarray
    rc: np.ndarray
    status: str
    info: dict


def solve(problem, warm_start=None, stream=None, **opts) -> Result:
    """Create, (optionally warm-start), solve, fetch, destroy."""
    h = pdlp_create(problem, stream=stream, **opts)
    try:
        if warm_start is not None:
            pdlp_set_warm_start(h, *warm_start)
        pdlp_solve(h)
        x, y, rc, info = pdlp_get_solution(h)
    finally:
        pdlp_destroy(h)
    return Result(x, y, rc, info["status_name"], info)
