"""Python binding of include/pdlp_gnn.h (argument marshalling only).

The network, its training and its inference run in the HIP library; this
module converts arguments.  Problems come as objects with numpy arrays (see
pdlp.pdlp_create)."""
from __future__ import annotations

import ctypes as C
from typing import Optional

import numpy as np

from . import pdlp as _P

PDLP_GNN_PARAMS = 50499
EXPORTED = ["pdlp_gnn_create", "pdlp_gnn_set_params", "pdlp_gnn_set_loss_weights", "pdlp_gnn_get_params",
            "pdlp_gnn_loss_grad",
            "pdlp_gnn_train_step", "pdlp_gnn_predict", "pdlp_gnn_last_error", "pdlp_gnn_destroy"]

_ready = False


def lib() -> C.CDLL:
    global _ready
    L = _P.lib()
    if not _ready:
        vp, i32, dbl = C.c_void_p, C.c_int32, C.c_double
        L.pdlp_gnn_create.argtypes = [C.POINTER(_P.pdlp_problem), i32, vp, vp, vp, vp, C.POINTER(vp)]
        L.pdlp_gnn_set_params.argtypes = [vp, vp]
        L.pdlp_gnn_get_params.argtypes = [vp, vp]
        L.pdlp_gnn_set_loss_weights.argtypes = [vp, dbl, dbl, dbl]
        L.pdlp_gnn_loss_grad.argtypes = [vp, i32, i32, C.POINTER(dbl), vp]
        L.pdlp_gnn_train_step.argtypes = [vp, i32, i32, C.c_float, C.POINTER(dbl)]
        L.pdlp_gnn_predict.argtypes = [vp, i32, i32, vp, vp, vp]
        L.pdlp_gnn_last_error.argtypes = [vp]
        L.pdlp_gnn_last_error.restype = C.c_char_p
        L.pdlp_gnn_destroy.argtypes = [vp]
        L.pdlp_gnn_destroy.restype = None
        for name in EXPORTED:
            if name not in ("pdlp_gnn_last_error", "pdlp_gnn_destroy"):
                getattr(L, name).restype = C.c_int
        _ready = True
    return L


def pdlp_gnn_last_error(g=None) -> str:
    return lib().pdlp_gnn_last_error(g.ptr if isinstance(g, GraphSet) else g).decode()


def _check(rc: int, g=None):
    if rc != _P.PDLP_OK:
        raise _P.PdlpError(rc, pdlp_gnn_last_error(g))


class GraphSet:
    """Owns a pdlp_gnn handle over `count` LPs."""

    def __init__(self, ptr, ms, ns, keep):
        self.ptr = ptr
        self.count = len(ms)
        self.ms = np.asarray(ms, np.int64)
        self.ns = np.asarray(ns, np.int64)
        self.row_off = np.concatenate([[0], np.cumsum(self.ms)])
        self.col_off = np.concatenate([[0], np.cumsum(self.ns)])
        self._keep = keep

    def __del__(self):
        try:
            pdlp_gnn_destroy(self)
        except Exception:
            pass


def pdlp_gnn_create(problems, x_star=None, y_star=None, omega_star=None, stream=None) -> GraphSet:
    """Graph set over a list of host problems; x_star / y_star packed (or a
    list of per-LP arrays), omega_star[count], or all None."""
    arrs = [_P._host_arrays(p) for p in problems]
    structs = (_P.pdlp_problem * max(len(arrs), 1))()
    for k, (p, a) in enumerate(zip(problems, arrs)):
        nnz = int(a["row_ptr"][-1]) if len(a["row_ptr"]) else 0
        structs[k] = _P.pdlp_problem(int(p.m), int(p.n), nnz, _P.PDLP_MEM_HOST,
                                     *[_P._ptr(a[key]) for key in
                                       ("row_ptr", "col_idx", "val", "c", "b", "l", "u", "row_type")])
    pack = lambda v: None if v is None else np.ascontiguousarray(
        np.concatenate(v) if isinstance(v, (list, tuple)) else v, dtype=np.float64)
    xs, ys, om = pack(x_star), pack(y_star), pack(omega_star)
    n_tot = sum(int(p.n) for p in problems)
    m_tot = sum(int(p.m) for p in problems)
    if xs is not None and xs.shape != (n_tot,):
        raise ValueError(f"x_star must have {n_tot} entries")
    if ys is not None and ys.shape != (m_tot,):
        raise ValueError(f"y_star must have {m_tot} entries")
    if om is not None and om.shape != (len(problems),):
        raise ValueError(f"omega_star must have {len(problems)} entries")
    ys_ptr = None if ys is None else (ys.ctypes.data if ys.size else C.addressof(C.c_double()))
    out = C.c_void_p()
    _check(lib().pdlp_gnn_create(structs, len(arrs), _P._ptr(xs), ys_ptr, _P._ptr(om),
                                 C.c_void_p(stream) if stream else None, C.byref(out)))
    return GraphSet(out.value, [int(p.m) for p in problems], [int(p.n) for p in problems],
                    (arrs, structs, xs, ys, om))


def pdlp_gnn_set_params(g: GraphSet, theta):
    th = np.ascontiguousarray(theta, dtype=np.float32)
    if th.shape != (PDLP_GNN_PARAMS,):
        raise ValueError(f"theta must have {PDLP_GNN_PARAMS} entries")
    _check(lib().pdlp_gnn_set_params(g.ptr, th.ctypes.data), g)


def pdlp_gnn_set_loss_weights(g: GraphSet, w_x: float, w_y: float, w_o: float):
    _check(lib().pdlp_gnn_set_loss_weights(g.ptr, float(w_x), float(w_y), float(w_o)), g)


def pdlp_gnn_get_params(g: GraphSet) -> np.ndarray:
    th = np.zeros(PDLP_GNN_PARAMS, np.float32)
    _check(lib().pdlp_gnn_get_params(g.ptr, th.ctypes.data), g)
    return th


def pdlp_gnn_loss_grad(g: GraphSet, first: int, count: int):
    L = C.c_double()
    grad = np.zeros(PDLP_GNN_PARAMS, np.float32)
    _check(lib().pdlp_gnn_loss_grad(g.ptr, int(first), int(count), C.byref(L), grad.ctypes.data), g)
    return L.value, grad


def pdlp_gnn_train_step(g: GraphSet, first: int, count: int, lr: float) -> float:
    L = C.c_double()
    _check(lib().pdlp_gnn_train_step(g.ptr, int(first), int(count), float(lr), C.byref(L)), g)
    return L.value


def pdlp_gnn_predict(g: GraphSet, first: int, count: int):
    """(x0 packed, y0 packed, omega0[count]) for LPs [first, first + count)."""
    nv = int(g.col_off[first + count] - g.col_off[first])
    nc = int(g.row_off[first + count] - g.row_off[first])
    x0 = np.zeros(nv); y0 = np.zeros(nc); om = np.zeros(count)
    _check(lib().pdlp_gnn_predict(g.ptr, int(first), int(count), x0.ctypes.data,
                                  y0.ctypes.data if nc else None, om.ctypes.data), g)
    return x0, y0, om


def pdlp_gnn_destroy(g: Optional[GraphSet]):
    if g is not None and g.ptr:
        lib().pdlp_gnn_destroy(g.ptr)
        g.ptr = None
