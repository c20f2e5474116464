"""C-ABI checks that need no GPU: the library loads, exports every function
include/pdlp.h declares, and rejects malformed input before touching HIP."""
import copy
import os
import re

import numpy as np
import pytest

import lpgen

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def P():
    from paper_2311_12180_amd import pdlp
    pdlp.lib()
    return pdlp


def declared_functions(header="pdlp.h"):
    text = open(os.path.join(ROOT, "include", header)).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pdlp_[a-z_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported(P):
    names = declared_functions()
    assert len(names) >= 13
    lib = P.lib()
    for name in names:
        assert hasattr(lib, name), name
    assert sorted(P.EXPORTED) == names


def test_network_symbols_are_exported(P):
    from paper_2311_12180_amd import gnn
    names = declared_functions("pdlp_gnn.h")
    assert sorted(gnn.EXPORTED) == names
    lib = gnn.lib()
    for name in names:
        assert hasattr(lib, name), name


def test_network_rejects_bad_input(P):
    from paper_2311_12180_amd import gnn
    good = lpgen.mixed_lp(0, m=10, n=12)
    bad = copy.deepcopy(good); bad.b[3] = np.inf
    with pytest.raises(P.PdlpError) as e:
        gnn.pdlp_gnn_create([good, bad])
    assert e.value.code == P.PDLP_ERR_DATA and "LP 1: b[3]" in str(e.value)
    x = np.zeros(24); y = np.zeros(20)
    with pytest.raises(P.PdlpError) as e:
        gnn.pdlp_gnn_create([good, good], x, y, np.array([1.0, -1.0]))
    assert e.value.code == P.PDLP_ERR_DATA and "omega_star" in str(e.value)
    with pytest.raises(P.PdlpError) as e:
        gnn.pdlp_gnn_create([good], x[:12], None, np.array([1.0]))
    assert e.value.code == P.PDLP_ERR_ARG
    lib = gnn.lib()
    assert lib.pdlp_gnn_create(None, 1, None, None, None, None, None) == P.PDLP_ERR_ARG
    assert lib.pdlp_gnn_set_params(None, None) == P.PDLP_ERR_ARG
    assert lib.pdlp_gnn_predict(None, 0, 1, None, None, None) == P.PDLP_ERR_ARG
    lib.pdlp_gnn_destroy(None)
    assert isinstance(gnn.pdlp_gnn_last_error(None), str)


def test_default_options(P):
    o = P.pdlp_default_options()
    assert o.eps_rel == 1e-4 and o.eval_period == 64 and o.ruiz_iters == 10
    assert o.pc_alpha == 1.0 and o.pw_theta == 0.5 and o.eps_zero == 1e-10
    assert (o.beta_suff, o.beta_nec, o.beta_art) == (0.2, 0.8, 0.36)
    assert o.a_precision == 0 and o.kkt_omega_power == 2


def _bad(p, P, code, fragment, **opts):
    with pytest.raises(P.PdlpError) as e:
        P.pdlp_create(p, **opts)
    assert e.value.code == code
    assert fragment in str(e.value)
    assert fragment in P.pdlp_last_error(None)


def test_rejects_malformed_problems(P):
    base = lpgen.mixed_lp(0, m=20, n=30)
    p = copy.deepcopy(base); p.col_idx[3] = p.n
    _bad(p, P, P.PDLP_ERR_DATA, "out of range")
    p = copy.deepcopy(base); r0, r1 = p.row_ptr[0], p.row_ptr[1]
    row = np.flatnonzero(np.diff(p.row_ptr) >= 2)[0]
    s = p.row_ptr[row]; p.col_idx[s + 1] = p.col_idx[s]
    _bad(p, P, P.PDLP_ERR_DATA, "duplicate column")
    p = copy.deepcopy(base); p.val[0] = np.nan
    _bad(p, P, P.PDLP_ERR_DATA, "not finite")
    p = copy.deepcopy(base); p.c[1] = np.inf
    _bad(p, P, P.PDLP_ERR_DATA, "c[1]")
    p = copy.deepcopy(base); p.b[2] = np.nan
    _bad(p, P, P.PDLP_ERR_DATA, "b[2]")
    p = copy.deepcopy(base); p.l[0] = 5.0; p.u[0] = 4.0
    _bad(p, P, P.PDLP_ERR_DATA, "bounds of x[0]")
    p = copy.deepcopy(base); p.l[1] = np.inf; p.u[1] = np.inf
    _bad(p, P, P.PDLP_ERR_DATA, "bounds of x[1]")
    p = copy.deepcopy(base); p.row_type[4] = 3
    _bad(p, P, P.PDLP_ERR_DATA, "row_type[4]")
    p = copy.deepcopy(base); p.row_ptr = p.row_ptr.copy(); p.row_ptr[5], p.row_ptr[6] = p.row_ptr[6], p.row_ptr[5]
    if p.row_ptr[5] > p.row_ptr[6]:
        _bad(p, P, P.PDLP_ERR_DATA, "row_ptr decreases")
    p = copy.deepcopy(base); p.row_ptr = p.row_ptr.copy(); p.row_ptr[0] = 1
    _bad(p, P, P.PDLP_ERR_DATA, "row_ptr[0]")


def test_rejects_bad_sizes_and_options(P):
    p = lpgen.mixed_lp(0, m=10, n=12)
    q = copy.deepcopy(p); q.n = 0
    _bad(q, P, P.PDLP_ERR_ARG, "sizes")
    _bad(p, P, P.PDLP_ERR_ARG, "eval_period", eval_period=0)
    _bad(p, P, P.PDLP_ERR_ARG, "a_precision", a_precision=7)
    _bad(p, P, P.PDLP_ERR_ARG, "pw_theta", pw_theta=1.5)
    _bad(p, P, P.PDLP_ERR_ARG, "eps_rel", eps_rel=float("nan"))
    _bad(p, P, P.PDLP_ERR_ARG, "max_iter", max_iter=-1)
    _bad(p, P, P.PDLP_ERR_ARG, "kkt_omega_power", kkt_omega_power=3)
    # layouts: 0, 1, 2 plus 4 (persistent grid) and/or 8 (wide step tiles), or
    # 3 + 16 cfg (LDS-staged step passes, cfg 0..2) with no other bit, or
    # 64 + 16 cfg (SELL-64 step passes, cfg 0..2) with no other bit
    for bad in (-2, 7, 11, 15, 16, 23, 27, 51, 65, 67, 68, 72, 112, 128):
        _bad(p, P, P.PDLP_ERR_ARG, "spmv_layout must be", spmv_layout=bad)
    for bad in (-3, 15, 16, 39, 51, 66, 76, 112):
        _bad(p, P, P.PDLP_ERR_ARG, "spmv_layout_kt must be", spmv_layout_kt=bad)
    for bad in (-1, 3):
        _bad(p, P, P.PDLP_ERR_ARG, "row_order must be", row_order=bad)


def test_batch_rejects_bad_members_and_options(P):
    good = lpgen.mixed_lp(0, m=10, n=12)
    bad = copy.deepcopy(good); bad.col_idx[2] = -1
    for probs, code, frag, opts in [([good, good, bad], P.PDLP_ERR_DATA, "LP 2: col_idx", {}),
                                    ([good], P.PDLP_ERR_ARG, "batch_lanes", {"batch_lanes": 3}),
                                    ([good], P.PDLP_ERR_ARG, "batch_lanes", {"batch_lanes": 128}),
                                    ([good], P.PDLP_ERR_ARG, "batch_grid", {"batch_grid": -2}),
                                    ([good], P.PDLP_ERR_ARG, "batch_handoff", {"batch_handoff": -1}),
                                    ([good], P.PDLP_ERR_ARG, "handoff_streams", {"handoff_streams": 0}),
                                    ([good], P.PDLP_ERR_ARG, "handoff_streams", {"handoff_streams": 17}),
                                    ([good], P.PDLP_ERR_ARG, "detect_infeas", {"detect_infeas": 2}),
                                    ([good], P.PDLP_ERR_ARG, "eps_infeas", {"eps_infeas": 0.0}),
                                    ([good], P.PDLP_ERR_ARG, "infeas_every", {"infeas_every": 0}),
                                    ([good], P.PDLP_ERR_ARG, "presolve", {"presolve": 2}),
                                    ([good], P.PDLP_ERR_ARG, "restart_metric", {"restart_metric": 2}),
                                    ([good], P.PDLP_ERR_ARG, "row_order", {"row_order": 3}),
                                    ([good], P.PDLP_ERR_UNSUPPORTED, "batch handles", {"presolve": 1}),
                                    ([], P.PDLP_ERR_ARG, "count", {})]:
        with pytest.raises(P.PdlpError) as e:
            P.pdlp_create_batch(probs, **opts)
        assert e.value.code == code and frag in str(e.value), str(e.value)


def test_null_arguments(P):
    lib = P.lib()
    assert lib.pdlp_default_options(None) == P.PDLP_ERR_ARG
    assert lib.pdlp_create(None, None, None, None) == P.PDLP_ERR_ARG
    assert lib.pdlp_solve(None) == P.PDLP_ERR_ARG
    assert lib.pdlp_get_solution(None, None, None, None, None) == P.PDLP_ERR_ARG
    assert lib.pdlp_set_termination(None, 1e-4, 10, 1.0) == P.PDLP_ERR_ARG
    assert lib.pdlp_create_batch(None, 1, None, None, None) == P.PDLP_ERR_ARG
    assert lib.pdlp_solve_batch(None) == P.PDLP_ERR_ARG
    assert lib.pdlp_get_solution_batch(None, 0, None, None, None, None) == P.PDLP_ERR_ARG
    assert lib.pdlp_set_warm_start_batch(None, 0, None, None, 0.0) == P.PDLP_ERR_ARG
    assert lib.pdlp_batch_schedule(None, None, None) == P.PDLP_ERR_ARG
    lib.pdlp_destroy(None)
    assert isinstance(P.pdlp_last_error(None), str)


def test_binding_fails_loudly_without_library(monkeypatch):
    from paper_2311_12180_amd import pdlp
    monkeypatch.setattr(pdlp, "_lib", None)
    monkeypatch.setattr(pdlp, "LIB_PATH", "/nonexistent/libpdlp_hip.so")
    with pytest.raises(ImportError):
        pdlp.lib()
