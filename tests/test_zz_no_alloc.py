"""pdlp_solve_noalloc (partial sums in the library's static device scratch,
no allocation during the solve) against pdlp_solve on the same handles.

Both run the same kernels in the same order on the same data, so the bar is
bitwise: x, y, reduced costs and the counters.  Two calls of the new entry
point in a row, the second on a smaller LP (the scratch keeps the first
call's contents, which the second must not see): a 20,000 x 40,000 skewed LP
with the headline LP's layouts (LDS-staged step passes of K, their dense
segment sums and the short rows' panel sums; SELL-64 passes of K'), then a
40 x 60 LP with every bound and row type on column panels with the
normalized-gap restarts (its partial sums too).  Infeasibility detection is on in both (its
partials as well)."""
import numpy as np
import pytest

import lpgen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    from paper_2311_12180_amd import pdlp
    pdlp.lib()
    return pdlp


def test_noalloc_matches_solve_on_two_calls_in_a_row(P):
    cases = [
        (lpgen.skewed_lp(3, m=20000, n=40000, nnz_target=400000, cap=8000),
         dict(eps_rel=1e-6, spmv_layout=35, spmv_layout_kt=64)),
        (lpgen.mixed_lp(1), dict(eps_rel=1e-6, spmv_layout=1, restart_metric=1)),
    ]
    handles, ref = [], []
    try:
        for p, opts in cases:
            h = P.pdlp_create(p, time_limit_s=60.0, max_iter=200000, **opts)
            handles.append(h)
            P.pdlp_solve(h)
            ref.append(P.pdlp_get_solution(h))
        info = P.pdlp_get_solution(handles[0])[3]
        assert (info["layout_k"], info["layout_kt"]) == (35, 64)
        for k, (p, _) in enumerate(cases):
            P.pdlp_solve_noalloc(handles[k])
            x, y, rc, I = P.pdlp_get_solution(handles[k])
            x0, y0, rc0, I0 = ref[k]
            print(f"{p.name}: {I['status_name']} after {I['iterations']} steps ({I['attempts']} attempts), "
                  f"pdlp_solve {I0['iterations']} ({I0['attempts']})")
            assert I["status_name"] == I0["status_name"] == "OPTIMAL"
            for key in ("iterations", "attempts", "restarts", "evaluations", "returned_avg"):
                assert I[key] == I0[key], (k, key)
            assert I["primal_obj"] == I0["primal_obj"] and I["rel_kkt"] == I0["rel_kkt"]
            np.testing.assert_array_equal(x, x0)
            np.testing.assert_array_equal(y, y0)
            np.testing.assert_array_equal(rc, rc0)
    finally:
        for h in handles:
            P.pdlp_destroy(h)


def test_noalloc_refuses_a_batch_handle(P):
    probs = [lpgen.mixed_lp(2), lpgen.mixed_lp(3)]
    h = P.pdlp_create_batch(probs, eps_rel=1e-6, time_limit_s=30.0)
    try:
        with pytest.raises(P.PdlpError) as e:
            P.pdlp_solve_noalloc(h)
        assert e.value.code == P.PDLP_ERR_STATE and "batch" in str(e.value)
    finally:
        P.pdlp_destroy(h)
