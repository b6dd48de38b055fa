"""psdproj_run_static (workspace in the library's static per-device scratch array, nothing
allocated by the call) against psdproj_run on the same plans and inputs: bitwise equal P and
result records, on consecutive calls whose later problems are smaller than the first, so the
array holds the previous call's contents when a call starts."""
import ctypes

import numpy as np
import pytest

import _gpu
from _gpu import matrix

pytestmark = pytest.mark.gpu


def _static_run(proj, At):
    import torch
    import paper_2410_19208_amd as pp
    from paper_2410_19208_amd.torch_api import read_results, stream_handle
    P = torch.full_like(At, float("nan"))
    res = torch.zeros(ctypes.sizeof(pp.Result), dtype=torch.uint8, device=At.device)
    pp.psdproj_run_static(proj.plan, At.data_ptr(), At.stride(0), P.data_ptr(), P.stride(0), res.data_ptr(),
                          stream_handle())
    return P, res


def test_run_static_equals_run():
    import torch
    import paper_2410_19208_amd as pp
    from paper_2410_19208_amd.torch_api import Projector, read_results
    dev = _gpu.device()
    cases = [(2000, 100, 10, 1, "scaled", "bf16x3"),   # the largest first
             (777, 40, 12, 1, "plain", "fp32"),
             (300, 24, 8, 0, "scaled", "fp64")]
    for i, (n, k, p, q, variant, prec) in enumerate(cases):
        A, _, _ = matrix("medium", n, 40 + i, n_pos=max(4, n // 10))
        At = _gpu.to_dev(A.astype(_gpu.storage(prec)), dev)
        proj = Projector(n, k, p, q, variant, prec, seed=9, device=dev)
        need, cap = pp.psdproj_static_scratch_bytes(proj.plan)
        assert need <= cap
        P_ref = proj(At)
        torch.cuda.synchronize()
        r_ref = proj.result()
        P_st, res = _static_run(proj, At)
        torch.cuda.synchronize()
        r_st = read_results(res, 1)[0]
        assert r_ref.status == 0 and r_st.status == 0
        assert (r_st.r_plus, r_st.alpha_used) == (r_ref.r_plus, r_ref.alpha_used)
        assert torch.equal(P_st, P_ref), f"call {i}: static-scratch run differs from psdproj_run"
    # a second static call of the first plan after the smaller ones: same result again
    n, k, p, q, variant, prec = cases[0]
    A, _, _ = matrix("medium", n, 40, n_pos=n // 10)
    At = _gpu.to_dev(A.astype(np.float32), dev)
    proj = Projector(n, k, p, q, variant, prec, seed=9, device=dev)
    P_ref = proj(At)
    P_st, _ = _static_run(proj, At)
    torch.cuda.synchronize()
    assert torch.equal(P_st, P_ref)


def test_run_static_rejects_oversized_problem():
    import paper_2410_19208_amd as pp
    _gpu.device()
    plan, _ = pp.psdproj_plan(20000, 200, 20, 1, pp.PLAIN, pp.BF16X3)
    try:
        need, cap = pp.psdproj_static_scratch_bytes(plan)
        assert need > cap
        st = pp.lib.psdproj_run_static(plan, ctypes.c_void_p(4096), 20000, ctypes.c_void_p(4096 + 2 * 1600000000),
                                       20000, ctypes.c_void_p(256), None)
        assert st == pp.E_SCRATCH
    finally:
        pp.psdproj_plan_destroy(plan)
