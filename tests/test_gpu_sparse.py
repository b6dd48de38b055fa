"""Sparse A (CSR, psdproj_run_csr) against the oracle on the same matrix made dense."""
import numpy as np
import pytest

import _gpu
import workloads
from _gpu import TOL, parity

pytestmark = pytest.mark.gpu


def _csr_to_dev(rp, ci, v, dev):
    import torch
    return (torch.from_numpy(rp).to(dev), torch.from_numpy(ci).to(dev), torch.from_numpy(v).to(dev))


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
@pytest.mark.parametrize("variant", ["plain", "scaled"])
@pytest.mark.parametrize("n,per_row,q", [(1500, 16, 1), (777, 40, 0)])
def test_sparse_parity(prec, variant, n, per_row, q):
    import torch
    from paper_2410_19208_amd.torch_api import SparseProjector
    from oracle import rnla
    dev = _gpu.device()
    k, p = 60, 10
    rp, ci, v, D = workloads.sparse_symmetric(n, per_row, 17, _gpu.storage(prec))
    proj = SparseProjector(n, k, p, q, variant, prec, seed=4, device=dev)
    P = proj(*_csr_to_dev(rp, ci, v, dev)).cpu().numpy()
    res = proj.result()
    ref = rnla.project(D, k, p, q, variant, seed=4, omega_dtype=_gpu.storage(prec))
    assert res.status == 0
    if variant == "scaled":
        assert abs(res.alpha_used - ref.alpha) < 1e-10 * ref.alpha
    err = parity(P, ref, D)
    print(f"sparse n={n} nnz/row={len(ci) / n:.1f} {prec} {variant} q={q}: parity {err:.3e} r+ {res.r_plus}/{ref.r_plus}")
    assert err < TOL[prec]
    assert np.array_equal(P, P.T)


def test_sparse_matches_dense_path():
    """The same matrix through psdproj_run (dense) and psdproj_run_csr: both within FP64 parity
    of the oracle, so within 2e-10 of each other."""
    import torch
    from paper_2410_19208_amd.torch_api import Projector, SparseProjector
    dev = _gpu.device()
    n = 900
    rp, ci, v, D = workloads.sparse_symmetric(n, 24, 5, np.float64)
    Ps = SparseProjector(n, 50, 10, 1, "scaled", "fp64", seed=2, device=dev)(*_csr_to_dev(rp, ci, v, dev))
    Pd = Projector(n, 50, 10, 1, "scaled", "fp64", seed=2, device=dev)(_gpu.to_dev(D, dev))
    torch.cuda.synchronize()
    Ps, Pd = Ps.cpu().numpy(), Pd.cpu().numpy()
    assert np.linalg.norm(Ps - Pd) <= 2e-10 * np.linalg.norm(Pd)


def test_sparse_bad_index_is_reported():
    import torch
    import paper_2410_19208_amd as pp
    from paper_2410_19208_amd.torch_api import SparseProjector
    dev = _gpu.device()
    n = 300
    rp, ci, v, D = workloads.sparse_symmetric(n, 8, 6, np.float32)
    ci = ci.copy()
    ci[5] = n + 7                      # a column index past n: skipped, reported
    proj = SparseProjector(n, 20, 5, 0, "plain", "fp32", device=dev)
    proj(*_csr_to_dev(rp, ci, v, dev))
    torch.cuda.synchronize()
    assert proj.result().status == pp.E_INVALID
    # a CSR plan is refused by the dense entry point (synchronously)
    A = torch.zeros(n, n, dtype=torch.float32, device=dev)
    with pytest.raises(pp.PsdprojError):
        pp.psdproj_run(proj.plan, A.data_ptr(), n, A.data_ptr(), n, proj.workspace.data_ptr(),
                       proj.result_buf.data_ptr(), 0)
