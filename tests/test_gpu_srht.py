"""The structured test matrix (PSDPROJ_FLAG_SRHT) on the GPU against the oracle: the matrix
bit for bit, and the projections built on it."""
import numpy as np
import pytest

import _gpu
from _gpu import TOL, matrix
from oracle import srht

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("seed,n,r", [(0, 1, 1), (3, 50, 20), (7, 512, 64), (11, 777, 52), (2**40 + 5, 20000, 220)])
def test_structured_matrix_bit_exact(seed, n, r):
    import torch
    import paper_2410_19208_amd as pp
    dev = _gpu.device()
    out = torch.zeros(n * r, dtype=torch.float64, device=dev)
    pp.psdproj_srht_matrix(seed, n, r, out.data_ptr(), 0)
    torch.cuda.synchronize()
    got = out.cpu().numpy().reshape(r, n).T
    if n * r <= 200000:
        assert np.array_equal(got, srht.test_matrix(seed, n, r))
    else:   # sampled entries, one column selection and sign vector computed by the oracle
        cols = srht.columns(seed, n, r)
        rows = np.random.default_rng(0).integers(0, n, 2000)
        d = srht.signs(seed, n)
        for i in rows[:200]:
            ref = d[i] * srht.hadamard_entry(np.full(r, i), cols)
            assert np.array_equal(got[i], ref)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
@pytest.mark.parametrize("variant", ["plain", "scaled"])
def test_structured_sketch_parity(prec, variant):
    import torch
    from paper_2410_19208_amd.torch_api import Projector
    from _gpu import parity, run_oracle
    from oracle import rnla
    dev = _gpu.device()
    n, k, p, q = 777, 40, 12, 1
    A, lam, U = matrix("medium", n, 5, n_pos=60)
    proj = Projector(n, k, p, q, variant, prec, seed=9, device=dev, sketch="srht")
    P = proj(_gpu.to_dev(A.astype(_gpu.storage(prec)), dev)).cpu().numpy()
    res = proj.result()
    A_in = A.astype(_gpu.storage(prec)).astype(np.float64)
    ref = rnla.project(A_in, k, p, q, variant, seed=9, omega_dtype=_gpu.storage(prec), sketch="srht")
    assert res.status == 0
    err = parity(P, ref, A)
    print(f"srht {prec} {variant}: parity {err:.3e} r+ {res.r_plus}/{ref.r_plus}")
    assert err < TOL[prec]
    assert np.array_equal(P, P.T)
