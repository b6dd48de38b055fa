"""Alg. 5 on the GPU against the oracle's literal two power iterations (Alg. 4 twice).

For N <= 32 the library runs both iterations over one stream of two-vector products and forms
the second run's iterates from a shifted Krylov basis at the end; for larger N it runs them one
after the other.  Both forms must give alpha, sigma_1 and sigma_2 of the literal iteration to
1e-10 relative, on spectra chosen to stress the basis (a matrix near a multiple of I, nearly PSD,
a large outlier, a wide uniform spectrum) as well as the workload spectra."""
import numpy as np
import pytest

import _gpu
import workloads
from oracle import rnla

pytestmark = pytest.mark.gpu


def _spectrum(kind, n, rng):
    if kind == "small":
        return workloads.spectrum_small(n, max(2, n // 10), 3)
    if kind == "uniform":
        return rng.uniform(-1.0, 1.0, n)
    if kind == "near_identity":
        return 1.0 + 1e-3 * rng.uniform(-1.0, 1.0, n)
    if kind == "near_minus_identity":
        return -1.0 + 1e-3 * rng.uniform(-1.0, 1.0, n)
    if kind == "nearly_psd":
        return np.r_[rng.uniform(0.0, 1.0, n - 1), -1e-2]
    if kind == "outlier":
        return np.r_[50.0, rng.uniform(-1.0, 1.0, n - 1)]
    raise ValueError(kind)


def _alpha_case(kind, n, N, prec, seed):
    rng = np.random.default_rng(seed)
    U = workloads.haar_orthogonal(n, seed)
    A = workloads.from_spectrum(U, _spectrum(kind, n, rng))
    A = A.astype(_gpu.storage(prec))
    proj, P, res = _gpu.run_gpu(A, 8, 4, 0, "scaled", prec, seed=seed, alpha_iters=N)
    a_ref, s1, s2 = rnla.min_eig(A.astype(np.float64), N, seed)
    return res, a_ref, s1, s2


@pytest.mark.parametrize("N", [1, 2, 10, 32, 33, 50])
@pytest.mark.parametrize("kind", ["small", "uniform", "near_identity", "near_minus_identity", "nearly_psd",
                                  "outlier"])
def test_alpha_both_forms(kind, N):
    res, a_ref, s1, s2 = _alpha_case(kind, 700, N, "fp64", 3)
    assert res.status == 0
    form = "paired" if N <= 32 else "sequential"
    print(f"{kind} N={N} ({form}): alpha {res.alpha_used:.15e} vs {a_ref:.15e}, "
          f"rel {abs(res.alpha_used - a_ref) / a_ref:.2e}")
    assert abs(res.sigma1 - s1) <= 1e-12 * s1
    assert abs(res.sigma2 - s2) <= 1e-10 * max(s2, 1e-300) + 1e-13 * s1
    assert abs(res.alpha_used - a_ref) <= 1e-10 * a_ref


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
@pytest.mark.parametrize("n", [255, 1024, 3000])
def test_alpha_fp32_storage(prec, n):
    """FP32 storage: the vectors and sums stay FP64, so alpha matches the oracle's on the same
    FP32-rounded matrix to the same bound; ragged and multi-block orders."""
    for kind in ("small", "near_identity"):
        res, a_ref, _, _ = _alpha_case(kind, n, 10, prec, 5)
        assert res.status == 0
        assert abs(res.alpha_used - a_ref) <= 1e-10 * a_ref, kind


def test_alpha_sparse_paired():
    """The sparse product (one thread per row) in the paired form."""
    import torch
    from paper_2410_19208_amd.torch_api import SparseProjector
    dev = _gpu.device()
    n = 900
    rp, ci, v, D = workloads.sparse_symmetric(n, 20, 8, np.float64)
    D = D + 3.0 * np.eye(n)          # shift the spectrum away from 0: the basis must follow it
    rows, cols = np.nonzero(D)
    order = np.lexsort((cols, rows))
    rows, cols = rows[order], cols[order]
    rp = np.zeros(n + 1, dtype=np.int32)
    np.add.at(rp, rows + 1, 1)
    rp = np.cumsum(rp).astype(np.int32)
    vals = D[rows, cols].astype(np.float64)
    proj = SparseProjector(n, 20, 5, 0, "scaled", "fp64", seed=6, device=dev)
    proj(torch.from_numpy(rp).to(dev), torch.from_numpy(cols.astype(np.int32)).to(dev),
         torch.from_numpy(vals).to(dev))
    torch.cuda.synchronize()
    res = proj.result()
    a_ref, _, _ = rnla.min_eig(D, 10, 6)
    assert res.status == 0
    assert abs(res.alpha_used - a_ref) <= 1e-10 * a_ref


def test_mixed_forms_in_one_batch_equal_single_runs():
    """Problems with N = 10 (paired) and N = 40 (sequential) in one grouped batch: each result is
    bitwise its single run."""
    import torch
    from paper_2410_19208_amd.torch_api import BatchProjector, Projector
    dev = _gpu.device()
    specs = [dict(n=600, k=30, p=8, q=1, variant="scaled", precision="bf16x3", seed=1, alpha_iters=10),
             dict(n=450, k=20, p=8, q=0, variant="scaled", precision="bf16x3", seed=2, alpha_iters=40),
             dict(n=800, k=40, p=8, q=1, variant="scaled", precision="fp64", seed=3, alpha_iters=5),
             dict(n=300, k=20, p=8, q=0, variant="plain", precision="fp32", seed=4)]
    As = []
    for i, s in enumerate(specs):
        A, _, _ = _gpu.matrix("small", s["n"], 40 + i, n_pos=max(2, s["n"] // 10))
        As.append(_gpu.to_dev(A.astype(_gpu.storage(s["precision"])), dev))
    bp = BatchProjector(specs, device=dev)
    Pb = bp(As)
    torch.cuda.synchronize()
    rb = bp.results()
    for i, s in enumerate(specs):
        s2 = dict(s)
        proj = Projector(s2.pop("n"), s2.pop("k"), s2.pop("p"), device=dev, **s2)
        P1 = proj(As[i])
        torch.cuda.synchronize()
        r1 = proj.result()
        assert r1.status == 0 and rb[i].status == 0
        assert (r1.alpha_used, r1.sigma1, r1.sigma2) == (rb[i].alpha_used, rb[i].sigma1, rb[i].sigma2)
        assert torch.equal(P1, Pb[i]), f"batch member {i} differs from its single run"
