"""The headline workload at its full size, in the launch configuration the benchmark times.

n = 20000, k = 200, p = 20, q = 1: A = U diag(lam) U^T with a Haar-orthogonal U and 5% of the
eigenvalues positive (the large workload), FP32 resident.  One step is one plain (Alg. 2) and
one scaled (Alg. 3, alpha by Alg. 5 with N = 10) projection as one grouped batch; three steps
run at once on three streams, each with its own workspaces and outputs.  Every slot's P must be
bitwise the same, and slot 0's P, alpha and r_plus must match the FP64 oracle on the same FP32
matrix and FP32-rounded test matrix (BF16X3 and FP32 within 1e-5, alpha within 1e-10)."""
import numpy as np
import pytest

import _gpu
import workloads
from oracle import rnla

pytestmark = pytest.mark.gpu

N, K, P_OS, Q = 20000, 200, 20, 1


@pytest.fixture(scope="module")
def headline():
    import torch
    dev = _gpu.device()
    U = workloads.haar_orthogonal(N, 3001, device="cuda")
    lam = workloads.spectrum_large(N, 0.05, 3001)
    A = workloads.from_spectrum(U, lam).to(torch.float32)
    del U
    torch.cuda.synchronize()
    A_host = A.cpu().numpy().astype(np.float64)
    o_plain = rnla.project(A_host, K, P_OS, Q, "plain", seed=0, omega_dtype=np.float32)
    o_scaled = rnla.project(A_host, K, P_OS, Q, "scaled", seed=0, alpha_iters=10, omega_dtype=np.float32)
    yield dev, A, float(np.linalg.norm(A_host)), o_plain, o_scaled
    del A


def _check(P, o, a_fro, tol, label):
    err = rnla.parity_error(P.cpu().numpy().astype(np.float64), o.P, a_fro)
    print(f"{label}: parity {err:.3e}")
    assert err < tol


def test_grouped_three_in_flight(headline):
    import torch
    from paper_2410_19208_amd.torch_api import BatchProjector
    dev, A, a_fro, o_plain, o_scaled = headline
    specs = [dict(n=N, k=K, p=P_OS, q=Q, variant="plain", precision="bf16x3", seed=0),
             dict(n=N, k=K, p=P_OS, q=Q, variant="scaled", precision="bf16x3", seed=0, alpha=0.0, alpha_iters=10)]
    streams = [None, torch.cuda.Stream(device=dev), torch.cuda.Stream(device=dev)]
    slots = [(BatchProjector(specs, device=dev), torch.empty_like(A), torch.empty_like(A)) for _ in streams]
    torch.cuda.synchronize()
    for (bp, P1, P2), st in zip(slots, streams):
        bp([A, A], [P1, P2], stream=st)
    torch.cuda.synchronize()
    for bp, _, _ in slots:
        assert [r.status for r in bp.results()] == [0, 0]
    for bp, P1, P2 in slots[1:]:
        assert torch.equal(P1, slots[0][1]) and torch.equal(P2, slots[0][2])
    r_plain, r_scaled = slots[0][0].results()
    assert r_plain.r_plus == o_plain.r_plus and r_scaled.r_plus == o_scaled.r_plus
    assert abs(r_scaled.alpha_used - o_scaled.alpha) < 1e-10 * o_scaled.alpha
    _check(slots[0][1], o_plain, a_fro, _gpu.TOL["bf16x3"], "n=20000 plain bf16x3 (grouped, 3 in flight)")
    _check(slots[0][2], o_scaled, a_fro, _gpu.TOL["bf16x3"], "n=20000 scaled bf16x3 (grouped, 3 in flight)")


def test_fp32_single_requests(headline):
    import torch
    from paper_2410_19208_amd.torch_api import Projector
    dev, A, a_fro, o_plain, o_scaled = headline
    for variant, o in (("plain", o_plain), ("scaled", o_scaled)):
        pr = Projector(N, K, P_OS, Q, variant, "fp32", seed=0, alpha=0.0, alpha_iters=10, device=dev)
        P = pr(A)
        torch.cuda.synchronize()
        res = pr.result()
        assert res.status == 0 and res.r_plus == o.r_plus
        _check(P, o, a_fro, _gpu.TOL["fp32"], f"n=20000 {variant} fp32 (single request)")
        del P
