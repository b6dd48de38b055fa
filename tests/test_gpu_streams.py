"""Grouped launch sequences issued round-robin to several HIP streams, each stream with its own
projectors, workspaces and outputs (the pattern of the throughput benchmark, where one step's
latency-bound stages overlap the other steps' streaming kernels): every output equals a lone run
of the same problems bit for bit, and no run reports an error."""
import pytest

import _gpu
from _gpu import matrix

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec", ["bf16x3", "fp32", "fp64"])
def test_round_robin_streams_equal_lone_run(prec):
    import torch
    from paper_2410_19208_amd.torch_api import BatchProjector
    dev = _gpu.device()
    n, k, p, q = 700, 40, 8, 1
    A_np, _, _ = matrix("small", n, 77, n_pos=60)
    A = _gpu.to_dev(A_np.astype(_gpu.storage(prec)), dev)
    specs = [dict(n=n, k=k, p=p, q=q, variant="plain", precision=prec, seed=3),
             dict(n=n, k=k, p=p, q=q, variant="scaled", precision=prec, seed=3, alpha=0.0, alpha_iters=10)]

    lone = BatchProjector(specs, device=dev)
    R1, R2 = torch.empty_like(A), torch.empty_like(A)
    lone([A, A], [R1, R2])
    torch.cuda.synchronize()
    assert all(r.status == 0 for r in lone.results())

    nslot = 3
    streams = [None] + [torch.cuda.Stream(device=dev) for _ in range(nslot - 1)]
    slots = [(BatchProjector(specs, device=dev), torch.full_like(A, float("nan")), torch.full_like(A, float("nan")), s)
             for s in streams]
    torch.cuda.synchronize()
    for i in range(3 * nslot):
        bp, P1, P2, s = slots[i % nslot]
        bp([A, A], [P1, P2], stream=s)
    torch.cuda.synchronize()
    for j, (bp, P1, P2, _) in enumerate(slots):
        assert all(r.status == 0 for r in bp.results()), f"slot {j}"
        assert torch.equal(P1, R1), f"slot {j}: plain output differs from the lone run"
        assert torch.equal(P2, R2), f"slot {j}: scaled output differs from the lone run"
