"""Captured launch sequences (HIP graphs): replays equal direct launches bit for bit.

Each replay is checked against the eager result, with eager work of the program's own and
synchronisations between the replays, and with the outputs poisoned before each replay so that
a replay that wrote nothing would be caught."""
import ctypes

import numpy as np
import pytest

import _gpu
from _gpu import matrix

pytestmark = pytest.mark.gpu

SPECS = [dict(n=900, k=60, p=10, q=1, variant="scaled", precision="bf16x3", seed=1),
         dict(n=500, k=30, p=10, q=0, variant="plain", precision="fp32", seed=2),
         dict(n=300, k=20, p=5, q=2, variant="plain", precision="fp64", seed=3)]


def _inputs(dev, shift=0):
    As = []
    for i, s in enumerate(SPECS):
        A, _, _ = matrix("small", s["n"], 60 + i + shift, n_pos=max(4, s["n"] // 8))
        As.append(_gpu.to_dev(A.astype(_gpu.storage(s["precision"])), dev))
    return As


def test_explicit_graph_replays_equal_batch():
    import torch
    import paper_2410_19208_amd as pp
    from paper_2410_19208_amd.torch_api import BatchProjector, Projector, stream_handle
    dev = _gpu.device()
    As = _inputs(dev)
    As2 = _inputs(dev, shift=10)
    eager = BatchProjector(SPECS, device=dev)
    ref1 = [p.clone() for p in eager(As)]
    torch.cuda.synchronize()
    ref2 = [p.clone() for p in eager(As2)]
    torch.cuda.synchronize()
    assert all(r.status == 0 for r in eager.results())

    # a graph bound to its own inputs, outputs and workspace
    g_in = [a.clone() for a in As]
    g_out = [torch.empty_like(a) for a in As]
    bp = BatchProjector(SPECS, device=dev)   # plans and a workspace of the right size
    graph = pp.psdproj_graph_create(bp.plans, [a.data_ptr() for a in g_in], [a.stride(0) for a in g_in],
                                    [p.data_ptr() for p in g_out], [p.stride(0) for p in g_out],
                                    bp.workspace.data_ptr(), bp.ws_bytes, bp.result_buf.data_ptr())
    other = Projector(400, 20, 5, 1, "plain", "bf16x3", seed=5, device=dev)
    A_other = _gpu.to_dev(matrix("small", 400, 77, n_pos=30)[0].astype(np.float32), dev)
    P_other = other(A_other).clone()
    try:
        for rep in range(4):
            use2 = rep % 2 == 1
            for a, src in zip(g_in, As2 if use2 else As):
                a.copy_(src)
            for p in g_out:
                p.fill_(float("nan"))
            pp.psdproj_graph_launch(graph, stream_handle())
            # eager work of the program between replays, on the same stream
            P_mid = other(A_other)
            x = torch.randn(1000, 1000, device=dev)
            (x @ x).sum().item()
            torch.cuda.synchronize()
            assert torch.equal(P_mid, P_other)
            assert all(r.status == 0 for r in bp.results())
            for i, (p, r) in enumerate(zip(g_out, ref2 if use2 else ref1)):
                assert torch.equal(p, r), f"replay {rep}: problem {i} differs from the eager batch"
    finally:
        pp.psdproj_graph_destroy(graph)


def test_run_cache_replays_equal_direct_launch():
    import torch
    import paper_2410_19208_amd as pp
    from paper_2410_19208_amd.torch_api import Projector
    dev = _gpu.device()
    n, k, p = 700, 40, 10
    A, _, _ = matrix("medium", n, 3, n_pos=70)
    At = _gpu.to_dev(A.astype(np.float32), dev)
    proj = Projector(n, k, p, 1, "scaled", "bf16x3", seed=8, device=dev)
    c0, r0 = pp.psdproj_graph_stats()
    first = proj(At).clone()     # direct launches (first time the sequence is seen)
    torch.cuda.synchronize()
    for rep in range(4):
        P = torch.full_like(At, float("nan"))
        proj(At, P)
        torch.cuda.synchronize()
        assert proj.result().status == 0
        assert torch.equal(P, first), f"run {rep + 2} differs from the first"
    c1, r1 = pp.psdproj_graph_stats()
    if not __import__("os").environ.get("PSDPROJ_GRAPHS", "1").startswith("0"):
        assert c1 >= c0 + 1 and r1 >= r0 + 3


def test_batch_cache_replays_equal_single_runs():
    import torch
    from paper_2410_19208_amd.torch_api import BatchProjector, Projector
    dev = _gpu.device()
    As = _inputs(dev)
    bp = BatchProjector(SPECS, device=dev)
    singles = []
    for s in SPECS:
        s2 = dict(s)
        singles.append(Projector(s2.pop("n"), s2.pop("k"), s2.pop("p"), device=dev, **s2))
    ref = [pr(a).clone() for pr, a in zip(singles, As)]
    torch.cuda.synchronize()
    for rep in range(3):
        Ps = [torch.full_like(a, float("nan")) for a in As]
        bp(As, Ps)
        torch.cuda.synchronize()
        for i, (p, r) in enumerate(zip(Ps, ref)):
            assert torch.equal(p, r), f"batch run {rep}: problem {i} differs from its single run"
