"""The request server (psdproj_server_*) on the GPU: every request's P equals a single run of
the same desc bit for bit, whatever else was in flight; admission respects the HBM budget;
the synchronous error paths."""
import threading

import numpy as np
import pytest

import _gpu
from _gpu import matrix

pytestmark = pytest.mark.gpu

SPECS = [
    dict(n=300, k=20, p=8, q=1, variant="plain", precision="bf16x3", seed=1),
    dict(n=1000, k=60, p=10, q=0, variant="scaled", precision="bf16x3", seed=2),
    dict(n=77, k=10, p=5, q=2, variant="scaled", precision="fp32", seed=3, alpha=0.5),
    dict(n=512, k=40, p=10, q=0, variant="plain", precision="fp64", seed=0),
    dict(n=650, k=20, p=8, q=1, variant="plain", precision="bf16x3", seed=5),
    dict(n=1200, k=100, p=12, q=1, variant="scaled", precision="fp32", seed=6),
]


def _inputs(dev):
    As = []
    for i, s in enumerate(SPECS):
        A, _, _ = matrix("small", s["n"], 40 + i, n_pos=max(2, s["n"] // 10))
        As.append(_gpu.to_dev(A.astype(_gpu.storage(s["precision"])), dev))
    return As


def _single(spec, A, dev):
    import torch
    from paper_2410_19208_amd.torch_api import Projector
    s = dict(spec)
    proj = Projector(s.pop("n"), s.pop("k"), s.pop("p"), device=dev, **s)
    P = proj(A)
    torch.cuda.synchronize()
    return P, proj.result()


def _submit(srv, spec, A):
    s = dict(spec)
    s.pop("n")
    k, p = s.pop("k"), s.pop("p")
    return srv.submit(A, k, p, **s)


@pytest.mark.parametrize("budget_mib,max_inflight", [(512, 16), (12, 16), (512, 1)])
def test_server_results_equal_single_runs(budget_mib, max_inflight):
    """(512 MiB, 16): requests share batches; 12 MiB: the budget admits about one at a time;
    max_inflight = 1: strictly one at a time.  Requests come from two host threads."""
    import torch
    from paper_2410_19208_amd.torch_api import Server
    dev = _gpu.device()
    As = _inputs(dev)
    ref = [_single(s, A, dev) for s, A in zip(SPECS, As)]
    srv = Server(budget_mib << 20, max_inflight, device=dev)
    tickets = [None] * len(SPECS)

    def worker(idx):
        for i in idx:
            tickets[i] = _submit(srv, SPECS[i], As[i])

    th = [threading.Thread(target=worker, args=(range(j, len(SPECS), 2),)) for j in range(2)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    for i, (t, P) in enumerate(tickets):
        res = srv.wait(t, 120.0)
        assert res.status == 0, f"request {i}: status {res.status}"
        assert res.r_plus == ref[i][1].r_plus
        assert torch.equal(P, ref[i][0]), f"request {i} differs from its single run"
        ts, ta, tf = srv.times(t)
        assert 0.0 <= ts <= ta <= tf
    srv.close()


def test_server_errors():
    import paper_2410_19208_amd as pp
    from paper_2410_19208_amd.torch_api import Server
    dev = _gpu.device()
    A = _gpu.to_dev(np.eye(600, dtype=np.float32), dev)
    srv = Server(6 << 20, 4, device=dev)
    with pytest.raises(pp.PsdprojError) as e:      # workspace (7.6 MiB) alone exceeds the 6 MiB budget
        srv.submit(A, 200, 20, precision="fp32")
    assert e.value.status == pp.E_BUDGET
    with pytest.raises(pp.PsdprojError) as e:      # k + p > n
        srv.submit(A[:10, :10].contiguous(), 8, 5, precision="fp32")
    assert e.value.status == pp.E_INVALID
    with pytest.raises(pp.PsdprojError):
        srv.poll(12345)                             # unknown ticket
    t, P = srv.submit(A, 4, 2, precision="fp32")
    res = srv.wait(t, 60.0)
    assert res.status == 0 and res.r_plus > 0
    srv.close()
