"""Shared helpers of the GPU tests: device selection, running the library and the oracle on
the same seeded inputs, and the parity metric."""
import numpy as np
import pytest

import workloads
from oracle import rnla

TOL = {"fp64": 1e-10, "fp32": 1e-5, "bf16x3": 1e-5}


def device():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def to_dev(A, dev):
    import torch
    return torch.from_numpy(np.ascontiguousarray(A)).to(dev)


def storage(prec):
    return np.float64 if prec == "fp64" else np.float32


def run_gpu(A_np, k, p, q, variant, prec, seed=0, alpha=0.0, alpha_iters=10, dev=None):
    import torch
    from paper_2410_19208_amd.torch_api import Projector
    dev = dev or device()
    n = A_np.shape[0]
    proj = Projector(n, k, p, q, variant, prec, seed=seed, alpha=alpha, alpha_iters=alpha_iters, device=dev)
    At = to_dev(A_np.astype(storage(prec)), dev)
    P = proj(At)
    torch.cuda.synchronize()
    return proj, P.cpu().numpy(), proj.result()


def run_oracle(A_np, k, p, q, variant, prec, seed=0, alpha=0.0, alpha_iters=10, keep_P=True):
    A = A_np.astype(storage(prec)).astype(np.float64)
    return rnla.project(A, k, p, q, variant, seed=seed, alpha=alpha if alpha > 0 else None,
                        alpha_iters=alpha_iters, omega_dtype=storage(prec), keep_P=keep_P)


def parity(P_gpu, ref, A_np):
    return rnla.parity_error(P_gpu.astype(np.float64), ref.P, float(np.linalg.norm(A_np.astype(np.float64))))


_CACHE = {}


def matrix(kind, n, seed, **kw):
    """Seeded workload matrix (float64), cached per process; callers get copies."""
    key = (kind, n, seed, tuple(sorted((k, tuple(v) if isinstance(v, (list, tuple, np.ndarray)) else v)
                                       for k, v in kw.items())))
    if key not in _CACHE:
        _CACHE[key] = workloads.make_matrix(kind, n, seed, storage="fp64", **kw)
    A, lam, U = _CACHE[key]
    return A.copy(), lam, U
