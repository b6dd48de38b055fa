"""Alg. 6 (dual gradient descent for the SDLS problem) on the GPU against the oracle's
oracle.sdls.dual_gd on the same seeded problem: the iterate y, the last projection X and ||g||.

Tolerance of y: one iteration changes y by beta g, and |g_i - g_i^oracle| = |Tr(A_i (P - P_or))|
<= ||A_i||_F ||P - P_or||_F <= e_par max(||P_or||_F, 1e-2 ||X||_F) (the generator normalises
||A_i||_F <= 1), so after one iteration |dy_i| <= beta TOL max(...); over M iterations the
difference also moves X by sum_i |dy_i| ||A_i||, which the bound below covers with a factor
(1 + beta m)^M."""
import numpy as np
import pytest

import _gpu
import workloads
from _gpu import TOL
from oracle import rnla, sdls

pytestmark = pytest.mark.gpu


def _problem(n, m, prec, seed):
    dt = np.float64 if prec == "fp64" else np.float32
    C, A, b, y0 = workloads.sdls_problem(n, m, seed, dtype=dt)
    return C, A, b, y0, dt


@pytest.mark.parametrize("scal,prec", [(0, "fp64"), (1, "fp64"), (0, "fp32"), (1, "bf16x3")])
@pytest.mark.parametrize("iters", [1, 4])
def test_sdls_iterates_match_oracle(scal, prec, iters):
    import torch
    from paper_2410_19208_amd.torch_api import SdlsSolver
    dev = _gpu.device()
    n, m, k, p, q, N, rho, beta, seed = 300, 3, 40, 10, 1, 10, 1.0, 0.5, 5
    C, A, b, y0, dt = _problem(n, m, prec, 31)
    solver = SdlsSolver(n, m, k, p, q, scal, prec, N, iters, rho, beta, 0.0, seed, device=dev)
    y, X, info = solver.solve(torch.from_numpy(C).to(dev), torch.from_numpy(A).to(dev), torch.from_numpy(b),
                              torch.from_numpy(y0))
    torch.cuda.synchronize()
    ref = sdls.dual_gd(C, A, b, rho, k, p, q, N, scal, 0.0, beta, iters, y0, seed=seed, omega_dtype=dt,
                       storage_dtype=dt)
    assert info.status == 0 and info.iters == iters == ref.iters
    y = y.cpu().numpy()
    X = X.cpu().numpy().astype(np.float64)
    x_fro = np.linalg.norm(sdls.form_x(C, A, ref.y + beta * ref.grad, rho))
    scale = max(np.linalg.norm(ref.X_plus), 1e-2 * x_fro)
    tol_y = 4 * iters * beta * TOL[prec] * scale * (1 + beta * m) ** (iters - 1)
    err_y = np.max(np.abs(y - ref.y))
    err_x = np.linalg.norm(X - ref.X_plus) / scale
    print(f"sdls scal={scal} {prec} M={iters}: |dy| {err_y:.2e} (bound {tol_y:.2e}), X {err_x:.2e}, "
          f"||g|| {info.grad_norm:.6e} vs {ref.history[-1]:.6e}")
    assert err_y <= tol_y
    assert err_x <= TOL[prec] * (1 + beta * m) ** (iters - 1)
    assert abs(info.grad_norm - ref.history[-1]) <= 4 * TOL[prec] * scale * np.sqrt(m) * (1 + beta * m) ** (iters - 1)
    assert np.array_equal(X, X.T)


def test_sdls_stops_at_tolerance():
    """eps large enough that the first ||g|| is below it: exactly one iteration; and the GPU's
    iteration count equals the oracle's for a tolerance reached part way."""
    import torch
    from paper_2410_19208_amd.torch_api import SdlsSolver
    dev = _gpu.device()
    n, m = 200, 2
    C, A, b, y0, dt = _problem(n, m, "fp64", 32)
    args = dict(k=60, p=10, q=2, scal=0, precision="fp64", alpha_iters=10, rho=1.0, beta=0.5, seed=1)
    s1 = SdlsSolver(n, m, max_iters=50, eps=1e30, device=dev, **args)
    _, _, info = s1.solve(*(torch.from_numpy(v).to(dev) for v in (C, A)), torch.from_numpy(b), torch.from_numpy(y0))
    assert info.iters == 1
    ref = sdls.dual_gd(C, A, b, 1.0, 60, 10, 2, 10, 0, 0.0, 0.5, 30, y0, seed=1)
    eps = ref.history[9] * 1.0001          # reached at iteration 10 by the oracle
    s2 = SdlsSolver(n, m, max_iters=30, eps=eps, device=dev, **args)
    _, _, info = s2.solve(*(torch.from_numpy(v).to(dev) for v in (C, A)), torch.from_numpy(b), torch.from_numpy(y0))
    expect = next(i + 1 for i, h in enumerate(ref.history) if h <= eps)
    assert info.iters == expect
