"""Dual gradient descent for the SDLS problem (Alg. 6), FP64, step by step (oracle; test
infrastructure only).

The semidefinite least-squares problem of the supplementary SDP section,
    min_{X PSD} 1/2 ||X - C/rho||_F^2   subject to  Tr(A_i^T X) = b_i, i = 1..m,
has the partial Lagrangian L(X; y) = 1/2 ||X - C/rho||^2 - sum_i y_i (Tr(A_i^T X) - b_i); its
inner minimiser is X*(y) = (C/rho + sum_i y_i A_i)_+ (the lemma on the analytical solution of
the dual), and the dual function theta(y) = L(X*(y); y) is concave with gradient
-(Tr(A_i^T X*(y)) - b_i)_i.  Alg. 6 ascends theta with the projection replaced by the exact one
(scal = -1, Thm 1), Alg. 2 (scal = 0) or Alg. 3 with alpha from Alg. 5 (scal = 1).

Readings taken where the printed algorithm is ambiguous (listed in the design notes):
  R14  The loop runs at most M iterations (M is "the max number of iterations"; the printed test
       i <= M before the increment would allow M + 1) and at least one: the printed gradient
       initialisation eps * ones(m) has norm eps sqrt(m), which exceeds eps only for m >= 2.
  R15  Iteration i (1-based) draws its test matrix and power-iteration start vectors from the
       Philox key seed + i - 1 (MATLAB draws fresh randn on every call).
  R16  The update is y <- y - beta g with g = (Tr(A_i^T Xhat_+) - b_i)_i, the printed line; it
       ascends theta because grad theta = -g.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import rnla

__all__ = ["SdlsResult", "form_x", "constraint_residual", "dual_value", "dual_gd"]


@dataclasses.dataclass
class SdlsResult:
    y: np.ndarray            # final dual variable
    X_plus: np.ndarray       # the last projection, the approximate primal solution
    iters: int               # iterations run
    grad: np.ndarray         # the last g = (Tr(A_i X_plus) - b_i)_i
    history: list            # ||g|| per iteration


def form_x(C, A, y, rho):
    """X = C/rho + sum_i y_i A_i (line 5 of Alg. 6); A has shape (m, n, n)."""
    X = np.asarray(C, np.float64) / rho
    for yi, Ai in zip(y, A):
        X = X + yi * np.asarray(Ai, np.float64)
    return X


def constraint_residual(A, b, X):
    """g_i = Tr(A_i^T X) - b_i (line 14 of Alg. 6, the gradient of Cor. 3 with its sign)."""
    return np.array([np.sum(np.asarray(Ai, np.float64) * X) for Ai in A]) - np.asarray(b, np.float64)


def dual_value(C, A, b, y, rho):
    """theta(y) = L(X*(y); y) with the exact projection X*(y) = (C/rho + sum y_i A_i)_+."""
    Xs = rnla.exact_projection(form_x(C, A, y, rho))
    Cr = np.asarray(C, np.float64) / rho
    return 0.5 * float(np.sum((Xs - Cr) ** 2)) - float(np.dot(y, constraint_residual(A, b, Xs)))


def dual_gd(C, A, b, rho, k, p, q, N, scal, eps, beta, M, y0, seed=0, omega_dtype=np.float64,
            storage_dtype=np.float64, project=None) -> SdlsResult:
    """Alg. 6.  storage_dtype: the precision X is held in when it is projected (FP32 for the
    FP32 and split-BF16 GPU paths, whose projection reads an FP32 matrix); project, if given,
    replaces the projection step (test hook)."""
    y = np.array(y0, dtype=np.float64)
    m = y.size
    g = eps * np.ones(m)
    history = []
    X_plus = None
    i = 0
    while i < M and (i == 0 or np.linalg.norm(g) > eps):   # R14
        i += 1
        X = form_x(C, A, y, rho).astype(storage_dtype).astype(np.float64)
        if project is not None:
            X_plus = project(X, i)
        elif scal == -1:
            X_plus = rnla.exact_projection(X)                           # Thm 1
        elif scal == 0:
            X_plus = rnla.ran_proj(X, k, p, q, seed=seed + i - 1, omega_dtype=omega_dtype).P     # Alg. 2
        elif scal == 1:
            alpha, _, _ = rnla.min_eig(X, N, seed=seed + i - 1)                                  # Alg. 5
            X_plus = rnla.ran_proj_scal(X, k, p, q, alpha, seed=seed + i - 1, omega_dtype=omega_dtype).P
        else:
            raise ValueError("scal must be -1, 0 or 1")
        X_plus = X_plus.astype(storage_dtype).astype(np.float64)
        g = constraint_residual(A, b, X_plus)
        history.append(float(np.linalg.norm(g)))
        y = y - beta * g                                                # R16
    return SdlsResult(y=y, X_plus=X_plus, iters=i, grad=g, history=history)
